// Device building blocks of the MPM transfers shared by the full-order
// kernels and the reduced-order substep.  Internal to libmpmrom.
#pragma once

#include "internal.h"

namespace mr {

// Stencil of one point in D dimensions.
template <int D>
struct Stencil {
    int base[3];
    float f[3];          // x/dx - base, in [0.5, 1.5)
    float w[3][3], dw[3][3];
};

template <int D>
__device__ __forceinline__ bool make_stencil(const GridK &g, const float *xp, Stencil<D> &s)
{
    bool ok = true;
    const int n[3] = {g.n0, g.n1, g.n2};
#pragma unroll
    for (int a = 0; a < D; ++a) {
        s.base[a] = bspline(xp[a], g.inv_dx, n[a], s.w[a], s.dw[a], ok);
        s.f[a] = xp[a] * g.inv_dx - (float)s.base[a];
    }
    return ok;
}

__device__ __forceinline__ int64_t node_lin(const GridK &g, int i, int j, int k)
{
    return (int64_t)i + (int64_t)g.n0 * ((int64_t)j + (int64_t)g.n1 * k);
}

// One Jacobi rotation of a symmetric 3x3 matrix A in the (p, q) plane (r
// the third index) that zeroes A[p][q]: with t = tan(phi) the smaller root
// of t^2 + 2 theta t - 1 = 0, theta = (A_qq - A_pp) / (2 A_pq), the diagonal
// moves by -+ t A_pq and the other row/column rotates; V accumulates the
// rotations (columns: eigenvectors).
template <int p, int q, int r>
__device__ __forceinline__ void jacobi_rotate3(float (&A)[3][3], float (&V)[3][3])
{
    const float apq = A[p][q];
    // below 1e-30 the entry is negligible against any stress this code
    // resolves, and its reciprocal could overflow
    if (fabsf(apq) < 1e-30f) return;
    // hardware reciprocal and reciprocal square root (1 ulp): the rotation
    // only needs to be orthogonal to rounding, and these keep the dependent
    // chain of the sweep short
    const float theta = (A[q][q] - A[p][p]) * __builtin_amdgcn_rcpf(2.0f * apq);
    const float at = fabsf(theta);
    // |theta| > 1e4: t = 1/(2 theta) to within theta^-3 (and theta^2 stays finite)
    const float h = at > 1e4f ? at : at * at + 1.0f;
    const float root = at > 1e4f ? at : h * __builtin_amdgcn_rsqf(h);
    const float t = copysignf(__builtin_amdgcn_rcpf(at + root), theta);
    const float c = __builtin_amdgcn_rsqf(t * t + 1.0f), s = t * c;
    A[p][p] -= t * apq;
    A[q][q] += t * apq;
    A[p][q] = A[q][p] = 0.0f;
    const float arp = A[r][p], arq = A[r][q];
    A[r][p] = A[p][r] = c * arp - s * arq;
    A[r][q] = A[q][r] = s * arp + c * arq;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float vp = V[k][p], vq = V[k][q];
        V[k][p] = c * vp - s * vq;
        V[k][q] = s * vp + c * vq;
    }
}

// Fixed-corotated rotation term in 3D: M = R F^T - I, R the rotation
// closest to F (the polar rotation when J > 0; for J <= 0 the sign moves
// onto the smallest singular value).  With F V = U Sigma' (V, U orthonormal,
// Sigma' the singular values with that sign), R F^T = U Sigma' U^T, so
// M = sum_i (sigma'_i - 1) u_i u_i^T.  The eigen-pairs come from cyclic
// Jacobi on E = F^T F - I = H + H^T + H^T H (H = F - I), whose eigenvalues
// e_i = sigma_i^2 - 1 keep their relative accuracy near the rest state, and
// sigma_i - 1 = e_i / (sqrt(1 + e_i) + 1); u_1, u_2 are the normalised,
// orthogonalised columns F v_1, F v_2 (by decreasing e) and u_3 = u_1 x u_2
// (its sign does not enter M).
__device__ __forceinline__ void corotated_term3(const float *F, const float *H, float Jm1,
                                                float *M)
{
    float E[3][3], V[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            float s = H[a * 3 + b] + H[b * 3 + a];
#pragma unroll
            for (int k = 0; k < 3; ++k) s += H[k * 3 + a] * H[k * 3 + b];
            E[a][b] = s;
            V[a][b] = a == b ? 1.0f : 0.0f;
        }
    for (int sweep = 0; sweep < 6; ++sweep) {
        const float off = E[0][1] * E[0][1] + E[0][2] * E[0][2] + E[1][2] * E[1][2];
        const float dg = E[0][0] * E[0][0] + E[1][1] * E[1][1] + E[2][2] * E[2][2];
        if (!(off > 1e-15f * dg)) break;
        jacobi_rotate3<0, 1, 2>(E, V);
        jacobi_rotate3<0, 2, 1>(E, V);
        jacobi_rotate3<1, 2, 0>(E, V);
    }
    // order by decreasing eigenvalue (permuting the columns of V)
    float e[3] = {E[0][0], E[1][1], E[2][2]};
    int o0 = 0, o1 = 1, o2 = 2, tmp;
    if (e[o0] < e[o1]) { tmp = o0; o0 = o1; o1 = tmp; }
    if (e[o0] < e[o2]) { tmp = o0; o0 = o2; o2 = tmp; }
    if (e[o1] < e[o2]) { tmp = o1; o1 = o2; o2 = tmp; }
    float u1[3], u2[3], u3[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        u1[a] = F[a * 3 + 0] * V[0][o0] + F[a * 3 + 1] * V[1][o0] + F[a * 3 + 2] * V[2][o0];
        u2[a] = F[a * 3 + 0] * V[0][o1] + F[a * 3 + 1] * V[1][o1] + F[a * 3 + 2] * V[2][o1];
    }
    float n1 = u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2];
    if (!(n1 > 1e-30f)) {            // F = 0: any orthonormal frame
        u1[0] = 1.0f; u1[1] = 0.0f; u1[2] = 0.0f;
        n1 = 1.0f;
    }
    const float r1 = __builtin_amdgcn_rsqf(n1);
#pragma unroll
    for (int a = 0; a < 3; ++a) u1[a] *= r1;
    const float d12 = u1[0] * u2[0] + u1[1] * u2[1] + u1[2] * u2[2];
#pragma unroll
    for (int a = 0; a < 3; ++a) u2[a] -= d12 * u1[a];
    float n2 = u2[0] * u2[0] + u2[1] * u2[1] + u2[2] * u2[2];
    if (!(n2 > 1e-30f)) {            // rank one: any unit vector normal to u1
        const int k = (fabsf(u1[0]) <= fabsf(u1[1]) && fabsf(u1[0]) <= fabsf(u1[2])) ? 0
                      : (fabsf(u1[1]) <= fabsf(u1[2]) ? 1 : 2);
        float ek[3] = {0.0f, 0.0f, 0.0f};
        ek[k] = 1.0f;
        u2[0] = u1[1] * ek[2] - u1[2] * ek[1];
        u2[1] = u1[2] * ek[0] - u1[0] * ek[2];
        u2[2] = u1[0] * ek[1] - u1[1] * ek[0];
        n2 = u2[0] * u2[0] + u2[1] * u2[1] + u2[2] * u2[2];
    }
    const float r2 = __builtin_amdgcn_rsqf(n2);
#pragma unroll
    for (int a = 0; a < 3; ++a) u2[a] *= r2;
    u3[0] = u1[1] * u2[2] - u1[2] * u2[1];
    u3[1] = u1[2] * u2[0] - u1[0] * u2[2];
    u3[2] = u1[0] * u2[1] - u1[1] * u2[0];
    const float ea = fmaxf(e[o0], -1.0f), eb = fmaxf(e[o1], -1.0f), ec = fmaxf(e[o2], -1.0f);
    const float s1 = ea / (sqrtf(1.0f + ea) + 1.0f);
    const float s2 = eb / (sqrtf(1.0f + eb) + 1.0f);
    const float s3 = Jm1 > -1.0f ? ec / (sqrtf(1.0f + ec) + 1.0f) : -sqrtf(1.0f + ec) - 1.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = a; b < 3; ++b) {
            const float m = s1 * u1[a] * u1[b] + s2 * u2[a] * u2[b] + s3 * u3[a] * u3[b];
            M[a * 3 + b] = m;
            M[b * 3 + a] = m;
        }
}

// Kirchhoff stress tau = P F^T (symmetric), written as tau[a*D+b].
// Neo-Hookean: tau = mu (F F^T - I) + la ln(J) I.
// Fixed-corotated: tau = 2 mu (F - R) F^T + la (J - 1) J I with R the
// rotation closest to F: in 2D the closed-form rotation by the angle of
// (F00 + F11, F10 - F01) (R = I when both vanish); in 3D
// (F - R) F^T = (F F^T - I) - (R F^T - I) with the second term from
// corotated_term3.  F F^T - I, J - 1 and ln J are formed from H = F - I to
// keep their relative accuracy near the rest state.
// Returns false for J <= 0 (Neo-Hookean) or a non-finite result.
template <int D>
__device__ __forceinline__ bool kirchhoff(int model, float mu, float la, const float *F, float *tau)
{
    float H[D * D];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) H[a * D + b] = F[a * D + b] - (a == b ? 1.0f : 0.0f);
    // J - 1 = tr H + (sum of principal 2x2 minors of H) + det H   (D == 3)
    float Jm1;
    if (D == 2) {
        Jm1 = H[0] + H[3] + (H[0] * H[3] - H[1] * H[2]);
    } else {
        float tr = H[0] + H[4] + H[8];
        float m2 = (H[0] * H[4] - H[1] * H[3]) + (H[0] * H[8] - H[2] * H[6]) +
                   (H[4] * H[8] - H[5] * H[7]);
        float d3 = H[0] * (H[4] * H[8] - H[5] * H[7]) - H[1] * (H[3] * H[8] - H[5] * H[6]) +
                   H[2] * (H[3] * H[7] - H[4] * H[6]);
        Jm1 = tr + m2 + d3;
    }
    if (model == MR_NEO_HOOKEAN) {
        if (!(Jm1 > -1.0f)) return false;
        float lnJ = log1pf(Jm1);
        // F F^T - I = H + H^T + H H^T
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int b = a; b < D; ++b) {
                float s = H[a * D + b] + H[b * D + a];
#pragma unroll
                for (int k = 0; k < D; ++k) s += H[a * D + k] * H[b * D + k];
                float t = mu * s + (a == b ? la * lnJ : 0.0f);
                tau[a * D + b] = t;
                tau[b * D + a] = t;
            }
        return isfinite(lnJ);
    }
    if constexpr (D == 3) {
        float M[9];
        corotated_term3(F, H, Jm1, M);
        const float vol = la * Jm1 * (1.0f + Jm1);
        bool fin = true;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = a; b < 3; ++b) {
                float s = H[a * 3 + b] + H[b * 3 + a];
#pragma unroll
                for (int k = 0; k < 3; ++k) s += H[a * 3 + k] * H[b * 3 + k];
                const float t = 2.0f * mu * (s - M[a * 3 + b]) + (a == b ? vol : 0.0f);
                tau[a * 3 + b] = t;
                tau[b * 3 + a] = t;
                fin = fin && isfinite(t);
            }
        return fin;
    }
    // fixed-corotated, D == 2
    float cs = F[0] + F[3], sn = F[2] - F[1];
    float h = sqrtf(cs * cs + sn * sn);
    float c = 1.0f, s = 0.0f;
    if (h > 0.0f) {
        c = cs / h;
        s = sn / h;
    }
    // F - R = H + (I - R);  1 - c = s^2 / (1 + c) when c > 0
    float omc = (c > 0.0f) ? (s * s) / (1.0f + c) : 1.0f - c;
    float D00 = H[0] + omc, D01 = H[1] + s, D10 = H[2] - s, D11 = H[3] + omc;
    float J = 1.0f + Jm1;
    float vol = la * Jm1 * J;
    // (F - R) F^T
    float t00 = 2.0f * mu * (D00 * F[0] + D01 * F[1]) + vol;
    float t01 = 2.0f * mu * (D00 * F[2] + D01 * F[3]);
    float t10 = 2.0f * mu * (D10 * F[0] + D11 * F[1]);
    float t11 = 2.0f * mu * (D10 * F[2] + D11 * F[3]) + vol;
    // exact symmetry holds in exact arithmetic; symmetrise the rounding
    float off = 0.5f * (t01 + t10);
    tau[0] = t00;
    tau[1] = off;
    tau[2] = off;
    tau[3] = t11;
    return isfinite(t00) && isfinite(off) && isfinite(t11);
}

// Grid boundary band applied to a node velocity (mass already positive).
template <int D>
__device__ __forceinline__ void apply_bc(const GridK &g, int i, int j, int k, float *v)
{
    if (g.bound <= 0) return;
    const int idx[3] = {i, j, k};
    const int n[3] = {g.n0, g.n1, g.n2};
    bool sticky = false, floor_band = false;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        bool lo = idx[a] < g.bound, hi = idx[a] >= n[a] - g.bound;
        if (g.floor_mode == MR_FLOOR_COULOMB && a == 1 && lo)
            floor_band = true;
        else if (lo || hi)
            sticky = true;
    }
    if (sticky) {
#pragma unroll
        for (int a = 0; a < D; ++a) v[a] = 0.0f;
    } else if (floor_band) {
        float vn = v[1];
        if (vn < 0.0f) {
            float nt2 = 0.0f;
#pragma unroll
            for (int a = 0; a < D; ++a)
                if (a != 1) nt2 += v[a] * v[a];
            float nt = sqrtf(nt2);
            if (nt <= -g.mu_f * vn) {
#pragma unroll
                for (int a = 0; a < D; ++a) v[a] = 0.0f;
            } else {
                float sc = 1.0f + g.mu_f * vn / nt;
#pragma unroll
                for (int a = 0; a < D; ++a) v[a] = (a == 1) ? 0.0f : v[a] * sc;
            }
        }
    }
}

// Per-particle quantities scattered by P2G:  node momentum contribution
//   w * (mv + mC (x_i - x_p)) - S grad w,   S = dt V0 tau.
template <int D>
struct P2GPayload {
    float m;
    float mv[D];
    float mC[D * D];
    float S[D * D];
};

// Contribution of one particle to stencil node (o0, o1, o2); returns mass
// and fills momentum.
template <int D>
__device__ __forceinline__ float p2g_node(const GridK &g, const Stencil<D> &st,
                                          const P2GPayload<D> &pl, int o0, int o1, int o2,
                                          float *mom)
{
    const int o[3] = {o0, o1, o2};
    float w = 1.0f, grad[D], dxi[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        w *= st.w[a][o[a]];
        dxi[a] = ((float)o[a] - st.f[a]) * g.dx;
    }
#pragma unroll
    for (int b = 0; b < D; ++b) {
        float gb = 1.0f;
#pragma unroll
        for (int a = 0; a < D; ++a) gb *= (a == b) ? st.dw[a][o[a]] : st.w[a][o[a]];
        grad[b] = gb;
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
        float acc = pl.mv[a];
#pragma unroll
        for (int b = 0; b < D; ++b) acc += pl.mC[a * D + b] * dxi[b];
        float f = 0.0f;
#pragma unroll
        for (int b = 0; b < D; ++b) f += pl.S[a * D + b] * grad[b];
        mom[a] = w * acc - f;
    }
    return w * pl.m;
}

// Separable evaluation of the P2G contributions of one particle to its 3^d
// stencil nodes.  With w = wx wy wz and grad w = (dwx wy wz, wx dwy wz,
// wx wy dwz), the momentum contribution
//   w (mv + mC (x_i - x_p)) - S grad w
// is, for fixed (o1, o2), wx (A + Bx dx0) - Sx dwx with
//   A  = wy wz (mv + mC[:,1] dx1 + mC[:,2] dx2) - (S[:,1] dwy wz + S[:,2] wy dwz),
//   Bx = wy wz mC[:,0],  Sx = wy wz S[:,0],
// so the (o1, o2) part is formed once per row instead of once per node.
// sink(o0, o1, o2, m, mom0, mom1, mom2) receives each node's contribution.
// ORDERED: each node's arithmetic is pinned after the previous node's sink
// (an empty asm that claims to modify the row factors), so that a sink with
// ordered memory side effects does not make the compiler precompute all 3^d
// contributions into registers ahead of them.
template <int D, typename Sink, bool ORDERED = false>
__device__ __forceinline__ void p2g_separable(const GridK &g, const Stencil<D> &st,
                                              const P2GPayload<D> &pl, Sink &&sink)
{
    float dx0[3];
#pragma unroll
    for (int o = 0; o < 3; ++o) dx0[o] = ((float)o - st.f[0]) * g.dx;
    const int oz = (D == 3) ? 3 : 1;
#pragma unroll
    for (int o2 = 0; o2 < oz; ++o2) {
#pragma unroll
        for (int o1 = 0; o1 < 3; ++o1) {
            const float wy = st.w[1][o1], dwy = st.dw[1][o1];
            const float wz = D == 3 ? st.w[2][o2] : 1.0f;
            const float dwz = D == 3 ? st.dw[2][o2] : 0.0f;
            const float wyz = wy * wz, gy = dwy * wz, gz = wy * dwz;
            const float dx1 = ((float)o1 - st.f[1]) * g.dx;
            const float dx2 = D == 3 ? ((float)o2 - st.f[2]) * g.dx : 0.0f;
            float A[D], Bx[D], Sx[D];
#pragma unroll
            for (int a = 0; a < D; ++a) {
                float t = pl.mv[a] + pl.mC[a * D + 1] * dx1;
                float s = pl.S[a * D + 1] * gy;
                if (D == 3) {
                    t += pl.mC[a * D + 2] * dx2;
                    s += pl.S[a * D + 2] * gz;
                }
                A[a] = wyz * t - s;
                Bx[a] = wyz * pl.mC[a * D + 0];
                Sx[a] = wyz * pl.S[a * D + 0];
            }
            const float myz = wyz * pl.m;
#pragma unroll
            for (int o0 = 0; o0 < 3; ++o0) {
                const float wx = st.w[0][o0], dwx = st.dw[0][o0];
                float mom[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int a = 0; a < D; ++a) mom[a] = wx * (A[a] + Bx[a] * dx0[o0]) - Sx[a] * dwx;
                sink(o0, o1, o2, myz * wx, mom[0], mom[1], mom[2]);
                if (ORDERED) {
                    if (D == 3)
                        asm volatile("" : "+v"(A[0]), "+v"(A[D - 2]), "+v"(A[D - 1]),
                                          "+v"(Bx[0]), "+v"(Bx[D - 2]), "+v"(Bx[D - 1]));
                    else
                        asm volatile("" : "+v"(A[0]), "+v"(A[D - 1]), "+v"(Bx[0]), "+v"(Bx[D - 1]));
                }
            }
        }
    }
}

// Separable G2P gather: for fixed (o1, o2) the x-row sums
//   s = sum wx v_i,  sb = sum wx dx0 v_i,  sg = sum dwx v_i
// are combined with the (o1, o2) factors into
//   v += wyz s;  B[:,0] += wyz sb;  B[:,1] += wyz dx1 s;  B[:,2] += wyz dx2 s;
//   gradv[:,0] += wyz sg;  gradv[:,1] += dwy wz s;  gradv[:,2] += wy dwz s.
// fetch(o0, o1, o2) returns the node velocity in .y, .z, .w.
template <int D, typename Fetch, bool ROWWISE = false>
__device__ __forceinline__ void g2p_separable(const GridK &g, const Stencil<D> &st, Fetch &&fetch,
                                              float *vp, float *Bp, float *gv)
{
    float dx0[3];
#pragma unroll
    for (int o = 0; o < 3; ++o) dx0[o] = ((float)o - st.f[0]) * g.dx;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        vp[a] = 0.0f;
#pragma unroll
        for (int b = 0; b < D; ++b) {
            Bp[a * D + b] = 0.0f;
            gv[a * D + b] = 0.0f;
        }
    }
    const int oz = (D == 3) ? 3 : 1;
#pragma unroll
    for (int o2 = 0; o2 < oz; ++o2) {
#pragma unroll
        for (int o1 = 0; o1 < 3; ++o1) {
            float s[D], sb[D], sg[D];
#pragma unroll
            for (int a = 0; a < D; ++a) s[a] = sb[a] = sg[a] = 0.0f;
#pragma unroll
            for (int o0 = 0; o0 < 3; ++o0) {
                const float4 q = fetch(o0, o1, o2);
                const float vi[3] = {q.y, q.z, q.w};
                const float wx = st.w[0][o0], wxd = wx * dx0[o0], dwx = st.dw[0][o0];
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    s[a] += wx * vi[a];
                    sb[a] += wxd * vi[a];
                    sg[a] += dwx * vi[a];
                }
            }
            const float wy = st.w[1][o1], dwy = st.dw[1][o1];
            const float wz = D == 3 ? st.w[2][o2] : 1.0f;
            const float dwz = D == 3 ? st.dw[2][o2] : 0.0f;
            const float wyz = wy * wz, gy = dwy * wz, gz = wy * dwz;
            const float dx1 = ((float)o1 - st.f[1]) * g.dx;
            const float dx2 = D == 3 ? ((float)o2 - st.f[2]) * g.dx : 0.0f;
            const float b1 = wyz * dx1, b2 = wyz * dx2;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                vp[a] += wyz * s[a];
                Bp[a * D + 0] += wyz * sb[a];
                Bp[a * D + 1] += b1 * s[a];
                gv[a * D + 0] += wyz * sg[a];
                gv[a * D + 1] += gy * s[a];
                if (D == 3) {
                    Bp[a * D + 2] += b2 * s[a];
                    gv[a * D + 2] += gz * s[a];
                }
            }
            // ROWWISE: keep the fetches of one x-row from being hoisted above
            // the previous row (bounds the registers held by loads in flight)
            if (ROWWISE) asm volatile("" ::: "memory");
        }
    }
}

// F_new = (I + dt gradv) F
template <int D>
__device__ __forceinline__ void update_F(const float *gv, const float *Fp, float dt, float *Fn)
{
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) {
            float s = Fp[a * D + b];
#pragma unroll
            for (int k = 0; k < D; ++k) s += dt * gv[a * D + k] * Fp[k * D + b];
            Fn[a * D + b] = s;
        }
}

}  // namespace mr
