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

// Kirchhoff stress tau = P F^T (symmetric), written as tau[a*D+b].
// Neo-Hookean: tau = mu (F F^T - I) + la ln(J) I.
// Fixed-corotated (D == 2): tau = 2 mu (F - R) F^T + la (J - 1) J I with R
// the rotation of the closed-form 2x2 polar decomposition (R = I when F is
// a pure zero of both invariants).  F F^T - I, J - 1 and ln J are formed
// from H = F - I to keep their relative accuracy near the rest state.
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

}  // namespace mr
