// Reduced-order-model step on gfx950 (paper Section 3.2, Algorithm 2):
// sample-point selection (Section 3.2.1), Lagrangian-quadrature kinematics
// (Algorithm 3), sample-point MPM substep (Algorithm 5) and projection
// (Algorithms 6 / 7), batched over B parameter instances with a fixed launch
// sequence per step so that K steps can be captured in one HIP graph.
//
// Per step and instance b:
//   1. samples: stratified counter-based draw (SplitMix64), no host input;
//   2. decode every reference particle at xhat_n (needed to find the
//      neighbours, Algorithm 3 step 3);
//   3. mark the 3^d stencil nodes of every sample in a node bitmap (the
//      active nodes I);
//   4. a particle is a quadrature point when any node of its stencil is
//      marked; quadrature points are compacted into Q_b (block scan plus one
//      atomic per block: order inside Q_b is by block, which only permutes
//      the float-atomic summation order of the next step);
//   5. decode x, F = dg/dX, v = (dg/dxhat) vhat at Q_b;
//   6. P2G of Q_b (plain transfer, C = 0, m_p, V0 = m_p / rho0, the
//      instance's Young's modulus) into the instance's grid, skipping nodes
//      outside I;
//   7. for every sample, the grid update of its 3^d nodes (v = p/m + dt g,
//      boundary band) fused into the trial G2P: v_trial, x_trial = x + dt v;
//   8. projection of (x_trial, v_trial) onto the manifold.
// With Eulerian quadrature (Algorithm 4) steps 2-5 become: decode the
// samples only; mark their stencil nodes I and, dilated by two cells, the
// stencil bases whose lattice points touch I (each base once, appended to a
// per-instance list); expand every base into its l^d lattice points; invert
// the decoder at them (a displacement step X = x - u(x) from a positions
// decode, then Newton steps: decoder launches with the spatial tangents and
// a per-point d x d solve); decode x, F, v at the result and keep a
// point when the residual is small, det F > 0 and its reference position
// lies in the body; its mass is rho0 (dx / l)^d / det F (Algorithm 4),
// times a body weight that is 1 inside the body and falls linearly to 0
// across the surface band.  The body test reads a smoothed reference
// density rho_ref, the particles' mass spread with the quadratic B-spline on
// the grid's node lattice (built once at creation): with s = rho_ref / rho0
// the weight is clamp(2 s - 1/2, 0, 1), so every point with s >= 3/4 (all
// of a body's interior at its nominal sampling density) carries exactly
// rho0 V / J and points with s <= 1/4 are dropped.
#include "mpm_kernels.h"
#include "project.h"

#include <math.h>

#include <algorithm>
#include <vector>

#include <stdlib.h>

#include <vector>

struct mr_rom {
    const mr_decoder *dec;
    int d, r;
    mr::GridK g;
    mr_rom_config cfg;
    mr_gn_opts opts;
    int B;
    int64_t P, ns_max, q_cap, nodes, words;
    float *X, *m, *E;      // X and m in the runner's particle order
    int32_t *internal_of;  // [P] caller's particle index -> runner's index
    int32_t *n_samples;
    int32_t *samples;   // [B][ns_max]
    float *x_all;       // [B][d][P]
    uint32_t *bitmap;   // [B][words]
    int32_t *Q;         // [B][q_cap]
    int32_t *q_count;   // [B]
    int32_t *n_active;  // [B]
    float *xQ, *FQ, *vQ;
    float *grid;        // [B][nodes][4]
    float *xs, *xt, *vt;
    double *z_next, *v_next;
    int32_t *status_step;  // [B]
    int64_t *counter;      // device step counter
    void *proj_ws;
    hipStream_t cap_stream;
    hipGraphExec_t graph;
    int graph_steps;
    double graph_dt;
    double *graph_ptrs[3];
    int32_t *graph_status;
    // Eulerian quadrature
    int quad, ell, newton_iters;
    float newton_tol;
    int64_t qb_cap;        // stencil bases per instance
    uint32_t *qb_bitmap;   // [B][words]
    int32_t *qbase;        // [B][qb_cap] node index of each base
    int32_t *qb_count;     // [B]
    float *XQ;             // [B][d][q_cap] reference positions (Newton iterate)
    float *mQ;             // [B][q_cap] point masses (0: discarded)
    float *rho;            // smoothed reference density on the grid's node lattice
    int rn[3];             // its nodes per axis (the grid's)
    // the per-instance grids and bitmaps are all zero between steps: a step
    // clears only what it marked; set when a step was left unfinished
    int dirty;
    // initial-condition correction fields (Lagrangian quadrature), runner
    // order: a, b [B][d][P], grad a, grad b [B][d*d][P]; used when fields_on
    float *fa, *fb, *fGa, *fGb;
    int fields_on;
};

namespace mr {

__device__ __forceinline__ uint64_t mix64(uint64_t c)
{
    uint64_t z = c + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void sample_kernel(uint64_t seed, const int64_t *counter, int64_t P, int ns_max,
                              const int32_t *n_samples, const int32_t *internal_of,
                              int32_t *samples)
{
    const int b = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ns_max) return;
    const int64_t S = n_samples[b];
    const uint64_t step = (uint64_t)(*counter);
    const uint64_t key = mix64(mix64(mix64(seed) ^ (uint64_t)b) ^ step);
    int32_t idx;
    if (k < S) {
        int64_t lo = ((int64_t)k * P) / S, hi = ((int64_t)(k + 1) * P) / S;
        idx = (int32_t)(lo + (int64_t)(mix64(key ^ (uint64_t)k) % (uint64_t)(hi - lo)));
    } else {
        idx = 0;  // padding entry, masked by the per-instance count
    }
    // draws are particle indices of the caller's order; the runner stores the
    // particles in its own (cell-coherent) order
    samples[(int64_t)b * ns_max + k] = internal_of[idx];
}

template <int D>
__global__ void gather_mark_kernel(GridK g, int64_t P, int ns_max, const int32_t *n_samples,
                                   const int32_t *samples, const float *x_all, float *xs,
                                   uint32_t *bitmap, int64_t words, int32_t *status)
{
    const int b = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ns_max) return;
    const int64_t q = samples[(int64_t)b * ns_max + k];
    float xp[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        xp[a] = x_all[((int64_t)b * D + a) * P + q];
        xs[((int64_t)b * D + a) * ns_max + k] = xp[a];
    }
    if (k >= n_samples[b]) return;
    Stencil<D> st;
    if (!make_stencil<D>(g, xp, st)) {
        atomicOr(status + b, MR_FLAG_DOMAIN);
        return;
    }
    uint32_t *bm = bitmap + (int64_t)b * words;
    const int oz = (D == 3) ? 3 : 1;
    for (int o2 = 0; o2 < oz; ++o2)
        for (int o1 = 0; o1 < 3; ++o1)
            for (int o0 = 0; o0 < 3; ++o0) {
                int64_t i = node_lin(g, st.base[0] + o0, st.base[1] + o1, D == 3 ? st.base[2] + o2 : 0);
                atomicOr(bm + (i >> 5), 1u << (i & 31));
            }
}

__device__ __forceinline__ bool bit_set(const uint32_t *bm, int64_t i)
{
    return (bm[i >> 5] >> (i & 31)) & 1u;
}

constexpr int NB_BLOCK = 1024;

template <int D>
__global__ void __launch_bounds__(NB_BLOCK) neighbour_kernel(GridK g, int64_t P, int64_t words,
                                                             const float *x_all,
                                                             const uint32_t *bitmap, int32_t *Q,
                                                             int64_t q_cap, int32_t *q_count,
                                                             int32_t *status)
{
    __shared__ int sh[NB_BLOCK];
    __shared__ int base_sh;
    const int b = blockIdx.y;
    const int64_t q = (int64_t)blockIdx.x * NB_BLOCK + threadIdx.x;
    int flag = 0;
    if (q < P) {
        float xp[D];
#pragma unroll
        for (int a = 0; a < D; ++a) xp[a] = x_all[((int64_t)b * D + a) * P + q];
        Stencil<D> st;
        if (make_stencil<D>(g, xp, st)) {
            const uint32_t *bm = bitmap + (int64_t)b * words;
            const int oz = (D == 3) ? 3 : 1;
            for (int o2 = 0; o2 < oz && !flag; ++o2)
                for (int o1 = 0; o1 < 3 && !flag; ++o1)
                    for (int o0 = 0; o0 < 3 && !flag; ++o0)
                        flag = bit_set(bm, node_lin(g, st.base[0] + o0, st.base[1] + o1,
                                                    D == 3 ? st.base[2] + o2 : 0));
        }
        // a decoded particle outside the lattice cannot touch the sample nodes
    }
    // block-wide exclusive scan of the flags (Hillis-Steele)
    const int t = threadIdx.x;
    sh[t] = flag;
    __syncthreads();
    for (int off = 1; off < NB_BLOCK; off <<= 1) {
        int add = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    int total = sh[NB_BLOCK - 1];
    if (t == 0) base_sh = total ? atomicAdd(q_count + b, total) : 0;
    __syncthreads();
    if (flag) {
        int64_t pos = (int64_t)base_sh + sh[t] - 1;
        if (pos < q_cap)
            Q[(int64_t)b * q_cap + pos] = (int32_t)q;
        else
            atomicOr(status + b, MR_FLAG_DOMAIN);  // quadrature capacity exceeded
    }
}

__global__ void clamp_count_kernel(int B, int32_t *q_count, int64_t q_cap)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B && q_count[b] > q_cap) q_count[b] = (int32_t)q_cap;
}

// P2G of Algorithm 5 over the quadrature list (C = 0, m = m_p, V0 = m_p / rho0),
// restricted to the marked nodes I.  Consecutive entries of the list
// (ascending particle index) mostly share a base cell and so the same 3^d
// nodes; the lanes of a wave first sum their contributions over each run of
// equal base cells (segmented suffix sums by shifts of 1, 2, 4, ... within the
// run) and only the run's first lane issues the HBM atomics.
template <int D>
__global__ void __launch_bounds__(256) p2g_quad_kernel(GridK g, int64_t q_cap, int64_t words,
                                                       const int32_t *q_count, const int32_t *Q,
                                                       const float *xQ, const float *FQ,
                                                       const float *vQ, const float *m_all,
                                                       const float *m_q,
                                                       float m_uniform, float inv_rho0,
                                                       const float *E, float nu, int model,
                                                       float dt, const uint32_t *bitmap,
                                                       float *grid, int64_t nodes, int32_t *status)
{
    constexpr int NS = (D == 3) ? 27 : 9;
    const int b = blockIdx.y;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool act = s < q_count[b];
    float val[NS][D + 1];
#pragma unroll
    for (int i = 0; i < NS; ++i)
#pragma unroll
        for (int c = 0; c <= D; ++c) val[i][c] = 0.0f;
    int key = -2 - lane;            // distinct for lanes without a contribution
    Stencil<D> st;
    const uint32_t *bm = bitmap + (int64_t)b * words;
    // point mass: per point (Eulerian quadrature; 0 marks a discarded point)
    // or the particle's
    float m = 0.0f;
    if (act) {
        if (m_q) {
            m = m_q[(int64_t)b * q_cap + s];
        } else {
            const int32_t q = Q[(int64_t)b * q_cap + s];
            m = m_all ? m_all[q] : m_uniform;
        }
    }
    if (act && m > 0.0f) {
        float xp[D], vp[D], Fp[D * D], tau[D * D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            xp[a] = xQ[((int64_t)b * D + a) * q_cap + s];
            vp[a] = vQ[((int64_t)b * D + a) * q_cap + s];
        }
#pragma unroll
        for (int k = 0; k < D * D; ++k) Fp[k] = FQ[((int64_t)b * D * D + k) * q_cap + s];
        Lame lm = lame_of(E[b], nu);
        bool ok = make_stencil<D>(g, xp, st);
        ok = kirchhoff<D>(model, lm.mu, lm.la, Fp, tau) && ok;
        if (!ok) {
            atomicOr(status + b, MR_FLAG_DOMAIN);
        } else {
            P2GPayload<D> pl;
            pl.m = m;
            const float sc = dt * m * inv_rho0;
#pragma unroll
            for (int a = 0; a < D; ++a) pl.mv[a] = m * vp[a];
#pragma unroll
            for (int k = 0; k < D * D; ++k) {
                pl.mC[k] = 0.0f;
                pl.S[k] = sc * tau[k];
            }
            key = (int)node_lin(g, st.base[0], st.base[1], D == 3 ? st.base[2] : 0);
#pragma unroll
            for (int o2 = 0; o2 < (D == 3 ? 3 : 1); ++o2)
#pragma unroll
                for (int o1 = 0; o1 < 3; ++o1)
#pragma unroll
                    for (int o0 = 0; o0 < 3; ++o0) {
                        const int i = o0 + 3 * (o1 + 3 * o2);
                        float mom[D];
                        val[i][0] = p2g_node<D>(g, st, pl, o0, o1, o2, mom);
#pragma unroll
                        for (int a = 0; a < D; ++a) val[i][1 + a] = mom[a];
                    }
        }
    }
    // runs of equal keys among consecutive lanes: run_end = last lane of mine
    const int key_next = __shfl_down(key, 1);
    const bool last = lane == 63 || key_next != key;
    const uint64_t lastmask = __ballot(last);
    const int run_end = __ffsll((long long)(lastmask & (~0ull << lane))) - 1;
    const int key_prev = __shfl_up(key, 1);
    const bool head = lane == 0 || key_prev != key;
    for (int dist = 1; dist < 64; dist <<= 1) {
        const bool take = lane + dist <= run_end;
        if (__ballot(take) == 0) break;
#pragma unroll
        for (int i = 0; i < NS; ++i)
#pragma unroll
            for (int c = 0; c <= D; ++c) {
                const float o = __shfl_down(val[i][c], dist);
                if (take) val[i][c] += o;
            }
    }
    if (!head || key < 0) return;
    float *gb = grid + (int64_t)b * nodes * 4;
#pragma unroll
    for (int o2 = 0; o2 < (D == 3 ? 3 : 1); ++o2)
#pragma unroll
        for (int o1 = 0; o1 < 3; ++o1)
#pragma unroll
            for (int o0 = 0; o0 < 3; ++o0) {
                const int64_t i = node_lin(g, st.base[0] + o0, st.base[1] + o1,
                                           D == 3 ? st.base[2] + o2 : 0);
                if (!bit_set(bm, i)) continue;
                const int k = o0 + 3 * (o1 + 3 * o2);
                float *gp = gb + 4 * i;
                atomicAdd(gp, val[k][0]);
#pragma unroll
                for (int a = 0; a < D; ++a) atomicAdd(gp + 1 + a, val[k][1 + a]);
            }
}

template <int D>
__global__ void g2p_trial_kernel(GridK g, int ns_max, const int32_t *n_samples, const float *xs,
                                 const float *grid, int64_t nodes, float dt, float *xt, float *vt)
{
    const int b = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ns_max) return;
    float xp[D];
#pragma unroll
    for (int a = 0; a < D; ++a) xp[a] = xs[((int64_t)b * D + a) * ns_max + k];
    Stencil<D> st;
    float vp[D] = {};
    if (k < n_samples[b] && make_stencil<D>(g, xp, st)) {
        const float4 *gb = reinterpret_cast<const float4 *>(grid) + (int64_t)b * nodes;
        const float gr[3] = {g.g0, g.g1, g.g2};
        const int oz = (D == 3) ? 3 : 1;
        for (int o2 = 0; o2 < oz; ++o2)
            for (int o1 = 0; o1 < 3; ++o1)
                for (int o0 = 0; o0 < 3; ++o0) {
                    int i0 = st.base[0] + o0, i1 = st.base[1] + o1, i2 = D == 3 ? st.base[2] + o2 : 0;
                    float4 q = gb[node_lin(g, i0, i1, i2)];
                    if (!(q.x > 0.0f)) continue;
                    float inv = 1.0f / q.x;
                    float vi[3] = {q.y * inv + dt * gr[0], q.z * inv + dt * gr[1],
                                   D == 3 ? q.w * inv + dt * gr[2] : 0.0f};
                    apply_bc<D>(g, i0, i1, i2, vi);
                    float w = st.w[0][o0] * st.w[1][o1] * (D == 3 ? st.w[2][o2] : 1.0f);
#pragma unroll
                    for (int a = 0; a < D; ++a) vp[a] += w * vi[a];
                }
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
        vt[((int64_t)b * D + a) * ns_max + k] = vp[a];
        xt[((int64_t)b * D + a) * ns_max + k] = xp[a] + dt * vp[a];
    }
}

// --- Eulerian quadrature (Algorithm 4) -------------------------------------

// lattice point `sub` (0 .. l^d - 1) of the stencil base with node index
// base_lin: per axis the l points (m + 1/2) dx / l, m = l b + l/2 + j, whose
// stencil base is b (they lie in ((b + 1/2) dx, (b + 3/2) dx))
template <int D>
__device__ __forceinline__ void eul_point(const GridK &g, int32_t base_lin, int sub, int L,
                                          float *xq)
{
    int bc[3];
    bc[0] = base_lin % g.n0;
    bc[1] = (base_lin / g.n0) % g.n1;
    bc[2] = base_lin / (g.n0 * g.n1);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const int j = sub % L;
        sub /= L;
        const int m = L * bc[a] + L / 2 + j;
        xq[a] = ((float)m + 0.5f) * (g.dx / (float)L);
    }
}

// one thread per (sample, offset in -2..2 per axis): marks the sample's
// stencil nodes in I (offsets 0..2) and the stencil bases within two cells
// (their lattice points touch I), appending each newly marked base once
template <int D>
__global__ void eul_mark_kernel(GridK g, int ns_max, const int32_t *n_samples, const float *xs,
                                uint32_t *bitmap, uint32_t *qb_bitmap, int64_t words,
                                int32_t *qbase, int64_t qb_cap, int32_t *qb_count,
                                int32_t *status)
{
    constexpr int NO = (D == 3) ? 125 : 25;
    const int b = blockIdx.y;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int k = (int)(t / NO), o = (int)(t % NO);
    if (k >= ns_max || k >= n_samples[b]) return;
    float xp[D];
#pragma unroll
    for (int a = 0; a < D; ++a) xp[a] = xs[((int64_t)b * D + a) * ns_max + k];
    Stencil<D> st;
    if (!make_stencil<D>(g, xp, st)) {
        if (o == 0) atomicOr(status + b, MR_FLAG_DOMAIN);
        return;
    }
    const int n[3] = {g.n0, g.n1, g.n2};
    int off[3] = {o % 5 - 2, (o / 5) % 5 - 2, D == 3 ? o / 25 - 2 : 0};
    int q[3] = {0, 0, 0};
    bool node = true, valid = true;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        q[a] = st.base[a] + off[a];
        node = node && off[a] >= 0;
        valid = valid && q[a] >= 0 && q[a] + 2 <= n[a] - 1;
    }
    const int64_t i = node_lin(g, q[0], q[1], q[2]);
    if (node) atomicOr(bitmap + (int64_t)b * words + (i >> 5), 1u << (i & 31));
    if (!valid) return;
    const uint32_t bit = 1u << (i & 31);
    const uint32_t old = atomicOr(qb_bitmap + (int64_t)b * words + (i >> 5), bit);
    if (old & bit) return;
    const int32_t pos = atomicAdd(qb_count + b, 1);
    if (pos < qb_cap)
        qbase[(int64_t)b * qb_cap + pos] = (int32_t)i;
    else
        atomicOr(status + b, MR_FLAG_DOMAIN);  // capacity exceeded
}

__global__ void eul_count_kernel(int B, const int32_t *qb_count, int64_t qb_cap, int LD,
                                 int32_t *q_count)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const int64_t nb = qb_count[b] < qb_cap ? qb_count[b] : qb_cap;
    q_count[b] = (int32_t)(nb * LD);
}

// Newton's starting point X = x^Q
template <int D>
__global__ void eul_init_kernel(GridK g, int64_t q_cap, const int32_t *q_count,
                                const int32_t *qbase, int64_t qb_cap, int L, int LD, float *XQ)
{
    const int b = blockIdx.y;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= q_count[b]) return;
    float xq[D];
    eul_point<D>(g, qbase[(int64_t)b * qb_cap + s / LD], (int)(s % LD), L, xq);
#pragma unroll
    for (int a = 0; a < D; ++a) XQ[((int64_t)b * D + a) * q_cap + s] = xq[a];
}

// determinant and solution of F y = r (Cramer's rule, d <= 3)
template <int D>
__device__ __forceinline__ float solve_small(const float *F, const float *r, float *y)
{
    if (D == 2) {
        const float det = F[0] * F[3] - F[1] * F[2];
        const float inv = 1.0f / det;
        y[0] = (F[3] * r[0] - F[1] * r[1]) * inv;
        y[1] = (F[0] * r[1] - F[2] * r[0]) * inv;
        return det;
    }
    const float c00 = F[4] * F[8] - F[5] * F[7];
    const float c01 = F[5] * F[6] - F[3] * F[8];
    const float c02 = F[3] * F[7] - F[4] * F[6];
    const float det = F[0] * c00 + F[1] * c01 + F[2] * c02;
    const float inv = 1.0f / det;
    // y = adj(F) r / det, adj(F) = cofactor matrix transposed
    const float c10 = F[2] * F[7] - F[1] * F[8];
    const float c11 = F[0] * F[8] - F[2] * F[6];
    const float c12 = F[1] * F[6] - F[0] * F[7];
    const float c20 = F[1] * F[5] - F[2] * F[4];
    const float c21 = F[2] * F[3] - F[0] * F[5];
    const float c22 = F[0] * F[4] - F[1] * F[3];
    y[0] = (c00 * r[0] + c10 * r[1] + c20 * r[2]) * inv;
    y[1] = (c01 * r[0] + c11 * r[1] + c21 * r[2]) * inv;
    y[2] = (c02 * r[0] + c12 * r[1] + c22 * r[2]) * inv;
    return det;
}

template <int D>
__device__ __forceinline__ float det_small(const float *F)
{
    if (D == 2) return F[0] * F[3] - F[1] * F[2];
    return F[0] * (F[4] * F[8] - F[5] * F[7]) + F[1] * (F[5] * F[6] - F[3] * F[8]) +
           F[2] * (F[3] * F[7] - F[4] * F[6]);
}

// one step X <- X - F^{-1} (g(X) - x^Q) from the decoded g and F (F null:
// the identity, i.e. X <- x^Q - u)
template <int D>
__global__ void eul_newton_kernel(GridK g, int64_t q_cap, const int32_t *q_count,
                                  const int32_t *qbase, int64_t qb_cap, int L, int LD,
                                  const float *xg, const float *FQ, float *XQ)
{
    const int b = blockIdx.y;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= q_count[b]) return;
    float xq[D], r[D], F[D * D], y[D];
    eul_point<D>(g, qbase[(int64_t)b * qb_cap + s / LD], (int)(s % LD), L, xq);
#pragma unroll
    for (int a = 0; a < D; ++a) r[a] = xg[((int64_t)b * D + a) * q_cap + s] - xq[a];
    if (FQ) {
#pragma unroll
        for (int k = 0; k < D * D; ++k) F[k] = FQ[((int64_t)b * D * D + k) * q_cap + s];
        const float det = solve_small<D>(F, r, y);
        if (!(det != 0.0f) || !isfinite(det)) return;   // left as is; rejected at the end
    } else {
#pragma unroll
        for (int a = 0; a < D; ++a) y[a] = r[a];
    }
#pragma unroll
    for (int a = 0; a < D; ++a) XQ[((int64_t)b * D + a) * q_cap + s] -= y[a];
}

// acceptance and mass; the point's position becomes the exact lattice point
template <int D>
__global__ void eul_finish_kernel(GridK g, int64_t q_cap, const int32_t *q_count,
                                  const int32_t *qbase, int64_t qb_cap, int L, int LD,
                                  const float *XQ, float *xQ, const float *FQ, const float *rho,
                                  int rn0, int rn1, int rn2, float rho0_vq, float inv_rho0,
                                  float tol, float *mQ)
{
    const int b = blockIdx.y;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= q_count[b]) return;
    float xq[D], F[D * D];
    eul_point<D>(g, qbase[(int64_t)b * qb_cap + s / LD], (int)(s % LD), L, xq);
    float res = 0.0f;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const int64_t o = ((int64_t)b * D + a) * q_cap + s;
        res = fmaxf(res, fabsf(xQ[o] - xq[a]));
        xQ[o] = xq[a];
    }
#pragma unroll
    for (int k = 0; k < D * D; ++k) F[k] = FQ[((int64_t)b * D * D + k) * q_cap + s];
    const float J = det_small<D>(F);
    // multilinear reading of the smoothed density at X (0 off the lattice)
    const int rn[3] = {rn0, rn1, rn2};
    const float inv_h = g.inv_dx;
    int i0[3] = {0, 0, 0};
    float fr[3] = {0.0f, 0.0f, 0.0f};
    bool on = true;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const float t = XQ[((int64_t)b * D + a) * q_cap + s] * inv_h;
        const float tf = floorf(t);
        on = on && tf >= 0.0f && tf <= (float)(rn[a] - 2);
        i0[a] = on ? (int)tf : 0;
        fr[a] = t - tf;
    }
    float dens = 0.0f;
    if (on) {
#pragma unroll
        for (int c = 0; c < (1 << D); ++c) {
            float w = 1.0f;
            int64_t idx = 0, stride = 1;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const int bit = (c >> a) & 1;
                w *= bit ? fr[a] : 1.0f - fr[a];
                idx += (int64_t)(i0[a] + bit) * stride;
                stride *= rn[a];
            }
            dens += w * rho[idx];
        }
    }
    const float wbody = fminf(fmaxf(2.0f * dens * inv_rho0 - 0.5f, 0.0f), 1.0f);
    const bool keep = res <= tol && J > 0.0f && wbody > 0.0f;
    mQ[(int64_t)b * q_cap + s] = keep ? wbody * rho0_vq / J : 0.0f;
}

__global__ void fill_u32_kernel(uint32_t *a, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0u;
}

__global__ void fill_f4_kernel(float4 *a, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        a[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

__global__ void advance_kernel(int B, int r, double *z, double *zp, double *v, const double *zn,
                               const double *vn, const int32_t *status_step, int32_t *status_out,
                               int64_t *counter)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < B * r) {
        zp[t] = z[t];
        z[t] = zn[t];
        v[t] = vn[t];
    }
    if (t < B && status_out) status_out[t] |= status_step[t];
    if (t == 0) *counter += 1;
}

__global__ void set_counter_kernel(int64_t *counter, int64_t v) { *counter = v; }

// --- initial-condition correction fields (Section 3.1, eq. defMapApproxForm)
// g~(X, xhat, t) = g(X; xhat) + a(X) + b(X) t, t = step counter x dt.

// decoded positions of every particle (runner order) += a + b t
__global__ void field_positions_kernel(int d, int64_t P, const int64_t *counter, double dt,
                                       const float *fa, const float *fb, float *x_all)
{
    const int b = blockIdx.y;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const float t = (float)((double)*counter * dt);
    for (int a = 0; a < d; ++a) {
        const int64_t i = ((int64_t)b * d + a) * P + p;
        x_all[i] += fa[i] + fb[i] * t;
    }
}

// quadrature kinematics: x += a + b t, F += grad a + t grad b, v += b
__global__ void field_quad_kernel(int d, int64_t P, int64_t q_cap, const int32_t *q_count,
                                  const int32_t *Q, const int64_t *counter, double dt,
                                  const float *fa, const float *fb, const float *fGa,
                                  const float *fGb, float *xQ, float *FQ, float *vQ)
{
    const int b = blockIdx.y;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= q_count[b]) return;
    const int64_t p = Q[(int64_t)b * q_cap + s];
    const float t = (float)((double)*counter * dt);
    for (int a = 0; a < d; ++a) {
        const int64_t i = ((int64_t)b * d + a) * P + p;
        const int64_t o = ((int64_t)b * d + a) * q_cap + s;
        xQ[o] += fa[i] + fb[i] * t;
        vQ[o] += fb[i];
    }
    for (int k = 0; k < d * d; ++k) {
        const int64_t i = ((int64_t)b * d * d + k) * P + p;
        FQ[((int64_t)b * d * d + k) * q_cap + s] += fGa[i] + fGb[i] * t;
    }
}

// the projection fits g~ at t + dt: with x_trial = g(xhat_n) + dt v_trial
// (positions on displacements), shifting the trial velocities by -b moves
// both fields to the targets (x_trial - a - b (t + dt), v_trial - b)
__global__ void field_velocity_kernel(int d, int64_t P, int ns_max, const int32_t *n_samples,
                                      const int32_t *samples, const float *fb, float *vt)
{
    const int b = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ns_max || k >= n_samples[b]) return;
    const int64_t p = samples[(int64_t)b * ns_max + k];
    for (int a = 0; a < d; ++a)
        vt[((int64_t)b * d + a) * ns_max + k] -= fb[((int64_t)b * d + a) * P + p];
}

// fields from the decodes at xhat0: a = X - g, grad a = I - dg/dX,
// b = V0 - (dg/dxhat) vhat0 (in place over the decoded x, F, v)
__global__ void field_init_kernel(int d, int64_t P, const float *X, const float *v0, float *fa,
                                  float *fb, float *fGa)
{
    const int b = blockIdx.y;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    for (int a = 0; a < d; ++a) {
        const int64_t i = ((int64_t)b * d + a) * P + p;
        fa[i] = X[(int64_t)a * P + p] - fa[i];
        fb[i] = v0[b * d + a] - fb[i];
    }
    for (int a = 0; a < d; ++a)
        for (int c = 0; c < d; ++c) {
            const int64_t i = ((int64_t)b * d * d + a * d + c) * P + p;
            fGa[i] = (a == c ? 1.0f : 0.0f) - fGa[i];
        }
}

// latents xhat0 +- eps_b vhat0 with eps_b = h / max_k |vhat0_k| (0 when
// vhat0 = 0); inv2e[b] = 1 / (2 eps_b) or 0
__global__ void field_fd_latents_kernel(int B, int r, double h, const double *z0, const double *v0,
                                        double *zp, double *zm, double *inv2e)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double m = 0.0;
    for (int k = 0; k < r; ++k) m = fmax(m, fabs(v0[b * r + k]));
    const double eps = m > 0.0 ? h / m : 0.0;
    for (int k = 0; k < r; ++k) {
        zp[b * r + k] = z0[b * r + k] + eps * v0[b * r + k];
        zm[b * r + k] = z0[b * r + k] - eps * v0[b * r + k];
    }
    inv2e[b] = m > 0.0 ? 0.5 / eps : 0.0;
}

// grad b = -(dg/dX (xhat0 + eps vhat0) - dg/dX (xhat0 - eps vhat0)) / (2 eps)
// for instances b0 .. b0 + gridDim.y - 1 (Fp in place)
__global__ void field_grad_b_kernel(int d, int64_t P, int b0, const double *inv2e, float *Fp,
                                    const float *Fm)
{
    const int bl = blockIdx.y;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const float s = (float)inv2e[b0 + bl];
    for (int k = 0; k < d * d; ++k) {
        const int64_t i = ((int64_t)bl * d * d + k) * P + p;
        Fp[i] = -(Fp[i] - Fm[i]) * s;
    }
}

// caller-order positions += a + b t (fields in runner order, internal_of
// maps the caller's particle to the runner's)
__global__ void field_caller_positions_kernel(int d, int64_t P, const int32_t *internal_of,
                                              float t, const float *fa, const float *fb, float *x)
{
    const int b = blockIdx.y;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int64_t q = internal_of[p];
    for (int a = 0; a < d; ++a) {
        const int64_t o = ((int64_t)b * d + a) * P;
        x[o + p] += fa[o + q] + fb[o + q] * t;
    }
}

// After the substep has read the grid: zero the grid nodes of every
// instance's marked set I and the marks themselves (node bitmap and, for the
// Eulerian quadrature, the stencil-base bitmap), so that the next step
// starts from zero grids without refilling them (all other nodes are still
// zero); counts |I| per instance on the way.  Grid (x blocks, B).
__global__ void clear_marked_kernel(int64_t words, int64_t nodes, uint32_t *bitmap,
                                    uint32_t *qb_bitmap, float4 *grid, int32_t *n_active)
{
    const int b = blockIdx.y;
    int cnt = 0;
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < words;
         w += (int64_t)gridDim.x * blockDim.x) {
        const int64_t wi = (int64_t)b * words + w;
        if (qb_bitmap && qb_bitmap[wi] != 0u) qb_bitmap[wi] = 0u;
        uint32_t m = bitmap[wi];
        if (m == 0u) continue;
        bitmap[wi] = 0u;
        cnt += __popc(m);
        while (m != 0u) {
            const int k = __ffs(m) - 1;
            m &= m - 1u;
            const int64_t i = 32 * w + k;
            if (i < nodes) grid[(int64_t)b * nodes + i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
    }
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_down(cnt, off);
    if ((threadIdx.x & 63) == 0 && cnt != 0) atomicAdd(n_active + b, cnt);
}

// every grid, bitmap and count of the runner to zero (creation, and after a
// step that was left unfinished)
void clear_all(mr_rom *R, hipStream_t st)
{
    const int TB = 256;
    const int64_t B = R->B;
    fill_u32_kernel<<<2048, TB, 0, st>>>(R->bitmap, B * R->words);
    if (R->qb_bitmap) fill_u32_kernel<<<2048, TB, 0, st>>>(R->qb_bitmap, B * R->words);
    fill_f4_kernel<<<4096, TB, 0, st>>>(reinterpret_cast<float4 *>(R->grid), B * R->nodes);
    fill_u32_kernel<<<(unsigned)ceil_div(B, TB), TB, 0, st>>>((uint32_t *)R->n_active, B);
}

int32_t rom_one_step(mr_rom *R, double dt, double *xhat, double *xhat_prev, double *vhat,
                     int32_t *status_out, hipStream_t st)
{
    const int B = R->B, d = R->d, r = R->r;
    const GridK &g = R->g;
    const int TB = 256;
    int32_t rc;
    dim3 gs((unsigned)ceil_div(R->ns_max, TB), (unsigned)B);
    fill_u32_kernel<<<(unsigned)ceil_div(B, TB), TB, 0, st>>>((uint32_t *)R->status_step, B);
    fill_u32_kernel<<<(unsigned)ceil_div(B, TB), TB, 0, st>>>((uint32_t *)R->q_count, B);
    fill_u32_kernel<<<(unsigned)ceil_div(B, TB), TB, 0, st>>>((uint32_t *)R->n_active, B);
    // the grids and bitmaps are zero here (cleared by the previous step)
    R->dirty = 1;
    sample_kernel<<<gs, TB, 0, st>>>(R->cfg.seed, R->counter, R->P, (int)R->ns_max, R->n_samples,
                                      R->internal_of, R->samples);
    MR_LAUNCH_CHECK();
    dim3 gq((unsigned)ceil_div(R->q_cap, TB), (unsigned)B);
    float inv_rho0 = 1.0f / R->cfg.rho0;
    if (R->quad == MR_QUAD_EULERIAN) {
        // Algorithm 4
        const int L = R->ell;
        const int LD = d == 3 ? L * L * L : L * L;
        fill_u32_kernel<<<(unsigned)ceil_div(B, TB), TB, 0, st>>>((uint32_t *)R->qb_count, B);
        rc = decode_jac_ex(R->dec, B, R->P, R->X, R->ns_max, R->samples, 1, R->n_samples, xhat,
                           nullptr, R->xs, nullptr, nullptr, nullptr, st);
        if (rc != MR_OK) return rc;
        const int no = d == 3 ? 125 : 25;
        dim3 gm((unsigned)ceil_div(R->ns_max * no, TB), (unsigned)B);
        if (d == 2)
            eul_mark_kernel<2><<<gm, TB, 0, st>>>(g, (int)R->ns_max, R->n_samples, R->xs, R->bitmap,
                                                  R->qb_bitmap, R->words, R->qbase, R->qb_cap,
                                                  R->qb_count, R->status_step);
        else
            eul_mark_kernel<3><<<gm, TB, 0, st>>>(g, (int)R->ns_max, R->n_samples, R->xs, R->bitmap,
                                                  R->qb_bitmap, R->words, R->qbase, R->qb_cap,
                                                  R->qb_count, R->status_step);
        eul_count_kernel<<<(unsigned)ceil_div(B, TB), TB, 0, st>>>(B, R->qb_count, R->qb_cap, LD,
                                                                   R->q_count);
        if (d == 2)
            eul_init_kernel<2><<<gq, TB, 0, st>>>(g, R->q_cap, R->q_count, R->qbase, R->qb_cap, L,
                                                  LD, R->XQ);
        else
            eul_init_kernel<3><<<gq, TB, 0, st>>>(g, R->q_cap, R->q_count, R->qbase, R->qb_cap, L,
                                                  LD, R->XQ);
        MR_LAUNCH_CHECK();
        const int64_t xstr = (int64_t)d * R->q_cap;
        // the first step takes the displacement guess X = x - u(x) (positions
        // only, Jacobian replaced by I); later steps are Newton steps
        for (int it = 0; it < R->newton_iters; ++it) {
            rc = decode_jac_ex(R->dec, B, R->q_cap, R->XQ, R->q_cap, nullptr, 0, R->q_count, xhat,
                               nullptr, R->xQ, it == 0 ? nullptr : R->FQ, nullptr, nullptr, st, 0,
                               xstr);
            if (rc != MR_OK) return rc;
            const float *Fit = it == 0 ? nullptr : R->FQ;
            if (d == 2)
                eul_newton_kernel<2><<<gq, TB, 0, st>>>(g, R->q_cap, R->q_count, R->qbase, R->qb_cap,
                                                        L, LD, R->xQ, Fit, R->XQ);
            else
                eul_newton_kernel<3><<<gq, TB, 0, st>>>(g, R->q_cap, R->q_count, R->qbase, R->qb_cap,
                                                        L, LD, R->xQ, Fit, R->XQ);
            MR_LAUNCH_CHECK();
        }
        rc = decode_jac_ex(R->dec, B, R->q_cap, R->XQ, R->q_cap, nullptr, 0, R->q_count, xhat,
                           vhat, R->xQ, R->FQ, R->vQ, nullptr, st, 0, xstr);
        if (rc != MR_OK) return rc;
        const double hq = (double)g.dx / L;
        const float rho0_vq = (float)(R->cfg.rho0 * (d == 3 ? hq * hq * hq : hq * hq));
        // a bf16 decoder's positions carry about 2^-8 of its output scale
        // (the inversion residual stalls there: 0.01-0.05 cells measured), so
        // the acceptance test allows four times that
        float tol = R->newton_tol * g.dx;
        if (decoder_precision(R->dec) == MR_PREC_BF16)
            tol = fmaxf(tol, 4.0f * 0.00390625f * decoder_out_scale(R->dec));
        if (d == 2)
            eul_finish_kernel<2><<<gq, TB, 0, st>>>(g, R->q_cap, R->q_count, R->qbase, R->qb_cap, L,
                                                    LD, R->XQ, R->xQ, R->FQ, R->rho, R->rn[0],
                                                    R->rn[1], R->rn[2], rho0_vq, inv_rho0, tol,
                                                    R->mQ);
        else
            eul_finish_kernel<3><<<gq, TB, 0, st>>>(g, R->q_cap, R->q_count, R->qbase, R->qb_cap, L,
                                                    LD, R->XQ, R->xQ, R->FQ, R->rho, R->rn[0],
                                                    R->rn[1], R->rn[2], rho0_vq, inv_rho0, tol,
                                                    R->mQ);
        MR_LAUNCH_CHECK();
    } else {
    // Algorithm 3: decode every particle, mark I, collect Q
    rc = rom_decode(R->dec, B, R->P, R->X, R->P, nullptr, xhat, R->x_all, st);
    if (rc != MR_OK) return rc;
    const dim3 gp((unsigned)ceil_div(R->P, TB), (unsigned)B);
    if (R->fields_on)
        field_positions_kernel<<<gp, TB, 0, st>>>(d, R->P, R->counter, dt, R->fa, R->fb, R->x_all);
    if (d == 2)
        gather_mark_kernel<2><<<gs, TB, 0, st>>>(g, R->P, (int)R->ns_max, R->n_samples, R->samples,
                                                 R->x_all, R->xs, R->bitmap, R->words, R->status_step);
    else
        gather_mark_kernel<3><<<gs, TB, 0, st>>>(g, R->P, (int)R->ns_max, R->n_samples, R->samples,
                                                 R->x_all, R->xs, R->bitmap, R->words, R->status_step);
    dim3 gn((unsigned)ceil_div(R->P, NB_BLOCK), (unsigned)B);
    if (d == 2)
        neighbour_kernel<2><<<gn, NB_BLOCK, 0, st>>>(g, R->P, R->words, R->x_all, R->bitmap, R->Q,
                                                     R->q_cap, R->q_count, R->status_step);
    else
        neighbour_kernel<3><<<gn, NB_BLOCK, 0, st>>>(g, R->P, R->words, R->x_all, R->bitmap, R->Q,
                                                     R->q_cap, R->q_count, R->status_step);
    clamp_count_kernel<<<(unsigned)ceil_div(B, TB), TB, 0, st>>>(B, R->q_count, R->q_cap);
    MR_LAUNCH_CHECK();
    // quadrature kinematics (Algorithm 3, step 4)
    rc = decode_jac_ex(R->dec, B, R->P, R->X, R->q_cap, R->Q, 1, R->q_count, xhat, vhat, R->xQ,
                       R->FQ, R->vQ, nullptr, st);
    if (rc != MR_OK) return rc;
    if (R->fields_on)
        field_quad_kernel<<<gq, TB, 0, st>>>(d, R->P, R->q_cap, R->q_count, R->Q, R->counter, dt,
                                             R->fa, R->fb, R->fGa, R->fGb, R->xQ, R->FQ, R->vQ);
    }
    // Algorithm 5
    const bool eul = R->quad == MR_QUAD_EULERIAN;
    if (d == 2)
        p2g_quad_kernel<2><<<gq, TB, 0, st>>>(g, R->q_cap, R->words, R->q_count, R->Q, R->xQ, R->FQ,
                                              R->vQ, R->m, eul ? R->mQ : nullptr, R->cfg.m_uniform,
                                              inv_rho0, R->E, R->cfg.nu, R->cfg.model, (float)dt,
                                              R->bitmap, R->grid, R->nodes, R->status_step);
    else
        p2g_quad_kernel<3><<<gq, TB, 0, st>>>(g, R->q_cap, R->words, R->q_count, R->Q, R->xQ, R->FQ,
                                              R->vQ, R->m, eul ? R->mQ : nullptr, R->cfg.m_uniform,
                                              inv_rho0, R->E, R->cfg.nu, R->cfg.model, (float)dt,
                                              R->bitmap, R->grid, R->nodes, R->status_step);
    if (d == 2)
        g2p_trial_kernel<2><<<gs, TB, 0, st>>>(g, (int)R->ns_max, R->n_samples, R->xs, R->grid,
                                               R->nodes, (float)dt, R->xt, R->vt);
    else
        g2p_trial_kernel<3><<<gs, TB, 0, st>>>(g, (int)R->ns_max, R->n_samples, R->xs, R->grid,
                                               R->nodes, (float)dt, R->xt, R->vt);
    {
        const int64_t per = std::min<int64_t>(ceil_div(R->words, TB), 256);
        clear_marked_kernel<<<dim3((unsigned)per, (unsigned)B), TB, 0, st>>>(
            R->words, R->nodes, R->bitmap, R->qb_bitmap, reinterpret_cast<float4 *>(R->grid),
            R->n_active);
    }
    MR_LAUNCH_CHECK();
    if (R->fields_on)
        field_velocity_kernel<<<gs, TB, 0, st>>>(d, R->P, (int)R->ns_max, R->n_samples, R->samples,
                                                 R->fb, R->vt);
    // Algorithm 6 / 7
    ProjWS w = proj_ws_carve(R->proj_ws, d, r, B, R->ns_max, R->opts.max_backtrack);
    rc = project_impl(R->dec, d, r, B, R->P, R->X, R->ns_max, R->samples, R->n_samples, nullptr,
                      R->vt, xhat, xhat_prev, dt, R->opts, R->z_next, R->v_next, nullptr, nullptr,
                      R->status_step, w, st, /*accumulate=*/1);
    if (rc != MR_OK) return rc;
    advance_kernel<<<(unsigned)ceil_div((int64_t)B * r, TB), TB, 0, st>>>(
        B, r, xhat, xhat_prev, vhat, R->z_next, R->v_next, R->status_step, status_out, R->counter);
    MR_LAUNCH_CHECK();
    R->dirty = 0;
    return MR_OK;
}

}  // namespace mr

using namespace mr;

extern "C" void rom_destroy(mr_rom *R)
{
    if (!R) return;
    void *bufs[] = {R->X, R->m, R->E, R->internal_of, R->n_samples, R->samples, R->x_all,
                    R->bitmap, R->Q,
                    R->q_count, R->n_active, R->xQ, R->FQ, R->vQ, R->grid, R->xs, R->xt, R->vt,
                    R->z_next, R->v_next, R->status_step, R->counter, R->proj_ws,
                    R->qb_bitmap, R->qbase, R->qb_count, R->XQ, R->mQ, R->rho,
                    R->fa, R->fb, R->fGa, R->fGb};
    for (void *p : bufs)
        if (p) (void)hipFree(p);
    if (R->graph) (void)hipGraphExecDestroy(R->graph);
    if (R->cap_stream) (void)hipStreamDestroy(R->cap_stream);
    free(R);
}

extern "C" int32_t rom_create(const mr_decoder *dec, const mr_grid *grid_desc,
                              const mr_rom_config *cfg, const float *X_all, const float *m_all,
                              const float *E, const int32_t *n_samples, const mr_gn_opts *opts,
                              mr_rom **out)
{
    GridK g;
    if (!dec || !out || !cfg || !X_all || !E || !n_samples || !opts_ok(opts) ||
        !grid_from_desc(grid_desc, g))
        return MR_EINVAL;
    int d = decoder_dim(dec), r = decoder_latent(dec);
    if (d != grid_desc->dim || cfg->B < 1 || cfg->B > 65535 || cfg->n_particles < 1 ||
        cfg->n_particles > INT32_MAX || cfg->n_samples_max < 1 ||
        cfg->n_samples_max > cfg->n_particles || !(cfg->rho0 > 0.0f))
        return MR_EINVAL;
    if ((int64_t)cfg->B * (opts->max_backtrack + 1) > 65535) return MR_EINVAL;
    if (cfg->quadrature != MR_QUAD_LAGRANGIAN && cfg->quadrature != MR_QUAD_EULERIAN)
        return MR_EINVAL;
    const int ell = cfg->quad_per_dim == 0 ? 2 : cfg->quad_per_dim;
    const int newton_iters = cfg->newton_iters == 0 ? 2 : cfg->newton_iters;
    const float newton_tol = cfg->newton_tol == 0.0f ? 1e-3f : cfg->newton_tol;
    if (cfg->quadrature == MR_QUAD_EULERIAN &&
        ((ell != 2 && ell != 4) || newton_iters < 1 || newton_iters > 16 ||
         !(newton_tol > 0.0f) || !(newton_tol < 1.0f)))
        return MR_EINVAL;
    mr_rom *R = (mr_rom *)calloc(1, sizeof(mr_rom));
    if (!R) return MR_ENOMEM;
    R->dec = dec;
    R->d = d;
    R->r = r;
    R->g = g;
    R->cfg = *cfg;
    R->opts = *opts;
    R->B = cfg->B;
    R->P = cfg->n_particles;
    R->ns_max = cfg->n_samples_max;
    R->nodes = grid_nodes(g);
    R->words = ceil_div(R->nodes, 32);
    R->quad = cfg->quadrature;
    R->ell = ell;
    R->newton_iters = newton_iters;
    R->newton_tol = newton_tol;
    const bool eul = R->quad == MR_QUAD_EULERIAN;
    // reference positions on the host: the stencil base cell of every
    // particle orders the runner's particles (below) and gives the densest
    // cell, which bounds the quadrature list
    const int64_t Pn = cfg->n_particles;
    std::vector<float> Xh((size_t)d * Pn);
    std::vector<int64_t> key(Pn);
    if (hipMemcpy(Xh.data(), X_all, 4 * d * Pn, hipMemcpyDeviceToHost) != hipSuccess) {
        free(R);
        return MR_EDEVICE;
    }
    int64_t ppc_max = 0;
    {
        const int nn[3] = {g.n0, g.n1, g.n2};
        std::vector<int32_t> per_cell(R->nodes, 0);
        for (int64_t p = 0; p < Pn; ++p) {
            int64_t kk = 0;
            for (int a = d - 1; a >= 0; --a) {
                float bf = floorf(Xh[(size_t)a * Pn + p] * g.inv_dx - 0.5f);
                int64_t bi = bf < 0.0f ? 0 : (bf > (float)(nn[a] - 1) ? nn[a] - 1 : (int64_t)bf);
                kk = kk * nn[a] + bi;
            }
            key[p] = kk;
            const int32_t c = ++per_cell[kk];
            if (c > ppc_max) ppc_max = c;
        }
    }
    // quadrature capacity: every sample's 3^d nodes are reached from a
    // (5 cells)^d box of stencil bases; Lagrangian: twice the densest
    // reference cell's particles per base cell (at least 16), room for
    // compression; Eulerian: every base of the box, l^d points each
    const int64_t box = (d == 3) ? 125 : 25;
    if (eul) {
        R->qb_cap = R->ns_max * box < R->nodes ? R->ns_max * box : R->nodes;
        R->q_cap = R->qb_cap * (d == 3 ? ell * ell * ell : ell * ell);
    } else {
        const int64_t per = box * (2 * ppc_max > 16 ? 2 * ppc_max : 16);
        R->q_cap = R->ns_max * per < R->P ? R->ns_max * per : R->P;
    }
    if (R->q_cap > INT32_MAX) {
        free(R);
        return MR_EINVAL;
    }
    const int64_t B = R->B, P = R->P;
    bool ok = true;
    auto alloc = [&](void **p, int64_t bytes) {
        if (ok && hipMalloc(p, bytes > 0 ? bytes : 4) != hipSuccess) ok = false;
    };
    alloc((void **)&R->X, 4 * d * P);
    alloc((void **)&R->internal_of, 4 * P);
    if (m_all) alloc((void **)&R->m, 4 * P);
    alloc((void **)&R->E, 4 * B);
    alloc((void **)&R->n_samples, 4 * B);
    alloc((void **)&R->samples, 4 * B * R->ns_max);
    if (!eul) {
        alloc((void **)&R->x_all, 4 * B * d * P);
        alloc((void **)&R->Q, 4 * B * R->q_cap);
    } else {
        alloc((void **)&R->qb_bitmap, 4 * B * R->words);
        alloc((void **)&R->qbase, 4 * B * R->qb_cap);
        alloc((void **)&R->qb_count, 4 * B);
        alloc((void **)&R->XQ, 4 * B * d * R->q_cap);
        alloc((void **)&R->mQ, 4 * B * R->q_cap);
        R->rn[0] = g.n0;
        R->rn[1] = g.n1;
        R->rn[2] = d == 3 ? g.n2 : 1;
        alloc((void **)&R->rho, 4 * (int64_t)R->rn[0] * R->rn[1] * R->rn[2]);
    }
    alloc((void **)&R->bitmap, 4 * B * R->words);
    alloc((void **)&R->q_count, 4 * B);
    alloc((void **)&R->n_active, 4 * B);
    alloc((void **)&R->xQ, 4 * B * d * R->q_cap);
    alloc((void **)&R->FQ, 4 * B * d * d * R->q_cap);
    alloc((void **)&R->vQ, 4 * B * d * R->q_cap);
    alloc((void **)&R->grid, 16 * B * R->nodes);
    alloc((void **)&R->xs, 4 * B * d * R->ns_max);
    alloc((void **)&R->xt, 4 * B * d * R->ns_max);
    alloc((void **)&R->vt, 4 * B * d * R->ns_max);
    alloc((void **)&R->z_next, 8 * B * r);
    alloc((void **)&R->v_next, 8 * B * r);
    alloc((void **)&R->status_step, 4 * B);
    alloc((void **)&R->counter, 8);
    alloc(&R->proj_ws, proj_ws_bytes(d, r, (int)B, R->ns_max, opts->max_backtrack));
    if (!ok) {
        rom_destroy(R);
        return MR_ENOMEM;
    }
    std::vector<int32_t> ns_host(B);
    if (hipMemcpy(ns_host.data(), n_samples, 4 * B, hipMemcpyDeviceToHost) != hipSuccess) {
        rom_destroy(R);
        return MR_EDEVICE;
    }
    for (int32_t v : ns_host)
        if (v < 1 || v > R->ns_max) {
            rom_destroy(R);
            return MR_EINVAL;
        }
    // The runner keeps the particles sorted by the base cell of their
    // reference position (stable): the quadrature list, collected in this
    // order, then holds runs of particles sharing a stencil, which the
    // quadrature P2G sums within a wave before its atomics.
    std::vector<float> Xs((size_t)d * P), mh, ms;
    std::vector<int32_t> order(P), inv(P);
    bool cp = true;
    if (m_all) {
        mh.resize(P);
        ms.resize(P);
        cp = hipMemcpy(mh.data(), m_all, 4 * P, hipMemcpyDeviceToHost) == hipSuccess;
    }
    if (cp) {
        for (int64_t p = 0; p < P; ++p) order[p] = (int32_t)p;
        std::stable_sort(order.begin(), order.end(),
                         [&](int32_t a, int32_t b) { return key[a] < key[b]; });
        for (int64_t i = 0; i < P; ++i) {
            inv[order[i]] = (int32_t)i;
            for (int a = 0; a < d; ++a) Xs[(size_t)a * P + i] = Xh[(size_t)a * P + order[i]];
            if (m_all) ms[i] = mh[order[i]];
        }
        cp = hipMemcpy(R->X, Xs.data(), 4 * d * P, hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(R->internal_of, inv.data(), 4 * P, hipMemcpyHostToDevice) == hipSuccess &&
             (!m_all || hipMemcpy(R->m, ms.data(), 4 * P, hipMemcpyHostToDevice) == hipSuccess);
        if (cp && eul) {
            // smoothed reference density: every particle's mass spread
            // with the quadratic B-spline over the 3^d grid nodes of its
            // stencil, divided by dx^d
            const double h = (double)g.dx;
            const int64_t nl = (int64_t)R->rn[0] * R->rn[1] * R->rn[2];
            std::vector<double> rho(nl, 0.0);
            const double inv_hd = d == 3 ? 1.0 / (h * h * h) : 1.0 / (h * h);
            for (int64_t p = 0; p < P; ++p) {
                int64_t bse[3] = {0, 0, 0};
                double w[3][3] = {{1, 0, 0}, {1, 0, 0}, {1, 0, 0}};
                bool in = true;
                for (int a = 0; a < d; ++a) {
                    const double t = (double)Xh[(size_t)a * P + p] / h;
                    const double bf = std::floor(t - 0.5);
                    in = in && bf >= 0.0 && bf + 2.0 <= (double)(R->rn[a] - 1);
                    bse[a] = (int64_t)bf;
                    const double f = t - bf;
                    w[a][0] = 0.5 * (1.5 - f) * (1.5 - f);
                    w[a][1] = 0.75 - (f - 1.0) * (f - 1.0);
                    w[a][2] = 0.5 * (f - 0.5) * (f - 0.5);
                }
                if (!in) continue;
                const double mp = (m_all ? (double)mh[p] : (double)cfg->m_uniform) * inv_hd;
                for (int o2 = 0; o2 < (d == 3 ? 3 : 1); ++o2)
                    for (int o1 = 0; o1 < 3; ++o1)
                        for (int o0 = 0; o0 < 3; ++o0) {
                            const int64_t i = (bse[0] + o0) +
                                              (int64_t)R->rn[0] * ((bse[1] + o1) +
                                                                   (int64_t)R->rn[1] * (bse[2] + o2));
                            rho[i] += mp * w[0][o0] * w[1][o1] * (d == 3 ? w[2][o2] : 1.0);
                        }
            }
            std::vector<float> rhof(rho.begin(), rho.end());
            cp = hipMemcpy(R->rho, rhof.data(), 4 * nl, hipMemcpyHostToDevice) == hipSuccess;
        }
    }
    cp = cp && hipMemcpy(R->E, E, 4 * B, hipMemcpyDeviceToDevice) == hipSuccess &&
         hipMemcpy(R->n_samples, n_samples, 4 * B, hipMemcpyDeviceToDevice) == hipSuccess;
    if (!cp || hipStreamCreateWithFlags(&R->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        rom_destroy(R);
        return MR_EDEVICE;
    }
    clear_all(R, R->cap_stream);
    if (hipStreamSynchronize(R->cap_stream) != hipSuccess) {
        rom_destroy(R);
        return MR_EDEVICE;
    }
    if (cfg->autotune) {
        // the four decoder launches of a step: every particle (positions),
        // the quadrature list (x, F, v), the samples (latent Jacobian) and
        // the line-search candidates (positions)
        // (Eulerian: the samples (positions) and the lattice points (x, F, v)
        // instead of every particle)
        const int32_t nc = opts->max_backtrack + 1;
        int32_t rc = decoder_autotune(dec, (int32_t)B, eul ? R->ns_max : P, 1, 3, R->cap_stream);
        if (rc == MR_OK) rc = decoder_autotune(dec, (int32_t)B, R->q_cap, 2, 3, R->cap_stream);
        if (rc == MR_OK) rc = decoder_autotune(dec, (int32_t)B, R->ns_max, 4, 3, R->cap_stream);
        if (rc == MR_OK) rc = decoder_autotune(dec, (int32_t)B * nc, R->ns_max, 1, 3, R->cap_stream);
        if (rc != MR_OK) {
            rom_destroy(R);
            return rc;
        }
    }
    *out = R;
    return MR_OK;
}

extern "C" int32_t rom_step(mr_rom *R, int32_t n_steps, int64_t step0, double dt, double *xhat,
                            double *xhat_prev, double *vhat, int32_t *status_out, int32_t use_graph,
                            void *stream)
{
    if (!R || n_steps < 0 || !xhat || !xhat_prev || !vhat || step0 < 0) return MR_EINVAL;
    hipStream_t st = as_stream(stream);
    if (R->dirty) {
        clear_all(R, st);
        R->dirty = 0;
    }
    set_counter_kernel<<<1, 1, 0, st>>>(R->counter, step0);
    MR_LAUNCH_CHECK();
    if (n_steps == 0) return MR_OK;
    if (!use_graph) {
        for (int32_t s = 0; s < n_steps; ++s) {
            int32_t rc = rom_one_step(R, dt, xhat, xhat_prev, vhat, status_out, st);
            if (rc != MR_OK) return rc;
        }
        return MR_OK;
    }
    bool reuse = R->graph && R->graph_steps == n_steps && R->graph_dt == dt &&
                 R->graph_ptrs[0] == xhat && R->graph_ptrs[1] == xhat_prev &&
                 R->graph_ptrs[2] == vhat && R->graph_status == status_out;
    if (!reuse) {
        if (R->graph) {
            (void)hipGraphExecDestroy(R->graph);
            R->graph = nullptr;
        }
        hipGraph_t graph;
        MR_CHECK_HIP(hipStreamBeginCapture(R->cap_stream, hipStreamCaptureModeThreadLocal));
        int32_t rc = MR_OK;
        for (int32_t s = 0; s < n_steps && rc == MR_OK; ++s)
            rc = rom_one_step(R, dt, xhat, xhat_prev, vhat, status_out, R->cap_stream);
        hipError_t e = hipStreamEndCapture(R->cap_stream, &graph);
        if (rc != MR_OK) return rc;
        if (e != hipSuccess) return MR_EDEVICE;
        e = hipGraphInstantiate(&R->graph, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            R->graph = nullptr;
            return MR_EDEVICE;
        }
        R->graph_steps = n_steps;
        R->graph_dt = dt;
        R->graph_ptrs[0] = xhat;
        R->graph_ptrs[1] = xhat_prev;
        R->graph_ptrs[2] = vhat;
        R->graph_status = status_out;
    }
    MR_CHECK_HIP(hipGraphLaunch(R->graph, st));
    return MR_OK;
}

extern "C" int32_t rom_last_counts(const mr_rom *R, int32_t b, int64_t *n_quad, int64_t *n_active,
                                   void *stream)
{
    if (!R || b < 0 || b >= R->B || !n_quad || !n_active) return MR_EINVAL;
    hipStream_t st = as_stream(stream);
    int32_t q = 0, a = 0;
    MR_CHECK_HIP(hipMemcpyAsync(&q, R->q_count + b, 4, hipMemcpyDeviceToHost, st));
    MR_CHECK_HIP(hipMemcpyAsync(&a, R->n_active + b, 4, hipMemcpyDeviceToHost, st));
    MR_CHECK_HIP(hipStreamSynchronize(st));
    *n_quad = q;
    *n_active = a;
    return MR_OK;
}

extern "C" int32_t rom_set_fields(mr_rom *R, const double *xhat0, const double *vhat0,
                                  const float *v0, void *stream)
{
    if (!R) return MR_EINVAL;
    if (!xhat0) {
        R->fields_on = 0;
        return MR_OK;
    }
    if (!vhat0 || !v0 || R->quad != MR_QUAD_LAGRANGIAN) return MR_EINVAL;
    const int d = R->d, r = R->r, B = R->B;
    const int64_t P = R->P;
    hipStream_t st = as_stream(stream);
    MR_CHECK_HIP(hipStreamSynchronize(st));
    if (!R->fa) {
        bool ok = hipMalloc(&R->fa, 4 * (int64_t)B * d * P) == hipSuccess &&
                  hipMalloc(&R->fb, 4 * (int64_t)B * d * P) == hipSuccess &&
                  hipMalloc(&R->fGa, 4 * (int64_t)B * d * d * P) == hipSuccess &&
                  hipMalloc(&R->fGb, 4 * (int64_t)B * d * d * P) == hipSuccess;
        if (!ok) {
            for (float **q : {&R->fa, &R->fb, &R->fGa, &R->fGb}) {
                if (*q) (void)hipFree(*q);
                *q = nullptr;
            }
            return MR_ENOMEM;
        }
    }
    R->fields_on = 0;
    const int TB = 256;
    float *v0d = nullptr;
    double *lat = nullptr;
    float *Fm = nullptr;
    const int CH = B < 8 ? B : 8;               // instances per difference pass
    int32_t rc = MR_OK;
    if (hipMalloc(&v0d, 4 * (int64_t)B * d) != hipSuccess ||
        hipMalloc(&lat, 8 * ((int64_t)2 * B * r + B)) != hipSuccess ||
        hipMalloc(&Fm, 4 * (int64_t)CH * d * d * P) != hipSuccess)
        rc = MR_ENOMEM;
    if (rc == MR_OK && hipMemcpyAsync(v0d, v0, 4 * (int64_t)B * d, hipMemcpyDefault, st) != hipSuccess)
        rc = MR_EDEVICE;
    // a, b, grad a from x, v, F at xhat0 (fp32 decodes)
    if (rc == MR_OK)
        rc = decode_jac_ex(R->dec, B, P, R->X, P, nullptr, 0, nullptr, xhat0, vhat0, R->fa, R->fGa,
                           R->fb, nullptr, st, 0, 0, 1);
    if (rc == MR_OK) {
        field_init_kernel<<<dim3((unsigned)ceil_div(P, TB), (unsigned)B), TB, 0, st>>>(
            d, P, R->X, v0d, R->fa, R->fb, R->fGa);
        // grad b by a central difference of dg/dX along vhat0: a latent step
        // of 1e-2 (max norm) keeps the truncation error near 1e-4 of grad b
        // and the fp32 rounding of the difference near 1e-4 as well
        double *zp = lat, *zm = lat + (int64_t)B * r, *inv2e = lat + (int64_t)2 * B * r;
        field_fd_latents_kernel<<<(unsigned)ceil_div(B, 64), 64, 0, st>>>(B, r, 1e-2, xhat0, vhat0,
                                                                           zp, zm, inv2e);
        if (hipGetLastError() != hipSuccess) rc = MR_EDEVICE;
        for (int b0 = 0; b0 < B && rc == MR_OK; b0 += CH) {
            const int nb = B - b0 < CH ? B - b0 : CH;
            float *Fp = R->fGb + (int64_t)b0 * d * d * P;
            rc = decode_jac_ex(R->dec, nb, P, R->X, P, nullptr, 0, nullptr, zp + (int64_t)b0 * r,
                               nullptr, nullptr, Fp, nullptr, nullptr, st, 0, 0, 1);
            if (rc == MR_OK)
                rc = decode_jac_ex(R->dec, nb, P, R->X, P, nullptr, 0, nullptr,
                                   zm + (int64_t)b0 * r, nullptr, nullptr, Fm, nullptr, nullptr, st,
                                   0, 0, 1);
            if (rc == MR_OK)
                field_grad_b_kernel<<<dim3((unsigned)ceil_div(P, TB), (unsigned)nb), TB, 0, st>>>(
                    d, P, b0, inv2e, Fp, Fm);
        }
    }
    if (rc == MR_OK && (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess))
        rc = MR_EDEVICE;
    if (v0d) (void)hipFree(v0d);
    if (lat) (void)hipFree(lat);
    if (Fm) (void)hipFree(Fm);
    if (rc == MR_OK) R->fields_on = 1;
    return rc;
}

extern "C" int32_t rom_positions(const mr_rom *R, const double *xhat, double t, float *x_out,
                                 void *stream)
{
    if (!R || !xhat || !x_out) return MR_EINVAL;
    hipStream_t st = as_stream(stream);
    // row p of the output is the caller's particle p, the runner's internal_of[p]
    int32_t rc = decode_jac_ex(R->dec, R->B, R->P, R->X, R->P, R->internal_of, 0, nullptr, xhat,
                               nullptr, x_out, nullptr, nullptr, nullptr, st);
    if (rc != MR_OK || !R->fields_on) return rc;
    field_caller_positions_kernel<<<dim3((unsigned)ceil_div(R->P, 256), (unsigned)R->B), 256, 0,
                                    st>>>(R->d, R->P, R->internal_of, (float)t, R->fa, R->fb,
                                          x_out);
    MR_LAUNCH_CHECK();
    return MR_OK;
}
