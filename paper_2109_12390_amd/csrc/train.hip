// Decoder training on gfx950 (paper Section 4.2, loss function; Appendix B,
// training details): forward pass with tangent streams, loss and its
// gradient, backward pass through the tangents (second derivatives of ELU),
// and Adam.
//
// A batch holds n_groups snapshots x rows_per_group particles; the rows of a
// group share the snapshot's latent code z_s and the velocity direction
// u_s = (z_{s+1} - z_s) / dt.  Every row carries S = d + 2 columns (streams):
// the primal, the d spatial tangents (for dg/dX) and the tangent along u_s
// (for (dg/dz) u_s).  Column c = row * S + stream.  Activations are stored
// column-major ([column][unit], unit contiguous) for the backward pass.
//
// Every dense product is one launch of a tiled matrix-core GEMM
// (64 x 64 block tile, 16x16 MFMA tiles, bf16 operands with fp32
// accumulation or fp32 operands) with arbitrary element strides, so the
// transposed products of the backward pass need no transposed copies; the
// weight gradients reduce over the batch columns with split-K and fp32
// atomics.  Element-wise work (activations, loss, latent gradients, Adam)
// runs in fp32 vector kernels.
#include "internal.h"

#include <stdlib.h>
#include <string.h>

#include <type_traits>

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

namespace mr {

__device__ __forceinline__ uint16_t to_bf16(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

struct GemmArgs {
    int M, N, K;
    const float *A;
    int64_t sam, sak;
    const float *B;
    int64_t sbk, sbn;
    float *C;
    int64_t scm, scn;
    int mode;     // 0: C = AB, 1: C += AB, 2: atomicAdd(C, AB)
    int k_chunk;  // K range per blockIdx.z
    int64_t scz;  // C offset per blockIdx.z (split-K slices; 0: one C)
};

constexpr int GBM = 64, GBN = 64, GBK = 32;

// Stages the 64 x GBK tile of an operand whose element (r, k) sits at
// P[r * sr + k * sk] into S[r][k] (as T); rows at or past rmax and k at or
// past ke read as zero.  The unit-stride dimension runs across consecutive
// threads.  VEC: that dimension is read four elements at a time (its
// extent and the other stride are multiples of 4 and P is 16-byte
// aligned, so a group of four is either all in range or all out).
template <typename T, int LDK, bool VEC>
__device__ __forceinline__ void stage_tile(T (*S)[LDK], const float *P, int64_t sr, int64_t sk,
                                           int r0, int rmax, int k0, int ke, int tid)
{
    constexpr int R = 64;
    if constexpr (VEC) {
#pragma unroll
        for (int e = 0; e < (R * GBK / 4) / 256; ++e) {
            const int idx = e * 256 + tid;
            if (sk == 1) {
                const int rr = idx / (GBK / 4), kk = (idx % (GBK / 4)) * 4;
                const int gr = r0 + rr, gk = k0 + kk;
                float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                if (gr < rmax && gk < ke) v = *reinterpret_cast<const float4 *>(P + (int64_t)gr * sr + gk);
                if constexpr (sizeof(T) == 2) {
                    uint2 w;
                    w.x = (uint32_t)to_bf16(v.x) | ((uint32_t)to_bf16(v.y) << 16);
                    w.y = (uint32_t)to_bf16(v.z) | ((uint32_t)to_bf16(v.w) << 16);
                    *reinterpret_cast<uint2 *>(&S[rr][kk]) = w;
                } else {
                    *reinterpret_cast<float4 *>(&S[rr][kk]) = v;
                }
            } else {
                const int kk = idx / (R / 4), rr = (idx % (R / 4)) * 4;
                const int gr = r0 + rr, gk = k0 + kk;
                float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                if (gr < rmax && gk < ke) v = *reinterpret_cast<const float4 *>(P + (int64_t)gk * sk + gr);
                const float c[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    if constexpr (sizeof(T) == 2)
                        S[rr + i][kk] = to_bf16(c[i]);
                    else
                        S[rr + i][kk] = c[i];
                }
            }
        }
    } else {
#pragma unroll
        for (int e = 0; e < (R * GBK) / 256; ++e) {
            const int idx = e * 256 + tid;
            int rr, kk;
            if (sk == 1) {
                rr = idx / GBK;
                kk = idx % GBK;
            } else {
                kk = idx / R;
                rr = idx % R;
            }
            const int gr = r0 + rr, gk = k0 + kk;
            const float v = (gr < rmax && gk < ke) ? P[(int64_t)gr * sr + (int64_t)gk * sk] : 0.0f;
            if constexpr (sizeof(T) == 2)
                S[rr][kk] = to_bf16(v);
            else
                S[rr][kk] = v;
        }
    }
}

// C(m, n) = sum_k A(m, k) B(k, n); block tile 64 x 64, four waves of 32 x 32
template <bool BF16, bool VA, bool VB>
__global__ void __launch_bounds__(256) gemm_kernel(GemmArgs g)
{
    constexpr int PAD = BF16 ? 8 : 4;
    constexpr int LDK = GBK + PAD;
    using T = typename std::conditional<BF16, uint16_t, float>::type;
    __shared__ __align__(16) T As[GBM][LDK];
    __shared__ __align__(16) T Bs[GBN][LDK];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.x * GBM, n0 = blockIdx.y * GBN;
    const int kb = blockIdx.z * g.k_chunk;
    const int ke = min(g.K, kb + g.k_chunk);
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int j = lane & 15, q4 = lane >> 4;
    f32x4_t acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = kb; k0 < ke; k0 += GBK) {
        // A (64 x 32) as A(m, k); B (32 x 64) as its transpose B(n, k)
        stage_tile<T, LDK, VA>(As, g.A, g.sam, g.sak, m0, g.M, k0, ke, tid);
        stage_tile<T, LDK, VB>(Bs, g.B, g.sbn, g.sbk, n0, g.N, k0, ke, tid);
        __syncthreads();
        if constexpr (BF16) {
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                bf16x8_t fa = *reinterpret_cast<const bf16x8_t *>(&As[wm + a * 16 + j][8 * q4]);
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    bf16x8_t fb = *reinterpret_cast<const bf16x8_t *>(&Bs[wn + b * 16 + j][8 * q4]);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb, acc[a][b], 0, 0, 0);
                }
            }
        } else {
#pragma unroll
            for (int ks = 0; ks < GBK; ks += 4)
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                            As[wm + a * 16 + j][ks + q4], Bs[wn + b * 16 + j][ks + q4], acc[a][b],
                            0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                int gm = m0 + wm + a * 16 + 4 * q4 + q;
                int gn = n0 + wn + b * 16 + j;
                if (gm >= g.M || gn >= g.N) continue;
                float *c = g.C + (int64_t)blockIdx.z * g.scz + (int64_t)gm * g.scm +
                           (int64_t)gn * g.scn;
                float v = acc[a][b][q];
                if (g.mode == 0)
                    *c = v;
                else if (g.mode == 1)
                    *c += v;
                else
                    atomicAdd(c, v);
            }
}

// whether an operand with element (r, k) at P[r * sr + k * sk], r < R and
// k < K, can be staged four elements at a time along its unit stride
static bool vec_ok(const float *P, int64_t sr, int64_t sk, int R, int K)
{
    if ((uintptr_t)P % 16 != 0) return false;
    if (sk == 1) return K % 4 == 0 && sr % 4 == 0;
    if (sr == 1) return R % 4 == 0 && sk % 4 == 0;
    return false;
}

// sums the split-K slices stage[z][m][n] (z = 0 .. splits - 1, in order)
// into C: C[m][n] += sum_z stage[z][m][n]
__global__ void split_reduce_kernel(int M, int N, int splits, const float *stage, float *C,
                                    int64_t scm, int64_t scn)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)M * N) return;
    float s = 0.0f;
    for (int z = 0; z < splits; ++z) s += stage[(int64_t)z * M * N + i];
    const int64_t m = i / N, n = i % N;
    C[m * scm + n * scn] += s;
}

// splits < 0: split the k range (a batch reduction, accumulated with
// atomics) so that about 1,024 blocks run, each over at least 256 k.
// stage (nullable): a buffer of at least 1024 x 64 x 64 floats; the split
// results then go to separate slices summed in slice order afterwards (no
// atomics: reproducible), instead of being added with atomics.
int32_t gemm(bool bf16, GemmArgs g, hipStream_t st, int splits = 1, float *stage = nullptr)
{
    if (g.M <= 0 || g.N <= 0) return MR_OK;
    if (g.K <= 0) return MR_OK;
    if (splits < 0) {
        const int64_t tiles = ceil_div(g.M, GBM) * ceil_div(g.N, GBN);
        const int64_t by_blocks = 1024 / tiles, by_k = g.K / 256;
        splits = (int)(by_blocks < by_k ? by_blocks : by_k);
    }
    if (splits < 1) splits = 1;
    int chunk = (int)ceil_div(ceil_div(g.K, splits), GBK) * GBK;
    splits = (int)ceil_div(g.K, chunk);
    g.k_chunk = chunk;
    float *C = g.C;
    const int64_t scm = g.scm, scn = g.scn;
    const bool staged = stage && splits > 1 && g.mode == 2;
    if (staged) {
        // slice z of C at stage + z M N (row-major); the kernel addresses
        // C + m scm + n scn, so the slice index rides on the z stride below
        g.C = stage;
        g.scm = g.N;
        g.scn = 1;
        g.scz = (int64_t)g.M * g.N;
        g.mode = 0;
    } else if (splits > 1) {
        g.mode = 2;
    }
    dim3 grid((unsigned)ceil_div(g.M, GBM), (unsigned)ceil_div(g.N, GBN), (unsigned)splits);
    const bool va = vec_ok(g.A, g.sam, g.sak, g.M, g.K);
    const bool vb = vec_ok(g.B, g.sbn, g.sbk, g.N, g.K);
    auto kern = bf16 ? (va ? (vb ? gemm_kernel<true, true, true> : gemm_kernel<true, true, false>)
                           : (vb ? gemm_kernel<true, false, true> : gemm_kernel<true, false, false>))
                     : (va ? (vb ? gemm_kernel<false, true, true> : gemm_kernel<false, true, false>)
                           : (vb ? gemm_kernel<false, false, true> : gemm_kernel<false, false, false>));
    kern<<<grid, 256, 0, st>>>(g);
    MR_LAUNCH_CHECK();
    if (staged) {
        const int64_t mn = (int64_t)g.M * g.N;
        split_reduce_kernel<<<(unsigned)ceil_div(mn, 256), 256, 0, st>>>(g.M, g.N, splits, stage, C,
                                                                         scm, scn);
        MR_LAUNCH_CHECK();
    }
    return MR_OK;
}

__device__ __forceinline__ float elu(float z) { return z > 0.0f ? z : expm1f(z); }
__device__ __forceinline__ float elu_d(float z) { return z > 0.0f ? 1.0f : expf(z); }
__device__ __forceinline__ float elu_dd(float z) { return z > 0.0f ? 0.0f : expf(z); }

struct TrainDims {
    int d, r, W, nh, S, K0, mode;
    float scale[3], shift[3], mean[3], stdv[3];
};

// input columns [Xn, z] / seeds of the tangent streams
__global__ void build_input_kernel(TrainDims td, int64_t rows, int rows_per_group, const float *X,
                                   const float *Z, const int32_t *snap, const int32_t *next,
                                   float inv_dt, float *A0)
{
    const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= rows * td.S) return;
    const int64_t row = col / td.S;
    const int st = (int)(col % td.S);
    const int grp = (int)(row / rows_per_group);
    const int s = snap[grp], nx = next[grp];
    float *a = A0 + col * td.K0;
    for (int k = 0; k < td.K0; ++k) a[k] = 0.0f;
    if (st == 0) {
        for (int c = 0; c < td.d; ++c) a[c] = X[row * td.d + c] * td.scale[c] + td.shift[c];
        for (int k = 0; k < td.r; ++k) a[td.d + k] = Z[(int64_t)s * td.r + k];
    } else if (st <= td.d) {
        a[st - 1] = td.scale[st - 1];
    } else if (nx >= 0) {
        for (int k = 0; k < td.r; ++k)
            a[td.d + k] = (Z[(int64_t)nx * td.r + k] - Z[(int64_t)s * td.r + k]) * inv_dt;
    }
}

// P (pre-activations, [col][W]) -> add the bias to primal columns, write the
// post-activations and the activated tangents
__global__ void activate_kernel(TrainDims td, int64_t rows, float *P, const float *bias, float *A)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * td.W) return;
    const int64_t row = t / td.W;
    const int i = (int)(t % td.W);
    const int64_t c0 = row * td.S;
    float p = P[c0 * td.W + i] + bias[i];
    P[c0 * td.W + i] = p;
    A[c0 * td.W + i] = elu(p);
    const float e = elu_d(p);
    for (int st = 1; st < td.S; ++st) A[(c0 + st) * td.W + i] = e * P[(c0 + st) * td.W + i];
}

__global__ void output_kernel(TrainDims td, int64_t rows, const float *X, const float *Y,
                              const float *bL, float *g, float *G, float *Gv)
{
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= rows) return;
    const int d = td.d;
    const int64_t c0 = row * td.S;
    for (int a = 0; a < d; ++a) {
        float val = td.mean[a] + td.stdv[a] * (Y[c0 * d + a] + bL[a]);
        if (td.mode == MR_OUT_DISPLACEMENT) val += X[row * d + a];
        g[row * d + a] = val;
        for (int b = 0; b < d; ++b)
            G[(row * d + a) * d + b] = td.stdv[a] * Y[(c0 + 1 + b) * d + a] +
                                       ((td.mode == MR_OUT_DISPLACEMENT && a == b) ? 1.0f : 0.0f);
        Gv[row * d + a] = td.stdv[a] * Y[(c0 + d + 1) * d + a];
    }
}

// adjoints of the last-layer outputs from the upstream gradients; bias grad
__global__ void output_adjoint_kernel(TrainDims td, int64_t rows, const float *dg, const float *dG,
                                      const float *dGv, float *Ybar, float *dbL)
{
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= rows) return;
    const int d = td.d;
    const int64_t c0 = row * td.S;
    for (int a = 0; a < d; ++a) {
        float yb = td.stdv[a] * dg[row * d + a];
        Ybar[c0 * d + a] = yb;
        if (dbL) atomicAdd(dbL + a, yb);
        for (int b = 0; b < d; ++b) Ybar[(c0 + 1 + b) * d + a] = td.stdv[a] * dG[(row * d + a) * d + b];
        Ybar[(c0 + d + 1) * d + a] = td.stdv[a] * dGv[row * d + a];
    }
}

// reproducible output-bias gradient: dbL[a] += sum over rows, in row order
// per thread and a fixed tree across the block (one block per component)
__global__ void __launch_bounds__(256) output_bias_kernel(TrainDims td, int64_t rows,
                                                          const float *Ybar, float *dbL)
{
    __shared__ float red[256];
    const int a = blockIdx.x;
    float s = 0.0f;
    for (int64_t row = threadIdx.x; row < rows; row += 256) s += Ybar[row * td.S * td.d + a];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) dbL[a] += red[0];
}

// db[u] += sum over the slots of part[slot][u]: one block per unit, thread t
// sums slots t, t + 256, ... in order, then a fixed tree (reproducible)
__global__ void __launch_bounds__(256) slot_reduce_kernel(int W, int64_t nslots,
                                                          const float *part, float *db)
{
    __shared__ float red[256];
    const int u = blockIdx.x;
    float s = 0.0f;
    for (int64_t k = threadIdx.x; k < nslots; k += 256) s += part[k * W + u];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) db[u] += red[0];
}

// adjoint of the pre-activations of a hidden layer:
//   primal: Pbar = e Abar + sum_t e' Pdot_t Abar_t ;  tangent t: Pbar_t = e Abar_t
// with e = ELU'(p), e' = ELU''(p); the bias gradient sums the primal Pbar
// For width W <= 256 a thread keeps one unit i (256 / W rows per pass,
// leftover lanes idle) and strides over rows, summing its bias gradient
// locally: one atomic per thread instead of one per row (all rows of a
// layer add into the same W addresses).  Wider layers: threads stride over
// units, the block over rows.
__device__ __forceinline__ float activate_backward_row(const TrainDims &td, int64_t row, int i,
                                                       const float *P, const float *Abar,
                                                       float *Pbar)
{
    const int64_t c0 = row * td.S;
    const float p = P[c0 * td.W + i];
    const float e = elu_d(p), e2 = elu_dd(p);
    float pb = e * Abar[c0 * td.W + i];
    for (int st = 1; st < td.S; ++st) {
        const float ab = Abar[(c0 + st) * td.W + i];
        pb += e2 * P[(c0 + st) * td.W + i] * ab;
        Pbar[(c0 + st) * td.W + i] = e * ab;
    }
    Pbar[c0 * td.W + i] = pb;
    return pb;
}

// part (nullable): the bias-gradient partial sums go to part[slot][unit]
// (W <= 256: slot = block x rows per pass + row lane; wider: slot = block)
// for slot_reduce_kernel, instead of atomics
__global__ void __launch_bounds__(256) activate_backward_kernel(TrainDims td, int64_t rows,
                                                                const float *P, const float *Abar,
                                                                float *Pbar, float *db, float *part)
{
    if (td.W <= 256) {
        const int rpp = 256 / td.W;
        if ((int)threadIdx.x >= rpp * td.W) return;      // no barriers below
        const int i = (int)(threadIdx.x % td.W);
        const int64_t r0 = (int64_t)blockIdx.x * rpp + threadIdx.x / td.W;
        const int64_t stride = (int64_t)gridDim.x * rpp;
        float bsum = 0.0f;
        for (int64_t row = r0; row < rows; row += stride)
            bsum += activate_backward_row(td, row, i, P, Abar, Pbar);
        if (part)
            part[r0 * td.W + i] = bsum;
        else if (r0 < rows)
            atomicAdd(db + i, bsum);
        return;
    }
    for (int i = threadIdx.x; i < td.W; i += blockDim.x) {
        float bsum = 0.0f;
        for (int64_t row = blockIdx.x; row < rows; row += gridDim.x)
            bsum += activate_backward_row(td, row, i, P, Abar, Pbar);
        if (part)
            part[(int64_t)blockIdx.x * td.W + i] = bsum;
        else if ((int64_t)blockIdx.x < rows)
            atomicAdd(db + i, bsum);
    }
}

// The same for W % 4 == 0, W <= 1024 and at most 5 streams: a thread keeps
// four units (float4 loads, all streams of a row issued together), 256 / (W / 4)
// rows per pass; the block sums its rows' bias gradients in LDS and adds W
// values.
constexpr int ABV_MAXS = 5;
__global__ void __launch_bounds__(256) activate_backward_vec_kernel(TrainDims td, int64_t rows,
                                                                    const float *P,
                                                                    const float *Abar, float *Pbar,
                                                                    float *db, float *part)
{
    __shared__ float red[1024];
    const int W = td.W, S = td.S, W4 = W / 4;
    const int rpp = 256 / W4;
    const int lane_row = (int)threadIdx.x / W4;
    const int i = 4 * ((int)threadIdx.x % W4);
    const bool active = lane_row < rpp;
    float4 bsum = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (active) {
        const int64_t stride = (int64_t)gridDim.x * rpp;
        for (int64_t row = (int64_t)blockIdx.x * rpp + lane_row; row < rows; row += stride) {
            const int64_t c0 = row * S;
            float4 p[ABV_MAXS], ab[ABV_MAXS];
#pragma unroll
            for (int st = 0; st < ABV_MAXS; ++st)
                if (st < S) {
                    p[st] = *reinterpret_cast<const float4 *>(P + (c0 + st) * W + i);
                    ab[st] = *reinterpret_cast<const float4 *>(Abar + (c0 + st) * W + i);
                }
            float pv[4] = {p[0].x, p[0].y, p[0].z, p[0].w};
            float e[4], e2[4], pb[4];
            const float a0[4] = {ab[0].x, ab[0].y, ab[0].z, ab[0].w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                e[q] = elu_d(pv[q]);
                e2[q] = elu_dd(pv[q]);
                pb[q] = e[q] * a0[q];
            }
#pragma unroll
            for (int st = 1; st < ABV_MAXS; ++st)
                if (st < S) {
                    const float t[4] = {p[st].x, p[st].y, p[st].z, p[st].w};
                    const float a[4] = {ab[st].x, ab[st].y, ab[st].z, ab[st].w};
#pragma unroll
                    for (int q = 0; q < 4; ++q) pb[q] += e2[q] * t[q] * a[q];
                    *reinterpret_cast<float4 *>(Pbar + (c0 + st) * W + i) =
                        make_float4(e[0] * a[0], e[1] * a[1], e[2] * a[2], e[3] * a[3]);
                }
            *reinterpret_cast<float4 *>(Pbar + c0 * W + i) = make_float4(pb[0], pb[1], pb[2], pb[3]);
            bsum.x += pb[0];
            bsum.y += pb[1];
            bsum.z += pb[2];
            bsum.w += pb[3];
        }
        *reinterpret_cast<float4 *>(&red[lane_row * W + i]) = bsum;
    }
    __syncthreads();
    // every block has at least one row (the grid is at most ceil(rows / rpp))
    for (int u = threadIdx.x; u < W; u += blockDim.x) {
        float sum = 0.0f;
        for (int k = 0; k < rpp; ++k) sum += red[k * W + u];
        if (part)
            part[(int64_t)blockIdx.x * W + u] = sum;
        else
            atomicAdd(db + u, sum);
    }
}

// latent gradients: primal column -> z_s; velocity column -> (z_next - z_s)/dt.
// Every row of a group shares its snapshot: one block per group sums the
// group's rows per latent component in LDS (256 threads: r components times
// floor(256 / r) row lanes, leftover lanes idle) and adds r (or 2r) values
// to dZ.
__global__ void __launch_bounds__(256) latent_grad_kernel(TrainDims td, int64_t rows,
                                                          int rows_per_group, const int32_t *snap,
                                                          const int32_t *next, float inv_dt,
                                                          const float *A0bar, float *dZ,
                                                          float *part)
{
    __shared__ float red0[256], red1[256];
    const int grp = blockIdx.x;
    const int lanes = 256 / td.r;                 // row lanes per component
    const int k = threadIdx.x % td.r, lr = threadIdx.x / td.r;
    const int s = snap[grp], nx = next[grp];
    float a0 = 0.0f, a1 = 0.0f;
    if (lr < lanes) {
        for (int q = lr; q < rows_per_group; q += lanes) {
            const int64_t row = (int64_t)grp * rows_per_group + q;
            if (row >= rows) break;
            const int64_t c0 = row * td.S;
            a0 += A0bar[c0 * td.r + k];
            if (nx >= 0) a1 += A0bar[(c0 + td.d + 1) * td.r + k];
        }
    }
    red0[threadIdx.x] = lr < lanes ? a0 : 0.0f;
    red1[threadIdx.x] = lr < lanes ? a1 : 0.0f;
    __syncthreads();
    if (threadIdx.x < td.r) {
        float t0 = 0.0f, t1 = 0.0f;
        for (int q = 0; q < lanes; ++q) {
            t0 += red0[q * td.r + threadIdx.x];
            t1 += red1[q * td.r + threadIdx.x];
        }
        const float w = nx >= 0 ? t1 * inv_dt : 0.0f;
        if (part) {
            part[((int64_t)grp * 2) * td.r + threadIdx.x] = t0;
            part[((int64_t)grp * 2 + 1) * td.r + threadIdx.x] = w;
            return;
        }
        atomicAdd(dZ + (int64_t)s * td.r + threadIdx.x, t0);
        if (nx >= 0) {
            atomicAdd(dZ + (int64_t)nx * td.r + threadIdx.x, w);
            atomicAdd(dZ + (int64_t)s * td.r + threadIdx.x, -w);
        }
    }
}

// the groups' latent gradients applied in group order (one thread per
// latent component): reproducible where groups share snapshots
__global__ void latent_apply_kernel(int r, int n_groups, const int32_t *snap, const int32_t *next,
                                    const float *part, float *dZ)
{
    const int k = threadIdx.x;
    if (k >= r) return;
    for (int grp = 0; grp < n_groups; ++grp) {
        const int s = snap[grp], nx = next[grp];
        const float t0 = part[((int64_t)grp * 2) * r + k];
        const float w = part[((int64_t)grp * 2 + 1) * r + k];
        dZ[(int64_t)s * r + k] += t0;
        if (nx >= 0) {
            dZ[(int64_t)nx * r + k] += w;
            dZ[(int64_t)s * r + k] -= w;
        }
    }
}

__global__ void __launch_bounds__(256) loss_kernel(int d, int64_t rows, int rows_per_group,
                                                   const int32_t *next, const float *g,
                                                   const float *G, const float *Gv,
                                                   const float *xt, const float *Ft,
                                                   const float *vt, float lam_F, float lam_v,
                                                   float *loss, float *dg, float *dG, float *dGv)
{
    __shared__ float red[256];
    float l = 0.0f;
    // one block: each thread takes rows t, t + 256, ... in order, then a
    // fixed tree (the objective is reproducible)
    for (int64_t row = threadIdx.x; row < rows; row += 256) {
        const float inv = 1.0f / (float)rows;
        float lr = 0.0f;
        const float mv = next[row / rows_per_group] >= 0 ? 1.0f : 0.0f;
        for (int a = 0; a < d; ++a) {
            float rx = g[row * d + a] - xt[row * d + a];
            float rv = Gv[row * d + a] - vt[row * d + a];
            lr += rx * rx + lam_v * mv * rv * rv;
            if (dg) dg[row * d + a] = 2.0f * rx * inv;
            if (dGv) dGv[row * d + a] = 2.0f * lam_v * mv * rv * inv;
            for (int b = 0; b < d; ++b) {
                float rF = G[(row * d + a) * d + b] - Ft[(row * d + a) * d + b];
                lr += lam_F * rF * rF;
                if (dG) dG[(row * d + a) * d + b] = 2.0f * lam_F * rF * inv;
            }
        }
        l += lr * inv;
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0];
}

__global__ void adam_kernel(int64_t n, float *p, const float *grad, float *m, float *v, float lr,
                            float b1, float b2, float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = grad[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// training rows: snapshot frames [n_frames][P_sub] of (x, F, v) on a shared
// reference set X_sub [P_sub][d]; the batch takes particles pid[row] of
// frame snap[row / rows_per_group]
__global__ void gather_rows_kernel(int d, int64_t rows, int rows_per_group, int64_t P_sub,
                                   const float *X_sub, const float *fx, const float *fF,
                                   const float *fv, const int32_t *snap, const int32_t *pid,
                                   float *X, float *xt, float *Ft, float *vt)
{
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= rows) return;
    const int64_t f = snap[row / rows_per_group];
    const int64_t p = pid[row];
    const int64_t q = f * P_sub + p;
    for (int a = 0; a < d; ++a) {
        X[row * d + a] = X_sub[p * d + a];
        xt[row * d + a] = fx[q * d + a];
        vt[row * d + a] = fv[q * d + a];
    }
    for (int k = 0; k < d * d; ++k) Ft[row * d * d + k] = fF[q * d * d + k];
}

}  // namespace mr

using namespace mr;

struct mr_trainer {
    TrainDims td;
    int width, prec;
    int64_t max_rows;
    size_t n_params;
    size_t oW[10], ob[10];  // parameter offsets of layer l
    float *A0, *P[9], *A[9], *Y, *Ybar, *Abar, *Pbar, *A0bar;
    // saved by the last forward
    int64_t rows;
    int rows_per_group;
    const float *params, *X;
    const int32_t *snap, *next;
    float inv_dt;
    // reproducible mode: split-K slices, bias partial sums, group latents
    int det;
    float *stage, *part, *gpart;
};

static size_t param_count(int d, int r, int width, int nh)
{
    return (size_t)width * (d + r) + width + (size_t)(nh - 1) * ((size_t)width * width + width) +
           (size_t)d * width + d;
}

extern "C" int64_t rom_train_param_count(int32_t d, int32_t r, int32_t width, int32_t n_hidden)
{
    if (d < 2 || d > 3 || r < 1 || width < 1 || n_hidden < 1) return -1;
    return (int64_t)param_count(d, r, width, n_hidden);
}

extern "C" void rom_trainer_destroy(mr_trainer *t)
{
    if (!t) return;
    float *bufs[] = {t->A0, t->Y, t->Ybar, t->Abar, t->Pbar, t->A0bar, t->stage, t->part,
                     t->gpart};
    for (float *b : bufs)
        if (b) (void)hipFree(b);
    for (int l = 0; l < 9; ++l) {
        if (t->P[l]) (void)hipFree(t->P[l]);
        if (t->A[l]) (void)hipFree(t->A[l]);
    }
    free(t);
}

extern "C" int32_t rom_trainer_create(int32_t d, int32_t r, int32_t width, int32_t n_hidden,
                                      int32_t precision, int64_t max_rows, const float *in_min,
                                      const float *in_max, const float *out_mean,
                                      const float *out_std, int32_t output_mode, mr_trainer **out)
{
    if (!out || !in_min || !in_max || !out_mean || !out_std) return MR_EINVAL;
    if ((d != 2 && d != 3) || r < 1 || r > 64 || width < 1 || width > 1024 || n_hidden < 1 ||
        n_hidden > 8 || max_rows < 1)
        return MR_EINVAL;
    if (precision != MR_PREC_FP32 && precision != MR_PREC_BF16) return MR_EINVAL;
    if (output_mode != MR_OUT_POSITION && output_mode != MR_OUT_DISPLACEMENT) return MR_EINVAL;
    for (int a = 0; a < d; ++a)
        if (!(in_max[a] > in_min[a])) return MR_EINVAL;
    mr_trainer *t = (mr_trainer *)calloc(1, sizeof(mr_trainer));
    if (!t) return MR_ENOMEM;
    TrainDims &td = t->td;
    td.d = d;
    td.r = r;
    td.W = width;
    td.nh = n_hidden;
    td.S = d + 2;
    td.K0 = d + r;
    td.mode = output_mode;
    for (int a = 0; a < 3; ++a) {
        if (a < d) {
            td.scale[a] = 2.0f / (in_max[a] - in_min[a]);
            td.shift[a] = -2.0f * in_min[a] / (in_max[a] - in_min[a]) - 1.0f;
            td.mean[a] = out_mean[a];
            td.stdv[a] = out_std[a];
        } else {
            td.scale[a] = td.shift[a] = td.mean[a] = td.stdv[a] = 0.0f;
        }
    }
    t->width = width;
    t->prec = precision;
    t->max_rows = max_rows;
    t->n_params = param_count(d, r, width, n_hidden);
    size_t off = 0;
    int in = d + r;
    for (int l = 0; l <= n_hidden; ++l) {
        int outd = (l == n_hidden) ? d : width;
        t->oW[l] = off;
        off += (size_t)outd * in;
        t->ob[l] = off;
        off += outd;
        in = width;
    }
    const int64_t cols = max_rows * td.S;
    bool ok = true;
    auto alloc = [&](float **p, int64_t nfl) {
        if (ok && hipMalloc((void **)p, sizeof(float) * (nfl > 0 ? nfl : 1)) != hipSuccess) ok = false;
    };
    alloc(&t->A0, cols * td.K0);
    for (int l = 0; l < n_hidden; ++l) {
        alloc(&t->P[l], cols * width);
        alloc(&t->A[l], cols * width);
    }
    alloc(&t->Y, cols * d);
    alloc(&t->Ybar, cols * d);
    alloc(&t->Abar, cols * width);
    alloc(&t->Pbar, cols * width);
    alloc(&t->A0bar, cols * r);
    if (!ok) {
        rom_trainer_destroy(t);
        return MR_ENOMEM;
    }
    *out = t;
    return MR_OK;
}

extern "C" int32_t rom_train_forward(mr_trainer *t, const float *params, const float *Z,
                                     const float *X, const int32_t *snap, const int32_t *next,
                                     int32_t n_groups, int32_t rows_per_group, float dt, float *g,
                                     float *G, float *Gv, void *stream)
{
    if (!t || !params || !Z || !X || !snap || !next || !g || !G || !Gv || n_groups < 1 ||
        rows_per_group < 1 || !(dt > 0.0f))
        return MR_EINVAL;
    const int64_t rows = (int64_t)n_groups * rows_per_group;
    if (rows > t->max_rows) return MR_EINVAL;
    hipStream_t st = as_stream(stream);
    const TrainDims &td = t->td;
    const bool bf = t->prec == MR_PREC_BF16;
    const int64_t cols = rows * td.S;
    const int TB = 256;
    t->rows = rows;
    t->rows_per_group = rows_per_group;
    t->params = params;
    t->X = X;
    t->snap = snap;
    t->next = next;
    t->inv_dt = 1.0f / dt;
    build_input_kernel<<<(unsigned)ceil_div(cols, TB), TB, 0, st>>>(td, rows, rows_per_group, X, Z,
                                                                    snap, next, t->inv_dt, t->A0);
    MR_LAUNCH_CHECK();
    int32_t rc;
    const float *in = t->A0;
    int K = td.K0;
    for (int l = 0; l < td.nh; ++l) {
        // P_l[col][i] = sum_k W_l[i][k] in[col][k]  (first layer in fp32: it
        // sees the raw coordinates and latents)
        GemmArgs ga{};
        ga.M = td.W; ga.N = (int)cols; ga.K = K;
        ga.A = params + t->oW[l]; ga.sam = K; ga.sak = 1;
        ga.B = in; ga.sbk = 1; ga.sbn = K;
        ga.C = t->P[l]; ga.scm = 1; ga.scn = td.W;
        ga.mode = 0;
        if ((rc = gemm(bf && l > 0, ga, st)) != MR_OK) return rc;
        activate_kernel<<<(unsigned)ceil_div(rows * td.W, TB), TB, 0, st>>>(td, rows, t->P[l],
                                                                           params + t->ob[l], t->A[l]);
        MR_LAUNCH_CHECK();
        in = t->A[l];
        K = td.W;
    }
    GemmArgs go{};
    go.M = td.d; go.N = (int)cols; go.K = td.W;
    go.A = params + t->oW[td.nh]; go.sam = td.W; go.sak = 1;
    go.B = in; go.sbk = 1; go.sbn = td.W;
    go.C = t->Y; go.scm = 1; go.scn = td.d;
    go.mode = 0;
    if ((rc = gemm(false, go, st)) != MR_OK) return rc;
    output_kernel<<<(unsigned)ceil_div(rows, TB), TB, 0, st>>>(td, rows, X, t->Y,
                                                               params + t->ob[td.nh], g, G, Gv);
    MR_LAUNCH_CHECK();
    return MR_OK;
}

extern "C" int32_t rom_train_backward(mr_trainer *t, const float *dg, const float *dG,
                                      const float *dGv, float *dparams, float *dZ, void *stream)
{
    if (!t || !dg || !dG || !dGv || !dparams || !dZ || t->rows < 1) return MR_EINVAL;
    hipStream_t st = as_stream(stream);
    const TrainDims &td = t->td;
    const bool bf = t->prec == MR_PREC_BF16;
    const int64_t rows = t->rows, cols = rows * td.S;
    const float *params = t->params;
    const int TB = 256;
    // the batch reductions of the weight gradients are split over ~1,024 blocks
    const int splits = -1;
    int32_t rc;
    float *stage = t->det ? t->stage : nullptr;
    output_adjoint_kernel<<<(unsigned)ceil_div(rows, TB), TB, 0, st>>>(
        td, rows, dg, dG, dGv, t->Ybar, t->det ? nullptr : dparams + t->ob[td.nh]);
    if (t->det)
        output_bias_kernel<<<(unsigned)td.d, 256, 0, st>>>(td, rows, t->Ybar, dparams + t->ob[td.nh]);
    MR_LAUNCH_CHECK();
    // dW_L[a][i] += sum_col Ybar[col][a] A_last[col][i]
    GemmArgs gw{};
    gw.M = td.d; gw.N = td.W; gw.K = (int)cols;
    gw.A = t->Ybar; gw.sam = 1; gw.sak = td.d;
    gw.B = t->A[td.nh - 1]; gw.sbk = td.W; gw.sbn = 1;
    gw.C = dparams + t->oW[td.nh]; gw.scm = td.W; gw.scn = 1;
    gw.mode = 2;
    if ((rc = gemm(false, gw, st, splits, stage)) != MR_OK) return rc;
    // Abar[col][i] = sum_a W_L[a][i] Ybar[col][a]
    GemmArgs ga{};
    ga.M = td.W; ga.N = (int)cols; ga.K = td.d;
    ga.A = params + t->oW[td.nh]; ga.sam = 1; ga.sak = td.W;
    ga.B = t->Ybar; ga.sbk = 1; ga.sbn = td.d;
    ga.C = t->Abar; ga.scm = 1; ga.scn = td.W;
    ga.mode = 0;
    if ((rc = gemm(false, ga, st)) != MR_OK) return rc;
    for (int l = td.nh - 1; l >= 0; --l) {
        float *part = t->det ? t->part : nullptr;
        int64_t nslots = 0;
        if (td.W % 4 == 0 && td.W <= 1024 && td.S <= ABV_MAXS) {
            const int64_t rpp = 256 / (td.W / 4);
            const int64_t passes = ceil_div(rows, rpp);
            const int64_t grid = passes < 1024 ? passes : 1024;
            activate_backward_vec_kernel<<<(unsigned)grid, 256, 0, st>>>(
                td, rows, t->P[l], t->Abar, t->Pbar, dparams + t->ob[l], part);
            nslots = grid;
        } else {
            const int64_t rpp = td.W <= 256 ? 256 / td.W : 1;
            const int64_t passes = ceil_div(rows, rpp);
            const int64_t grid = passes < 1024 ? passes : 1024;
            activate_backward_kernel<<<(unsigned)grid, 256, 0, st>>>(
                td, rows, t->P[l], t->Abar, t->Pbar, dparams + t->ob[l], part);
            nslots = grid * rpp;
        }
        if (part)
            slot_reduce_kernel<<<(unsigned)td.W, 256, 0, st>>>(td.W, nslots, part,
                                                               dparams + t->ob[l]);
        MR_LAUNCH_CHECK();
        const int Kin = (l == 0) ? td.K0 : td.W;
        const float *in = (l == 0) ? t->A0 : t->A[l - 1];
        // dW_l[i][k] += sum_col Pbar[col][i] in[col][k]
        GemmArgs gd{};
        gd.M = td.W; gd.N = Kin; gd.K = (int)cols;
        gd.A = t->Pbar; gd.sam = 1; gd.sak = td.W;
        gd.B = in; gd.sbk = Kin; gd.sbn = 1;
        gd.C = dparams + t->oW[l]; gd.scm = Kin; gd.scn = 1;
        gd.mode = 2;
        if ((rc = gemm(bf && l > 0, gd, st, splits, stage)) != MR_OK) return rc;
        if (l > 0) {
            // Abar[col][k] = sum_i W_l[i][k] Pbar[col][i]
            GemmArgs gi{};
            gi.M = td.W; gi.N = (int)cols; gi.K = td.W;
            gi.A = params + t->oW[l]; gi.sam = 1; gi.sak = td.W;
            gi.B = t->Pbar; gi.sbk = 1; gi.sbn = td.W;
            gi.C = t->Abar; gi.scm = 1; gi.scn = td.W;
            gi.mode = 0;
            if ((rc = gemm(bf, gi, st)) != MR_OK) return rc;
        } else {
            // latent part of the first layer's input adjoint
            GemmArgs gz{};
            gz.M = td.r; gz.N = (int)cols; gz.K = td.W;
            gz.A = params + t->oW[0] + td.d; gz.sam = 1; gz.sak = td.K0;
            gz.B = t->Pbar; gz.sbk = 1; gz.sbn = td.W;
            gz.C = t->A0bar; gz.scm = 1; gz.scn = td.r;
            gz.mode = 0;
            if ((rc = gemm(false, gz, st)) != MR_OK) return rc;
        }
    }
    const int64_t n_groups = ceil_div(rows, (int64_t)t->rows_per_group);
    latent_grad_kernel<<<(unsigned)n_groups, 256, 0, st>>>(
        td, rows, t->rows_per_group, t->snap, t->next, t->inv_dt, t->A0bar, dZ,
        t->det ? t->gpart : nullptr);
    if (t->det)
        latent_apply_kernel<<<1, 64, 0, st>>>(td.r, (int)n_groups, t->snap, t->next, t->gpart, dZ);
    MR_LAUNCH_CHECK();
    return MR_OK;
}

extern "C" int32_t rom_train_loss(int32_t d, int32_t n_groups, int32_t rows_per_group,
                                  const int32_t *next, const float *g, const float *G,
                                  const float *Gv, const float *x_t, const float *F_t,
                                  const float *v_t, float lam_F, float lam_v, float *loss,
                                  float *dg, float *dG, float *dGv, void *stream)
{
    if ((d != 2 && d != 3) || n_groups < 1 || rows_per_group < 1 || !next || !g || !G || !Gv ||
        !x_t || !F_t || !v_t || !loss)
        return MR_EINVAL;
    const int64_t rows = (int64_t)n_groups * rows_per_group;
    hipStream_t st = as_stream(stream);
    loss_kernel<<<1, 256, 0, st>>>(d, rows, rows_per_group, next, g, G, Gv, x_t, F_t, v_t, lam_F,
                                   lam_v, loss, dg, dG, dGv);
    MR_LAUNCH_CHECK();
    return MR_OK;
}

extern "C" int32_t rom_adam_step(int64_t n, float *param, const float *grad, float *m, float *v,
                                 float lr, float beta1, float beta2, float eps, int32_t step,
                                 void *stream)
{
    if (n < 0 || (n > 0 && (!param || !grad || !m || !v)) || step < 1) return MR_EINVAL;
    if (n == 0) return MR_OK;
    const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
    adam_kernel<<<(unsigned)ceil_div(n, 256), 256, 0, as_stream(stream)>>>(n, param, grad, m, v, lr,
                                                                         beta1, beta2, eps, c1, c2);
    MR_LAUNCH_CHECK();
    return MR_OK;
}

extern "C" int32_t rom_train_gather(int32_t d, int32_t n_groups, int32_t rows_per_group,
                                    int64_t P_sub, const float *X_sub, const float *frame_x,
                                    const float *frame_F, const float *frame_v,
                                    const int32_t *snap, const int32_t *pid, float *X, float *x_t,
                                    float *F_t, float *v_t, void *stream)
{
    if ((d != 2 && d != 3) || n_groups < 1 || rows_per_group < 1 || P_sub < 1 || !X_sub ||
        !frame_x || !frame_F || !frame_v || !snap || !pid || !X || !x_t || !F_t || !v_t)
        return MR_EINVAL;
    const int64_t rows = (int64_t)n_groups * rows_per_group;
    gather_rows_kernel<<<(unsigned)ceil_div(rows, 256), 256, 0, as_stream(stream)>>>(
        d, rows, rows_per_group, P_sub, X_sub, frame_x, frame_F, frame_v, snap, pid, X, x_t, F_t,
        v_t);
    MR_LAUNCH_CHECK();
    return MR_OK;
}

extern "C" int32_t rom_trainer_set_deterministic(mr_trainer *t, int32_t on)
{
    if (!t) return MR_EINVAL;
    if (on && !t->stage) {
        // split-K slices: splits x M x N <= 1024 x 64 x 64 (gemm's rule);
        // bias partials: at most 1024 blocks x 256 row lanes or 1024 x W;
        // group latents: 2 r per group, at most max_rows groups
        const int64_t W = t->td.W;
        const int64_t nbias = W <= 256 ? 1024 * 256 : 1024 * W;
        if (hipMalloc(&t->stage, sizeof(float) * 1024 * 64 * 64) != hipSuccess ||
            hipMalloc(&t->part, sizeof(float) * nbias) != hipSuccess ||
            hipMalloc(&t->gpart, sizeof(float) * 2 * t->td.r * t->max_rows) != hipSuccess) {
            for (float **q : {&t->stage, &t->part, &t->gpart}) {
                if (*q) (void)hipFree(*q);
                *q = nullptr;
            }
            return MR_ENOMEM;
        }
    }
    t->det = on ? 1 : 0;
    return MR_OK;
}
