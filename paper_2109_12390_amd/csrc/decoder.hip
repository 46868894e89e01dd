// Neural deformation-map decoder g(X; xhat) with forward-mode derivatives on
// gfx950 matrix cores (paper Section 3.1, eqs. kinematicRestriction, defGrad
// and timederOne; Section 4 network: MLP with ELU).
//
// One wave evaluates NP x 16 points of one instance together with S - 1
// tangent streams per point (directions e_a in X for F = dg/dX, vhat for
// v = (dg/dxhat) vhat, e_k in xhat for the latent Jacobian).  A column of the
// wave's activation panel is one (point, stream) pair; the panel lives in LDS
// as [column][unit] (unit-contiguous, row stride padded against bank
// conflicts).  The width x width hidden layers are 16x16 MFMA tiles:
//   bf16 operands with fp32 accumulation (v_mfma_f32_16x16x32_bf16), or
//   fp32 operands (v_mfma_f32_16x16x4_f32) in the fp32 precision mode.
// The first layer (d + r inputs, folded as W_X Xn + (W_z xhat + b) with the
// latent part computed once per instance) and the last layer (width -> d),
// the ELU and its derivative, stay in fp32 vector arithmetic.  Tangents
// obey t' = ELU'(z) (W t), with z the primal pre-activation of the same
// point, which the MFMA output layout places in the same lane and register.
#include "project.h"

#include <stdlib.h>
#include <string.h>

#include <vector>

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// launch shapes of the decoder kernels (see launch_w)
enum DecVariant { DEC_COL = 0, DEC_COL_NP2 = 1, DEC_COL_NP4 = 2, DEC_ROWS = 3, DEC_REG = 4,
                  DEC_NVARIANT = 5 };
constexpr int DEC_BUCKETS = 32;   // size classes: floor(log2(instances x points))

struct mr_decoder {
    int d, r, width, W, nh, mode, prec;
    // autotuned shape per stream configuration (1, 5, 9) and size class;
    // -1: not tuned (a size rule applies)
    mutable int8_t tuned[3][DEC_BUCKETS];
    float *dev;          // padded fp32 parameters (one allocation)
    uint16_t *hid_bf16;  // hidden weights in bf16, (nh - 1) x W x W
    size_t n_params;     // unpadded parameter count
    float *staging;      // device copy of unpadded params for set_params
    float scale[3], shift[3], mean[3], stdv[3];
    // offsets (floats) inside dev
    size_t oW0, ob0, oWh, obh, oWL, obL;
};

namespace mr {

enum StreamKind { SK_PRIMAL = 0, SK_SPATIAL = 1, SK_VELOCITY = 2, SK_LATENT = 3, SK_ZERO = 4 };

constexpr int MAXS = 9;

struct DecK {
    int d, r, W, nh, mode;
    const float *W0, *b0, *Wh, *bh, *WL, *bL;
    const uint16_t *Whb;
    float scale[3], shift[3], mean[3], stdv[3];
};

struct StreamSpec {
    int kind[MAXS];
    int arg[MAXS];
    int zk;   // latent streams of block z take latent arg + zk * z (0: one z)
};

struct DecIO {
    int B;
    int64_t n_ref, n;
    const float *X;
    const int32_t *idx;
    int idx_per_inst;
    int idx_div;  // idx row of instance b is b / idx_div (when idx_per_inst)
    const int32_t *n_inst;  // nullable: points s >= n_inst[b] are skipped
    int64_t x_stride;       // instance b reads its inputs at X + b * x_stride (0: shared)
    int disp_only;          // displacement mode: write g - X instead of g
    const double *xhat, *vhat;
    float *x, *F, *v, *Jz;
    int jz_k0;  // first latent index of this launch's latent streams
};

__device__ __forceinline__ float elu(float z) { return z > 0.0f ? z : expm1f(z); }
__device__ __forceinline__ float elu_d(float z) { return z > 0.0f ? 1.0f : expf(z); }

// kind and argument of stream st in this block (latent streams shifted by
// zk * blockIdx.z; past the last latent they are zero streams)
__device__ __forceinline__ void stream_of(const StreamSpec &ss, int r, int st, int &kind, int &arg)
{
    kind = ss.kind[st];
    arg = ss.arg[st];
    if (kind == SK_LATENT) {
        arg += ss.zk * (int)blockIdx.z;
        if (arg >= r) kind = SK_ZERO;
    }
}

// blocks along z of a launch
inline unsigned z_blocks(const StreamSpec &ss, int r)
{
    return ss.zk > 0 ? (unsigned)((r + ss.zk - 1) / ss.zk) : 1u;
}

// ELU and its derivative from one hardware exponential, for activations that
// are stored in bf16: e^z - 1 is formed by subtraction, whose absolute error
// (a few 1e-8) is far below the bf16 rounding of the unit-sized activations
// it is summed with in the next layer.  For z > 0 the exponential (possibly
// +inf) is discarded by the selects, so it needs no clamp.
__device__ __forceinline__ void elu_fast(float z, float &h, float &e)
{
    const float ex = __expf(z);
    h = z > 0.0f ? z : ex - 1.0f;
    e = z > 0.0f ? 1.0f : ex;
}

// round-to-nearest-even fp32 -> bf16 bit pattern (finite inputs)
__host__ __device__ __forceinline__ uint16_t bf16_bits(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

// Unit order of bf16 activation panels and of the bf16 copy of the hidden
// weights (the k dimension of every hidden-layer product): within each block
// of 32 units, unit u = 32 m + 16 h + 4 g + q (h in 0..1, g in 0..3, q in
// 0..3) sits at position 32 m + 8 g + 4 h + q.  A 16x16 MFMA output tile
// pair (row tiles 2m and 2m + 1) leaves lane l holding units 32 m + 4 g + q
// and 32 m + 16 + 4 g + q of one column, g = l / 16; the B operand of a
// 16x16x32 k-step takes positions 32 m + 8 g + 0..7 of a column from lane l.
// With this order the two coincide, so one layer's activated accumulators
// are the next layer's B operands without leaving the registers.  The order
// is a relabelling of k applied to activations and weights alike.
__host__ __device__ constexpr int unit_pos(int u)
{
    return (u & ~31) | (((u >> 2) & 3) << 3) | (((u >> 4) & 1) << 2) | (u & 3);
}
__host__ __device__ constexpr int pos_unit(int p)
{
    return (p & ~31) | (((p >> 2) & 1) << 4) | (((p >> 3) & 3) << 2) | (p & 3);
}
static_assert(unit_pos(pos_unit(45)) == 45 && pos_unit(unit_pos(53)) == 53 &&
                  unit_pos(16 + 4) == 12 && unit_pos(4) == 8,
              "unit order");

template <typename T>
struct Elem;
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

// Panel element type: fp32 (accurate ELU, libm exponentials) or bf16 (fast
// ELU, hardware round-to-nearest-even conversion).  store4 writes four
// consecutive units of one column (16 or 8 bytes, aligned: the panel row
// stride and the unit offset 4 (lane / 16) are multiples of 4 elements).
template <>
struct Elem<float> {
    static constexpr int KS = 4;    // k per MFMA
    static constexpr int PAD = 4;   // row padding (elements)
    __device__ static void act(float z, float &h, float &e)
    {
        h = elu(z);
        e = elu_d(z);
    }
    __device__ static void store4(float *p, f32x4 v) { *reinterpret_cast<f32x4 *>(p) = v; }
    __device__ static f32x4 load4(const float *p) { return *reinterpret_cast<const f32x4 *>(p); }
    // panel position of unit u (a multiple of 4) and unit at position p
    __device__ static constexpr int pos(int u) { return u; }
    __device__ static constexpr int unit(int p) { return p; }
};
template <>
struct Elem<uint16_t> {
    static constexpr int KS = 32;
    static constexpr int PAD = 8;
    __device__ static void act(float z, float &h, float &e) { elu_fast(z, h, e); }
    __device__ static void store4(uint16_t *p, f32x4 v)
    {
        *reinterpret_cast<bf16x4 *>(p) = __builtin_convertvector(v, bf16x4);
    }
    __device__ static f32x4 load4(const uint16_t *p)
    {
        return __builtin_convertvector(*reinterpret_cast<const bf16x4 *>(p), f32x4);
    }
    __device__ static constexpr int pos(int u) { return unit_pos(u); }
    __device__ static constexpr int unit(int p) { return pos_unit(p); }
};

// One MFMA k-step: acc += A(16 x KS) * B(KS x 16).
//  fp32:  lane l holds A[l%16][k0 + l/16], B[k0 + l/16][l%16]
//  bf16:  lane l holds A[l%16][k0 + 8(l/16) + 0..7], B[k0 + 8(l/16) + 0..7][l%16]
// A row-major in global memory (row stride W), B from the LDS panel
// (column-major: B[k][j] at Hc[j*ld + k]).
__device__ __forceinline__ f32x4 mfma_step(const float *Arow, const float *Bcol, f32x4 acc,
                                           int lane)
{
    int g = lane >> 4;
    return __builtin_amdgcn_mfma_f32_16x16x4f32(Arow[g], Bcol[g], acc, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma_step(const uint16_t *Arow, const uint16_t *Bcol, f32x4 acc,
                                           int lane)
{
    int g = lane >> 4;
    bf16x8 a = *reinterpret_cast<const bf16x8 *>(Arow + 8 * g);
    bf16x8 b = *reinterpret_cast<const bf16x8 *>(Bcol + 8 * g);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
}

// Output of one (point s, stream st, component a) of instance b, from the
// last layer's dot product y = W_L[a] . h: the position (plus b_L, the
// output scaling and, in displacement mode, X), a column of F = dg/dX, the
// velocity, or a latent-Jacobian entry.
__device__ __forceinline__ void emit_output(const DecK &P, const StreamSpec &ss, const DecIO &io,
                                            int b, int64_t s, int st, int a, float y)
{
    const int D = P.d;
    int kind, arg;
    stream_of(ss, P.r, st, kind, arg);
    const int64_t n = io.n;
    const size_t bo = (size_t)b;
    if (kind == SK_PRIMAL) {
        if (io.x && blockIdx.z == 0) {
            float val = P.mean[a] + P.stdv[a] * (y + P.bL[a]);
            if (P.mode == MR_OUT_DISPLACEMENT && !io.disp_only) {
                int64_t row = io.idx ? (int64_t)io.idx[(io.idx_per_inst ? (int64_t)(b / io.idx_div) * n : 0) + s] : s;
                val += io.X[(int64_t)b * io.x_stride + a * io.n_ref + row];
            }
            io.x[(bo * D + a) * n + s] = val;
        }
    } else if (kind == SK_SPATIAL) {
        if (io.F) {
            float val = P.stdv[a] * y + ((P.mode == MR_OUT_DISPLACEMENT && a == arg) ? 1.0f : 0.0f);
            io.F[(bo * D * D + a * D + arg) * n + s] = val;
        }
    } else if (kind == SK_VELOCITY) {
        if (io.v) io.v[(bo * D + a) * n + s] = P.stdv[a] * y;
    } else if (kind == SK_LATENT) {
        if (io.Jz) io.Jz[(bo * D * P.r + (size_t)a * P.r + arg) * n + s] = P.stdv[a] * y;
    }
}

// launch shapes: point tiles per wave of the primal-only evaluation, and
// whether the primal-only / five-stream evaluations keep one row tile of
// accumulators (double-buffered panel) instead of the whole layer
#ifndef MR_DEC_PRIMAL_NP
#define MR_DEC_PRIMAL_NP 1
#endif
#ifndef MR_DEC_PRIMAL_DB
#define MR_DEC_PRIMAL_DB false
#endif
#ifndef MR_DEC_TANGENT_DB
#define MR_DEC_TANGENT_DB false
#endif
#ifndef MR_DEC_PRIMAL_WPB
#define MR_DEC_PRIMAL_WPB 16
#endif
#ifndef MR_DEC_TANGENT_WPB
#define MR_DEC_TANGENT_WPB 4
#endif

// Shared memory of a block: the per-instance vectors c0 and u (2 W floats),
// in bf16 mode the current hidden layer's weights (W rows, padded stride),
// then one activation panel per wave (two in the double-buffered shape).
// Staging the weights once per block and layer turns the MFMA A-operand
// fetches into LDS reads; from global memory every k-step waited on a
// cache round trip.
// Fixed block LDS: c0 and u (W floats each), the first layer's spatial
// weights W0[:, 0..d) and the output layer's weights (3 W floats each, d
// padded to 3; read by every lane, so kept next to the compute instead of
// behind a global load per use), then (bf16) a hidden layer's weights.
template <typename T, int W>
struct DecSmem {
    static constexpr bool WLDS = sizeof(T) == 2;
    static constexpr int LD = W + Elem<T>::PAD;
    static constexpr size_t vec = 8 * W * sizeof(float);
    static constexpr size_t fixed = vec + (WLDS ? (size_t)W * LD * sizeof(T) : 0);
};

// c0 = W_z xhat + b0 and u = W_z vhat of instance b, the spatial columns of
// W0 and the output weights into the block's fixed LDS
template <int W, bool WLS = true>
__device__ __forceinline__ void load_block_vectors(const DecK &P, const double *xh,
                                                   const double *vh, float *c0, float *u,
                                                   float *w0x, float *wls)
{
    const int in0 = P.d + P.r;
    for (int i = threadIdx.x; i < W; i += blockDim.x) {
        double s0 = P.b0[i], s1 = 0.0;
        for (int k = 0; k < P.r; ++k) {
            double w = P.W0[(size_t)i * in0 + P.d + k];
            s0 += w * xh[k];
            if (vh) s1 += w * vh[k];
        }
        c0[i] = (float)s0;
        u[i] = (float)s1;
    }
    for (int i = threadIdx.x; i < 3 * W; i += blockDim.x) {
        const int row = i / 3, a = i % 3;
        w0x[i] = a < P.d ? P.W0[(size_t)row * in0 + a] : 0.0f;
        if (WLS) wls[i] = i / W < P.d ? P.WL[i] : 0.0f;
    }
}

template <typename T, int W, int S, int NP, bool DB, int WPB>
__global__ void __launch_bounds__(64 * WPB) decoder_kernel(DecK P, StreamSpec ss, DecIO io)
{
    using E = Elem<T>;
    using SM = DecSmem<T, W>;
    constexpr int NCT = NP * S;          // column tiles per wave
    constexpr int COLS = NCT * 16;       // columns per wave
    constexpr int LD = W + E::PAD;       // panel and staged-weight row stride
    constexpr int NRT = W / 16;          // row tiles
    constexpr int NKS = W / E::KS;       // k-steps per row tile
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    constexpr int nwaves = WPB;
    const int b = blockIdx.y;
    const int64_t n_b = io.n_inst ? (int64_t)io.n_inst[b] : io.n;
    // a block entirely past this instance's points leaves before any barrier
    if ((int64_t)blockIdx.x * nwaves * (NP * 16) >= n_b) return;
    // per-instance vectors: c0 = W_z xhat + b0, u = W_z vhat
    float *c0 = reinterpret_cast<float *>(smem);
    float *u = c0 + W;
    float *w0x = u + W;
    float *wls = w0x + 3 * W;
    T *wsh = reinterpret_cast<T *>(smem + SM::vec);
    T *panel = reinterpret_cast<T *>(smem + SM::fixed) + (size_t)wave * (DB ? 2 : 1) * COLS * LD;
    T *pin = panel;
    T *pout = DB ? panel + COLS * LD : panel;
    const double *xh = io.xhat + (size_t)b * P.r;
    const double *vh = io.vhat ? io.vhat + (size_t)b * P.r : nullptr;
    load_block_vectors<W>(P, xh, vh, c0, u, w0x, wls);
    __syncthreads();

    // ---- first layer: lane handles point column j = lane % 16 of each point
    // tile and units 16 m + 4 (lane / 16) + q, q = 0..3 (the layout of an MFMA
    // output tile), stored four units at a time
    const int64_t wbase = ((int64_t)blockIdx.x * nwaves + wave) * (NP * 16);
    const int j = lane & 15;
    const int g = lane >> 4;
    const int in0 = P.d + P.r;
#pragma unroll
    for (int pt = 0; pt < NP; ++pt) {
        int64_t s = wbase + pt * 16 + j;
        float Xn[3] = {0.0f, 0.0f, 0.0f};
        if (s < n_b) {
            int64_t row = io.idx ? (int64_t)io.idx[(io.idx_per_inst ? (int64_t)(b / io.idx_div) * io.n : 0) + s] : s;
            for (int a = 0; a < P.d; ++a) Xn[a] = io.X[(int64_t)b * io.x_stride + a * io.n_ref + row] * P.scale[a] + P.shift[a];
        }
        for (int m = 0; m < NRT; ++m) {
            const int i0 = 16 * m + 4 * g;
            f32x4 h4, e4;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float *w0 = w0x + (i0 + q) * 3;
                float z = c0[i0 + q];
                for (int a = 0; a < P.d; ++a) z += w0[a] * Xn[a];
                float h, e;
                E::act(z, h, e);
                h4[q] = h;
                e4[q] = e;
            }
#pragma unroll
            for (int st = 0; st < S; ++st) {
                int kind, arg;
    stream_of(ss, P.r, st, kind, arg);
                f32x4 val;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (kind == SK_PRIMAL) val[q] = h4[q];
                    else if (kind == SK_SPATIAL) val[q] = e4[q] * w0x[(i0 + q) * 3 + arg] * P.scale[arg];
                    else if (kind == SK_VELOCITY) val[q] = e4[q] * u[i0 + q];
                    else if (kind == SK_LATENT) val[q] = e4[q] * P.W0[(size_t)(i0 + q) * in0 + P.d + arg];
                    else val[q] = 0.0f;
                }
                E::store4(pin + ((pt * S + st) * 16 + j) * LD + E::pos(i0), val);
            }
        }
    }
    __syncthreads();

    // ---- hidden layers on matrix cores
    for (int l = 0; l < P.nh - 1; ++l) {
        const T *Wl;
        int lda = W;
        if constexpr (SM::WLDS) {
            const T *src = reinterpret_cast<const T *>(P.Whb) + (size_t)l * W * W;
            __syncthreads();   // every wave is done with the previous layer's weights
            constexpr int V = W / 8;   // 16-byte vectors per row
            for (int t = threadIdx.x; t < W * V; t += 64 * WPB) {
                const int row = t / V, c8 = t % V;
                *reinterpret_cast<uint4 *>(wsh + row * LD + 8 * c8) =
                    reinterpret_cast<const uint4 *>(src)[t];
            }
            __syncthreads();
            Wl = wsh;
            lda = LD;
        } else {
            Wl = reinterpret_cast<const T *>(P.Wh) + (size_t)l * W * W;
        }
        const float *bl = P.bh + (size_t)l * W;
        if constexpr (!DB) {
            // primal columns start from the bias, tangent columns from zero
            f32x4 acc[NRT][NCT];
#pragma unroll
            for (int rt = 0; rt < NRT; ++rt) {
                f32x4 b4;
#pragma unroll
                for (int q = 0; q < 4; ++q) b4[q] = bl[rt * 16 + 4 * g + q];
#pragma unroll
                for (int ct = 0; ct < NCT; ++ct)
                    acc[rt][ct] = (ct % S == 0) ? b4 : f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            }
#pragma unroll
            for (int rt = 0; rt < NRT; ++rt) {
                const T *Arow = Wl + (size_t)(rt * 16 + j) * lda;
#pragma unroll
                for (int ks = 0; ks < NKS; ++ks)
#pragma unroll
                    for (int ct = 0; ct < NCT; ++ct)
                        acc[rt][ct] = mfma_step(Arow + ks * E::KS,
                                                pin + (ct * 16 + j) * LD + ks * E::KS, acc[rt][ct],
                                                lane);
            }
            // the panel is this wave's own: its reads above precede the
            // in-place writes below in the wave's in-order LDS stream
#pragma unroll
            for (int rt = 0; rt < NRT; ++rt) {
                const int i0 = rt * 16 + 4 * g;
#pragma unroll
                for (int pt = 0; pt < NP; ++pt) {
                    f32x4 h4, e4;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        float h, e;
                        E::act(acc[rt][pt * S][q], h, e);
                        h4[q] = h;
                        e4[q] = e;
                    }
                    E::store4(pout + ((pt * S) * 16 + j) * LD + E::pos(i0), h4);
#pragma unroll
                    for (int st = 1; st < S; ++st)
                        E::store4(pout + ((pt * S + st) * 16 + j) * LD + E::pos(i0),
                                  e4 * acc[rt][pt * S + st]);
                }
            }
        } else {
#pragma unroll 1
            for (int rt = 0; rt < NRT; ++rt) {
                f32x4 acc[NCT];
                f32x4 b4;
#pragma unroll
                for (int q = 0; q < 4; ++q) b4[q] = bl[rt * 16 + 4 * g + q];
#pragma unroll
                for (int ct = 0; ct < NCT; ++ct)
                    acc[ct] = (ct % S == 0) ? b4 : f32x4{0.0f, 0.0f, 0.0f, 0.0f};
                const T *Arow = Wl + (size_t)(rt * 16 + j) * lda;
#pragma unroll
                for (int ks = 0; ks < NKS; ++ks)
#pragma unroll
                    for (int ct = 0; ct < NCT; ++ct)
                        acc[ct] = mfma_step(Arow + ks * E::KS,
                                            pin + (ct * 16 + j) * LD + ks * E::KS, acc[ct], lane);
                const int i0 = rt * 16 + 4 * g;
#pragma unroll
                for (int pt = 0; pt < NP; ++pt) {
                    f32x4 h4, e4;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        float h, e;
                        E::act(acc[pt * S][q], h, e);
                        h4[q] = h;
                        e4[q] = e;
                    }
                    E::store4(pout + ((pt * S) * 16 + j) * LD + E::pos(i0), h4);
#pragma unroll
                    for (int st = 1; st < S; ++st)
                        E::store4(pout + ((pt * S + st) * 16 + j) * LD + E::pos(i0), e4 * acc[pt * S + st]);
                }
            }
            T *tmp = pin;
            pin = pout;
            pout = tmp;
        }
    }

    // ---- output layer (fp32): y_a = WL[a] . h (+ bL[a] for the primal)
    const int D = P.d;
    const int total = NCT * 16 * D;
    for (int it = lane; it < total; it += 64) {
        int col = it / D, a = it % D;
        int ct = col >> 4, jj = col & 15;
        int pt = ct / S, st = ct % S;
        int64_t s = wbase + pt * 16 + jj;
        if (s >= n_b) continue;
        const T *h = pin + (size_t)col * LD;
        const float *wl = wls + a * W;
        float y = 0.0f;
        for (int i = 0; i < W; i += 4) {
            const f32x4 h4 = E::load4(h + i);
            const int k = E::unit(i);
            y += wl[k] * h4[0] + wl[k + 1] * h4[1] + wl[k + 2] * h4[2] + wl[k + 3] * h4[3];
        }
        emit_output(P, ss, io, b, s, st, a, y);
    }
}


// Row-split shape, for small point sets: a block of W/16 waves evaluates one
// tile of 16 points with all S streams; wave w owns output units
// 16 w .. 16 w + 15 of every layer, the activation panel is shared by the
// block (double-buffered) and the layer's weights are staged once per block.
// The per-element arithmetic and its order are those of decoder_kernel, so
// both shapes give identical results.
template <typename T, int W, int S>
__global__ void __launch_bounds__(64 * (W / 16)) decoder_rows_kernel(DecK P, StreamSpec ss,
                                                                     DecIO io)
{
    using E = Elem<T>;
    using SM = DecSmem<T, W>;
    constexpr int NW = W / 16;           // waves = row tiles
    constexpr int COLS = S * 16;
    constexpr int LD = W + E::PAD;
    constexpr int NKS = W / E::KS;
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int j = lane & 15, g = lane >> 4;
    const int b = blockIdx.y;
    const int64_t n_b = io.n_inst ? (int64_t)io.n_inst[b] : io.n;
    const int64_t s0 = (int64_t)blockIdx.x * 16;
    if (s0 >= n_b) return;                                  // block-uniform
    float *c0 = reinterpret_cast<float *>(smem);
    float *u = c0 + W;
    float *w0x = u + W;
    float *wls = w0x + 3 * W;
    T *wsh = reinterpret_cast<T *>(smem + SM::vec);
    T *pin = reinterpret_cast<T *>(smem + SM::fixed);
    T *pout = pin + COLS * LD;
    const double *xh = io.xhat + (size_t)b * P.r;
    const double *vh = io.vhat ? io.vhat + (size_t)b * P.r : nullptr;
    load_block_vectors<W>(P, xh, vh, c0, u, w0x, wls);
    __syncthreads();
    // first layer: this wave's 16 units for the tile's 16 points
    const int in0 = P.d + P.r;
    const int i0 = 16 * wave + 4 * g;
    {
        const int64_t s = s0 + j;
        float Xn[3] = {0.0f, 0.0f, 0.0f};
        if (s < n_b) {
            int64_t row = io.idx ? (int64_t)io.idx[(io.idx_per_inst ? (int64_t)(b / io.idx_div) * io.n : 0) + s] : s;
            for (int a = 0; a < P.d; ++a) Xn[a] = io.X[(int64_t)b * io.x_stride + a * io.n_ref + row] * P.scale[a] + P.shift[a];
        }
        f32x4 h4, e4;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float *w0 = w0x + (i0 + q) * 3;
            float z = c0[i0 + q];
            for (int a = 0; a < P.d; ++a) z += w0[a] * Xn[a];
            float h, e;
            E::act(z, h, e);
            h4[q] = h;
            e4[q] = e;
        }
#pragma unroll
        for (int st = 0; st < S; ++st) {
            int kind, arg;
    stream_of(ss, P.r, st, kind, arg);
            f32x4 val;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (kind == SK_PRIMAL) val[q] = h4[q];
                else if (kind == SK_SPATIAL) val[q] = e4[q] * w0x[(i0 + q) * 3 + arg] * P.scale[arg];
                else if (kind == SK_VELOCITY) val[q] = e4[q] * u[i0 + q];
                else if (kind == SK_LATENT) val[q] = e4[q] * P.W0[(size_t)(i0 + q) * in0 + P.d + arg];
                else val[q] = 0.0f;
            }
            E::store4(pin + (st * 16 + j) * LD + E::pos(i0), val);
        }
    }
    __syncthreads();
    // hidden layers
    for (int l = 0; l < P.nh - 1; ++l) {
        const T *Wl;
        int lda = W;
        if constexpr (SM::WLDS) {
            const T *src = reinterpret_cast<const T *>(P.Whb) + (size_t)l * W * W;
            constexpr int V = W / 8;
            for (int t = threadIdx.x; t < W * V; t += 64 * NW) {
                const int row = t / V, c8 = t % V;
                *reinterpret_cast<uint4 *>(wsh + row * LD + 8 * c8) =
                    reinterpret_cast<const uint4 *>(src)[t];
            }
            __syncthreads();
            Wl = wsh;
            lda = LD;
        } else {
            Wl = reinterpret_cast<const T *>(P.Wh) + (size_t)l * W * W;
        }
        const float *bl = P.bh + (size_t)l * W;
        f32x4 acc[S];
        f32x4 b4;
#pragma unroll
        for (int q = 0; q < 4; ++q) b4[q] = bl[i0 + q];
        acc[0] = b4;
#pragma unroll
        for (int ct = 1; ct < S; ++ct) acc[ct] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        const T *Arow = Wl + (size_t)(16 * wave + j) * lda;
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks)
#pragma unroll
            for (int ct = 0; ct < S; ++ct)
                acc[ct] = mfma_step(Arow + ks * E::KS, pin + (ct * 16 + j) * LD + ks * E::KS,
                                    acc[ct], lane);
        f32x4 h4, e4;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float h, e;
            E::act(acc[0][q], h, e);
            h4[q] = h;
            e4[q] = e;
        }
        E::store4(pout + j * LD + E::pos(i0), h4);
#pragma unroll
        for (int st = 1; st < S; ++st) E::store4(pout + (st * 16 + j) * LD + E::pos(i0), e4 * acc[st]);
        __syncthreads();   // the new panel is complete; the old one and the weights are free
        T *tmp = pin;
        pin = pout;
        pout = tmp;
    }
    // output layer
    const int D = P.d;
    for (int it = threadIdx.x; it < COLS * D; it += 64 * NW) {
        const int col = it / D, a = it % D;
        const int st = col >> 4, jj = col & 15;
        const int64_t s = s0 + jj;
        if (s >= n_b) continue;
        const T *h = pin + (size_t)col * LD;
        const float *wl = wls + a * W;
        float y = 0.0f;
        for (int i = 0; i < W; i += 4) {
            const f32x4 h4 = E::load4(h + i);
            const int k = E::unit(i);
            y += wl[k] * h4[0] + wl[k + 1] * h4[1] + wl[k + 2] * h4[2] + wl[k + 3] * h4[3];
        }
        emit_output(P, ss, io, b, s, st, a, y);
    }
}

// Register-resident shape (bf16): waves split the points as in
// decoder_kernel, but the hidden layers keep their activations in registers.
// Under the panel unit order a lane's activated, converted accumulators of
// row tiles 2m and 2m + 1 are exactly its B operand of k-step m for the next
// layer, so only the staged weights (A operands) come from LDS.  The
// output layer runs on the matrix cores too, from those registers: its fp32
// weights are split into bf16 high and low parts (hi = bf16(w), lo =
// bf16(w - hi), rows 0..d-1 of two A operands), the products with the bf16
// activations are exact in fp32 and the MFMA sums them in fp32, so the layer
// keeps fp32 accuracy (the split leaves an error below 2^-16 of each weight)
// and only its summation order differs from the panel shapes'.  Every hidden
// activation is formed by the same arithmetic in the same order as there.
typedef __bf16 bf16x8v __attribute__((ext_vector_type(8)));

template <int W, int S, int NP, int WPB>
__global__ void __launch_bounds__(64 * WPB) decoder_reg_kernel(DecK P, StreamSpec ss, DecIO io)
{
    using T = uint16_t;
    using E = Elem<T>;
    using SM = DecSmem<T, W>;
    constexpr int NCT = NP * S;          // column tiles per wave
    constexpr int LD = W + E::PAD;
    constexpr int NRT = W / 16;          // row tiles
    constexpr int NKS = W / 32;          // k-steps
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int b = blockIdx.y;
    const int64_t n_b = io.n_inst ? (int64_t)io.n_inst[b] : io.n;
    if ((int64_t)blockIdx.x * WPB * (NP * 16) >= n_b) return;    // block-uniform
    float *c0 = reinterpret_cast<float *>(smem);
    float *u = c0 + W;
    float *w0x = u + W;
    float *wls = w0x + 3 * W;
    T *wsh = reinterpret_cast<T *>(smem + SM::vec);
    const double *xh = io.xhat + (size_t)b * P.r;
    const double *vh = io.vhat ? io.vhat + (size_t)b * P.r : nullptr;
    load_block_vectors<W, false>(P, xh, vh, c0, u, w0x, wls);
    // the output weights' bf16 high and low parts in panel order, [part][a][p],
    // in the slot of the fp32 copy (3 W floats = 2 x 3 W bf16)
    T *wob = reinterpret_cast<T *>(wls);
    for (int i = threadIdx.x; i < 3 * W; i += 64 * WPB) {
        const int a = i / W;
        const float w = a < P.d ? P.WL[(size_t)a * W + pos_unit(i % W)] : 0.0f;
        const uint16_t hi = bf16_bits(w);
        wob[i] = hi;
        wob[3 * W + i] = bf16_bits(w - __uint_as_float((uint32_t)hi << 16));
    }
    __syncthreads();

    const int64_t wbase = ((int64_t)blockIdx.x * WPB + wave) * (NP * 16);
    const int j = lane & 15;
    const int g = lane >> 4;
    bf16x8v Bop[NKS][NCT];
    bf16x4 lo[NCT];

    // ---- first layer (fp32 vector arithmetic, the same products as in
    // decoder_kernel)
    if constexpr (S == 1) {
        // the primal alone: straight-line code, the row tiles outer so that
        // one tile's first-layer weights serve both point tiles, and all
        // three input terms (w0x and Xn are zero beyond d).  (With tangent
        // streams this form leaves the B operands where the hidden loop's
        // register assignment needs copies, and spills at five streams.)
        float Xn[NP][3];
#pragma unroll
        for (int pt = 0; pt < NP; ++pt) {
            const int64_t s = wbase + pt * 16 + j;
#pragma unroll
            for (int a = 0; a < 3; ++a) Xn[pt][a] = 0.0f;
            if (s < n_b) {
                int64_t row = io.idx ? (int64_t)io.idx[(io.idx_per_inst ? (int64_t)(b / io.idx_div) * io.n : 0) + s] : s;
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    if (a < P.d) Xn[pt][a] = io.X[(int64_t)b * io.x_stride + a * io.n_ref + row] * P.scale[a] + P.shift[a];
            }
        }
#pragma unroll
        for (int m = 0; m < NRT; ++m) {
            const int i0 = 16 * m + 4 * g;
            float cw[4], ww[4][3];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                cw[q] = c0[i0 + q];
#pragma unroll
                for (int a = 0; a < 3; ++a) ww[q][a] = w0x[(i0 + q) * 3 + a];
            }
#pragma unroll
            for (int pt = 0; pt < NP; ++pt) {
                f32x4 h4;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float z = cw[q];
#pragma unroll
                    for (int a = 0; a < 3; ++a) z += ww[q][a] * Xn[pt][a];
                    float h, e;
                    E::act(z, h, e);
                    h4[q] = h;
                }
                const bf16x4 v4 = __builtin_convertvector(h4, bf16x4);
                if (m & 1)
                    Bop[m >> 1][pt] = __builtin_shufflevector(lo[pt], v4, 0, 1, 2, 3, 4, 5, 6, 7);
                else
                    lo[pt] = v4;
            }
        }
    } else {
        // tangent streams: each scales ELU' by a column of one LDS table
        // (w0x for a spatial tangent, u for the velocity; a zero stream by
        // 0), chosen once here instead of per element (the launcher admits
        // only these kinds).  The products are those of the panel shapes:
        // (e w0x) scale, (e u) 1.
        const float *cft[S];
        int cfk[S];
        float cfs[S];
#pragma unroll
        for (int st = 1; st < S; ++st) {
            int kind, arg;
            stream_of(ss, P.r, st, kind, arg);
            cft[st] = kind == SK_SPATIAL ? w0x + arg : u;
            cfk[st] = kind == SK_SPATIAL ? 3 : 1;
            cfs[st] = kind == SK_SPATIAL ? P.scale[arg] : (kind == SK_VELOCITY ? 1.0f : 0.0f);
        }
#pragma unroll
        for (int pt = 0; pt < NP; ++pt) {
            const int64_t s = wbase + pt * 16 + j;
            float Xn[3] = {0.0f, 0.0f, 0.0f};
            if (s < n_b) {
                int64_t row = io.idx ? (int64_t)io.idx[(io.idx_per_inst ? (int64_t)(b / io.idx_div) * io.n : 0) + s] : s;
                for (int a = 0; a < P.d; ++a) Xn[a] = io.X[(int64_t)b * io.x_stride + a * io.n_ref + row] * P.scale[a] + P.shift[a];
            }
#pragma unroll
            for (int m = 0; m < NRT; ++m) {
                const int i0 = 16 * m + 4 * g;
                f32x4 h4, e4;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float *w0 = w0x + (i0 + q) * 3;
                    float z = c0[i0 + q];
                    for (int a = 0; a < P.d; ++a) z += w0[a] * Xn[a];
                    float h, e;
                    E::act(z, h, e);
                    h4[q] = h;
                    e4[q] = e;
                }
#pragma unroll
                for (int st = 0; st < S; ++st) {
                    f32x4 val;
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        val[q] = st == 0 ? h4[q] : e4[q] * cft[st][(i0 + q) * cfk[st]] * cfs[st];
                    const bf16x4 v4 = __builtin_convertvector(val, bf16x4);
                    if (m & 1)
                        Bop[m >> 1][pt * S + st] = __builtin_shufflevector(lo[pt * S + st], v4, 0, 1, 2, 3, 4, 5, 6, 7);
                    else
                        lo[pt * S + st] = v4;
                }
            }
        }
    }

    // ---- hidden layers on matrix cores, activations in registers
    for (int l = 0; l < P.nh - 1; ++l) {
        const T *src = reinterpret_cast<const T *>(P.Whb) + (size_t)l * W * W;
        __syncthreads();   // every wave is done with the previous layer's weights
        constexpr int V = W / 8;
        for (int t = threadIdx.x; t < W * V; t += 64 * WPB) {
            const int row = t / V, c8 = t % V;
            *reinterpret_cast<uint4 *>(wsh + row * LD + 8 * c8) = reinterpret_cast<const uint4 *>(src)[t];
        }
        __syncthreads();
        const float *bl = P.bh + (size_t)l * W;
        bf16x8v Bn[NKS][NCT];
#pragma unroll
        for (int rt = 0; rt < NRT; ++rt) {
            f32x4 acc[NCT];
            f32x4 b4;
#pragma unroll
            for (int q = 0; q < 4; ++q) b4[q] = bl[rt * 16 + 4 * g + q];
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct)
                acc[ct] = (ct % S == 0) ? b4 : f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            const T *Arow = wsh + (rt * 16 + j) * LD + 8 * g;
#pragma unroll
            for (int ks = 0; ks < NKS; ++ks) {
                const bf16x8v a = *reinterpret_cast<const bf16x8v *>(Arow + ks * 32);
#pragma unroll
                for (int ct = 0; ct < NCT; ++ct)
                    acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, Bop[ks][ct], acc[ct], 0, 0, 0);
            }
#pragma unroll
            for (int pt = 0; pt < NP; ++pt) {
                f32x4 h4, e4;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float h, e;
                    E::act(acc[pt * S][q], h, e);
                    h4[q] = h;
                    e4[q] = e;
                }
#pragma unroll
                for (int st = 0; st < S; ++st) {
                    const f32x4 val = st == 0 ? h4 : e4 * acc[pt * S + st];
                    const bf16x4 v4 = __builtin_convertvector(val, bf16x4);
                    if (rt & 1)
                        Bn[rt >> 1][pt * S + st] = __builtin_shufflevector(lo[pt * S + st], v4, 0, 1, 2, 3, 4, 5, 6, 7);
                    else
                        lo[pt * S + st] = v4;
                }
            }
        }
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks)
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct) Bop[ks][ct] = Bn[ks][ct];
    }

    // ---- output layer on matrix cores: lane (j, g = 0) ends with outputs
    // a = 0..3 of point j of the column tile (rows 3 and up of A are zero)
    const int D = P.d;
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
        f32x4 y = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) {
            bf16x8v ahi = {}, alo = {};
            if (j < 3) {
                ahi = *reinterpret_cast<const bf16x8v *>(wob + j * W + ks * 32 + 8 * g);
                alo = *reinterpret_cast<const bf16x8v *>(wob + 3 * W + j * W + ks * 32 + 8 * g);
            }
            y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, Bop[ks][ct], y, 0, 0, 0);
            y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, Bop[ks][ct], y, 0, 0, 0);
        }
        const int pt = ct / S, st = ct % S;
        const int64_t s = wbase + pt * 16 + j;
        if (g == 0 && s < n_b) {
#pragma unroll
            for (int a = 0; a < 3; ++a)
                if (a < D) emit_output(P, ss, io, b, s, st, a, y[a]);
        }
    }
}

template <typename T, int W, int S, int NP, bool DB, int WPB>
int32_t launch_one(const DecK &P, const StreamSpec &ss, const DecIO &io, hipStream_t st)
{
    using E = Elem<T>;
    constexpr int COLS = NP * S * 16;
    constexpr size_t per_wave = (size_t)(DB ? 2 : 1) * COLS * (W + E::PAD) * sizeof(T);
    constexpr size_t lds = DecSmem<T, W>::fixed + (size_t)WPB * per_wave;
    static_assert(WPB >= 1 && lds <= 160 * 1024, "decoder block does not fit the LDS of a compute unit");
    const int64_t pts_per_block = (int64_t)WPB * NP * 16;
    dim3 grid((unsigned)ceil_div(io.n, pts_per_block), (unsigned)io.B, z_blocks(ss, P.r));
    auto kern = decoder_kernel<T, W, S, NP, DB, WPB>;
    static bool attr_set = false;  // the LDS size of an instantiation is fixed
    if (!attr_set) {
        MR_CHECK_HIP(hipFuncSetAttribute((const void *)kern,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        attr_set = true;
    }
    kern<<<grid, 64 * WPB, lds, st>>>(P, ss, io);
    MR_LAUNCH_CHECK();
    return MR_OK;
}

// waves per block of a shape: as many as fit the 160 KB of LDS, at most `cap`
template <typename T, int W, int S, int NP, bool DB>
constexpr int dec_wpb(int cap)
{
    constexpr size_t per_wave = (size_t)(DB ? 2 : 1) * NP * S * 16 * (W + Elem<T>::PAD) * sizeof(T);
    constexpr size_t fixed = DecSmem<T, W>::fixed;
    int w = (int)((160 * 1024 - fixed) / per_wave);
    return w < cap ? w : cap;
}

template <typename T, int W, int S>
int32_t launch_rows(const DecK &P, const StreamSpec &ss, const DecIO &io, hipStream_t st)
{
    constexpr size_t lds = DecSmem<T, W>::fixed + 2 * (size_t)S * 16 * (W + Elem<T>::PAD) * sizeof(T);
    static_assert(lds <= 160 * 1024, "decoder block does not fit the LDS of a compute unit");
    dim3 grid((unsigned)ceil_div(io.n, 16), (unsigned)io.B, z_blocks(ss, P.r));
    auto kern = decoder_rows_kernel<T, W, S>;
    static bool attr_set = false;
    if (!attr_set) {
        MR_CHECK_HIP(hipFuncSetAttribute((const void *)kern,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        attr_set = true;
    }
    kern<<<grid, 64 * (W / 16), lds, st>>>(P, ss, io);
    MR_LAUNCH_CHECK();
    return MR_OK;
}

// waves per block of the register-resident shape
#ifndef MR_DEC_REG_WPB
#define MR_DEC_REG_WPB 8
#endif

template <int W, int S, int NP>
int32_t launch_reg(const DecK &P, const StreamSpec &ss, const DecIO &io, hipStream_t st)
{
    constexpr int WPB = MR_DEC_REG_WPB;
    constexpr size_t lds = DecSmem<uint16_t, W>::fixed;
    static_assert(lds <= 160 * 1024, "decoder block does not fit the LDS of a compute unit");
    dim3 grid((unsigned)ceil_div(io.n, (int64_t)WPB * NP * 16), (unsigned)io.B, z_blocks(ss, P.r));
    // the first layer takes stream 0 to be the primal and the others to be
    // spatial, velocity or zero streams
    if (ss.kind[0] != SK_PRIMAL) return MR_EINVAL;
    for (int st = 1; st < S; ++st)
        if (ss.kind[st] != SK_SPATIAL && ss.kind[st] != SK_VELOCITY && ss.kind[st] != SK_ZERO)
            return MR_EINVAL;
    auto kern = decoder_reg_kernel<W, S, NP, WPB>;
    static bool attr_set = false;
    if (!attr_set) {
        MR_CHECK_HIP(hipFuncSetAttribute((const void *)kern,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        attr_set = true;
    }
    kern<<<grid, 64 * WPB, lds, st>>>(P, ss, io);
    MR_LAUNCH_CHECK();
    return MR_OK;
}

// Launch shapes per stream configuration (1: primal only, 5: x, F, v;
// 9: x and 8 latent-Jacobian columns):
//   DEC_COL      one or more point tiles per wave, waves split the points
//   DEC_COL_NP2  two point tiles per wave (primal only)
//   DEC_COL_NP4  four point tiles per wave (primal only)
//   DEC_ROWS     waves of a block split a layer's units (small point sets)
//   DEC_REG      waves split the points, hidden activations in registers
//                (bf16 only; two point tiles per wave for cfg 1, one for
//                cfg 5; not offered for cfg 9, whose 9 streams would not fit)
template <typename T, int W>
int32_t launch_w(int cfg, int variant, const DecK &P, const StreamSpec &ss, const DecIO &io,
                 hipStream_t st)
{
    constexpr int NP1 = MR_DEC_PRIMAL_NP;
    constexpr bool DB1 = MR_DEC_PRIMAL_DB, DB5 = MR_DEC_TANGENT_DB;
    if constexpr (sizeof(T) == 2 && W >= 32) {   // bf16 decoders have W >= 32
        if (variant == DEC_REG && cfg == 1) return launch_reg<W, 1, 2>(P, ss, io, st);
        if (variant == DEC_REG && cfg == 5) return launch_reg<W, 5, 1>(P, ss, io, st);
        if (variant == DEC_REG && cfg == 4) return launch_reg<W, 4, 1>(P, ss, io, st);
    }
    if (variant == DEC_REG) variant = DEC_COL;
    // x and F without v: the other shapes run the five-stream kernels with
    // the velocity stream zero
    if (cfg == 4) cfg = 5;
    if (cfg == 1) {
        if (variant == DEC_ROWS) return launch_rows<T, W, 1>(P, ss, io, st);
        if (variant == DEC_COL_NP2)
            return launch_one<T, W, 1, 2, false, dec_wpb<T, W, 1, 2, false>(12)>(P, ss, io, st);
        if (variant == DEC_COL_NP4)
            return launch_one<T, W, 1, 4, false, dec_wpb<T, W, 1, 4, false>(6)>(P, ss, io, st);
        return launch_one<T, W, 1, NP1, DB1, dec_wpb<T, W, 1, NP1, DB1>(MR_DEC_PRIMAL_WPB)>(P, ss, io,
                                                                                          st);
    }
    if (cfg == 5) {
        if (variant == DEC_ROWS) return launch_rows<T, W, 5>(P, ss, io, st);
        return launch_one<T, W, 5, 1, DB5, dec_wpb<T, W, 5, 1, DB5>(MR_DEC_TANGENT_WPB)>(P, ss, io, st);
    }
    if (variant == DEC_ROWS) return launch_rows<T, W, 9>(P, ss, io, st);
    return launch_one<T, W, 9, 1, true, dec_wpb<T, W, 9, 1, true>(4)>(P, ss, io, st);
}

// Decoder without hidden layers (the linear manifold): y = W0 [Xn, xhat] + b0.
// One thread per (instance, point) writes every requested output.
__global__ void linear_decoder_kernel(DecK P, DecIO io)
{
    const int b = blockIdx.y;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n_b = io.n_inst ? (int64_t)io.n_inst[b] : io.n;
    if (s >= n_b) return;
    const int D = P.d, in0 = P.d + P.r;
    const int64_t n = io.n;
    const int64_t row = io.idx ? (int64_t)io.idx[(io.idx_per_inst ? (int64_t)(b / io.idx_div) * n : 0) + s] : s;
    const double *xh = io.xhat + (size_t)b * P.r;
    const double *vh = io.vhat ? io.vhat + (size_t)b * P.r : nullptr;
    float Xr[3], Xn[3];
    for (int a = 0; a < D; ++a) {
        Xr[a] = io.X[(int64_t)b * io.x_stride + a * io.n_ref + row];
        Xn[a] = Xr[a] * P.scale[a] + P.shift[a];
    }
    const size_t bo = (size_t)b;
    for (int a = 0; a < D; ++a) {
        const float *w = P.W0 + (size_t)a * in0;
        if (io.x) {
            double y = P.b0[a];
            for (int k = 0; k < D; ++k) y += (double)w[k] * Xn[k];
            for (int k = 0; k < P.r; ++k) y += (double)w[D + k] * xh[k];
            float val = P.mean[a] + P.stdv[a] * (float)y;
            if (P.mode == MR_OUT_DISPLACEMENT && !io.disp_only) val += Xr[a];
            io.x[(bo * D + a) * n + s] = val;
        }
        if (io.F)
            for (int c = 0; c < D; ++c)
                io.F[(bo * D * D + a * D + c) * n + s] =
                    P.stdv[a] * w[c] * P.scale[c] + ((P.mode == MR_OUT_DISPLACEMENT && a == c) ? 1.0f : 0.0f);
        if (io.v && vh) {
            double y = 0.0;
            for (int k = 0; k < P.r; ++k) y += (double)w[D + k] * vh[k];
            io.v[(bo * D + a) * n + s] = P.stdv[a] * (float)y;
        }
        if (io.Jz)
            for (int k = 0; k < P.r; ++k)
                io.Jz[(bo * D * P.r + (size_t)a * P.r + k) * n + s] = P.stdv[a] * w[D + k];
    }
}

// tuning slot of a configuration (4, x and F only, shares the slot of 5)
inline int cfg_index(int cfg) { return cfg == 1 ? 0 : (cfg == 5 || cfg == 4 ? 1 : 2); }

// whether a shape can run configuration cfg of this decoder
inline bool shape_available(const mr_decoder *dec, int cfg, int v)
{
    if (v < 0 || v >= DEC_NVARIANT) return false;
    if (cfg != 1 && (v == DEC_COL_NP2 || v == DEC_COL_NP4)) return false;
    if (v == DEC_REG) return dec->prec == MR_PREC_BF16 && cfg != 9;
    return true;
}

// size class of a launch: floor(log2(instances x points))
inline int size_bucket(int64_t pts)
{
    int b = 0;
    while (b < DEC_BUCKETS - 1 && ((int64_t)2 << b) <= pts) ++b;
    return b;
}

// Shape for a launch: the autotuned choice of the nearest tuned size class
// (within a factor 4), else the size rule: row split up to 8192 points,
// above that registers-resident activations where available (bf16, cfg 1
// and 5), else point split.
int dec_variant(const mr_decoder *dec, int cfg, int64_t pts)
{
    const int ci = cfg_index(cfg), bk = size_bucket(pts);
    for (int dist = 0; dist <= 2; ++dist)
        for (int sgn = -1; sgn <= 1; sgn += 2) {
            const int q = bk + sgn * dist;
            if (q >= 0 && q < DEC_BUCKETS && dec->tuned[ci][q] >= 0) return dec->tuned[ci][q];
        }
    if (pts <= 8192) return DEC_ROWS;
    return shape_available(dec, cfg, DEC_REG) ? DEC_REG : DEC_COL;
}

// force_fp32: run a bf16 decoder's launch on its fp32 parameters (the fp32
// kernels at the same padded width; shapes by the size rule, since the tuned
// table holds bf16 choices)
int32_t launch_cfg(const mr_decoder *dec, int cfg, const StreamSpec &ss, const DecIO &io,
                   hipStream_t st, int variant_override = -1, int force_fp32 = 0)
{
    DecK P;
    P.d = dec->d;
    P.r = dec->r;
    P.W = dec->W;
    P.nh = dec->nh;
    P.mode = dec->mode;
    P.W0 = dec->dev + dec->oW0;
    P.b0 = dec->dev + dec->ob0;
    P.Wh = dec->dev + dec->oWh;
    P.bh = dec->dev + dec->obh;
    P.WL = dec->dev + dec->oWL;
    P.bL = dec->dev + dec->obL;
    P.Whb = dec->hid_bf16;
    for (int a = 0; a < 3; ++a) {
        P.scale[a] = dec->scale[a];
        P.shift[a] = dec->shift[a];
        P.mean[a] = dec->mean[a];
        P.stdv[a] = dec->stdv[a];
    }
    if (dec->nh == 0) {
        dim3 grid((unsigned)ceil_div(io.n, 256), (unsigned)io.B);
        linear_decoder_kernel<<<grid, 256, 0, st>>>(P, io);
        MR_LAUNCH_CHECK();
        return MR_OK;
    }
    const bool bf = dec->prec == MR_PREC_BF16 && !force_fp32;
    int variant = variant_override >= 0 ? variant_override
                                        : dec_variant(dec, cfg, (int64_t)io.B * io.n);
    if (dec->prec == MR_PREC_BF16 && !bf && variant_override < 0)
        variant = (int64_t)io.B * io.n <= 8192 ? DEC_ROWS : DEC_COL;
    switch (dec->W) {
    case 16: return bf ? launch_w<uint16_t, 16>(cfg, variant, P, ss, io, st) : launch_w<float, 16>(cfg, variant, P, ss, io, st);
    case 32: return bf ? launch_w<uint16_t, 32>(cfg, variant, P, ss, io, st) : launch_w<float, 32>(cfg, variant, P, ss, io, st);
    case 64: return bf ? launch_w<uint16_t, 64>(cfg, variant, P, ss, io, st) : launch_w<float, 64>(cfg, variant, P, ss, io, st);
    case 128: return bf ? launch_w<uint16_t, 128>(cfg, variant, P, ss, io, st) : launch_w<float, 128>(cfg, variant, P, ss, io, st);
    default: return MR_EINVAL;
    }
}

// --- parameter packing: unpadded [W0, b0, W1, b1, ..., WL, bL] -> padded
__global__ void pack_params_kernel(const float *src, float *dst, uint16_t *hid, int d, int r,
                                   int width, int W, int nh, size_t oW0, size_t ob0, size_t oWh,
                                   size_t obh, size_t oWL, size_t obL)
{
    const int in0 = d + r;
    if (nh == 0) {  // linear decoder: dense (d x in0) matrix and d biases
        size_t tot = (size_t)d * in0 + d;
        for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot;
             t += (size_t)gridDim.x * blockDim.x) {
            if (t < (size_t)d * in0)
                dst[oW0 + t] = src[t];
            else
                dst[ob0 + (t - (size_t)d * in0)] = src[t];
        }
        return;
    }
    size_t total = (size_t)W * in0 + W + (size_t)(nh - 1) * (W * W + W) + (size_t)d * W + d;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (size_t)gridDim.x * blockDim.x) {
        size_t q = t;
        // source layout offsets
        size_t s_W0 = 0, s_b0 = (size_t)width * in0;
        size_t s_h = s_b0 + width;
        size_t hsz = (size_t)width * width + width;
        size_t s_WL = s_h + (size_t)(nh - 1) * hsz, s_bL = s_WL + (size_t)d * width;
        float val = 0.0f;
        if (q < (size_t)W * in0) {
            int i = (int)(q / in0), k = (int)(q % in0);
            if (i < width) val = src[s_W0 + (size_t)i * in0 + k];
            dst[oW0 + q] = val;
            continue;
        }
        q -= (size_t)W * in0;
        if (q < (size_t)W) {
            if ((int)q < width) val = src[s_b0 + q];
            dst[ob0 + q] = val;
            continue;
        }
        q -= W;
        if (q < (size_t)(nh - 1) * W * W) {
            int l = (int)(q / ((size_t)W * W));
            size_t rem = q % ((size_t)W * W);
            int i = (int)(rem / W), k = (int)(rem % W);
            if (i < width && k < width) val = src[s_h + l * hsz + (size_t)i * width + k];
            dst[oWh + q] = val;
            // bf16 copy in the panel unit order (W >= 32 in bf16 mode; the
            // copy of an fp32 decoder is never read)
            hid[q - k + (W % 32 == 0 ? unit_pos(k) : k)] = bf16_bits(val);
            continue;
        }
        q -= (size_t)(nh - 1) * W * W;
        if (q < (size_t)(nh - 1) * W) {
            int l = (int)(q / W), i = (int)(q % W);
            if (i < width) val = src[s_h + l * hsz + (size_t)width * width + i];
            dst[obh + q] = val;
            continue;
        }
        q -= (size_t)(nh - 1) * W;
        if (q < (size_t)d * W) {
            int a = (int)(q / W), i = (int)(q % W);
            if (i < width) val = src[s_WL + (size_t)a * width + i];
            dst[oWL + q] = val;
            continue;
        }
        q -= (size_t)d * W;
        dst[obL + q] = src[s_bL + q];
    }
}

}  // namespace mr

using namespace mr;

static size_t unpadded_count(int d, int r, int width, int nh)
{
    if (nh == 0) return (size_t)d * (d + r) + d;
    return (size_t)width * (d + r) + width + (size_t)(nh - 1) * ((size_t)width * width + width) +
           (size_t)d * width + d;
}

extern "C" int32_t rom_decoder_set_params(mr_decoder *dec, const float *params,
                                          int32_t params_on_device, void *stream)
{
    if (!dec || !params) return MR_EINVAL;
    hipStream_t st = as_stream(stream);
    const float *src = params;
    if (!params_on_device) {
        MR_CHECK_HIP(hipMemcpyAsync(dec->staging, params, dec->n_params * sizeof(float),
                                    hipMemcpyHostToDevice, st));
        src = dec->staging;
    }
    pack_params_kernel<<<256, 256, 0, st>>>(src, dec->dev, dec->hid_bf16, dec->d, dec->r, dec->width,
                                            dec->W, dec->nh, dec->oW0, dec->ob0, dec->oWh, dec->obh,
                                            dec->oWL, dec->obL);
    MR_LAUNCH_CHECK();
    if (!params_on_device) MR_CHECK_HIP(hipStreamSynchronize(st));
    return MR_OK;
}

namespace mr {

// stream specification of a configuration as decode_jac_ex builds it
static StreamSpec spec_of(int cfg, int d)
{
    StreamSpec ss{};
    ss.kind[0] = SK_PRIMAL;
    if (cfg == 5) {
        for (int a = 0; a < 3; ++a) {
            ss.kind[1 + a] = a < d ? SK_SPATIAL : SK_ZERO;
            ss.arg[1 + a] = a;
        }
        ss.kind[4] = SK_VELOCITY;
    } else if (cfg == 9) {
        for (int q = 0; q < 8; ++q) {
            ss.kind[1 + q] = SK_LATENT;
            ss.arg[1 + q] = q;
        }
    }
    return ss;
}

int32_t decoder_autotune(const mr_decoder *dec, int32_t B, int64_t n, int32_t cfg_mask,
                         int32_t reps, hipStream_t st)
{
    if (!dec || B < 1 || n < 1 || reps < 1 || (cfg_mask & ~7)) return MR_EINVAL;
    if (dec->nh == 0) return MR_OK;   // the linear decoder has one shape
    const int d = dec->d, r = dec->r;
    const int64_t pts = (int64_t)B * n;
    int32_t rc = MR_OK;
    for (int ci = 0; ci < 3 && rc == MR_OK; ++ci) {
        if (!(cfg_mask & (1 << ci))) continue;
        const int cfg = ci == 0 ? 1 : (ci == 1 ? 5 : 9);
        // representative size: the same instances and points when affordable,
        // else one instance with a capped point count
        const int64_t cap = ci == 2 ? ((int64_t)1 << 20) : ((int64_t)1 << 22);
        int32_t Bt = B;
        int64_t nt = n;
        if (pts > cap) {
            Bt = 1;
            nt = cap;
        }
        const int64_t rj = ci == 2 ? (int64_t)d * (r > 8 ? r : 8) : 0;
        const int64_t out_floats = (int64_t)Bt * nt * (ci == 0 ? d : (ci == 1 ? d + d * d + d : d + rj));
        float *X = nullptr, *out = nullptr;
        double *lat = nullptr;
        if (hipMalloc(&X, sizeof(float) * d * nt) != hipSuccess ||
            hipMalloc(&out, sizeof(float) * out_floats) != hipSuccess ||
            hipMalloc(&lat, sizeof(double) * 2 * Bt * r) != hipSuccess) {
            (void)hipFree(X);
            (void)hipFree(out);
            (void)hipFree(lat);
            return MR_ENOMEM;
        }
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (hipMemsetAsync(X, 0, sizeof(float) * d * nt, st) != hipSuccess ||
            hipMemsetAsync(lat, 0, sizeof(double) * 2 * Bt * r, st) != hipSuccess ||
            hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
            rc = MR_EDEVICE;
        DecIO io{};
        io.B = Bt;
        io.n_ref = nt;
        io.n = nt;
        io.X = X;
        io.idx_div = 1;
        io.xhat = lat;
        io.vhat = lat + (size_t)Bt * r;
        io.x = out;
        if (ci == 1) {
            io.F = out + (size_t)Bt * d * nt;
            io.v = io.F + (size_t)Bt * d * d * nt;
        } else if (ci == 2) {
            io.Jz = out + (size_t)Bt * d * nt;
        }
        const StreamSpec ss = spec_of(cfg, d);
        const int cand[5] = {DEC_COL, DEC_COL_NP2, DEC_COL_NP4, DEC_ROWS, DEC_REG};
        float best = 0.0f;
        int best_v = DEC_COL;
        for (int k = 0; k < 5 && rc == MR_OK; ++k) {
            const int v = cand[k];
            if (cfg != 1 && (v == DEC_COL_NP2 || v == DEC_COL_NP4)) continue;
            if (v == DEC_REG && !shape_available(dec, cfg, v)) continue;
            rc = launch_cfg(dec, cfg, ss, io, st, v);   // warm-up (and LDS attribute)
            if (rc != MR_OK) break;
            if (hipEventRecord(e0, st) != hipSuccess) rc = MR_EDEVICE;
            for (int q = 0; q < reps && rc == MR_OK; ++q) rc = launch_cfg(dec, cfg, ss, io, st, v);
            if (rc == MR_OK && (hipEventRecord(e1, st) != hipSuccess ||
                                hipEventSynchronize(e1) != hipSuccess))
                rc = MR_EDEVICE;
            float ms = 0.0f;
            if (rc == MR_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = MR_EDEVICE;
            if (rc == MR_OK && (k == 0 || ms < best)) {
                best = ms;
                best_v = v;
            }
        }
        if (rc == MR_OK) dec->tuned[ci][size_bucket(pts)] = (int8_t)best_v;
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipStreamSynchronize(st);
        (void)hipFree(X);
        (void)hipFree(out);
        (void)hipFree(lat);
    }
    return rc;
}

}  // namespace mr

extern "C" int32_t rom_decoder_autotune(mr_decoder *dec, int32_t B, int64_t n, int32_t cfg_mask,
                                        int32_t reps, void *stream)
{
    return decoder_autotune(dec, B, n, cfg_mask, reps, as_stream(stream));
}

extern "C" int32_t rom_decoder_shape(const mr_decoder *dec, int32_t cfg, int32_t B, int64_t n)
{
    if (!dec || B < 1 || n < 0 || (cfg != 1 && cfg != 5 && cfg != 9)) return MR_EINVAL;
    if (dec->nh == 0) return DEC_COL;
    return dec_variant(dec, cfg, (int64_t)B * n);
}

extern "C" int32_t rom_decoder_set_shape(mr_decoder *dec, int32_t cfg, int32_t B, int64_t n,
                                         int32_t shape)
{
    if (!dec || B < 1 || n < 1 || (cfg != 1 && cfg != 5 && cfg != 9)) return MR_EINVAL;
    if (!shape_available(dec, cfg, shape)) return MR_EINVAL;
    dec->tuned[cfg_index(cfg)][size_bucket((int64_t)B * n)] = (int8_t)shape;
    return MR_OK;
}

extern "C" int32_t rom_decoder_create(int32_t d, int32_t r, int32_t width, int32_t n_hidden,
                                      const float *params, const float *in_min,
                                      const float *in_max, const float *out_mean,
                                      const float *out_std, int32_t output_mode,
                                      int32_t precision, mr_decoder **out)
{
    if (!out || !params || !in_min || !in_max || !out_mean || !out_std) return MR_EINVAL;
    if ((d != 2 && d != 3) || r < 1 || r > 32 || width < 1 || width > 128 || n_hidden < 0 ||
        n_hidden > 8)
        return MR_EINVAL;
    if (output_mode != MR_OUT_POSITION && output_mode != MR_OUT_DISPLACEMENT) return MR_EINVAL;
    if (precision != MR_PREC_FP32 && precision != MR_PREC_BF16) return MR_EINVAL;
    for (int a = 0; a < d; ++a)
        if (!(in_max[a] > in_min[a])) return MR_EINVAL;
    // padded width: a power of two >= 16 (>= 32 with bf16, whose matrix-core
    // step consumes 32 units of k); padded units have zero weights and bias,
    // so they stay exactly zero through ELU and contribute nothing
    int W = precision == MR_PREC_BF16 ? 32 : 16;
    while (W < width) W *= 2;
    mr_decoder *dec = (mr_decoder *)calloc(1, sizeof(mr_decoder));
    if (!dec) return MR_ENOMEM;
    memset(dec->tuned, 0xff, sizeof(dec->tuned));   // nothing tuned yet
    dec->d = d;
    dec->r = r;
    dec->width = width;
    dec->W = W;
    dec->nh = n_hidden;
    dec->mode = output_mode;
    dec->prec = precision;
    dec->n_params = unpadded_count(d, r, width, n_hidden);
    for (int a = 0; a < 3; ++a) {
        if (a < d) {
            dec->scale[a] = 2.0f / (in_max[a] - in_min[a]);
            dec->shift[a] = -2.0f * in_min[a] / (in_max[a] - in_min[a]) - 1.0f;
            dec->mean[a] = out_mean[a];
            dec->stdv[a] = out_std[a];
        } else {
            dec->scale[a] = dec->shift[a] = dec->mean[a] = dec->stdv[a] = 0.0f;
        }
    }
    size_t off = 0;
    auto take = [&](size_t nfl) {
        size_t o = off;
        off += (nfl + 63) & ~(size_t)63;
        return o;
    };
    dec->oW0 = take((size_t)W * (d + r));
    dec->ob0 = take(W);
    const size_t nhh = n_hidden > 0 ? (size_t)(n_hidden - 1) : 0;
    dec->oWh = take(nhh * W * W + 1);
    dec->obh = take(nhh * W + 1);
    dec->oWL = take((size_t)d * W);
    dec->obL = take(d);
    if (hipMalloc(&dec->dev, off * sizeof(float)) != hipSuccess ||
        hipMalloc(&dec->hid_bf16, (nhh * W * W + 8) * sizeof(uint16_t)) !=
            hipSuccess ||
        hipMalloc(&dec->staging, dec->n_params * sizeof(float)) != hipSuccess) {
        rom_decoder_destroy(dec);
        return MR_ENOMEM;
    }
    if (hipMemset(dec->dev, 0, off * sizeof(float)) != hipSuccess) {
        rom_decoder_destroy(dec);
        return MR_EDEVICE;
    }
    int32_t rc = rom_decoder_set_params(dec, params, 0, nullptr);
    if (rc != MR_OK) {
        rom_decoder_destroy(dec);
        return rc;
    }
    *out = dec;
    return MR_OK;
}

extern "C" void rom_decoder_destroy(mr_decoder *dec)
{
    if (!dec) return;
    if (dec->dev) (void)hipFree(dec->dev);
    if (dec->hid_bf16) (void)hipFree(dec->hid_bf16);
    if (dec->staging) (void)hipFree(dec->staging);
    free(dec);
}

static bool dec_io_ok(const mr_decoder *dec, int32_t B, int64_t n_ref, const float *X, int64_t n,
                      const int32_t *idx, const double *xhat)
{
    if (!dec || B < 1 || B > 65535 || n_ref < 0 || n < 0 || !X || !xhat) return false;
    if (!idx && n != n_ref) return false;
    return true;
}

extern "C" int32_t rom_decode(const mr_decoder *dec, int32_t B, int64_t n_ref, const float *X,
                              int64_t n, const int32_t *idx, const double *xhat, float *x_out,
                              void *stream)
{
    if (!dec_io_ok(dec, B, n_ref, X, n, idx, xhat) || !x_out) return MR_EINVAL;
    if (n == 0) return MR_OK;
    DecIO io{};
    io.B = B;
    io.n_ref = n_ref;
    io.n = n;
    io.X = X;
    io.idx = idx;
    io.idx_per_inst = 0;
    io.idx_div = 1;
    io.xhat = xhat;
    io.x = x_out;
    StreamSpec ss{};
    ss.kind[0] = SK_PRIMAL;
    return launch_cfg(dec, 1, ss, io, as_stream(stream));
}

namespace mr {
int32_t decode_jac_ex(const mr_decoder *dec, int32_t B, int64_t n_ref, const float *X, int64_t n,
                      const int32_t *idx, int32_t idx_per_instance, const int32_t *n_inst,
                      const double *xhat, const double *vhat, float *x, float *F, float *v,
                      float *Jz, hipStream_t st, int disp_only, int64_t x_stride, int force_fp32)
{
    if (n == 0) return MR_OK;
    DecIO io{};
    io.x_stride = x_stride;
    io.n_inst = n_inst;
    io.disp_only = disp_only;
    io.B = B;
    io.n_ref = n_ref;
    io.n = n;
    io.X = X;
    io.idx = idx;
    io.idx_per_inst = idx_per_instance ? 1 : 0;
    io.idx_div = idx_per_instance > 1 ? idx_per_instance : 1;
    io.xhat = xhat;
    io.vhat = vhat;
    io.x = x;
    io.F = F;
    io.v = v;
    int32_t rc;
    bool wrote_x = false;
    if (F || v) {
        StreamSpec ss{};
        ss.kind[0] = SK_PRIMAL;
        for (int a = 0; a < 3; ++a) {
            ss.kind[1 + a] = (a < dec->d && F) ? SK_SPATIAL : SK_ZERO;
            ss.arg[1 + a] = a;
        }
        ss.kind[4] = v ? SK_VELOCITY : SK_ZERO;
        rc = launch_cfg(dec, (F && !v) ? 4 : 5, ss, io, st, -1, force_fp32);
        if (rc != MR_OK) return rc;
        wrote_x = true;
    }
    if (Jz) {
        io.Jz = Jz;
        io.F = nullptr;
        io.v = nullptr;
        // one launch: block z takes latent columns 8z .. 8z + 7
        StreamSpec ss{};
        ss.kind[0] = SK_PRIMAL;
        for (int q = 0; q < 8; ++q) {
            ss.kind[1 + q] = SK_LATENT;
            ss.arg[1 + q] = q;
        }
        ss.zk = 8;
        io.x = wrote_x ? nullptr : x;
        rc = launch_cfg(dec, 9, ss, io, st, -1, force_fp32);
        if (rc != MR_OK) return rc;
        wrote_x = wrote_x || x;
    }
    if (!wrote_x && x) {
        StreamSpec ss{};
        ss.kind[0] = SK_PRIMAL;
        io.x = x;
        io.Jz = nullptr;
        return launch_cfg(dec, 1, ss, io, st, -1, force_fp32);
    }
    return MR_OK;
}
}  // namespace mr

extern "C" int32_t rom_decode_jac(const mr_decoder *dec, int32_t B, int64_t n_ref, const float *X,
                                  int64_t n, const int32_t *idx, int32_t idx_per_instance,
                                  const double *xhat, const double *vhat, float *x, float *F,
                                  float *v, float *Jz, void *stream)
{
    if (!dec_io_ok(dec, B, n_ref, X, n, idx, xhat)) return MR_EINVAL;
    if (idx_per_instance && !idx) return MR_EINVAL;
    if (idx_per_instance < 0 || (idx_per_instance > 1 && B % idx_per_instance != 0)) return MR_EINVAL;
    if (v && !vhat) return MR_EINVAL;
    return decode_jac_ex(dec, B, n_ref, X, n, idx, idx_per_instance, nullptr, xhat, vhat, x, F, v,
                         Jz, as_stream(stream));
}

namespace mr {
int decoder_dim(const mr_decoder *dec) { return dec->d; }
int decoder_latent(const mr_decoder *dec) { return dec->r; }
int decoder_output_mode(const mr_decoder *dec) { return dec->mode; }
int decoder_precision(const mr_decoder *dec) { return dec->prec; }
float decoder_out_scale(const mr_decoder *dec)
{
    float m = 0.0f;
    for (int a = 0; a < dec->d; ++a) m = fmaxf(m, fabsf(dec->stdv[a]));
    return m;
}
}  // namespace mr
