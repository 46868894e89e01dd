// Encoder network on gfx950 (paper Section 4.1, layer shapes of Table 1):
// concatenated point positions -> single-channel 1D convolutions (kernel 6,
// stride 2, ELU) down to the shortest length not below 32 -> dense 32
// (ELU) -> dense r.  Forward and backward passes for training.
//
// Every layer is streaming work: a convolution reads its input once and
// writes half as many outputs (6 multiply-adds each), so the encoder of a
// 65,536-point snapshot moves about 2 x 0.8 MB and does about 2.4 MFLOP;
// it is bound by HBM bandwidth and launch latency, not by arithmetic, and
// runs on the vector units in fp32.  One thread per output element; the
// stride-2 windows of neighbouring threads overlap, so each input element
// is fetched from HBM once and re-read from the caches.  The weight
// gradients are reduced per block in LDS and added with one atomic per
// parameter and block.
#include "internal.h"

#include <vector>

namespace mr {

constexpr int ENC_K = 6, ENC_S = 2, ENC_MIN = 32, ENC_H = 32;
constexpr int ENC_TB = 256;

struct EncLayout {
    std::vector<int64_t> len;   // len[0] = input length, len[l + 1] = output of conv l
    int nc;                     // convolutions
    int64_t dc;                 // d_conv
    int64_t n_params, act_floats, work_floats;
    int64_t plane_floats, dense_floats, conv_blocks;
    std::vector<int64_t> act_off;   // offset of conv l's output in a frame's record
    int64_t h1_off;
};

bool enc_layout(int64_t in_len, int r, EncLayout &L)
{
    if (in_len < ENC_MIN || r < 1 || r > 64) return false;
    L.len.assign(1, in_len);
    for (;;) {
        const int64_t cur = L.len.back();
        const int64_t nxt = (cur - ENC_K) / ENC_S + 1;
        if (cur < ENC_K || nxt < ENC_MIN) break;
        L.len.push_back(nxt);
    }
    L.nc = (int)L.len.size() - 1;
    L.dc = L.len.back();
    L.n_params = (int64_t)L.nc * (ENC_K + 1) + ENC_H * L.dc + ENC_H + (int64_t)r * ENC_H + r;
    L.act_off.resize(L.nc);
    int64_t o = 0;
    for (int l = 0; l < L.nc; ++l) {
        L.act_off[l] = o;
        o += L.len[l + 1];
    }
    L.h1_off = o;
    L.act_floats = o + ENC_H;
    // two gradient planes of the longest convolution output (or of d_conv),
    // then (reproducible mode) the frame's dense-layer gradient and the
    // per-block convolution partial sums of its longest layer
    const int64_t l1 = L.nc > 0 ? L.len[1] : L.dc;
    L.plane_floats = l1;
    L.dense_floats = ENC_H * L.dc + ENC_H + (int64_t)r * ENC_H + r;
    L.conv_blocks = (l1 + ENC_TB - 1) / ENC_TB;
    L.work_floats = 2 * l1 + L.dense_floats + (ENC_K + 1) * L.conv_blocks;
    return true;
}

__device__ __forceinline__ float elu_f(float s) { return s > 0.0f ? s : expm1f(s); }
// ELU' from the activation: 1 where positive, else exp(s) = elu(s) + 1
__device__ __forceinline__ float elu_prime_a(float a) { return a > 0.0f ? 1.0f : a + 1.0f; }

struct EncNorm {
    int d;
    float scale[3], shift[3];
};

// element j of layer l's input for frame f: the normalised position
// coordinate (first layer) or the previous activation
__device__ __forceinline__ float enc_in(const float *in, int64_t j, const EncNorm &nm, bool first)
{
    if (!first) return in[j];
    const int a = (int)(j % nm.d);
    return nm.scale[a] * in[j] + nm.shift[a];
}

// y[f][i] = elu(b + sum_k w[k] x[f][2 i + k]); grid (ceil(Lout / TB), n)
__global__ void __launch_bounds__(ENC_TB) enc_conv_fwd_kernel(
    const float *x, const int32_t *frame_idx, int64_t in_stride, const float *act_prev,
    int64_t act_stride, int64_t Lin, int64_t Lout, const float *wb, EncNorm nm, float *out)
{
    const int f = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * ENC_TB + threadIdx.x;
    if (i >= Lout) return;
    const bool first = act_prev == nullptr;
    const float *in = first ? x + (int64_t)(frame_idx ? frame_idx[f] : f) * in_stride
                            : act_prev + (int64_t)f * act_stride;
    float s = wb[ENC_K];
#pragma unroll
    for (int k = 0; k < ENC_K; ++k) s = fmaf(wb[k], enc_in(in, ENC_S * i + k, nm, first), s);
    (void)Lin;
    out[(int64_t)f * act_stride + i] = elu_f(s);
}

// the two dense layers of one frame: h1 = elu(W1 a + b1), z = W2 h1 + b2
__global__ void __launch_bounds__(64) enc_dense_fwd_kernel(float *act, int64_t act_stride,
                                                           int64_t a_off, int64_t h1_off, int dc,
                                                           int r, const float *W1, const float *b1,
                                                           const float *W2, const float *b2,
                                                           float *z)
{
    __shared__ float a[2 * ENC_MIN + ENC_K];
    __shared__ float h[ENC_H];
    const int f = blockIdx.x, t = threadIdx.x;
    float *rec = act + (int64_t)f * act_stride;
    for (int i = t; i < dc; i += 64) a[i] = rec[a_off + i];
    __syncthreads();
    if (t < ENC_H) {
        float s = b1[t];
        for (int i = 0; i < dc; ++i) s = fmaf(W1[t * dc + i], a[i], s);
        h[t] = elu_f(s);
        rec[h1_off + t] = h[t];
    }
    __syncthreads();
    if (t < r) {
        float s = b2[t];
        for (int o = 0; o < ENC_H; ++o) s = fmaf(W2[t * ENC_H + o], h[o], s);
        z[(int64_t)f * r + t] = s;
    }
}

// backward of the dense layers for one frame: parameter gradients (atomics
// per frame) and the gradient of the last convolution's output
// fgrad (nullable): this frame's gradient record (W1, b1, W2, b2 layout) at
// fgrad + f fstride, written instead of the atomics (reproducible mode)
__global__ void __launch_bounds__(64) enc_dense_bwd_kernel(const float *act, int64_t act_stride,
                                                           int64_t a_off, int64_t h1_off, int dc,
                                                           int r, const float *W1, const float *W2,
                                                           const float *dz, float *gW1, float *gb1,
                                                           float *gW2, float *gb2, float *da,
                                                           int64_t da_stride, float *fgrad,
                                                           int64_t fstride)
{
    __shared__ float a[2 * ENC_MIN + ENC_K];
    __shared__ float ds1[ENC_H];
    __shared__ float g[64];
    const int f = blockIdx.x, t = threadIdx.x;
    const float *rec = act + (int64_t)f * act_stride;
    for (int i = t; i < dc; i += 64) a[i] = rec[a_off + i];
    if (t < r) g[t] = dz[(int64_t)f * r + t];
    if (fgrad) {
        // the frame's own record: plain stores, summed over frames in order
        float *o = fgrad + (int64_t)f * fstride;
        gW1 = o;
        gb1 = o + ENC_H * dc;
        gW2 = gb1 + ENC_H;
        gb2 = gW2 + r * ENC_H;
    }
    __syncthreads();
    if (t < ENC_H) {
        const float h = rec[h1_off + t];
        float s = 0.0f;
        for (int q = 0; q < r; ++q) {
            s = fmaf(W2[q * ENC_H + t], g[q], s);
            if (fgrad)
                gW2[q * ENC_H + t] = g[q] * h;
            else
                atomicAdd(gW2 + q * ENC_H + t, g[q] * h);
        }
        ds1[t] = s * elu_prime_a(h);
        if (fgrad)
            gb1[t] = ds1[t];
        else
            atomicAdd(gb1 + t, ds1[t]);
    }
    if (t < r) {
        if (fgrad)
            gb2[t] = g[t];
        else
            atomicAdd(gb2 + t, g[t]);
    }
    __syncthreads();
    for (int i = t; i < dc; i += 64) {
        float s = 0.0f;
        for (int o = 0; o < ENC_H; ++o) {
            s = fmaf(W1[o * dc + i], ds1[o], s);
            if (fgrad)
                gW1[o * dc + i] = ds1[o] * a[i];
            else
                atomicAdd(gW1 + o * dc + i, ds1[o] * a[i]);
        }
        da[(int64_t)f * da_stride + i] = s;
    }
}

// input gradient of a convolution: dx[j] = sum over the outputs i with
// 2 i + k = j of w[k] ds[i], ds = da elu'(y); grid (ceil(Lin / TB), n)
__global__ void __launch_bounds__(ENC_TB) enc_conv_bwd_data_kernel(
    const float *da, int64_t da_stride, const float *y, int64_t y_stride, int64_t Lin,
    int64_t Lout, const float *wb, float *dx, int64_t dx_stride)
{
    const int f = blockIdx.y;
    const int64_t j = (int64_t)blockIdx.x * ENC_TB + threadIdx.x;
    if (j >= Lin) return;
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < ENC_K; ++k) {
        const int64_t q = j - k;
        if (q < 0 || (q & 1)) continue;
        const int64_t i = q >> 1;
        if (i >= Lout) continue;
        const float yy = y[(int64_t)f * y_stride + i];
        s = fmaf(wb[k], da[(int64_t)f * da_stride + i] * elu_prime_a(yy), s);
    }
    dx[(int64_t)f * dx_stride + j] = s;
}

// weight and bias gradients of a convolution: sum over frames and outputs
// of ds[i] x[2 i + k] and ds[i]; grid (ceil(Lout / TB), n)
__global__ void __launch_bounds__(ENC_TB) enc_conv_bwd_weight_kernel(
    const float *x, const int32_t *frame_idx, int64_t in_stride, const float *act_prev,
    int64_t act_stride, const float *da, int64_t da_stride, const float *y, int64_t Lout,
    EncNorm nm, float *gwb, float *part)
{
    __shared__ float red[ENC_K + 1][ENC_TB / 64];
    const int f = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * ENC_TB + threadIdx.x;
    float v[ENC_K + 1];
#pragma unroll
    for (int k = 0; k <= ENC_K; ++k) v[k] = 0.0f;
    if (i < Lout) {
        const bool first = act_prev == nullptr;
        const float *in = first ? x + (int64_t)(frame_idx ? frame_idx[f] : f) * in_stride
                                : act_prev + (int64_t)f * act_stride;
        const float ds = da[(int64_t)f * da_stride + i] * elu_prime_a(y[(int64_t)f * act_stride + i]);
#pragma unroll
        for (int k = 0; k < ENC_K; ++k) v[k] = ds * enc_in(in, ENC_S * i + k, nm, first);
        v[ENC_K] = ds;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k <= ENC_K; ++k) {
        float s = v[k];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off);
        if (lane == 0) red[k][wv] = s;
    }
    __syncthreads();
    if (threadIdx.x <= ENC_K) {
        float s = 0.0f;
        for (int w = 0; w < ENC_TB / 64; ++w) s += red[threadIdx.x][w];
        if (part)   // block (x, frame y) -> slot y gridDim.x + x
            part[((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * (ENC_K + 1) + threadIdx.x] = s;
        else
            atomicAdd(gwb + threadIdx.x, s);
    }
}

// grad[k] += sum over many slots of part[slot][k] for a few k: one block per
// k, thread t sums slots t, t + 256, ... in order, then a fixed tree
// (reproducible, and parallel over the tens of thousands of block partials)
__global__ void __launch_bounds__(256) enc_slot_tree_kernel(int64_t nslots, int64_t stride,
                                                            const float *part, float *grad)
{
    __shared__ float red[256];
    const int k = blockIdx.x;
    float s = 0.0f;
    for (int64_t q = threadIdx.x; q < nslots; q += 256) s += part[q * stride + k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) grad[k] += red[0];
}

// grad[k] += sum over the slots of part[slot][k], in slot order
__global__ void enc_slot_reduce_kernel(int64_t width, int64_t nslots, int64_t stride,
                                       const float *part, float *grad)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= width) return;
    float s = 0.0f;
    for (int64_t q = 0; q < nslots; ++q) s += part[q * stride + k];
    grad[k] += s;
}

__global__ void enc_fill_kernel(float *a, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0.0f;
}

bool enc_norm(int d, const float *in_min, const float *in_max, EncNorm &nm)
{
    if ((d != 2 && d != 3) || !in_min || !in_max) return false;
    nm.d = d;
    for (int a = 0; a < 3; ++a) {
        if (a < d) {
            if (!(in_max[a] > in_min[a])) return false;
            nm.scale[a] = 2.0f / (in_max[a] - in_min[a]);
            nm.shift[a] = -2.0f * in_min[a] / (in_max[a] - in_min[a]) - 1.0f;
        } else {
            nm.scale[a] = nm.shift[a] = 0.0f;
        }
    }
    return true;
}

}  // namespace mr

using namespace mr;

extern "C" int32_t rom_encoder_layout(int64_t in_len, int32_t r, int32_t *n_conv, int64_t *d_conv,
                                      int64_t *n_params, int64_t *act_floats,
                                      int64_t *work_floats)
{
    EncLayout L;
    if (!enc_layout(in_len, r, L)) return MR_EINVAL;
    if (n_conv) *n_conv = L.nc;
    if (d_conv) *d_conv = L.dc;
    if (n_params) *n_params = L.n_params;
    if (act_floats) *act_floats = L.act_floats;
    if (work_floats) *work_floats = L.work_floats;
    return MR_OK;
}

extern "C" int32_t rom_encoder_forward(int32_t d, int32_t r, int64_t in_len, int32_t n,
                                       const float *x, const int32_t *frame_idx,
                                       const float *params, const float *in_min,
                                       const float *in_max, float *act, float *z, void *stream)
{
    EncLayout L;
    EncNorm nm;
    if (!enc_layout(in_len, r, L) || !enc_norm(d, in_min, in_max, nm) || in_len % d != 0 ||
        n < 0 || n > 65535 || (n > 0 && (!x || !params || !act || !z)))
        return MR_EINVAL;
    if (n == 0) return MR_OK;
    hipStream_t st = as_stream(stream);
    const float *prev = nullptr;
    for (int l = 0; l < L.nc; ++l) {
        const int64_t Lout = L.len[l + 1];
        dim3 grid((unsigned)ceil_div(Lout, ENC_TB), (unsigned)n);
        enc_conv_fwd_kernel<<<grid, ENC_TB, 0, st>>>(
            x, frame_idx, in_len, prev, L.act_floats, L.len[l], Lout, params + l * (ENC_K + 1), nm,
            act + L.act_off[l]);
        prev = act + L.act_off[l];
    }
    MR_LAUNCH_CHECK();
    const float *W1 = params + (int64_t)L.nc * (ENC_K + 1);
    const float *b1 = W1 + ENC_H * L.dc;
    const float *W2 = b1 + ENC_H;
    const float *b2 = W2 + (int64_t)r * ENC_H;
    if (L.nc == 0) return MR_EINVAL;   // the dense layers read the last convolution's output
    enc_dense_fwd_kernel<<<(unsigned)n, 64, 0, st>>>(act, L.act_floats, L.act_off[L.nc - 1],
                                                     L.h1_off, (int)L.dc, r, W1, b1, W2, b2, z);
    MR_LAUNCH_CHECK();
    return MR_OK;
}

extern "C" int32_t rom_encoder_backward(int32_t d, int32_t r, int64_t in_len, int32_t n,
                                        const float *x, const int32_t *frame_idx,
                                        const float *params, const float *in_min,
                                        const float *in_max, const float *act, const float *dz,
                                        float *grad, float *work, int32_t deterministic,
                                        void *stream)
{
    EncLayout L;
    EncNorm nm;
    if (!enc_layout(in_len, r, L) || !enc_norm(d, in_min, in_max, nm) || in_len % d != 0 ||
        n < 0 || n > 65535 || L.nc == 0 || !grad ||
        (n > 0 && (!x || !params || !act || !dz || !work)))
        return MR_EINVAL;
    hipStream_t st = as_stream(stream);
    enc_fill_kernel<<<(unsigned)std::min<int64_t>(ceil_div(L.n_params, 256), 1024), 256, 0, st>>>(
        grad, L.n_params);
    MR_LAUNCH_CHECK();
    if (n == 0) return MR_OK;
    const float *W1 = params + (int64_t)L.nc * (ENC_K + 1);
    const float *W2 = W1 + ENC_H * L.dc + ENC_H;
    float *gW1 = grad + (int64_t)L.nc * (ENC_K + 1);
    float *gb1 = gW1 + ENC_H * L.dc;
    float *gW2 = gb1 + ENC_H;
    float *gb2 = gW2 + (int64_t)r * ENC_H;
    // two gradient planes per frame, alternating between layers; then the
    // per-frame dense gradients and the convolution block partials
    const int64_t ws = L.plane_floats;
    float *plane[2] = {work, work + (int64_t)n * ws};
    float *fgrad = deterministic ? work + 2 * (int64_t)n * ws : nullptr;
    float *cpart = deterministic ? fgrad + (int64_t)n * L.dense_floats : nullptr;
    int cur = 0;
    enc_dense_bwd_kernel<<<(unsigned)n, 64, 0, st>>>(act, L.act_floats, L.act_off[L.nc - 1],
                                                     L.h1_off, (int)L.dc, r, W1, W2, dz, gW1, gb1,
                                                     gW2, gb2, plane[cur], ws, fgrad,
                                                     L.dense_floats);
    if (fgrad)
        enc_slot_reduce_kernel<<<(unsigned)ceil_div(L.dense_floats, 256), 256, 0, st>>>(
            L.dense_floats, n, L.dense_floats, fgrad, gW1);
    MR_LAUNCH_CHECK();
    for (int l = L.nc - 1; l >= 0; --l) {
        const int64_t Lin = L.len[l], Lout = L.len[l + 1];
        const float *wb = params + l * (ENC_K + 1);
        const float *y = act + L.act_off[l];
        const float *prev = l > 0 ? act + L.act_off[l - 1] : nullptr;
        dim3 gw((unsigned)ceil_div(Lout, ENC_TB), (unsigned)n);
        enc_conv_bwd_weight_kernel<<<gw, ENC_TB, 0, st>>>(x, frame_idx, in_len, prev, L.act_floats,
                                                          plane[cur], ws, y, Lout, nm,
                                                          grad + l * (ENC_K + 1), cpart);
        if (cpart)
            enc_slot_tree_kernel<<<ENC_K + 1, 256, 0, st>>>((int64_t)gw.x * n, ENC_K + 1, cpart,
                                                            grad + l * (ENC_K + 1));
        if (l > 0) {
            dim3 gd((unsigned)ceil_div(Lin, ENC_TB), (unsigned)n);
            enc_conv_bwd_data_kernel<<<gd, ENC_TB, 0, st>>>(plane[cur], ws, y, L.act_floats, Lin,
                                                            Lout, wb, plane[cur ^ 1], ws);
            cur ^= 1;
        }
        MR_LAUNCH_CHECK();
    }
    return MR_OK;
}
