// Measurement aid, not part of the method: a dense bf16 matrix-core loop
// that gives the MFMA rate this part sustains, reported beside the nominal
// peak when the decoder's throughput is set against its roofline.
#include "internal.h"

namespace mr {

typedef __bf16 bf16x8p __attribute__((ext_vector_type(8)));
typedef float f32x4p __attribute__((ext_vector_type(4)));

// every wave runs `iters` rounds of 8 independent 16x16x32 bf16 products
// (16,384 FLOP each) on register operands, then stores one value per lane
__global__ void __launch_bounds__(256) mfma_probe_kernel(int32_t iters, float *sink)
{
    const int lane = threadIdx.x & 63;
    bf16x8p a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        a[e] = (__bf16)(1.0f + 0.001f * (float)(lane + e));
        b[e] = (__bf16)(0.5f - 0.001f * (float)e);
    }
    f32x4p acc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = f32x4p{0.0f, 0.0f, 0.0f, 0.0f};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < 8; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    sink[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace mr

using namespace mr;

extern "C" int32_t mr_mfma_probe(int32_t blocks, int32_t iters, float *sink, void *stream)
{
    if (blocks < 1 || iters < 1 || !sink) return MR_EINVAL;
    mfma_probe_kernel<<<(unsigned)blocks, 256, 0, as_stream(stream)>>>(iters, sink);
    MR_LAUNCH_CHECK();
    return MR_OK;
}
