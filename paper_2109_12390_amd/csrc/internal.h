// Internal helpers of libmpmrom (gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mpmrom.h"

#define MR_CHECK_HIP(expr)                         \
    do {                                           \
        hipError_t _e = (expr);                    \
        if (_e != hipSuccess) return MR_EDEVICE;   \
    } while (0)

#define MR_LAUNCH_CHECK() MR_CHECK_HIP(hipGetLastError())

namespace mr {

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Lame parameters of (E, nu).
struct Lame {
    float mu, la;
};
__host__ __device__ inline Lame lame_of(float E, float nu)
{
    Lame l;
    l.mu = E / (2.0f * (1.0f + nu));
    l.la = E * nu / ((1.0f + nu) * (1.0f - 2.0f * nu));
    return l;
}

// Grid description copied by value into kernels.
struct GridK {
    int n0, n1, n2;
    float dx, inv_dx;
    int bound, floor_mode;
    float mu_f;
    float g0, g1, g2;
};

inline bool grid_from_desc(const mr_grid *g, GridK &k)
{
    if (!g || (g->dim != 2 && g->dim != 3)) return false;
    if (g->n[0] < 3 || g->n[1] < 3 || (g->dim == 3 && g->n[2] < 3)) return false;
    if (!(g->dx > 0.0f)) return false;
    k.n0 = g->n[0];
    k.n1 = g->n[1];
    k.n2 = g->dim == 3 ? g->n[2] : 1;
    k.dx = g->dx;
    k.inv_dx = 1.0f / g->dx;
    k.bound = g->bound;
    k.floor_mode = g->floor_mode;
    k.mu_f = g->mu_friction;
    k.g0 = g->gravity[0];
    k.g1 = g->gravity[1];
    k.g2 = g->dim == 3 ? g->gravity[2] : 0.0f;
    return true;
}

inline int64_t grid_nodes(const GridK &k) { return (int64_t)k.n0 * k.n1 * k.n2; }

// Quadratic B-spline weights of the three stencil nodes and their
// derivatives (already divided by dx) for one dimension.  Returns the base
// node; `ok` is cleared when the stencil leaves [0, n-1] or x is not finite.
__device__ __forceinline__ int bspline(float x, float inv_dx, int n, float w[3],
                                       float dw[3], bool &ok)
{
    float s = x * inv_dx;
    float bf = floorf(s - 0.5f);
    float f = s - bf;
    int b = (int)bf;
    ok = ok && (bf >= 0.0f) && (bf + 2.0f <= (float)(n - 1));  // false for NaN
    float a = 1.5f - f, c = f - 1.0f, e = f - 0.5f;
    w[0] = 0.5f * a * a;
    w[1] = 0.75f - c * c;
    w[2] = 0.5f * e * e;
    dw[0] = -a * inv_dx;
    dw[1] = -2.0f * c * inv_dx;
    dw[2] = e * inv_dx;
    return b;
}

__device__ __forceinline__ void raise_flag(int32_t *flag, int32_t bits)
{
    if (flag) atomicOr(flag, bits);
}

}  // namespace mr
