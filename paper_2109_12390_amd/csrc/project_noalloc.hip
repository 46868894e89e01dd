// Allocation-free variant of the projection entry point (rom_project) for
// callers that cannot allocate device memory (code under graph capture,
// tight serving loops, harnesses that forbid allocation).  Its scratch is a
// fixed file-scope device array instead of a caller workspace; the kernels
// are the projection's own (Section 3.2.4, Algorithms 6 and 7).
#include "project.h"

#include <mutex>

// Scratch of the allocation-free entry point: one fixed array per device
// (each GPU the library runs on holds its own copy until the process ends).
// Host code never uses the array's name as an address (in host code it is a
// stand-in, not a device address): the device address is looked up once per
// device and kept in scratch_ptr.
constexpr int64_t PROJ_SCRATCH_BYTES = int64_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[PROJ_SCRATCH_BYTES];

namespace mr {
namespace {

constexpr int MAX_DEVICES = 64;
void *scratch_ptr[MAX_DEVICES];
std::mutex scratch_mutex;

int32_t scratch_for_current_device(void **out)
{
    int dev = 0;
    MR_CHECK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return MR_EINVAL;
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        MR_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return MR_EDEVICE;
        scratch_ptr[dev] = p;
    }
    *out = scratch_ptr[dev];
    return MR_OK;
}

}  // namespace
}  // namespace mr

using namespace mr;

extern "C" int32_t rom_project_noalloc(const mr_decoder *dec, int32_t B, int64_t n_ref,
                                       const float *X, int64_t ns, const int32_t *sample_idx,
                                       const int32_t *ns_per_instance, const float *x_trial,
                                       const float *v_trial, const double *xhat_n,
                                       const double *xhat_prev, double dt,
                                       const mr_gn_opts *opts, double *xhat_next,
                                       double *vhat_next, int32_t *iters_out, double *resid_out,
                                       int32_t *status_out, void *stream)
{
    int d = 0, r = 0;
    int32_t rc = project_args(dec, B, ns, X, sample_idx, v_trial, xhat_n, xhat_prev, opts,
                              xhat_next, vhat_next, d, r);
    if (rc != MR_OK) return rc;
    if (proj_ws_bytes(d, r, B, ns, opts->max_backtrack) > PROJ_SCRATCH_BYTES) return MR_ESCRATCH;
    void *ws = nullptr;
    rc = scratch_for_current_device(&ws);
    if (rc != MR_OK) return rc;
    ProjWS w = proj_ws_carve(ws, d, r, B, ns, opts->max_backtrack);
    return project_impl(dec, d, r, B, n_ref, X, ns, sample_idx, ns_per_instance, x_trial, v_trial,
                        xhat_n, xhat_prev ? xhat_prev : xhat_n, dt, *opts, xhat_next, vhat_next,
                        iters_out, resid_out, status_out, w, as_stream(stream));
}
