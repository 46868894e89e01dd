// Internal interfaces shared by the projection and the reduced-order step.
#pragma once

#include "internal.h"

namespace mr {

int decoder_dim(const mr_decoder *dec);
int decoder_latent(const mr_decoder *dec);
int decoder_output_mode(const mr_decoder *dec);
int decoder_precision(const mr_decoder *dec);
float decoder_out_scale(const mr_decoder *dec);   // largest output standard deviation
int32_t decoder_autotune(const mr_decoder *dec, int32_t B, int64_t n, int32_t cfg_mask,
                         int32_t reps, hipStream_t st);
int32_t decode_jac_ex(const mr_decoder *dec, int32_t B, int64_t n_ref, const float *X, int64_t n,
                      const int32_t *idx, int32_t idx_per_instance, const int32_t *n_inst,
                      const double *xhat, const double *vhat, float *x, float *F, float *v,
                      float *Jz, hipStream_t st, int disp_only = 0, int64_t x_stride = 0,
                      int force_fp32 = 0);

struct ProjWS {
    float *Jz, *x, *xc, *xt;
    double *A, *part, *g, *delta, *z, *v, *zc, *f, *fe, *fc, *fce, *fnew, *step;
    int32_t *status, *singular;
};

int64_t proj_ws_bytes(int d, int r, int B, int64_t ns, int max_backtrack);
ProjWS proj_ws_carve(void *base, int d, int r, int B, int64_t ns, int max_backtrack);
bool opts_ok(const mr_gn_opts *o);
int32_t project_args(const mr_decoder *dec, int32_t B, int64_t ns, const float *X,
                     const int32_t *sample_idx, const float *v_trial, const double *xhat_n,
                     const double *xhat_prev, const mr_gn_opts *opts, const double *xhat_next,
                     const double *vhat_next, int &d, int &r);

int32_t project_impl(const mr_decoder *dec, int d, int r, int32_t B, int64_t n_ref, const float *X,
                     int64_t ns, const int32_t *idx, const int32_t *ns_inst, const float *x_trial,
                     const float *v_trial, const double *zn, const double *zp, double dt,
                     const mr_gn_opts &o, double *z_out, double *v_out, int32_t *iters_out,
                     double *resid_out, int32_t *status_out, const ProjWS &w, hipStream_t st,
                     int accumulate = 0);

}  // namespace mr
