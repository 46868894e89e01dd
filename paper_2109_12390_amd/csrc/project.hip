// Reduced-space dynamics on gfx950 (paper Section 3.2.4, Algorithms 6 and 7):
// velocity least squares and Gauss-Newton position projection over the
// sample points, batched over B instances.
//
//  * normal equations: one workgroup per (instance, chunk of 64 samples)
//    stages the chunk's latent Jacobian (fp32, from the decoder kernels) in
//    LDS as fp64 and forms partial J^T J, J^T y and 0.5 |y|^2 (products of
//    fp32 values are exact in fp64, so only the summation rounds); a second
//    kernel adds the partials in chunk order;
//  * the r x r solve is an fp64 Cholesky factorisation, one wave per
//    instance;
//  * backtracking: the max_backtrack + 1 trial step lengths 1, 1/2, 1/4, ...
//    are decoded together in one launch (B (max_backtrack + 1) instances)
//    and the first one passing the Armijo test is taken, so each iteration
//    has a fixed launch sequence (no host decisions, graph-capturable).
#include "project.h"

namespace mr {

constexpr int NE_THREADS = 256;

__global__ void zero_i32_kernel(int32_t *a, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0;
}
constexpr int NE_CH = 64;             // samples per partial-sum workgroup
constexpr int NE_LD = NE_CH + 1;      // LDS row stride (doubles), off the bank period

__host__ __device__ inline int ne_chunks(int64_t ns) { return (int)((ns + NE_CH - 1) / NE_CH); }
__host__ __device__ inline int ne_entries(int r) { return r * r + r + 2; }

// sum over one chunk of p[c] q[c] (ABS: |p[c]| q[c]), four partial sums
template <bool ABS>
__device__ __forceinline__ double chunk_dot(const double *p, const double *q)
{
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < NE_CH; ++c) acc[c & 3] += (ABS ? fabs(p[c]) : p[c]) * q[c];
    return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

// Partial sums of the normal equations over one chunk of NE_CH samples of
// one instance (grid: chunks x B).  Entry e of the chunk's record:
//   e < r^2        (J^T J)[k1][k2]       = sum_a,s J[a k1][s] J[a k2][s]
//   e < r^2 + r    (J^T y)[k]            = sum_a,s J[a k][s] y[a][s]
//   e = r^2 + r    0.5 |y|^2                       (MODE 1)
//   e = r^2 + r + 1  sum |y| (|x| + |x_trial|) 2^-23 (MODE 1): a bound on
//                  the change of the objective caused by fp32 rounding
// with y = v_trial (MODE 0) or y = x - x_trial (MODE 1).  The fp32 inputs
// are widened to fp64 once when staged; their products are exact in fp64,
// so only the summation rounds.
template <int MODE>
__global__ void __launch_bounds__(NE_THREADS) normal_eq_partial_kernel(
    int d, int r, int64_t ns, const int32_t *ns_inst, const float *Jz, const float *y,
    const float *x, double *part)
{
    extern __shared__ __align__(8) double smd[];
    const int ch = blockIdx.x, nch = gridDim.x, b = blockIdx.y;
    const int64_t cnt = ns_inst ? (int64_t)ns_inst[b] : ns;
    const int64_t s0 = (int64_t)ch * NE_CH;
    const int len = s0 >= cnt ? 0 : (int)((cnt - s0) < NE_CH ? (cnt - s0) : NE_CH);
    const int dr = d * r;
    double *Js = smd;                   // [dr][NE_LD]
    double *Ys = Js + dr * NE_LD;       // [d][NE_LD]
    double *Ms = Ys + d * NE_LD;        // [d][NE_LD]
    const float *Jb = Jz + (size_t)b * dr * ns;
    const float *yb = y + (size_t)b * d * ns;
    const float *xb = MODE == 1 ? x + (size_t)b * d * ns : nullptr;
    for (int t = threadIdx.x; t < dr * NE_CH; t += NE_THREADS) {
        const int row = t / NE_CH, c = t % NE_CH;
        Js[row * NE_LD + c] = c < len ? (double)Jb[(size_t)row * ns + s0 + c] : 0.0;
    }
    for (int t = threadIdx.x; t < d * NE_CH; t += NE_THREADS) {
        const int a = t / NE_CH, c = t % NE_CH;
        double val = 0.0, mag = 0.0;
        if (c < len) {
            const float yv = yb[(size_t)a * ns + s0 + c];
            if (MODE == 1) {
                const float xv = xb[(size_t)a * ns + s0 + c];
                mag = (double)fabsf(xv) + (double)fabsf(yv);
                val = (double)(xv - yv);
            } else {
                val = (double)yv;
            }
        }
        Ys[a * NE_LD + c] = val;
        Ms[a * NE_LD + c] = mag;
    }
    __syncthreads();
    const int nent = ne_entries(r);
    double *pb = part + ((size_t)b * nch + ch) * nent;
    // Rows are zero past len, so every sum runs over the whole chunk (a
    // fixed trip count: the LDS loads of the loop are issued together).
    for (int e = threadIdx.x; e < nent; e += NE_THREADS) {
        double s = 0.0;
        if (e < r * r) {
            const int k1 = e / r, k2 = e % r;
            for (int a = 0; a < d; ++a)
                s += chunk_dot<false>(Js + (a * r + k1) * NE_LD, Js + (a * r + k2) * NE_LD);
        } else if (e < r * r + r) {
            const int k = e - r * r;
            for (int a = 0; a < d; ++a) s += chunk_dot<false>(Js + (a * r + k) * NE_LD, Ys + a * NE_LD);
        } else if (MODE == 1 && e == r * r + r) {
            for (int a = 0; a < d; ++a) s += chunk_dot<false>(Ys + a * NE_LD, Ys + a * NE_LD);
            s *= 0.5;
        } else if (MODE == 1) {
            for (int a = 0; a < d; ++a) s += chunk_dot<true>(Ys + a * NE_LD, Ms + a * NE_LD);
            s *= 0x1p-23;
        }
        pb[e] = s;
    }
}

// Sum of the chunk records in chunk order (deterministic) into A, rhs, f, fe.
__global__ void __launch_bounds__(NE_THREADS) normal_eq_reduce_kernel(int r, int nch,
                                                                      const double *part,
                                                                      double *A, double *rhs,
                                                                      double *f, double *fe)
{
    const int b = blockIdx.x;
    const int nent = ne_entries(r);
    for (int e = threadIdx.x; e < nent; e += NE_THREADS) {
        double s = 0.0;
        for (int ch = 0; ch < nch; ++ch) s += part[((size_t)b * nch + ch) * nent + e];
        if (e < r * r)
            A[(size_t)b * r * r + e] = s;
        else if (e < r * r + r)
            rhs[(size_t)b * r + (e - r * r)] = s;
        else if (e == r * r + r && f)
            f[b] = s;
        else if (e == r * r + r + 1 && fe)
            fe[b] = s;
    }
}

template <int MODE>
void normal_eq(int d, int r, int B, int64_t ns, const int32_t *ns_inst, const float *Jz,
               const float *y, const float *x, double *part, double *A, double *rhs, double *f,
               double *fe, hipStream_t st)
{
    const int nch = ne_chunks(ns);
    const size_t lds = sizeof(double) * (size_t)(d * r + 2 * d) * NE_LD;
    normal_eq_partial_kernel<MODE><<<dim3((unsigned)nch, (unsigned)B), NE_THREADS, lds, st>>>(
        d, r, ns, ns_inst, Jz, y, x, part);
    normal_eq_reduce_kernel<<<(unsigned)B, NE_THREADS, 0, st>>>(r, nch, part, A, rhs, f, fe);
}

// 0.5 |x - x_trial|^2 per candidate instance c (samples of instance c / group)
__global__ void __launch_bounds__(256) objective_kernel(int d, int64_t ns, int group,
                                                        const int32_t *ns_inst, const float *x,
                                                        const float *xt, double *f, double *fe)
{
    __shared__ double red[256];
    __shared__ double red2[256];
    const int c = blockIdx.x;
    const int b = c / group;
    const int64_t cnt = ns_inst ? (int64_t)ns_inst[b] : ns;
    double s = 0.0, se = 0.0;
    for (int64_t t = threadIdx.x; t < cnt * d; t += blockDim.x) {
        int a = (int)(t / cnt);
        int64_t i = t % cnt;
        double xv = x[((size_t)c * d + a) * ns + i], tv = xt[((size_t)b * d + a) * ns + i];
        double v = xv - tv;
        s += 0.5 * v * v;
        se += fabs(v) * (fabs(xv) + fabs(tv)) * 0x1p-23;
    }
    red[threadIdx.x] = s;
    red2[threadIdx.x] = se;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            red[threadIdx.x] += red[threadIdx.x + o];
            red2[threadIdx.x] += red2[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        f[c] = red[0];
        fe[c] = red2[0];
    }
}

// Solve (A + damping I) y = sign * rhs by Cholesky, one wave per instance
// (r <= 32): the matrix sits in LDS; column j of L is formed by lanes i >= j
// in parallel (left-looking), and the two triangular solves keep y_i in lane
// i, updating the remaining lanes after each pivot.  A pivot below 1e-12 of
// its original diagonal (or not positive) marks the instance singular:
// y = 0 and MR_FLAG_SINGULAR.
__global__ void __launch_bounds__(64) cholesky_solve_kernel(int B, int r, const double *A,
                                                            const double *rhs, double damping,
                                                            double sign, double *y,
                                                            int32_t *status, int32_t *singular)
{
    __shared__ double Ls[32][33];
    __shared__ double dg[32];
    __shared__ double inv[32];  // 1 / L[j][j]
    const int b = blockIdx.x;
    const int lane = threadIdx.x;
    if (b >= B) return;                                   // block-uniform
    const double *Ab = A + (size_t)b * r * r;
    for (int t = lane; t < r * r; t += 64) {
        const int i = t / r, k = t % r;
        Ls[i][k] = Ab[t] + (i == k ? damping : 0.0);
    }
    if (lane < r) dg[lane] = Ab[lane * r + lane] + damping;
    __syncthreads();
    bool ok = true;
    for (int j = 0; j < r; ++j) {
        const bool act = lane >= j && lane < r;
        double s = 0.0;
        if (act) {
            // L[lane][j] - sum_k L[lane][k] L[j][k], four partial sums
            double p[4] = {0.0, 0.0, 0.0, 0.0};
            int k = 0;
            for (; k + 4 <= j; k += 4)
#pragma unroll
                for (int q = 0; q < 4; ++q) p[q] += Ls[lane][k + q] * Ls[j][k + q];
            for (; k < j; ++k) p[0] += Ls[lane][k] * Ls[j][k];
            s = Ls[lane][j] - ((p[0] + p[1]) + (p[2] + p[3]));
        }
        const double piv = __shfl(s, j);
        if (!(piv > 1e-12 * dg[j]) || !(piv > 0.0)) {   // wave-uniform
            ok = false;
            break;
        }
        const double ljj = sqrt(piv);
        const double rl = 1.0 / ljj;
        if (act) Ls[lane][j] = lane == j ? ljj : s * rl;
        if (lane == j) inv[j] = rl;
        __syncthreads();
    }
    double* yb = y + (size_t)b * r;
    if (!ok) {
        if (lane < r) yb[lane] = 0.0;
        if (lane == 0) {
            if (status) status[b] |= MR_FLAG_SINGULAR;
            if (singular) singular[b] = 1;
        }
        return;
    }
    // forward: L w = sign rhs ; backward: L^T y = w
    double yk = lane < r ? sign * rhs[(size_t)b * r + lane] : 0.0;
    for (int i = 0; i < r; ++i) {
        const double wi = __shfl(yk, i) * inv[i];
        if (lane == i) yk = wi;
        else if (lane > i && lane < r) yk -= Ls[lane][i] * wi;
    }
    for (int i = r - 1; i >= 0; --i) {
        const double yi = __shfl(yk, i) * inv[i];
        if (lane == i) yk = yi;
        else if (lane < i) yk -= Ls[i][lane] * yi;
    }
    if (lane < r) yb[lane] = yk;
}

// trial point of Algorithm 5 from the decoded current point: x_n + dt v_trial
__global__ void trial_from_velocity_kernel(int64_t total, double dt, const float *xn,
                                           const float *vt, float *xt)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < total) xt[i] = xn[i] + (float)dt * vt[i];
}

__global__ void init_guess_kernel(int B, int r, int mode, double dt, const double *zn,
                                  const double *zp, const double *vhat, const int32_t *singular,
                                  double *z, double *vout)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B * r) return;
    int b = t / r;
    bool sing = singular[b] != 0;
    double v = sing ? 0.0 : vhat[t];
    vout[t] = v;
    if (mode == MR_VEL_ONLY)
        z[t] = zn[t] + dt * v;
    else
        z[t] = sing ? zn[t] : 2.0 * zn[t] - zp[t];
}

// candidate latents z + alpha_j delta, alpha_j = 2^-j, j = 0..nc-1
__global__ void candidates_kernel(int B, int r, int nc, const double *z, const double *delta,
                                  double *zc)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B * nc * r) return;
    int k = t % r;
    int c = t / r;
    int b = c / nc, jj = c % nc;
    double alpha = ldexp(1.0, -jj);
    zc[t] = z[(size_t)b * r + k] + alpha * delta[(size_t)b * r + k];
}

// pick the first Armijo-admissible step; g = J^T res (gradient of f)
__global__ void select_kernel(int B, int r, int nc, double c_armijo, double tol_step,
                              const double *f, const double *fe, const double *g,
                              const double *delta, const double *fc, const double *fce,
                              const int32_t *singular, double *z,
                              double *fnew, double *step_norm, int32_t *status, int last)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double slope = 0.0;
    for (int k = 0; k < r; ++k) slope += g[(size_t)b * r + k] * delta[(size_t)b * r + k];
    // A Gauss-Newton step below the fp32 resolution of the decoder means the
    // instance has converged: the objective is then at its rounding floor and
    // the Armijo comparison is noise, so the (tiny) step is taken untested.
    double dn2 = 0.0, z2 = 0.0;
    for (int k = 0; k < r; ++k) {
        dn2 += delta[(size_t)b * r + k] * delta[(size_t)b * r + k];
        z2 += z[(size_t)b * r + k] * z[(size_t)b * r + k];
    }
    const bool converged = sqrt(dn2) <= 1e-7 * (1.0 + sqrt(z2));
    int pick = converged ? 0 : -1;
    for (int jj = 0; jj < nc && pick < 0; ++jj) {
        double alpha = ldexp(1.0, -jj);
        // Armijo test, widened by the rounding bound of the two objective
        // evaluations (fp32 positions): a step whose decrease cannot be
        // resolved is accepted rather than rejected as an ascent
        if (fc[(size_t)b * nc + jj] <=
            f[b] + c_armijo * alpha * slope + fe[b] + fce[(size_t)b * nc + jj]) {
            pick = jj;
            break;
        }
    }
    double sn = 0.0, zn2 = 0.0;
    if (pick >= 0 && !singular[b]) {
        double alpha = ldexp(1.0, -pick);
        for (int k = 0; k < r; ++k) {
            double s = alpha * delta[(size_t)b * r + k];
            z[(size_t)b * r + k] += s;
            sn += s * s;
            zn2 += z[(size_t)b * r + k] * z[(size_t)b * r + k];
        }
        fnew[b] = fc[(size_t)b * nc + pick];
    } else {
        fnew[b] = f[b];
        if (pick < 0 && status) status[b] |= MR_FLAG_LINESEARCH;
    }
    step_norm[b] = sqrt(sn);
    if (last && tol_step > 0.0 && sqrt(sn) > tol_step * (1.0 + sqrt(zn2)) && status)
        status[b] |= MR_FLAG_NOCONV;
}

__global__ void finish_kernel(int B, int r, const double *z, const double *v, const double *fnew,
                              int iters, double *z_out, double *v_out, int32_t *iters_out,
                              double *resid_out, const int32_t *status_in, int32_t *status_out,
                              int accumulate)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B * r) return;
    z_out[t] = z[t];
    v_out[t] = v[t];
    if (t % r == 0) {
        int b = t / r;
        if (iters_out) iters_out[b] = iters;
        if (resid_out) resid_out[b] = fnew ? fnew[b] : 0.0;
        if (status_out) status_out[b] = accumulate ? (status_out[b] | status_in[b]) : status_in[b];
    }
}

int64_t proj_ws_bytes(int d, int r, int B, int64_t ns, int max_backtrack)
{
    int nc = max_backtrack + 1;
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        int64_t o = off;
        off += (bytes + 255) & ~(int64_t)255;
        return o;
    };
    take(4LL * B * d * r * ns);       // Jz
    take(4LL * B * d * ns);           // x
    take(4LL * B * nc * d * ns);      // candidate x
    take(4LL * B * d * ns);           // trial positions / displacements
    take(8LL * B * r * r);            // A
    take(8LL * B * ne_chunks(ns) * ne_entries(r));   // normal-equation partial sums
    take(8LL * B * r);                // rhs / g
    take(8LL * B * r);                // delta
    take(8LL * B * r);                // z
    take(8LL * B * r);                // v
    take(8LL * B * nc * r);           // candidate z
    take(8LL * B);                    // f
    take(8LL * B);                    // fe
    take(8LL * B * nc);               // fc
    take(8LL * B * nc);               // fce
    take(8LL * B);                    // fnew
    take(8LL * B);                    // step norm
    take(4LL * B);                    // status
    take(4LL * B);                    // singular
    return off;
}

ProjWS proj_ws_carve(void *base, int d, int r, int B, int64_t ns, int max_backtrack)
{
    int nc = max_backtrack + 1;
    char *p = (char *)base;
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        char *q = p + off;
        off += (bytes + 255) & ~(int64_t)255;
        return q;
    };
    ProjWS w;
    w.Jz = (float *)take(4LL * B * d * r * ns);
    w.x = (float *)take(4LL * B * d * ns);
    w.xc = (float *)take(4LL * B * nc * d * ns);
    w.xt = (float *)take(4LL * B * d * ns);
    w.A = (double *)take(8LL * B * r * r);
    w.part = (double *)take(8LL * B * ne_chunks(ns) * ne_entries(r));
    w.g = (double *)take(8LL * B * r);
    w.delta = (double *)take(8LL * B * r);
    w.z = (double *)take(8LL * B * r);
    w.v = (double *)take(8LL * B * r);
    w.zc = (double *)take(8LL * B * nc * r);
    w.f = (double *)take(8LL * B);
    w.fe = (double *)take(8LL * B);
    w.fc = (double *)take(8LL * B * nc);
    w.fce = (double *)take(8LL * B * nc);
    w.fnew = (double *)take(8LL * B);
    w.step = (double *)take(8LL * B);
    w.status = (int32_t *)take(4LL * B);
    w.singular = (int32_t *)take(4LL * B);
    return w;
}

int32_t project_impl(const mr_decoder *dec, int d, int r, int32_t B, int64_t n_ref, const float *X,
                     int64_t ns, const int32_t *idx, const int32_t *ns_inst, const float *x_trial,
                     const float *v_trial, const double *zn, const double *zp, double dt,
                     const mr_gn_opts &o, double *z_out, double *v_out, int32_t *iters_out,
                     double *resid_out, int32_t *status_out, const ProjWS &w, hipStream_t st,
                     int accumulate)
{
    const int nc = o.max_backtrack + 1;
    const int TB = 256;
    int32_t rc;
    zero_i32_kernel<<<(unsigned)ceil_div(B, TB), TB, 0, st>>>(w.status, B);
    zero_i32_kernel<<<(unsigned)ceil_div(B, TB), TB, 0, st>>>(w.singular, B);
    // With x_trial == NULL the trial positions are those of Algorithm 5,
    // g(X_p; xhat_n) + dt v_trial, and with a displacement-mode decoder the
    // whole position projection runs on displacements g - X: the residual
    // g(X; z) - x_trial is then formed from numbers of the size of the
    // motion, not of the coordinates, so fp32 keeps its relative accuracy.
    const int disp = (!x_trial && decoder_output_mode(dec) == MR_OUT_DISPLACEMENT) ? 1 : 0;
    // velocity least squares at zn
    // positions (objective, line search) and latent Jacobian, each in fp32
    // or in the decoder's precision (proj_fp32 1: positions, 2: both)
    const int f32x = o.proj_fp32 >= 1 ? 1 : 0, f32j = o.proj_fp32 >= 2 ? 1 : 0;
    auto positions_and_jacobian = [&](const double *zq) -> int32_t {
        if (f32x == f32j)
            return decode_jac_ex(dec, B, n_ref, X, ns, idx, 1, ns_inst, zq, nullptr, w.x, nullptr,
                                 nullptr, w.Jz, st, disp, 0, f32x);
        int32_t e = decode_jac_ex(dec, B, n_ref, X, ns, idx, 1, ns_inst, zq, nullptr, nullptr,
                                  nullptr, nullptr, w.Jz, st, disp, 0, f32j);
        if (e != MR_OK) return e;
        return decode_jac_ex(dec, B, n_ref, X, ns, idx, 1, ns_inst, zq, nullptr, w.x, nullptr,
                             nullptr, nullptr, st, disp, 0, f32x);
    };
    rc = positions_and_jacobian(zn);
    if (rc != MR_OK) return rc;
    const float *xtp = x_trial;
    if (!x_trial) {
        int64_t tot = (int64_t)B * d * ns;
        trial_from_velocity_kernel<<<(unsigned)ceil_div(tot, TB), TB, 0, st>>>(tot, dt, w.x, v_trial,
                                                                                w.xt);
        xtp = w.xt;
    }
    normal_eq<0>(d, r, B, ns, ns_inst, w.Jz, v_trial, nullptr, w.part, w.A, w.g, nullptr, nullptr,
                 st);
    cholesky_solve_kernel<<<(unsigned)B, 64, 0, st>>>(B, r, w.A, w.g, o.damping, 1.0, w.v,
                                                      w.status, w.singular);
    init_guess_kernel<<<(unsigned)ceil_div((int64_t)B * r, TB), TB, 0, st>>>(
        B, r, o.mode, dt, zn, zp, w.v, w.singular, w.z, w.v);
    MR_LAUNCH_CHECK();
    int iters = 0;
    const double *fres = nullptr;
    if (o.mode == MR_POS_VEL) {
        for (int it = 0; it < o.max_iter; ++it) {
            rc = positions_and_jacobian(w.z);
            if (rc != MR_OK) return rc;
            normal_eq<1>(d, r, B, ns, ns_inst, w.Jz, xtp, w.x, w.part, w.A, w.g, w.f, w.fe, st);
            cholesky_solve_kernel<<<(unsigned)B, 64, 0, st>>>(B, r, w.A, w.g, o.damping, -1.0,
                                                              w.delta, w.status, nullptr);
            candidates_kernel<<<(unsigned)ceil_div((int64_t)B * nc * r, TB), TB, 0, st>>>(
                B, r, nc, w.z, w.delta, w.zc);
            MR_LAUNCH_CHECK();
            rc = decode_jac_ex(dec, B * nc, n_ref, X, ns, idx, nc, nullptr, w.zc, nullptr, w.xc,
                               nullptr, nullptr, nullptr, st, disp, 0, f32x);
            if (rc != MR_OK) return rc;
            objective_kernel<<<B * nc, 256, 0, st>>>(d, ns, nc, ns_inst, w.xc, xtp, w.fc, w.fce);
            select_kernel<<<(unsigned)ceil_div(B, 64), 64, 0, st>>>(
                B, r, nc, o.armijo_c, o.tol_step, w.f, w.fe, w.g, w.delta, w.fc, w.fce, w.singular,
                w.z, w.fnew,
                w.step, w.status, it == o.max_iter - 1 ? 1 : 0);
            MR_LAUNCH_CHECK();
        }
        iters = o.max_iter;
        fres = o.max_iter > 0 ? w.fnew : nullptr;
    }
    finish_kernel<<<(unsigned)ceil_div((int64_t)B * r, TB), TB, 0, st>>>(
        B, r, w.z, w.v, fres, iters, z_out, v_out, iters_out, resid_out, w.status, status_out,
        accumulate);
    MR_LAUNCH_CHECK();
    return MR_OK;
}

bool opts_ok(const mr_gn_opts *o)
{
    return o && (o->mode == MR_POS_VEL || o->mode == MR_VEL_ONLY) && o->max_iter >= 0 &&
           o->max_iter <= 64 && o->max_backtrack >= 0 && o->max_backtrack <= 30 &&
           o->damping >= 0.0 && o->proj_fp32 >= 0 && o->proj_fp32 <= 2;
}

// argument checks shared by the projection entry points; fills the sizes
int32_t project_args(const mr_decoder *dec, int32_t B, int64_t ns, const float *X,
                     const int32_t *sample_idx, const float *v_trial, const double *xhat_n,
                     const double *xhat_prev, const mr_gn_opts *opts, const double *xhat_next,
                     const double *vhat_next, int &d, int &r)
{
    if (!dec || B < 1 || ns < 1 || !X || !sample_idx || !v_trial || !xhat_n || !opts_ok(opts) ||
        !xhat_next || !vhat_next)
        return MR_EINVAL;
    if (opts->mode == MR_POS_VEL && !xhat_prev) return MR_EINVAL;
    if ((int64_t)B * (opts->max_backtrack + 1) > 65535) return MR_EINVAL;
    d = decoder_dim(dec);
    r = decoder_latent(dec);
    return MR_OK;
}

}  // namespace mr

using namespace mr;

extern "C" int64_t rom_project_workspace_bytes(const mr_decoder *dec, int32_t B, int64_t ns,
                                               const mr_gn_opts *opts)
{
    if (!dec || B < 1 || ns < 1 || !opts_ok(opts)) return MR_EINVAL;
    return proj_ws_bytes(decoder_dim(dec), decoder_latent(dec), B, ns, opts->max_backtrack);
}

extern "C" int32_t rom_project(const mr_decoder *dec, int32_t B, int64_t n_ref, const float *X,
                               int64_t ns, const int32_t *sample_idx,
                               const int32_t *ns_per_instance, const float *x_trial,
                               const float *v_trial, const double *xhat_n,
                               const double *xhat_prev, double dt, const mr_gn_opts *opts,
                               double *xhat_next, double *vhat_next, int32_t *iters_out,
                               double *resid_out, int32_t *status_out, void *workspace,
                               size_t ws_bytes, void *stream)
{
    int d = 0, r = 0;
    int32_t rc = project_args(dec, B, ns, X, sample_idx, v_trial, xhat_n, xhat_prev, opts,
                              xhat_next, vhat_next, d, r);
    if (rc != MR_OK) return rc;
    if (!workspace || (int64_t)ws_bytes < proj_ws_bytes(d, r, B, ns, opts->max_backtrack) ||
        (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return MR_EINVAL;
    ProjWS w = proj_ws_carve(workspace, d, r, B, ns, opts->max_backtrack);
    return project_impl(dec, d, r, B, n_ref, X, ns, sample_idx, ns_per_instance, x_trial, v_trial,
                        xhat_n, xhat_prev ? xhat_prev : xhat_n, dt, *opts, xhat_next, vhat_next,
                        iters_out, resid_out, status_out, w, as_stream(stream));
}
