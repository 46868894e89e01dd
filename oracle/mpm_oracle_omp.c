/*
 * Threaded variant of the FP64 oracle step (Algorithm 1), for timing the
 * oracle on every host core.
 *
 * TEST INFRASTRUCTURE ONLY.  It calls the plain oracle functions of
 * mpm_oracle.c on contiguous particle chunks, one chunk per thread:
 *   - particle-to-grid: each thread scatters its chunk into private grid
 *     arrays; the private arrays are then summed node by node in thread order
 *     (a fixed order for a given thread count, so a run is reproducible; with
 *     one thread the result is the plain oracle's bit for bit);
 *   - grid update: the plain function on the whole grid (one thread);
 *   - grid-to-particle: each thread updates its chunk (particles are
 *     independent there).
 * Only the node range a chunk can touch is scanned in the sum: its stencil
 * bases' linear indices, extended by the stencil (for particles stored in
 * lattice order a chunk is a slab).
 */
#include <omp.h>
#include <stdlib.h>
#include <string.h>

int orc_p2g(int dim, const int *n, double dx, long np, const long *subset,
            const double *x, const double *v, const double *C, const double *F,
            const double *m, const double *V0, int model, double mu, double la,
            int apic, double *gm, double *gmv, double *gf);
void orc_grid_update(int dim, const int *n, double dt, const double *gravity,
                     int bound, int floor_mode, double mu_f,
                     const double *gm, const double *gmv, const double *gf,
                     double *gv);
int orc_g2p(int dim, const int *n, double dx, double dt, long np,
            const long *subset, int apic, int update_F, const double *gv,
            double *x, double *v, double *C, double *F,
            double *trial_x, double *trial_v);
void orc_cell_keys(int dim, const int *n, double dx, long np, const double *x,
                   long *keys);

/* One step on `threads` threads (<= 0: the OpenMP default).  Arrays as in
 * the plain functions; x, v, C, F are updated in place.  Scratch (the
 * private grids, threads x nodes x (1 + 2 dim) doubles) is allocated per
 * call.  Returns 0, -2 when the scratch cannot be allocated, or -6 (a stencil
 * off the lattice, J <= 0) from any thread. */
int orc_step_threaded(int dim, const int *n, double dx, double dt, long np,
                      double *x, double *v, double *C, double *F,
                      const double *m, const double *V0, int model, double mu,
                      double la, int apic, const double *gravity, int bound,
                      int floor_mode, double mu_f, int threads)
{
    int T = threads > 0 ? threads : omp_get_max_threads();
    long nn = 1;
    for (int a = 0; a < dim; ++a) nn *= n[a];
    const int dd = dim * dim;
    const long per = 1 + 2 * dim;                  /* mass, momentum, force */
    double *priv = (double *)calloc((size_t)T * nn * per, sizeof(double));
    double *gm = (double *)calloc((size_t)nn * per, sizeof(double));
    double *gv = (double *)calloc((size_t)nn * dim, sizeof(double));
    long *lo = (long *)malloc(sizeof(long) * T), *hi = (long *)malloc(sizeof(long) * T);
    int rc = 0;
    if (!priv || !gm || !gv || !lo || !hi) {
        free(priv); free(gm); free(gv); free(lo); free(hi);
        return -2;
    }
    double *gmv = gm + nn, *gf = gm + nn * (1 + dim);
    long reach = 2;                                 /* linear index of node (2, 2, 2) */
    for (int a = 1, s = 1; a < dim; ++a) { s *= n[a - 1]; reach += 2L * s; }
#pragma omp parallel num_threads(T) reduction(| : rc)
    {
        const int t = omp_get_thread_num();
        const long b = np * t / T, e = np * (t + 1) / T;
        double *pm = priv + (size_t)t * nn * per;
        lo[t] = nn;
        hi[t] = -1;
        if (e > b) {
            long *keys = (long *)malloc(sizeof(long) * (e - b));
            orc_cell_keys(dim, n, dx, e - b, x + b * dim, keys);
            for (long i = 0; i < e - b; ++i) {
                if (keys[i] < 0) continue;
                if (keys[i] < lo[t]) lo[t] = keys[i];
                if (keys[i] + reach > hi[t]) hi[t] = keys[i] + reach;
            }
            free(keys);
            rc |= orc_p2g(dim, n, dx, e - b, NULL, x + b * dim, v + b * dim, C + b * dd,
                          F + b * dd, m + b, V0 + b, model, mu, la, apic, pm, pm + nn,
                          pm + nn * (1 + dim));
        }
    }
    if (rc == 0) {
        /* node sums in thread order */
#pragma omp parallel for num_threads(T) schedule(static)
        for (long i = 0; i < nn; ++i) {
            for (int t = 0; t < T; ++t) {
                if (i < lo[t] || i > hi[t]) continue;
                const double *pm = priv + (size_t)t * nn * per;
                gm[i] += pm[i];
                for (int a = 0; a < dim; ++a) {
                    gmv[i * dim + a] += pm[nn + i * dim + a];
                    gf[i * dim + a] += pm[nn * (1 + dim) + i * dim + a];
                }
            }
        }
        orc_grid_update(dim, n, dt, gravity, bound, floor_mode, mu_f, gm, gmv, gf, gv);
#pragma omp parallel num_threads(T) reduction(| : rc)
        {
            const int t = omp_get_thread_num();
            const long b = np * t / T, e = np * (t + 1) / T;
            if (e > b)
                rc |= orc_g2p(dim, n, dx, dt, e - b, NULL, apic, 1, gv, x + b * dim,
                              v + b * dim, C + b * dd, F + b * dd, NULL, NULL);
        }
    }
    free(priv); free(gm); free(gv); free(lo); free(hi);
    return rc == 0 ? 0 : -6;
}
