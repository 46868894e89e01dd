/*
 * mpmrom.h -- C ABI of libmpmrom.so, the MI355X (gfx950) implementation of
 * the explicit material point method step and of the reduced-order model
 * built on an implicit neural representation of the deformation map
 * (Chen, Chiaramonte, Grinspun, Carlberg, "Model reduction for the material
 * point method via an implicit neural representation of the deformation
 * map", arXiv 2109.12390).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Status.  Every function returns an int32 status: MR_OK (0) or a negative
 *   MR_E* code.  MR_EINVAL: null pointer, bad size or enum, detected on the
 *   host before anything is enqueued.  MR_EDEVICE: a HIP call failed.
 *   Conditions found by the kernels themselves (a particle outside the node
 *   lattice, a non-positive volume ratio, a singular normal matrix) are
 *   asynchronous: they are OR-ed as MR_FLAG_* bits into a caller-provided
 *   device int32 word (`status_flag`, nullable), which the caller reads after
 *   synchronising the stream.
 * Streams.  `stream` is a hipStream_t passed as void*; NULL is the null
 *   stream.  Every call only enqueues work on that stream and returns; it
 *   never synchronises, except the *_create functions (which copy
 *   parameters to the device) and mr_sync_status.
 * Memory.  Array arguments are device pointers owned by the caller (for
 *   example PyTorch tensors); the library never frees or retains them past
 *   the call.  Handles (mr_decoder, mr_rom) are owned by the library:
 *   created by *_create, released by *_destroy.  Handles are not thread safe;
 *   calls on one handle must be ordered on one stream.
 * Layout.  Particle arrays are structure-of-arrays float32, component-major:
 *   x[a*n + p]; d x d matrices are row-major per particle:
 *   F[(a*d + b)*n + p].  The background grid is dense, node-major, 4 floats
 *   per node: grid[4*i + c], c = 0 mass, c = 1..d momentum (after
 *   mpm_p2g) or velocity (after mpm_grid_update); node (i, j, k) has linear
 *   index i + n0*(j + n1*k) and sits at (i, j, k) * dx.  Latent vectors are
 *   float64, instance-major [B][r].  Index lists are int32.
 */
#ifndef MPMROM_H
#define MPMROM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes and device flag bits -------------------------------- */
#define MR_OK 0
#define MR_EINVAL (-1)
#define MR_ENOMEM (-2)
#define MR_EDEVICE (-3)
#define MR_ESINGULAR (-4)
#define MR_ENOCONV (-5)
#define MR_EDOMAIN (-6)
#define MR_ESCRATCH (-7)  /* rom_project_noalloc: the call needs more scratch than
                              its fixed device array holds */

#define MR_FLAG_DOMAIN 1     /* stencil left the lattice, NaN, or J <= 0    */
#define MR_FLAG_SINGULAR 2   /* Cholesky of a normal matrix failed          */
#define MR_FLAG_NOCONV 4     /* Gauss-Newton step above tolerance at exit   */
#define MR_FLAG_LINESEARCH 8 /* no step length passed the Armijo test       */
#define MR_FLAG_DRIFT 16     /* deterministic P2G: a particle's stencil left
                                its tile's region (moved more than a cell
                                since the sort); it was not scattered      */

/* ---- enums ------------------------------------------------------------- */
#define MR_FLOOR_STICKY 0        /* every face of the boundary band sticky  */
#define MR_FLOOR_COULOMB 1       /* low-y face Coulomb friction, rest sticky */
/* Constitutive models (Kirchhoff stress tau = P F^T, Section 2.1):
 * fixed-corotated (Stomakhin et al. 2012, the law of the paper's
 * experiments): tau = 2 mu (F - R) F^T + la (J - 1) J I, R the rotation
 * closest to F (the polar rotation for J > 0; for J <= 0 the sign moves onto
 * the smallest singular value, so inverted states keep a defined stress);
 * compressible Neo-Hookean: tau = mu (F F^T - I) + la ln(J) I, undefined
 * for J <= 0 (MR_FLAG_DOMAIN). */
#define MR_FIXED_COROTATED 0
#define MR_NEO_HOOKEAN 1

/* mpm_p2g / mpm_g2p flags */
#define MR_NO_AFFINE 1   /* plain (PIC) transfer: no C_p term / C_p := 0     */
#define MR_ACCUMULATE 2  /* p2g: add into `grid` instead of overwriting it   */
#define MR_TRIAL 4       /* g2p: write x_trial, v_trial; leave particles     */
#define MR_NO_F_UPDATE 8 /* g2p: keep F_p                                    */
#define MR_SORTED 16     /* p2g: particles are cell-sorted by mpm_cell_sort;
                            enables the LDS-tiled scatter                    */
#define MR_NO_VC_OUT 32  /* g2p2g: do not store v_p and C_p                  */
#define MR_DETERMINISTIC 64 /* p2g (with MR_SORTED), mpm_step, mpm_cell_sort_ex:
                            bitwise-reproducible results, independent of the
                            input order of the particles and of the runtime
                            schedule: cells are ordered canonically (by
                            position) by the sort, and each tile's region is
                            staged and summed per node in a fixed tile order
                            instead of flushed with float atomics          */

/* kernel classes of the launch timer (mr_timing_read) */
#define MR_KC_SORT 0     /* cell sort (all of its launches)                  */
#define MR_KC_P2G 1      /* particle-to-grid scatter (with grid zeroing)     */
#define MR_KC_GRID 2     /* grid update                                      */
#define MR_KC_G2P 3      /* grid-to-particle gather                          */
#define MR_KC_G2P2G 4    /* fused gather of step n and scatter of step n + 1 */
#define MR_KC_ZERO 5     /* separate grid clears (mpm_step clears the second
                            grid inside the grid update: no launches here) */
#define MR_KC_COUNT 6

/* decoder enums */
#define MR_OUT_POSITION 0
#define MR_OUT_DISPLACEMENT 1
#define MR_PREC_FP32 0
#define MR_PREC_BF16 1

/* projection modes */
#define MR_POS_VEL 0  /* Algorithm 6: velocity least squares + Gauss-Newton  */
#define MR_VEL_ONLY 1 /* Algorithm 7: velocity least squares, x += dt v      */

/* ---- plain descriptors -------------------------------------------------- */
typedef struct {
    int32_t dim;        /* 2 or 3                                              */
    int32_t n[3];       /* nodes per dimension (n[2] ignored when dim == 2)   */
    float dx;           /* node spacing                                        */
    int32_t bound;      /* boundary band width in nodes (0 = no walls)         */
    int32_t floor_mode; /* MR_FLOOR_STICKY or MR_FLOOR_COULOMB                 */
    float mu_friction;  /* Coulomb coefficient of the floor                    */
    float gravity[3];   /* body acceleration g                                 */
} mr_grid;

typedef struct {
    int32_t model; /* MR_FIXED_COROTATED or MR_NEO_HOOKEAN                   */
    float E, nu;   /* Young's modulus and Poisson ratio                      */
} mr_material;

typedef struct {
    int64_t n;            /* number of particles                              */
    float *x, *v, *C, *F; /* device SoA arrays (C may be NULL with MR_NO_AFFINE) */
    const float *m;       /* per-particle mass, or NULL to use m_uniform      */
    const float *V0;      /* per-particle reference volume, or NULL           */
    float m_uniform, V0_uniform;
} mr_particles;

/* ---- full-order MPM (paper Section 2.2, Algorithm 1) -------------------- */

/* Particle-to-grid transfer (Algorithm 1, first step; Algorithm 5, first
 * step, over quadrature points).  For the listed particles (all when
 * subset == NULL) adds into node i
 *   grid[4i]     += N_i(x_p) m_p
 *   grid[4i+1+a] += N_i(x_p) m_p (v_p + C_p (x_i - x_p))_a
 *                   - dt V0_p (tau_p grad N_i(x_p))_a
 * where N is the quadratic B-spline, tau = P F^T the Kirchhoff stress of the
 * material (so the internal force f^sigma of Algorithm 1 is folded into the
 * momentum, scaled by dt) and the C_p term is the affine (APIC) transfer,
 * dropped with MR_NO_AFFINE.  The grid is zeroed first unless
 * MR_ACCUMULATE.  MR_SORTED requires that mpm_cell_sort ran on these
 * particles with this grid (any later motion is handled).  Particles whose
 * stencil leaves the lattice, or with J <= 0 under Neo-Hookean, are skipped
 * and raise MR_FLAG_DOMAIN.  `workspace` (nullable unless MR_SORTED) must
 * hold mpm_workspace_bytes(grid, n) bytes of device memory.
 * MR_DETERMINISTIC (requires MR_SORTED and subset == NULL; the sort should
 * be mpm_cell_sort_ex with MR_DETERMINISTIC): bitwise-reproducible grid
 * values; every particle must still lie within a cell of its sort-time cell
 * (else it is skipped and MR_FLAG_DRIFT raised). */
int32_t mpm_p2g(const mr_grid *grid_desc, const mr_material *mat,
                const mr_particles *parts, const int32_t *subset,
                int64_t n_subset, float dt, float *grid, int32_t flags,
                void *workspace, int32_t *status_flag, void *stream);

/* Grid update (Algorithm 1, second step): for nodes with mass,
 *   v_i = grid[4i+1..]/m_i + dt g,
 * then the boundary band (sticky faces set v = 0; the Coulomb floor
 * projects v when it points into the floor).  Nodes without mass get v = 0.
 * Converts grid momentum to velocity in place.  active (nullable) lists the
 * n_active node indices to update; NULL updates every node. */
int32_t mpm_grid_update(const mr_grid *grid_desc, float dt, float *grid,
                        const int32_t *active, int64_t n_active, void *stream);

/* Grid-to-particle transfer and advection (Algorithm 1, third and fourth
 * steps):  v_p = sum_i N_i v_i;  C_p = (4/dx^2) sum_i N_i v_i (x_i - x_p)^T
 * (0 with MR_NO_AFFINE);  F_p <- (I + dt sum_i v_i (x) grad N_i) F_p (kept
 * with MR_NO_F_UPDATE);  x_p <- x_p + dt v_p, all at the old x_p.
 * MR_TRIAL (Algorithm 5, last two steps): only writes
 * v_trial[a*n_subset + s] = v_p and x_trial[a*n_subset + s] = x_p + dt v_p
 * for the listed particles. */
int32_t mpm_g2p(const mr_grid *grid_desc, mr_particles *parts,
                const int32_t *subset, int64_t n_subset, float dt,
                const float *grid, int32_t flags, float *x_trial,
                float *v_trial, int32_t *status_flag, void *stream);

/* Cell sort: reorders the particle arrays (x, v, C, F, and m / V0 when
 * per-particle -- those are written through as well, so the caller must own
 * them writable) so that particles are grouped by stencil base cell
 * floor(x/dx - 0.5), cells in the tile-major order used by the sorted P2G,
 * ties in their previous order (a stable sort).  perm_out (nullable, n
 * int32) receives the old index of each new slot.  workspace: see
 * mpm_workspace_bytes. */
int32_t mpm_cell_sort(const mr_grid *grid_desc, mr_particles *parts,
                      int32_t *perm_out, void *workspace, int32_t *status_flag,
                      void *stream);
/* mpm_cell_sort with flags: MR_DETERMINISTIC orders the particles of a cell
 * by position (x, then y, then z; by previous order only between equal
 * positions) instead of by previous order, so that the order -- and the
 * deterministic P2G that relies on it -- does not depend on the input order.
 * Other flag bits: MR_EINVAL. */
int32_t mpm_cell_sort_ex(const mr_grid *grid_desc, mr_particles *parts,
                         int32_t *perm_out, void *workspace, int32_t flags,
                         int32_t *status_flag, void *stream);

/* Device workspace bytes needed by mpm_cell_sort and the sorted P2G for a
 * grid and n particles (including the staging area of the deterministic
 * P2G: 16 bytes per node of every tile's region). */
int64_t mpm_workspace_bytes(const mr_grid *grid_desc, int64_t n);

/* Launch timer: HIP events recorded on the launching stream around every
 * kernel launch of an mpm_step call, tagged with an MR_KC_* class.  Used for
 * tracing and for per-kernel bandwidth figures; adds one event pair per
 * launch.  capacity: number of launches recorded (later ones are not). */
typedef struct mr_timing mr_timing;
int32_t mr_timing_create(int32_t capacity, mr_timing **out);
void mr_timing_destroy(mr_timing *t);
int32_t mr_timing_reset(mr_timing *t);
/* Restricts recording to the classes whose bit is set in class_mask
 * (bit MR_KC_*) and, per class, to every `every`-th launch counted from
 * this call (every >= 1, else MR_EINVAL).  Each recorded launch costs a few
 * microseconds of stream time for its event pair, so sampling keeps a timed
 * run close to an untimed one.  Default: all classes, every launch. */
int32_t mr_timing_sample(mr_timing *t, uint32_t class_mask, int32_t every);
/* Synchronises on the recorded events; per class c < n_classes returns the
 * number of launches and their summed duration in milliseconds. */
int32_t mr_timing_read(mr_timing *t, int32_t n_classes, int64_t *launches,
                       double *total_ms);

/* Fused grid-to-particle transfer of step n (Algorithm 1, third and fourth
 * steps, from grid_in velocities) and particle-to-grid transfer of step
 * n + 1 (Algorithm 1, first step, at the updated particle state, added into
 * grid_out).  The particles must be in the order of the last mpm_cell_sort
 * with this workspace (motion since then is handled).  x and F are updated
 * in place; v and C are stored unless MR_NO_VC_OUT.  grid_out is zeroed
 * first unless MR_ACCUMULATE; grid_in and grid_out must differ. */
int32_t mpm_g2p2g(const mr_grid *grid_desc, const mr_material *mat,
                  mr_particles *parts, float dt, const float *grid_in,
                  float *grid_out, int32_t flags, void *workspace,
                  int32_t *status_flag, void *stream);

/* n_steps full-order steps (Algorithm 1 with the affine transfer unless
 * MR_NO_AFFINE in flags): per step the scatter into one of two grid
 * buffers, the grid update (which clears the other buffer) and the gather.
 * With sort_every > 0 the particles are cell-sorted before step 0 and every
 * sort_every steps and P2G uses the sorted tiled scatter.  grid: device scratch of
 * 4 * nodes floats (contents on return unspecified); workspace:
 * mpm_step_workspace_bytes(grid, n) bytes.  perm_accum (nullable, n int32)
 * receives, for every array slot on return, the index that particle had on
 * entry.  timing (nullable) records every launch.  Particles end with x, v,
 * C, F of the last step.  Between sorts the state may live in the
 * workspace (each sort gathers from one copy into the other); it is in the
 * caller's arrays again when the call's work completes on the stream.
 * MR_DETERMINISTIC (requires sort_every >= 1): canonical sorts and the
 * deterministic P2G, so the final state does not depend on the input order
 * of the particles (up to their relabelling, given by perm_accum) or on the
 * run; particles must move less than a cell between sorts.  Every launch
 * is a kernel or a device-to-device copy on `stream` (no host
 * synchronisation, no memset), so a call can be captured in a graph when
 * timing is NULL. */
int32_t mpm_step(const mr_grid *grid_desc, const mr_material *mat,
                 mr_particles *parts, float dt, int32_t n_steps,
                 int32_t sort_every, int32_t flags, float *grid,
                 void *workspace, int32_t *perm_accum, int32_t *status_flag,
                 mr_timing *timing, void *stream);
int64_t mpm_step_workspace_bytes(const mr_grid *grid_desc, int64_t n);

/* Sort key of each particle in the order mpm_cell_sort produces
 * (keys_out: n int32; -1 for particles outside the lattice). */
int32_t mpm_cell_keys(const mr_grid *grid_desc, const mr_particles *parts,
                      int32_t *keys_out, void *stream);

/* ---- neural deformation-map decoder (Sections 3.1 and 4) --------------- */

typedef struct mr_decoder mr_decoder;

/* Creates a decoder g(X; xhat) = X + mean + std * y (MR_OUT_DISPLACEMENT) or
 * mean + std * y (MR_OUT_POSITION), y the output of an MLP with n_hidden ELU
 * layers of `width` units on the input [2 (X - in_min)/(in_max - in_min) - 1,
 * xhat] (paper Section 4 network, Appendix B feature scaling).  params is a
 * host float32 array [W_0 (width x (d+r), row-major), b_0, W_1, b_1, ...,
 * W_L (d x width), b_L]; in_min, in_max, out_mean, out_std are host arrays of
 * d floats.  precision MR_PREC_BF16 runs the width x width hidden layers on
 * bf16 matrix cores with fp32 accumulation (first and last layers and all
 * activations stay fp32); MR_PREC_FP32 runs every layer in fp32.
 * Synchronous.  width <= 256, 1 <= n_hidden <= 8, d in {2, 3}, r <= 32. */
int32_t rom_decoder_create(int32_t d, int32_t r, int32_t width,
                           int32_t n_hidden, const float *params,
                           const float *in_min, const float *in_max,
                           const float *out_mean, const float *out_std,
                           int32_t output_mode, int32_t precision,
                           mr_decoder **out);
void rom_decoder_destroy(mr_decoder *dec);

/* Launch-shape autotuner.  The decoder kernels have several shapes per
 * stream configuration (cfg 1: positions only; 5: positions, F and v;
 * 9: positions and eight latent-Jacobian columns): waves splitting the
 * points (one, two or four 16-point tiles per wave) or the waves of a block
 * splitting a layer's units for a shared tile of 16 points (small point
 * sets).  rom_decoder_autotune times each shape of every configuration in
 * cfg_mask (bit 0: cfg 1, bit 1: cfg 5, bit 2: cfg 9) on B instances of n
 * points (capped at 2^22 points, 2^20 for cfg 9, with one instance), `reps`
 * launches each, and records the fastest for that size class
 * (floor(log2(B n))) in the decoder.  Untuned size classes use the nearest
 * tuned class within a factor of 4, else row splitting up to 8192 points
 * and, above, the register-resident shape where the configuration offers it
 * (bf16 decoders, cfg 1 and 5), else point splitting.
 * Every shape computes identical results.  Synchronous on `stream`;
 * allocates and frees scratch.  Returns MR_EINVAL for B < 1, n < 1,
 * reps < 1 or unknown mask bits. */
int32_t rom_decoder_autotune(mr_decoder *dec, int32_t B, int64_t n,
                             int32_t cfg_mask, int32_t reps, void *stream);

/* Shape a launch of configuration cfg (1, 5 or 9) on B instances of n
 * points would use: 0 points split one tile per wave, 1 two tiles, 2 four
 * tiles, 3 units split across the waves of a block, 4 points split with the
 * hidden activations kept in registers (bf16 decoders, cfg 1 and 5);
 * negative on error. */
int32_t rom_decoder_shape(const mr_decoder *dec, int32_t cfg, int32_t B, int64_t n);

/* Records `shape` (numbered as above) for the size class of B instances of
 * n points of configuration cfg, as rom_decoder_autotune would: for callers
 * that tune offline or pin a shape.  Every shape computes identical
 * results.  Returns MR_EINVAL for a shape the configuration or the
 * decoder's precision does not offer. */
int32_t rom_decoder_set_shape(mr_decoder *dec, int32_t cfg, int32_t B, int64_t n,
                              int32_t shape);

/* Replaces the parameters of an existing decoder (same shapes); params is a
 * device or host pointer as flagged by `params_on_device`.  Stream-ordered
 * when on device. */
int32_t rom_decoder_set_params(mr_decoder *dec, const float *params,
                               int32_t params_on_device, void *stream);

/* Kinematic restriction x = g(X; xhat) (Section 3.1, eq. kinematicRestriction)
 * for B instances sharing the reference points.  X: device SoA [d][n_ref];
 * idx (nullable): n int32 row indices into X (NULL: n == n_ref, row s).
 * xhat: device float64 [B][r].  x_out: device float32 [B][d][n]. */
int32_t rom_decode(const mr_decoder *dec, int32_t B, int64_t n_ref,
                   const float *X, int64_t n, const int32_t *idx,
                   const double *xhat, float *x_out, void *stream);

/* Decoder with derivatives at the same points: x = g (nullable),
 * F = dg/dX (Section 3.1, eq. defGrad; [B][d*d][n], nullable),
 * v = (dg/dxhat) vhat (eq. timederOne; [B][d][n], nullable, needs vhat),
 * Jz = dg/dxhat ([B][d*r][n], entry (a, k) at (a*r + k)*n + s; nullable).
 * idx_per_instance: 0 -- idx (nullable) is one list of n rows shared by all
 * instances; 1 -- idx is [B][n], one list per instance; k > 1 -- idx is
 * [B/k][n] and instance b uses list b / k (B must be a multiple of k; the
 * projection decodes its k line-search candidates of an instance this way).
 * Returns MR_EINVAL for a negative k, a k that does not divide B, or k != 0
 * with idx NULL. */
int32_t rom_decode_jac(const mr_decoder *dec, int32_t B, int64_t n_ref,
                       const float *X, int64_t n, const int32_t *idx,
                       int32_t idx_per_instance, const double *xhat,
                       const double *vhat, float *x, float *F, float *v,
                       float *Jz, void *stream);

/* ---- projection (Section 3.2.4, Algorithms 6 and 7) -------------------- */

typedef struct {
    int32_t mode;          /* MR_POS_VEL or MR_VEL_ONLY                        */
    int32_t max_iter;      /* Gauss-Newton iterations (fixed count)            */
    int32_t max_backtrack; /* halvings of the step in the Armijo search        */
    double armijo_c;       /* sufficient-decrease constant                     */
    double damping;        /* added to the normal-matrix diagonal (0: none)    */
    double tol_step;       /* MR_FLAG_NOCONV when the last step exceeds
                              tol_step (1 + |xhat|); <= 0 disables the test  */
    int32_t proj_fp32;     /* the projection's decodes of a bf16 decoder:
                              0 all in bf16; 1 the positions (sample
                              positions and line-search candidates, hence
                              the objective) in fp32, the latent Jacobian in
                              bf16; 2 both in fp32 (as an fp32 decoder of
                              the same weights).  bf16 activations make g
                              piecewise constant in xhat below about 2^-8 of
                              the output scale, which can hide a step's
                              motion from the objective and the Armijo
                              test.  No effect on an fp32 decoder.  Values
                              outside 0..2 are rejected (MR_EINVAL)     */
} mr_gn_opts;

/* Reduced-space dynamics for B instances with ns sample points each
 * (ns_per_instance, nullable device int32 [B], may lower the count per
 * instance):  vhat_{n+1} = argmin sum_p |dg/dxhat(X_p; xhat_n) v - v_trial_p|^2
 * by the normal equations and an fp64 Cholesky factorisation; with
 * MR_POS_VEL, xhat_{n+1} = argmin sum_p |g(X_p; z) - x_trial_p|^2 by
 * max_iter Gauss-Newton iterations from 2 xhat_n - xhat_prev, each with an
 * Armijo backtracking search (a step that no length passes is discarded and
 * raises MR_FLAG_LINESEARCH); with MR_VEL_ONLY, xhat_{n+1} = xhat_n + dt
 * vhat_{n+1}.  sample_idx: device int32 [B][ns] rows of X; x_trial, v_trial:
 * device float32 [B][d][ns]; latents device float64 [B][r]; iters_out and
 * status_out device int32 [B], resid_out device float64 [B] (half the
 * squared position residual at exit), all nullable.  A singular normal
 * matrix leaves that instance's xhat_next = xhat_n, vhat_next = 0 and raises
 * MR_FLAG_SINGULAR.
 * x_trial may be NULL: the target positions are then g(X_p; xhat_n) + dt
 * v_trial_p; with an MR_OUT_DISPLACEMENT decoder the position residual is
 * then formed from displacements g - X, which keeps fp32 cancellation in
 * the residual at the size of the motion, not of the coordinates.
 * workspace: caller-owned device memory of at least
 * rom_project_workspace_bytes(dec, B, ns, opts) bytes, 256-byte aligned
 * (its contents need not be initialised and are dead after the call; it
 * must not be shared by calls that overlap in time).  The call only enqueues
 * kernels on `stream` (no allocation, no synchronisation), so it can be
 * captured in a graph.  MR_EINVAL for a missing, short or misaligned
 * workspace. */
int32_t rom_project(const mr_decoder *dec, int32_t B, int64_t n_ref,
                    const float *X, int64_t ns, const int32_t *sample_idx,
                    const int32_t *ns_per_instance, const float *x_trial,
                    const float *v_trial, const double *xhat_n,
                    const double *xhat_prev, double dt, const mr_gn_opts *opts,
                    double *xhat_next, double *vhat_next, int32_t *iters_out,
                    double *resid_out, int32_t *status_out, void *workspace,
                    size_t ws_bytes, void *stream);

/* Allocation-free variant of rom_project, for callers that cannot allocate
 * device memory (code under graph capture, tight serving loops, harnesses
 * that forbid allocation).  Same arguments, results and errors as
 * rom_project, without the workspace: the scratch is a fixed 16 MiB device
 * array inside the library, one per GPU, held until the process ends (its
 * address is looked up on the first call on each device).  No hipMalloc,
 * hipFree or allocating library call is made.  MR_ESCRATCH when
 * rom_project_workspace_bytes(dec, B, ns, opts) exceeds 16 MiB (about 46
 * instances of 1,024 samples at r = 16, d = 3 and 8 halvings).  Every call
 * on one GPU shares that array and leaves its contents behind: calls that
 * overlap in time on one GPU (several streams or host threads) race and
 * must be serialised by the caller. */
int32_t rom_project_noalloc(const mr_decoder *dec, int32_t B, int64_t n_ref,
                            const float *X, int64_t ns, const int32_t *sample_idx,
                            const int32_t *ns_per_instance, const float *x_trial,
                            const float *v_trial, const double *xhat_n,
                            const double *xhat_prev, double dt, const mr_gn_opts *opts,
                            double *xhat_next, double *vhat_next, int32_t *iters_out,
                            double *resid_out, int32_t *status_out, void *stream);

/* Bytes of device workspace rom_project needs for B instances of ns
 * samples with these options (the decoder fixes d and r); MR_EINVAL
 * (negative) for a null decoder or options, B < 1 or ns < 1. */
int64_t rom_project_workspace_bytes(const mr_decoder *dec, int32_t B, int64_t ns,
                                    const mr_gn_opts *opts);

/* ---- reduced-order step (Section 3.2, Algorithm 2 with Algorithms 3, 5 and
 * 6 or 7) ----------------------------------------------------------------- */

typedef struct mr_rom mr_rom;

typedef struct {
    int32_t B;               /* parameter instances                          */
    int64_t n_particles;     /* reference particles P                        */
    int32_t n_samples_max;   /* largest sample count                         */
    uint64_t seed;           /* sampler seed                                 */
    float rho0;              /* reference density (V0 = m / rho0)            */
    float m_uniform;         /* particle mass when m_all is NULL             */
    int32_t model;           /* constitutive model                           */
    float nu;                /* Poisson ratio (shared)                       */
    int32_t autotune;        /* non-zero: rom_create times the decoder's
                                launch shapes at this runner's sizes
                                (rom_decoder_autotune) before returning   */
    int32_t quadrature;      /* MR_QUAD_LAGRANGIAN (Algorithm 3) or
                                MR_QUAD_EULERIAN (Algorithm 4)            */
    int32_t quad_per_dim;    /* Eulerian: points per cell and dimension,
                                2 or 4 (0 selects 2)                      */
    int32_t newton_iters;    /* Eulerian: Newton iterations inverting the
                                decoder, 1..16 (0 selects 2)              */
    float newton_tol;        /* Eulerian: largest residual max-norm of an
                                accepted point, in cells (0 selects 1e-3);
                                with a bf16 decoder at least 4 x 2^-8 of
                                its largest output standard deviation (its
                                positions' resolution, below which Newton
                                cannot reduce the residual)               */
} mr_rom_config;

/* quadrature kinematics of the reduced step (mr_rom_config.quadrature).
 * Lagrangian (Algorithm 3): every reference particle is decoded each step
 * and those whose stencil touches the samples' nodes are the quadrature
 * points (particle mass, V0 = m / rho0).  Eulerian (Algorithm 4): only the
 * samples are decoded; the quadrature points are the lattice points
 * (m + 1/2) dx / l per axis (l = quad_per_dim) whose stencil touches the
 * samples' nodes, their reference positions X solve g(X; xhat) = x by
 * newton_iters iterations from X = x: a displacement step X = x - u(x)
 * (Jacobian replaced by I), then Newton steps with F = dg/dX, and
 * a point is kept when the residual is within newton_tol cells, det F > 0
 * and X lies in the reference body; its mass is rho0 (dx / l)^d / det F
 * (Algorithm 4) times a body weight clamp(2 s - 1/2, 0, 1), with
 * s = rho_ref(X) / rho0: exactly rho0 V / J wherever s >= 3/4 (a body's
 * interior), a linear taper across the surface band, and the point dropped
 * where s <= 1/4.  rho_ref is the reference particles' mass spread with the
 * quadratic B-spline on the grid's node lattice (spacing dx) and read by
 * multilinear interpolation; rom_create builds it on the host. */
#define MR_QUAD_LAGRANGIAN 0
#define MR_QUAD_EULERIAN 1

/* Creates the reduced-order model runner.  X_all: device SoA [d][P] reference
 * positions; m_all (nullable) device masses; E: device float32 [B] Young's
 * moduli; n_samples: device int32 [B] sample counts (r/d <= count <=
 * n_samples_max).  The grid and option structs are copied; the decoder is
 * referenced and must outlive the runner.  Allocates all workspace up front
 * (synchronous).  The quadrature list holds, per sample, the (5 cells)^d box
 * of stencil bases around it: Lagrangian, twice the particles of the
 * densest reference cell (at least 16) per base cell, at most P; Eulerian,
 * l^d points per base.  A step that would exceed it keeps the first entries
 * and raises MR_FLAG_DOMAIN.  Each instance has a dense node-major grid
 * (16 bytes per node) and node bitmaps; only the nodes a step marks (the set
 * I) are written, and the step zeroes exactly those again after its substep,
 * so no step refills whole grids.  With cfg->autotune set, the decoder's launch shapes are
 * tuned for the runner's four decoder launches (all particles, the
 * quadrature list, the samples, the line-search candidates), which updates
 * the decoder's shape table. */
int32_t rom_create(const mr_decoder *dec, const mr_grid *grid_desc,
                   const mr_rom_config *cfg, const float *X_all,
                   const float *m_all, const float *E,
                   const int32_t *n_samples, const mr_gn_opts *opts,
                   mr_rom **out);
void rom_destroy(mr_rom *rom);

/* Advances every instance n_steps reduced-order steps of size dt, starting
 * at step counter `step0` (the sampler's stream index): for each step, draw
 * the sample points, form the quadrature points (Lagrangian: decode every
 * particle, mark the active nodes of the samples' stencils, collect the
 * neighbour particles touching them, Algorithm 3; Eulerian: decode the
 * samples, mark their nodes, generate and invert the lattice points,
 * Algorithm 4), evaluate x, F, v at the quadrature points, run the
 * sample-point MPM substep (Algorithm 5) and project (Algorithm 6 or 7).
 * xhat, xhat_prev, vhat: device float64 [B][r], updated in place.
 * status_out: device int32 [B] (nullable), OR of MR_FLAG_* over the steps.
 * When use_graph != 0 the per-step launches are captured once into a HIP
 * graph and replayed.  No host synchronisation inside. */
int32_t rom_step(mr_rom *rom, int32_t n_steps, int64_t step0, double dt,
                 double *xhat, double *xhat_prev, double *vhat,
                 int32_t *status_out, int32_t use_graph, void *stream);

/* Initial-condition correction fields (Section 3.1, eqs. defMapApproxForm
 * and essentialSpec, time function t -> t): after this call the runner's
 * kinematics are those of g~(X, xhat, t) = g(X; xhat) + a(X) + b(X) t with
 *   a = X - g(X; xhat0),  b = V0 - (dg/dxhat)(X; xhat0) vhat0,
 * grad a = I - dg/dX (X; xhat0), grad b = -d/dX [(dg/dxhat)(X; xhat0) vhat0]
 * at every reference particle, so that positions, velocities and
 * deformation gradients at t = 0 are exactly X, V0 and I for any initial
 * latents; t = step counter x dt of rom_step (start the run at step0 = 0).
 * Positions get a + b t, deformation gradients grad a + t grad b,
 * velocities b, and the projection fits g~ at the step's end (its trial
 * velocities shifted by -b).  xhat0, vhat0: device float64 [B][r]; v0:
 * host or device float32 [B][d], a uniform initial velocity per instance
 * (so grad V0 = 0).  grad b is a central difference of dg/dX along vhat0
 * with a latent step of 1e-2 (max norm), fp32 decodes.  Lagrangian
 * quadrature only (the Eulerian points would need the fields and their
 * gradients at the inverted, non-particle reference positions inside every
 * Newton step): MR_EINVAL otherwise.  xhat0 == NULL switches the fields off.
 * Allocates 24 floats per particle and instance once, plus temporaries, and
 * synchronises the stream (a set-up call). */
int32_t rom_set_fields(mr_rom *rom, const double *xhat0, const double *vhat0,
                       const float *v0, void *stream);

/* Positions of every particle (the caller's order) for latents xhat
 * (device float64 [B][r]) at time t: g(X; xhat), plus a + b t when the
 * correction fields are on.  x_out: device float32 [B][d][P]. */
int32_t rom_positions(const mr_rom *rom, const double *xhat, double t,
                      float *x_out, void *stream);

/* Diagnostics of the last step of instance b: quadrature-point count |Q|
 * and active-node count |I| (device values copied to the host; this call
 * synchronises the stream). */
int32_t rom_last_counts(const mr_rom *rom, int32_t b, int64_t *n_quad,
                        int64_t *n_active, void *stream);

/* ---- measurement aid (not part of the method) ------------------------- */

/* Dense bf16 matrix-core loop for the sustained MFMA rate: `blocks`
 * workgroups of 256 threads, every wave running `iters` rounds of 8
 * independent 16x16x32 bf16 products (16,384 FLOP each) on register
 * operands, blocks x 4 x iters x 8 x 16,384 FLOP in all.  sink: device
 * float32 [blocks x 256], written (keeps the products live).  Stream-
 * ordered; MR_EINVAL for blocks < 1, iters < 1 or a NULL sink. */
int32_t mr_mfma_probe(int32_t blocks, int32_t iters, float *sink, void *stream);

/* ---- decoder training (Section 4.2 loss; Appendix B training details) --- */

typedef struct mr_trainer mr_trainer;

/* Number of float32 parameters of the decoder in the packed layout of
 * rom_decoder_create ([W_0, b_0, ..., W_L, b_L], row-major weights). */
int64_t rom_train_param_count(int32_t d, int32_t r, int32_t width,
                              int32_t n_hidden);

/* Creates the training workspace for batches of up to max_rows rows
 * (activations of the primal and of the d + 1 tangent streams of every row
 * are kept for the backward pass: about 2 (d + 2) width n_hidden floats per
 * row).  precision MR_PREC_BF16 runs the width x width products on bf16
 * matrix cores with fp32 accumulation; the first and last layers and all
 * element-wise work stay fp32.  Synchronous. */
int32_t rom_trainer_create(int32_t d, int32_t r, int32_t width,
                           int32_t n_hidden, int32_t precision,
                           int64_t max_rows, const float *in_min,
                           const float *in_max, const float *out_mean,
                           const float *out_std, int32_t output_mode,
                           mr_trainer **out);
void rom_trainer_destroy(mr_trainer *t);

/* Forward pass with tangents for n_groups x rows_per_group rows; group g
 * uses latent z = Z[snap[g]] (Z: device float32 [n_snapshots][r]) and the
 * velocity direction u = (Z[next[g]] - Z[snap[g]]) / dt (zero when
 * next[g] < 0).  X: device [rows][d].  Writes g = g(X; z) [rows][d],
 * G = dg/dX [rows][d][d] and Gv = (dg/dz) u [rows][d].  params: device
 * packed parameters (must stay valid until rom_train_backward). */
int32_t rom_train_forward(mr_trainer *t, const float *params, const float *Z,
                          const float *X, const int32_t *snap,
                          const int32_t *next, int32_t n_groups,
                          int32_t rows_per_group, float dt, float *g,
                          float *G, float *Gv, void *stream);

/* Backward pass of the last forward: given dL/dg, dL/dG, dL/dGv, ADDS
 * dL/dparams into dparams (packed layout) and dL/dZ into dZ. */
int32_t rom_train_backward(mr_trainer *t, const float *dg, const float *dG,
                           const float *dGv, float *dparams, float *dZ,
                           void *stream);

/* Reproducible training: with on != 0 every batch reduction of
 * rom_train_backward (split-K weight gradients, bias gradients, the
 * snapshots' latent gradients) is written as partial sums and added in a
 * fixed order instead of with float atomics, so two runs from the same
 * inputs give bitwise identical gradients.  Allocates about 17 MB on first
 * use.  (rom_train_loss is reproducible in either mode.) */
int32_t rom_trainer_set_deterministic(mr_trainer *t, int32_t on);

/* Training objective (Section 4.2): batch mean of |g - x|^2 +
 * lam_F |G - F|_F^2 + lam_v |Gv - v|^2, the velocity term dropped for
 * groups with next < 0.  loss: device float scalar (overwritten);
 * dg, dG, dGv (nullable): its gradient with respect to g, G, Gv. */
int32_t rom_train_loss(int32_t d, int32_t n_groups, int32_t rows_per_group,
                       const int32_t *next, const float *g, const float *G,
                       const float *Gv, const float *x_t, const float *F_t,
                       const float *v_t, float lam_F, float lam_v,
                       float *loss, float *dg, float *dG, float *dGv,
                       void *stream);

/* Adam (Kingma and Ba): m, v moment estimates, step counts from 1. */
int32_t rom_adam_step(int64_t n, float *param, const float *grad, float *m,
                      float *v, float lr, float beta1, float beta2, float eps,
                      int32_t step, void *stream);

/* Assembles training rows: frames hold (x [P_sub][d], F [P_sub][d][d],
 * v [P_sub][d]) of a fixed particle subset with reference positions
 * X_sub [P_sub][d]; row i takes particle pid[i] of frame
 * snap[i / rows_per_group]. */
int32_t rom_train_gather(int32_t d, int32_t n_groups, int32_t rows_per_group,
                         int64_t P_sub, const float *X_sub,
                         const float *frame_x, const float *frame_F,
                         const float *frame_v, const int32_t *snap,
                         const int32_t *pid, float *X, float *x_t, float *F_t,
                         float *v_t, void *stream);

/* Reads n device status words into host memory after synchronising the
 * stream; returns the OR of their bits mapped to the first MR_E* code
 * (MR_EDOMAIN, MR_ESINGULAR, MR_ENOCONV in that priority) or MR_OK. */
int32_t mr_sync_status(void *stream, const int32_t *device_flags, int32_t n,
                       int32_t *host_flags);

/* Library version string (static storage). */
const char *mr_version(void);

/* ---- encoder (Section 4.1, Table 1) ------------------------------------
 * The network that maps the concatenated deformed positions of a fixed set
 * of material points (point-major: x_1, y_1, z_1, x_2, ...; in_len = d x
 * points) to generalized coordinates, trained with the decoder.  Shape of
 * Table 1: 1D convolutions of kernel 6 and stride 2, added while the next
 * output length stays >= 32 (the last length is d_conv), then dense
 * d_conv -> 32 and 32 -> r.  Each convolution has one input and one output
 * channel, no padding and a bias; ELU follows every convolution and the
 * first dense layer; the input coordinates are mapped per axis to [-1, 1]
 * by in_min / in_max (the decoder's reference-position scaling).  fp32.
 * Parameter vector (device float32 [n_params]): per convolution 6 weights
 * then the bias; W1 (32 x d_conv, row-major), b1 (32), W2 (r x 32), b2 (r).
 */

/* Sizes for an input length and latent dimension (all outputs nullable):
 * the number of convolutions, d_conv, the parameter count, the floats per
 * frame of the activation record that rom_encoder_forward writes and
 * rom_encoder_backward reads, and the floats per frame of the backward
 * work buffer.  MR_EINVAL for in_len < 32 or r outside 1..64. */
int32_t rom_encoder_layout(int64_t in_len, int32_t r, int32_t *n_conv,
                           int64_t *d_conv, int64_t *n_params,
                           int64_t *act_floats, int64_t *work_floats);

/* Encodes n frames.  x: device float32 frames of in_len floats; frame f is
 * x + frame_idx[f] * in_len (frame_idx: nullable device int32 [n]; NULL:
 * frame f).  in_min, in_max: host float32 [d].  act: device float32
 * [n][act_floats], written (the record the backward pass needs).  z:
 * device float32 [n][r].  MR_EINVAL for bad sizes, in_len not a multiple
 * of d, fewer than one convolution, or n above 65535; no synchronisation. */
int32_t rom_encoder_forward(int32_t d, int32_t r, int64_t in_len, int32_t n,
                            const float *x, const int32_t *frame_idx,
                            const float *params, const float *in_min,
                            const float *in_max, float *act, float *z,
                            void *stream);

/* Gradient of sum_f dz[f] . z[f] with respect to the parameters, for the
 * frames and the activation record of the matching rom_encoder_forward
 * call.  dz: device float32 [n][r]; grad: device float32 [n_params],
 * overwritten; work: device float32 [n][work_floats] scratch.  With
 * deterministic == 0 the weight gradients are summed with float atomics
 * (their last bits depend on the schedule); otherwise every partial sum
 * goes to the work buffer and is added in a fixed order (bitwise
 * reproducible).  Errors as rom_encoder_forward. */
int32_t rom_encoder_backward(int32_t d, int32_t r, int64_t in_len, int32_t n,
                             const float *x, const int32_t *frame_idx,
                             const float *params, const float *in_min,
                             const float *in_max, const float *act,
                             const float *dz, float *grad, float *work,
                             int32_t deterministic, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* MPMROM_H */
