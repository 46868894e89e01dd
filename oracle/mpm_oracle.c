/*
 * Plain FP64 CPU oracle of the explicit material point method step.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the HIP kernels are checked against.  It shares no code,
 * header, table or constant with the GPU library, and the product path never
 * links or calls it.
 *
 * What it computes (paper, Section 2.2, Algorithm 1 "MPM Algorithm"):
 *   particle-to-grid transfer   m_i = sum_p N_i(x_p) m_p
 *                               m_i v_i = sum_p N_i(x_p) m_p v_p   (+ APIC term)
 *                               f^sigma_i = -sum_p (J/rho0) sigma grad N_i m_p
 *   grid update                 v_i <- v_i + dt (f^sigma_i + f^e_i) / m_i
 *   grid-to-particle transfer   v_p = sum_i N_i v_i
 *                               F_p <- (1 + dt sum_i v_i (x) grad N_i) F_p
 *   position update             x_p <- x_p + dt v_p
 *
 * Readings taken where the paper is silent (each one is listed with its
 * reason in the design notes of the repository):
 *   - N_i is the tensor-product quadratic B-spline on a node lattice with
 *     node i at i*dx; the stencil base of a point is floor(x/dx - 0.5).
 *   - The internal force uses J sigma = P F^T (Section 2.1, relation between
 *     the first Piola-Kirchhoff and Cauchy stress) and m_p / rho0 = V0_p, so
 *     f^sigma_i = -sum_p V0_p tau_p grad N_i with tau = P F^T.
 *   - For gravity, J b = B = rho0 g (footnote on the Lagrangian/Eulerian body
 *     force relation), so f^e_i = m_i g.
 *   - The optional affine (APIC) transfer adds m_p C_p (x_i - x_p) to the
 *     momentum and reconstructs C_p = (4/dx^2) sum_i N_i v_i (x_i - x_p)^T,
 *     the quadratic-B-spline inertia D = dx^2/4 I.  With apic = 0 the code is
 *     the literal PIC transfer of Algorithm 1.
 *   - Nodes with m_i == 0 keep velocity 0.
 *   - Grid boundary conditions act on a band of `bound` nodes at every face:
 *     sticky (v = 0), or a Coulomb floor on the low-y face.
 *
 * Layout (oracle-private): particles array-of-structs, x[p*dim + a],
 * F[p*dim*dim + a*dim + b]; grid nodes linear index i + n0*(j + n1*k).
 * All arithmetic is double precision; loops are plain and in index order.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EDOMAIN (-6)

/* Quadratic B-spline weights and their derivatives (per unit of dx) for the
 * three nodes base, base+1, base+2, where f = x/dx - base lies in [0.5, 1.5). */
void orc_bspline_1d(double f, double *w, double *dw)
{
    double a = 1.5 - f;
    double b = f - 1.0;
    double c = f - 0.5;
    w[0] = 0.5 * a * a;
    w[1] = 0.75 - b * b;
    w[2] = 0.5 * c * c;
    dw[0] = -a;
    dw[1] = -2.0 * b;
    dw[2] = c;
}

/* Stencil of one point: base node per dimension, 1D weights and gradients.
 * Returns ORC_EDOMAIN if the 3^d stencil leaves the node lattice. */
static int stencil(int dim, const int *n, double dx, const double *xp,
                   int *base, double w[3][3], double dw[3][3])
{
    for (int a = 0; a < dim; ++a) {
        double s = xp[a] / dx;
        if (!(s == s)) return ORC_EDOMAIN; /* NaN */
        double bf = floor(s - 0.5);
        if (bf < 0.0 || bf + 2.0 > (double)(n[a] - 1)) return ORC_EDOMAIN;
        base[a] = (int)bf;
        orc_bspline_1d(s - bf, w[a], dw[a]);
        for (int k = 0; k < 3; ++k) dw[a][k] /= dx;
    }
    return ORC_OK;
}

static long node_index(int dim, const int *n, const int *ijk)
{
    long idx = ijk[dim - 1];
    for (int a = dim - 2; a >= 0; --a) idx = idx * n[a] + ijk[a];
    return idx;
}

/* Iterate over the 3^d offsets of a stencil. */
static int next_offset(int dim, int *o)
{
    for (int a = 0; a < dim; ++a) {
        if (++o[a] < 3) return 1;
        o[a] = 0;
    }
    return 0;
}

static double det(int dim, const double *F)
{
    if (dim == 2) return F[0] * F[3] - F[1] * F[2];
    return F[0] * (F[4] * F[8] - F[5] * F[7])
         - F[1] * (F[3] * F[8] - F[5] * F[6])
         + F[2] * (F[3] * F[7] - F[4] * F[6]);
}

/* Cyclic Jacobi eigenvalue iteration for a symmetric 4x4 matrix A (textbook
 * form: each rotation in the (p, q) plane zeroes A[p][q]).  On return the
 * diagonal of A holds the eigenvalues and the columns of V the eigenvectors. */
static void jacobi_eig4(double A[4][4], double V[4][4])
{
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) V[i][j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int p = 0; p < 4; ++p) {
            diag += A[p][p] * A[p][p];
            for (int q = p + 1; q < 4; ++q) off += A[p][q] * A[p][q];
        }
        if (off <= 1e-34 * (diag + off) || off == 0.0) break;
        for (int p = 0; p < 4; ++p)
            for (int q = p + 1; q < 4; ++q) {
                if (A[p][q] == 0.0) continue;
                /* J = [[c, s], [-s, c]] in the (p, q) plane; A <- J^T A J
                 * zeroes A[p][q] when cot(2 phi) = (A_qq - A_pp) / (2 A_pq)
                 * and t = tan(phi) is the smaller root of t^2 + 2 theta t - 1 */
                double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < 4; ++k) {
                    double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - sn * akq;
                    A[k][q] = sn * akp + c * akq;
                }
                for (int k = 0; k < 4; ++k) {
                    double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - sn * aqk;
                    A[q][k] = sn * apk + c * aqk;
                }
                for (int k = 0; k < 4; ++k) {
                    double vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = c * vkp - sn * vkq;
                    V[k][q] = sn * vkp + c * vkq;
                }
            }
    }
}

/* The rotation R (det R = +1) closest to F in the Frobenius norm, i.e. the
 * one maximising tr(R^T F).  For det F > 0 it is the rotation factor of the
 * polar decomposition F = R S with S symmetric positive definite; for
 * det F <= 0 it is the rotation the fixed-corotated model of Stomakhin et
 * al. (2012) uses for inverted elements.
 * d = 2: R is the rotation by the angle of (F00 + F11, F10 - F01); R = I
 * when both vanish.
 * d = 3: with R(q) the rotation of the unit quaternion q = (w, x, y, z),
 * tr(R(q)^T F) is the quadratic form q^T K q of the symmetric 4x4 matrix K
 * below (expanded from the entries of R(q)), so the best q is the
 * eigenvector of K's largest eigenvalue (a Rayleigh quotient over the unit
 * sphere); the eigenvectors come from cyclic Jacobi rotations. */
void orc_closest_rotation(int dim, const double *F, double *R)
{
    if (dim == 2) {
        double cs = F[0] + F[3], sn = F[2] - F[1];
        double h = sqrt(cs * cs + sn * sn);
        double c = 1.0, s = 0.0;
        if (h > 0.0) {
            c = cs / h;
            s = sn / h;
        }
        R[0] = c; R[1] = -s; R[2] = s; R[3] = c;
        return;
    }
    const double F00 = F[0], F01 = F[1], F02 = F[2], F10 = F[3], F11 = F[4], F12 = F[5],
                 F20 = F[6], F21 = F[7], F22 = F[8];
    double K[4][4], V[4][4];
    K[0][0] = F00 + F11 + F22;
    K[1][1] = F00 - F11 - F22;
    K[2][2] = -F00 + F11 - F22;
    K[3][3] = -F00 - F11 + F22;
    K[0][1] = K[1][0] = F21 - F12;
    K[0][2] = K[2][0] = F02 - F20;
    K[0][3] = K[3][0] = F10 - F01;
    K[1][2] = K[2][1] = F01 + F10;
    K[1][3] = K[3][1] = F02 + F20;
    K[2][3] = K[3][2] = F12 + F21;
    jacobi_eig4(K, V);
    int best = 0;
    for (int i = 1; i < 4; ++i)
        if (K[i][i] > K[best][best]) best = i;
    double w = V[0][best], x = V[1][best], y = V[2][best], z = V[3][best];
    double nq = sqrt(w * w + x * x + y * y + z * z);
    w /= nq; x /= nq; y /= nq; z /= nq;
    R[0] = w * w + x * x - y * y - z * z;
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = w * w - x * x + y * y - z * z;
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = w * w - x * x - y * y + z * z;
}

/* Kirchhoff stress tau = P F^T.
 * model 0: fixed-corotated (Stomakhin et al. 2012, the constitutive law of
 *          the paper's experiments), tau = 2 mu (F - R) F^T + la (J-1) J I,
 *          R the rotation closest to F (orc_closest_rotation).
 * model 1: compressible Neo-Hookean, tau = mu (F F^T - I) + la ln(J) I.
 * Returns ORC_EDOMAIN for J <= 0 with the Neo-Hookean model. */
int orc_kirchhoff(int dim, int model, double mu, double la, const double *F,
                  double *tau)
{
    double J = det(dim, F);
    double FFt[9];
    for (int a = 0; a < dim; ++a)
        for (int b = 0; b < dim; ++b) {
            double s = 0.0;
            for (int k = 0; k < dim; ++k) s += F[a * dim + k] * F[b * dim + k];
            FFt[a * dim + b] = s;
        }
    if (model == 0) {
        double R[9];
        orc_closest_rotation(dim, F, R);
        /* tau = 2 mu (F F^T - R F^T) + la (J - 1) J I */
        for (int a = 0; a < dim; ++a)
            for (int b = 0; b < dim; ++b) {
                double RFt = 0.0;
                for (int k = 0; k < dim; ++k) RFt += R[a * dim + k] * F[b * dim + k];
                tau[a * dim + b] = 2.0 * mu * (FFt[a * dim + b] - RFt)
                                 + (a == b ? la * (J - 1.0) * J : 0.0);
            }
        return ORC_OK;
    }
    if (!(J > 0.0)) return ORC_EDOMAIN;
    double lnJ = log(J);
    for (int a = 0; a < dim; ++a)
        for (int b = 0; b < dim; ++b)
            tau[a * dim + b] = mu * (FFt[a * dim + b] - (a == b ? 1.0 : 0.0))
                             + (a == b ? la * lnJ : 0.0);
    return ORC_OK;
}

/* Particle-to-grid transfer (Algorithm 1, first step; Algorithm 5, first
 * step, when `subset` lists the quadrature points).  Adds into gm (mass),
 * gmv (momentum, dim per node) and gf (internal force, dim per node), which
 * the caller zeroes.  mu and la are the Lame parameters of the material.
 * subset == NULL means all np particles in index order. */
int orc_p2g(int dim, const int *n, double dx, long np, const long *subset,
            const double *x, const double *v, const double *C, const double *F,
            const double *m, const double *V0, int model, double mu, double la,
            int apic, double *gm, double *gmv, double *gf)
{
    int dd = dim * dim;
    for (long s = 0; s < np; ++s) {
        long p = subset ? subset[s] : s;
        const double *xp = x + p * dim;
        int base[3];
        double w[3][3], dw[3][3];
        if (stencil(dim, n, dx, xp, base, w, dw) != ORC_OK) return ORC_EDOMAIN;
        double tau[9];
        if (orc_kirchhoff(dim, model, mu, la, F + p * dd, tau) != ORC_OK)
            return ORC_EDOMAIN;
        int o[3] = {0, 0, 0};
        do {
            int ijk[3];
            double wip = 1.0, grad[3], dxi[3];
            for (int a = 0; a < dim; ++a) {
                ijk[a] = base[a] + o[a];
                wip *= w[a][o[a]];
                dxi[a] = ijk[a] * dx - xp[a];
            }
            for (int b = 0; b < dim; ++b) {
                double g = 1.0;
                for (int a = 0; a < dim; ++a) g *= (a == b) ? dw[a][o[a]] : w[a][o[a]];
                grad[b] = g;
            }
            long i = node_index(dim, n, ijk);
            gm[i] += wip * m[p];
            for (int a = 0; a < dim; ++a) {
                double vel = v[p * dim + a];
                if (apic)
                    for (int b = 0; b < dim; ++b) vel += C[p * dd + a * dim + b] * dxi[b];
                gmv[i * dim + a] += wip * m[p] * vel;
                double f = 0.0;
                for (int b = 0; b < dim; ++b) f += tau[a * dim + b] * grad[b];
                gf[i * dim + a] += -V0[p] * f;
            }
        } while (next_offset(dim, o));
    }
    return ORC_OK;
}

/* Grid update (Algorithm 1, second step): for nodes with mass,
 *   v_i = (m_i v_i)/m_i + dt (f^sigma_i / m_i + g),
 * then the boundary band.  floor_mode 0: all faces sticky.  floor_mode 1:
 * the low-y face is a Coulomb floor with friction coefficient mu_f and
 * normal +y, the other faces sticky.  Writes gv (dim per node). */
void orc_grid_update(int dim, const int *n, double dt, const double *gravity,
                     int bound, int floor_mode, double mu_f,
                     const double *gm, const double *gmv, const double *gf,
                     double *gv)
{
    long nn = 1;
    for (int a = 0; a < dim; ++a) nn *= n[a];
    for (long i = 0; i < nn; ++i) {
        double *vi = gv + i * dim;
        for (int a = 0; a < dim; ++a) vi[a] = 0.0;
        if (!(gm[i] > 0.0)) continue;
        for (int a = 0; a < dim; ++a)
            vi[a] = gmv[i * dim + a] / gm[i] + dt * (gf[i * dim + a] / gm[i] + gravity[a]);
        /* node coordinates */
        int ijk[3];
        long r = i;
        for (int a = 0; a < dim; ++a) { ijk[a] = (int)(r % n[a]); r /= n[a]; }
        int sticky = 0, floor_band = 0;
        for (int a = 0; a < dim; ++a) {
            int lo = ijk[a] < bound, hi = ijk[a] >= n[a] - bound;
            if (floor_mode == 1 && a == 1 && lo) floor_band = 1;
            else if (lo || hi) sticky = 1;
        }
        if (sticky) {
            for (int a = 0; a < dim; ++a) vi[a] = 0.0;
        } else if (floor_band) {
            double vn = vi[1];
            if (vn < 0.0) {
                double vt[3], nt = 0.0;
                for (int a = 0; a < dim; ++a) vt[a] = (a == 1) ? 0.0 : vi[a];
                for (int a = 0; a < dim; ++a) nt += vt[a] * vt[a];
                nt = sqrt(nt);
                if (nt <= -mu_f * vn) {
                    for (int a = 0; a < dim; ++a) vi[a] = 0.0;
                } else {
                    double s = 1.0 + mu_f * vn / nt;
                    for (int a = 0; a < dim; ++a) vi[a] = vt[a] * s;
                }
            }
        }
    }
}

/* Grid-to-particle transfer and advection (Algorithm 1, third and fourth
 * steps; Algorithm 5, last two steps when trial_x/trial_v are given).
 *   full mode  (trial_x == NULL): updates v, C (APIC, else zero), F (if
 *              update_F) and x of the listed particles in place;
 *   trial mode (trial_x != NULL): writes v_trial and x_trial = x + dt v_trial
 *              for the listed particles (s-th entry at s*dim) and leaves the
 *              particle state untouched. */
int orc_g2p(int dim, const int *n, double dx, double dt, long np,
            const long *subset, int apic, int update_F, const double *gv,
            double *x, double *v, double *C, double *F,
            double *trial_x, double *trial_v)
{
    int dd = dim * dim;
    double dinv = 4.0 / (dx * dx);
    for (long s = 0; s < np; ++s) {
        long p = subset ? subset[s] : s;
        double *xp = x + p * dim;
        int base[3];
        double w[3][3], dw[3][3];
        if (stencil(dim, n, dx, xp, base, w, dw) != ORC_OK) return ORC_EDOMAIN;
        double vp[3] = {0, 0, 0}, Bp[9], gradv[9];
        memset(Bp, 0, sizeof Bp);
        memset(gradv, 0, sizeof gradv);
        int o[3] = {0, 0, 0};
        do {
            int ijk[3];
            double wip = 1.0, grad[3], dxi[3];
            for (int a = 0; a < dim; ++a) {
                ijk[a] = base[a] + o[a];
                wip *= w[a][o[a]];
                dxi[a] = ijk[a] * dx - xp[a];
            }
            for (int b = 0; b < dim; ++b) {
                double g = 1.0;
                for (int a = 0; a < dim; ++a) g *= (a == b) ? dw[a][o[a]] : w[a][o[a]];
                grad[b] = g;
            }
            const double *vi = gv + node_index(dim, n, ijk) * dim;
            for (int a = 0; a < dim; ++a) {
                vp[a] += wip * vi[a];
                for (int b = 0; b < dim; ++b) {
                    Bp[a * dim + b] += wip * vi[a] * dxi[b];
                    gradv[a * dim + b] += vi[a] * grad[b];
                }
            }
        } while (next_offset(dim, o));
        if (trial_x) {
            for (int a = 0; a < dim; ++a) {
                trial_v[s * dim + a] = vp[a];
                trial_x[s * dim + a] = xp[a] + dt * vp[a];
            }
            continue;
        }
        for (int a = 0; a < dim; ++a) v[p * dim + a] = vp[a];
        for (int k = 0; k < dd; ++k) C[p * dd + k] = apic ? dinv * Bp[k] : 0.0;
        if (update_F) {
            double Fn[9];
            double *Fp = F + p * dd;
            for (int a = 0; a < dim; ++a)
                for (int b = 0; b < dim; ++b) {
                    double sacc = Fp[a * dim + b];
                    for (int k = 0; k < dim; ++k) sacc += dt * gradv[a * dim + k] * Fp[k * dim + b];
                    Fn[a * dim + b] = sacc;
                }
            memcpy(Fp, Fn, sizeof(double) * dd);
        }
        for (int a = 0; a < dim; ++a) xp[a] += dt * vp[a];
    }
    return ORC_OK;
}

/* Linear index of the stencil base cell of every particle (the cell-sort
 * key); -1 where the stencil leaves the lattice. */
void orc_cell_keys(int dim, const int *n, double dx, long np, const double *x,
                   long *keys)
{
    for (long p = 0; p < np; ++p) {
        int base[3];
        double w[3][3], dw[3][3];
        if (stencil(dim, n, dx, x + p * dim, base, w, dw) != ORC_OK) {
            keys[p] = -1;
            continue;
        }
        keys[p] = node_index(dim, n, base);
    }
}
