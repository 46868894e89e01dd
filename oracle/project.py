"""FP64 oracle of the reduced-space dynamics: projection of the sample
points' trial positions and velocities onto the manifold.

TEST INFRASTRUCTURE ONLY.

Follows Section 3.2.4:
  - Algorithm 6 (position-velocity projection):
        vhat_{n+1} = argmin_v  sum_p || dg/dxhat(X_p; xhat_n) v - v_trial_p ||^2
        xhat_{n+1} = argmin_z  sum_p || g(X_p; z) - x_trial_p ||^2
    the second solved by Gauss-Newton with backtracking, from the initial
    guess 2 xhat_n - xhat_{n-1} (Section 5, implementation details).
  - Algorithm 7 (velocity-only projection): the same vhat_{n+1}, then
        xhat_{n+1} = xhat_n + dt vhat_{n+1}.
Readings: Armijo sufficient-decrease test f(z + a d) <= f(z) + c a grad.d with
c = 1e-4, step halved at most max_backtrack times, and a rejected step
(no acceptable a) ends the iteration with the step discarded; stopping rule
||a d||_2 <= tol_step (1 + ||z||_2) or max_iter iterations, or exactly
max_iter iterations in fixed-iteration mode.

The least-squares subproblems use numpy.linalg.lstsq on the stacked
(d*S) x r system (or the damped normal equations when damping > 0).
"""
import numpy as np

from . import decoder as _dec

MODE_POS_VEL = 0
MODE_VEL_ONLY = 1

STATUS_OK = 0
STATUS_SINGULAR = 1
STATUS_NOCONV = 2
STATUS_LINESEARCH = 4


class GNOptions:
    def __init__(self, mode=MODE_POS_VEL, max_iter=20, max_backtrack=8,
                 armijo_c=1e-4, tol_step=1e-10, damping=0.0, fixed_iters=False):
        self.mode = mode
        self.max_iter = max_iter
        self.max_backtrack = max_backtrack
        self.armijo_c = armijo_c
        self.tol_step = tol_step
        self.damping = damping
        self.fixed_iters = fixed_iters


def _solve_ls(A, b, damping=0.0):
    """argmin_y ||A y - b||^2 (+ damping ||y||^2)."""
    if damping > 0.0:
        N = A.T @ A + damping * np.eye(A.shape[1])
        return np.linalg.solve(N, A.T @ b)
    y, _, rank, _ = np.linalg.lstsq(A, b, rcond=None)
    if rank < A.shape[1]:
        raise np.linalg.LinAlgError("rank-deficient least-squares system")
    return y


def velocity_ls(J, v_trial, damping=0.0):
    """Generalized velocity from J (S, d, r) and trial velocities (S, d)."""
    S, d, r = J.shape
    return _solve_ls(J.reshape(S * d, r), np.asarray(v_trial).reshape(S * d), damping)


def objective(dec, X_s, x_trial, z):
    res = _dec.decode(dec, X_s, z) - x_trial
    return 0.5 * float(np.sum(res * res))


def gauss_newton(dec, X_s, x_trial, z0, opts):
    """Minimise 0.5 sum_p ||g(X_p; z) - x_trial_p||^2 from z0.
    Returns (z, iterations, final objective, status bits)."""
    z = np.array(z0, dtype=np.float64)
    x_trial = np.asarray(x_trial, dtype=np.float64)
    S, d = x_trial.shape
    status = STATUS_OK
    it = 0
    f = objective(dec, X_s, x_trial, z)
    converged = False
    while it < opts.max_iter:
        x, _, J, _ = _dec.decode_jac(dec, X_s, z)
        res = (x - x_trial).reshape(S * d)
        A = J.reshape(S * d, -1)
        try:
            delta = -_solve_ls(A, res, opts.damping)
        except np.linalg.LinAlgError:
            status |= STATUS_SINGULAR
            break
        slope = float((A.T @ res) @ delta)
        alpha = 1.0
        accepted = False
        for _ in range(opts.max_backtrack + 1):
            f_new = objective(dec, X_s, x_trial, z + alpha * delta)
            if f_new <= f + opts.armijo_c * alpha * slope:
                accepted = True
                break
            alpha *= 0.5
        it += 1
        if not accepted:
            status |= STATUS_LINESEARCH
            break
        z = z + alpha * delta
        f = f_new
        if not opts.fixed_iters:
            if np.linalg.norm(alpha * delta) <= opts.tol_step * (1.0 + np.linalg.norm(z)):
                converged = True
                break
    if not opts.fixed_iters and not converged and not (status & STATUS_SINGULAR):
        status |= STATUS_NOCONV
    return z, it, f, status


def project(dec, X_s, x_trial, v_trial, zhat_n, zhat_prev, dt, opts):
    """Reduced-space dynamics (Algorithm 6 or 7).  Returns
    (zhat_{n+1}, vhat_{n+1}, iterations, objective, status)."""
    _, _, J, _ = _dec.decode_jac(dec, X_s, zhat_n)
    try:
        vhat = velocity_ls(J, v_trial, opts.damping)
    except np.linalg.LinAlgError:
        r = J.shape[2]
        return np.array(zhat_n, dtype=float), np.zeros(r), 0, np.inf, STATUS_SINGULAR
    if opts.mode == MODE_VEL_ONLY:
        z = np.asarray(zhat_n, dtype=np.float64) + dt * vhat
        return z, vhat, 0, objective(dec, X_s, x_trial, z) if x_trial is not None else 0.0, STATUS_OK
    z0 = 2.0 * np.asarray(zhat_n, dtype=np.float64) - np.asarray(zhat_prev, dtype=np.float64)
    z, it, f, status = gauss_newton(dec, X_s, x_trial, z0, opts)
    return z, vhat, it, f, status
