"""FP64 oracle of one reduced-order-model time step (Section 3.2,
Algorithm 2) with Lagrangian-quadrature kinematics (Algorithm 3) or
Eulerian-quadrature kinematics (Algorithm 4), the sample-point full-space
dynamics (Algorithm 5) and the projection (Algorithm 6 or 7); plus the
least-squares initial latents (Section 3.1, eq. essentialSpecInt) and the
error metrics of Section 5.

TEST INFRASTRUCTURE ONLY.

Readings:
  - The neighbour test uses stencil membership: a point touches node i when
    i is one of the 3^d nodes base..base+2 of its stencil (a node whose
    quadratic B-spline weight is exactly zero at a support edge is still in
    the stencil; its contribution is zero either way).
  - Quadrature points carry the particle mass m_p and reference volume
    V0_p = m_p / rho0 (Algorithm 3, last step) and no affine velocity
    (Algorithm 5 uses the plain transfer).
  - The grid boundary band of the full-order model applies to the substep.
  Eulerian quadrature (Algorithm 4):
  - Points sit at (m + 1/2) dx / ell along each axis (ell per cell and
    dimension, evenly spaced, volume (dx / ell)^d); the quadrature points of
    a step are those whose stencil touches an active node (the nodes of the
    samples' stencils), the same test as for the Lagrangian neighbours.
  - The map is inverted from X = x^Q by a displacement step X <- x^Q -
    (g(X) - X) (a Newton step with F replaced by I: the guess x - u(x))
    followed by Newton steps with F = dg/dX at the current iterate, for a
    fixed total number of iterations; a point is kept when the final
    residual max-norm is within a tolerance, det F > 0 at the result and X
    lies in the reference body.
  - Mass (Algorithm 4, last step): m^Q = rho0 V^Q / J with V^Q = (dx / ell)^d
    and J = det F, for every point inside the reference body.  The paper does
    not say how a point is found to be in the body; reading used here: the
    reference particles' mass spread with the quadratic B-spline on the
    grid's node lattice (spacing dx), read at X by multilinear interpolation,
    gives a smoothed density rho_ref; with s = rho_ref(X) / rho0 the point
    carries the weight tau(s) = clamp(2 s - 1/2, 0, 1): 1 (mass exactly
    rho0 V^Q / J) wherever s >= 3/4, i.e. everywhere inside a body sampled
    at its nominal density, a linear taper across the surface band (where
    rho_ref falls from rho0 to 0 over about a cell, centred on the half
    level s = 1/2), and 0 (point discarded) where s <= 1/4.  V0 = m^Q / rho0.
    Sample points are not quadrature points.
"""
import numpy as np

from . import decoder as _dec
from . import mpm as _mpm
from . import project as _proj
from . import sampler as _sampler


def stencil_bases(dx, x):
    """Stencil base node per point and dimension: floor(x/dx - 0.5)."""
    return np.floor(np.asarray(x, dtype=np.float64) / dx - 0.5).astype(np.int64)


def _linear(n, ijk):
    idx = ijk[..., -1]
    for a in range(ijk.shape[-1] - 2, -1, -1):
        idx = idx * n[a] + ijk[..., a]
    return idx


def _offsets(dim):
    grids = np.meshgrid(*([np.arange(3)] * dim), indexing="ij")
    return np.stack([g.reshape(-1) for g in grids], axis=1)


def neighbour_set(dim, n, dx, x_all, samples):
    """Algorithm 3, steps 2-3.  Returns (I, Q, N): the sorted active node
    indices, the sorted quadrature-point indices (samples and neighbours),
    and the sorted neighbour indices alone."""
    base = stencil_bases(dx, x_all)
    n_arr = np.asarray(n)
    if np.any(base < 0) or np.any(base + 2 > n_arr - 1):
        raise _mpm.OracleDomainError("decoded point outside the lattice")
    offs = _offsets(dim)
    samples = np.asarray(samples, dtype=np.int64)
    marked = np.zeros(int(np.prod(n)), dtype=bool)
    for o in offs:
        marked[_linear(n, base[samples] + o)] = True
    touches = np.zeros(x_all.shape[0], dtype=bool)
    for o in offs:
        touches |= marked[_linear(n, base + o)]
    is_sample = np.zeros(x_all.shape[0], dtype=bool)
    is_sample[samples] = True
    N = np.nonzero(touches & ~is_sample)[0]
    Q = np.nonzero(touches | is_sample)[0]
    I = np.nonzero(marked)[0]
    return I, Q, N


def neighbour_set_bruteforce(dim, n, dx, x_all, samples):
    """Same sets by direct pairwise comparison of stencils (small inputs)."""
    base = stencil_bases(dx, x_all)
    offs = [tuple(o) for o in _offsets(dim)]
    I = set()
    for p in samples:
        for o in offs:
            I.add(tuple(int(base[p][a] + o[a]) for a in range(dim)))
    S = set(int(s) for s in samples)
    N = []
    for q in range(x_all.shape[0]):
        if q in S:
            continue
        st = set(tuple(int(base[q][a] + o[a]) for a in range(dim)) for o in offs)
        if st & I:
            N.append(q)
    Il = sorted(int(_linear(n, np.array(i))) for i in I)
    return np.array(Il), np.array(sorted(S | set(N))), np.array(N)


def substep(scene, x_Q, F_Q, v_Q, m_Q, V0_Q, x_samples, dt):
    """Algorithm 5: P2G over the quadrature points, grid update, trial G2P
    for the sample points.  Returns (x_trial, v_trial)."""
    dim, n, dx = scene["dim"], scene["n"], scene["dx"]
    Qn = x_Q.shape[0]
    zeroC = np.zeros((Qn, dim, dim))
    gm, gmv, gf = _mpm.p2g(dim, n, dx, x_Q, v_Q, zeroC, F_Q, m_Q, V0_Q,
                           scene["model"], scene["mu"], scene["la"], apic=False)
    gv = _mpm.grid_update(dim, n, dt, scene["gravity"], scene["bound"],
                          scene["floor_mode"], scene["mu_f"], gm, gmv, gf)
    S = x_samples.shape[0]
    return _mpm.g2p(dim, n, dx, dt, gv, x_samples, np.zeros((S, dim)),
                    np.zeros((S, dim, dim)), np.tile(np.eye(dim), (S, 1, 1)),
                    apic=False, trial=True)


def active_nodes(dim, n, dx, x_samples):
    """The nodes of the samples' stencils (Algorithm 3 / 4, step 2), sorted."""
    base = stencil_bases(dx, x_samples)
    n_arr = np.asarray(n)
    if np.any(base < 0) or np.any(base + 2 > n_arr - 1):
        raise _mpm.OracleDomainError("decoded sample outside the lattice")
    nodes = [_linear(n, base + o) for o in _offsets(dim)]
    return np.unique(np.concatenate(nodes)) if len(base) else np.zeros(0, dtype=np.int64)


def density_lattice_shape(n):
    """Nodes per axis of the reference-density lattice (the grid's nodes)."""
    return list(n)


def reference_density(dim, n, dx, X_all, m_all):
    """rho_ref on the grid's node lattice (spacing h = dx): sum over
    reference particles of m_p N((X_k - X_p) / h) / h^d with the tensor
    quadratic B-spline N (stencil base floor(X / h - 1/2)); particles whose
    stencil leaves the lattice are skipped.  Returns a flat array (x
    fastest)."""
    h = dx
    shape = density_lattice_shape(n)
    rho = np.zeros(int(np.prod(shape)))
    X = np.asarray(X_all, dtype=np.float64)
    m = np.broadcast_to(np.asarray(m_all, dtype=np.float64), (X.shape[0],))
    base = np.floor(X / h - 0.5).astype(np.int64)
    ok = np.all((base >= 0) & (base + 2 <= np.asarray(shape) - 1), axis=1)
    X, m, base = X[ok], m[ok], base[ok]
    f = X / h - base
    # quadratic B-spline weights of the three nodes base..base+2 (the MPM
    # kernel of Section 2.2) at offset f in [1/2, 3/2)
    w = [np.stack([0.5 * (1.5 - f[:, a]) ** 2, 0.75 - (f[:, a] - 1.0) ** 2,
                   0.5 * (f[:, a] - 0.5) ** 2], axis=1) for a in range(dim)]
    for o in _offsets(dim):
        wt = np.ones(len(X))
        for a in range(dim):
            wt = wt * w[a][:, o[a]]
        np.add.at(rho, _linear(shape, base + o), m * wt / h ** dim)
    return rho


def density_at(rho, dim, n, dx, X):
    """Multilinear interpolation of the node-lattice density at points X (0
    outside the lattice)."""
    h = dx
    shape = np.asarray(density_lattice_shape(n))
    t = np.asarray(X, dtype=np.float64) / h
    i0 = np.floor(t).astype(np.int64)
    fr = t - i0
    ok = np.all((i0 >= 0) & (i0 + 1 <= shape - 1), axis=1)
    out = np.zeros(len(t))
    for c in _offsets(dim):
        if np.any(c > 1):
            continue
        wt = np.ones(len(t))
        for a in range(dim):
            wt = wt * np.where(c[a] == 1, fr[:, a], 1.0 - fr[:, a])
        idx = np.where(ok[:, None], i0 + c, 0)
        out += np.where(ok, wt * rho[_linear(list(shape), idx)], 0.0)
    return out


def quadrature_lattice(dim, n, dx, ell):
    """Every Eulerian quadrature point of the domain, (m + 1/2) dx / ell per
    axis over the n - 1 cells per axis; returns (points (M, d), base (M, d))."""
    axes = [(np.arange((n[a] - 1) * ell) + 0.5) * (dx / ell) for a in range(dim)]
    grids = np.meshgrid(*axes, indexing="ij")
    pts = np.stack([g.reshape(-1) for g in grids], axis=1)
    return pts, stencil_bases(dx, pts)


def eulerian_points(dim, n, dx, ell, I):
    """Algorithm 4, step 3: the quadrature points whose stencil lies in the
    lattice and touches a node of I."""
    pts, base = quadrature_lattice(dim, n, dx, ell)
    n_arr = np.asarray(n)
    inside = np.all((base >= 0) & (base + 2 <= n_arr - 1), axis=1)
    pts, base = pts[inside], base[inside]
    marked = np.zeros(int(np.prod(n)), dtype=bool)
    marked[np.asarray(I, dtype=np.int64)] = True
    touch = np.zeros(len(pts), dtype=bool)
    for o in _offsets(dim):
        touch |= marked[_linear(n, base + o)]
    return pts[touch]


def invert_map(jac_fn, x_target, iters):
    """Solves g(X) = x_target from X0 = x_target: the first iteration is
    X <- X - (g(X) - x_target) (Jacobian replaced by I), every later one a
    Newton step X <- X - F(X)^{-1} (g(X) - x_target); `iters` iterations in
    all.  jac_fn(X) returns (g, F)."""
    X = np.array(x_target, dtype=np.float64)
    for k in range(iters):
        g, F = jac_fn(X)
        if k == 0:
            X = X - (g - x_target)
        else:
            X = X - np.linalg.solve(F, (g - x_target)[..., None])[..., 0]
    return X


def body_weight(s):
    """Weight of a quadrature point whose reference position has smoothed
    relative density s = rho_ref / rho0: 1 for s >= 3/4, 0 for s <= 1/4,
    linear in between (the surface band)."""
    return np.clip(2.0 * np.asarray(s, dtype=np.float64) - 0.5, 0.0, 1.0)


def eulerian_quadrature(dec, dim, n, dx, x_samples, zhat, vhat, ell, iters, tol, rho0,
                        rho_ref):
    """Algorithm 4: quadrature points, their reference positions (inverse
    map), F, v and masses m^Q = tau rho0 V^Q / J (rho_ref: reference_density
    on the node lattice, tau = body_weight(rho_ref / rho0)).  Returns a dict
    with the kept points' xQ, FQ, vQ, mQ, V0Q, their reference positions XQ,
    and I and the candidate count."""
    I = active_nodes(dim, n, dx, x_samples)
    xq = eulerian_points(dim, n, dx, ell, I)
    jac = lambda X: _dec.decode_jac(dec, X, zhat)[:2]
    X = invert_map(jac, xq, iters)
    x, F, _, v = _dec.decode_jac(dec, X, zhat, vhat)
    det = np.linalg.det(F) if len(F) else np.zeros(0)
    conv = np.max(np.abs(x - xq), axis=1) <= tol if len(x) else np.zeros(0, dtype=bool)
    rho = density_at(rho_ref, dim, n, dx, X)
    tau = body_weight(rho / rho0)
    keep = conv & (det > 0.0) & (tau > 0.0)
    Vq = (dx / ell) ** dim
    m = tau[keep] * rho0 * Vq / det[keep]
    return {"xQ": xq[keep], "XQ": X[keep], "FQ": F[keep], "vQ": v[keep], "mQ": m,
            "V0Q": m / rho0, "I": I, "n_candidates": len(xq), "keep": keep,
            "X_all": X, "x_candidates": xq, "rho": rho, "tau": tau}


def initial_fields(dec, X_all, xhat0, vhat0, V0):
    """The correction fields that make the initial conditions exact
    (Section 3.1, eqs. defMapApproxForm and essentialSpec, with the time
    function t -> t) for a uniform initial velocity V0 (d,):
        a(X) = X - g(X; xhat0)             grad a = I - dg/dX (X; xhat0)
        b(X) = V0 - dg/dxhat (X; xhat0) vhat0
        grad b = - d/dX [dg/dxhat (X; xhat0) vhat0]   (grad V0 = 0)
    at every row of X_all.  Returns dict a, b (P, d), Ga, Gb (P, d, d)."""
    X = np.asarray(X_all, dtype=np.float64)
    x0, F0, _, v = _dec.decode_jac(dec, X, xhat0, vhat0)
    d = X.shape[1]
    return {"a": X - x0, "b": np.asarray(V0, dtype=np.float64)[None] - v,
            "Ga": np.eye(d)[None] - F0, "Gb": -_dec.mixed_jac(dec, X, xhat0, vhat0)}


def rom_step(dec, scene, X_all, m_all, V0_all, zhat, zhat_prev, vhat, dt,
             samples, opts, quadrature="lagrangian", ell=2, newton_iters=2, newton_tol=None,
             rho0=None, rho_ref=None, fields=None, t=0.0):
    """One ROM step (Algorithm 2) with Lagrangian (Algorithm 3) or Eulerian
    (Algorithm 4) quadrature kinematics.  Returns (zhat_next, vhat_next,
    info).  Eulerian: rho0 and the reference density lattice are required;
    newton_tol defaults to 1e-3 dx.  fields (Lagrangian only): the output
    of initial_fields; the kinematics are then those of
    g~(X, xhat, t) = g(X; xhat) + a(X) + b(X) t at the step's start time t
    (positions g + a + b t, deformation gradient dg/dX + grad a + t grad b,
    velocity (dg/dxhat) vhat + b), and the projection fits g~ at t + dt:
    positions to x_trial - a - b (t + dt), velocities to v_trial - b."""
    dim, n, dx = scene["dim"], scene["n"], scene["dx"]
    samples = np.asarray(samples, dtype=np.int64)
    if fields is not None and quadrature != "lagrangian":
        raise ValueError("correction fields need the Lagrangian quadrature")
    if quadrature == "eulerian":
        x_s = _dec.decode(dec, X_all[samples], zhat)
        tol = 1e-3 * dx if newton_tol is None else newton_tol
        eq = eulerian_quadrature(dec, dim, n, dx, x_s, zhat, vhat, ell, newton_iters, tol, rho0,
                                 rho_ref)
        x_trial, v_trial = substep(scene, eq["xQ"], eq["FQ"], eq["vQ"], eq["mQ"], eq["V0Q"], x_s,
                                   dt)
        info = {"I": eq["I"], "eulerian": eq}
    else:
        x_all = _dec.decode(dec, X_all, zhat)
        if fields is not None:
            x_all = x_all + fields["a"] + fields["b"] * t
        I, Q, N = neighbour_set(dim, n, dx, x_all, samples)
        xQ, FQ, JQ, vQ = _dec.decode_jac(dec, X_all[Q], zhat, vhat)
        if fields is not None:
            xQ = xQ + fields["a"][Q] + fields["b"][Q] * t
            FQ = FQ + fields["Ga"][Q] + fields["Gb"][Q] * t
            vQ = vQ + fields["b"][Q]
        pos = np.searchsorted(Q, samples)
        x_trial, v_trial = substep(scene, xQ, FQ, vQ, np.asarray(m_all)[Q],
                                   np.asarray(V0_all)[Q], xQ[pos], dt)
        info = {"I": I, "Q": Q, "N": N}
    if fields is not None:
        # g~ at t + dt is g + a + b (t + dt): the fields move to the targets
        x_fit = x_trial - fields["a"][samples] - fields["b"][samples] * (t + dt)
        v_fit = v_trial - fields["b"][samples]
    else:
        x_fit, v_fit = x_trial, v_trial
    z, vh, it, f, status = _proj.project(dec, X_all[samples], x_fit, v_fit,
                                         zhat, zhat_prev, dt, opts)
    info.update({"x_trial": x_trial, "v_trial": v_trial, "iters": it, "objective": f,
                 "status": status})
    return z, vh, info


# failures that hand the run over to the full-order model
FALLBACK_STATUS = _proj.STATUS_SINGULAR | _proj.STATUS_NOCONV
STATUS_DOMAIN = 1 << 8      # stress undefined (J <= 0), NaN, or a point off the lattice


def full_state_from_latent(dec, X_all, zhat, vhat):
    """The full-order state the reduced one stands for (Section 3.1:
    x = g(X; xhat), F = dg/dX, v = (dg/dxhat) vhat), with C = 0 since the
    reduced substep carries no affine term."""
    x, F, _, v = _dec.decode_jac(dec, X_all, zhat, vhat)
    return {"x": x, "v": v, "C": np.zeros_like(F), "F": F}


def run_with_fallback(dec, scene, X_all, zhat, zhat_prev, vhat, dt, n_steps, sample_fn, opts,
                      apic=False, **rom_kwargs):
    """Reduced steps (rom_step with scene["m"], scene["V0"]) until one fails
    (a singular normal matrix, Gauss-Newton above tolerance, or a domain
    error); from the last good latent state the full-order state is
    reconstructed and the remaining steps, the failed one included, run
    with Algorithm 1.  sample_fn(step) gives the sample indices.
    Returns (state, fallback step or None, failing status, full-order
    status): state is the full-order state at the end (reconstructed from
    the final latents when no step failed)."""
    m_all, V0_all = scene["m"], scene["V0"]
    for k in range(n_steps):
        try:
            zn, vn, info = rom_step(dec, scene, X_all, m_all, V0_all, zhat, zhat_prev, vhat, dt,
                                    sample_fn(k), opts, **rom_kwargs)
            bad = info["status"] & FALLBACK_STATUS
            if not bad and not (np.all(np.isfinite(zn)) and np.all(np.isfinite(vn))):
                bad = STATUS_DOMAIN
        except _mpm.OracleDomainError:
            bad = STATUS_DOMAIN
        if bad:
            state = full_state_from_latent(dec, X_all, zhat, vhat)
            fom_status = 0
            try:
                for _ in range(k, n_steps):
                    state = _mpm.step(scene, state, dt, apic=apic)
            except _mpm.OracleDomainError:
                fom_status = STATUS_DOMAIN
            return state, k, bad, fom_status
        zhat_prev, zhat, vhat = zhat, zn, vn
    return full_state_from_latent(dec, X_all, zhat, vhat), None, 0, 0


def rom_init(dec, X, V, opts, z0=None):
    """Least-squares initial latents (eq. essentialSpecInt by point
    quadrature): xhat_0 minimises sum ||X - g(X; z)||^2 by Gauss-Newton
    from z0 (zero by default); vhat_0 minimises sum ||V - J(X; xhat_0) v||^2.
    Returns (xhat_0, vhat_0, status)."""
    r = dec.r
    z0 = np.zeros(r) if z0 is None else np.asarray(z0, dtype=np.float64)
    z, _, _, status = _proj.gauss_newton(dec, X, np.asarray(X, dtype=np.float64), z0, opts)
    _, _, J, _ = _dec.decode_jac(dec, X, z)
    vh = _proj.velocity_ls(J, V, opts.damping)
    return z, vh, status


def sample_indices(seed, instance, step, n_samples, n_particles):
    return np.array(_sampler.stratified_samples(seed, instance, step, n_samples,
                                                n_particles), dtype=np.int64)


class ErrorAccumulator:
    """Accumulates the error sums of Section 5 over steps, particles and
    instances: the paper's position error 100 sqrt(sum|x_rom - x|^2) /
    sqrt(sum|x|^2) and the displacement-relative error
    sqrt(sum|x_rom - x|^2) / sqrt(sum|x - X|^2)."""

    def __init__(self):
        self.num = 0.0
        self.den_pos = 0.0
        self.den_disp = 0.0

    def add(self, x_rom, x_full, X):
        x_rom = np.asarray(x_rom, dtype=np.float64)
        x_full = np.asarray(x_full, dtype=np.float64)
        self.num += float(np.sum((x_rom - x_full) ** 2))
        self.den_pos += float(np.sum(x_full ** 2))
        self.den_disp += float(np.sum((x_full - np.asarray(X, dtype=np.float64)) ** 2))

    def position_percent(self):
        return 100.0 * np.sqrt(self.num) / np.sqrt(self.den_pos)

    def displacement_relative(self):
        return np.sqrt(self.num) / np.sqrt(self.den_disp)
