"""Reduced-order run with the full-order model as its fallback.

The reduced model stands for the full-order state x = g(X; xhat),
F = dg/dX, v = (dg/dxhat) vhat (Section 3.1, eqs. kinematicRestriction,
defGrad, timederOne).  When a reduced step fails -- the normal matrix of
the projection is singular (too few or degenerate samples, Section 3.2.1),
Gauss-Newton stops above its tolerance, or a quadrature point has J <= 0,
a NaN or a stencil off the lattice -- the run hands over to the full-order
model (Algorithm 1) from that state, reconstructed at the last latent state
known to be good, and the full-order model redoes the remaining steps.

The reduced steps run in chunks (one HIP graph per chunk); the status word
of a chunk is read after it, so the hand-over happens at the start of the
failing chunk (chunk = 1 hands over at the failing step itself).  Every
step runs in the library's kernels; this module only sequences them.
"""
import numpy as np
import torch

from . import binding as B

FALLBACK_FLAGS = B.FLAG_SINGULAR | B.FLAG_NOCONV | B.FLAG_DOMAIN


def full_state_from_latent(dec, X, zhat, vhat, m_uniform, V0_uniform):
    """Particles (reference order) of the full-order state a latent state
    stands for: x, F and v decoded at every reference position X (d, P);
    C = 0 (the reduced substep carries no affine term)."""
    d, P = X.shape
    x = torch.empty(1, d, P, device=X.device)
    F = torch.empty(1, d * d, P, device=X.device)
    v = torch.empty(1, d, P, device=X.device)
    B.rom_decode_jac(dec, X, zhat[:1].contiguous(), vhat=vhat[:1].contiguous(), x=x, F=F, v=v)
    return B.Particles(x[0].contiguous(), v[0].contiguous(), torch.zeros(d * d, P, device=X.device),
                       F[0].contiguous(), m_uniform=m_uniform, V0_uniform=V0_uniform)


def run_with_fallback(dec, scene, E, zhat, zhat_prev, vhat, n_steps, n_samples, opts,
                      chunk=10, sort_every=10, affine=False, seed=7, use_graph=True, **rom_kwargs):
    """n_steps reduced steps of one instance (Young's modulus E) from the
    latent state (zhat, zhat_prev, vhat: (1, r) float64 device tensors,
    advanced in place while the reduced model runs), falling back to the
    full-order model on failure.  Returns a dict: "x", "v", "F" (d, P) of
    the final full-order state in reference order, "fallback_step" (step
    at which the full-order model took over, or None), "status" (flags of
    the failing chunk, 0 when none failed) and "fom_status" (flags the
    full-order run raised)."""
    X = torch.tensor(np.ascontiguousarray(scene["X"].T), device=zhat.device)
    d, P = X.shape
    grid = B.Grid(scene["dim"], scene["n"], scene["dx"], scene["bound"], scene["floor_mode"],
                  scene["mu_f"], scene["gravity"])
    rom = B.Rom(dec, grid, X, torch.tensor([float(E)], device=X.device),
                torch.tensor([n_samples], dtype=torch.int32, device=X.device), opts, seed=seed,
                rho0=float(scene["rho"]), m_uniform=float(scene["m"]), model=scene["model"],
                nu=scene["nu"], **rom_kwargs)
    m_u, V0_u = float(scene["m"]), float(scene["V0"])
    st = torch.zeros(1, dtype=torch.int32, device=X.device)
    done = 0
    try:
        while done < n_steps:
            k = min(chunk, n_steps - done)
            good = (zhat.clone(), zhat_prev.clone(), vhat.clone())
            st.zero_()
            rom.step(k, done, scene["dt"], zhat, zhat_prev, vhat, status=st, use_graph=use_graph)
            flags = int(st.item())
            finite = bool(torch.isfinite(zhat).all() and torch.isfinite(vhat).all())
            if (flags & FALLBACK_FLAGS) or not finite:
                parts = full_state_from_latent(dec, X, good[0], good[2], m_u, V0_u)
                fom_flags = _full_order(scene, E, parts, n_steps - done, sort_every, affine, grid)
                return {"x": parts.x, "v": parts.v, "F": parts.F, "fallback_step": done,
                        "status": flags if flags & FALLBACK_FLAGS else B.FLAG_DOMAIN,
                        "fom_status": fom_flags}
            done += k
    finally:
        rom.close()
    parts = full_state_from_latent(dec, X, zhat, vhat, m_u, V0_u)
    return {"x": parts.x, "v": parts.v, "F": parts.F, "fallback_step": None, "status": 0,
            "fom_status": 0}


def _full_order(scene, E, parts, n_steps, sort_every, affine, grid):
    """Advances the particles n_steps with mpm_step and restores the
    reference order in place; returns the raised flags."""
    P = parts.n
    dev = parts.x.device
    gbuf = torch.zeros(grid.nodes() * 4, device=dev)
    ws = torch.zeros(B.mpm_step_workspace_bytes(grid, P), dtype=torch.uint8, device=dev)
    perm = torch.zeros(P, dtype=torch.int32, device=dev)
    flag = torch.zeros(1, dtype=torch.int32, device=dev)
    if n_steps > 0:
        B.mpm_step(grid, (scene["model"], float(E), scene["nu"]), parts, scene["dt"], n_steps,
                   sort_every, 0 if affine else B.NO_AFFINE, gbuf, ws, perm_accum=perm,
                   status=flag)
        inv = torch.empty(P, dtype=torch.long, device=dev)
        inv[perm.long()] = torch.arange(P, device=dev)
        for name in ("x", "v", "C", "F"):
            setattr(parts, name, getattr(parts, name)[:, inv].contiguous())
    return int(flag.item())
