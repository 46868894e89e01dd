"""Reduced-order model against the full-order model on the same parameters
(paper Section 5: the full-order solution judges the reduced one).

`fom_positions` runs mpm_step and records particle positions (in reference
order); `rom_positions` initialises the latent state by the least-squares
initial conditions (Section 3.1, eq. essentialSpecInt, by point quadrature
over a particle subset: rom_project with x_trial = X, then the velocity
problem at that latent), runs rom_step and decodes every particle at the
recorded steps (rom_decode); `displacement_error` accumulates
sqrt(sum |x_rom - x_fom|^2) / sqrt(sum |x_fom - X|^2) over steps and
particles, and the paper's position error in percent.
"""
import numpy as np
import torch

from . import binding as B


def _grid(scene):
    return B.Grid(scene["dim"], scene["n"], scene["dx"], scene["bound"], scene["floor_mode"],
                  scene["mu_f"], scene["gravity"])


def fom_positions(scene, E, v0, n_steps, record_every, sort_every=10, affine=True,
                  device="cuda"):
    """Full-order positions at steps 0, record_every, ... (reference order),
    as a list of (d, P) float32 device tensors.  affine=False runs the
    transfers without the APIC affine term (the PIC scheme of Algorithm 1,
    which the reduced-order substep of Algorithm 5 also uses)."""
    d, P = scene["dim"], scene["P"]
    soa = lambda a: torch.tensor(np.ascontiguousarray(a.reshape(P, -1).T), device=device)
    v = np.tile(np.asarray(v0, dtype=np.float32), (P, 1))
    parts = B.Particles(soa(scene["X"]), soa(v), torch.zeros(d * d, P, device=device),
                        soa(np.tile(np.eye(d, dtype=np.float32), (P, 1, 1))),
                        m_uniform=float(scene["m"]), V0_uniform=float(scene["V0"]))
    grid = _grid(scene)
    gbuf = torch.zeros(grid.nodes() * 4, device=device)
    ws = torch.zeros(B.mpm_step_workspace_bytes(grid, P), dtype=torch.uint8, device=device)
    perm = torch.zeros(P, dtype=torch.int32, device=device)
    flag = torch.zeros(1, dtype=torch.int32, device=device)
    slot_of = torch.arange(P, device=device)
    out = [parts.x.clone()]
    done = 0
    while done < n_steps:
        k = min(record_every, n_steps - done)
        B.mpm_step(grid, (scene["model"], float(E), scene["nu"]), parts, scene["dt"], k,
                   sort_every, 0 if affine else B.NO_AFFINE, gbuf, ws, perm_accum=perm,
                   status=flag)
        inv = torch.empty(P, dtype=torch.long, device=device)
        inv[perm.long()] = torch.arange(P, device=device)
        slot_of = inv[slot_of]
        done += k
        out.append(parts.x[:, slot_of].contiguous())
    rc, fl = B.sync_status(flag)
    if rc != 0:
        raise RuntimeError("full-order model raised %s" % fl)
    return out


def rom_initial_state(dec, scene, v0, z_guess=None, n_quad=65536, seed=0, iters=8,
                      device="cuda"):
    """Least-squares initial latent position and velocity over a random
    subset of n_quad particles (point quadrature of the two integrals).  The
    Gauss-Newton iteration starts at z_guess (default 0): the latent codes a
    decoder was trained with for the initial frame of its simulations (all
    of which start from the reference configuration) are the natural start,
    since a network can map several codes to the same configuration and the
    dynamics are only trained along the codes it has seen."""
    P, d, r = scene["P"], scene["dim"], dec.r
    rng = np.random.default_rng(seed)
    q = np.sort(rng.choice(P, size=min(n_quad, P), replace=False)).astype(np.int32)
    X = torch.tensor(np.ascontiguousarray(scene["X"].T), device=device)
    idx = torch.tensor(q[None, :], device=device)
    x_trial = X[:, idx[0].long()].contiguous()[None]
    v_trial = torch.tensor(np.tile(np.asarray(v0, np.float32)[:, None], (1, len(q))), device=device)[None]
    z0 = torch.zeros(1, r, dtype=torch.float64, device=device)
    if z_guess is not None:
        z0[0] = torch.as_tensor(np.asarray(z_guess, dtype=np.float64), device=device)
    z = torch.zeros_like(z0)
    vh = torch.zeros_like(z0)
    B.rom_project(dec, X, idx, x_trial.contiguous(), v_trial.contiguous(), z0, z0, 1.0,
                  B.gn_opts(mode=B.POS_VEL, max_iter=iters, proj_fp32=2), z, vh)
    vh2 = torch.zeros_like(z0)
    zz = torch.zeros_like(z0)
    B.rom_project(dec, X, idx, x_trial.contiguous(), v_trial.contiguous(), z, z, 0.0,
                  B.gn_opts(mode=B.VEL_ONLY, max_iter=0, proj_fp32=2), zz, vh2)
    return z, vh2


def rom_initial_states(dec, scene, v0s, z_candidates, n_quad=65536, seed=0, iters=8, chunk=64,
                       device="cuda"):
    """rom_initial_state for many initial velocities.  The position problem
    (x = X at t = 0) is solved from each candidate code (z_candidates: [c][r],
    e.g. the codes a decoder was trained with for the initial frames of its
    simulations, which all start from the reference configuration); a
    network can hold the reference configuration at several codes whose
    tangent spaces differ, so each instance starts at the candidate whose
    latent Jacobian J best represents its initial velocity: with v uniform
    over the points, the least-squares residual is the quadratic form
    v^T (n I - M (J^T J)^-1 M^T) v, M = sum_p J_p (d x r), formed once per
    candidate.  The velocity problems then run at the chosen codes in
    batched rom_project calls of `chunk` instances.  Returns z, vh: [len(v0s),
    r] float64 device tensors and the chosen candidate per instance."""
    P, d, r = scene["P"], scene["dim"], dec.r
    rng = np.random.default_rng(seed)
    q = np.sort(rng.choice(P, size=min(n_quad, P), replace=False)).astype(np.int32)
    nq = len(q)
    X = torch.tensor(np.ascontiguousarray(scene["X"].T), device=device)
    qi = torch.tensor(q, device=device).long()
    Xq = X[:, qi].contiguous()
    cand = torch.as_tensor(np.asarray(z_candidates, dtype=np.float64), device=device)
    nc = cand.shape[0]
    # position least squares from every candidate (one batched projection)
    idx = torch.tensor(np.tile(q[None, :], (nc, 1)), device=device)
    x_trial = Xq[None].expand(nc, d, nq).contiguous()
    v_zero = torch.zeros(nc, d, nq, device=device)
    zc = torch.zeros_like(cand)
    junk = torch.zeros_like(cand)
    B.rom_project(dec, X, idx, x_trial, v_zero, cand.contiguous(), cand.contiguous(), 1.0,
                  B.gn_opts(mode=B.POS_VEL, max_iter=iters, proj_fp32=2), zc, junk)
    # per candidate: J^T J and M = sum_p J_p from the latent Jacobian
    Jz = torch.zeros(nc, d * r, nq, device=device)
    B.rom_decode_jac(dec, Xq, zc, Jz=Jz)
    J = Jz.double().reshape(nc, d, r, nq).permute(0, 3, 1, 2).reshape(nc, nq * d, r)
    JtJ = J.transpose(1, 2) @ J                               # [c][r][r]
    M = Jz.double().reshape(nc, d, r, nq).sum(-1)             # [c][d][r]
    Q = nq * torch.eye(d, dtype=torch.float64, device=device)[None] - \
        M @ torch.linalg.solve(JtJ, M.transpose(1, 2))        # [c][d][d]
    V = torch.as_tensor(np.asarray(v0s, dtype=np.float64), device=device)   # [b][d]
    res = torch.einsum("bi,cij,bj->bc", V, Q, V)
    choice = res.argmin(1)
    z = zc[choice].contiguous()
    Bn = len(v0s)
    vh = torch.zeros(Bn, r, dtype=torch.float64, device=device)
    opts = B.gn_opts(mode=B.VEL_ONLY, max_iter=0, proj_fp32=2)
    for c0 in range(0, Bn, chunk):
        c1 = min(Bn, c0 + chunk)
        nb = c1 - c0
        idx = torch.tensor(np.tile(q[None, :], (nb, 1)), device=device)
        x_t = Xq[None].expand(nb, d, nq).contiguous()
        v_t = V[c0:c1].float()[:, :, None].expand(nb, d, nq).contiguous()
        zz = z[c0:c1].contiguous()
        zo = torch.zeros_like(zz)
        vv = torch.zeros_like(zz)
        B.rom_project(dec, X, idx, x_t, v_t, zz, zz, 0.0, opts, zo, vv)
        vh[c0:c1] = vv
    return z, vh, choice.cpu().numpy()


def nearest_codes(dec, scene, frames, codes, n_sub=4096, seed=1, device="cuda"):
    """For each frame (d, P), the row of codes whose decoding of a random
    subset of n_sub particles is closest to the frame on that subset: a
    starting point for the projection of a frame of an unseen simulation."""
    P, d = scene["P"], scene["dim"]
    rng = np.random.default_rng(seed)
    q = torch.tensor(np.sort(rng.choice(P, size=min(n_sub, P), replace=False)), device=device).long()
    X = torch.tensor(np.ascontiguousarray(scene["X"].T), device=device)
    Xq = X[:, q].contiguous()
    C = torch.as_tensor(np.asarray(codes, dtype=np.float64), device=device).contiguous()
    xb = torch.zeros(C.shape[0], d, len(q), device=device)
    B.rom_decode(dec, Xq, C, xb)
    out = []
    for f in frames:
        res = ((xb - f[:, q][None]) ** 2).sum((1, 2))
        out.append(C[int(res.argmin().item())].cpu().numpy())
    return out


def best_projection(dec, scene, frames, z_guesses, n_quad=65536, seed=0, iters=6,
                    device="cuda"):
    """The decoder's best approximation of given full-order frames (the
    error floor of any reduced trajectory on its manifold): for each frame,
    the latent that minimises sum |g(X_p; z) - x_p|^2 over a random subset
    of n_quad particles, by Gauss-Newton (rom_project) from z_guesses[k],
    then every particle decoded there.  Returns the decoded frames."""
    P, d, r = scene["P"], scene["dim"], dec.r
    rng = np.random.default_rng(seed)
    q = np.sort(rng.choice(P, size=min(n_quad, P), replace=False)).astype(np.int32)
    X = torch.tensor(np.ascontiguousarray(scene["X"].T), device=device)
    idx = torch.tensor(q[None, :], device=device)
    qi = idx[0].long()
    v_trial = torch.zeros(1, d, len(q), device=device)
    opts = B.gn_opts(mode=B.POS_VEL, max_iter=iters, proj_fp32=2)
    ws = torch.empty(B.rom_project_workspace_bytes(dec, 1, len(q), opts), dtype=torch.uint8,
                     device=device)
    xbuf = torch.zeros(1, d, P, device=device)
    out = []
    for k, xf in enumerate(frames):
        z0 = torch.as_tensor(np.asarray(z_guesses[k], dtype=np.float64), device=device)[None]
        z = torch.zeros_like(z0)
        vh = torch.zeros_like(z0)
        B.rom_project(dec, X, idx, xf[:, qi].contiguous()[None], v_trial, z0.contiguous(),
                      z0.contiguous(), 1.0, opts, z, vh, workspace=ws)
        B.rom_decode(dec, X, z, xbuf)
        out.append(xbuf[0].clone())
    return out


def rom_positions(dec, scene, E, v0, n_steps, record_every, n_samples, opts, seed=7,
                  use_graph=True, z_guess=None, device="cuda", progress=None, exact_ic=False,
                  **rom_kwargs):
    """Reduced-order positions of every particle at the recorded steps and
    the step statistics.  rom_kwargs go to the runner (e.g. the Eulerian
    quadrature options); progress(step) is called after each recorded
    chunk.  exact_ic: the runner carries the initial-condition correction
    fields of the least-squares initial latents (rom_set_fields), and the
    positions include them."""
    P, d = scene["P"], scene["dim"]
    X = torch.tensor(np.ascontiguousarray(scene["X"].T), device=device)
    grid = _grid(scene)
    rom = B.Rom(dec, grid, X, torch.tensor([float(E)], device=device),
                torch.tensor([n_samples], dtype=torch.int32, device=device), opts, seed=seed,
                rho0=float(scene["rho"]), m_uniform=float(scene["m"]),
                model=scene["model"], nu=scene["nu"], **rom_kwargs)
    z, vh = rom_initial_state(dec, scene, v0, z_guess=z_guess, device=device)
    if exact_ic:
        rom.set_fields(z.clone(), vh.clone(), np.asarray(v0, np.float64)[None])
    zp = z.clone()
    st = torch.zeros(1, dtype=torch.int32, device=device)
    xbuf = torch.zeros(1, d, P, device=device)
    rom.positions(z, 0.0, xbuf)
    out = [xbuf[0].clone()]
    done = 0
    times = []
    while done < n_steps:
        k = min(record_every, n_steps - done)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        rom.step(k, done, scene["dt"], z, zp, vh, status=st, use_graph=use_graph)
        b.record()
        rom.positions(z, (done + k) * scene["dt"], xbuf)
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b) / k)
        done += k
        out.append(xbuf[0].clone())
        if progress is not None:
            progress(done)
    nq, na = rom.last_counts(0)
    rom.close()
    return out, {"status": int(st.item()), "ms_per_step": float(np.mean(times[1:] if len(times) > 1 else times)),
                 "n_quadrature_points": nq, "n_active_nodes": na}


def rom_positions_batched(dec, scene, Es, v0s, n_steps, record_every, n_samples, opts,
                          z_guesses=None, seed=7, use_graph=True, device="cuda"):
    """Several parameter instances (Young's moduli Es, initial velocities
    v0s) advanced together by one batched runner (rom_step with B
    instances); returns, per instance, the positions of every particle at
    the recorded steps, and the mean step time of the batch."""
    P, d = scene["P"], scene["dim"]
    Bn = len(Es)
    X = torch.tensor(np.ascontiguousarray(scene["X"].T), device=device)
    grid = _grid(scene)
    rom = B.Rom(dec, grid, X, torch.tensor(np.asarray(Es, np.float32), device=device),
                torch.full((Bn,), n_samples, dtype=torch.int32, device=device), opts, seed=seed,
                rho0=float(scene["rho"]), m_uniform=float(scene["m"]), model=scene["model"],
                nu=scene["nu"])
    zs, vs = [], []
    for b in range(Bn):
        zg = None if z_guesses is None else z_guesses[b]
        z, vh = rom_initial_state(dec, scene, v0s[b], z_guess=zg, device=device)
        zs.append(z)
        vs.append(vh)
    z = torch.cat(zs).contiguous()
    vh = torch.cat(vs).contiguous()
    zp = z.clone()
    st = torch.zeros(Bn, dtype=torch.int32, device=device)
    xbuf = torch.zeros(Bn, d, P, device=device)
    B.rom_decode(dec, X, z, xbuf)
    out = [[xbuf[b].clone()] for b in range(Bn)]
    done = 0
    times = []
    while done < n_steps:
        k = min(record_every, n_steps - done)
        a = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        a.record()
        rom.step(k, done, scene["dt"], z, zp, vh, status=st, use_graph=use_graph)
        e.record()
        B.rom_decode(dec, X, z, xbuf)
        torch.cuda.synchronize()
        times.append(a.elapsed_time(e) / k)
        done += k
        for b in range(Bn):
            out[b].append(xbuf[b].clone())
    rom.close()
    return out, {"status": st.cpu().numpy().tolist(),
                 "ms_per_batched_step": float(np.mean(times[1:] if len(times) > 1 else times))}


def displacement_error(x_rom, x_fom, X):
    """(displacement-relative error, position error in percent) accumulated
    over the recorded steps and all particles."""
    num = den_d = den_p = 0.0
    Xt = torch.as_tensor(np.ascontiguousarray(X.T), device=x_fom[0].device).double()
    for a, b in zip(x_rom, x_fom):
        a = a.double()
        b = b.double()
        num += float(((a - b) ** 2).sum())
        den_d += float(((b - Xt) ** 2).sum())
        den_p += float((b ** 2).sum())
    return (num / den_d) ** 0.5, 100.0 * (num / den_p) ** 0.5
