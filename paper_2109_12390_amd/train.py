"""Decoder training driver (paper Section 4.2 loss, Appendix B training
details) on the library's training kernels.

`DecoderTrainFn` and `TrainLossFn` are torch.autograd.Functions whose
forward and backward passes are the C-ABI kernels rom_train_forward /
rom_train_backward and rom_train_loss; the Adam update is rom_adam_step and
batch assembly rom_train_gather.  PyTorch only allocates memory and chains
the two Functions.  Snapshots come from the library's own full-order model
(mpm_step).
"""
import ctypes
import math

import numpy as np
import torch

from . import binding as B


class Trainer:
    """Owns an mr_trainer handle (rom_trainer_create / rom_trainer_destroy)."""

    def __init__(self, d, r, width, n_hidden, precision, max_rows, in_min, in_max, out_mean,
                 out_std, output_mode=B.OUT_DISPLACEMENT):
        lib = B.load()
        self.d, self.r, self.width, self.n_hidden = d, r, width, n_hidden
        f = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.float32))
        self._norm = [f(in_min), f(in_max), f(out_mean), f(out_std)]
        h = ctypes.c_void_p()
        B._check("rom_trainer_create", lib.rom_trainer_create(
            d, r, width, n_hidden, precision, max_rows,
            *[ctypes.c_void_p(a.ctypes.data) for a in self._norm], output_mode, ctypes.byref(h)))
        self.handle = h
        self.n_params = int(lib.rom_train_param_count(d, r, width, n_hidden))

    def close(self):
        if self.handle:
            B.load().rom_trainer_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DecoderTrainFn(torch.autograd.Function):
    """(params, Z) -> (g, G, Gv) for a batch of n_groups x rows_per_group rows."""

    @staticmethod
    def forward(ctx, params, Z, X, snap, nxt, trainer, n_groups, rows_per_group, dt):
        d = trainer.d
        rows = n_groups * rows_per_group
        dev = params.device
        g = torch.empty(rows, d, device=dev)
        G = torch.empty(rows, d, d, device=dev)
        Gv = torch.empty(rows, d, device=dev)
        lib = B.load()
        B._check("rom_train_forward", lib.rom_train_forward(
            trainer.handle, B._ptr(params, torch.float32), B._ptr(Z, torch.float32),
            B._ptr(X, torch.float32), B._ptr(snap, torch.int32), B._ptr(nxt, torch.int32),
            n_groups, rows_per_group, dt, B._ptr(g), B._ptr(G), B._ptr(Gv), B._stream(None)))
        ctx.trainer = trainer
        ctx.keep = (params, Z, X, snap, nxt)
        return g, G, Gv

    @staticmethod
    def backward(ctx, dg, dG, dGv):
        params, Z, _, _, _ = ctx.keep
        dparams = torch.zeros_like(params)
        dZ = torch.zeros_like(Z)
        B._check("rom_train_backward", B.load().rom_train_backward(
            ctx.trainer.handle, B._ptr(dg.contiguous()), B._ptr(dG.contiguous()),
            B._ptr(dGv.contiguous()), B._ptr(dparams), B._ptr(dZ), B._stream(None)))
        return dparams, dZ, None, None, None, None, None, None, None


class TrainLossFn(torch.autograd.Function):
    """Training objective (batch mean of the three penalised residuals)."""

    @staticmethod
    def forward(ctx, g, G, Gv, x_t, F_t, v_t, nxt, n_groups, rows_per_group, lam_F, lam_v):
        d = g.shape[1]
        loss = torch.zeros(1, device=g.device)
        dg, dG, dGv = torch.empty_like(g), torch.empty_like(G), torch.empty_like(Gv)
        B._check("rom_train_loss", B.load().rom_train_loss(
            d, n_groups, rows_per_group, B._ptr(nxt, torch.int32), B._ptr(g), B._ptr(G),
            B._ptr(Gv), B._ptr(x_t), B._ptr(F_t), B._ptr(v_t), lam_F, lam_v, B._ptr(loss),
            B._ptr(dg), B._ptr(dG), B._ptr(dGv), B._stream(None)))
        ctx.grads = (dg, dG, dGv)
        return loss[0]

    @staticmethod
    def backward(ctx, dloss):
        dg, dG, dGv = ctx.grads
        return dg * dloss, dG * dloss, dGv * dloss, None, None, None, None, None, None, None, None


class EncoderFn(torch.autograd.Function):
    """(encoder params) -> z [n][r] for the frames frame_idx of x [frames][in_len]
    (rom_encoder_forward / rom_encoder_backward)."""

    @staticmethod
    def forward(ctx, params, x, frame_idx, r, d, in_min, in_max, deterministic=False):
        n = frame_idx.numel()
        _, _, _, actf, workf = B.encoder_layout(x.shape[1], r)
        act = torch.empty(n, actf, device=x.device)
        z = torch.empty(n, r, device=x.device)
        B.encoder_forward(d, r, x, params, in_min, in_max, act, z, frame_idx=frame_idx)
        ctx.keep = (params, x, frame_idx, act, r, d, in_min, in_max, workf, deterministic)
        return z

    @staticmethod
    def backward(ctx, dz):
        params, x, frame_idx, act, r, d, in_min, in_max, workf, det = ctx.keep
        g = torch.empty_like(params)
        work = torch.empty(frame_idx.numel(), workf, device=x.device)
        B.encoder_backward(d, r, x, params, in_min, in_max, act, dz.contiguous(), g, work,
                           frame_idx=frame_idx, deterministic=det)
        return g, None, None, None, None, None, None, None


def encoder_init(in_len, r, seed):
    """Glorot-uniform encoder parameters (Appendix B), zero biases, in the
    library's layout (rom_encoder_layout)."""
    nc, dc, npar, _, _ = B.encoder_layout(in_len, r)
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(nc):
        a = math.sqrt(6.0 / 12.0)               # 6 taps in, 6 out
        out.extend(rng.uniform(-a, a, 6).tolist() + [0.0])
    a = math.sqrt(6.0 / (dc + 32))
    out.extend(rng.uniform(-a, a, 32 * dc).tolist() + [0.0] * 32)
    a = math.sqrt(6.0 / (32 + r))
    out.extend(rng.uniform(-a, a, r * 32).tolist() + [0.0] * r)
    assert len(out) == npar
    return np.asarray(out, dtype=np.float32)


def encode(params, frames, r, d, in_min, in_max, chunk=128):
    """Codes of frames [n][in_len] (device) under encoder params (device)."""
    n = frames.shape[0]
    out = torch.empty(n, r, device=frames.device)
    with torch.no_grad():
        for c0 in range(0, n, chunk):
            idx = torch.arange(c0, min(n, c0 + chunk), dtype=torch.int32, device=frames.device)
            out[c0:c0 + idx.numel()] = EncoderFn.apply(params, frames, idx, r, d, in_min, in_max)
    return out


def adam_step(param, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    B._check("rom_adam_step", B.load().rom_adam_step(
        param.numel(), B._ptr(param), B._ptr(grad), B._ptr(m), B._ptr(v), lr, beta1, beta2, eps,
        step, B._stream(None)))


class SnapshotSet:
    """Frames of (x, F, v) of a fixed particle subset, on the device:
    x [n_frames][P_sub][d], F [n_frames][P_sub][d][d], v [n_frames][P_sub][d];
    X_sub [P_sub][d]; next_frame[f] = f + 1 inside a simulation, -1 at its end."""

    def __init__(self, X_sub, fx, fF, fv, next_frame, dt_frame, sub=None):
        self.X_sub, self.fx, self.fF, self.fv = X_sub, fx, fF, fv
        self.next_frame = next_frame
        self.dt_frame = dt_frame
        self.sub = sub          # indices of the subset in the scene's particles

    @property
    def n_frames(self):
        return self.fx.shape[0]

    @property
    def P_sub(self):
        return self.X_sub.shape[0]


def generate_snapshots(scene, instances, n_steps, every, n_sub, seed, sort_every=10,
                       affine=True, device="cuda"):
    """Runs the full-order model (mpm_step) for every (E, v0) instance from
    the scene's initial state and records frames every `every` steps
    (including the initial state) for a fixed random subset of n_sub
    particles.  affine=False drops the APIC affine term (PIC transfers)."""
    d = scene["dim"]
    P = scene["P"]
    rng = np.random.default_rng(seed)
    sub = np.sort(rng.choice(P, size=n_sub, replace=False))
    sub_t = torch.tensor(sub, device=device, dtype=torch.long)
    grid = B.Grid(d, scene["n"], scene["dx"], scene["bound"], scene["floor_mode"], scene["mu_f"],
                  scene["gravity"])
    gbuf = torch.zeros(grid.nodes() * 4, device=device)
    ws = torch.zeros(B.mpm_step_workspace_bytes(grid, P), dtype=torch.uint8, device=device)
    perm = torch.zeros(P, dtype=torch.int32, device=device)
    flag = torch.zeros(1, dtype=torch.int32, device=device)
    frames_x, frames_F, frames_v, nxt = [], [], [], []
    soa = lambda a: torch.tensor(np.ascontiguousarray(a.reshape(P, -1).T), device=device)
    n_frames_per = n_steps // every + 1
    for (E, v0) in instances:
        X = scene["X"]
        v = np.tile(np.asarray(v0, dtype=np.float32), (P, 1))
        parts = B.Particles(soa(X), soa(v), torch.zeros(d * d, P, device=device),
                            soa(np.tile(np.eye(d, dtype=np.float32), (P, 1, 1))),
                            m_uniform=float(scene["m"]), V0_uniform=float(scene["V0"]))
        slot_of = torch.arange(P, device=device)        # slot of each original particle
        for f in range(n_frames_per):
            if f > 0:
                B.mpm_step(grid, (scene["model"], float(E), scene["nu"]), parts, scene["dt"], every,
                           sort_every, 0 if affine else B.NO_AFFINE, gbuf, ws, perm_accum=perm,
                           status=flag)
                # slot -> entry index of this call; compose with the running map
                inv = torch.empty_like(perm, dtype=torch.long)
                inv[perm.long()] = torch.arange(P, device=device)
                slot_of = inv[slot_of]
            s = slot_of[sub_t]
            frames_x.append(parts.x[:, s].T.contiguous())
            frames_F.append(parts.F[:, s].T.contiguous().reshape(n_sub, d, d))
            frames_v.append(parts.v[:, s].T.contiguous())
            nxt.append(1 if f < n_frames_per - 1 else 0)
    rc, fl = B.sync_status(flag)
    if rc != 0:
        raise RuntimeError("full-order model raised status flags %s" % fl)
    fx = torch.stack(frames_x)
    fF = torch.stack(frames_F)
    fv = torch.stack(frames_v)
    n_frames = fx.shape[0]
    next_frame = np.array([i + 1 if nxt[i] else -1 for i in range(n_frames)], dtype=np.int32)
    X_sub = torch.tensor(scene["X"][sub], device=device)
    return SnapshotSet(X_sub, fx, fF, fv, next_frame, every * scene["dt"], sub=sub)


def balanced_penalties(snap):
    """Penalty weights that put the three terms of the objective on the
    scale of the position term for this data: lam_F = E|u|^2 / E|F - I|^2 and
    lam_v = E|u|^2 / E|v|^2 over the snapshot rows (u the displacement).
    The paper's lam_F = 100, lam_v = 0.01 are tied to its scenes' units."""
    d = snap.X_sub.shape[1]
    u2 = float(((snap.fx - snap.X_sub[None]) ** 2).sum(-1).mean())
    f2 = float(((snap.fF - torch.eye(d, device=snap.fF.device)) ** 2).sum((-1, -2)).mean())
    v2 = float((snap.fv ** 2).sum(-1).mean())
    return (u2 / f2 if f2 > 0 else 1.0), (u2 / v2 if v2 > 0 else 1.0)


def normalisation(snap):
    """Min-max input range of the reference positions and mean / standard
    deviation of the displacements (Appendix B feature scaling)."""
    d = snap.X_sub.shape[1]
    X = snap.X_sub.cpu().numpy().astype(np.float64)
    # over every row of every frame, in float64 on the device (the frames
    # can hold hundreds of millions of rows)
    u = (snap.fx - snap.X_sub[None]).reshape(-1, d).double()
    mean = u.mean(0)
    std = torch.sqrt(((u - mean) ** 2).mean(0)).cpu().numpy()
    std = np.where(std > 0, std, 1.0)
    return X.min(0), X.max(0), mean.cpu().numpy(), std


def train(snap, width, n_hidden, r, steps, n_groups, rows_per_group, precision=B.PREC_BF16,
          lr0=1e-3, lr1=1e-6, lam_F=100.0, lam_v=0.01, seed=0, log_every=0, init=None,
          eval_rows_per_frame=64, encoder=False, encoder_lr_scale=1.0, deterministic=False,
          device="cuda"):
    """Trains decoder weights and the snapshots' latent codes with Adam, the
    learning rate decaying exponentially from lr0 to lr1.  The codes are
    free per-snapshot variables, or with encoder=True the encoder network of
    Section 4.1 applied to each snapshot's concatenated positions, trained
    with the decoder (each step encodes the batch's snapshots and their
    successors).  Returns (weights, biases, Z, normalisation, loss history)
    and, with encoder=True, the encoder parameters as a sixth item (Z then
    holds every snapshot's code under the trained encoder); with
    log_every > 0 the history holds (step, objective) on a fixed evaluation
    batch of eval_rows_per_frame random particles of every frame, before
    step 0, every log_every steps and after the last step.  The encoder's
    learning rate is encoder_lr_scale times the decoder's.  deterministic:
    every gradient reduction in a fixed order (bitwise reproducible runs)."""
    from . import scenes
    d = snap.X_sub.shape[1]
    in_min, in_max, mean, std = normalisation(snap)
    rows = n_groups * rows_per_group
    eval_rows = snap.n_frames * eval_rows_per_frame if log_every else 0
    tr = Trainer(d, r, width, n_hidden, precision, max(rows, eval_rows), in_min, in_max, mean,
                 std)
    if deterministic:
        B._check("rom_trainer_set_deterministic",
                 B.load().rom_trainer_set_deterministic(tr.handle, 1))
    if init is None:
        Ws, bs = scenes.xavier_decoder(d, r, width, n_hidden, seed)
    else:
        Ws, bs = init
    params = torch.tensor(B.pack_params(Ws, bs), device=device)
    Z = torch.zeros(snap.n_frames, r, device=device)
    m_p, v_p = torch.zeros_like(params), torch.zeros_like(params)
    m_z, v_z = torch.zeros_like(Z), torch.zeros_like(Z)
    if encoder:
        frames = snap.fx.reshape(snap.n_frames, -1)
        pe = torch.tensor(encoder_init(frames.shape[1], r, seed + 3), device=device)
        m_e, v_e = torch.zeros_like(pe), torch.zeros_like(pe)
        enc_args = (r, d, in_min.astype(np.float32), in_max.astype(np.float32))

        def codes(frame_ids):
            """Z with the rows frame_ids encoded (differentiable), others 0."""
            z = EncoderFn.apply(pe_var, frames, frame_ids, *enc_args, deterministic)
            return torch.zeros(snap.n_frames, r, device=device).index_copy(0, frame_ids.long(), z)
    nf = torch.tensor(snap.next_frame, device=device)
    rng = np.random.default_rng(seed + 1)
    X = torch.empty(rows, d, device=device)
    xt = torch.empty(rows, d, device=device)
    Ft = torch.empty(rows, d, d, device=device)
    vt = torch.empty(rows, d, device=device)
    lib = B.load()
    history = []
    if log_every:
        erng = np.random.default_rng(seed + 2)
        e_fr = torch.arange(snap.n_frames, dtype=torch.int32, device=device)
        e_pid = torch.tensor(erng.integers(0, snap.P_sub, size=eval_rows).astype(np.int32),
                             device=device)
        e_nxt = nf[e_fr.long()].contiguous()
        eX = torch.empty(eval_rows, d, device=device)
        ext = torch.empty(eval_rows, d, device=device)
        eFt = torch.empty(eval_rows, d, d, device=device)
        evt = torch.empty(eval_rows, d, device=device)
        B._check("rom_train_gather", lib.rom_train_gather(
            d, snap.n_frames, eval_rows_per_frame, snap.P_sub, B._ptr(snap.X_sub), B._ptr(snap.fx),
            B._ptr(snap.fF), B._ptr(snap.fv), B._ptr(e_fr, torch.int32), B._ptr(e_pid, torch.int32),
            B._ptr(eX), B._ptr(ext), B._ptr(eFt), B._ptr(evt), B._stream(None)))

        def evaluate():
            with torch.no_grad():
                if encoder:
                    Z.copy_(encode(pe, frames, *enc_args))
                g, G, Gv = DecoderTrainFn.apply(params, Z, eX, e_fr, e_nxt, tr, snap.n_frames,
                                                eval_rows_per_frame, float(snap.dt_frame))
                return float(TrainLossFn.apply(g, G, Gv, ext, eFt, evt, e_nxt, snap.n_frames,
                                               eval_rows_per_frame, lam_F, lam_v).item())
        history.append((0, evaluate()))
    for it in range(steps):
        lr = lr0 * (lr1 / lr0) ** (it / max(steps - 1, 1))
        fr = rng.integers(0, snap.n_frames, size=n_groups).astype(np.int32)
        pid = rng.integers(0, snap.P_sub, size=rows).astype(np.int32)
        fr_t = torch.tensor(fr, device=device)
        pid_t = torch.tensor(pid, device=device)
        nxt_t = nf[fr_t.long()].contiguous()
        B._check("rom_train_gather", lib.rom_train_gather(
            d, n_groups, rows_per_group, snap.P_sub, B._ptr(snap.X_sub), B._ptr(snap.fx),
            B._ptr(snap.fF), B._ptr(snap.fv), B._ptr(fr_t, torch.int32), B._ptr(pid_t, torch.int32),
            B._ptr(X), B._ptr(xt), B._ptr(Ft), B._ptr(vt), B._stream(None)))
        p = params.detach().requires_grad_(True)
        if encoder:
            pe_var = pe.detach().requires_grad_(True)
            need = torch.unique(torch.cat([fr_t, nxt_t[nxt_t >= 0]])).to(torch.int32)
            z = codes(need)
        else:
            z = Z.detach().requires_grad_(True)
        g, G, Gv = DecoderTrainFn.apply(p, z, X, fr_t, nxt_t, tr, n_groups, rows_per_group,
                                        float(snap.dt_frame))
        loss = TrainLossFn.apply(g, G, Gv, xt, Ft, vt, nxt_t, n_groups, rows_per_group, lam_F, lam_v)
        loss.backward()
        adam_step(params, p.grad.contiguous(), m_p, v_p, it + 1, lr)
        if encoder:
            adam_step(pe, pe_var.grad.contiguous(), m_e, v_e, it + 1, lr * encoder_lr_scale)
        else:
            adam_step(Z, z.grad.contiguous(), m_z, v_z, it + 1, lr)
        if log_every and ((it + 1) % log_every == 0 or it == steps - 1):
            history.append((it + 1, evaluate()))
    sizes = [d + r] + [width] * n_hidden + [d]
    flat = params.cpu().numpy()
    Ws, bs, o = [], [], 0
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        Ws.append(flat[o:o + fi * fo].reshape(fo, fi)); o += fi * fo
        bs.append(flat[o:o + fo]); o += fo
    tr.close()
    if encoder:
        Z = encode(pe, frames, *enc_args)
        return Ws, bs, Z.cpu().numpy(), (in_min, in_max, mean, std), history, pe.cpu().numpy()
    return Ws, bs, Z.cpu().numpy(), (in_min, in_max, mean, std), history


def train_linear(snap, r, steps, rows=16384, lr0=1e-2, lr1=1e-4, lam_F=100.0, lam_v=0.01,
                 seed=0, device="cuda"):
    """The linear-manifold baseline (a single linear layer g = X + mean +
    std * (W [X~; z] + b), no activation, the comparison of the paper's
    Section 5): its weights, bias and per-snapshot latent codes trained on
    the same objective as the network (batch mean of the position, lam_F
    deformation-gradient and lam_v velocity residuals) with Adam and the same
    exponentially decaying learning rate.  Training runs as PyTorch
    operations: this one-layer map is a baseline for comparison, outside the
    reduced-order path (which evaluates it with the library's kernels).
    Returns (weights, biases, Z, normalisation) like `train`."""
    d = snap.X_sub.shape[1]
    in_min, in_max, mean, std = normalisation(snap)
    f32 = lambda a: torch.tensor(np.asarray(a, dtype=np.float32), device=device)
    lo, hi, mu, sd = f32(in_min), f32(in_max), f32(mean), f32(std)
    gen = torch.Generator(device="cpu").manual_seed(seed)
    a = math.sqrt(6.0 / (d + r + d))
    W = ((torch.rand(d, d + r, generator=gen) * 2 - 1) * a).to(device).requires_grad_(True)
    b = torch.zeros(d, device=device, requires_grad=True)
    Z = torch.zeros(snap.n_frames, r, device=device, requires_grad=True)
    opt = torch.optim.Adam([W, b, Z], lr=lr0)
    nxt = torch.tensor(snap.next_frame, device=device, dtype=torch.long)
    scale_X = 2.0 / (hi - lo)
    eye = torch.eye(d, device=device)
    for it in range(steps):
        for gr in opt.param_groups:
            gr["lr"] = lr0 * (lr1 / lr0) ** (it / max(steps - 1, 1))
        fr = torch.randint(0, snap.n_frames, (rows,), generator=gen).to(device)
        pi = torch.randint(0, snap.P_sub, (rows,), generator=gen).to(device)
        X = snap.X_sub[pi]
        Xn = (X - lo) * scale_X - 1.0
        g = X + mu + sd * (torch.cat([Xn, Z[fr]], 1) @ W.T + b)
        Fg = eye + sd[:, None] * W[:, :d] * scale_X[None, :]
        loss_x = ((g - snap.fx[fr, pi]) ** 2).sum(-1)
        loss_F = ((Fg[None] - snap.fF[fr, pi]) ** 2).sum((-1, -2))
        has = nxt[fr] >= 0
        dz = (Z[nxt[fr].clamp(min=0)] - Z[fr]) / snap.dt_frame
        gv = (sd[None, :] * (dz @ W[:, d:].T))
        loss_v = torch.where(has, ((gv - snap.fv[fr, pi]) ** 2).sum(-1), torch.zeros_like(loss_x))
        loss = (loss_x + lam_F * loss_F + lam_v * loss_v).mean()
        opt.zero_grad()
        loss.backward()
        opt.step()
    Ws = [W.detach().cpu().numpy().astype(np.float32)]
    bs = [b.detach().cpu().numpy().astype(np.float32)]
    return Ws, bs, Z.detach().cpu().numpy(), (in_min, in_max, mean, std)
