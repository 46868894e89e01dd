"""Checkpoint and resume as .npz files (plain arrays, no pickled objects).

Full-order state: x, v, C, F (SoA float32, as the library holds them),
per-particle m and V0 or their uniform values, the step counter and the
reference label of every slot (mpm_step keeps the particles cell-sorted,
so slot i holds reference particle `label[i]`).

Reduced state: xhat_n, xhat_{n-1}, vhat_n (float64, one row per instance),
the step counter and the sampler seed.  The sampler is counter based: the
sample points of step k depend on the seed, the instance and k alone, so
the counter is all the random state there is, and rom_step resumes with
step0 = the saved counter.

Decoder: weights, biases, input box, output mean and scale, output mode
and precision, enough to rebuild the same decoder.

A resumed run starts from bit-identical inputs.  Whether it then continues
bit for bit depends on the run: the full-order model does with
MR_DETERMINISTIC when the resume point lies on the sort schedule (a
multiple of sort_every, since mpm_step sorts before its first step); runs
that sum with float atomics agree to rounding.
"""
import numpy as np
import torch

from . import binding as B

_FORMAT = 1


def _np(t):
    return t.detach().cpu().numpy()


def save_particles(path, parts, step, label=None):
    """Full-order particle state at `step`; label (int64, per slot) is the
    reference particle each slot holds (identity when None)."""
    P = parts.n
    arrays = {"format": np.int64(_FORMAT), "kind": np.array("particles"),
              "step": np.int64(step), "x": _np(parts.x), "v": _np(parts.v),
              "C": _np(parts.C), "F": _np(parts.F),
              "m_uniform": np.float32(parts.m_uniform), "V0_uniform": np.float32(parts.V0_uniform),
              "label": np.arange(P, dtype=np.int64) if label is None
              else np.asarray(label, dtype=np.int64)}
    if parts.m is not None:
        arrays["m"] = _np(parts.m)
    if parts.V0 is not None:
        arrays["V0"] = _np(parts.V0)
    np.savez(path, **arrays)


def _open(path, kind):
    z = np.load(path, allow_pickle=False)
    if int(z["format"]) != _FORMAT or str(z["kind"]) != kind:
        raise ValueError("%s is not a %s checkpoint of format %d" % (path, kind, _FORMAT))
    return z


def load_particles(path, device="cuda"):
    """Returns (Particles on `device`, step, label)."""
    z = _open(path, "particles")
    t = lambda a: torch.tensor(np.ascontiguousarray(a), device=device)
    parts = B.Particles(t(z["x"]), t(z["v"]), t(z["C"]), t(z["F"]),
                        t(z["m"]) if "m" in z.files else None,
                        t(z["V0"]) if "V0" in z.files else None,
                        m_uniform=float(z["m_uniform"]), V0_uniform=float(z["V0_uniform"]))
    return parts, int(z["step"]), z["label"].copy()


def save_latents(path, xhat, xhat_prev, vhat, step, seed):
    """Reduced state of B instances at `step` (latents float64 (B, r))."""
    np.savez(path, format=np.int64(_FORMAT), kind=np.array("latents"), step=np.int64(step),
             seed=np.uint64(seed), xhat=_np(xhat).astype(np.float64),
             xhat_prev=_np(xhat_prev).astype(np.float64), vhat=_np(vhat).astype(np.float64))


def load_latents(path, device="cuda"):
    """Returns a dict: xhat, xhat_prev, vhat (float64 tensors on `device`),
    step, seed."""
    z = _open(path, "latents")
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=device)
    return {"xhat": t(z["xhat"]), "xhat_prev": t(z["xhat_prev"]), "vhat": t(z["vhat"]),
            "step": int(z["step"]), "seed": int(z["seed"])}


def save_decoder(path, weights, biases, in_min, in_max, out_mean, out_std,
                 output_mode=B.OUT_DISPLACEMENT, precision=B.PREC_FP32):
    arrays = {"format": np.int64(_FORMAT), "kind": np.array("decoder"),
              "n_layers": np.int64(len(weights)), "output_mode": np.int64(output_mode),
              "precision": np.int64(precision),
              "in_min": np.asarray(in_min, np.float32), "in_max": np.asarray(in_max, np.float32),
              "out_mean": np.asarray(out_mean, np.float32),
              "out_std": np.asarray(out_std, np.float32)}
    for i, (W, b) in enumerate(zip(weights, biases)):
        arrays["W%d" % i] = np.asarray(W, np.float32)
        arrays["b%d" % i] = np.asarray(b, np.float32)
    np.savez(path, **arrays)


def load_decoder_arrays(path):
    """(weights, biases, in_min, in_max, out_mean, out_std, output_mode,
    precision) as saved."""
    z = _open(path, "decoder")
    n = int(z["n_layers"])
    return ([z["W%d" % i].copy() for i in range(n)], [z["b%d" % i].copy() for i in range(n)],
            z["in_min"].copy(), z["in_max"].copy(), z["out_mean"].copy(), z["out_std"].copy(),
            int(z["output_mode"]), int(z["precision"]))


def load_decoder(path):
    """The saved decoder as a library decoder (B.Decoder)."""
    Ws, bs, lo, hi, mean, std, mode, prec = load_decoder_arrays(path)
    return B.Decoder(Ws, bs, lo, hi, mean, std, mode, prec)
