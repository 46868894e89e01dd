"""The reduced run with the full-order model as its fallback, on the GPU.

A singular normal matrix (a latent the decoder ignores) and Gauss-Newton
stopped above its tolerance are forced from the host through the decoder and
the projection options.  The hand-over state (x, F, v decoded from the last
good latents) and the full-order steps after it are compared with the
oracle's driver on the same inputs, and on the translation manifold with the
symplectic-Euler free-fall closed form.  A run with no failure must finish
in the reduced model, chunked or not, with the same result.

Tolerances: positions to 1e-5 relative L2 (the fp32 bar of one full-order
step; here a handful of steps of a body at rest in its own frame); F and v
to 1e-4 of their scale (fp32 decoder output, as in the decoder parity
tests)."""
import numpy as np
import pytest

from oracle import decoder as OD
from oracle import project as OP
from oracle import rom as OR
from paper_2109_12390_amd import binding as B
from paper_2109_12390_amd import fallback as FB
from paper_2109_12390_amd import scenes
from tests.helpers import aos, oracle_scene, rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
dev = "cuda"


def _scene():
    """4,096 Neo-Hookean particles (8^3 cells, 8 per cell) in the middle of a
    32^3 grid with no wall band: a few steps stay far from every boundary."""
    return scenes.make_scene(3, 32, (8, 8, 8), (0.375, 0.375, 0.375), 2, 1000.0, 5.0e4, 0.3,
                             scenes.MODEL_NEO_HOOKEAN, (0.0, -9.8, 0.0), scenes.FLOOR_STICKY, 0.0,
                             0, 5.0e-5, 11)


def _lat(a):
    return torch.tensor(np.asarray(a, np.float64)[None, :], device=dev)


def _translation_decoder(s, r_extra=0):
    """g = X + xhat[:3]; r_extra further latents the decoder ignores."""
    d = 3
    W = np.concatenate([np.zeros((d, d)), np.eye(d), np.zeros((d, r_extra))], axis=1)
    X = s["X"]
    return B.Decoder([W.astype(np.float32)], [np.zeros(d, np.float32)], X.min(0), X.max(0),
                     np.zeros(d, np.float32), np.ones(d, np.float32))


def _free_fall(s, x0, v0, k):
    dt, g = s["dt"], np.array(s["gravity"])
    return x0 + dt * (k * v0 + dt * g * k * (k + 1) / 2), v0 + k * dt * g


def _check_free_fall(s, out, x0, v0, k):
    x, v = _free_fall(s, x0, v0, k)
    ex = rel_l2(aos(out["x"].cpu().numpy(), 3), x)
    ev = np.max(np.abs(aos(out["v"].cpu().numpy(), 3) - v)) / np.max(np.abs(v))
    eF = np.max(np.abs(aos(out["F"].cpu().numpy(), 3, mat=True) - np.eye(3)))
    print("free fall after %d steps: rel L2 x %.2e, v %.2e, |F - I| %.2e" % (k, ex, ev, eF))
    assert ex < 1e-5 and ev < 1e-4 and eF < 1e-4


def test_singular_normal_matrix_hands_over_to_free_fall(gpu):
    s = _scene()
    dec = _translation_decoder(s, r_extra=1)
    z = _lat([0.01, -0.02, 0.0, 0.5])
    vh = _lat([0.3, 0.1, -0.2, 7.0])
    steps = 6
    out = FB.run_with_fallback(dec, s, s["E"], z, z.clone(), vh, steps, 16,
                               B.gn_opts(mode=B.POS_VEL, max_iter=3), chunk=4)
    print("fallback step", out["fallback_step"], "status", out["status"], "fom", out["fom_status"])
    assert out["fallback_step"] == 0 and out["status"] & B.FLAG_SINGULAR
    assert out["fom_status"] == 0
    _check_free_fall(s, out, s["X"].astype(np.float64) + [0.01, -0.02, 0.0],
                     np.array([0.3, 0.1, -0.2]), steps)


def test_gauss_newton_above_tolerance_hands_over(gpu):
    s = _scene()
    dec = _translation_decoder(s)
    z = _lat([0.0, 0.0, 0.0])
    v0 = np.array([0.2, -0.1, 0.05])
    steps = 5
    out = FB.run_with_fallback(dec, s, s["E"], z, z.clone(), _lat(v0), steps, 16,
                               B.gn_opts(mode=B.POS_VEL, max_iter=1, tol_step=1e-30), chunk=1)
    assert out["fallback_step"] == 0 and out["status"] & B.FLAG_NOCONV
    assert out["fom_status"] == 0
    _check_free_fall(s, out, s["X"].astype(np.float64), v0, steps)


@pytest.mark.parametrize("chunk,use_graph", [(3, True), (7, False)])
def test_run_without_failure_stays_reduced(gpu, chunk, use_graph):
    """7 steps in chunks of 3 (a ragged last chunk) or at once: no hand-over,
    and the decoded final state is the free fall."""
    s = _scene()
    dec = _translation_decoder(s)
    z = _lat([0.0, 0.0, 0.0])
    v0 = np.array([0.2, -0.1, 0.05])
    steps = 7
    vh = _lat(v0)
    out = FB.run_with_fallback(dec, s, s["E"], z, z.clone(), vh, steps, 16,
                               B.gn_opts(mode=B.POS_VEL, max_iter=2), chunk=chunk,
                               use_graph=use_graph)
    assert out["fallback_step"] is None and out["status"] == 0
    _check_free_fall(s, out, s["X"].astype(np.float64), v0, steps)


def test_hand_over_matches_oracle_driver(gpu):
    """Random 3-hidden-layer decoder whose last latent is inert: both drivers
    fail at the first step, rebuild x, F, v from the latents (a deformed
    body with a non-uniform velocity) and run the full-order model (no
    affine term) for the remaining steps."""
    s = _scene()
    d, r = 3, 6
    Ws, bs = scenes.random_decoder(d, r, 32, 3, 61, scale=1.0, bias_scale=0.1)
    Ws[0][:, d + r - 1] = 0.0
    X = s["X"]
    lo, hi = X.min(0).astype(np.float32), X.max(0).astype(np.float32)
    mean = np.zeros(d, np.float32)
    std = np.full(d, 0.01, np.float32)
    odec = OD.Decoder(Ws, bs, lo, hi, mean, std, OD.OUT_DISPLACEMENT)
    gdec = B.Decoder(Ws, bs, lo, hi, mean, std)
    rng = np.random.default_rng(3)
    z0 = 0.3 * rng.standard_normal(r)
    v0 = 2.0 * rng.standard_normal(r)
    steps = 4
    out = FB.run_with_fallback(gdec, s, s["E"], _lat(z0), _lat(z0), _lat(v0), steps, 24,
                               B.gn_opts(mode=B.POS_VEL, max_iter=3))
    sc = oracle_scene(s)
    Xd = X.astype(np.float64)
    state, k, bad, fom = OR.run_with_fallback(
        odec, sc, Xd, z0, z0, v0, s["dt"], steps, lambda i: OR.sample_indices(7, 0, i, 24, s["P"]),
        OP.GNOptions(mode=OP.MODE_POS_VEL, max_iter=3))
    assert k == 0 and bad & OP.STATUS_SINGULAR and fom == 0
    assert out["fallback_step"] == 0 and out["status"] & B.FLAG_SINGULAR and out["fom_status"] == 0
    x = aos(out["x"].cpu().numpy(), 3)
    v = aos(out["v"].cpu().numpy(), 3)
    F = aos(out["F"].cpu().numpy(), 3, mat=True)
    ex = rel_l2(x - Xd, state["x"] - Xd)
    ex_abs = rel_l2(x, state["x"])
    ev = np.max(np.abs(v - state["v"])) / np.max(np.abs(state["v"]))
    eF = np.max(np.abs(F - state["F"])) / np.max(np.abs(state["F"] - np.eye(3)))
    print("hand-over parity: rel L2 x %.2e (of the displacement %.2e), v %.2e, F %.2e"
          % (ex_abs, ex, ev, eF))
    assert ex_abs < 1e-5 and ev < 1e-4 and eF < 1e-4
