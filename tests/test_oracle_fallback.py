"""The fallback from the reduced to the full-order model, forced from the
host on the oracle: a singular normal matrix (a latent direction the
decoder ignores), Gauss-Newton stopped above tolerance, and J <= 0 at the
quadrature points (a reflecting position-mode decoder).  Each must hand
over at the failing step with the full-order state reconstructed from the
last good latent state; where the full-order model can continue, its free
fall is checked against the symplectic-Euler closed form."""
import numpy as np

from oracle import decoder as D
from oracle import mpm
from oracle import project as PR
from oracle import rom

DIM, N, P = 3, 16, 150
DT = 1e-3
GRAV = np.array([0.0, -9.8, 0.0])


def _scene():
    mu, la = mpm.lame(1e4, 0.3)
    return dict(dim=DIM, n=[N] * DIM, dx=1.0 / N, bound=0, floor_mode=0, mu_f=0.0,
                gravity=list(GRAV), model=mpm_model(), mu=mu, la=la,
                m=np.full(P, 1e-3), V0=np.full(P, 1e-6))


def mpm_model():
    return 1  # Neo-Hookean


def _X():
    return np.random.default_rng(9).uniform(0.35, 0.65, size=(P, DIM))


def _free_fall(x0, v0, steps):
    """Symplectic Euler under gravity alone: v_k = v0 + k dt g, x_k = x0 + dt sum v_j."""
    v = v0 + steps * DT * GRAV
    x = x0 + DT * (steps * v0 + DT * GRAV * steps * (steps + 1) / 2)
    return x, v


def test_singular_normal_matrix_hands_over_with_the_latent_state():
    """r = 4 with the fourth latent ignored: J^T J is singular from the first
    step; the hand-over state is x = X + xhat[:3], v = vhat[:3], F = I."""
    W = np.concatenate([np.zeros((DIM, DIM)), np.eye(DIM), np.zeros((DIM, 1))], axis=1)
    dec = D.Decoder([W], [np.zeros(DIM)], np.zeros(DIM), np.ones(DIM), np.zeros(DIM),
                    np.ones(DIM))
    X = _X()
    z = np.array([0.01, -0.02, 0.0, 0.5])
    vh = np.array([0.3, 0.1, -0.2, 7.0])
    opts = PR.GNOptions(mode=PR.MODE_POS_VEL, max_iter=3)
    steps = 5
    state, k, bad, fom = rom.run_with_fallback(dec, _scene(), X, z, z, vh, DT, steps,
                                               lambda s: rom.sample_indices(3, 0, s, 8, P), opts)
    assert k == 0 and bad & PR.STATUS_SINGULAR and fom == 0
    x, v = _free_fall(X + z[:3], vh[:3], steps)
    np.testing.assert_allclose(state["v"], np.broadcast_to(v, (P, DIM)), atol=1e-12)
    np.testing.assert_allclose(state["x"], x, atol=1e-12)
    np.testing.assert_allclose(state["F"], np.broadcast_to(np.eye(DIM), (P, DIM, DIM)), atol=1e-12)


def test_gauss_newton_above_tolerance_hands_over():
    """One Gauss-Newton iteration with a strict step tolerance: the step is
    never seen to converge (MR_FLAG_NOCONV); two good steps pass first when
    the iteration cap allows it."""
    W = np.concatenate([np.zeros((DIM, DIM)), np.eye(DIM)], axis=1)
    dec = D.Decoder([W], [np.zeros(DIM)], np.zeros(DIM), np.ones(DIM), np.zeros(DIM),
                    np.ones(DIM))
    X = _X()
    z0 = np.zeros(DIM)
    v0 = np.array([0.2, -0.1, 0.05])
    steps = 4
    sample = lambda s: rom.sample_indices(5, 0, s, 6, P)
    strict = PR.GNOptions(mode=PR.MODE_POS_VEL, max_iter=1, tol_step=1e-30)
    state, k, bad, fom = rom.run_with_fallback(dec, _scene(), X, z0, z0, v0, DT, steps, sample,
                                               strict)
    assert k == 0 and bad & PR.STATUS_NOCONV and fom == 0
    x, v = _free_fall(X, v0, steps)
    np.testing.assert_allclose(state["x"], x, atol=1e-12)
    np.testing.assert_allclose(state["v"], np.broadcast_to(v, (P, DIM)), atol=1e-12)
    # without the failure the reduced run finishes and stands for the same
    # free fall (translation manifold)
    ok = PR.GNOptions(mode=PR.MODE_POS_VEL, max_iter=3, fixed_iters=True)
    state2, k2, bad2, _ = rom.run_with_fallback(dec, _scene(), X, z0, z0, v0, DT, steps, sample, ok)
    assert k2 is None and bad2 == 0
    np.testing.assert_allclose(state2["x"], x, atol=1e-12)


def test_inverted_map_hands_over_and_reports_the_full_order_failure():
    """Position-mode linear decoder with dg/dX = diag(-1, 1, 1) (a
    reflection): J = -1 at every quadrature point, so the reduced step fails
    at once; the reconstructed state is the reflected body, on which the
    full-order model fails as well (its stress is undefined too)."""
    X = _X()
    lo, hi = X.min(0), X.max(0)
    c = 0.5 * (lo + hi)
    half = 0.5 * (hi - lo)
    # y = W0 Xn with Xn = 2 (X - lo)/(hi - lo) - 1; g = c + half * y
    W = np.concatenate([np.diag([-1.0, 1.0, 1.0]), np.zeros((DIM, 2))], axis=1)
    dec = D.Decoder([W], [np.zeros(DIM)], lo, hi, c, half, D.OUT_POSITION)
    z = np.zeros(2)
    opts = PR.GNOptions(mode=PR.MODE_VEL_ONLY)
    state, k, bad, fom = rom.run_with_fallback(dec, _scene(), X, z, z, z, DT, 3,
                                               lambda s: rom.sample_indices(1, 0, s, 8, P), opts)
    assert k == 0 and bad == rom.STATUS_DOMAIN and fom == rom.STATUS_DOMAIN
    want = X.copy()
    want[:, 0] = 2 * c[0] - X[:, 0]
    np.testing.assert_allclose(state["x"], want, atol=1e-12)
    np.testing.assert_allclose(np.linalg.det(state["F"]), -1.0, atol=1e-12)
