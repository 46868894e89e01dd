"""Pins of the training-objective oracle: finite differences of the loss in
weights, biases and latent codes; zero loss and zero gradient at the
generating network; the dropped velocity term of a simulation's last
snapshot; and the closed-form first Adam step."""
import numpy as np
import pytest

from oracle import decoder as D
from oracle import train as TR
from paper_2109_12390_amd import scenes


def tiny(seed=0, d=3, r=3, width=5, nh=2):
    Ws, bs = scenes.random_decoder(d, r, width, nh, seed, scale=1.3, bias_scale=0.3)
    return D.Decoder([w.astype(np.float64) for w in Ws], [b.astype(np.float64) for b in bs],
                     -np.ones(d), np.ones(d), np.full(d, 0.1), np.full(d, 0.5))


def batch(rng, d=3, r=3, N=6, n_snap=4):
    X = rng.uniform(-1, 1, size=(N, d))
    snap = rng.integers(0, n_snap, size=N)
    nxt = np.where(snap < n_snap - 1, snap + 1, -1)
    Z = 0.3 * rng.standard_normal((n_snap, r))
    x_t = X + 0.1 * rng.standard_normal((N, d))
    F_t = np.eye(d) + 0.1 * rng.standard_normal((N, d, d))
    v_t = rng.standard_normal((N, d))
    return Z, X, snap, nxt, x_t, F_t, v_t


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(0)
    dec = tiny()
    Z, X, snap, nxt, x_t, F_t, v_t = batch(rng)
    args = (X, snap, nxt, x_t, F_t, v_t, 0.05, 10.0, 0.5)
    L, gW, gb, gZ = TR.loss_and_grads(dec, Z, *args)
    h = 1e-6
    for l in range(len(dec.weights)):
        for (i, j) in [(0, 0), (1, 2), (dec.weights[l].shape[0] - 1, dec.weights[l].shape[1] - 1)]:
            dp = [w.copy() for w in dec.weights]
            dm = [w.copy() for w in dec.weights]
            dp[l][i, j] += h
            dm[l][i, j] -= h
            Lp = TR.loss_value(D.Decoder(dp, dec.biases, dec.in_min, dec.in_max, dec.out_mean, dec.out_std), Z, *args)
            Lm = TR.loss_value(D.Decoder(dm, dec.biases, dec.in_min, dec.in_max, dec.out_mean, dec.out_std), Z, *args)
            assert gW[l][i, j] == pytest.approx((Lp - Lm) / (2 * h), rel=1e-6, abs=1e-8)
        bp = [b.copy() for b in dec.biases]
        bm = [b.copy() for b in dec.biases]
        bp[l][0] += h
        bm[l][0] -= h
        Lp = TR.loss_value(D.Decoder(dec.weights, bp, dec.in_min, dec.in_max, dec.out_mean, dec.out_std), Z, *args)
        Lm = TR.loss_value(D.Decoder(dec.weights, bm, dec.in_min, dec.in_max, dec.out_mean, dec.out_std), Z, *args)
        assert gb[l][0] == pytest.approx((Lp - Lm) / (2 * h), rel=1e-6, abs=1e-8)
    for (s, k) in [(0, 0), (1, 2), (3, 1)]:
        Zp, Zm = Z.copy(), Z.copy()
        Zp[s, k] += h
        Zm[s, k] -= h
        fd = (TR.loss_value(dec, Zp, *args) - TR.loss_value(dec, Zm, *args)) / (2 * h)
        assert gZ[s, k] == pytest.approx(fd, rel=1e-6, abs=1e-8)


def test_zero_loss_and_gradient_at_the_generating_network():
    rng = np.random.default_rng(1)
    dec = tiny(seed=3)
    Z, X, snap, nxt, _, _, _ = batch(rng)
    dt = 0.05
    x_t, F_t, J, _ = D.decode_jac(dec, X[:1], Z[snap[0]])
    xs, Fs, vs = [], [], []
    for i in range(len(X)):
        xi, Fi, Ji, _ = D.decode_jac(dec, X[i:i + 1], Z[snap[i]])
        u = (Z[nxt[i]] - Z[snap[i]]) / dt if nxt[i] >= 0 else np.zeros(Z.shape[1])
        xs.append(xi[0]); Fs.append(Fi[0]); vs.append(Ji[0] @ u)
    L, gW, gb, gZ = TR.loss_and_grads(dec, Z, X, snap, nxt, np.array(xs), np.array(Fs), np.array(vs),
                                      dt, 100.0, 0.01)
    assert L < 1e-25
    for g in gW + gb + [gZ]:
        assert np.max(np.abs(g)) < 1e-10


def test_last_snapshot_velocity_term_is_dropped():
    rng = np.random.default_rng(2)
    dec = tiny()
    Z, X, snap, nxt, x_t, F_t, v_t = batch(rng, N=8)
    snap[0], nxt[0] = 3, -1
    L1 = TR.loss_value(dec, Z, X, snap, nxt, x_t, F_t, v_t, 0.05, 10.0, 1.0)
    v2 = v_t.copy()
    v2[0] += 100.0
    L2 = TR.loss_value(dec, Z, X, snap, nxt, x_t, F_t, v2, 0.05, 10.0, 1.0)
    assert L1 == pytest.approx(L2, rel=1e-14)
    v2[1] += 1.0
    if nxt[1] >= 0:
        assert TR.loss_value(dec, Z, X, snap, nxt, x_t, F_t, v2, 0.05, 10.0, 1.0) != pytest.approx(L1)


def test_adam_first_step_closed_form():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    new, m, v = TR.adam_update(p, g, np.zeros(3), np.zeros(3), 1, 1e-3)
    # after one step mhat = g, vhat = g^2: the update is lr g / (|g| + eps)
    np.testing.assert_allclose(new, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
