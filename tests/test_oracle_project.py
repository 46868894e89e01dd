"""Pins of the FP64 projection oracle: exact recovery in the consistent
case, agreement with the normal-equation route, one-step convergence for
linear decoders, monotone Armijo decrease, and the Appendix A identity
between one Gauss-Newton step and the velocity-only update."""
import numpy as np
import pytest

from oracle import decoder as D
from oracle import project as PR
from paper_2109_12390_amd import scenes


def tiny(d=3, r=4, width=8, nh=3, seed=0):
    Ws, bs = scenes.random_decoder(d, r, width, nh, seed, scale=1.2, bias_scale=0.2)
    return D.Decoder(Ws, bs, -np.ones(d), np.ones(d), np.zeros(d), np.full(d, 0.3))


def test_velocity_ls_recovers_consistent_velocity():
    dec = tiny()
    rng = np.random.default_rng(0)
    X = rng.uniform(-1, 1, size=(20, 3))
    z = rng.standard_normal(4) * 0.3
    _, _, J, _ = D.decode_jac(dec, X, z)
    vstar = rng.standard_normal(4)
    v_trial = np.einsum("pdr,r->pd", J, vstar)
    np.testing.assert_allclose(PR.velocity_ls(J, v_trial), vstar, rtol=1e-10)
    # inconsistent data: equals the normal-equation solution
    noisy = v_trial + 0.1 * rng.standard_normal(v_trial.shape)
    A = J.reshape(-1, 4)
    ne = np.linalg.solve(A.T @ A, A.T @ noisy.reshape(-1))
    np.testing.assert_allclose(PR.velocity_ls(J, noisy), ne, rtol=1e-9)


def test_gn_linear_decoder_converges_in_one_iteration():
    # a linear decoder has the same latent Jacobian at every point, so the
    # stacked system has rank <= d: take r < d
    d, r = 3, 2
    rng = np.random.default_rng(1)
    W = rng.standard_normal((d, d + r))
    dec = D.Decoder([W], [rng.standard_normal(d)], -np.ones(d), np.ones(d), np.zeros(d), np.ones(d))
    X = rng.uniform(-1, 1, size=(10, d))
    x_trial = X + rng.standard_normal((10, d))
    opts = PR.GNOptions(max_iter=1, fixed_iters=True)
    z, it, f, status = PR.gauss_newton(dec, X, x_trial, np.zeros(r), opts)
    # linear least squares in z: the lstsq solution of the stacked system
    Xn = 2 * (X + 1) / 2 - 1
    A = np.tile(W[:, d:], (10, 1))
    b = (x_trial - X - (Xn @ W[:, :d].T + dec.biases[0])).reshape(-1)
    zs = np.linalg.lstsq(A, b, rcond=None)[0]
    np.testing.assert_allclose(z, zs, rtol=1e-11)
    assert it == 1 and status == PR.STATUS_OK


def test_gn_recovers_latent_of_consistent_positions():
    dec = tiny(seed=3)
    rng = np.random.default_rng(2)
    X = rng.uniform(-1, 1, size=(40, 3))
    zstar = rng.standard_normal(4) * 0.4
    x_trial = D.decode(dec, X, zstar)
    z, it, f, status = PR.gauss_newton(dec, X, x_trial, zstar + 0.05 * rng.standard_normal(4),
                                       PR.GNOptions(max_iter=30))
    assert status == PR.STATUS_OK
    np.testing.assert_allclose(z, zstar, atol=1e-9)
    assert f < 1e-20


def test_gn_objective_non_increasing():
    dec = tiny(seed=4)
    rng = np.random.default_rng(3)
    X = rng.uniform(-1, 1, size=(30, 3))
    x_trial = D.decode(dec, X, rng.standard_normal(4)) + 0.05 * rng.standard_normal((30, 3))
    z = rng.standard_normal(4)
    f_prev = PR.objective(dec, X, x_trial, z)
    for _ in range(6):
        z, _, f, status = PR.gauss_newton(dec, X, x_trial, z, PR.GNOptions(max_iter=1, fixed_iters=True))
        assert f <= f_prev + 1e-15
        f_prev = f


def test_appendix_a_identity():
    """With x_p = g(X_p; zhat_n) and x_trial = x_p + dt v_trial, one undamped
    Gauss-Newton step from zhat_n is zhat_n + dt vhat of the velocity
    least-squares problem."""
    dec = tiny(seed=5)
    rng = np.random.default_rng(4)
    X = rng.uniform(-1, 1, size=(25, 3))
    zn = rng.standard_normal(4) * 0.3
    dt = 1e-3
    x_n = D.decode(dec, X, zn)
    v_trial = rng.standard_normal((25, 3))
    x_trial = x_n + dt * v_trial
    _, _, J, _ = D.decode_jac(dec, X, zn)
    vhat = PR.velocity_ls(J, v_trial)
    opts = PR.GNOptions(max_iter=1, fixed_iters=True)
    z1, _, _, status = PR.gauss_newton(dec, X, x_trial, zn, opts)
    assert status == PR.STATUS_OK
    np.testing.assert_allclose(z1, zn + dt * vhat, rtol=0, atol=1e-14)
    # and the projection driver in velocity-only mode gives the same point
    zv, vv, _, _, _ = PR.project(dec, X, x_trial, v_trial, zn, zn, dt,
                                 PR.GNOptions(mode=PR.MODE_VEL_ONLY))
    np.testing.assert_allclose(zv, z1, atol=1e-14)
    np.testing.assert_allclose(vv, vhat, atol=1e-14)


def test_rank_deficient_sample_set_is_reported():
    """Fewer than r/d sample points leave the normal matrix singular."""
    dec = tiny(r=4)
    X = np.zeros((1, 3))
    _, _, J, _ = D.decode_jac(dec, X, np.zeros(4))
    with pytest.raises(np.linalg.LinAlgError):
        PR.velocity_ls(J, np.ones((1, 3)))
    z, vh, it, f, status = PR.project(dec, X, np.ones((1, 3)), np.ones((1, 3)),
                                      np.zeros(4), np.zeros(4), 1e-3, PR.GNOptions())
    assert status & PR.STATUS_SINGULAR
