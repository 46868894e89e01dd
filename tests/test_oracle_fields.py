"""Pins of the oracle's initial-condition correction fields (Section 3.1,
eqs. defMapApproxForm and essentialSpec) and of the mixed second derivative
they need: the derivative against central differences taken two ways
(along the latent direction of dg/dX, and along X of the latent tangent),
the fields against the initial conditions they exist to satisfy, and a
reduced run on a translation manifold started from arbitrary latents,
which the fields must turn into the ballistic trajectory of the true
initial state."""
import numpy as np
import pytest

from oracle import decoder as D
from oracle import project as PR
from oracle import rom
from tests.test_oracle_sampler_rom import _scene, translation_decoder


def _random_decoder(d, r, seed, width=12, layers=3):
    rng = np.random.default_rng(seed)
    sizes = [d + r] + [width] * layers + [d]
    Ws = [rng.standard_normal((o, i)) * (1.2 / np.sqrt(i)) for i, o in zip(sizes[:-1], sizes[1:])]
    bs = [0.3 * rng.standard_normal(o) for o in sizes[1:]]
    return D.Decoder(Ws, bs, np.zeros(d), np.ones(d), 0.01 * rng.standard_normal(d),
                     np.full(d, 0.05), D.OUT_DISPLACEMENT)


@pytest.mark.parametrize("d", [2, 3])
def test_mixed_derivative_is_the_latent_derivative_of_F(d):
    r = 4
    dec = _random_decoder(d, r, 10 + d)
    rng = np.random.default_rng(1)
    X = rng.uniform(0.1, 0.9, size=(7, d))
    z = 0.5 * rng.standard_normal(r)
    u = rng.standard_normal(r)
    M = D.mixed_jac(dec, X, z, u)
    h = 1e-5
    Fp = D.decode_jac(dec, X, z + h * u)[1]
    Fm = D.decode_jac(dec, X, z - h * u)[1]
    np.testing.assert_allclose(M, (Fp - Fm) / (2 * h), rtol=1e-6, atol=1e-10)


def test_mixed_derivative_is_the_spatial_derivative_of_the_latent_tangent():
    d, r = 3, 5
    dec = _random_decoder(d, r, 21)
    rng = np.random.default_rng(2)
    X = rng.uniform(0.1, 0.9, size=(5, d))
    z = 0.5 * rng.standard_normal(r)
    u = rng.standard_normal(r)
    M = D.mixed_jac(dec, X, z, u)
    h = 1e-5
    for i in range(d):
        e = np.zeros(d)
        e[i] = h
        vp = D.decode_jac(dec, X + e, z, u)[3]
        vm = D.decode_jac(dec, X - e, z, u)[3]
        np.testing.assert_allclose(M[:, :, i], (vp - vm) / (2 * h), rtol=1e-6, atol=1e-10)


def test_fields_make_the_initial_conditions_exact():
    d, r = 3, 4
    dec = _random_decoder(d, r, 31)
    rng = np.random.default_rng(3)
    X = rng.uniform(0.1, 0.9, size=(40, d))
    z0 = rng.standard_normal(r)
    v0h = rng.standard_normal(r)
    V0 = np.array([0.3, -1.2, 0.5])
    f = rom.initial_fields(dec, X, z0, v0h, V0)
    x, F, J, v = D.decode_jac(dec, X, z0, v0h)
    # position and deformation gradient at t = 0: X and I
    np.testing.assert_allclose(x + f["a"], X, atol=1e-14)
    np.testing.assert_allclose(F + f["Ga"], np.broadcast_to(np.eye(d), F.shape), atol=1e-14)
    # velocity at t = 0: the prescribed V0
    np.testing.assert_allclose(v + f["b"], np.broadcast_to(V0, v.shape), atol=1e-14)
    # velocity gradient at t = 0 along the latent path z0 + t v0h: grad V0 = 0
    h = 1e-5
    Fp = D.decode_jac(dec, X, z0 + h * v0h)[1]
    Fm = D.decode_jac(dec, X, z0 - h * v0h)[1]
    np.testing.assert_allclose((Fp - Fm) / (2 * h) + f["Gb"], 0.0, atol=1e-8)


@pytest.mark.parametrize("mode", [PR.MODE_POS_VEL, PR.MODE_VEL_ONLY])
def test_fields_turn_any_initial_latents_into_the_true_trajectory(mode):
    """Translation manifold g = X + xhat, free fall: started from arbitrary
    latents (x0, v0h) with the correction fields of the true initial state
    (positions X, velocity V0), the reduced positions g + a + b t follow
    the symplectic-Euler trajectory of X with V0 (without the fields they
    would follow X + x0 with v0h)."""
    dim, n, P = 3, 16, 200
    rng = np.random.default_rng(5)
    X = rng.uniform(0.35, 0.65, size=(P, dim))
    dec = translation_decoder(dim)
    sc = _scene(dim, n, P, model=1)
    g = np.array(sc["gravity"])
    V0 = np.array([0.2, -0.4, 0.1])
    z = 0.05 * rng.standard_normal(dim)
    vh = rng.standard_normal(dim)
    f = rom.initial_fields(dec, X, z, vh, V0)
    zp = z.copy()
    dt = 1e-3
    opts = PR.GNOptions(mode=mode, max_iter=3, fixed_iters=True)
    nst = 5
    for k in range(nst):
        samples = rom.sample_indices(7, 0, k, 4, P)
        zn, vn, info = rom.rom_step(dec, sc, X, sc["m"], sc["V0"], z, zp, vh, dt, samples, opts,
                                    fields=f, t=k * dt)
        zp, z, vh = z, zn, vn
    t = nst * dt
    x = D.decode(dec, X, z) + f["a"] + f["b"] * t
    v = D.decode_jac(dec, X, z, vh)[3] + f["b"]
    vexp = V0 + nst * dt * g
    xexp = X + nst * dt * V0 + dt * dt * g * nst * (nst + 1) / 2
    np.testing.assert_allclose(v, np.broadcast_to(vexp, v.shape), atol=1e-12)
    np.testing.assert_allclose(x, xexp, atol=1e-13)
