"""Pins of the sampler and reduced-order step oracles: sampler invariants,
neighbour sets against brute force, the translation-manifold ROM against
the symplectic-Euler closed form, the Algorithm 5 / Algorithm 1 limit, the
least-squares initial latents and the error metrics."""
import os

import numpy as np
import pytest

from oracle import decoder as D
from oracle import mpm
from oracle import project as PR
from oracle import rom
from oracle import sampler


def _golden_splitmix64():
    path = os.path.join(os.path.dirname(__file__), "golden", "splitmix64.txt")
    rows = []
    for line in open(path):
        line = line.strip()
        if line and not line.startswith("#"):
            vals = [int(t) for t in line.split()]
            rows.append((vals[0], vals[1:]))
    return rows


def test_mix_reproduces_published_splitmix64_outputs():
    """SplitMix64 run as a generator (state advanced by the golden gamma
    before each output) must give the published sequences; mix(c) is the
    output for state c, i.e. the k-th output from seed s is
    mix(s + (k - 1) gamma)."""
    rows = _golden_splitmix64()
    assert len(rows) == 2
    for seed, outs in rows:
        state = seed
        for want in outs:
            assert sampler.mix(state) == want
            state = (state + sampler.GOLDEN) & sampler.MASK


def test_mix_is_injective_on_a_range_and_well_spread():
    outs = [sampler.mix(c) for c in range(20000)]
    assert len(set(outs)) == len(outs)
    bits = np.array([[(o >> b) & 1 for b in range(64)] for o in outs[:4000]])
    assert np.all(np.abs(bits.mean(0) - 0.5) < 0.04)


@pytest.mark.parametrize("S,P", [(1, 10), (7, 100), (512, 2097152), (100, 100), (64, 65)])
def test_stratified_samples_invariants(S, P):
    s = sampler.stratified_samples(11, 3, 42, S, P)
    assert len(s) == S
    for k, idx in enumerate(s):
        lo, hi = (k * P) // S, ((k + 1) * P) // S
        assert lo <= idx < hi
    assert len(set(s)) == S and s == sorted(s)
    if S == P:
        assert s == list(range(P))


def test_sampler_is_deterministic_and_redraws_per_step():
    a = sampler.stratified_samples(1, 0, 5, 64, 10000)
    assert a == sampler.stratified_samples(1, 0, 5, 64, 10000)
    assert a != sampler.stratified_samples(1, 0, 6, 64, 10000)
    assert a != sampler.stratified_samples(1, 1, 5, 64, 10000)
    assert a != sampler.stratified_samples(2, 0, 5, 64, 10000)


def test_sampler_is_uniform_within_strata():
    counts = np.zeros(10)
    for step in range(4000):
        idx = sampler.stratified_samples(9, 0, step, 1, 10)[0]
        counts[idx] += 1
    chi2 = np.sum((counts - 400.0) ** 2 / 400.0)
    assert chi2 < 30.0    # 9 dof, p ~ 4e-4


def test_sampler_rejects_bad_sizes():
    with pytest.raises(ValueError):
        sampler.stratified_samples(0, 0, 0, 11, 10)
    with pytest.raises(ValueError):
        sampler.stratified_samples(0, 0, 0, 0, 10)


@pytest.mark.parametrize("dim", [2, 3])
def test_neighbour_set_matches_bruteforce(dim):
    rng = np.random.default_rng(0)
    n = [12] * dim
    x = rng.uniform(0.3, 0.7, size=(150, dim))
    samples = np.sort(rng.choice(150, size=5, replace=False))
    I, Q, N = rom.neighbour_set(dim, n, 1 / 12, x, samples)
    Ib, Qb, Nb = rom.neighbour_set_bruteforce(dim, n, 1 / 12, x, samples)
    np.testing.assert_array_equal(I, Ib)
    np.testing.assert_array_equal(Q, Qb)
    np.testing.assert_array_equal(N, Nb)
    assert len(I) <= 5 * 3 ** dim
    assert set(samples) <= set(Q) and not (set(samples) & set(N))


def translation_decoder(d):
    W = np.concatenate([np.zeros((d, d)), np.eye(d)], axis=1)
    return D.Decoder([W], [np.zeros(d)], np.zeros(d), np.ones(d), np.zeros(d), np.ones(d))


def _scene(dim, n, P, model=1, E=1e4, gravity=None):
    mu, la = mpm.lame(E, 0.3)
    g = [0.0] * dim
    g[1] = -9.8
    return dict(dim=dim, n=[n] * dim, dx=1.0 / n, bound=0, floor_mode=0, mu_f=0.0,
                gravity=g if gravity is None else gravity, model=model, mu=mu, la=la,
                m=np.full(P, 1e-3), V0=np.full(P, 1e-6))


@pytest.mark.parametrize("mode", [PR.MODE_POS_VEL, PR.MODE_VEL_ONLY])
@pytest.mark.parametrize("dim", [2, 3])
def test_translation_manifold_rom_equals_symplectic_euler(mode, dim):
    """g = X + xhat (r = d), free fall, no walls: F = I, tau = 0 everywhere,
    so the ROM reproduces v_{n+1} = v_n + dt g, x_{n+1} = x_n + dt v_{n+1}
    for any sample set."""
    rng = np.random.default_rng(1)
    n = 16
    P = 200
    X = rng.uniform(0.35, 0.65, size=(P, dim))
    dec = translation_decoder(dim)
    sc = _scene(dim, n, P, model=1)
    g = np.array(sc["gravity"])
    z = np.zeros(dim); zp = z.copy(); vh = rng.standard_normal(dim) * 0.2
    z0, v0 = z.copy(), vh.copy()
    dt = 1e-3
    opts = PR.GNOptions(mode=mode, max_iter=3, fixed_iters=True)
    for k in range(5):
        samples = rom.sample_indices(7, 0, k, 4, P)
        zn, vn, info = rom.rom_step(dec, sc, X, sc["m"], sc["V0"], z, zp, vh, dt, samples, opts)
        zp, z, vh = z, zn, vn
    nst = 5
    np.testing.assert_allclose(vh, v0 + nst * dt * g, atol=1e-12)
    np.testing.assert_allclose(z, z0 + nst * dt * v0 + dt * dt * g * nst * (nst + 1) / 2, atol=1e-13)


def test_substep_with_all_points_is_one_pic_step():
    """With every particle a sample (no neighbours), the quadrature
    kinematics equal to the particle state and C = 0, Algorithm 5 gives the
    position and velocity of one step of Algorithm 1 with the plain
    transfer."""
    rng = np.random.default_rng(2)
    dim, n, P = 3, 16, 120
    x = rng.uniform(0.35, 0.65, size=(P, dim))
    v = rng.standard_normal((P, dim)) * 0.1
    F = np.eye(dim) + 0.02 * rng.standard_normal((P, dim, dim))
    sc = _scene(dim, n, P)
    sc["bound"] = 3
    sc["floor_mode"] = 1
    sc["mu_f"] = 0.3
    xt, vt = rom.substep(sc, x, F, v, sc["m"], sc["V0"], x, 1e-4)
    full = mpm.step(sc, {"x": x, "v": v, "C": np.zeros((P, dim, dim)), "F": F}, 1e-4, apic=False)
    np.testing.assert_allclose(vt, full["v"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(xt, full["x"], rtol=0, atol=1e-15)


def test_rom_init_translation_manifold():
    rng = np.random.default_rng(3)
    X = rng.uniform(0.2, 0.8, size=(100, 3))
    V = np.tile([0.5, -1.0, 0.25], (100, 1))
    z, vh, status = rom.rom_init(translation_decoder(3), X, V, PR.GNOptions(max_iter=5))
    np.testing.assert_allclose(z, 0.0, atol=1e-15)
    np.testing.assert_allclose(vh, [0.5, -1.0, 0.25], atol=1e-15)
    assert status == PR.STATUS_OK


def test_error_metrics():
    rng = np.random.default_rng(4)
    X = rng.uniform(size=(50, 3))
    x = X + 0.01 * rng.standard_normal((50, 3))
    acc = rom.ErrorAccumulator()
    acc.add(x, x, X)
    assert acc.displacement_relative() == 0.0 and acc.position_percent() == 0.0
    a1, a2 = rom.ErrorAccumulator(), rom.ErrorAccumulator()
    xr = x + 1e-4 * rng.standard_normal((50, 3))
    a1.add(xr, x, X)
    a2.add(3 * xr, 3 * x, 3 * X)
    assert a1.displacement_relative() == pytest.approx(a2.displacement_relative(), rel=1e-12)
    assert a1.position_percent() == pytest.approx(a2.position_percent(), rel=1e-12)
