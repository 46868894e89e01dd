"""Pins of the Eulerian-quadrature oracle (Algorithm 4): point counts in
closed form, the point set against a pure-Python enumeration, the Newton
inversion against the exact inverse of an affine map and against an
independent root finder, masses and reference positions under a
translation, and the translation-manifold ROM with Eulerian quadrature
against the symplectic-Euler closed form."""
import itertools

import numpy as np
import pytest
from scipy import optimize

from oracle import decoder as D
from oracle import mpm
from oracle import project as PR
from oracle import rom


def translation_decoder(d):
    W = np.concatenate([np.zeros((d, d)), np.eye(d)], axis=1)
    return D.Decoder([W], [np.zeros(d)], np.zeros(d), np.ones(d), np.zeros(d), np.ones(d))


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("ell", [2, 4])
def test_one_interior_sample_point_count(dim, ell):
    """One sample: I is its 3^d stencil; a point touches I iff its base is
    within -2..2 of the sample's base per axis, and ell points per axis have
    a given base, so |points| = (5 ell)^d."""
    n = [16] * dim
    dx = 1 / 16
    xs = np.full((1, dim), 0.5 + 0.3 * dx)
    I = rom.active_nodes(dim, n, dx, xs)
    assert len(I) == 3 ** dim
    pts = rom.eulerian_points(dim, n, dx, ell, I)
    assert len(pts) == (5 * ell) ** dim
    # evenly spaced at dx / ell, volume (dx / ell)^d each
    frac = pts / (dx / ell) - 0.5
    np.testing.assert_allclose(frac, np.round(frac), atol=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_points_match_python_enumeration(dim):
    rng = np.random.default_rng(4)
    n = [8] * dim
    dx = 1 / 8
    ell = 2
    xs = rng.uniform(0.3, 0.7, size=(3, dim))
    I = rom.active_nodes(dim, n, dx, xs)
    pts = rom.eulerian_points(dim, n, dx, ell, I)
    # enumerate every lattice point in plain Python
    Iset = set()
    for x in xs:
        b = [int(np.floor(x[a] / dx - 0.5)) for a in range(dim)]
        for o in itertools.product(range(3), repeat=dim):
            Iset.add(tuple(b[a] + o[a] for a in range(dim)))
    want = []
    for m in itertools.product(range((n[0] - 1) * ell), repeat=dim):
        p = [(mi + 0.5) * dx / ell for mi in m]
        b = [int(np.floor(p[a] / dx - 0.5)) for a in range(dim)]
        if any(bi < 0 or bi + 2 > n[0] - 1 for bi in b):
            continue
        st = {tuple(b[a] + o[a] for a in range(dim)) for o in itertools.product(range(3), repeat=dim)}
        if st & Iset:
            want.append(p)
    got = sorted(map(tuple, np.round(pts, 12)))
    assert got == sorted(map(tuple, np.round(np.array(want), 12)))


def test_newton_inverts_an_affine_map_in_one_iteration():
    """W = [S | 0]: g(X) = X + S (2X - 1) + c, so X = (I + 2S)^{-1} (x + S 1 - c);
    after the displacement step, one Newton step is exact on an affine map;
    the displacement step alone is exact when the map is a translation."""
    rng = np.random.default_rng(5)
    d, r = 3, 2
    S = 0.1 * rng.standard_normal((d, d))
    c = 0.05 * rng.standard_normal(d)
    W = np.concatenate([S, np.zeros((d, r))], axis=1)
    dec = D.Decoder([W], [c], np.zeros(d), np.ones(d), np.zeros(d), np.ones(d))
    x = rng.uniform(0.2, 0.8, size=(40, d))
    z = rng.standard_normal(r)
    exact = np.linalg.solve(np.eye(d) + 2 * S, (x + S.sum(1) - c).T).T
    X1 = rom.invert_map(lambda X: D.decode_jac(dec, X, z)[:2], x, 1)
    np.testing.assert_allclose(X1, x - (D.decode(dec, x, z) - x), atol=1e-15)
    X2 = rom.invert_map(lambda X: D.decode_jac(dec, X, z)[:2], x, 2)
    np.testing.assert_allclose(X2, exact, atol=1e-13)
    X4 = rom.invert_map(lambda X: D.decode_jac(dec, X, z)[:2], x, 4)
    np.testing.assert_allclose(X4, exact, atol=1e-13)
    t = np.array([0.02, -0.01, 0.03])
    tdec = D.Decoder([np.zeros((d, d + r))], [t], np.zeros(d), np.ones(d), np.zeros(d),
                     np.ones(d))
    np.testing.assert_allclose(rom.invert_map(lambda X: D.decode_jac(tdec, X, z)[:2], x, 1),
                               x - t, atol=1e-15)


def test_newton_matches_an_independent_root_finder():
    rng = np.random.default_rng(6)
    d, r, w = 3, 2, 8
    Ws = [0.3 * rng.standard_normal((w, d + r)), 0.3 * rng.standard_normal((w, w)),
          0.3 * rng.standard_normal((d, w))]
    bs = [0.1 * rng.standard_normal(w), 0.1 * rng.standard_normal(w), 0.05 * rng.standard_normal(d)]
    dec = D.Decoder(Ws, bs, np.zeros(d), np.ones(d), np.zeros(d), 0.05 * np.ones(d))
    z = rng.standard_normal(r)
    x = rng.uniform(0.3, 0.7, size=(12, d))
    X = rom.invert_map(lambda Y: D.decode_jac(dec, Y, z)[:2], x, 12)
    for k in range(len(x)):
        sol = optimize.root(lambda Y: D.decode(dec, Y[None], z)[0] - x[k], x[k], tol=1e-14)
        assert sol.success
        np.testing.assert_allclose(X[k], sol.x, atol=1e-11)
    np.testing.assert_allclose(D.decode(dec, X, z), x, atol=1e-12)


def _lattice_nodes(shape, h):
    """Node positions of a lattice in flat order, x fastest."""
    idx = np.indices(tuple(shape[::-1])).reshape(len(shape), -1)[::-1].T
    return idx * h


def _box_particles(dim, n, lo, hi, ppc=2):
    """Particles at (c + (j + 1/2) / ppc) dx in every cell of [lo, hi)^d."""
    dx = 1 / n
    c0, c1 = int(round(lo * n)), int(round(hi * n))
    ax = (np.arange(c0 * ppc, c1 * ppc) + 0.5) * dx / ppc
    g = np.meshgrid(*([ax] * dim), indexing="ij")
    return np.stack([a.reshape(-1) for a in g], axis=1)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("ppc", [1, 2])
def test_reference_density_partition_of_unity_and_mass(dim, ppc):
    """Particles on a regular lattice of spacing dx / ppc with m = rho0
    (dx / ppc)^d: rho_ref = rho0 at every node whose whole stencil
    neighbourhood is inside the sampled box (the quadratic B-spline's
    integer shifts sum to 1, so its shifts by 1/ppc sum to ppc per axis), 0
    two spacings outside, and the lattice holds the particles' total mass."""
    n, rho0 = 16, 1000.0
    dx = 1 / n
    X_all = _box_particles(dim, n, 0.25, 0.75, ppc=ppc)
    X_all = X_all[X_all[:, 0] < 0.625]          # asymmetric: the box is [0.25, 0.625) in x
    m = rho0 * (dx / ppc) ** dim
    rho = rom.reference_density(dim, [n] * dim, dx, X_all, m)
    shape = rom.density_lattice_shape([n] * dim)
    nodes = _lattice_nodes(shape, dx)
    hi = np.array([0.625, 0.75, 0.75][:dim])
    inner = np.all((nodes >= 0.25 + 1.5 * dx) & (nodes <= hi - 1.5 * dx), axis=1)
    outer = np.any((nodes <= 0.25 - 2 * dx) | (nodes >= hi + 2 * dx), axis=1)
    np.testing.assert_allclose(rho[inner], rho0, rtol=1e-12)
    assert np.all(rho[outer] == 0.0)
    np.testing.assert_allclose(rho.sum() * dx ** dim, m * len(X_all), rtol=1e-12)
    # multilinear reading: exact at nodes, rho0 between inner nodes
    np.testing.assert_allclose(rom.density_at(rho, dim, [n] * dim, dx, nodes[inner]),
                               rho0, rtol=1e-12)


def test_density_reading_is_exact_for_linear_fields():
    dim, n = 3, 8
    dx = 1 / n
    shape = rom.density_lattice_shape([n] * dim)
    nodes = _lattice_nodes(shape, dx)
    coef = np.array([1.0, -2.0, 0.5])
    rho = 3.0 + nodes @ coef
    X = np.random.default_rng(8).uniform(0.1, 0.8, size=(50, dim))
    np.testing.assert_allclose(rom.density_at(rho, dim, [n] * dim, dx, X), 3.0 + X @ coef,
                               rtol=1e-12)


def test_body_weight_ramp():
    """tau(s): 0 up to s = 1/4, 1 from s = 3/4, linear in between, 1/2 at the
    half level."""
    s = np.array([0.0, 0.25, 0.375, 0.5, 0.625, 0.75, 0.9, 1.7])
    np.testing.assert_allclose(rom.body_weight(s), [0, 0, 0.25, 0.5, 0.75, 1, 1, 1], atol=1e-15)


@pytest.mark.parametrize("dim", [2, 3])
def test_translation_positions_and_masses(dim):
    """g = X + t: X^Q = x^Q - t exactly, J = 1; the mass is rho0 (dx / ell)^d
    well inside the box and zero (point dropped) well outside it."""
    n, ell, rho0 = 16, 2, 1000.0
    dx = 1 / n
    h = dx / ell
    X_all = _box_particles(dim, n, 0.25, 0.75)
    rho = rom.reference_density(dim, [n] * dim, dx, X_all, rho0 * h ** dim)
    t = np.array([2 * dx, -1 * dx, dx][:dim])
    dec = translation_decoder(dim)
    xs = np.array([[0.7, 0.45, 0.5][:dim], [0.3, 0.6, 0.4][:dim]])
    eq = rom.eulerian_quadrature(dec, dim, [n] * dim, dx, xs, t, np.zeros(dim), ell, 3,
                                 1e-3 * dx, rho0, rho)
    Xc = eq["x_candidates"] - t
    np.testing.assert_allclose(eq["X_all"], Xc, atol=1e-15)
    np.testing.assert_allclose(np.linalg.det(eq["FQ"]), 1.0, atol=1e-15)
    inner = np.all((Xc >= 0.25 + 2 * h) & (Xc <= 0.75 - 2 * h), axis=1)
    outer = np.any((Xc <= 0.25 - 2 * dx) | (Xc >= 0.75 + 2 * dx), axis=1)
    assert inner.any() and outer.any()
    assert np.all(eq["keep"][inner]) and not np.any(eq["keep"][outer])
    kept_inner = inner[eq["keep"]]
    np.testing.assert_allclose(eq["mQ"][kept_inner], rho0 * h ** dim, rtol=1e-15)


def _jittered_cube(n, cells, lo, seed, sub=2):
    """A cube of cells^3 grid cells with sub^3 particles per cell, each
    uniform in its sub-cell (the benchmark scenes' sampling)."""
    dx = 1 / n
    rng = np.random.default_rng(seed)
    idx = np.indices((cells * sub,) * 3).reshape(3, -1).T.astype(np.float64)
    return np.asarray(lo) + (idx + rng.random(idx.shape)) * (dx / sub)


@pytest.mark.parametrize("kind", ["translation", "stretch"])
def test_jittered_body_interior_masses_are_rho0_V_over_J(kind):
    """Algorithm 4's mass m^Q = rho0 V^Q / J on a jittered body: every
    lattice point whose reference position lies at least 1.5 dx inside the
    cube carries exactly rho0 V^Q / J (the particles' scatter in the
    smoothed density does not enter), points 2 dx outside are dropped, and
    the kept mass equals the cube's mass up to its rounded edges and
    corners.  Maps: a translation g = X + t (J = 1) and a uniform stretch
    g = c + (1 + e)(X - c) (J = (1 + e)^3)."""
    n, ell, rho0, cells = 32, 2, 1000.0, 8
    dx = 1 / n
    lo = np.array([0.5 - 4 * dx, 0.3, 0.5 - 4 * dx])
    X_all = _jittered_cube(n, cells, lo, seed=11)
    mp = rho0 * (dx / 2) ** 3
    rho = rom.reference_density(3, [n] * 3, dx, X_all, mp)
    d, r = 3, 3
    if kind == "translation":
        t = np.array([0.6, -1.3, 0.2]) * dx
        W = np.concatenate([np.zeros((d, d)), np.eye(d)], axis=1)
        dec = D.Decoder([W], [np.zeros(d)], np.zeros(d), np.ones(d), np.zeros(d), np.ones(d))
        z, J, inv = t, 1.0, (lambda x: x - t)
    else:
        # normalised input 2X - 1 (in_min 0, in_max 1): g = X + (e/2)(2X - 1) + b
        e = 0.04
        c = lo + 4 * dx
        W = np.concatenate([0.5 * e * np.eye(d), np.zeros((d, r))], axis=1)
        b = 0.5 * e * np.ones(d) - e * c
        dec = D.Decoder([W], [b], np.zeros(d), np.ones(d), np.zeros(d), np.ones(d))
        z, J, inv = np.zeros(r), (1 + e) ** 3, (lambda x: c + (x - c) / (1 + e))
    xs = D.decode(dec, X_all, z)
    eq = rom.eulerian_quadrature(dec, 3, [n] * 3, dx, xs, z, np.zeros(r), ell, 3, 1e-3 * dx,
                                 rho0, rho)
    Xc = inv(eq["x_candidates"])
    np.testing.assert_allclose(eq["X_all"], Xc, atol=1e-13)
    inner = np.all((Xc >= lo + 1.5 * dx) & (Xc <= lo + cells * dx - 1.5 * dx), axis=1)
    outer = np.any((Xc <= lo - 2 * dx) | (Xc >= lo + cells * dx + 2 * dx), axis=1)
    assert inner.sum() > 500 and outer.any()
    Vq = (dx / ell) ** 3
    assert np.all(eq["keep"][inner]) and not np.any(eq["keep"][outer])
    kept_inner = inner[eq["keep"]]
    np.testing.assert_allclose(eq["mQ"][kept_inner], rho0 * Vq / J, rtol=1e-12)
    # the smoothed density itself scatters well away from rho0 here, and
    # only the weight is cut off by it
    s_in = eq["rho"][inner] / rho0
    assert s_in.min() >= 0.75 and s_in.std() > 0.01
    # total kept mass (in the reference measure: m J = tau rho0 V^Q) within
    # the rounding of the cube's 12 edges and 8 corners
    body = rho0 * (cells * dx) ** 3
    kept = float(np.sum(eq["mQ"] * np.linalg.det(eq["FQ"])))
    assert abs(kept - body) / body < 0.1, kept / body


@pytest.mark.parametrize("mode", [PR.MODE_POS_VEL, PR.MODE_VEL_ONLY])
@pytest.mark.parametrize("dim", [2, 3])
def test_translation_manifold_eulerian_rom_equals_symplectic_euler(mode, dim):
    """Free fall of a filled box under g = X + xhat: every quadrature point
    has F = I and the instance velocity, every node near the samples has
    mass, so the ROM with Eulerian quadrature reproduces symplectic Euler."""
    n = 32
    dx = 1 / n
    X_all = _box_particles(dim, n, 0.25, 0.75)
    P = len(X_all)
    rho = rom.reference_density(dim, [n] * dim, dx, X_all, 1000.0 * (dx / 2) ** dim)
    dec = translation_decoder(dim)
    mu, la = mpm.lame(1e4, 0.3)
    grav = [0.0] * dim
    grav[1] = -9.8
    sc = dict(dim=dim, n=[n] * dim, dx=dx, bound=0, floor_mode=0, mu_f=0.0, gravity=grav,
              model=1, mu=mu, la=la)
    interior = np.nonzero(np.all((X_all > 0.25 + 4 * dx) & (X_all < 0.75 - 4 * dx), axis=1))[0]
    rng = np.random.default_rng(7)
    z = np.zeros(dim)
    zp = z.copy()
    vh = np.array([0.3, -0.2, 0.1][:dim])
    z0, v0 = z.copy(), vh.copy()
    dt = 1e-3
    opts = PR.GNOptions(mode=mode, max_iter=3, fixed_iters=True)
    nst = 4
    for k in range(nst):
        samples = np.sort(rng.choice(interior, size=3, replace=False))
        zn, vn, info = rom.rom_step(dec, sc, X_all, None, None, z, zp, vh, dt, samples, opts,
                                    quadrature="eulerian", ell=2, newton_iters=2, rho0=1000.0,
                                    rho_ref=rho)
        assert info["eulerian"]["keep"].all()
        zp, z, vh = z, zn, vn
    g = np.array(grav)
    np.testing.assert_allclose(vh, v0 + nst * dt * g, atol=1e-12)
    np.testing.assert_allclose(z, z0 + nst * dt * v0 + dt * dt * g * nst * (nst + 1) / 2,
                               atol=1e-13)
