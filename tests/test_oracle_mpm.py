"""Pins of the FP64 MPM oracle against what the method fixes: B-spline
closed forms and invariants, conservation in the transfers, exact APIC
reproduction of affine fields, the ballistic closed form, stress closed
forms and energy derivatives, and hand-computed boundary cases."""
import numpy as np
import pytest

from oracle import mpm


def textbook_bspline(xi):
    """Quadratic B-spline N(xi) of a node at signed distance xi (in cells)."""
    a = abs(xi)
    if a < 0.5:
        return 0.75 - a * a
    if a < 1.5:
        return 0.5 * (1.5 - a) ** 2
    return 0.0


@pytest.mark.parametrize("f", [0.5, 0.51, 0.75, 1.0, 1.2345, 1.4999])
def test_bspline_matches_textbook_and_moments(f):
    w, dw = mpm.bspline_1d(f)
    for k in range(3):
        assert w[k] == pytest.approx(textbook_bspline(k - f), abs=1e-15)
    rel = np.arange(3) - f          # (x_i - x_p)/dx
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert (w * rel).sum() == pytest.approx(0.0, abs=1e-15)
    assert (w * rel * rel).sum() == pytest.approx(0.25, abs=1e-15)   # dx^2/4
    assert dw.sum() == pytest.approx(0.0, abs=1e-15)
    assert (dw * np.arange(3)).sum() == pytest.approx(1.0, abs=1e-15)  # sum x_i grad w = I
    h = 1e-6
    for k in range(3):
        fd = (textbook_bspline(k - (f + h)) - textbook_bspline(k - (f - h))) / (2 * h)
        # central differences straddle the C1 junctions at |xi| = 0.5: O(h) error
        assert dw[k] == pytest.approx(fd, abs=2e-6)


def test_bspline_node_and_midpoint_values():
    w, _ = mpm.bspline_1d(1.0)
    np.testing.assert_allclose(w, [1 / 8, 3 / 4, 1 / 8], atol=0)
    w, _ = mpm.bspline_1d(0.5)
    np.testing.assert_allclose(w, [1 / 2, 1 / 2, 0.0], atol=0)


def _random_particles(rng, dim, n, P, lo=0.3, hi=0.7):
    x = rng.uniform(lo, hi, size=(P, dim))
    v = rng.standard_normal((P, dim))
    C = rng.standard_normal((P, dim, dim))
    F = np.eye(dim) + 0.05 * rng.standard_normal((P, dim, dim))
    m = rng.uniform(0.5, 2.0, size=P)
    V0 = rng.uniform(0.5, 2.0, size=P) * 1e-3
    return x, v, C, F, m, V0


@pytest.mark.parametrize("dim", [2, 3])
def test_single_particle_grid_mass_is_tensor_product(dim):
    rng = np.random.default_rng(0)
    n = [16] * dim
    dx = 1.0 / 16
    xp = rng.uniform(0.3, 0.7, size=(1, dim))
    gm, _, _ = mpm.p2g(dim, n, dx, xp, np.zeros((1, dim)), np.zeros((1, dim, dim)),
                       np.eye(dim)[None], np.ones(1), np.ones(1), 1, 1.0, 1.0)
    grid = gm.reshape(n[::-1])  # index [k][j][i] (or [j][i])
    base = np.floor(xp[0] / dx - 0.5).astype(int)
    for node in np.argwhere(grid > 0):
        ijk = node[::-1]
        expect = np.prod([textbook_bspline(ijk[a] - xp[0][a] / dx) for a in range(dim)])
        assert grid[tuple(node)] == pytest.approx(expect, abs=1e-15)
    assert np.count_nonzero(grid) <= 3 ** dim
    assert np.all(np.argwhere(grid > 0)[:, ::-1] >= base)


@pytest.mark.parametrize("dim,model", [(2, 0), (3, 1)])
def test_p2g_conserves_mass_momentum_and_force_balance(dim, model):
    rng = np.random.default_rng(1)
    n = [32] * dim
    x, v, C, F, m, V0 = _random_particles(rng, dim, n, 500)
    gm, gmv, gf = mpm.p2g(dim, n, 1 / 32, x, v, C, F, m, V0, model, 3.0, 5.0, apic=True)
    assert gm.sum() == pytest.approx(m.sum(), rel=1e-14)
    np.testing.assert_allclose(gmv.sum(0), (m[:, None] * v).sum(0), rtol=0, atol=1e-12)
    # internal forces are a discrete divergence: they sum to zero
    scale = np.abs(gf).sum()
    np.testing.assert_allclose(gf.sum(0), 0.0, atol=1e-13 * scale)


def test_p2g_exact_mass_with_representable_inputs():
    """Binary-fraction positions and masses: every weight product is exact,
    so the lumped mass sums to the particle mass exactly."""
    x = np.array([[0.5, 0.5], [0.40625, 0.59375], [0.53125, 0.4375]])
    m = np.array([1.0, 0.5, 0.25])
    gm, _, _ = mpm.p2g(2, [16, 16], 1 / 16, x, np.zeros((3, 2)), np.zeros((3, 2, 2)),
                       np.tile(np.eye(2), (3, 1, 1)), m, m, 1, 1.0, 1.0)
    assert gm.sum() == m.sum()


def _free_scene(dim, n, m, V0, model=1, mu=0.0, la=0.0, gravity=None):
    return dict(dim=dim, n=[n] * dim, dx=1.0 / n, bound=0, floor_mode=0, mu_f=0.0,
                gravity=gravity if gravity is not None else [0.0] * dim,
                model=model, mu=mu, la=la, m=m, V0=V0)


@pytest.mark.parametrize("dim", [2, 3])
def test_apic_reproduces_affine_velocity_exactly(dim):
    rng = np.random.default_rng(2)
    P = 400
    x = rng.uniform(0.3, 0.7, size=(P, dim))
    a = rng.standard_normal(dim)
    A = rng.standard_normal((dim, dim))
    v = a + x @ A.T
    C = np.tile(A, (P, 1, 1))
    F = np.tile(np.eye(dim), (P, 1, 1))
    m = rng.uniform(0.5, 2.0, size=P)
    sc = _free_scene(dim, 32, m, m * 1e-3, mu=10.0, la=10.0)
    out = mpm.step(sc, {"x": x, "v": v, "C": C, "F": F}, dt=1e-4)
    # velocities and affine matrices are reproduced at the old positions
    np.testing.assert_allclose(out["v"], v, rtol=0, atol=1e-12)
    np.testing.assert_allclose(out["C"], C, rtol=0, atol=1e-11)
    np.testing.assert_allclose(out["x"], x + 1e-4 * v, rtol=0, atol=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_rigid_translation_is_exact(dim):
    rng = np.random.default_rng(3)
    P = 300
    x0 = rng.uniform(0.4, 0.6, size=(P, dim))
    vel = rng.standard_normal(dim) * 0.5
    st = {"x": x0, "v": np.tile(vel, (P, 1)), "C": np.zeros((P, dim, dim)),
          "F": np.tile(np.eye(dim), (P, 1, 1))}
    sc = _free_scene(dim, 32, np.ones(P), np.full(P, 1e-3), mu=100.0, la=100.0)
    dt = 1e-3
    for _ in range(10):
        st = mpm.step(sc, st, dt)
    np.testing.assert_allclose(st["x"], x0 + 10 * dt * vel, rtol=0, atol=1e-13)
    np.testing.assert_allclose(st["F"], np.tile(np.eye(dim), (P, 1, 1)), atol=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_ballistic_closed_form(dim):
    """Zero stiffness, gravity only, no walls: symplectic Euler in closed form
    v_n = v0 + n dt g,  x_n = x0 + n dt v0 + dt^2 g n(n+1)/2."""
    rng = np.random.default_rng(4)
    P = 200
    x0 = rng.uniform(0.45, 0.55, size=(P, dim))
    v0 = np.zeros(dim); v0[0] = 0.3
    g = np.zeros(dim); g[1] = -9.8
    st = {"x": x0, "v": np.tile(v0, (P, 1)), "C": np.zeros((P, dim, dim)),
          "F": np.tile(np.eye(dim), (P, 1, 1))}
    sc = _free_scene(dim, 32, np.ones(P), np.full(P, 1e-3), gravity=list(g))
    dt, nst = 1e-4, 100
    for _ in range(nst):
        st = mpm.step(sc, st, dt)
    np.testing.assert_allclose(st["v"], np.tile(v0 + nst * dt * g, (P, 1)), atol=1e-12)
    expect = x0 + nst * dt * v0 + dt * dt * g * nst * (nst + 1) / 2
    np.testing.assert_allclose(st["x"], expect, atol=1e-13)
    assert expect[0, 1] - x0[0, 1] == pytest.approx(-4.949e-4, rel=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_g2p_conserves_momentum_without_walls(dim):
    rng = np.random.default_rng(5)
    P = 300
    n = [32] * dim
    x, v, C, F, m, V0 = _random_particles(rng, dim, n, P)
    model = 0 if dim == 2 else 1
    gm, gmv, gf = mpm.p2g(dim, n, 1 / 32, x, v, C, F, m, V0, model, 2.0, 3.0)
    gv = mpm.grid_update(dim, n, 1e-3, [0.0] * dim, 0, 0, 0.0, gm, gmv, gf)
    _, vn, _, _ = mpm.g2p(dim, n, 1 / 32, 1e-3, gv, x, v, C, F)
    np.testing.assert_allclose((m[:, None] * vn).sum(0), (gm[:, None] * gv).sum(0),
                               atol=1e-12)
    # and the grid momentum is the particle momentum plus dt times the
    # (zero-sum) internal force
    np.testing.assert_allclose((gm[:, None] * gv).sum(0), (m[:, None] * v).sum(0),
                               atol=1e-11)


def _rot(dim, rng):
    Q, R = np.linalg.qr(rng.standard_normal((dim, dim)))
    Q = Q @ np.diag(np.sign(np.diag(R)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    return Q


def psi_fcr(F, mu, la):
    s = np.linalg.svd(F, compute_uv=False)
    J = np.linalg.det(F)
    return mu * np.sum((s - 1.0) ** 2) + 0.5 * la * (J - 1.0) ** 2


def psi_nh(F, mu, la):
    J = np.linalg.det(F)
    d = F.shape[0]
    return 0.5 * mu * (np.trace(F.T @ F) - d) - mu * np.log(J) + 0.5 * la * np.log(J) ** 2


@pytest.mark.parametrize("dim,model", [(2, 0), (2, 1), (3, 0), (3, 1)])
def test_stress_zero_at_rest_and_rotation(dim, model):
    rng = np.random.default_rng(6)
    np.testing.assert_allclose(mpm.kirchhoff(dim, model, 3.0, 4.0, np.eye(dim)), 0, atol=0)
    R = _rot(dim, rng)
    np.testing.assert_allclose(mpm.kirchhoff(dim, model, 3.0, 4.0, R), 0, atol=1e-14)


@pytest.mark.parametrize("dim,model,psi", [(2, 0, psi_fcr), (2, 1, psi_nh), (3, 0, psi_fcr),
                                           (3, 1, psi_nh)])
def test_stress_is_energy_derivative(dim, model, psi):
    """P = dPsi/dF by central differences; tau = P F^T."""
    rng = np.random.default_rng(7)
    mu, la = 3.0, 5.0
    for _ in range(5):
        F = np.eye(dim) + 0.3 * rng.standard_normal((dim, dim))
        if np.linalg.det(F) < 0.2:
            continue
        tau = mpm.kirchhoff(dim, model, mu, la, F)
        P = tau @ np.linalg.inv(F).T
        h = 1e-6
        Pfd = np.zeros((dim, dim))
        for a in range(dim):
            for b in range(dim):
                E = np.zeros((dim, dim)); E[a, b] = h
                Pfd[a, b] = (psi(F + E, mu, la) - psi(F - E, mu, la)) / (2 * h)
        np.testing.assert_allclose(P, Pfd, rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("dim,model", [(2, 0), (2, 1), (3, 0), (3, 1)])
def test_stress_small_strain_limit(dim, model):
    """F = I + e, e symmetric: tau = 2 mu e + la tr(e) I + O(|e|^2).  The
    remainder is bounded by (2 mu + 4 la) |e|_F^2: the mu term by
    2 mu |e^2| (fixed-corotated, R = I) or mu |e^2| (Neo-Hookean), the la
    term by la (tr(e)^2 + |sum of 2x2 minors| + higher), each at most
    d |e|_F^2 <= 3 |e|_F^2 and |e|_F^2."""
    rng = np.random.default_rng(8)
    mu, la = 3.0, 5.0
    eps = 1e-6
    H = rng.standard_normal((dim, dim))
    e = eps * 0.5 * (H + H.T)
    tau = mpm.kirchhoff(dim, model, mu, la, np.eye(dim) + e)
    lin = 2 * mu * e + la * np.trace(e) * np.eye(dim)
    np.testing.assert_allclose(tau, lin, atol=(2 * mu + 4 * la) * np.sum(e * e))


def _kabsch(F):
    """Closest rotation from numpy's SVD: U diag(1, .., det(U V^T)) V^T."""
    U, _, Vt = np.linalg.svd(F)
    D = np.eye(F.shape[0])
    D[-1, -1] = np.sign(np.linalg.det(U @ Vt))
    return U @ D @ Vt


def _random_F(rng, dim, n, inverted=False):
    out = []
    while len(out) < n:
        F = np.eye(dim) + 0.6 * rng.standard_normal((dim, dim))
        J = np.linalg.det(F)
        s = np.linalg.svd(F, compute_uv=False)
        # away from the degenerate cases (repeated or vanishing singular values)
        if (J < 0) == inverted and abs(J) > 0.05 and np.min(np.abs(np.diff(s))) > 0.05:
            out.append(F)
    return out


@pytest.mark.parametrize("dim", [2, 3])
def test_closest_rotation_is_the_polar_rotation(dim):
    """det F > 0: the rotation factor of F = R S with S symmetric positive
    definite, as scipy's polar decomposition gives it."""
    from scipy.linalg import polar
    rng = np.random.default_rng(31)
    for F in _random_F(rng, dim, 20):
        R = mpm.closest_rotation(dim, F)
        np.testing.assert_allclose(R, polar(F)[0], atol=1e-12)
        S = R.T @ F
        np.testing.assert_allclose(S, S.T, atol=1e-12)
        assert np.all(np.linalg.eigvalsh(0.5 * (S + S.T)) > 0)


@pytest.mark.parametrize("dim", [2, 3])
def test_closest_rotation_of_inverted_elements(dim):
    """det F < 0: the rotation of the SVD with the sign moved onto the
    smallest singular value (the Kabsch construction), and it maximises
    tr(R^T F) over 4,000 random rotations."""
    rng = np.random.default_rng(32)
    for F in _random_F(rng, dim, 20, inverted=True):
        R = mpm.closest_rotation(dim, F)
        np.testing.assert_allclose(R.T @ R, np.eye(dim), atol=1e-13)
        assert np.linalg.det(R) == pytest.approx(1.0, abs=1e-13)
        np.testing.assert_allclose(R, _kabsch(F), atol=1e-11)
    F = _random_F(rng, dim, 1, inverted=True)[0]
    best = np.trace(mpm.closest_rotation(dim, F).T @ F)
    trials = [np.trace(_rot(dim, rng).T @ F) for _ in range(4000)]
    assert best >= max(trials) - 1e-12


def test_closest_rotation_reduces_to_the_2d_closed_form():
    """F = blockdiag(F2, 1): the 3D rotation is blockdiag(R2, 1), R2 from
    the closed-form 2D rotation, and a known rotation times a symmetric
    positive definite stretch gives that rotation back."""
    rng = np.random.default_rng(33)
    for F2 in _random_F(rng, 2, 10):
        F = np.eye(3)
        F[:2, :2] = F2
        R = mpm.closest_rotation(3, F)
        want = np.eye(3)
        want[:2, :2] = mpm.closest_rotation(2, F2)
        np.testing.assert_allclose(R, want, atol=1e-12)
    for _ in range(10):
        R0 = _rot(3, rng)
        A = rng.standard_normal((3, 3))
        S = A @ A.T + 0.3 * np.eye(3)
        np.testing.assert_allclose(mpm.closest_rotation(3, R0 @ S), R0, atol=1e-11)


def test_fcr_stress_is_rotation_covariant_and_defined_when_inverted():
    """tau(Q F) = Q tau(F) Q^T; for det F < 0 the stress is the derivative
    of the energy with the signed smallest singular value (the inverted
    branch of the fixed-corotated model), by central differences."""
    rng = np.random.default_rng(34)
    mu, la = 3.0, 5.0
    for F in _random_F(rng, 3, 5):
        Q = _rot(3, rng)
        np.testing.assert_allclose(mpm.kirchhoff(3, 0, mu, la, Q @ F),
                                   Q @ mpm.kirchhoff(3, 0, mu, la, F) @ Q.T, atol=1e-11)

    def psi_signed(F):
        s = np.linalg.svd(F, compute_uv=False)
        J = np.linalg.det(F)
        s[-1] *= np.sign(J)
        return mu * np.sum((s - 1.0) ** 2) + 0.5 * la * (J - 1.0) ** 2

    for F in _random_F(rng, 3, 5, inverted=True):
        P = mpm.kirchhoff(3, 0, mu, la, F) @ np.linalg.inv(F).T
        h = 1e-6
        Pfd = np.zeros((3, 3))
        for a in range(3):
            for b in range(3):
                E = np.zeros((3, 3))
                E[a, b] = h
                Pfd[a, b] = (psi_signed(F + E) - psi_signed(F - E)) / (2 * h)
        np.testing.assert_allclose(P, Pfd, rtol=1e-6, atol=1e-6)


def test_nh_rejects_inverted_element():
    F = np.diag([-1.0, 1.0, 1.0])
    with pytest.raises(mpm.OracleDomainError):
        mpm.kirchhoff(3, 1, 1.0, 1.0, F)


def _one_node_grid(dim, n, ijk, vel, mass=2.0):
    nn = n ** dim
    gm = np.zeros(nn); gmv = np.zeros((nn, dim)); gf = np.zeros((nn, dim))
    idx = ijk[-1]
    for a in range(dim - 2, -1, -1):
        idx = idx * n + ijk[a]
    gm[idx] = mass
    gmv[idx] = mass * np.asarray(vel, dtype=float)
    return gm, gmv, gf, idx


@pytest.mark.parametrize("vel,expect", [
    ((0.1, -1.0, 0.0), (0.0, 0.0, 0.0)),      # stick: |v_t| <= mu |v_n|
    ((1.0, -1.0, 0.0), (0.7, 0.0, 0.0)),      # slip: v_t scaled by 1 - mu |v_n| / |v_t|
    ((0.0, -2.0, 1.0), (0.0, 0.0, 0.4)),
    ((1.0, 1.0, 0.5), (1.0, 1.0, 0.5)),       # separating: untouched
])
def test_coulomb_floor_cases(vel, expect):
    n = 16
    gm, gmv, gf, idx = _one_node_grid(3, n, (8, 1, 8), vel)
    gv = mpm.grid_update(3, [n] * 3, 1e-3, [0, 0, 0], 3, 1, 0.3, gm, gmv, gf)
    np.testing.assert_allclose(gv[idx], expect, atol=1e-15)


@pytest.mark.parametrize("ijk", [(1, 8, 8), (8, 8, 14), (8, 13, 8), (2, 1, 8)])
def test_sticky_walls(ijk):
    n = 16
    gm, gmv, gf, idx = _one_node_grid(3, n, ijk, (0.5, -0.5, 0.25))
    gv = mpm.grid_update(3, [n] * 3, 1e-3, [0, 0, 0], 3, 1, 0.3, gm, gmv, gf)
    np.testing.assert_allclose(gv[idx], 0.0, atol=0)


def test_interior_node_and_empty_node():
    n = 16
    gm, gmv, gf, idx = _one_node_grid(2, n, (8, 8), (0.5, -0.5))
    gf[idx] = [2.0, 4.0]
    gv = mpm.grid_update(2, [n] * 2, 0.1, [0.0, -10.0], 3, 0, 0.0, gm, gmv, gf)
    np.testing.assert_allclose(gv[idx], [0.5 + 0.1 * 1.0, -0.5 + 0.1 * (2.0 - 10.0)], atol=1e-15)
    assert np.count_nonzero(gv) == 2


def test_two_dimensional_block_is_stable():
    from paper_2109_12390_amd import scenes
    s = scenes.scene_2d()
    mu, la = mpm.lame(s["E"], s["nu"])
    sc = dict(dim=2, n=s["n"], dx=s["dx"], bound=3, floor_mode=0, mu_f=0.0,
              gravity=s["gravity"], model=0, mu=mu, la=la,
              m=np.full(s["P"], float(s["m"])), V0=np.full(s["P"], float(s["V0"])))
    st = {k: v.astype(np.float64) for k, v in scenes.initial_state(s).items()}
    for _ in range(50):
        st = mpm.step(sc, st, s["dt"])
    J = np.linalg.det(st["F"])
    assert 0.99 < J.min() and J.max() < 1.01
    assert np.abs(st["v"]).max() < 0.1


def test_cell_keys_and_stable_sort():
    rng = np.random.default_rng(9)
    x = rng.uniform(0.2, 0.8, size=(1000, 3))
    x[500:600] = x[100:200]   # duplicate cells keep input order
    keys = mpm.cell_keys(3, [16] * 3, 1 / 16, x)
    b = np.floor(x * 16 - 0.5).astype(int)
    np.testing.assert_array_equal(keys, b[:, 0] + 16 * (b[:, 1] + 16 * b[:, 2]))
    perm = mpm.cell_sort_permutation(3, [16] * 3, 1 / 16, x)
    sk = keys[perm]
    assert np.all(np.diff(sk) >= 0)
    for k in np.unique(keys):
        idx = perm[sk == k]
        assert np.all(np.diff(idx) > 0)
    x[0] = [0.01, 0.5, 0.5]
    assert mpm.cell_keys(3, [16] * 3, 1 / 16, x)[0] == -1


@pytest.mark.parametrize("threads", [1, 4])
def test_threaded_step_matches_the_plain_oracle(threads):
    """The OpenMP driver (private grids summed in thread order) against the
    plain step: bitwise with one thread, to summation-order rounding with
    four, over steps with contact on the Coulomb floor."""
    from paper_2109_12390_amd import scenes
    s = scenes.scene_3d(n=32, cube_cells=8, seed=9, v0=(0.3, -2.0, 0.1))
    st = {k: v.astype(np.float64) for k, v in scenes.initial_state(s).items()}
    mu, la = mpm.lame(s["E"], s["nu"])
    sc = dict(dim=3, n=s["n"], dx=s["dx"], bound=s["bound"], floor_mode=s["floor_mode"],
              mu_f=s["mu_f"], gravity=s["gravity"], model=s["model"], mu=mu, la=la,
              m=np.full(s["P"], float(s["m"])), V0=np.full(s["P"], float(s["V0"])))
    a, b = st, st
    for _ in range(5):
        a = mpm.step(sc, a, s["dt"])
        b = mpm.step_threaded(sc, b, s["dt"], threads=threads)
    for k in ("x", "v", "C", "F"):
        if threads == 1:
            assert np.array_equal(a[k], b[k]), k
        else:
            # C is a velocity gradient (rounding noise on a near-rigid body):
            # measured against |v| / dx
            scale = np.max(np.abs(a[k])) if k != "C" else np.max(np.abs(a["v"])) / s["dx"]
            assert np.max(np.abs(a[k] - b[k])) <= 1e-12 * scale, k
