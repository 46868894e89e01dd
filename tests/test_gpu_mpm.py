"""Parity of the HIP MPM kernels (mpm_p2g, mpm_grid_update, mpm_g2p,
mpm_cell_sort, mpm_step) with the FP64 oracle on the same seeded inputs.

Tolerances (fp32 kernels against fp64 on fp32-rounded inputs): every node or
particle value is a short sum of fp32 products (a few ulps each, 2^-24 =
6e-8 relative), so single-kernel outputs are compared per element with an
absolute tolerance of 2e-5 times the largest magnitude of that channel
(momentum and force terms cancel, so a relative bound per element would be
meaningless).  Whole steps use the stated targets: relative L2 of particle
positions <= 1e-5 after one step and <= 1e-3 after 100 steps, plus the
stricter checks on velocities listed in each test."""
import os

import numpy as np
import pytest

from oracle import mpm as OM
from paper_2109_12390_amd import binding as B
from paper_2109_12390_amd import scenes
from tests.helpers import aos, oracle_scene, rel_l2, soa, tile_slot_order

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

dev = "cuda"


def T(a, dtype=torch.float32):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=dev)


def make_parts(_B, x, v, C, F, m=None, V0=None, m_u=0.0, V0_u=0.0):
    return B.Particles(T(soa(x)), T(soa(v)), T(soa(C)), T(soa(F)),
                       None if m is None else T(np.asarray(m, dtype=np.float32)),
                       None if V0 is None else T(np.asarray(V0, dtype=np.float32)), m_u, V0_u)


def random_state(rng, dim, P, lo=0.3, hi=0.7, Fs=0.05):
    x = rng.uniform(lo, hi, size=(P, dim)).astype(np.float32)
    v = rng.standard_normal((P, dim)).astype(np.float32)
    C = (5 * rng.standard_normal((P, dim, dim))).astype(np.float32)
    F = (np.eye(dim) + Fs * rng.standard_normal((P, dim, dim))).astype(np.float32)
    m = rng.uniform(0.5, 2.0, size=P).astype(np.float32) * 1e-3
    V0 = rng.uniform(0.5, 2.0, size=P).astype(np.float32) * 1e-6
    return x, v, C, F, m, V0


def close_channels(got, ref, frac=2e-5, name=""):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.max(np.abs(ref), axis=0, keepdims=True)
    scale = np.where(scale > 0, scale, 1.0)
    err = np.max(np.abs(got - ref) / scale)
    print("%s: max err / channel scale = %.3e" % (name, err))
    assert err <= frac, name


@pytest.mark.parametrize("dim,model,apic", [(2, 0, True), (3, 1, True), (3, 1, False), (2, 1, False),
                                            (3, 0, True), (3, 0, False)])
@pytest.mark.parametrize("P", [1, 777, 5000])
def test_p2g_matches_oracle(gpu, dim, model, apic, P):
    rng = np.random.default_rng(10 + dim + P)
    n = [24] * dim
    dx = 1.0 / 24
    x, v, C, F, m, V0 = random_state(rng, dim, P)
    mu, la = OM.lame(1e4, 0.3)
    dt = 1e-4
    gm, gmv, gf = OM.p2g(dim, n, dx, x, v, C, F, m, V0, model, mu, la, apic=apic)
    grid = B.Grid(dim, n, dx, bound=3)
    gbuf = torch.full((int(np.prod(n)) * 4,), 7.0, device=dev)   # p2g must overwrite
    parts = make_parts(B, x, v, C, F, m, V0)
    B.mpm_p2g(grid, (model, 1e4, 0.3), parts, gbuf, dt, flags=0 if apic else B.NO_AFFINE)
    g = gbuf.cpu().numpy().reshape(-1, 4)
    close_channels(g[:, 0], gm, name="mass")
    close_channels(g[:, 1:1 + dim], gmv + dt * gf, name="momentum")
    assert np.all(g[:, 1 + dim:] == 0)


def _large_deformations(rng, P):
    """Every third particle a rotation with 1e-4 strain; the others
    rotations times symmetric stretches (singular values 0.3-2.5), half of
    them reflected (det F < 0) with the two smallest singular values at
    least 0.1 apart.  (A reflection with nearly equal smallest singular
    values has two almost equally close rotations, and its stress jumps
    between them: no finite precision resolves which one, so such states
    are left out.)"""
    out = np.empty((P, 3, 3))
    for p in range(P):
        Q, R = np.linalg.qr(rng.standard_normal((3, 3)))
        Q = Q @ np.diag(np.sign(np.diag(R)))
        if np.linalg.det(Q) < 0:
            Q[:, 0] = -Q[:, 0]
        W, _ = np.linalg.qr(rng.standard_normal((3, 3)))
        if p % 3 == 0:
            sv = 1.0 + 1e-4 * rng.standard_normal(3)
        else:
            while True:
                sv = np.sort(rng.uniform(0.3, 2.5, size=3))[::-1].copy()
                if sv[1] - sv[2] >= 0.1:
                    break
            if p % 2:
                sv[2] = -sv[2]
        out[p] = Q @ W @ np.diag(sv) @ W.T
    return out.astype(np.float32)


@pytest.mark.parametrize("P", [2, 3000])
def test_fixed_corotated_forces_under_large_deformation(gpu, P):
    """3D fixed-corotated internal forces (v = C = 0, so the momentum
    channel is dt f) for rotated, stretched and inverted deformation
    gradients against the oracle's closest-rotation stress, to 1e-4 of the
    channel scale.  (The rotated small-strain particles carry an fp32 error
    of about 1e-7 of 2 mu, from forming F F^T - I out of O(1) entries.)"""
    rng = np.random.default_rng(71 + P)
    dim, n, dx, dt = 3, [24] * 3, 1.0 / 24, 1e-4
    x = rng.uniform(0.3, 0.7, size=(P, dim)).astype(np.float32)
    F = _large_deformations(rng, P)
    zeros = np.zeros((P, dim), np.float32)
    m = np.full(P, 1e-3, np.float32)
    V0 = np.full(P, 1e-6, np.float32)
    mu, la = OM.lame(1e4, 0.3)
    gm, gmv, gf = OM.p2g(dim, n, dx, x, zeros, np.zeros((P, 3, 3)), F, m, V0, 0, mu, la, apic=False)
    gbuf = torch.zeros(int(np.prod(n)) * 4, device=dev)
    parts = make_parts(B, x, zeros, np.zeros((P, 3, 3), np.float32), F, m, V0)
    B.mpm_p2g(B.Grid(dim, n, dx, bound=3), (B.FIXED_COROTATED, 1e4, 0.3), parts, gbuf, dt,
              flags=B.NO_AFFINE)
    g = gbuf.cpu().numpy().reshape(-1, 4)
    close_channels(g[:, 1:4] / dt, gf, frac=1e-4, name="force")


@pytest.mark.parametrize("dim", [2, 3])
def test_grid_update_matches_oracle(gpu, dim):
    rng = np.random.default_rng(20 + dim)
    n = [16] * dim
    nn = 16 ** dim
    g = np.zeros((nn, 4), dtype=np.float32)
    mask = rng.random(nn) < 0.7
    g[mask, 0] = rng.uniform(0.1, 2.0, size=mask.sum())
    g[mask, 1:1 + dim] = rng.standard_normal((mask.sum(), dim))
    gravity = [0.0, -9.8, 0.0][:dim] if dim == 3 else [0.0, -9.8]
    for floor_mode, muf in [(0, 0.0), (1, 0.3)]:
        if dim == 2 and floor_mode == 1:
            floor_mode = 0
        gv = OM.grid_update(dim, n, 1e-2, gravity, 3, floor_mode, muf, g[:, 0].astype(np.float64),
                            g[:, 1:1 + dim].astype(np.float64), np.zeros((nn, dim)))
        gbuf = T(g.reshape(-1))
        B.mpm_grid_update(B.Grid(dim, n, 1 / 16, 3, floor_mode, muf, gravity), 1e-2, gbuf)
        out = gbuf.cpu().numpy().reshape(-1, 4)
        close_channels(out[:, 1:1 + dim], gv, name="grid velocity")
        np.testing.assert_array_equal(out[:, 0], g[:, 0])
    # active-list form: only listed nodes change
    act = np.sort(rng.choice(nn, size=50, replace=False)).astype(np.int32)
    gbuf = T(g.reshape(-1))
    B.mpm_grid_update(B.Grid(dim, n, 1 / 16, 3, 0, 0.0, gravity), 1e-2, gbuf, active=T(act, torch.int32))
    out = gbuf.cpu().numpy().reshape(-1, 4)
    untouched = np.setdiff1d(np.arange(nn), act)
    np.testing.assert_array_equal(out[untouched], g[untouched])


@pytest.mark.parametrize("dim,apic", [(2, True), (3, True), (3, False)])
def test_g2p_matches_oracle(gpu, dim, apic):
    rng = np.random.default_rng(30 + dim)
    n = [24] * dim
    dx = 1 / 24
    P = 3000
    x, v, C, F, m, V0 = random_state(rng, dim, P)
    gv = rng.standard_normal((24 ** dim, dim)).astype(np.float32)
    gbuf = np.zeros((24 ** dim, 4), dtype=np.float32)
    gbuf[:, 0] = 1.0
    gbuf[:, 1:1 + dim] = gv
    dt = 1e-3
    xo, vo, Co, Fo = OM.g2p(dim, n, dx, dt, gv.astype(np.float64), x, v, C, F, apic=apic)
    parts = make_parts(B, x, v, C, F)
    B.mpm_g2p(B.Grid(dim, n, dx), parts, dt, T(gbuf.reshape(-1)), flags=0 if apic else B.NO_AFFINE)
    close_channels(aos(parts.v.cpu().numpy(), dim), vo, name="v")
    close_channels(aos(parts.C.cpu().numpy(), dim, True).reshape(P, -1), Co.reshape(P, -1), name="C")
    np.testing.assert_allclose(aos(parts.F.cpu().numpy(), dim, True), Fo, atol=2e-6)
    np.testing.assert_allclose(aos(parts.x.cpu().numpy(), dim), xo, atol=2e-7)
    # trial mode on a subset (Algorithm 5, last steps)
    sub = np.sort(rng.choice(P, size=100, replace=False))
    xt, vt = OM.g2p(dim, n, dx, dt, gv.astype(np.float64), x, v, C, F, subset=sub, trial=True)
    parts = make_parts(B, x, v, C, F)
    x_tr = torch.zeros(dim * 100, device=dev)
    v_tr = torch.zeros(dim * 100, device=dev)
    B.mpm_g2p(B.Grid(dim, n, dx), parts, dt, T(gbuf.reshape(-1)), subset=T(sub, torch.int32),
              flags=B.TRIAL, x_trial=x_tr, v_trial=v_tr)
    np.testing.assert_allclose(x_tr.cpu().numpy().reshape(dim, 100).T, xt, atol=2e-7)
    close_channels(v_tr.cpu().numpy().reshape(dim, 100).T, vt, name="v_trial")
    np.testing.assert_array_equal(parts.x.cpu().numpy(), soa(x))   # untouched


@pytest.mark.parametrize("dim,P", [(3, 4096), (3, 20000), (2, 4096), (3, 0)])
def test_cell_sort_permutation_is_bit_exact(gpu, dim, P):
    rng = np.random.default_rng(40 + P)
    n = [32] * dim
    dx = 1 / 32
    x, v, C, F, m, V0 = random_state(rng, dim, P, lo=0.12, hi=0.88)
    if P > 10:
        x[5] = x[7]        # shared cells keep their order
        x[9] = 0.01        # outside the lattice: last, flagged
    grid = B.Grid(dim, n, dx)
    parts = make_parts(B, x, v, C, F, m, V0)
    ws = B.new_workspace(grid, P)
    perm = torch.zeros(max(P, 1), dtype=torch.int32, device=dev)[:P]
    flag = torch.zeros(1, dtype=torch.int32, device=dev)
    B.mpm_cell_sort(grid, parts, ws, perm_out=perm if P else None, status=flag)
    if P == 0:
        return
    expect = tile_slot_order(dim, n, dx, x)
    got = perm.cpu().numpy()
    np.testing.assert_array_equal(got, expect)
    np.testing.assert_array_equal(parts.x.cpu().numpy(), soa(x[expect]))
    np.testing.assert_array_equal(parts.F.cpu().numpy(), soa(F[expect]))
    np.testing.assert_array_equal(parts.m.cpu().numpy(), m[expect])
    assert flag.item() & B.FLAG_DOMAIN


@pytest.mark.parametrize("dim,P,move,opts", [
    (3, 20000, "random", ""), (2, 6000, "random", ""),
    (3, 20000, "none", ""), (2, 6000, "none", ""),
    (3, 20000, "rigid", ""), (2, 6000, "rigid", ""),
    (3, 60000, "dense", ""),
    (3, 20000, "random", "uniform"), (3, 20000, "random", "noaffine"),
    (3, 20000, "random", "corotated"), (3, 60000, "dense", "uniform"),
    (3, 9000, "random", "odd"), (3, 9000, "none", "odd-uniform")])
def test_sorted_tiled_p2g_matches_oracle(gpu, dim, P, move, opts):
    """Cell-sort, then the tiled P2G with the particles moved since the sort:
    random: by up to 1.4 cells each (mixed drifts, some beyond the drift
    margin: deferred particles, claims and the global fallback); none: every
    particle in its sort-time cell; rigid: all translated by one cell
    diagonally (every lane drifted, distinct base cells); dense: 60,000
    particles in a 4-cell cube moved randomly, thousands of drifted
    particles per tile (the deferred list fills and the rest wait in the
    tile's spill range).  Options: uniform masses and volumes instead of
    per-particle arrays, the plain transfer (no affine term), the
    fixed-corotated law, and an odd tile count per axis (22 nodes: 5 tiles,
    a ragged brick of the XCD-aware tile order)."""
    rng = np.random.default_rng(50 + dim + len(opts))
    nn = 22 if "odd" in opts else 40
    n = [nn] * dim
    dx = 1 / nn
    lo, hi = (0.45, 0.55) if move == "dense" else (0.2, 0.8)
    x, v, C, F, m, V0 = random_state(rng, dim, P, lo=lo, hi=hi)
    uniform = "uniform" in opts
    if uniform:
        m[:] = np.float32(1.3e-3)
        V0[:] = np.float32(0.9e-6)
    grid = B.Grid(dim, n, dx)
    parts = (make_parts(B, x, v, C, F, m_u=float(m[0]), V0_u=float(V0[0])) if uniform
             else make_parts(B, x, v, C, F, m, V0))
    ws = B.new_workspace(grid, P)
    perm = torch.zeros(P, dtype=torch.int32, device=dev)
    B.mpm_cell_sort(grid, parts, ws, perm_out=perm)
    p = perm.cpu().numpy()
    if move in ("random", "dense"):
        xs = x[p] + (rng.uniform(-1.4, 1.4, size=(P, dim)) * dx).astype(np.float32)
    elif move == "rigid":
        xs = x[p] + np.float32(dx) * np.array([1.0, -1.0, 1.0][:dim], dtype=np.float32)
    else:
        xs = x[p].copy()
    parts.x.copy_(T(soa(xs)))
    model = 0 if (dim == 2 or opts == "corotated") else 1
    apic = opts != "noaffine"
    mu, la = OM.lame(1e4, 0.3)
    gm, gmv, gf = OM.p2g(dim, n, dx, xs, v[p], C[p], F[p], m[p], V0[p], model, mu, la, apic=apic)
    gbuf = torch.zeros(int(np.prod(n)) * 4, device=dev)
    flags = B.SORTED | (0 if apic else B.NO_AFFINE)
    B.mpm_p2g(grid, (model, 1e4, 0.3), parts, gbuf, 1e-4, flags=flags, workspace=ws)
    g = gbuf.cpu().numpy().reshape(-1, 4)
    close_channels(g[:, 0], gm, name="mass")
    close_channels(g[:, 1:1 + dim], gmv + 1e-4 * gf, name="momentum")


@pytest.mark.parametrize("dim,P", [(3, 20000), (2, 6000)])
def test_deterministic_p2g_is_bitwise_reproducible(gpu, dim, P):
    """MR_DETERMINISTIC: after the canonical sort the grid is bitwise the
    same for a shuffled input order and on a repeated run, every node is
    written (no zeroing needed), and it matches the oracle; particles moved
    beyond the drift margin raise MR_FLAG_DRIFT."""
    rng = np.random.default_rng(60 + dim)
    n = [40] * dim
    dx = 1 / 40
    x, v, C, F, m, V0 = random_state(rng, dim, P, lo=0.2, hi=0.8)
    grid = B.Grid(dim, n, dx)
    model = 0 if dim == 2 else 1
    nodes = int(np.prod(n))
    grids = []
    for order in (np.arange(P), rng.permutation(P), np.arange(P)):
        parts = make_parts(B, x[order], v[order], C[order], F[order], m[order], V0[order])
        ws = B.new_workspace(grid, P)
        flag = torch.zeros(1, dtype=torch.int32, device=dev)
        B.mpm_cell_sort_ex(grid, parts, ws, B.DETERMINISTIC, status=flag)
        gbuf = torch.full((nodes * 4,), 7.0, device=dev)
        B.mpm_p2g(grid, (model, 1e4, 0.3), parts, gbuf, 1e-4, flags=B.SORTED | B.DETERMINISTIC,
                  workspace=ws, status=flag)
        assert flag.item() == 0
        grids.append(gbuf.cpu().numpy())
    assert np.array_equal(grids[0], grids[1]) and np.array_equal(grids[0], grids[2])
    mu, la = OM.lame(1e4, 0.3)
    gm, gmv, gf = OM.p2g(dim, n, dx, x, v, C, F, m, V0, model, mu, la)
    g = grids[0].reshape(-1, 4)
    close_channels(g[:, 0], gm, name="mass")
    close_channels(g[:, 1:1 + dim], gmv + 1e-4 * gf, name="momentum")
    # motion beyond the margin since the sort is reported, not scattered
    parts = make_parts(B, x, v, C, F, m, V0)
    ws = B.new_workspace(grid, P)
    perm = torch.zeros(P, dtype=torch.int32, device=dev)
    B.mpm_cell_sort_ex(grid, parts, ws, B.DETERMINISTIC, perm_out=perm)
    p = perm.cpu().numpy()
    xs = x[p] + (rng.uniform(-1.4, 1.4, size=(P, dim)) * dx).astype(np.float32)
    parts.x.copy_(T(soa(xs)))
    flag = torch.zeros(1, dtype=torch.int32, device=dev)
    gbuf = torch.zeros(nodes * 4, device=dev)
    B.mpm_p2g(grid, (model, 1e4, 0.3), parts, gbuf, 1e-4, flags=B.SORTED | B.DETERMINISTIC,
              workspace=ws, status=flag)
    assert flag.item() & B.FLAG_DRIFT


def test_deterministic_steps_are_bitwise_reproducible(gpu):
    """mpm_step with MR_DETERMINISTIC from the same state in two input
    orders: after relabelling by perm_accum the final x, v, C, F agree bit
    for bit (and with a repeated run), and stay within rounding of the
    default schedule."""
    s = scenes.scene_3d(n=32, cube_cells=8, seed=5, v0=(0.3, -2.0, 0.1))
    st0 = scenes.initial_state(s)
    P = s["P"]
    grid = _gpu_scene(B, s)
    rng = np.random.default_rng(61)
    outs = []
    for order, det in ((np.arange(P), True), (rng.permutation(P), True), (np.arange(P), True),
                       (np.arange(P), False)):
        parts = make_parts(B, st0["x"][order], st0["v"][order], st0["C"][order], st0["F"][order],
                           m_u=float(s["m"]), V0_u=float(s["V0"]))
        gbuf = torch.zeros(grid.nodes() * 4, device=dev)
        ws = torch.zeros(B.mpm_step_workspace_bytes(grid, P), dtype=torch.uint8, device=dev)
        perm = torch.zeros(P, dtype=torch.int32, device=dev)
        flag = torch.zeros(1, dtype=torch.int32, device=dev)
        B.mpm_step(grid, (s["model"], s["E"], s["nu"]), parts, s["dt"], 30, 10,
                   B.DETERMINISTIC if det else 0, gbuf, ws, perm_accum=perm, status=flag)
        assert flag.item() == 0
        ident = order[perm.cpu().numpy()]           # original label of every slot
        inv = np.empty(P, dtype=np.int64)
        inv[ident] = np.arange(P)
        outs.append({k: getattr(parts, k).cpu().numpy()[:, inv] for k in ("x", "v", "C", "F")})
    for k in ("x", "v", "C", "F"):
        assert np.array_equal(outs[0][k], outs[1][k]), k
        assert np.array_equal(outs[0][k], outs[2][k]), k
    print("deterministic vs default schedule after 30 steps: x %.2e" % rel_l2(outs[0]["x"], outs[3]["x"]))
    assert rel_l2(outs[0]["x"], outs[3]["x"]) < 1e-6


def _run_oracle(sc, st, dt, steps):
    st = {k: np.asarray(v, dtype=np.float64) for k, v in st.items()}
    for _ in range(steps):
        st = OM.step(sc, st, dt)
    return st


def _gpu_scene(B, s):
    return B.Grid(s["dim"], s["n"], s["dx"], s["bound"], s["floor_mode"], s["mu_f"], s["gravity"])


@pytest.mark.parametrize("steps,sort_every", [(1, 0), (100, 0), (100, 10)])
def test_two_dimensional_scene_trajectory(gpu, steps, sort_every):
    s = scenes.scene_2d()
    st0 = scenes.initial_state(s)
    ref = _run_oracle(oracle_scene(s), st0, s["dt"], steps)
    parts = make_parts(B, st0["x"], st0["v"], st0["C"], st0["F"], m_u=float(s["m"]), V0_u=float(s["V0"]))
    grid = _gpu_scene(B, s)
    gbuf = torch.zeros(grid.nodes() * 4, device=dev)
    ws = torch.zeros(B.mpm_step_workspace_bytes(grid, s["P"]), dtype=torch.uint8, device=dev)
    perm = torch.zeros(s["P"], dtype=torch.int32, device=dev)
    flag = torch.zeros(1, dtype=torch.int32, device=dev)
    B.mpm_step(grid, (s["model"], s["E"], s["nu"]), parts, s["dt"], steps, sort_every, 0, gbuf, ws,
               perm_accum=perm, status=flag)
    p = perm.cpu().numpy()
    inv = np.empty_like(p)
    inv[p] = np.arange(len(p))
    x = aos(parts.x.cpu().numpy(), 2)[inv]
    v = aos(parts.v.cpu().numpy(), 2)[inv]
    F = aos(parts.F.cpu().numpy(), 2, True)[inv]
    ex = rel_l2(x, ref["x"])
    ev = rel_l2(v, ref["v"])
    # F - I after one step is ~1e-6, below fp32 resolution of F itself
    # (ulp(1) = 1.2e-7), so F is compared in absolute terms
    eF = float(np.max(np.abs(F - ref["F"])))
    ed = rel_l2(x - s["X"], ref["x"] - s["X"])
    print("2D steps=%d sort=%d: x %.3e  v %.3e  max|dF| %.3e  displacement %.3e" % (steps, sort_every, ex, ev, eF, ed))
    assert flag.item() == 0
    assert ex <= (1e-5 if steps == 1 else 1e-3)
    assert ev <= (1e-4 if steps == 1 else 1e-2)
    assert eF <= (1e-6 if steps == 1 else 1e-4)


def test_three_dimensional_scene_small(gpu):
    """3D Neo-Hookean cube on a Coulomb floor, 20^3... 8^3-cell cube on a
    32^3 grid, 100 steps with sorting every 10."""
    s = scenes.scene_3d(n=32, cube_cells=8, seed=5, v0=(0.3, -2.0, 0.1))
    st0 = scenes.initial_state(s)
    steps = 100
    ref = _run_oracle(oracle_scene(s), st0, s["dt"], steps)
    parts = make_parts(B, st0["x"], st0["v"], st0["C"], st0["F"], m_u=float(s["m"]), V0_u=float(s["V0"]))
    grid = _gpu_scene(B, s)
    gbuf = torch.zeros(grid.nodes() * 4, device=dev)
    ws = torch.zeros(B.mpm_step_workspace_bytes(grid, s["P"]), dtype=torch.uint8, device=dev)
    perm = torch.zeros(s["P"], dtype=torch.int32, device=dev)
    B.mpm_step(grid, (s["model"], s["E"], s["nu"]), parts, s["dt"], steps, 10, 0, gbuf, ws, perm_accum=perm)
    p = perm.cpu().numpy()
    inv = np.empty_like(p)
    inv[p] = np.arange(len(p))
    x = aos(parts.x.cpu().numpy(), 3)[inv]
    v = aos(parts.v.cpu().numpy(), 3)[inv]
    ex, ev = rel_l2(x, ref["x"]), rel_l2(v, ref["v"])
    ed = rel_l2(x - s["X"], ref["x"] - s["X"])
    print("3D small 100 steps: x %.3e v %.3e displacement %.3e" % (ex, ev, ed))
    assert ex <= 1e-3 and ev <= 1e-2 and ed <= 1e-2


def _gpu_trajectory(s, st0, steps, sort_every=10, model=None):
    parts = make_parts(B, st0["x"], st0["v"], st0["C"], st0["F"], m_u=float(s["m"]),
                       V0_u=float(s["V0"]))
    grid = _gpu_scene(B, s)
    gbuf = torch.zeros(grid.nodes() * 4, device=dev)
    ws = torch.zeros(B.mpm_step_workspace_bytes(grid, s["P"]), dtype=torch.uint8, device=dev)
    perm = torch.zeros(s["P"], dtype=torch.int32, device=dev)
    flag = torch.zeros(1, dtype=torch.int32, device=dev)
    B.mpm_step(grid, (s["model"] if model is None else model, s["E"], s["nu"]), parts, s["dt"],
               steps, sort_every, 0, gbuf, ws, perm_accum=perm, status=flag)
    p = perm.cpu().numpy()
    inv = np.empty_like(p)
    inv[p] = np.arange(len(p))
    return (aos(parts.x.cpu().numpy(), 3)[inv], aos(parts.v.cpu().numpy(), 3)[inv],
            aos(parts.F.cpu().numpy(), 3, True)[inv], flag.item())


@pytest.mark.parametrize("model", [scenes.MODEL_NEO_HOOKEAN, scenes.MODEL_FIXED_COROTATED])
def test_three_dimensional_contact_100_steps(gpu, model):
    """An 8^3-cell jittered cube released just above the Coulomb floor band
    and thrown down and sideways, 100 steps with sorting every 10: the bottom
    layers reach the floor band early in the run, stick or slide there (in
    the oracle's run the lowest particles end above their free-flight height
    and the bottom layer loses a third of its sideways speed to friction),
    and the trajectory stays within the 1e-3 bound of the oracle."""
    dx = 1 / 32
    s = scenes.make_scene(3, 32, (8, 8, 8), (0.5 - 4 * dx, 3.8 * dx, 0.5 - 4 * dx), 2, 1000.0, 5.0e4,
                          0.3, model, (0.0, -9.8, 0.0), scenes.FLOOR_COULOMB, 0.3, 3, 5.0e-5,
                          seed=13, v0=(1.5, -6.0, 0.8))
    st0 = scenes.initial_state(s)
    steps = 100
    ref = _run_oracle(oracle_scene(s), st0, s["dt"], steps)
    # contact happened in the reference: the lowest particles stopped above
    # where free flight would have taken them
    t = steps * s["dt"]
    y0 = s["X"][:, 1].astype(np.float64)
    free = y0 - 6.0 * t - 0.5 * 9.8 * t * t
    bottom = y0 < y0.min() + 0.5 * dx
    assert np.mean(ref["x"][bottom, 1] - free[bottom]) > 0.03 * dx
    assert np.mean(ref["v"][bottom, 0]) < 0.8 * 1.5
    x, v, F, flag = _gpu_trajectory(s, st0, steps)
    ex, ev = rel_l2(x, ref["x"]), rel_l2(v, ref["v"])
    ed = rel_l2(x - s["X"], ref["x"] - s["X"])
    eF = float(np.max(np.abs(F - ref["F"])))
    print("3D contact model %d: x %.3e v %.3e displacement %.3e max|dF| %.3e; bottom layer "
          "sideways speed %.3f (released at 1.5)" % (model, ex, ev, ed, eF,
                                                     float(np.mean(ref["v"][bottom, 0]))))
    assert flag == 0
    assert ex <= 1e-3 and ev <= 1e-2 and ed <= 1e-2 and eF <= 1e-3


def test_three_dimensional_full_size_100_steps(gpu):
    """The 2,097,152-particle benchmark scene in the benchmark's launch
    configuration (mpm_step, sort every 10), 100 steps against the threaded
    FP64 oracle on every particle: relative L2 of positions within 1e-3."""
    s = scenes.scene_3d()
    st0 = scenes.initial_state(s)
    steps = 100
    sc = oracle_scene(s)
    ref = {k: np.asarray(v, dtype=np.float64) for k, v in st0.items()}
    for _ in range(steps):
        ref = OM.step_threaded(sc, ref, s["dt"], threads=int(os.environ.get("OMP_NUM_THREADS",
                                                                              "0") or 0))
    x, v, F, flag = _gpu_trajectory(s, st0, steps)
    ex, ev = rel_l2(x, ref["x"]), rel_l2(v, ref["v"])
    ed = rel_l2(x - s["X"], ref["x"] - s["X"])
    print("3D full size, 100 steps: x %.3e v %.3e displacement %.3e" % (ex, ev, ed))
    assert flag == 0
    assert ex <= 1e-3 and ev <= 1e-2 and ed <= 1e-2


def test_three_dimensional_fixed_corotated_scene(gpu):
    """The 3D scene above with the fixed-corotated law (the paper's
    constitutive model), 100 steps, sorting every 10."""
    s = scenes.scene_3d(n=32, cube_cells=8, seed=5, v0=(0.3, -2.0, 0.1))
    s["model"] = scenes.MODEL_FIXED_COROTATED
    st0 = scenes.initial_state(s)
    steps = 100
    ref = _run_oracle(oracle_scene(s), st0, s["dt"], steps)
    parts = make_parts(B, st0["x"], st0["v"], st0["C"], st0["F"], m_u=float(s["m"]), V0_u=float(s["V0"]))
    grid = _gpu_scene(B, s)
    gbuf = torch.zeros(grid.nodes() * 4, device=dev)
    ws = torch.zeros(B.mpm_step_workspace_bytes(grid, s["P"]), dtype=torch.uint8, device=dev)
    perm = torch.zeros(s["P"], dtype=torch.int32, device=dev)
    flag = torch.zeros(1, dtype=torch.int32, device=dev)
    B.mpm_step(grid, (s["model"], s["E"], s["nu"]), parts, s["dt"], steps, 10, 0, gbuf, ws,
               perm_accum=perm, status=flag)
    p = perm.cpu().numpy()
    inv = np.empty_like(p)
    inv[p] = np.arange(len(p))
    x = aos(parts.x.cpu().numpy(), 3)[inv]
    v = aos(parts.v.cpu().numpy(), 3)[inv]
    ex, ev = rel_l2(x, ref["x"]), rel_l2(v, ref["v"])
    ed = rel_l2(x - s["X"], ref["x"] - s["X"])
    print("3D fixed-corotated 100 steps: x %.3e v %.3e displacement %.3e" % (ex, ev, ed))
    assert flag.item() == 0
    assert ex <= 1e-3 and ev <= 1e-2 and ed <= 1e-2


def test_launch_timer_sampling(gpu):
    """mr_timing_sample: only the chosen classes, every k-th launch of each;
    the timed run's state matches an untimed run's (up to the order of the
    grid's float atomics)."""
    s = scenes.scene_3d(n=32, cube_cells=8, seed=5, v0=(0.3, -2.0, 0.1))
    st0 = scenes.initial_state(s)
    grid = _gpu_scene(B, s)
    steps, every = 25, 3
    xs = []
    for timed in (False, True):
        parts = make_parts(B, st0["x"], st0["v"], st0["C"], st0["F"], m_u=float(s["m"]),
                           V0_u=float(s["V0"]))
        gbuf = torch.zeros(grid.nodes() * 4, device=dev)
        ws = torch.zeros(B.mpm_step_workspace_bytes(grid, s["P"]), dtype=torch.uint8, device=dev)
        tm = None
        if timed:
            tm = B.Timing(256)
            tm.sample(every, ["p2g", "cell_sort"])
        B.mpm_step(grid, (s["model"], s["E"], s["nu"]), parts, s["dt"], steps, 10, 0, gbuf, ws,
                   timing=tm)
        xs.append(parts.x.cpu().numpy())
        if timed:
            r = tm.read()
            tm.close()
    # launches: one scatter per step; sorts before steps 0, 10 and 20
    assert set(r) == {"p2g", "cell_sort"}
    assert r["p2g"][0] == -(-steps // every)
    assert r["cell_sort"][0] == 1
    assert all(ms > 0 for _, ms in r.values())
    assert rel_l2(xs[1], xs[0]) < 1e-6
    with pytest.raises(B.MrError):
        B.Timing(4).sample(0)


def test_three_dimensional_full_size_one_step(gpu):
    """The 2,097,152-particle scene in the benchmark's launch configuration
    (mpm_step with cell sorting), one step against the oracle on every
    particle."""
    s = scenes.scene_3d()
    st0 = scenes.initial_state(s)
    ref = _run_oracle(oracle_scene(s), st0, s["dt"], 1)
    parts = make_parts(B, st0["x"], st0["v"], st0["C"], st0["F"], m_u=float(s["m"]), V0_u=float(s["V0"]))
    grid = _gpu_scene(B, s)
    gbuf = torch.zeros(grid.nodes() * 4, device=dev)
    ws = torch.zeros(B.mpm_step_workspace_bytes(grid, s["P"]), dtype=torch.uint8, device=dev)
    perm = torch.zeros(s["P"], dtype=torch.int32, device=dev)
    flag = torch.zeros(1, dtype=torch.int32, device=dev)
    B.mpm_step(grid, (s["model"], s["E"], s["nu"]), parts, s["dt"], 1, 10, 0, gbuf, ws,
               perm_accum=perm, status=flag)
    p = perm.cpu().numpy()
    assert np.array_equal(np.sort(p), np.arange(s["P"]))
    inv = np.empty_like(p)
    inv[p] = np.arange(len(p))
    x = aos(parts.x.cpu().numpy(), 3)[inv]
    v = aos(parts.v.cpu().numpy(), 3)[inv]
    ex, ev = rel_l2(x, ref["x"]), rel_l2(v, ref["v"])
    print("3D full one step: x %.3e v %.3e" % (ex, ev))
    assert flag.item() == 0
    assert ex <= 1e-5 and ev <= 1e-4


def test_domain_errors_are_flagged(gpu):
    rng = np.random.default_rng(60)
    x, v, C, F, m, V0 = random_state(rng, 3, 10)
    x[3] = [0.01, 0.5, 0.5]                    # stencil leaves the lattice
    F[4] = np.diag([-1.0, 1.0, 1.0])           # J < 0 under Neo-Hookean
    grid = B.Grid(3, [16] * 3, 1 / 16)
    gbuf = torch.zeros(16 ** 3 * 4, device=dev)
    flag = torch.zeros(1, dtype=torch.int32, device=dev)
    B.mpm_p2g(grid, (B.NEO_HOOKEAN, 1e4, 0.3), make_parts(B, x, v, C, F, m, V0), gbuf, 1e-4, status=flag)
    assert flag.item() & B.FLAG_DOMAIN
    keep = np.array([i for i in range(10) if i not in (3, 4)])
    mu, la = OM.lame(1e4, 0.3)
    gm, _, _ = OM.p2g(3, [16] * 3, 1 / 16, x[keep], v[keep], C[keep], F[keep], m[keep], V0[keep], 1, mu, la)
    close_channels(gbuf.cpu().numpy().reshape(-1, 4)[:, 0], gm, name="mass without bad particles")
    rc, _ = B.sync_status(flag)
    assert rc == B.MR_EDOMAIN


def test_invalid_arguments_rejected(gpu):
    rng = np.random.default_rng(61)
    x, v, C, F, m, V0 = random_state(rng, 3, 10)
    gbuf = torch.zeros(16 ** 3 * 4, device=dev)
    with pytest.raises(B.MrError) as e:
        B.mpm_p2g(B.Grid(3, [16] * 3, 1 / 16), (7, 1e4, 0.3),      # no such model
                  make_parts(B, x, v, C, F, m, V0), gbuf, 1e-4)
    assert e.value.code == B.MR_EINVAL
    with pytest.raises(B.MrError):
        B.mpm_p2g(B.Grid(3, [16] * 3, 1 / 16), (B.NEO_HOOKEAN, 1e4, 0.3),
                  make_parts(B, x, v, C, F, m, V0), gbuf, 1e-4, flags=B.SORTED)


@pytest.mark.parametrize("dim,apic", [(3, True), (2, True), (3, False)])
def test_fused_g2p2g_matches_oracle(gpu, dim, apic):
    """mpm_g2p2g = G2P from grid_in (Algorithm 1, steps 3-4) followed by P2G
    at the updated state (Algorithm 1, step 1), on sorted particles whose
    positions were then jittered by up to 1.4 cells (some beyond the drift
    margin, exercising the HBM fallbacks of both halves)."""
    rng = np.random.default_rng(70 + dim)
    n = [32] * dim
    dx = 1 / 32
    P = 12000 if dim == 3 else 3000
    x, v, C, F, m, V0 = random_state(rng, dim, P, lo=0.2, hi=0.8)
    grid = B.Grid(dim, n, dx)
    parts = make_parts(B, x, v, C, F, m, V0)
    ws = B.new_workspace(grid, P)
    perm = torch.zeros(P, dtype=torch.int32, device=dev)
    B.mpm_cell_sort(grid, parts, ws, perm_out=perm)
    p = perm.cpu().numpy()
    xs = x[p] + (rng.uniform(-1.4, 1.4, size=(P, dim)) * dx).astype(np.float32)
    parts.x.copy_(T(soa(xs)))
    gv = (0.5 * rng.standard_normal((32 ** dim, dim))).astype(np.float32)
    gin = np.zeros((32 ** dim, 4), np.float32)
    gin[:, 0] = 1.0
    gin[:, 1:1 + dim] = gv
    dt = 1e-3
    model = 0 if dim == 2 else 1
    mu, la = OM.lame(1e4, 0.3)
    xo, vo, Co, Fo = OM.g2p(dim, n, dx, dt, gv.astype(np.float64), xs, v[p], C[p], F[p], apic=apic)
    gm, gmv, gf = OM.p2g(dim, n, dx, xo, vo, Co, Fo, m[p], V0[p], model, mu, la, apic=apic)
    gout = torch.full((32 ** dim * 4,), 5.0, device=dev)
    flag = torch.zeros(1, dtype=torch.int32, device=dev)
    B.mpm_g2p2g(grid, (model, 1e4, 0.3), parts, dt, T(gin.reshape(-1)), gout, ws,
                flags=0 if apic else B.NO_AFFINE, status=flag)
    g = gout.cpu().numpy().reshape(-1, 4)
    assert flag.item() == 0
    close_channels(g[:, 0], gm, name="fused mass")
    close_channels(g[:, 1:1 + dim], gmv + dt * gf, name="fused momentum")
    np.testing.assert_allclose(aos(parts.x.cpu().numpy(), dim), xo, atol=2e-7)
    np.testing.assert_allclose(aos(parts.F.cpu().numpy(), dim, True), Fo, atol=2e-6)
    close_channels(aos(parts.v.cpu().numpy(), dim), vo, name="fused v")
    if apic:
        close_channels(aos(parts.C.cpu().numpy(), dim, True).reshape(P, -1), Co.reshape(P, -1),
                       name="fused C")


def test_empty_particle_set(gpu):
    z = torch.zeros(3, 0, device=dev)
    z9 = torch.zeros(9, 0, device=dev)
    parts = B.Particles(z, z.clone(), z9, z9.clone(), m_uniform=1.0, V0_uniform=1.0)
    gbuf = torch.full((16 ** 3 * 4,), 3.0, device=dev)
    grid = B.Grid(3, [16] * 3, 1 / 16)
    B.mpm_p2g(grid, (B.NEO_HOOKEAN, 1e4, 0.3), parts, gbuf, 1e-4)
    assert float(gbuf.abs().sum()) == 0.0
    B.mpm_g2p(grid, parts, 1e-4, gbuf)
    torch.cuda.synchronize()


def test_time_loop_captured_in_a_graph(gpu):
    """mpm_step launches only kernels and device copies, so a call can be
    captured in a graph.  Three replays from the initial state, with eager
    work (state reset, grid clear) and synchronisation between them, each
    match the eager run bit for bit (deterministic mode)."""
    s = scenes.scene_3d(n=32, cube_cells=8, seed=5, v0=(0.3, -2.0, 0.1))
    st0 = scenes.initial_state(s)
    P = s["P"]
    grid = _gpu_scene(B, s)
    mat = (s["model"], s["E"], s["nu"])

    def fresh():
        return make_parts(B, st0["x"], st0["v"], st0["C"], st0["F"], m_u=float(s["m"]),
                          V0_u=float(s["V0"]))

    gbuf = torch.zeros(grid.nodes() * 4, device=dev)
    ws = torch.zeros(B.mpm_step_workspace_bytes(grid, P), dtype=torch.uint8, device=dev)
    perm = torch.zeros(P, dtype=torch.int32, device=dev)
    eager = fresh()
    B.mpm_step(grid, mat, eager, s["dt"], 20, 10, B.DETERMINISTIC, gbuf, ws, perm_accum=perm)
    torch.cuda.synchronize()
    want = {k: getattr(eager, k).clone() for k in ("x", "v", "C", "F")}
    want_perm = perm.clone()
    static = fresh()
    init = fresh()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):       # warm-up outside the capture
        B.mpm_step(grid, mat, static, s["dt"], 1, 10, B.DETERMINISTIC, gbuf, ws, perm_accum=perm)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        B.mpm_step(grid, mat, static, s["dt"], 20, 10, B.DETERMINISTIC, gbuf, ws, perm_accum=perm)
    for rep in range(3):
        for k in ("x", "v", "C", "F"):
            getattr(static, k).copy_(getattr(init, k))
        gbuf.zero_()
        perm.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for k in ("x", "v", "C", "F"):
            assert torch.equal(getattr(static, k), want[k]), (rep, k)
        assert torch.equal(perm, want_perm), rep
