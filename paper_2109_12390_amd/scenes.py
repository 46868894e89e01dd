"""Seeded synthetic inputs shared by the HIP path's tests, the benchmark and
the oracle's tests.

This module only generates inputs (particle lattices with jitter, material
and parameter-instance draws, network initialisation); it holds none of the
method's arithmetic.  Every array is drawn in float64 with numpy's PCG64
generator and rounded to float32, so the GPU path and the oracle consume the
same values.

Scenes stand in for the paper's geometries (its cylinder, cuboid and tower
assets and their Poisson-disk particle sets are not available): blocks of
jittered particles, d-cubed sub-cells per grid cell, in the lattice order of
the cells (spatially coherent reference order).
"""
import numpy as np

MODEL_FIXED_COROTATED = 0
MODEL_NEO_HOOKEAN = 1
FLOOR_STICKY = 0
FLOOR_COULOMB = 1


def _jittered_block(rng, dim, lo, cells, dx, sub):
    """Particles on `sub` jittered sub-cells per cell per dimension, cells in
    lattice order (x fastest), sub-cells in lattice order inside each cell."""
    cells = list(cells)
    idx = np.indices(cells[::-1]).reshape(dim, -1)[::-1].T          # (ncell, dim), x fastest
    sidx = np.indices([sub] * dim).reshape(dim, -1)[::-1].T          # (nsub, dim)
    base = idx[:, None, :] * sub + sidx[None, :, :]                  # (ncell, nsub, dim)
    base = base.reshape(-1, dim).astype(np.float64)
    jit = rng.random(base.shape)
    pos = np.asarray(lo, dtype=np.float64) + (base + jit) * (dx / sub)
    return pos


def make_scene(dim, n, cells, lo, sub, rho, E, nu, model, gravity, floor_mode,
               mu_f, bound, dt, seed, v0=None):
    rng = np.random.default_rng(seed)
    dx = 1.0 / n
    X = _jittered_block(rng, dim, lo, cells, dx, sub).astype(np.float32)
    P = X.shape[0]
    V0 = np.float32(dx ** dim / sub ** dim)
    m = np.float32(rho * float(V0))
    v = np.zeros((P, dim), dtype=np.float32)
    if v0 is not None:
        v[:] = np.asarray(v0, dtype=np.float32)
    return {
        "dim": dim, "n": [n] * dim, "dx": dx, "bound": bound,
        "floor_mode": floor_mode, "mu_f": mu_f,
        "gravity": [float(g) for g in gravity], "model": model,
        "E": E, "nu": nu, "rho": rho, "dt": dt,
        "X": X, "v0": v, "m": m, "V0": V0, "P": P,
    }


def scene_2d(seed=1, literal_block=False):
    """2D full-order scene: 64 x 64 nodes (dx = 1/64), fixed-corotated block
    E = 1e4, nu = 0.3, density 1, gravity -9.8, sticky walls, 4 particles per
    cell; 4,096 particles in a 0.5 x 0.5 block (or the literal 0.25 x 0.5
    block, 2,048 particles)."""
    n = 64
    dx = 1.0 / n
    cells = (16, 32) if literal_block else (32, 32)
    lo = (0.25, 2.5 * dx)
    return make_scene(2, n, cells, lo, 2, 1.0, 1.0e4, 0.3, MODEL_FIXED_COROTATED,
                      (0.0, -9.8), FLOOR_STICKY, 0.0, 3, 1.0e-4, seed)


def scene_3d(n=128, cube_cells=64, seed=2, E=5.0e4, v0=(0.0, -1.0, 0.0), sub=2):
    """3D full-order scene: n^3 nodes (dx = 1/n), a jittered Neo-Hookean cube
    of cube_cells^3 cells with sub particles per cell per dimension (8 per
    cell, 2,097,152 at the default size; sub = 4 is the same body sampled 2x
    finer), density 1000, E = 5e4, nu = 0.3, dropped with v0 onto a Coulomb
    floor (mu = 0.3), other faces sticky, band 3 nodes, dt = 5e-5."""
    dx = 1.0 / n
    side = cube_cells * dx
    lo = (0.5 - side / 2, 5.12 * dx, 0.5 - side / 2)
    return make_scene(3, n, (cube_cells,) * 3, lo, sub, 1000.0, E, 0.3,
                      MODEL_NEO_HOOKEAN, (0.0, -9.8, 0.0), FLOOR_COULOMB, 0.3, 3,
                      5.0e-5, seed, v0=v0)


def initial_state(scene):
    """x = X, v = v0, C = 0, F = I as float32 arrays (oracle convention
    shapes (P, d), (P, d, d))."""
    P, dim = scene["P"], scene["dim"]
    return {
        "x": scene["X"].copy(),
        "v": scene["v0"].copy(),
        "C": np.zeros((P, dim, dim), dtype=np.float32),
        "F": np.tile(np.eye(dim, dtype=np.float32), (P, 1, 1)),
    }


def parameter_instances(n_inst, seed, E_range=(1.0e3, 1.0e5), v_range=2.0, dim=3):
    """Young's moduli (log-uniform in E_range) and initial velocities
    (uniform in [-v_range, v_range]^d) for n_inst parameter instances."""
    rng = np.random.default_rng(seed)
    logE = rng.uniform(np.log(E_range[0]), np.log(E_range[1]), size=n_inst)
    E = np.exp(logE)
    v0 = rng.uniform(-v_range, v_range, size=(n_inst, dim))
    return E, v0


def xavier_decoder(d, r, width, n_hidden, seed):
    """Glorot-uniform weights (gain 1) and zero biases for an MLP
    (d + r) -> width x n_hidden -> d; returns lists of float32 arrays,
    weights shaped (out, in)."""
    rng = np.random.default_rng(seed)
    sizes = [d + r] + [width] * n_hidden + [d]
    Ws, bs = [], []
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        a = np.sqrt(6.0 / (fi + fo))
        Ws.append(rng.uniform(-a, a, size=(fo, fi)).astype(np.float32))
        bs.append(np.zeros(fo, dtype=np.float32))
    return Ws, bs


def random_decoder(d, r, width, n_hidden, seed, scale=1.0, bias_scale=0.1):
    """A random (untrained) MLP with non-zero biases, for derivative and
    parity tests."""
    rng = np.random.default_rng(seed)
    sizes = [d + r] + [width] * n_hidden + [d]
    Ws, bs = [], []
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        a = scale * np.sqrt(6.0 / (fi + fo))
        Ws.append(rng.uniform(-a, a, size=(fo, fi)).astype(np.float32))
        bs.append((bias_scale * rng.standard_normal(fo)).astype(np.float32))
    return Ws, bs
