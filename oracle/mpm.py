"""FP64 oracle of the explicit MPM step (paper Section 2.2, Algorithm 1) and of
the sample-point dynamics (Section 3.2.3, Algorithm 5).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU
baseline leg of the benchmark, never by the product path.

The arithmetic lives in ``mpm_oracle.c`` (plain loops, double precision);
this module marshals numpy arrays to it.  Shapes (oracle convention):
positions and velocities (P, d), matrices (P, d, d), grid mass (nodes,),
grid vectors (nodes, d) with node index i + n0*(j + n1*k).
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_lp = ctypes.POINTER(ctypes.c_long)
_ip = ctypes.POINTER(ctypes.c_int)


def _load():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        lib = ctypes.CDLL(path)
        lib.orc_bspline_1d.argtypes = [ctypes.c_double, _dp, _dp]
        lib.orc_kirchhoff.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                      ctypes.c_double, _dp, _dp]
        lib.orc_kirchhoff.restype = ctypes.c_int
        lib.orc_closest_rotation.argtypes = [ctypes.c_int, _dp, _dp]
        lib.orc_closest_rotation.restype = None
        lib.orc_p2g.argtypes = [ctypes.c_int, _ip, ctypes.c_double, ctypes.c_long, _lp,
                                _dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_int,
                                ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                _dp, _dp, _dp]
        lib.orc_p2g.restype = ctypes.c_int
        lib.orc_grid_update.argtypes = [ctypes.c_int, _ip, ctypes.c_double, _dp,
                                        ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                        _dp, _dp, _dp, _dp]
        lib.orc_grid_update.restype = None
        lib.orc_g2p.argtypes = [ctypes.c_int, _ip, ctypes.c_double, ctypes.c_double,
                                ctypes.c_long, _lp, ctypes.c_int, ctypes.c_int, _dp,
                                _dp, _dp, _dp, _dp, _dp, _dp]
        lib.orc_g2p.restype = ctypes.c_int
        lib.orc_cell_keys.argtypes = [ctypes.c_int, _ip, ctypes.c_double, ctypes.c_long,
                                      _dp, _lp]
        lib.orc_cell_keys.restype = None
        lib.orc_step_threaded.argtypes = [ctypes.c_int, _ip, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_long, _dp, _dp, _dp, _dp, _dp, _dp,
                                          ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_double, ctypes.c_int]
        lib.orc_step_threaded.restype = ctypes.c_int
        _lib = lib
    return _lib


class OracleDomainError(RuntimeError):
    """A stencil left the node lattice, a NaN appeared, or J <= 0 (Neo-Hookean)."""


def _d(a):
    return a.ctypes.data_as(_dp)


def _f64(a, shape=None):
    out = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        out = out.reshape(shape)
    return out


def _ivec(n):
    arr = (ctypes.c_int * 3)(*(list(n) + [1] * (3 - len(n))))
    return arr


MODEL_FIXED_COROTATED = 0
MODEL_NEO_HOOKEAN = 1


def lame(E, nu):
    """Lame parameters (mu, lambda) of Young's modulus E and Poisson ratio nu."""
    mu = E / (2.0 * (1.0 + nu))
    la = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return mu, la


def bspline_1d(f):
    """Quadratic B-spline weights and x-derivatives (per unit dx) of the three
    nodes base..base+2 for a fractional offset f = x/dx - base in [0.5, 1.5)."""
    lib = _load()
    w = np.zeros(3)
    dw = np.zeros(3)
    lib.orc_bspline_1d(float(f), _d(w), _d(dw))
    return w, dw


def kirchhoff(dim, model, mu, la, F):
    """Kirchhoff stress tau = P F^T of one deformation gradient F (d x d)."""
    lib = _load()
    F = _f64(F, (dim, dim))
    tau = np.zeros((dim, dim))
    rc = lib.orc_kirchhoff(dim, model, mu, la, _d(F), _d(tau))
    if rc != 0:
        raise OracleDomainError("stress undefined (J <= 0 or unsupported model)")
    return tau


def closest_rotation(dim, F):
    """The rotation (det +1) closest to F in the Frobenius norm, which the
    fixed-corotated stress uses (the polar rotation when det F > 0)."""
    lib = _load()
    F = _f64(F, (dim, dim))
    R = np.zeros((dim, dim))
    lib.orc_closest_rotation(dim, _d(F), _d(R))
    return R


def num_nodes(n):
    return int(np.prod(n))


def p2g(dim, n, dx, x, v, C, F, m, V0, model, mu, la, apic=True, subset=None):
    """Particle-to-grid transfer.  Returns (m_i, m_i v_i, f^sigma_i) as arrays
    of shape (nodes,), (nodes, d), (nodes, d)."""
    lib = _load()
    P = x.shape[0]
    x = _f64(x, (P, dim)); v = _f64(v, (P, dim))
    C = _f64(C, (P, dim, dim)); F = _f64(F, (P, dim, dim))
    m = _f64(np.broadcast_to(m, (P,))); V0 = _f64(np.broadcast_to(V0, (P,)))
    nn = num_nodes(n)
    gm = np.zeros(nn); gmv = np.zeros((nn, dim)); gf = np.zeros((nn, dim))
    if subset is None:
        sub_ptr, count = None, P
    else:
        sub = np.ascontiguousarray(subset, dtype=np.int64)
        sub_ptr, count = sub.ctypes.data_as(_lp), sub.shape[0]
    rc = lib.orc_p2g(dim, _ivec(n), dx, count, sub_ptr, _d(x), _d(v), _d(C), _d(F),
                     _d(m), _d(V0), model, mu, la, int(bool(apic)),
                     _d(gm), _d(gmv), _d(gf))
    if rc != 0:
        raise OracleDomainError("p2g: particle outside the lattice or J <= 0")
    return gm, gmv, gf


def grid_update(dim, n, dt, gravity, bound, floor_mode, mu_f, gm, gmv, gf):
    """Grid velocity update with boundary band; returns v_i of shape (nodes, d)."""
    lib = _load()
    nn = num_nodes(n)
    gm = _f64(gm, (nn,)); gmv = _f64(gmv, (nn, dim)); gf = _f64(gf, (nn, dim))
    g = _f64(list(gravity) + [0.0] * (3 - len(gravity)))
    gv = np.zeros((nn, dim))
    lib.orc_grid_update(dim, _ivec(n), dt, _d(g), int(bound), int(floor_mode),
                        float(mu_f), _d(gm), _d(gmv), _d(gf), _d(gv))
    return gv


def g2p(dim, n, dx, dt, gv, x, v, C, F, apic=True, update_F=True, subset=None,
        trial=False):
    """Grid-to-particle transfer.  Full mode returns updated copies
    (x, v, C, F); trial mode returns (x_trial, v_trial) of the listed points."""
    lib = _load()
    P = x.shape[0]
    x = _f64(x, (P, dim)).copy(); v = _f64(v, (P, dim)).copy()
    C = _f64(C, (P, dim, dim)).copy(); F = _f64(F, (P, dim, dim)).copy()
    gv = _f64(gv, (num_nodes(n), dim))
    if subset is None:
        sub_ptr, count = None, P
    else:
        sub = np.ascontiguousarray(subset, dtype=np.int64)
        sub_ptr, count = sub.ctypes.data_as(_lp), sub.shape[0]
    if trial:
        tx = np.zeros((count, dim)); tv = np.zeros((count, dim))
        tx_ptr, tv_ptr = _d(tx), _d(tv)
    else:
        tx_ptr = tv_ptr = None
    rc = lib.orc_g2p(dim, _ivec(n), dx, dt, count, sub_ptr, int(bool(apic)),
                     int(bool(update_F)), _d(gv), _d(x), _d(v), _d(C), _d(F),
                     tx_ptr, tv_ptr)
    if rc != 0:
        raise OracleDomainError("g2p: particle outside the lattice")
    if trial:
        return tx, tv
    return x, v, C, F


def step(scene, state, dt, apic=True):
    """One explicit MPM step (Algorithm 1, with the affine transfer when apic).

    scene: dict with dim, n, dx, bound, floor_mode, mu_f, gravity, model, mu,
    la, m (P,) and V0 (P,).  state: dict with x, v, C, F.  Returns the new
    state dict (inputs are not modified)."""
    dim, n, dx = scene["dim"], scene["n"], scene["dx"]
    gm, gmv, gf = p2g(dim, n, dx, state["x"], state["v"], state["C"], state["F"],
                      scene["m"], scene["V0"], scene["model"], scene["mu"],
                      scene["la"], apic=apic)
    gv = grid_update(dim, n, dt, scene["gravity"], scene["bound"],
                     scene["floor_mode"], scene["mu_f"], gm, gmv, gf)
    x, v, C, F = g2p(dim, n, dx, dt, gv, state["x"], state["v"], state["C"],
                     state["F"], apic=apic)
    return {"x": x, "v": v, "C": C, "F": F}


def step_threaded(scene, state, dt, threads=0, apic=True):
    """The same step as `step`, on `threads` host threads (0: all): particle
    chunks scatter into private grids summed in thread order, then the grid
    update and a chunked gather (mpm_oracle_omp.c).  Returns the new state."""
    lib = _load()
    dim, n, dx = scene["dim"], scene["n"], scene["dx"]
    P = state["x"].shape[0]
    x = _f64(state["x"], (P, dim)).copy(); v = _f64(state["v"], (P, dim)).copy()
    C = _f64(state["C"], (P, dim, dim)).copy(); F = _f64(state["F"], (P, dim, dim)).copy()
    m = _f64(np.broadcast_to(scene["m"], (P,))); V0 = _f64(np.broadcast_to(scene["V0"], (P,)))
    g = _f64(list(scene["gravity"]) + [0.0] * (3 - len(scene["gravity"])))
    rc = lib.orc_step_threaded(dim, _ivec(n), dx, dt, P, _d(x), _d(v), _d(C), _d(F), _d(m),
                               _d(V0), scene["model"], scene["mu"], scene["la"],
                               int(bool(apic)), _d(g), int(scene["bound"]),
                               int(scene["floor_mode"]), float(scene["mu_f"]), int(threads))
    if rc == -2:
        raise MemoryError("step_threaded: private grids")
    if rc != 0:
        raise OracleDomainError("step_threaded: particle outside the lattice or J <= 0")
    return {"x": x, "v": v, "C": C, "F": F}


def cell_keys(dim, n, dx, x):
    """Linear index (i + n0*(j + n1*k)) of every particle's stencil base node;
    -1 for particles whose stencil leaves the lattice."""
    lib = _load()
    P = x.shape[0]
    x = _f64(x, (P, dim))
    keys = np.zeros(P, dtype=np.int64)
    lib.orc_cell_keys(dim, _ivec(n), dx, P, _d(x), keys.ctypes.data_as(_lp))
    return keys


def cell_sort_permutation(dim, n, dx, x):
    """Stable ordering of particles by stencil base cell: perm such that
    x[perm] is grouped by cell, ties kept in input order."""
    keys = cell_keys(dim, n, dx, x)
    return np.argsort(keys, kind="stable")
