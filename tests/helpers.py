"""Shared test utilities: layout conversions between the oracle's
array-of-structs convention and the library's structure-of-arrays device
layout, and scene descriptors for both sides.  Holds none of the method's
arithmetic."""
import numpy as np

from oracle import mpm as OM


def soa(a):
    """(P, d) or (P, d, d) -> (d, P) or (d*d, P) float32."""
    a = np.asarray(a)
    P = a.shape[0]
    k = int(np.prod(a.shape[1:]))
    return np.ascontiguousarray(a.reshape(P, k).T.astype(np.float32))


def aos(a, dim, mat=False):
    """(d, P) or (d*d, P) -> (P, d) or (P, d, d) float64."""
    a = np.asarray(a, dtype=np.float64)
    P = a.shape[-1]
    out = a.reshape(-1, P).T
    return out.reshape(P, dim, dim) if mat else out.reshape(P, dim)


def oracle_scene(s, P=None):
    """Oracle scene dict (float64 masses) from a scenes.make_scene dict."""
    P = s["P"] if P is None else P
    mu, la = OM.lame(s["E"], s["nu"])
    return dict(dim=s["dim"], n=s["n"], dx=s["dx"], bound=s["bound"],
                floor_mode=s["floor_mode"], mu_f=s["mu_f"], gravity=s["gravity"],
                model=s["model"], mu=mu, la=la,
                m=np.full(P, float(np.float32(s["m"]))), V0=np.full(P, float(np.float32(s["V0"]))))


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def tile_slot_order(dim, n, dx, x):
    """Expected cell-sort permutation: particles grouped by tile of stencil
    base cells (4^3 cells in 3D, 8^2 in 2D, tiles and cells x-fastest),
    inside a tile ordered by rank within their cell (previous order), then
    by cell.  Written from the layout the library documents; particles
    outside the lattice go last in input order."""
    TS = 4 if dim == 3 else 8
    base = np.floor(np.asarray(x, dtype=np.float64) / dx - 0.5).astype(np.int64)
    n = np.asarray(n)
    nt = -(-(n - 2) // TS)
    ok = np.all((base >= 0) & (base + 2 <= n - 1), axis=1)
    t = base // TS
    c = base % TS
    tile = t[:, 0] + nt[0] * (t[:, 1] + (nt[1] * t[:, 2] if dim == 3 else 0))
    cell = c[:, 0] + TS * (c[:, 1] + (TS * c[:, 2] if dim == 3 else 0))
    key = tile * 64 + cell
    ntiles = int(np.prod(nt))
    key = np.where(ok, key, ntiles * 64)
    P = len(key)
    order = np.argsort(key, kind="stable")
    rank = np.zeros(P, dtype=np.int64)
    sk = key[order]
    start = 0
    for i in range(1, P + 1):
        if i == P or sk[i] != sk[start]:
            rank[order[start:i]] = np.arange(i - start)
            start = i
    big = np.where(ok, 0, 1)
    return np.lexsort((np.where(ok, cell, np.arange(P)), np.where(ok, rank, 0), np.where(ok, tile, 0), big))
