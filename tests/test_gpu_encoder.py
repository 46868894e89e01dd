"""Parity of the HIP encoder (rom_encoder_forward / rom_encoder_backward,
Section 4.1, Table 1) with the FP64 oracle.

Tolerance: every output is a chain of fp32 sums of at most 6 (convolutions)
or 67 (dense) products through at most 13 layers, so the relative error is
a few units of 2^-24 times the depth and the fan-in; 1e-4 of the output
scale is a wide bound.  The weight gradients are sums over frames and up
to 10^5 outputs per layer, added with fp32 atomics in blocks of 256: their
error grows with the square root of the count, and 1e-3 of each parameter
block's largest gradient bounds it."""
import numpy as np
import pytest

from oracle import encoder as OE
from paper_2109_12390_amd import binding as B

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
dev = "cuda"


def _case(L, r, n_frames, pick, seed):
    rng = np.random.default_rng(seed)
    d = 3
    lo, hi = np.array([0.2, 0.1, 0.3]), np.array([0.8, 0.9, 0.6])
    X = rng.uniform(lo, hi, size=(n_frames, L // d, d)).reshape(n_frames, L)
    p = OE.xavier(L, r, seed + 1) + 0.05 * rng.standard_normal(OE.param_count(L, r))
    idx = np.asarray(pick, dtype=np.int32)
    dz = rng.standard_normal((len(idx), r))
    return d, X, p.astype(np.float32), idx, dz, lo.astype(np.float32), hi.astype(np.float32)


def _run(d, r, X, p, idx, dz, lo, hi, deterministic=False):
    L = X.shape[1]
    nc, dc, npar, actf, workf = B.encoder_layout(L, r)
    n = len(idx)
    x = torch.tensor(X.astype(np.float32), device=dev)
    pt = torch.tensor(p, device=dev)
    it = torch.tensor(idx, device=dev)
    act = torch.zeros(n, actf, device=dev)
    z = torch.zeros(n, r, device=dev)
    B.encoder_forward(d, r, x, pt, lo, hi, act, z, frame_idx=it)
    g = torch.zeros(npar, device=dev)
    work = torch.zeros(n, workf, device=dev)
    B.encoder_backward(d, r, x, pt, lo, hi, act, torch.tensor(dz.astype(np.float32), device=dev),
                       g, work, frame_idx=it, deterministic=deterministic)
    torch.cuda.synchronize()
    return z.cpu().numpy(), g.cpu().numpy()


def _blocks(L, r):
    """Parameter index ranges: each convolution, W1, b1, W2, b2."""
    lens = OE.conv_lengths(L)
    out, o = [], 0
    for _ in range(len(lens) - 1):
        out.append((o, o + 7))
        o += 7
    for n in (32 * lens[-1], 32, r * 32, r):
        out.append((o, o + n))
        o += n
    return out


@pytest.mark.parametrize("L,r,n_frames,pick", [
    (78, 3, 3, [2, 0]),                     # one convolution
    (3 * 4000, 16, 6, [5, 1, 3, 3]),        # nine convolutions, a repeated frame
    (3 * 65536, 16, 4, [0, 1, 2, 3]),       # the training snapshots' length
])
def test_encoder_matches_oracle(gpu, L, r, n_frames, pick):
    d, X, p, idx, dz, lo, hi = _case(L, r, n_frames, pick, 40 + L % 97)
    z, g = _run(d, r, X, p, idx, dz, lo, hi)
    zr, cache = OE.forward(p.astype(np.float64), X[idx], r, d, lo, hi)
    gr = OE.backward(p.astype(np.float64), cache, dz, r)
    ez = np.max(np.abs(z - zr)) / np.max(np.abs(zr))
    print("L %d: %d convolutions, z err %.2e of scale" % (L, len(OE.conv_lengths(L)) - 1, ez))
    assert ez < 1e-4
    for (a, b) in _blocks(L, r):
        sc = np.max(np.abs(gr[a:b]))
        eg = np.max(np.abs(g[a:b] - gr[a:b])) / sc
        assert eg < 1e-3, (a, b, eg)


def test_encoder_rejects_bad_sizes(gpu):
    x = torch.zeros(2, 90, device=dev)
    p = torch.zeros(2000, device=dev)
    act = torch.zeros(2, 200, device=dev)
    z = torch.zeros(2, 3, device=dev)
    with pytest.raises(B.MrError):           # in_len not a multiple of d
        B.encoder_forward(3, 3, torch.zeros(2, 91, device=dev), p, [0] * 3, [1] * 3, act, z)
    with pytest.raises(B.MrError):           # d outside 2..3
        B.encoder_forward(4, 3, torch.zeros(2, 92, device=dev), p, [0] * 4, [1] * 4, act, z)
    with pytest.raises(B.MrError):           # shorter than 32
        B.encoder_forward(3, 3, torch.zeros(2, 30, device=dev), p, [0] * 3, [1] * 3, act, z)
    with pytest.raises(B.MrError):           # empty box
        B.encoder_forward(3, 3, x, p, [0] * 3, [0] * 3, act, z)


def test_encoder_backward_reproducible_mode(gpu):
    """deterministic = 1: the gradient matches the oracle like the atomic
    mode and two calls agree bit for bit (the training snapshots' length)."""
    L, r = 3 * 65536, 16
    d, X, p, idx, dz, lo, hi = _case(L, r, 5, [4, 0, 2, 1, 3], 61)
    z1, g1 = _run(d, r, X, p, idx, dz, lo, hi, deterministic=True)
    z2, g2 = _run(d, r, X, p, idx, dz, lo, hi, deterministic=True)
    assert np.array_equal(g1, g2) and np.array_equal(z1, z2)
    zr, cache = OE.forward(p.astype(np.float64), X[idx], r, d, lo, hi)
    gr = OE.backward(p.astype(np.float64), cache, dz, r)
    for (a, b) in _blocks(L, r):
        eg = np.max(np.abs(g1[a:b] - gr[a:b])) / np.max(np.abs(gr[a:b]))
        assert eg < 1e-3, (a, b, eg)
