"""Pins of the FP64 encoder oracle (paper Section 4.1, Table 1) against
what its definition fixes: the layer lengths of Table 1 worked by hand,
the strided convolution as a library cross-correlation, the whole network
as a product of dense matrices, and its gradient against central finite
differences."""
import numpy as np
import pytest

from oracle import encoder as OE


def test_conv_lengths_follow_table_1():
    # 65,536 points in 3D: twelve halvings of (L - 6) / 2 + 1 down to 44;
    # one more would give 20 < 32
    assert OE.conv_lengths(196608) == [196608, 98302, 49149, 24572, 12284, 6140, 3068, 1532,
                                       764, 380, 188, 92, 44]
    assert OE.conv_lengths(80) == [80, 38]
    assert OE.conv_lengths(32) == [32]          # no convolution fits
    with pytest.raises(ValueError):
        OE.conv_lengths(31)


def test_parameter_count_matches_the_layout():
    for L, r in ((80, 3), (196608, 16), (300, 5)):
        p = np.arange(OE.param_count(L, r), dtype=np.float64)
        convs, W1, b1, W2, b2 = OE.unpack(p, L, r)
        dc = OE.conv_lengths(L)[-1]
        assert W1.shape == (32, dc) and W2.shape == (r, 32) and b2.shape == (r,)
        assert len(convs) == len(OE.conv_lengths(L)) - 1
        # first conv: weights 0..5, bias 6
        if convs:
            assert list(convs[0][0]) == [0, 1, 2, 3, 4, 5] and convs[0][1] == 6


def test_conv_is_a_strided_library_correlation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal(97)
    w = rng.standard_normal(6)
    y = OE.conv1d(x, w, 0.3)
    ref = np.correlate(x, w, mode="valid")[::2] + 0.3
    assert y.shape == ((97 - 6) // 2 + 1,)
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-13)


def test_normalisation_maps_the_box_to_minus_one_one():
    lo, hi = np.array([0.1, 0.2, 0.3]), np.array([0.5, 1.2, 0.4])
    x = np.concatenate([lo, hi, 0.5 * (lo + hi)])
    np.testing.assert_allclose(OE.normalise(x, 3, lo, hi), [-1, -1, -1, 1, 1, 1, 0, 0, 0],
                               atol=1e-14)


def _dense_forward(params, x, r, d, lo, hi):
    """The same network written with one dense matrix per convolution."""
    L = x.shape[-1]
    convs, W1, b1, W2, b2 = OE.unpack(params, L, r)
    a = OE.normalise(x, d, lo, hi)
    for (w, b) in convs:
        Lin = a.shape[-1]
        Lout = (Lin - 6) // 2 + 1
        C = np.zeros((Lout, Lin))
        for i in range(Lout):
            C[i, 2 * i:2 * i + 6] = w
        s = a @ C.T + b
        a = np.where(s > 0, s, np.exp(np.minimum(s, 0)) - 1)
    s1 = a @ W1.T + b1
    h = np.where(s1 > 0, s1, np.exp(np.minimum(s1, 0)) - 1)
    return h @ W2.T + b2


def test_forward_equals_dense_matrix_composition():
    rng = np.random.default_rng(1)
    L, r, d = 3 * 60, 4, 3
    p = OE.xavier(L, r, 2) + 0.05 * rng.standard_normal(OE.param_count(L, r))
    x = rng.uniform(0.2, 0.8, size=(5, L))
    lo, hi = np.full(3, 0.2), np.full(3, 0.8)
    z, _ = OE.forward(p, x, r, d, lo, hi)
    np.testing.assert_allclose(z, _dense_forward(p, x, r, d, lo, hi), rtol=1e-12, atol=1e-13)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    L, r, d = 3 * 40, 3, 3
    p = OE.xavier(L, r, 4) + 0.1 * rng.standard_normal(OE.param_count(L, r))
    x = rng.uniform(0.0, 1.0, size=(2, L))
    lo, hi = np.zeros(3), np.ones(3)
    dz = rng.standard_normal((2, r))
    z, cache = OE.forward(p, x, r, d, lo, hi)
    g = OE.backward(p, cache, dz, r)
    h = 1e-6
    fd = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        zp, _ = OE.forward(p + e, x, r, d, lo, hi)
        zm, _ = OE.forward(p - e, x, r, d, lo, hi)
        fd[i] = np.sum(dz * (zp - zm)) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-8)


def test_library_layout_matches_the_oracle():
    """The library's encoder layout query (host code, no GPU) gives the
    oracle's lengths and parameter count."""
    from paper_2109_12390_amd import binding as B
    for L, r in ((196608, 16), (80, 3), (3 * 1000, 8), (32 * 3 + 6, 5)):
        lens = OE.conv_lengths(L)
        if len(lens) == 1:
            continue
        nc, dc, npar, act, work = B.encoder_layout(L, r)
        assert (nc, dc, npar) == (len(lens) - 1, lens[-1], OE.param_count(L, r))
        dense = 32 * lens[-1] + 32 + 32 * r + r
        assert act == sum(lens[1:]) + 32
        assert work == 2 * lens[1] + dense + 7 * ((lens[1] + 255) // 256)
