"""FP64 oracle of the encoder network (paper Section 4.1 and Table 1).

Test infrastructure only: used by tests/, never by the library.

The encoder maps the concatenated deformed positions of a fixed set of
material points (point-major: x_1, y_1, z_1, x_2, ...) to generalized
coordinates.  Table 1 fixes its shape: 1D convolutions of kernel size 6
and stride 2, as many as keep the length at or above 32 (the last length
is d_conv), then a fully connected layer d_conv -> 32 and one 32 -> r.

Readings (the paper gives kernel size and stride only): each convolution
has a single input and output channel, no padding, a bias, and an ELU
after it; the first fully connected layer has an ELU, the last none (the
decoder's activation, Section 4.1); the input coordinates are mapped by
the same per-axis min-max normalisation as the decoder's reference
positions (Appendix B feature scaling).

Parameter vector layout: for each convolution its 6 weights then its
bias; then W1 (32 x d_conv, row-major) and b1 (32); then W2 (r x 32) and
b2 (r).
"""
import numpy as np

KERNEL = 6
STRIDE = 2
MIN_LEN = 32
HIDDEN = 32


def conv_lengths(in_len):
    """Lengths after each convolution: layers are added while the next
    output length stays >= MIN_LEN (Table 1: d_conv as low as possible but
    not below 32).  Returns [in_len, L1, ..., d_conv]."""
    if in_len < MIN_LEN:
        raise ValueError("input shorter than the smallest convolution output")
    lens = [in_len]
    while True:
        nxt = (lens[-1] - KERNEL) // STRIDE + 1
        if lens[-1] < KERNEL or nxt < MIN_LEN:
            break
        lens.append(nxt)
    return lens


def param_count(in_len, r):
    nc = len(conv_lengths(in_len)) - 1
    dc = conv_lengths(in_len)[-1]
    return nc * (KERNEL + 1) + HIDDEN * dc + HIDDEN + r * HIDDEN + r


def unpack(params, in_len, r):
    """Splits the parameter vector into conv (w, b) pairs, W1, b1, W2, b2."""
    lens = conv_lengths(in_len)
    nc, dc = len(lens) - 1, lens[-1]
    p = np.asarray(params, dtype=np.float64)
    o = 0
    convs = []
    for _ in range(nc):
        convs.append((p[o:o + KERNEL], p[o + KERNEL]))
        o += KERNEL + 1
    W1 = p[o:o + HIDDEN * dc].reshape(HIDDEN, dc); o += HIDDEN * dc
    b1 = p[o:o + HIDDEN]; o += HIDDEN
    W2 = p[o:o + r * HIDDEN].reshape(r, HIDDEN); o += r * HIDDEN
    b2 = p[o:o + r]; o += r
    assert o == p.size
    return convs, W1, b1, W2, b2


def elu(s):
    return np.where(s > 0.0, s, np.expm1(np.minimum(s, 0.0)))


def elu_prime(s):
    return np.where(s > 0.0, 1.0, np.exp(np.minimum(s, 0.0)))


def conv1d(x, w, b):
    """One convolution of the encoder: y[i] = b + sum_k w[k] x[STRIDE i + k]
    over the valid outputs (a cross-correlation, as in neural networks)."""
    L = (x.shape[-1] - KERNEL) // STRIDE + 1
    y = np.full(x.shape[:-1] + (L,), b, dtype=np.float64)
    for k in range(KERNEL):
        y += w[k] * x[..., k:k + STRIDE * (L - 1) + 1:STRIDE]
    return y


def normalise(x, d, in_min, in_max):
    """Per-axis min-max map to [-1, 1] of concatenated positions (last
    axis, point-major with d coordinates per point)."""
    lo = np.asarray(in_min, np.float64)
    hi = np.asarray(in_max, np.float64)
    scale = 2.0 / (hi - lo)
    shift = -2.0 * lo / (hi - lo) - 1.0
    n = x.shape[-1] // d
    sc = np.tile(scale, n)
    sh = np.tile(shift, n)
    return np.asarray(x, np.float64) * sc + sh


def forward(params, x, r, d, in_min, in_max):
    """Encoder of a batch of concatenated position vectors x [n][in_len]:
    returns z [n][r] and the cache for `backward`."""
    x = np.atleast_2d(np.asarray(x, np.float64))
    in_len = x.shape[1]
    convs, W1, b1, W2, b2 = unpack(params, in_len, r)
    a = normalise(x, d, in_min, in_max)
    pre = []
    acts = [a]
    for (w, b) in convs:
        s = conv1d(a, w, b)
        pre.append(s)
        a = elu(s)
        acts.append(a)
    s1 = a @ W1.T + b1
    h1 = elu(s1)
    z = h1 @ W2.T + b2
    return z, (acts, pre, s1, h1)


def backward(params, cache, dz, r):
    """Gradient of sum(dz * z) with respect to the parameter vector, by the
    chain rule through the layers of `forward` (reverse order)."""
    acts, pre, s1, h1 = cache
    in_len = acts[0].shape[1]
    convs, W1, b1, W2, b2 = unpack(params, in_len, r)
    dz = np.atleast_2d(np.asarray(dz, np.float64))
    gW2 = dz.T @ h1
    gb2 = dz.sum(0)
    ds1 = (dz @ W2) * elu_prime(s1)
    gW1 = ds1.T @ acts[-1]
    gb1 = ds1.sum(0)
    da = ds1 @ W1
    gconv = []
    for li in range(len(convs) - 1, -1, -1):
        w, _ = convs[li]
        ds = da * elu_prime(pre[li])
        xin = acts[li]
        L = ds.shape[1]
        gw = np.array([np.sum(ds * xin[:, k:k + STRIDE * (L - 1) + 1:STRIDE]) for k in range(KERNEL)])
        gb = ds.sum()
        gconv.append((gw, gb))
        dx = np.zeros_like(xin)
        for k in range(KERNEL):
            dx[:, k:k + STRIDE * (L - 1) + 1:STRIDE] += w[k] * ds
        da = dx
    gconv.reverse()
    out = []
    for gw, gb in gconv:
        out.extend(gw.tolist())
        out.append(gb)
    return np.concatenate([np.asarray(out), gW1.ravel(), gb1, gW2.ravel(), gb2])


def xavier(in_len, r, seed):
    """Glorot-uniform initial parameters (Appendix B), zero biases."""
    rng = np.random.default_rng(seed)
    lens = conv_lengths(in_len)
    dc = lens[-1]
    out = []
    for _ in range(len(lens) - 1):
        a = np.sqrt(6.0 / (KERNEL + KERNEL))      # fan-in = fan-out = 6 taps
        out.extend(rng.uniform(-a, a, KERNEL).tolist())
        out.append(0.0)
    a = np.sqrt(6.0 / (dc + HIDDEN))
    out.extend(rng.uniform(-a, a, HIDDEN * dc).tolist())
    out.extend([0.0] * HIDDEN)
    a = np.sqrt(6.0 / (HIDDEN + r))
    out.extend(rng.uniform(-a, a, r * HIDDEN).tolist())
    out.extend([0.0] * r)
    return np.asarray(out)
