"""Pins of the FP64 decoder oracle: central finite differences of g in X and
xhat on tiny networks, exact block Jacobians of linear decoders, and an
independent autograd evaluation (torch CPU float64)."""
import numpy as np
import pytest

from oracle import decoder as D
from paper_2109_12390_amd import scenes


def tiny_decoder(d=3, r=4, width=6, n_hidden=3, seed=0, mode=D.OUT_DISPLACEMENT):
    Ws, bs = scenes.random_decoder(d, r, width, n_hidden, seed, scale=1.5, bias_scale=0.3)
    rng = np.random.default_rng(seed + 100)
    return D.Decoder(Ws, bs, in_min=-rng.uniform(0.5, 1.0, d), in_max=rng.uniform(0.5, 1.0, d),
                     out_mean=rng.standard_normal(d) * 0.1, out_std=rng.uniform(0.5, 2.0, d),
                     output_mode=mode)


@pytest.mark.parametrize("mode", [D.OUT_DISPLACEMENT, D.OUT_POSITION])
@pytest.mark.parametrize("d,r,width,nh", [(3, 4, 6, 3), (2, 3, 4, 2), (3, 16, 8, 5)])
def test_jacobians_match_central_differences(mode, d, r, width, nh):
    dec = tiny_decoder(d, r, width, nh, seed=d * 10 + r, mode=mode)
    rng = np.random.default_rng(1)
    X = rng.uniform(-0.5, 0.5, size=(7, d))
    z = rng.standard_normal(r) * 0.5
    vh = rng.standard_normal(r)
    x, F, J, v = D.decode_jac(dec, X, z, vh)
    np.testing.assert_allclose(x, D.decode(dec, X, z), rtol=0, atol=1e-15)
    h = 1e-6
    for a in range(d):
        e = np.zeros(d); e[a] = h
        fd = (D.decode(dec, X + e, z) - D.decode(dec, X - e, z)) / (2 * h)
        np.testing.assert_allclose(F[:, :, a], fd, rtol=1e-7, atol=1e-8)
    for k in range(r):
        e = np.zeros(r); e[k] = h
        fd = (D.decode(dec, X, z + e) - D.decode(dec, X, z - e)) / (2 * h)
        np.testing.assert_allclose(J[:, :, k], fd, rtol=1e-7, atol=1e-8)
    np.testing.assert_allclose(v, np.einsum("pdr,r->pd", J, vh), atol=1e-14)


def test_linear_decoder_has_exact_block_jacobians():
    d, r = 3, 5
    rng = np.random.default_rng(2)
    W = rng.standard_normal((d, d + r)); b = rng.standard_normal(d)
    lo, hi = -np.ones(d) * 0.3, np.ones(d) * 0.7
    std = np.array([0.5, 2.0, 1.5]); mean = np.array([0.1, -0.2, 0.3])
    dec = D.Decoder([W], [b], lo, hi, mean, std)
    X = rng.uniform(0, 0.5, size=(4, d)); z = rng.standard_normal(r)
    x, F, J, _ = D.decode_jac(dec, X, z)
    Fexp = np.eye(d) + std[:, None] * W[:, :d] * (2.0 / (hi - lo))[None, :]
    Jexp = std[:, None] * W[:, d:]
    np.testing.assert_allclose(F, np.broadcast_to(Fexp, F.shape), atol=1e-14)
    np.testing.assert_allclose(J, np.broadcast_to(Jexp, J.shape), atol=1e-14)
    Xn = 2 * (X - lo) / (hi - lo) - 1
    xexp = X + mean + std * (np.concatenate([Xn, np.tile(z, (4, 1))], 1) @ W.T + b)
    np.testing.assert_allclose(x, xexp, atol=1e-14)


def test_translation_decoder():
    """g = X + xhat (r = d): F = I, J = I."""
    d = 3
    W = np.concatenate([np.zeros((d, d)), np.eye(d)], axis=1)
    dec = D.Decoder([W], [np.zeros(d)], -np.ones(d), np.ones(d), np.zeros(d), np.ones(d))
    X = np.random.default_rng(3).uniform(size=(5, d))
    z = np.array([0.1, -0.2, 0.3])
    x, F, J, v = D.decode_jac(dec, X, z, np.array([1.0, 2.0, 3.0]))
    np.testing.assert_allclose(x, X + z, atol=1e-15)
    np.testing.assert_allclose(F, np.broadcast_to(np.eye(d), F.shape), atol=0)
    np.testing.assert_allclose(J, np.broadcast_to(np.eye(d), J.shape), atol=0)
    np.testing.assert_allclose(v, np.tile([1.0, 2.0, 3.0], (5, 1)), atol=0)


def test_elu_values():
    z = np.array([-2.0, -1e-3, 0.0, 1e-3, 3.0])
    np.testing.assert_allclose(D.elu(z), [np.exp(-2) - 1, np.exp(-1e-3) - 1, 0.0, 1e-3, 3.0], rtol=1e-12)
    np.testing.assert_allclose(D.elu_prime(z), [np.exp(-2), np.exp(-1e-3), 1.0, 1.0, 1.0], rtol=1e-15)


def test_matches_torch_autograd_float64():
    torch = pytest.importorskip("torch")
    dec = tiny_decoder(3, 16, 8, 5, seed=7)
    rng = np.random.default_rng(4)
    X = rng.uniform(-0.5, 0.5, size=(3, 3))
    z = rng.standard_normal(16) * 0.3
    x, F, J, _ = D.decode_jac(dec, X, z)

    def g(Xt, zt):
        Xn = 2 * (Xt - torch.tensor(dec.in_min)) / torch.tensor(dec.in_max - dec.in_min) - 1
        h = torch.cat([Xn, zt])
        for l, (W, b) in enumerate(zip(dec.weights, dec.biases)):
            h = torch.tensor(W) @ h + torch.tensor(b)
            if l < len(dec.weights) - 1:
                h = torch.nn.functional.elu(h)
        return Xt + torch.tensor(dec.out_mean) + torch.tensor(dec.out_std) * h

    for p in range(3):
        Xt = torch.tensor(X[p]); zt = torch.tensor(z)
        JX, Jz = torch.autograd.functional.jacobian(g, (Xt, zt))
        np.testing.assert_allclose(F[p], JX.numpy(), atol=1e-12)
        np.testing.assert_allclose(J[p], Jz.numpy(), atol=1e-12)
        np.testing.assert_allclose(x[p], g(Xt, zt).numpy(), atol=1e-14)
