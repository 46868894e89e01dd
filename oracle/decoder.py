"""FP64 oracle of the implicit-neural-representation decoder g(X; xhat) and
its derivatives.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU
baseline leg of the benchmark, never by the product path.

Definitions followed:
  - Kinematic restriction x = g(X; xhat) (Section 3.1, eqs. manifoldDecoder
    and kinematicRestriction).
  - Deformation gradient F = dg/dX (Section 3.1, eq. defGrad) and velocity
    v = (dg/dxhat) vhat (eq. timederOne).
  - The network is a multilayer perceptron with ELU activations on every
    hidden layer and a linear output layer (Section 4, network figure and
    architecture table); the input [X, xhat] has X min-max normalised and the
    output standardised (Appendix B, training details).
Readings: ELU with alpha = 1; X mapped to [-1, 1] per component; in
"displacement" output mode the network output is the standardised
displacement, g = X + mean + std * y, in "position" mode g = mean + std * y.

Derivatives are formed by the chain rule with explicit Jacobian matrices per
point (T_{l+1} = diag(ELU'(z_l)) W_l T_l), i.e. the definition written out,
not a tangent/adjoint scheme.
"""
import numpy as np

OUT_POSITION = "position"
OUT_DISPLACEMENT = "displacement"


class Decoder:
    """Parameters of g: weights[l] has shape (out, in), biases[l] (out,).
    The first layer takes d + r inputs, the last has d outputs; every layer
    but the last is followed by ELU."""

    def __init__(self, weights, biases, in_min, in_max, out_mean, out_std,
                 output_mode=OUT_DISPLACEMENT):
        self.weights = [np.asarray(w, dtype=np.float64) for w in weights]
        self.biases = [np.asarray(b, dtype=np.float64) for b in biases]
        self.in_min = np.asarray(in_min, dtype=np.float64)
        self.in_max = np.asarray(in_max, dtype=np.float64)
        self.out_mean = np.asarray(out_mean, dtype=np.float64)
        self.out_std = np.asarray(out_std, dtype=np.float64)
        self.output_mode = output_mode
        self.d = self.out_mean.shape[0]
        self.r = self.weights[0].shape[1] - self.d


def elu(z):
    return np.where(z > 0.0, z, np.expm1(np.minimum(z, 0.0)))


def elu_prime(z):
    return np.where(z > 0.0, 1.0, np.exp(np.minimum(z, 0.0)))


def _input(dec, X, xhat):
    Xn = 2.0 * (X - dec.in_min) / (dec.in_max - dec.in_min) - 1.0
    Z = np.broadcast_to(np.asarray(xhat, dtype=np.float64), (X.shape[0], dec.r))
    return np.concatenate([Xn, Z], axis=1)


def decode(dec, X, xhat):
    """x = g(X; xhat) for every row of X (P, d); returns (P, d)."""
    X = np.asarray(X, dtype=np.float64)
    h = _input(dec, X, xhat)
    L = len(dec.weights)
    for l in range(L):
        z = h @ dec.weights[l].T + dec.biases[l]
        h = elu(z) if l < L - 1 else z
    g = dec.out_mean + dec.out_std * h
    if dec.output_mode == OUT_DISPLACEMENT:
        g = g + X
    return g


def decode_jac(dec, X, xhat, vhat=None, chunk=1024):
    """Returns (x, F, J, v):
         x (P, d)     = g(X; xhat)
         F (P, d, d)  = dg/dX
         J (P, d, r)  = dg/dxhat
         v (P, d)     = J vhat   (None when vhat is None)."""
    X = np.asarray(X, dtype=np.float64)
    P, d, r = X.shape[0], dec.d, dec.r
    xs, Fs, Js = [], [], []
    seed = np.zeros((d + r, d + r))
    seed[:d, :d] = np.diag(2.0 / (dec.in_max - dec.in_min))
    seed[d:, d:] = np.eye(r)
    L = len(dec.weights)
    for s in range(0, P, chunk):
        Xc = X[s:s + chunk]
        h = _input(dec, Xc, xhat)
        T = np.broadcast_to(seed, (Xc.shape[0], d + r, d + r))
        for l in range(L):
            W = dec.weights[l]
            z = h @ W.T + dec.biases[l]
            Tz = np.matmul(W, T)                 # W T_l for every point
            if l < L - 1:
                h = elu(z)
                T = elu_prime(z)[:, :, None] * Tz
            else:
                h, T = z, Tz
        g = dec.out_mean + dec.out_std * h
        Jfull = dec.out_std[None, :, None] * T
        Fc = Jfull[:, :, :d].copy()
        if dec.output_mode == OUT_DISPLACEMENT:
            g = g + Xc
            Fc = Fc + np.eye(d)[None]
        xs.append(g)
        Fs.append(Fc)
        Js.append(Jfull[:, :, d:].copy())
    x = np.concatenate(xs) if xs else np.zeros((0, d))
    F = np.concatenate(Fs) if Fs else np.zeros((0, d, d))
    J = np.concatenate(Js) if Js else np.zeros((0, d, r))
    v = None
    if vhat is not None:
        v = np.einsum("pdr,r->pd", J, np.asarray(vhat, dtype=np.float64))
    return x, F, J, v


def mixed_jac(dec, X, xhat, u):
    """The mixed second derivative d/de [dg/dX (X; xhat + e u)] at e = 0,
    (P, d, d), by forward mode over forward mode: along the layers, with s
    the pre-activation, T the spatial tangents, t the tangent along u and M
    the mixed tangents, M' = elu''(s) (W T)(W t) + elu'(s) W M; elu'' is
    exp(s) for s <= 0 and 0 above (the derivative of elu' away from 0)."""
    X = np.asarray(X, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    P, d, r = X.shape[0], dec.d, dec.r
    h = _input(dec, X, xhat)
    T = np.zeros((P, d + r, d))
    T[:, :d, :] = np.diag(2.0 / (dec.in_max - dec.in_min))[None]
    t = np.zeros((P, d + r))
    t[:, d:] = u[None]
    M = np.zeros((P, d + r, d))
    L = len(dec.weights)
    for l in range(L):
        W = dec.weights[l]
        s = h @ W.T + dec.biases[l]
        WT = np.matmul(W, T)
        Wt = t @ W.T
        WM = np.matmul(W, M)
        if l < L - 1:
            e1 = elu_prime(s)
            e2 = np.where(s > 0.0, 0.0, np.exp(np.minimum(s, 0.0)))
            h = elu(s)
            M = (e2 * Wt)[:, :, None] * WT + e1[:, :, None] * WM
            T = e1[:, :, None] * WT
            t = e1 * Wt
        else:
            M = WM
    return dec.out_std[None, :, None] * M


def flatten_params(dec):
    """Pack [W_0 (row-major), b_0, W_1, b_1, ...] into one float64 vector."""
    parts = []
    for W, b in zip(dec.weights, dec.biases):
        parts.append(W.reshape(-1))
        parts.append(b.reshape(-1))
    return np.concatenate(parts)
