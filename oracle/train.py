"""FP64 oracle of the decoder's training objective and its gradients
(Section 4.2, loss function; Appendix B, training details).

TEST INFRASTRUCTURE ONLY.

For a batch of snapshot rows (X_p, snapshot s, targets x = phi, F = grad phi,
v = phi-dot), the objective is the batch mean of
    |g(X; z_s) - x|^2 + lam_F |dg/dX(X; z_s) - F|_F^2
                       + lam_v |dg/dz(X; z_s) (z_{s+1} - z_s)/dt - v|^2,
where z_s are per-snapshot latent codes optimised with the weights (the
alternative to the encoder that Section 4.1 describes), dt the snapshot
interval, and the velocity term is dropped for the last snapshot of a
simulation (it has no successor).  Readings: batch mean instead of the sum
(a rescaling of the learning rate); snapshot codes instead of the encoder.

The objective is written out with plain PyTorch float64 CPU operations, and
its gradients with respect to every weight, bias and latent code come from
torch.autograd on that written-out expression (the gradient of the
definition).  It is pinned in the tests by central finite differences.
"""
import numpy as np
import torch

from . import decoder as _dec


def _mlp(weights, biases, inp):
    h = inp
    L = len(weights)
    for l in range(L):
        h = h @ weights[l].T + biases[l]
        if l < L - 1:
            h = torch.nn.functional.elu(h)
    return h


def loss_terms(dec, weights, biases, Z, X, snap, nxt, x_t, F_t, v_t, dt, lam_F, lam_v):
    """Returns (total, position term, gradient term, velocity term) as 0-d
    float64 tensors, differentiable in weights, biases and Z.
    X (N, d), snap (N,) snapshot index of each row, nxt (N,) index of its
    successor snapshot or -1, targets x_t (N, d), F_t (N, d, d), v_t (N, d)."""
    d = dec.d
    X = torch.as_tensor(X, dtype=torch.float64)
    lo = torch.as_tensor(dec.in_min)
    hi = torch.as_tensor(dec.in_max)
    mean = torch.as_tensor(dec.out_mean)
    std = torch.as_tensor(dec.out_std)
    snap = torch.as_tensor(snap, dtype=torch.long)
    nxt = torch.as_tensor(nxt, dtype=torch.long)
    has_next = nxt >= 0
    z = Z[snap]
    zn = Z[torch.where(has_next, nxt, snap)]
    u = (zn - z) / dt

    def g_single(Xp, zp):
        Xn = 2.0 * (Xp - lo) / (hi - lo) - 1.0
        y = _mlp(weights, biases, torch.cat([Xn, zp]))
        out = mean + std * y
        if dec.output_mode == _dec.OUT_DISPLACEMENT:
            out = out + Xp
        return out

    N = X.shape[0]
    gs, Gs, Gvs = [], [], []
    for i in range(N):
        xi = X[i]
        zi = z[i]
        gi = g_single(xi, zi)
        # forward-mode derivatives through double-differentiable autograd
        JX = torch.autograd.functional.jacobian(lambda a: g_single(a, zi), xi, create_graph=True)
        Jz = torch.autograd.functional.jacobian(lambda b: g_single(xi, b), zi, create_graph=True)
        gs.append(gi)
        Gs.append(JX)
        Gvs.append(Jz @ u[i])
    g = torch.stack(gs)
    G = torch.stack(Gs)
    Gv = torch.stack(Gvs)
    x_t = torch.as_tensor(x_t, dtype=torch.float64)
    F_t = torch.as_tensor(F_t, dtype=torch.float64)
    v_t = torch.as_tensor(v_t, dtype=torch.float64)
    lp = ((g - x_t) ** 2).sum(1)
    lf = ((G - F_t) ** 2).sum((1, 2))
    lv = torch.where(has_next, ((Gv - v_t) ** 2).sum(1), torch.zeros(N, dtype=torch.float64))
    pos, grad, vel = lp.mean(), lf.mean(), lv.mean()
    return pos + lam_F * grad + lam_v * vel, pos, grad, vel


def loss_and_grads(dec, Z, X, snap, nxt, x_t, F_t, v_t, dt, lam_F, lam_v):
    """Objective value and its gradients: (loss, [dW_l], [db_l], dZ) as numpy
    float64 arrays."""
    Ws = [torch.tensor(W, dtype=torch.float64, requires_grad=True) for W in dec.weights]
    bs = [torch.tensor(b, dtype=torch.float64, requires_grad=True) for b in dec.biases]
    Zt = torch.tensor(np.asarray(Z, dtype=np.float64), requires_grad=True)
    total, _, _, _ = loss_terms(dec, Ws, bs, Zt, X, snap, nxt, x_t, F_t, v_t, dt, lam_F, lam_v)
    total.backward()
    return (float(total), [W.grad.numpy() for W in Ws], [b.grad.numpy() for b in bs],
            Zt.grad.numpy())


def loss_value(dec, Z, X, snap, nxt, x_t, F_t, v_t, dt, lam_F, lam_v):
    Ws = [torch.tensor(W, dtype=torch.float64) for W in dec.weights]
    bs = [torch.tensor(b, dtype=torch.float64) for b in dec.biases]
    Zt = torch.tensor(np.asarray(Z, dtype=np.float64))
    total, _, _, _ = loss_terms(dec, Ws, bs, Zt, X, snap, nxt, x_t, F_t, v_t, dt, lam_F, lam_v)
    return float(total)


def adam_update(param, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba 2015, Algorithm 1) on numpy arrays;
    returns (param, m, v).  step counts from 1."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return param - lr * mhat / (np.sqrt(vhat) + eps), m, v
