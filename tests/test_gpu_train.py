"""Parity of the training kernels (rom_train_forward / backward / loss,
rom_adam_step) with the FP64 training oracle, and end-to-end training on
snapshots from the library's own full-order model.

Tolerances: fp32 mode -- the loss and every gradient entry agree with the
oracle to 1e-4 of the largest gradient magnitude of that parameter block
(fp32 products over at most a few hundred terms).  bf16 mode -- the
width x width products round both operands to bf16 (unit roundoff 2^-9,
about 2e-3); through five such layers, forward and backward, each with
128-term sums, the relative error of a whole gradient block is of order
2e-3 * sqrt(128) * (a few) ~ a few percent, so bf16 gradients are checked
by the relative Frobenius error of each block (5e-2); single entries of a
block can cancel to near zero and carry no useful relative bound."""
import numpy as np
import pytest

from oracle import decoder as OD
from oracle import train as OT
from paper_2109_12390_amd import binding as B
from paper_2109_12390_amd import scenes
from paper_2109_12390_amd import train as TR

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
dev = "cuda"


def _batch(rng, d, r, n_groups, rpg, n_snap):
    rows = n_groups * rpg
    X = rng.uniform(0.2, 0.8, size=(rows, d)).astype(np.float32)
    snap = rng.integers(0, n_snap, size=n_groups).astype(np.int32)
    nxt = np.where(snap < n_snap - 1, snap + 1, -1).astype(np.int32)
    nxt[0] = -1          # one group without a successor: velocity term dropped
    Z = (0.3 * rng.standard_normal((n_snap, r))).astype(np.float32)
    xt = (X + 0.02 * rng.standard_normal((rows, d))).astype(np.float32)
    Ft = (np.eye(d) + 0.05 * rng.standard_normal((rows, d, d))).astype(np.float32)
    vt = (0.5 * rng.standard_normal((rows, d))).astype(np.float32)
    return X, snap, nxt, Z, xt, Ft, vt


@pytest.mark.parametrize("prec", [B.PREC_FP32, B.PREC_BF16])
@pytest.mark.parametrize("d,r,width,nh", [(3, 3, 8, 2), (3, 16, 128, 5), (2, 4, 32, 3), (3, 5, 24, 2),
                                         (2, 3, 300, 1), (3, 6, 30, 2)])
def test_loss_and_gradients_match_oracle(gpu, prec, d, r, width, nh):
    rng = np.random.default_rng(width + r + prec)
    n_groups, rpg, n_snap = 3, 7, 5
    X, snap, nxt, Z, xt, Ft, vt = _batch(rng, d, r, n_groups, rpg, n_snap)
    Ws, bs = scenes.random_decoder(d, r, width, nh, 7, scale=1.0, bias_scale=0.1)
    lo, hi = np.zeros(d, np.float32), np.ones(d, np.float32)
    mean, std = np.full(d, 0.01, np.float32), np.full(d, 0.05, np.float32)
    dt, lam_F, lam_v = 0.01, 100.0, 0.01
    rows = n_groups * rpg
    tr = TR.Trainer(d, r, width, nh, prec, rows, lo, hi, mean, std)
    params = torch.tensor(B.pack_params(Ws, bs), device=dev, requires_grad=True)
    Zt = torch.tensor(Z, device=dev, requires_grad=True)
    T = lambda a, dt_=torch.float32: torch.tensor(np.ascontiguousarray(a), device=dev, dtype=dt_)
    g, G, Gv = TR.DecoderTrainFn.apply(params, Zt, T(X), T(snap, torch.int32), T(nxt, torch.int32), tr,
                                       n_groups, rpg, dt)
    loss = TR.TrainLossFn.apply(g, G, Gv, T(xt), T(Ft), T(vt), T(nxt, torch.int32), n_groups, rpg,
                                lam_F, lam_v)
    loss.backward()
    odec = OD.Decoder([w.astype(np.float64) for w in Ws], [b.astype(np.float64) for b in bs],
                      lo, hi, mean, std)
    row_snap = np.repeat(snap, rpg)
    row_nxt = np.repeat(nxt, rpg)
    L, gW, gb, gZ = OT.loss_and_grads(odec, Z, X, row_snap, row_nxt, xt, Ft, vt, dt, lam_F, lam_v)
    tol = 1e-4 if prec == B.PREC_FP32 else 5e-2
    el = abs(loss.item() - L) / abs(L)
    print("prec %d w%d: loss %.6e oracle %.6e rel %.2e" % (prec, width, loss.item(), L, el))
    assert el < tol
    flat = params.grad.cpu().numpy()
    if prec == B.PREC_FP32:
        err = lambda got, ref: np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-30)
    else:
        err = lambda got, ref: np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-30)
    o = 0
    worst = 0.0
    for l, (W, b) in enumerate(zip(gW, gb)):
        for ref in (W, b):
            got = flat[o:o + ref.size].reshape(ref.shape)
            o += ref.size
            worst = max(worst, err(got, ref))
    ez = err(Zt.grad.cpu().numpy(), gZ)
    print("  worst parameter-block gradient error %.2e, latent gradient error %.2e" % (worst, ez))
    assert worst < tol and ez < tol
    tr.close()


def test_adam_matches_oracle(gpu):
    rng = np.random.default_rng(5)
    p = rng.standard_normal(1000).astype(np.float32)
    m = np.zeros(1000, np.float32)
    v = np.zeros(1000, np.float32)
    pt, mt, vt = (torch.tensor(a, device=dev) for a in (p, m, v))
    pr, mr, vr = p.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for step in range(1, 6):
        g = rng.standard_normal(1000).astype(np.float32)
        TR.adam_step(pt, torch.tensor(g, device=dev), mt, vt, step, 1e-2)
        pr, mr, vr = OT.adam_update(pr, g.astype(np.float64), mr, vr, step, 1e-2)
    np.testing.assert_allclose(pt.cpu().numpy(), pr, rtol=1e-5, atol=1e-6)


def test_training_on_full_order_snapshots_reduces_the_loss(gpu):
    """Snapshots from the library's own full-order model (a small 3D cube,
    two parameter instances), then Adam on the decoder weights and latent
    codes with the bf16 training kernels."""
    s = scenes.scene_3d(n=32, cube_cells=8, seed=8)
    inst = [(2e4, (0.5, -1.0, 0.0)), (5e4, (-0.5, -2.0, 0.3))]
    snap = TR.generate_snapshots(s, inst, n_steps=100, every=5, n_sub=1024, seed=3)
    assert snap.n_frames == 2 * 21
    Ws, bs, Z, norm, hist = TR.train(snap, width=64, n_hidden=3, r=4, steps=400, n_groups=16,
                                     rows_per_group=64, log_every=50, lr0=1e-2, lr1=1e-4)
    print("objective on the evaluation batch", hist)
    # the same schedule in float32 torch on the CPU (oracle snapshots, torch Adam)
    # lowers this objective about 13-fold
    assert hist[-1][1] < 0.3 * hist[0][1]
    assert np.all(np.isfinite(Z))


def test_encoder_chain_gradient_matches_oracle(gpu):
    """Codes from the encoder (Section 4.1): the gradient of the training
    objective with respect to the encoder's parameters, through the decoder's
    training kernels and the encoder's backward pass (chained by autograd),
    against the oracle's loss gradient with respect to the codes pushed
    through the oracle encoder's backward pass.  fp32 kernels."""
    from oracle import encoder as OE
    rng = np.random.default_rng(77)
    d, r, width, nh = 3, 4, 32, 2
    n_groups, rpg, n_snap, P_sub = 3, 7, 5, 40
    X, snap, nxt, _, xt, Ft, vt = _batch(rng, d, r, n_groups, rpg, n_snap)
    frames = rng.uniform(0.2, 0.8, size=(n_snap, P_sub * d)).astype(np.float32)
    L_in = P_sub * d
    pe = (OE.xavier(L_in, r, 5) + 0.05 * rng.standard_normal(OE.param_count(L_in, r))).astype(np.float32)
    Ws, bs = scenes.random_decoder(d, r, width, nh, 9, scale=1.0, bias_scale=0.1)
    lo, hi = np.zeros(d, np.float32), np.ones(d, np.float32)
    mean, std = np.full(d, 0.01, np.float32), np.full(d, 0.05, np.float32)
    elo, ehi = np.full(d, 0.2, np.float32), np.full(d, 0.8, np.float32)
    dt, lam_F, lam_v = 0.01, 100.0, 0.01
    T = lambda a, dt_=torch.float32: torch.tensor(np.ascontiguousarray(a), device=dev, dtype=dt_)
    tr = TR.Trainer(d, r, width, nh, B.PREC_FP32, n_groups * rpg, lo, hi, mean, std)
    params = T(B.pack_params(Ws, bs))
    pe_t = T(pe).requires_grad_(True)
    need = np.unique(np.concatenate([snap, nxt[nxt >= 0]])).astype(np.int32)
    z = TR.EncoderFn.apply(pe_t, T(frames), T(need, torch.int32), r, d, elo, ehi)
    Zfull = torch.zeros(n_snap, r, device=dev).index_copy(0, T(need, torch.int64), z)
    g, G, Gv = TR.DecoderTrainFn.apply(params, Zfull, T(X), T(snap, torch.int32),
                                       T(nxt, torch.int32), tr, n_groups, rpg, dt)
    loss = TR.TrainLossFn.apply(g, G, Gv, T(xt), T(Ft), T(vt), T(nxt, torch.int32), n_groups, rpg,
                                lam_F, lam_v)
    loss.backward()
    zo, cache = OE.forward(pe.astype(np.float64), frames[need], r, d, elo, ehi)
    Zo = np.zeros((n_snap, r))
    Zo[need] = zo
    odec = OD.Decoder([w.astype(np.float64) for w in Ws], [b.astype(np.float64) for b in bs],
                      lo, hi, mean, std)
    L, _, _, gZ = OT.loss_and_grads(odec, Zo, X, np.repeat(snap, rpg), np.repeat(nxt, rpg), xt, Ft,
                                    vt, dt, lam_F, lam_v)
    ge = OE.backward(pe.astype(np.float64), cache, gZ[need], r)
    got = pe_t.grad.cpu().numpy()
    err = np.max(np.abs(got - ge)) / np.max(np.abs(ge))
    print("encoder chain: loss rel %.2e, gradient err %.2e of its scale"
          % (abs(loss.item() - L) / abs(L), err))
    assert abs(loss.item() - L) < 1e-4 * abs(L)
    assert err < 1e-3
    tr.close()


def test_training_with_the_encoder_reduces_the_loss(gpu):
    """The snapshots of the test above, trained with codes from the encoder
    network instead of free per-snapshot codes (bf16 decoder kernels, fp32
    encoder)."""
    s = scenes.scene_3d(n=32, cube_cells=8, seed=8)
    inst = [(2e4, (0.5, -1.0, 0.0)), (5e4, (-0.5, -2.0, 0.3))]
    snap = TR.generate_snapshots(s, inst, n_steps=100, every=5, n_sub=1024, seed=3)
    Ws, bs, Z, norm, hist, pe = TR.train(snap, width=64, n_hidden=3, r=4, steps=400, n_groups=16,
                                         rows_per_group=64, log_every=50, lr0=1e-2, lr1=1e-4,
                                         encoder=True)
    print("objective on the evaluation batch (encoder codes)", hist)
    assert hist[-1][1] < 0.3 * hist[0][1]
    assert np.all(np.isfinite(Z)) and np.all(np.isfinite(pe))
    # distinct snapshots get distinct codes
    assert np.min(np.linalg.norm(Z[1:] - Z[:-1], axis=1)) > 0.0


@pytest.mark.parametrize("prec", [B.PREC_FP32, B.PREC_BF16])
def test_reproducible_training_gradients(gpu, prec):
    """rom_trainer_set_deterministic: the gradients of a batch match the
    oracle as in the atomic mode, and two backward passes give bitwise
    identical parameter and latent gradients (several groups share
    snapshots, so the latent sums overlap)."""
    rng = np.random.default_rng(91 + prec)
    d, r, width, nh = 3, 16, 128, 5
    n_groups, rpg, n_snap = 24, 96, 5
    X, snap, nxt, Z, xt, Ft, vt = _batch(rng, d, r, n_groups, rpg, n_snap)
    Ws, bs = scenes.random_decoder(d, r, width, nh, 7, scale=1.0, bias_scale=0.1)
    lo, hi = np.zeros(d, np.float32), np.ones(d, np.float32)
    mean, std = np.full(d, 0.01, np.float32), np.full(d, 0.05, np.float32)
    dt, lam_F, lam_v = 0.01, 100.0, 0.01
    T = lambda a, dt_=torch.float32: torch.tensor(np.ascontiguousarray(a), device=dev, dtype=dt_)
    tr = TR.Trainer(d, r, width, nh, prec, n_groups * rpg, lo, hi, mean, std)
    B._check("rom_trainer_set_deterministic", B.load().rom_trainer_set_deterministic(tr.handle, 1))
    outs = []
    for rep in range(2):
        params = torch.tensor(B.pack_params(Ws, bs), device=dev, requires_grad=True)
        Zt = torch.tensor(Z, device=dev, requires_grad=True)
        g, G, Gv = TR.DecoderTrainFn.apply(params, Zt, T(X), T(snap, torch.int32),
                                           T(nxt, torch.int32), tr, n_groups, rpg, dt)
        loss = TR.TrainLossFn.apply(g, G, Gv, T(xt), T(Ft), T(vt), T(nxt, torch.int32), n_groups,
                                    rpg, lam_F, lam_v)
        loss.backward()
        outs.append((loss.item(), params.grad.cpu().numpy(), Zt.grad.cpu().numpy()))
    assert outs[0][0] == outs[1][0]
    assert np.array_equal(outs[0][1], outs[1][1]) and np.array_equal(outs[0][2], outs[1][2])
    odec = OD.Decoder([w.astype(np.float64) for w in Ws], [b.astype(np.float64) for b in bs],
                      lo, hi, mean, std)
    L, gW, gb, gZ = OT.loss_and_grads(odec, Z, X, np.repeat(snap, rpg), np.repeat(nxt, rpg), xt, Ft,
                                      vt, dt, lam_F, lam_v)
    tol = 1e-4 if prec == B.PREC_FP32 else 5e-2
    flat = outs[0][1]
    o = 0
    worst = 0.0
    for W, b in zip(gW, gb):
        for ref in (W, b):
            got = flat[o:o + ref.size].reshape(ref.shape)
            o += ref.size
            if prec == B.PREC_FP32:
                worst = max(worst, np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
            else:
                worst = max(worst, np.linalg.norm(got - ref) / np.linalg.norm(ref))
    ez = np.linalg.norm(outs[0][2] - gZ) / np.linalg.norm(gZ)
    print("reproducible mode prec %d: worst block %.2e, latent %.2e" % (prec, worst, ez))
    assert worst < tol and ez < tol
    tr.close()


def test_reproducible_training_runs_agree_bitwise(gpu):
    """Two training runs with deterministic=True (bf16 decoder kernels,
    encoder codes) end with bitwise identical parameters and codes."""
    s = scenes.scene_3d(n=32, cube_cells=8, seed=8)
    inst = [(2e4, (0.5, -1.0, 0.0)), (5e4, (-0.5, -2.0, 0.3))]
    snap = TR.generate_snapshots(s, inst, n_steps=60, every=5, n_sub=1024, seed=3)
    runs = [TR.train(snap, width=64, n_hidden=3, r=4, steps=60, n_groups=16, rows_per_group=64,
                     lr0=1e-3, lr1=1e-5, encoder=True, deterministic=True) for _ in range(2)]
    for a, b in zip(runs[0][0] + runs[0][1], runs[1][0] + runs[1][1]):
        assert np.array_equal(a, b)
    assert np.array_equal(runs[0][2], runs[1][2]) and np.array_equal(runs[0][5], runs[1][5])
