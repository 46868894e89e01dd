"""Decoder launch shapes and their autotuner (rom_decoder_autotune,
rom_decoder_shape): every shape evaluates the same arithmetic in the same
order per output, so a decode that runs with the point-splitting shape (large
point count) and the same points decoded through the unit-splitting shape
(small point count, or a forced choice after tuning) agree to fp32 rounding
of differently contracted sums."""
import numpy as np
import pytest

from paper_2109_12390_amd import binding as B
from paper_2109_12390_amd import scenes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
dev = "cuda"


def _dec(prec, width=128, nh=5, r=16, seed=3):
    Ws, bs = scenes.random_decoder(3, r, width, nh, seed, scale=1.0, bias_scale=0.1)
    return B.Decoder(Ws, bs, np.zeros(3, np.float32), np.ones(3, np.float32),
                     np.zeros(3, np.float32), np.full(3, 0.05, np.float32), B.OUT_DISPLACEMENT, prec)


def _decode_all(dec, X, z, vh, idx=None):
    n = X.shape[1] if idx is None else idx.numel()
    out = dict(x=torch.zeros(1, 3, n, device=dev), F=torch.zeros(1, 9, n, device=dev),
               v=torch.zeros(1, 3, n, device=dev), Jz=torch.zeros(1, 48, n, device=dev))
    B.rom_decode_jac(dec, X, z, idx=idx, vhat=vh, **out)
    xo = torch.zeros(1, 3, n, device=dev)
    B.rom_decode(dec, X, z, xo, idx=idx)
    out["x_only"] = xo
    return out


@pytest.mark.parametrize("prec", [B.PREC_FP32, B.PREC_BF16])
def test_shapes_agree_and_autotune(gpu, prec):
    rng = np.random.default_rng(7)
    n = 40000
    X = torch.tensor(rng.uniform(0, 1, size=(3, n)).astype(np.float32), device=dev)
    z = torch.tensor(0.3 * rng.standard_normal((1, 16)), device=dev)
    vh = torch.tensor(0.3 * rng.standard_normal((1, 16)), device=dev)
    dec = _dec(prec)
    # untuned size rule: units split for 2,000 points; for 40,000 points the
    # register-resident shape (bf16) or points split (fp32)
    assert dec.shape(1, 1, n) == (4 if prec == B.PREC_BF16 else 0)
    assert dec.shape(1, 1, 2000) == 3 and dec.shape(9, 1, n) == 0
    big = _decode_all(dec, X, z, vh)
    idx = torch.arange(0, n, 20, dtype=torch.int32, device=dev)
    small = _decode_all(dec, X, z, vh, idx=idx)
    worst = 0.0
    for k in big:
        a = big[k][:, :, idx.long()]
        b = small[k]
        e = float((a - b).abs().max() / (a.abs().max() + 1e-30))
        worst = max(worst, e)
    print("prec %d: point-split vs unit-split shapes, worst relative difference %.2e" % (prec, worst))
    assert worst < 1e-5
    dec.autotune(1, n, cfg_mask=7, reps=2)
    tuned = [dec.shape(c, 1, n) for c in (1, 5, 9)]
    print("tuned shapes at %d points (cfg 1, 5, 9):" % n, tuned)
    assert all(0 <= t <= 4 for t in tuned)
    again = _decode_all(dec, X, z, vh)
    for k in big:
        e = float((again[k] - big[k]).abs().max() / (big[k].abs().max() + 1e-30))
        assert e < 1e-5, k
    dec.close()


@pytest.mark.parametrize("width,nh", [(128, 5), (32, 2)])
def test_every_shape_agrees(gpu, width, nh):
    """Each shape pinned in turn (rom_decoder_set_shape) for the primal and
    the five-stream configurations of a bf16 decoder, against the first:
    the register-resident shape keeps the hidden activations in registers
    under the panel unit order, with the same arithmetic."""
    rng = np.random.default_rng(11)
    n = 20000 + 37                      # several blocks and a ragged tail
    X = torch.tensor(rng.uniform(0, 1, size=(3, n)).astype(np.float32), device=dev)
    z = torch.tensor(0.3 * rng.standard_normal((1, 16)), device=dev)
    vh = torch.tensor(0.3 * rng.standard_normal((1, 16)), device=dev)
    dec = _dec(B.PREC_BF16, width=width, nh=nh)
    outs = {}
    for shape in (0, 1, 2, 3, 4):
        dec.set_shape(1, 1, n, shape)
        if shape in (0, 3, 4):
            dec.set_shape(5, 1, n, shape)
        assert dec.shape(1, 1, n) == shape
        xo = torch.zeros(1, 3, n, device=dev)
        B.rom_decode(dec, X, z, xo)
        o = {"x_only": xo}
        if shape in (0, 3, 4):
            o.update(x=torch.zeros(1, 3, n, device=dev), F=torch.zeros(1, 9, n, device=dev),
                     v=torch.zeros(1, 3, n, device=dev))
            B.rom_decode_jac(dec, X, z, vhat=vh, x=o["x"], F=o["F"], v=o["v"])
            # x and F without v (the four-stream launch)
            o.update(x4=torch.zeros(1, 3, n, device=dev), F4=torch.zeros(1, 9, n, device=dev))
            B.rom_decode_jac(dec, X, z, x=o["x4"], F=o["F4"])
            assert torch.equal(o["F4"], o["F"]) and torch.equal(o["x4"], o["x"])
        outs[shape] = o
    worst = 0.0
    for shape, o in outs.items():
        for k, t in o.items():
            ref = outs[0][k]
            e = float((t - ref).abs().max() / (ref.abs().max() + 1e-30))
            worst = max(worst, e)
            assert e < 1e-5, (shape, k, e)
    print("width %d: all shapes against shape 0, worst relative difference %.2e" % (width, worst))
    dec.close()


def test_every_shape_agrees_in_two_dimensions(gpu):
    """The same agreement for a planar (d = 2) bf16 decoder, where the
    first layer's third input term and the third spatial tangent are zero
    (the register-resident shape sums all three terms and runs a zero
    stream)."""
    rng = np.random.default_rng(12)
    n, r = 20000 + 37, 8
    Ws, bs = scenes.random_decoder(2, r, 128, 5, 5, scale=1.0, bias_scale=0.1)
    dec = B.Decoder(Ws, bs, np.zeros(2, np.float32), np.ones(2, np.float32),
                    np.zeros(2, np.float32), np.full(2, 0.05, np.float32), B.OUT_DISPLACEMENT,
                    B.PREC_BF16)
    X = torch.tensor(rng.uniform(0, 1, size=(2, n)).astype(np.float32), device=dev)
    z = torch.tensor(0.3 * rng.standard_normal((1, r)), device=dev)
    vh = torch.tensor(0.3 * rng.standard_normal((1, r)), device=dev)
    outs = {}
    for shape in (0, 1, 2, 3, 4):
        dec.set_shape(1, 1, n, shape)
        if shape in (0, 3, 4):
            dec.set_shape(5, 1, n, shape)
        xo = torch.zeros(1, 2, n, device=dev)
        B.rom_decode(dec, X, z, xo)
        o = {"x_only": xo}
        if shape in (0, 3, 4):
            o.update(x=torch.zeros(1, 2, n, device=dev), F=torch.zeros(1, 4, n, device=dev),
                     v=torch.zeros(1, 2, n, device=dev))
            B.rom_decode_jac(dec, X, z, vhat=vh, x=o["x"], F=o["F"], v=o["v"])
        outs[shape] = o
    for shape, o in outs.items():
        for k, t in o.items():
            ref = outs[0][k]
            e = float((t - ref).abs().max() / (ref.abs().max() + 1e-30))
            assert e < 1e-5, (shape, k, e)
    dec.close()


def test_set_shape_rejects_unavailable_shapes(gpu):
    dec32 = _dec(B.PREC_FP32, width=32, nh=2, r=4)
    dec16 = _dec(B.PREC_BF16, width=32, nh=2, r=4)
    lib = B.load()
    assert lib.rom_decoder_set_shape(dec32.handle, 1, 1, 1000, 4) == B.MR_EINVAL   # fp32
    assert lib.rom_decoder_set_shape(dec16.handle, 9, 1, 1000, 4) == B.MR_EINVAL   # 9 streams
    assert lib.rom_decoder_set_shape(dec16.handle, 5, 1, 1000, 1) == B.MR_EINVAL   # primal only
    assert lib.rom_decoder_set_shape(dec16.handle, 1, 1, 1000, 5) == B.MR_EINVAL
    assert lib.rom_decoder_set_shape(dec16.handle, 1, 1, 1000, 4) == B.MR_OK
    dec32.close()
    dec16.close()


def test_autotune_rejects_bad_arguments(gpu):
    dec = _dec(B.PREC_BF16, width=32, nh=2, r=4)
    lib = B.load()
    assert lib.rom_decoder_autotune(dec.handle, 0, 100, 1, 1, None) == B.MR_EINVAL
    assert lib.rom_decoder_autotune(dec.handle, 1, 100, 8, 1, None) == B.MR_EINVAL
    assert lib.rom_decoder_autotune(dec.handle, 1, 100, 1, 0, None) == B.MR_EINVAL
    assert lib.rom_decoder_shape(dec.handle, 2, 1, 100) == B.MR_EINVAL
    dec.close()


def test_mfma_probe_runs(gpu):
    """The matrix-core probe (a measurement aid) writes finite values and
    rejects bad arguments."""
    sink = torch.zeros(4 * 256, device=dev)
    B.mfma_probe(4, 10, sink)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(sink).all()) and float(sink.abs().sum()) > 0
    lib = B.load()
    assert lib.mr_mfma_probe(0, 10, B._ptr(sink, torch.float32), None) == B.MR_EINVAL
    assert lib.mr_mfma_probe(4, 0, B._ptr(sink, torch.float32), None) == B.MR_EINVAL
