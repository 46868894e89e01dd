"""Checkpoint files round-trip bit for bit (host side; no GPU needed)."""
import numpy as np
import pytest

from paper_2109_12390_amd import binding as B
from paper_2109_12390_amd import checkpoint as CK

torch = pytest.importorskip("torch")


def test_particles_round_trip(tmp_path):
    rng = np.random.default_rng(1)
    P = 1001
    t = lambda a: torch.tensor(a.astype(np.float32))
    parts = B.Particles(t(rng.random((3, P))), t(rng.random((3, P))), t(rng.random((9, P))),
                        t(rng.random((9, P))), t(rng.random(P)), None, m_uniform=0.0,
                        V0_uniform=1.5e-7)
    label = rng.permutation(P)
    CK.save_particles(tmp_path / "p.npz", parts, 1234, label)
    q, step, lab = CK.load_particles(tmp_path / "p.npz", device="cpu")
    assert step == 1234 and np.array_equal(lab, label)
    for k in ("x", "v", "C", "F", "m"):
        assert torch.equal(getattr(q, k), getattr(parts, k)), k
    assert q.V0 is None and q.V0_uniform == np.float32(1.5e-7)


def test_latents_and_decoder_round_trip(tmp_path):
    rng = np.random.default_rng(2)
    z = torch.tensor(rng.standard_normal((4, 16)))
    CK.save_latents(tmp_path / "l.npz", z, z * 0.5, z * 2.0, 77, 2 ** 63 + 5)
    L = CK.load_latents(tmp_path / "l.npz", device="cpu")
    assert L["step"] == 77 and L["seed"] == 2 ** 63 + 5
    assert torch.equal(L["xhat"], z) and torch.equal(L["xhat_prev"], z * 0.5)
    assert torch.equal(L["vhat"], z * 2.0)
    Ws = [rng.standard_normal((8, 5)).astype(np.float32), rng.standard_normal((3, 8)).astype(np.float32)]
    bs = [rng.standard_normal(8).astype(np.float32), rng.standard_normal(3).astype(np.float32)]
    CK.save_decoder(tmp_path / "d.npz", Ws, bs, [0, 0, 0], [1, 1, 1], [0.1, 0.2, 0.3],
                    [1e-3] * 3, B.OUT_POSITION, B.PREC_BF16)
    Ws2, bs2, lo, hi, mean, std, mode, prec = CK.load_decoder_arrays(tmp_path / "d.npz")
    assert all(np.array_equal(a, b) for a, b in zip(Ws, Ws2))
    assert all(np.array_equal(a, b) for a, b in zip(bs, bs2))
    assert mode == B.OUT_POSITION and prec == B.PREC_BF16
    assert np.array_equal(mean, np.float32([0.1, 0.2, 0.3]))
    with pytest.raises(ValueError):
        CK.load_particles(tmp_path / "d.npz", device="cpu")
