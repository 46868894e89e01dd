"""Resume from a checkpoint on the GPU.

Full-order: 40 deterministic steps (MR_DETERMINISTIC, sort every 10) in one
call against 20 steps, a checkpoint written and read back into fresh
tensors, and 20 more: bit-identical x, v, C, F per reference particle.
Reduced: 12 steps at once against 6 + checkpoint (latents, counter, seed,
decoder) + 6 in a new runner: the sampler resumes its stream from the
counter.  The reduced step is not bitwise reproducible across runners (its
quadrature list is collected and scattered with atomics; two fresh runners
differ by about 2e-6 in the latents here), so the bound is the one the
reduced step's parity with the oracle uses, 1e-5 of 1 + max |xhat|; a
resume from the wrong counter draws other samples and must miss it."""
import numpy as np
import pytest

from paper_2109_12390_amd import binding as B
from paper_2109_12390_amd import checkpoint as CK
from paper_2109_12390_amd import scenes
from tests.helpers import soa

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
dev = "cuda"


def _fom_parts(s):
    st = scenes.initial_state(s)
    t = lambda a: torch.tensor(soa(a), device=dev)
    return B.Particles(t(st["x"]), t(st["v"]), t(st["C"]), t(st["F"]), m_uniform=float(s["m"]),
                       V0_uniform=float(s["V0"]))


def _run(s, parts, steps, label):
    grid = B.Grid(3, s["n"], s["dx"], s["bound"], s["floor_mode"], s["mu_f"], s["gravity"])
    P = parts.n
    gbuf = torch.zeros(grid.nodes() * 4, device=dev)
    ws = torch.zeros(B.mpm_step_workspace_bytes(grid, P), dtype=torch.uint8, device=dev)
    perm = torch.zeros(P, dtype=torch.int32, device=dev)
    flag = torch.zeros(1, dtype=torch.int32, device=dev)
    B.mpm_step(grid, (s["model"], s["E"], s["nu"]), parts, s["dt"], steps, 10, B.DETERMINISTIC,
               gbuf, ws, perm_accum=perm, status=flag)
    assert flag.item() == 0
    return label[perm.cpu().numpy()]


def _by_label(parts, label):
    inv = np.empty_like(label)
    inv[label] = np.arange(len(label))
    return {k: getattr(parts, k).cpu().numpy()[:, inv] for k in ("x", "v", "C", "F")}


def test_full_order_resume_is_bitwise(gpu, tmp_path):
    s = scenes.scene_3d(n=32, cube_cells=8, seed=5, v0=(0.3, -2.0, 0.1))
    P = s["P"]
    straight = _fom_parts(s)
    lab_s = _run(s, straight, 40, np.arange(P))
    first = _fom_parts(s)
    lab = _run(s, first, 20, np.arange(P))
    CK.save_particles(tmp_path / "fom.npz", first, 20, lab)
    del first
    resumed, step, lab = CK.load_particles(tmp_path / "fom.npz")
    assert step == 20
    lab = _run(s, resumed, 20, lab)
    a, b = _by_label(straight, lab_s), _by_label(resumed, lab)
    for k in ("x", "v", "C", "F"):
        assert np.array_equal(a[k], b[k]), k


def test_reduced_order_resume(gpu, tmp_path):
    s = scenes.scene_3d(n=32, cube_cells=8, seed=6)
    d, r = 3, 8
    X = s["X"]
    Ws, bs = scenes.random_decoder(d, r, 32, 3, 51, scale=1.0, bias_scale=0.1)
    norm = (X.min(0), X.max(0), np.zeros(d, np.float32), np.full(d, 0.01, np.float32))
    CK.save_decoder(tmp_path / "dec.npz", Ws, bs, *norm)
    grid = B.Grid(3, s["n"], s["dx"], s["bound"], s["floor_mode"], s["mu_f"], s["gravity"])
    Xg = torch.tensor(soa(X), device=dev)
    E = torch.tensor([5e4], dtype=torch.float32, device=dev)
    ns = torch.tensor([24], dtype=torch.int32, device=dev)
    opts = B.gn_opts(mode=B.POS_VEL, max_iter=3)
    rng = np.random.default_rng(52)
    z0 = torch.tensor(0.2 * rng.standard_normal((1, r)), device=dev)
    v0 = torch.tensor(0.5 * rng.standard_normal((1, r)), device=dev)

    def runner(dec):
        return B.Rom(dec, grid, Xg, E, ns, opts, seed=99, rho0=1000.0, m_uniform=float(s["m"]))

    dec = B.Decoder(Ws, bs, *norm)
    rom = runner(dec)
    z, zp, vh = z0.clone(), z0.clone(), v0.clone()
    rom.step(12, 0, s["dt"], z, zp, vh, use_graph=True)
    straight = (z.clone(), vh.clone())
    z, zp, vh = z0.clone(), z0.clone(), v0.clone()
    rom.step(6, 0, s["dt"], z, zp, vh, use_graph=True)
    CK.save_latents(tmp_path / "lat.npz", z, zp, vh, 6, 99)
    mid = z.clone()
    rom.close()
    dec.close()
    dec2 = CK.load_decoder(tmp_path / "dec.npz")
    L = CK.load_latents(tmp_path / "lat.npz")
    rom2 = runner(dec2)
    rom2.step(6, L["step"], s["dt"], L["xhat"], L["xhat_prev"], L["vhat"], use_graph=True)
    zscale = 1.0 + straight[0].abs().max().item()
    dz = (L["xhat"] - straight[0]).abs().max().item() / zscale
    dv = (L["vhat"] - straight[1]).abs().max().item() / straight[1].abs().max().item()
    change = (straight[0] - mid).abs().max().item() / zscale
    print("resumed vs straight: latent err %.2e, velocity err %.2e (latent change over the last "
          "6 steps %.2e)" % (dz, dv, change))
    assert dz < 1e-5 and dv < 1e-3
    # a resume from the wrong counter draws other samples
    rom3 = runner(dec2)
    L = CK.load_latents(tmp_path / "lat.npz")
    rom3.step(6, 0, s["dt"], L["xhat"], L["xhat_prev"], L["vhat"], use_graph=True)
    wrong = (L["xhat"] - straight[0]).abs().max().item() / zscale
    print("resumed from counter 0 instead: latent err %.2e" % wrong)
    assert wrong > 1e-4
    rom2.close()
    rom3.close()
    dec2.close()
