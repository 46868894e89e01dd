"""The learned part end to end: the full-order model generates snapshots,
the decoder is trained on them with the library's training kernels, the
reduced-order model (Lagrangian quadrature, 256 sample points, position-
velocity projection) runs from the least-squares initial state, and the
full-order model judges it (displacement-relative error over the recorded
frames).  The same reduced-order run with the untrained network (the
initialisation the training starts from, same normalisation) is the method
without the learned part.

The reduced substep (Algorithm 5) transfers momentum without an affine
term, so its reference is the full-order model with the same transfers
(Algorithm 1 as printed: MR_NO_AFFINE); on this scene that model and the
APIC one differ by about 15% of the displacement, which no reduced model
of the former can close.  The error against the APIC model is printed.

Scene: a 3D Neo-Hookean cube (8^3 cells, 4,096 particles) on a 32^3 grid,
released just above the Coulomb floor with a downward and sideways
velocity, so that contact compresses and shears it within the run.
Penalty weights: the position term of this scene is ~7e-4 per particle
(rms displacement 2.7e-2), the velocity one ~2.3 (rms velocity 1.5) and
the gradient one ~6e-3; lam_F = 1 and lam_v = 1e-4 put the three on one
scale (the paper's 100 and 0.01 were chosen for its own scenes' units)."""
import numpy as np
import pytest

from paper_2109_12390_amd import binding as B
from paper_2109_12390_amd import evaluate as EV
from paper_2109_12390_amd import scenes
from paper_2109_12390_amd import train as TR

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N_STEPS, RECORD = 300, 10


def _scene(sub=2, seed=5):
    n = 32
    dx = 1.0 / n
    return scenes.make_scene(3, n, (8, 8, 8), (0.375, 3.4 * dx, 0.375), sub, 1000.0, 5.0e4, 0.3,
                             scenes.MODEL_NEO_HOOKEAN, (0.0, -9.8, 0.0), scenes.FLOOR_COULOMB,
                             0.3, 3, 1.0e-4, seed)


@pytest.fixture(scope="module")
def fom_and_training(gpu):
    s = _scene()
    E, v0 = 5.0e4, (0.4, -1.5, 0.0)
    fom = EV.fom_positions(s, E, v0, N_STEPS, RECORD, affine=False)
    fom_apic = EV.fom_positions(s, E, v0, N_STEPS, RECORD, affine=True)
    snap = TR.generate_snapshots(s, [(E, v0)], n_steps=N_STEPS, every=5, n_sub=s["P"], seed=1,
                                 affine=False)
    r, width, nh = 8, 64, 3
    Ws, bs, Z, norm, hist = TR.train(snap, width=width, n_hidden=nh, r=r, steps=4000, n_groups=16,
                                     rows_per_group=64, lr0=1e-2, lr1=1e-4, lam_F=1.0, lam_v=1e-4,
                                     log_every=1000)
    print("training objective on the evaluation batch", hist)
    init = scenes.xavier_decoder(3, r, width, nh, 0)     # what train() starts from
    # the linear-manifold baseline: one linear layer, same r, same objective
    Wl, bl, Zl, norml = TR.train_linear(snap, r, 4000, rows=1024, lam_F=1.0, lam_v=1e-4)
    # initial latent: projection of the rest configuration, started from the
    # code the training gave the first frame (zero for the untrained network)
    return (s, E, v0, (fom, fom_apic), (Ws, bs, Z[0]), init + (None,), norm,
            ((Wl, bl, Zl[0]), norml, Z, Zl))


def _rom_error(s, E, v0, foms, weights, norm, prec, n_samples=256, mode=None, **rom_kwargs):
    Ws, bs, z_guess = weights
    lo, hi, mean, std = norm
    dec = B.Decoder(Ws, bs, lo, hi, mean, std, B.OUT_DISPLACEMENT, prec)
    # a bf16 decoder's projection decodes its positions in fp32 (its own
    # positions are piecewise constant in the latents below a step's motion)
    x_rom, st = EV.rom_positions(dec, s, E, v0, N_STEPS, RECORD, n_samples=n_samples,
                                 opts=B.gn_opts(mode=B.POS_VEL if mode is None else mode,
                                                max_iter=3,
                                                proj_fp32=1 if prec == B.PREC_BF16 else 0),
                                 z_guess=z_guess, **rom_kwargs)
    dec.close()
    return [EV.displacement_error(x_rom, f, s["X"]) for f in foms], st


@pytest.mark.parametrize("prec", [B.PREC_FP32, B.PREC_BF16])
def test_trained_decoder_beats_the_untrained_one(fom_and_training, prec):
    s, E, v0, foms, trained, init, norm, _ = fom_and_training
    ((e_tr, p_tr), (e_tr_apic, _)), st_tr = _rom_error(s, E, v0, foms, trained, norm, prec)
    ((e_un, p_un), _), st_un = _rom_error(s, E, v0, foms, init, norm, prec)
    print("prec %d: displacement error trained %.3e (position %.4f%%), untrained %.3e "
          "(position %.4f%%); trained vs the APIC full-order model %.3e; quadrature points %d, "
          "active nodes %d" % (prec, e_tr, p_tr, e_un, p_un, e_tr_apic,
                               st_tr["n_quadrature_points"], st_tr["n_active_nodes"]))
    # measured: trained ~0.19-0.21 in fp32 and bf16; untrained ~1.06 (fp32)
    # and 0.54-0.72 (bf16, whose rounding perturbs the random network); training
    # on this small set is not deterministic (atomic gradient sums), so the
    # bounds leave room for its spread
    assert np.isfinite(e_tr) and np.isfinite(e_un)
    assert e_tr < 0.5 * e_un
    assert e_tr < 0.3


def test_trained_network_beats_the_linear_manifold(fom_and_training):
    """The learned nonlinear manifold against the paper's linear-manifold
    baseline (a single linear layer, no activation, same latent dimension
    and objective): the network's best approximation of the full-order
    frames (the latent fitting all particles, per frame) and its reduced
    trajectory are both better than the linear layer's; the linear
    manifold can only translate the body and apply one fixed affine map."""
    s, E, v0, foms, trained, init, norm, (lin, norml, Z, Zl) = fom_and_training
    fom = foms[0]
    Ws, bs, _ = trained
    dec = B.Decoder(Ws, bs, *norm, B.OUT_DISPLACEMENT, B.PREC_FP32)
    ldec = B.Decoder(lin[0], lin[1], *norml, B.OUT_DISPLACEMENT, B.PREC_FP32)
    # recorded every 10 steps, snapshots every 5: frame k <-> code 2k
    guess = lambda Zs: [Zs[min(2 * k, len(Zs) - 1)] for k in range(len(fom))]
    bp_nn = EV.displacement_error(EV.best_projection(dec, s, fom, guess(Z)), fom, s["X"])[0]
    bp_lin = EV.displacement_error(EV.best_projection(ldec, s, fom, guess(Zl)), fom, s["X"])[0]
    dec.close()
    ldec.close()
    ((e_nn, _), _), _ = _rom_error(s, E, v0, foms, trained, norm, B.PREC_FP32)
    ((e_lin, _), _), st = _rom_error(s, E, v0, foms, lin, norml, B.PREC_FP32)
    print("best projection: network %.3e, linear %.3e; reduced model: network %.3e, linear %.3e "
          "(status %d)" % (bp_nn, bp_lin, e_nn, e_lin, st["status"]))
    assert bp_nn < 0.5 * bp_lin
    assert not np.isfinite(e_lin) or e_nn < 0.5 * e_lin


@pytest.mark.parametrize("n_samples,mode", [(256, B.POS_VEL), (32, B.VEL_ONLY)])
def test_eulerian_quadrature_accuracy(fom_and_training, n_samples, mode):
    """The trained decoder with Eulerian quadrature (Algorithm 4: lattice
    points inverted through the decoder instead of the neighbour particles)
    against the same run with Lagrangian quadrature, both judged by the
    full-order model."""
    s, E, v0, foms, trained, init, norm, _ = fom_and_training
    ((e_eu, p_eu), _), st_eu = _rom_error(s, E, v0, foms, trained, norm, B.PREC_BF16,
                                          n_samples=n_samples, mode=mode,
                                          quadrature=B.QUAD_EULERIAN)
    ((e_la, p_la), _), st_la = _rom_error(s, E, v0, foms, trained, norm, B.PREC_BF16,
                                          n_samples=n_samples, mode=mode)
    print("samples %d mode %d: displacement error Eulerian %.3e (%d lattice points), "
          "Lagrangian %.3e (%d quadrature particles)"
          % (n_samples, mode, e_eu, st_eu["n_quadrature_points"], e_la,
             st_la["n_quadrature_points"]))
    # measured on the 2.1M-particle scene: Eulerian 0.13 vs Lagrangian 0.14
    # (512 samples), 0.18 vs 0.19 (50 samples, velocity-only)
    assert np.isfinite(e_eu)
    assert e_eu < 0.3 and e_eu < 1.5 * e_la + 0.02


@pytest.mark.parametrize("quad", [B.QUAD_LAGRANGIAN, B.QUAD_EULERIAN])
def test_zero_shot_super_resolution(fom_and_training, quad):
    """The decoder trained on the 4,096-particle set runs, unchanged, on the
    same body sampled 2x finer per dimension (32,768 particles, 4 per cell
    per dimension, a new jitter) that it never saw, and is judged against
    the full-order model run on that finer set (Section 5, zero-shot
    super-resolution: the decoder is a function of the reference position,
    so any particle set of the body can be evaluated)."""
    s, E, v0, foms, trained, init, norm, _ = fom_and_training
    fine = _scene(sub=4, seed=15)
    assert fine["P"] == 8 * s["P"]
    fom_f = EV.fom_positions(fine, E, v0, N_STEPS, RECORD, affine=False)
    [(e_f, p_f)], st_f = _rom_error(fine, E, v0, [fom_f], trained, norm, B.PREC_BF16,
                                    quadrature=quad)
    [(e_c, p_c)], st_c = _rom_error(s, E, v0, foms[:1], trained, norm, B.PREC_BF16,
                                    quadrature=quad)
    print("quadrature %d: displacement error on the 2x finer set %.3e (position %.4f%%, %d "
          "quadrature points), on the training set %.3e (%d quadrature points)"
          % (quad, e_f, p_f, st_f["n_quadrature_points"], e_c, st_c["n_quadrature_points"]))
    assert np.isfinite(e_f)
    assert e_f < 0.3 and e_f < 1.5 * e_c + 0.02


def test_batched_instances_error_distribution(gpu):
    """One decoder trained on four parameter instances (Young's modulus and
    initial velocity) of the contact scene; the four and two held-out
    instances advance together in one batched runner (rom_step, B = 6), each
    judged against its own full-order run (PIC transfers, as above)."""
    s = _scene()
    train_inst = [(5.0e4, (0.4, -1.5, 0.0)), (2.0e4, (-0.3, -1.2, 0.2)),
                  (8.0e4, (0.0, -1.8, -0.3)), (3.0e4, (0.2, -1.0, 0.3))]
    held_out = [(4.0e4, (0.1, -1.4, 0.1)), (6.0e4, (-0.2, -1.6, -0.1))]
    snap = TR.generate_snapshots(s, train_inst, n_steps=N_STEPS, every=5, n_sub=s["P"], seed=2,
                                 affine=False)
    Ws, bs, Z, norm, hist = TR.train(snap, width=64, n_hidden=3, r=8, steps=6000, n_groups=32,
                                     rows_per_group=64, lr0=1e-2, lr1=1e-4, lam_F=1.0, lam_v=1e-4,
                                     log_every=2000)
    print("training objective on the evaluation batch", hist)
    lo, hi, mean, std = norm
    dec = B.Decoder(Ws, bs, lo, hi, mean, std, B.OUT_DISPLACEMENT, B.PREC_BF16)
    inst = train_inst + held_out
    frames_per = N_STEPS // 5 + 1
    z0 = Z[0]      # initial-frame code of the first training simulation
    x_rom, info = EV.rom_positions_batched(dec, s, [e for e, _ in inst], [v for _, v in inst],
                                           N_STEPS, RECORD, n_samples=256,
                                           opts=B.gn_opts(mode=B.POS_VEL, max_iter=3),
                                           z_guesses=[Z[b * frames_per] if b < 4 else z0
                                                      for b in range(len(inst))])
    dec.close()
    errs = []
    for b, (E, v0) in enumerate(inst):
        fom = EV.fom_positions(s, E, v0, N_STEPS, RECORD, affine=False)
        errs.append(EV.displacement_error(x_rom[b], fom, s["X"])[0])
    errs = np.array(errs)
    print("batched runner (B = %d): %.3f ms per batched step, status %s" % (
        len(inst), info["ms_per_batched_step"], info["status"]))
    print("displacement error, training instances:", np.round(errs[:4], 4),
          " held-out instances:", np.round(errs[4:], 4))
    # measured: training instances 0.26-0.38, held-out 0.28-0.40 (bf16
    # decoder; status words carry MR_FLAG_LINESEARCH: some Gauss-Newton steps
    # were discarded)
    assert np.all(np.isfinite(errs))
    assert np.median(errs[:4]) < 0.5 and np.max(errs) < 1.0
