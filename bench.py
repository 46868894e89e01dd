"""Benchmark of the full-order MPM step on the 3D scene: 128^3 nodes,
2,097,152 particles (8 per cell) in a jittered Neo-Hookean cube (E = 5e4,
nu = 0.3, density 1000) dropped onto a Coulomb floor (mu = 0.3), dt = 5e-5,
particles cell-sorted every 10 steps.  Synthetic, seeded input.

The timed region is one mpm_step call (C ABI) advancing K steps: a cell
sort every 10th step followed by P2G (sorted, LDS-tiled), and in between the
fused gather-of-step-n / scatter-of-step-n+1 kernel, each followed by the
grid update.  HIP events bracket the whole region; the library's launch
timer records an event pair around every launch inside it on the same
stream, which gives the per-kernel average durations of the roofline entry.
The JSON line also carries the reduced-order step on the same scene: its
throughput with one instance and with 256 instances in one graph (random
decoder of the benchmarked shape), and a trained decoder's reduced model
judged against the full-order model over 500 steps.
Prints one JSON line on stdout.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-rom]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_BF16_PEAK_TFLOPS = 2500.0     # dense bf16 matrix cores, nominal
SORT_EVERY = 10
# launch-timer sampling interval: coprime with SORT_EVERY, so the sampled
# scatters cover every number of steps since the last sort (the scatter
# slows by ~20% over the ten steps as particles drift from their sorted
# cells; a multiple of the sort interval would sample one phase only)
TIMING_EVERY = 7


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("mpm.hip", "mpm_kernels.h", "internal.h"):
        with open(os.path.join(ROOT, "paper_2109_12390_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, src_hash):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    only if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        return None
    ent = data.get(kernel)
    if not ent or ent.get("source_hash") != src_hash:
        return None
    return ent.get("bytes_per_launch")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(scene, steps_single=2, steps_threaded=6):
    """The FP64 oracle on the same full-size scene: the threaded driver
    (private grids summed in thread order) on the host's threads -- the
    baseline value -- and the plain single-threaded loop beside it.  The
    thread count is OMP_NUM_THREADS when set (the host's share of cores),
    else every core."""
    from oracle import mpm as OM
    st0 = {k: v.astype(np.float64) for k, v in __import__(
        "paper_2109_12390_amd.scenes", fromlist=["x"]).initial_state(scene).items()}
    mu, la = OM.lame(scene["E"], scene["nu"])
    sc = dict(dim=3, n=scene["n"], dx=scene["dx"], bound=scene["bound"],
              floor_mode=scene["floor_mode"], mu_f=scene["mu_f"], gravity=scene["gravity"],
              model=scene["model"], mu=mu, la=la,
              m=np.full(scene["P"], float(scene["m"])), V0=np.full(scene["P"], float(scene["V0"])))
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    st = OM.step_threaded(sc, st0, scene["dt"], threads=threads)    # warm-up (loads the oracle)
    t0 = time.perf_counter()
    for _ in range(steps_threaded):
        st = OM.step_threaded(sc, st, scene["dt"], threads=threads)
    el_t = time.perf_counter() - t0
    st = st0
    t0 = time.perf_counter()
    for _ in range(steps_single):
        st = OM.step(sc, st, scene["dt"])
    el_1 = time.perf_counter() - t0
    return {"value": scene["P"] * steps_threaded / el_t, "unit": "particle-steps/s",
            "cores": threads, "kind": "oracle",
            "sample": "%d steps of the full %d-particle scene, FP64, %d threads (OpenMP driver: "
                      "private grids summed in thread order)" % (steps_threaded, scene["P"], threads),
            "single_thread": {"value": scene["P"] * steps_single / el_1, "cores": 1,
                              "sample": "%d steps, plain loop" % steps_single},
            "host": {"nproc": os.cpu_count(), "cpu_model": cpu_model()}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-rom", action="store_true")
    ap.add_argument("--no-fcr", action="store_true",
                    help="skip the fixed-corotated variant of the full-order scene")
    ap.add_argument("--rom-steps", type=int, default=100)
    ap.add_argument("--rom-instances", type=int, default=256)
    ap.add_argument("--rom-accuracy-steps", type=int, default=500,
                    help="steps of the trained reduced model judged against the full-order "
                         "model (0: skip)")
    ap.add_argument("--train-steps", type=int, default=4000)
    ap.add_argument("--rom-batched-steps", type=int, default=4)
    ap.add_argument("--rom-batched-error-steps", type=int, default=100,
                    help="steps of the batched reduced model (decoder trained with the encoder "
                         "on 8 instances) judged per instance against the full-order model "
                         "(0: skip)")
    ap.add_argument("--rom-study", action="store_true",
                    help="the reduced model's error attribution and sample-count sweep with a "
                         "trained decoder (adds a few minutes)")
    ap.add_argument("--batched-study", action="store_true",
                    help="train on several instances, then judge every instance of the batched "
                         "reduced model against its own full-order run (adds several minutes)")
    ap.add_argument("--batched-study-instances", type=int, default=256)
    ap.add_argument("--batched-study-steps", type=int, default=400)
    ap.add_argument("--batched-study-train-steps", type=int, default=8000)
    ap.add_argument("--batched-study-codes", default="encoder", choices=("encoder", "free"))
    ap.add_argument("--batched-study-quadratures", default="lagrangian,eulerian")
    ap.add_argument("--rom-pareto-steps", type=int, default=30,
                    help="steps per point of the quadrature / samples / projection sweep (0: off)")
    ap.add_argument("--decoder-profile", action="store_true",
                    help="only run the reduced step's two decoder launches (positions of every "
                         "particle; x, F, v at a quadrature-sized subset), for counter runs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 256 MiB ten times (the reference "
                         "kernel that scales the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2109_12390_amd import binding as B
    from paper_2109_12390_amd import scenes

    if args.copy_calibration:
        a = torch.ones(64 << 20, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(10):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": b.numel() * 4,
                          "launches": 10}), flush=True)
        return
    B.load()
    dev = "cuda:0"
    s = scenes.scene_3d()
    P = s["P"]
    if args.decoder_profile:
        print(json.dumps(decoder_profile(B, scenes, s)), flush=True)
        return
    st = scenes.initial_state(s)
    soa = lambda a: torch.tensor(np.ascontiguousarray(a.reshape(P, -1).T), device=dev)
    parts = B.Particles(soa(st["x"]), soa(st["v"]), soa(st["C"]), soa(st["F"]),
                        m_uniform=float(s["m"]), V0_uniform=float(s["V0"]))
    grid = B.Grid(3, s["n"], s["dx"], s["bound"], s["floor_mode"], s["mu_f"], s["gravity"])
    gbuf = torch.zeros(grid.nodes() * 4, device=dev)
    ws = torch.zeros(B.mpm_step_workspace_bytes(grid, P), dtype=torch.uint8, device=dev)
    flag = torch.zeros(1, dtype=torch.int32, device=dev)
    mat = (s["model"], s["E"], s["nu"])
    dt = s["dt"]

    timing = B.Timing(capacity=16 * (args.steps + 8))
    # one launch in TIMING_EVERY of each kernel class is bracketed by HIP
    # events on the launch stream (an event pair costs a few microseconds of
    # stream time, 6% of the step when every launch is timed)
    timing.sample(TIMING_EVERY)
    # untimed warm-up: compiles nothing, but brings the caches, the
    # allocator and the clocks to steady state
    B.mpm_step(grid, mat, parts, dt, args.warmup, SORT_EVERY, 0, gbuf, ws, status=flag)
    torch.cuda.synchronize()
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    t_start.record()
    B.mpm_step(grid, mat, parts, dt, args.steps, SORT_EVERY, 0, gbuf, ws, status=flag, timing=timing)
    t_end.record()
    torch.cuda.synchronize()
    total_ms = t_start.elapsed_time(t_end)
    rc, fl = B.sync_status(flag)
    if rc != 0:
        log("status flags raised during the run:", fl)
    # launches of each class in the run (the loop of mpm_step: a sort before
    # step 0 and every SORT_EVERY steps, one scatter, grid update and gather
    # per step)
    run_launches = {"cell_sort": 1 + (args.steps - 1) // SORT_EVERY, "p2g": args.steps,
                    "grid_update": args.steps, "g2p": args.steps}
    per_kernel = {k: {"timed_launches": n, "avg_ms": ms / n,
                      "run_ms": ms / n * run_launches.get(k, n)}
                  for k, (n, ms) in timing.read().items()}
    log("per-kernel:", json.dumps(per_kernel))

    # algorithmic bytes per launch (float32 particle state; the grid region
    # touched is measured from the node masses of one more scatter of the
    # final state, outside the timed region: the grid buffers' contents after
    # mpm_step are unspecified)
    B.mpm_p2g(grid, mat, parts, gbuf, dt)
    g = gbuf.view(-1, 4)
    active_nodes = int((g[:, 0] > 0).sum().item())
    grid_bytes = 16 * active_nodes
    algo = {
        "g2p2g": 96 * P + 2 * grid_bytes,           # read and write x, F; read and flush the touched nodes
        "p2g": 96 * P + grid_bytes,                 # read x, v, C, F; flush the touched nodes
        "g2p": 48 * P + grid_bytes + 96 * P,        # read x, F and the grid; write x, v, C, F
        "grid_update": 48 * grid.nodes(),           # read and write every node, clear the other grid
        "zero_grid": 16 * grid.nodes(),             # clear the second grid
        "cell_sort": (2 * 96 + 16) * P,             # gather-permute the state, keys and indices
    }
    dom = max(per_kernel, key=lambda k: per_kernel[k]["run_ms"])
    achieved = algo[dom] / (per_kernel[dom]["avg_ms"] * 1e-3) / 1e9
    src_hash = kernel_source_hash()
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(dom, src_hash),
                "algorithmic_bytes_per_launch": algo[dom]}
    ms_per_step = total_ms / args.steps
    value = P * args.steps / (total_ms * 1e-3)
    out = {
        "metric": "MPM particle-steps/s",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "3D full-order MPM, 128^3 grid, 2,097,152 particles, Neo-Hookean "
                               "cube on a Coulomb floor, dt 5e-5, cell sort every 10 steps",
                   "particles": P, "grid": s["n"], "sort_every": SORT_EVERY},
        "roofline": roofline,
        "per_kernel_ms": {k: round(v["avg_ms"], 5) for k, v in per_kernel.items()},
        "active_nodes": active_nodes,
        "kernel_source_hash": src_hash,
    }
    peaks = measured_peaks(B)
    out["peaks_measured"] = peaks
    roofline["measured_peak"] = peaks["hbm_copy_GBps"]
    roofline["frac_measured"] = round(achieved / peaks["hbm_copy_GBps"], 4)
    log("measured peaks:", json.dumps(peaks))
    if not args.no_fcr:
        out["fixed_corotated"] = fom_fixed_corotated(B, scenes, s, min(args.steps, 200),
                                                     args.warmup)
        log("fixed-corotated:", json.dumps(out["fixed_corotated"]))
        out["two_dimensional"] = fom_two_dimensional(B, scenes)
        log("2D:", json.dumps(out["two_dimensional"]))
    if not args.no_rom:
        out["rom"] = rom_throughput(B, scenes, s, args.rom_steps, peaks=peaks)
        log("decoder roofline:", json.dumps(out["rom"]["decoder_roofline"]))
        if args.rom_pareto_steps > 0:
            out["rom_pareto"] = rom_pareto(B, scenes, s, args.rom_pareto_steps)
        if args.rom_instances > 0:
            out["rom_batched"] = rom_batched_throughput(B, scenes, s, args.rom_instances,
                                                        args.rom_batched_steps)
            if args.rom_batched_error_steps > 0:
                log("batched instances judged against their own full-order runs ...")
                out["rom_batched"]["error_vs_full_order"] = batched_study(
                    B, scenes, s, n_inst=args.rom_instances, n_steps=args.rom_batched_error_steps,
                    train_steps=8000, codes="encoder", quadratures=("lagrangian",),
                    trainings=("bf16_encoder",))
        if args.rom_accuracy_steps > 0:
            log("training a decoder on full-order snapshots and judging the reduced model ...")
            out["rom_trained"] = rom_trained_accuracy(B, scenes, s, args.rom_accuracy_steps,
                                                      args.train_steps)
            if out["rom_trained"]["status"]:
                log("the trained reduced run raised status flags:",
                    out["rom_trained"]["status_flags"])
    if args.rom_study:
        log("reduced-model study ...")
        out["rom_study"] = rom_study(B, scenes, s)
    if args.batched_study:
        log("batched reduced-model study ...")
        out["batched_study"] = batched_study(B, scenes, s, n_inst=args.batched_study_instances,
                                             n_steps=args.batched_study_steps,
                                             train_steps=args.batched_study_train_steps,
                                             codes=args.batched_study_codes,
                                             quadratures=args.batched_study_quadratures.split(","))
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host ...")
        out["cpu_baseline"] = cpu_baseline(s)
    print(json.dumps(out), flush=True)


def measured_peaks(B):
    """What this GPU sustains, beside the nominal peaks: a plain 1 GiB
    device-to-device copy (bytes read + written per second, best of 5) and
    the dense bf16 matrix-core loop of mr_mfma_probe (2,048 workgroups)."""
    import torch
    dev = "cuda:0"
    a = torch.ones(256 << 20, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    best = None
    for _ in range(5):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    hbm = 2 * a.numel() * 4 / (best * 1e-3) / 1e9
    del a, b
    blocks, iters = 2048, 20000
    sink = torch.empty(blocks * 256, device=dev)
    B.mfma_probe(blocks, 100, sink)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    B.mfma_probe(blocks, iters, sink)
    e1.record()
    torch.cuda.synchronize()
    flop = blocks * 4 * iters * 8 * 16384
    mfma = flop / (e0.elapsed_time(e1) * 1e-3) / 1e12
    return {"hbm_copy_GBps": round(hbm, 1), "mfma_bf16_TFLOPs": round(mfma, 1)}


def decoder_profile(B, scenes, s, reps=10, n_tan=435_200, r=16, width=128, n_hidden=5):
    """The reduced step's two decoder launches alone (bf16, random weights),
    each repeated `reps` times: the positions of every particle of the 3D
    scene (one primal stream) and x, F and v (the primal and four tangent
    streams) at a quadrature-sized subset of it.  Reports the time per launch
    and the hidden layers' matrix-core FLOP, which the bf16 MFMA counters
    (512 FLOP per MOPS unit) should reproduce."""
    import torch
    dev = "cuda:0"
    X = s["X"]
    P = s["P"]
    Ws, bs = scenes.xavier_decoder(3, r, width, n_hidden, 11)
    dec = B.Decoder(Ws, bs, X.min(0), X.max(0), np.zeros(3, np.float32),
                    np.full(3, 1e-3, np.float32), B.OUT_DISPLACEMENT, B.PREC_BF16)
    Xg = torch.tensor(np.ascontiguousarray(X.T), device=dev)
    rng = np.random.default_rng(5)
    z = torch.tensor(rng.uniform(-0.5, 0.5, (1, r)), device=dev)
    vh = torch.tensor(rng.uniform(-0.5, 0.5, (1, r)), device=dev)
    idx = torch.tensor(np.sort(rng.choice(P, n_tan, replace=False)).astype(np.int32), device=dev)
    xo = torch.empty(1, 3, P, device=dev)
    xt = torch.empty(1, 3, n_tan, device=dev)
    Ft = torch.empty(1, 9, n_tan, device=dev)
    vt = torch.empty(1, 3, n_tan, device=dev)
    hidden_flop = 2 * (n_hidden - 1) * width * width
    out = {"decoder": "%d x %d bf16, r = %d" % (width, n_hidden, r), "reps": reps}
    for name, run, n, streams in (
            ("positions_all", lambda: B.rom_decode(dec, Xg, z, xo), P, 1),
            ("x_F_v_subset", lambda: B.rom_decode_jac(dec, Xg, z, idx=idx, vhat=vh, x=xt, F=Ft, v=vt),
             n_tan, 5)):
        run()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            run()
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        flop = n * streams * hidden_flop
        out[name] = {"points": n, "streams": streams, "ms": round(ms, 4),
                     "hidden_mfma_flop": flop, "tflops": round(flop / (ms * 1e-3) / 1e12, 1)}
    dec.close()
    return out


def fom_two_dimensional(B, scenes, steps=100, sort_every=10):
    """The 2D scene (64^2 grid, 4,096 particles, fixed-corotated): its
    working set stays in the caches and the run is bound by launch latency,
    so only the absolute rate is reported."""
    import torch
    dev = "cuda:0"
    s = scenes.scene_2d()
    P = s["P"]
    st = scenes.initial_state(s)
    soa = lambda a: torch.tensor(np.ascontiguousarray(a.reshape(P, -1).T), device=dev)
    parts = B.Particles(soa(st["x"]), soa(st["v"]), soa(st["C"]), soa(st["F"]),
                        m_uniform=float(s["m"]), V0_uniform=float(s["V0"]))
    grid = B.Grid(2, s["n"], s["dx"], s["bound"], s["floor_mode"], s["mu_f"], s["gravity"])
    gbuf = torch.zeros(grid.nodes() * 4, device=dev)
    ws = torch.zeros(B.mpm_step_workspace_bytes(grid, P), dtype=torch.uint8, device=dev)
    mat = (s["model"], s["E"], s["nu"])
    B.mpm_step(grid, mat, parts, s["dt"], 10, sort_every, 0, gbuf, ws)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    B.mpm_step(grid, mat, parts, s["dt"], steps, sort_every, 0, gbuf, ws)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    # the same steps captured once in a graph and replayed (mpm_step launches
    # only kernels and device copies)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        B.mpm_step(grid, mat, parts, s["dt"], 1, sort_every, 0, gbuf, ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        B.mpm_step(grid, mat, parts, s["dt"], steps, sort_every, 0, gbuf, ws)
    graph.replay()
    torch.cuda.synchronize()
    e0.record()
    graph.replay()
    e1.record()
    torch.cuda.synchronize()
    ms_g = e0.elapsed_time(e1) / steps
    return {"workload": "2D full-order MPM, 64^2 grid, 4,096 particles, fixed-corotated, "
                        "dt 1e-4, sort every %d steps" % sort_every,
            "ms_per_step": round(ms, 4), "particle_steps_per_s": P / (ms * 1e-3),
            "graph_ms_per_step": round(ms_g, 4), "graph_particle_steps_per_s": P / (ms_g * 1e-3),
            "graph_speedup": round(ms / ms_g, 2), "steps": steps}


def fom_fixed_corotated(B, scenes, s, steps, warmup):
    """The same scene and loop with the fixed-corotated law (the paper's
    constitutive model; a closest-rotation eigen-solve per particle inside
    the scatter): time per step and the scatter's average launch time."""
    import torch
    dev = "cuda:0"
    P = s["P"]
    st = scenes.initial_state(s)
    soa = lambda a: torch.tensor(np.ascontiguousarray(a.reshape(P, -1).T), device=dev)
    parts = B.Particles(soa(st["x"]), soa(st["v"]), soa(st["C"]), soa(st["F"]),
                        m_uniform=float(s["m"]), V0_uniform=float(s["V0"]))
    grid = B.Grid(3, s["n"], s["dx"], s["bound"], s["floor_mode"], s["mu_f"], s["gravity"])
    gbuf = torch.zeros(grid.nodes() * 4, device=dev)
    ws = torch.zeros(B.mpm_step_workspace_bytes(grid, P), dtype=torch.uint8, device=dev)
    flag = torch.zeros(1, dtype=torch.int32, device=dev)
    mat = (scenes.MODEL_FIXED_COROTATED, s["E"], s["nu"])
    timing = B.Timing(capacity=16 * (steps + 8))
    timing.sample(TIMING_EVERY, ["p2g"])
    B.mpm_step(grid, mat, parts, s["dt"], warmup, SORT_EVERY, 0, gbuf, ws, status=flag)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    B.mpm_step(grid, mat, parts, s["dt"], steps, SORT_EVERY, 0, gbuf, ws, status=flag,
               timing=timing)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    n, p2g_ms = timing.read()["p2g"]
    timing.close()
    return {"ms_per_step": round(ms, 4), "particle_steps_per_s": P / (ms * 1e-3),
            "p2g_avg_ms": round(p2g_ms / n, 5), "steps": steps, "status": int(flag.item())}


def rom_throughput(B, scenes, s, steps, n_samples=512, r=16, width=128, n_hidden=5,
                   quadrature=None, mode=None, peaks=None):
    """Reduced-order steps on the same 2,097,152-particle scene: one
    instance, r = 16, 512 sample points per step, Lagrangian quadrature
    (all particles decoded to find the neighbours), bf16 decoder of width
    128 with 5 hidden layers, position-velocity projection with 3
    Gauss-Newton iterations (damping 1e-4); the per-step launches are
    replayed from a HIP graph.  The decoder here is randomly initialised
    (throughput only; the trained leg measures accuracy).  quadrature and
    mode select the Eulerian quadrature and the velocity-only projection."""
    import torch
    dev = "cuda:0"
    quadrature = B.QUAD_LAGRANGIAN if quadrature is None else quadrature
    mode = B.POS_VEL if mode is None else mode
    X = s["X"]
    P = s["P"]
    Ws, bs = scenes.xavier_decoder(3, r, width, n_hidden, 11)
    lo, hi = X.min(0), X.max(0)
    dec = B.Decoder(Ws, bs, lo, hi, np.zeros(3, np.float32), np.full(3, 1e-3, np.float32),
                    B.OUT_DISPLACEMENT, B.PREC_BF16)
    grid = B.Grid(3, s["n"], s["dx"], s["bound"], s["floor_mode"], s["mu_f"], s["gravity"])
    Xg = torch.tensor(np.ascontiguousarray(X.T), device=dev)
    E = torch.tensor([s["E"]], dtype=torch.float32, device=dev)
    ns = torch.tensor([n_samples], dtype=torch.int32, device=dev)
    rom = B.Rom(dec, grid, Xg, E, ns, B.gn_opts(mode=mode, max_iter=3, damping=1e-4), seed=4,
                rho0=1000.0, m_uniform=float(s["m"]), autotune=True, quadrature=quadrature)
    shapes = decoder_shapes(dec, 1, P, n_samples)
    z = torch.zeros(1, r, dtype=torch.float64, device=dev)
    zp = z.clone()
    vh = torch.zeros(1, r, dtype=torch.float64, device=dev)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    k = 10
    rom.step(k, 0, s["dt"], z, zp, vh, status=st, use_graph=True)     # capture + warm-up
    torch.cuda.synchronize()
    times = []
    n_rep = max(1, steps // k)
    for i in range(n_rep):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        rom.step(k, k * (i + 1), s["dt"], z, zp, vh, status=st, use_graph=True)
        b.record()
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b) / k)
    n_quad, n_active = rom.last_counts(0)
    rom.close()
    # the dominant launch of the step, alone: positions of every particle
    xo = torch.empty(1, 3, P, device=dev)
    B.rom_decode(dec, Xg, z, xo)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(5):
        B.rom_decode(dec, Xg, z, xo)
    b.record()
    torch.cuda.synchronize()
    dec_ms = a.elapsed_time(b) / 5
    flop_pt = 2 * (width * (3 + r) + (n_hidden - 1) * width * width + 3 * width)
    tflops = P * flop_pt / (dec_ms * 1e-3) / 1e12
    dec_roof = {"bound": "mfma", "kernel": "bf16 decoder, positions of all %d particles" % P,
                "shape": SHAPE_NAMES[dec.shape(1, 1, P)], "ms": round(dec_ms, 4),
                "flop_per_point": flop_pt, "achieved": round(tflops, 1), "peak": MFMA_BF16_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(tflops / MFMA_BF16_PEAK_TFLOPS, 4)}
    if peaks:
        dec_roof["measured_peak"] = peaks["mfma_bf16_TFLOPs"]
        dec_roof["frac_measured"] = round(tflops / peaks["mfma_bf16_TFLOPs"], 4)
    dec.close()
    times = np.array(times)
    return {"metric": "ROM latent steps/s", "value": float(1e3 / times.mean()), "unit": "latent steps/s",
            "decoder_shapes": shapes, "decoder_roofline": dec_roof,
            "ms_per_step": float(times.mean()), "p50_ms": float(np.percentile(times, 50)),
            "p99_ms": float(np.percentile(times, 99)), "steps": int(n_rep * k),
            "n_quadrature_points": int(n_quad), "n_active_nodes": int(n_active),
            "config": {"instances": 1, "particles": P, "samples": n_samples, "r": r,
                       "decoder": "bf16 MLP %d x %d, random init" % (width, n_hidden),
                       "quadrature": "Eulerian (l = 2, a displacement step and one Newton step)"
                       if quadrature == B.QUAD_EULERIAN else "Lagrangian",
                       "projection": "position-velocity, 3 Gauss-Newton iterations"
                       if mode == B.POS_VEL else "velocity only",
                       "graph": "HIP graph of %d steps" % k},
            "displacement_error": None}


def rom_pareto(B, scenes, s, steps):
    """Latent steps/s over the paper's axes of the reduced model's cost:
    quadrature (Lagrangian: every particle decoded each step; Eulerian:
    samples and lattice points only), sample count and projection scheme,
    on the 2.1M-particle scene with the randomly initialised decoder."""
    rows = []
    for quad, qn in ((B.QUAD_LAGRANGIAN, "lagrangian"), (B.QUAD_EULERIAN, "eulerian")):
        for ns in (50, 512):
            for mode, mn in ((B.POS_VEL, "position-velocity"), (B.VEL_ONLY, "velocity-only")):
                r = rom_throughput(B, scenes, s, steps, n_samples=ns, quadrature=quad, mode=mode)
                rows.append({"quadrature": qn, "samples": ns, "projection": mn,
                             "latent_steps_per_s": round(r["value"], 1),
                             "ms_per_step": round(r["ms_per_step"], 4),
                             "quadrature_points": r["n_quadrature_points"],
                             "active_nodes": r["n_active_nodes"]})
                log("pareto:", json.dumps(rows[-1]))
    return rows


def rom_trained_accuracy(B, scenes, s, n_steps, train_steps, r=16, width=128, n_hidden=5,
                         n_samples=512, codes="encoder"):
    """The reduced model with a trained decoder on the same 2,097,152-particle
    scene and parameters (E = 5e4, v0 = (0, -1, 0)): full-order snapshots
    (every 5th step of n_steps, 65,536 particles), GPU training (bf16
    kernels, Adam with the learning rate decaying exponentially 1e-2 -> 1e-4
    over train_steps batches of 16,384 rows, penalty weights balanced to the
    data scale), then n_steps reduced steps (512 samples, position-velocity
    projection, 3 Gauss-Newton iterations, normal equations damped by 1e-4)
    judged every 10 steps against the full-order model with the transfers of
    the reduced substep (no affine term).  The same decoder then runs on the
    body sampled 2x finer per dimension (16,777,216 particles it never saw),
    judged against the full-order model on that set."""
    import torch
    from paper_2109_12390_amd import evaluate as EV
    from paper_2109_12390_amd import train as TR
    E, v0 = float(s["E"]), (0.0, -1.0, 0.0)
    t0 = time.perf_counter()
    fom = EV.fom_positions(s, E, v0, n_steps, 10, affine=False)
    snap = TR.generate_snapshots(s, [(E, v0)], n_steps=n_steps, every=5, n_sub=65536, seed=4,
                                 affine=False)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    lam_F, lam_v = TR.balanced_penalties(snap)
    t0 = time.perf_counter()
    # codes from the encoder network (Section 4.1) at the paper's starting
    # rate 1e-3, or free per-snapshot codes at 1e-2
    enc = codes == "encoder"
    lr0 = 1e-3 if enc else 1e-2
    out = TR.train(snap, width=width, n_hidden=n_hidden, r=r, steps=train_steps, n_groups=64,
                   rows_per_group=256, lr0=lr0, lr1=lr0 * 1e-2, lam_F=lam_F, lam_v=lam_v,
                   log_every=train_steps, encoder=enc, deterministic=True)
    Ws, bs, Z, norm, hist = out[:5]
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    lo, hi, mean, std = norm
    dec = B.Decoder(Ws, bs, lo, hi, mean, std, B.OUT_DISPLACEMENT, B.PREC_BF16)
    opts = B.gn_opts(mode=B.POS_VEL, max_iter=3, damping=1e-4, proj_fp32=1)
    x_rom, st = EV.rom_positions(dec, s, E, v0, n_steps, 10, n_samples=n_samples, opts=opts,
                                 z_guess=Z[0])
    err, pos = EV.displacement_error(x_rom, fom, s["X"])
    del x_rom
    # error floor: the decoder's best approximation of every recorded frame
    # (frames every 10 steps, codes every 5)
    Zs = [Z[min(2 * k, Z.shape[0] - 1)] for k in range(len(fom))]
    proj = EV.best_projection(dec, s, fom, Zs)
    err_proj = EV.displacement_error(proj, fom, s["X"])[0]
    del proj
    # the linear-manifold baseline (one linear layer, same r and objective)
    Wl, bl, Zl, norml = TR.train_linear(snap, r, train_steps, lam_F=lam_F, lam_v=lam_v)
    ldec = B.Decoder(Wl, bl, *norml, B.OUT_DISPLACEMENT, B.PREC_FP32)
    proj = EV.best_projection(ldec, s, fom, [Zl[min(2 * k, Zl.shape[0] - 1)]
                                              for k in range(len(fom))])
    lin = {"best_projection_displacement_error": round(EV.displacement_error(proj, fom, s["X"])[0], 4)}
    del proj
    xl, sl = EV.rom_positions(ldec, s, E, v0, n_steps, 10, n_samples=n_samples,
                              opts=opts,
                              z_guess=Zl[0])
    lin.update({"displacement_error": round(EV.displacement_error(xl, fom, s["X"])[0], 4),
                "status": sl["status"], "status_flags": B.flag_names(sl["status"]),
                "decoder": "one linear layer, r = %d, fp32" % r})
    del xl
    ldec.close()
    log("linear manifold:", json.dumps(lin))
    # the same decoder under the other quadrature and the paper's fast
    # configuration (few samples, velocity-only projection)
    variants = []
    for qn, quad, ns, mode, mn, pf in (("eulerian", B.QUAD_EULERIAN, n_samples, B.POS_VEL,
                                        "position-velocity", 1),
                                       ("lagrangian", B.QUAD_LAGRANGIAN, n_samples, B.POS_VEL,
                                        "position-velocity, all decodes in bf16", 0),
                                       ("lagrangian", B.QUAD_LAGRANGIAN, n_samples, B.POS_VEL,
                                        "position-velocity, initial-condition fields", 1),
                                       ("lagrangian", B.QUAD_LAGRANGIAN, 50, B.VEL_ONLY,
                                        "velocity-only", 0),
                                       ("eulerian", B.QUAD_EULERIAN, 50, B.VEL_ONLY,
                                        "velocity-only", 0)):
        xr, sv = EV.rom_positions(dec, s, E, v0, n_steps, 10, n_samples=ns,
                                  opts=B.gn_opts(mode=mode, max_iter=3, damping=1e-4, proj_fp32=pf),
                                  z_guess=Z[0], quadrature=quad, exact_ic="fields" in mn)
        e2, p2 = EV.displacement_error(xr, fom, s["X"])
        variants.append({"quadrature": qn, "samples": ns, "projection": mn,
                         "latent_steps_per_s": round(1e3 / sv["ms_per_step"], 1),
                         "ms_per_step": round(sv["ms_per_step"], 4),
                         "displacement_error": round(e2, 4), "position_error_percent": round(p2, 4),
                         "status": sv["status"], "status_flags": B.flag_names(sv["status"])})
        log("trained variant:", json.dumps(variants[-1]))
    # zero-shot super-resolution: the same body sampled 2x finer per
    # dimension (4 particles per cell per dimension, a new jitter), which the
    # decoder never saw, judged against the full-order model on that set
    del fom
    fine = scenes.scene_3d(seed=3, sub=4)
    fom_f = EV.fom_positions(fine, E, v0, n_steps, 10, affine=False)
    super_res = []
    for qn, quad in (("eulerian", B.QUAD_EULERIAN), ("lagrangian", B.QUAD_LAGRANGIAN)):
        xr, sv = EV.rom_positions(dec, fine, E, v0, n_steps, 10, n_samples=n_samples,
                                  opts=opts,
                                  z_guess=Z[0], quadrature=quad)
        e2, p2 = EV.displacement_error(xr, fom_f, fine["X"])
        del xr
        super_res.append({"particles": fine["P"], "quadrature": qn, "samples": n_samples,
                          "projection": "position-velocity",
                          "latent_steps_per_s": round(1e3 / sv["ms_per_step"], 1),
                          "ms_per_step": round(sv["ms_per_step"], 4),
                          "quadrature_points": sv["n_quadrature_points"],
                          "displacement_error": round(e2, 4), "position_error_percent": round(p2, 4),
                          "status": sv["status"], "status_flags": B.flag_names(sv["status"])})
        log("super-resolution:", json.dumps(super_res[-1]))
    del fom_f
    dec.close()
    return {"metric": "ROM latent steps/s at the measured displacement error",
            "value": float(1e3 / st["ms_per_step"]), "unit": "latent steps/s",
            "ms_per_step": st["ms_per_step"], "displacement_error": err,
            "position_error_percent": pos, "status": st["status"],
            "status_flags": B.flag_names(st["status"]), "steps": n_steps,
            "best_projection_displacement_error": round(err_proj, 4),
            "linear_manifold": lin,
            "train": {"steps": train_steps, "rows_per_step": 64 * 256, "objective": hist,
                      "codes": codes, "learning_rate": [lr0, lr0 * 1e-2], "reproducible": True,
                      "rows_per_s": train_steps * 64 * 256 / t_train,
                      "lam_F": lam_F, "lam_v": lam_v, "seconds": t_train,
                      "snapshot_seconds": t_data, "frames": snap.n_frames, "particles": 65536},
            "config": {"instances": 1, "particles": s["P"], "samples": n_samples, "r": r,
                       "decoder": "bf16 MLP %d x %d, trained" % (width, n_hidden),
                       "projection": "position-velocity, 3 Gauss-Newton iterations, damping 1e-4, "
                                     "positions of the projection decoded in fp32",
                       "codes": codes, "quadrature": "Lagrangian",
                       "reference": "full-order model without the affine transfer term"},
            "variants": variants, "super_resolution": super_res}


def rom_study(B, scenes, s, n_steps=500, train_steps=4000, r=16, width=128, n_hidden=5):
    """Where the reduced model's error comes from, on the 2,097,152-particle
    scene (E = 5e4, v0 = (0, -1, 0), n_steps steps, errors every 10 steps)
    with one trained bf16 decoder (as in rom_trained_accuracy: encoder codes,
    reproducible training, projection positions in fp32):
      - error floors: the decoder's best projection of every full-order frame
        (the latent fitting all positions, by Gauss-Newton), and the reduced
        model with every particle sampled (Lagrangian quadrature);
      - the sample-count sweep |P| in {10, 50, 100, 512} x {position-velocity,
        velocity-only} x {Lagrangian, Eulerian quadrature}, plus the
        position-velocity scheme at 512 with damping 1e-5, 1e-6 and 0 and
        with the initial-condition correction fields;
      - the same weights with fp32 hidden layers at 512 samples;
      - the linear-manifold baseline (one linear layer, same r and objective)
        at 512 samples, with its own best projection;
    each against the full-order model without the affine transfer term (the
    reduced substep's transfers) and with it (APIC).  Latent steps/s are
    reported beside each error."""
    import torch
    from paper_2109_12390_amd import evaluate as EV
    from paper_2109_12390_amd import train as TR
    E, v0 = float(s["E"]), (0.0, -1.0, 0.0)
    rec = 10
    fom_pic = EV.fom_positions(s, E, v0, n_steps, rec, affine=False)
    fom_apic = EV.fom_positions(s, E, v0, n_steps, rec, affine=True)
    snap = TR.generate_snapshots(s, [(E, v0)], n_steps=n_steps, every=5, n_sub=65536, seed=4,
                                 affine=False)
    lam_F, lam_v = TR.balanced_penalties(snap)
    # encoder codes (Section 4.1), the paper's starting rate, reproducible
    out_t = TR.train(snap, width=width, n_hidden=n_hidden, r=r, steps=train_steps, n_groups=64,
                     rows_per_group=256, lr0=1e-3, lr1=1e-5, lam_F=lam_F, lam_v=lam_v,
                     encoder=True, deterministic=True)
    Ws, bs, Z, norm = out_t[:4]
    lo, hi, mean, std = norm
    dec = B.Decoder(Ws, bs, lo, hi, mean, std, B.OUT_DISPLACEMENT, B.PREC_BF16)
    Zs = [Z[min(2 * k, Z.shape[0] - 1)] for k in range(len(fom_pic))]   # frames every 5 steps
    X = s["X"]

    def errs(x):
        e1, p1 = EV.displacement_error(x, fom_pic, X)
        e2, _ = EV.displacement_error(x, fom_apic, X)
        return {"e_u_vs_pic": round(e1, 4), "e_u_vs_apic": round(e2, 4),
                "position_error_percent_vs_pic": round(p1, 4)}

    out = {"config": {"particles": s["P"], "steps": n_steps, "r": r,
                      "decoder": "bf16 MLP %d x %d, trained with encoder codes" % (width, n_hidden),
                      "damping": 1e-4, "gauss_newton_iterations": 3,
                      "projection_positions": "fp32"},
           "fom_pic_vs_apic": errs(fom_pic)["e_u_vs_apic"]}
    proj = EV.best_projection(dec, s, fom_pic, Zs)
    out["best_projection"] = errs(proj)
    del proj
    log("study: best projection", json.dumps(out["best_projection"]))
    runs = []

    def run(quad, qn, ns, mode, mn, damping=1e-4, d=dec, zg=Z[0], tag=None, exact_ic=False):
        prog = (lambda k: log("study: %d samples, step %d" % (ns, k)) if k % 100 == 0 else None)
        x, st = EV.rom_positions(d, s, E, v0, n_steps, rec, n_samples=ns,
                                 opts=B.gn_opts(mode=mode, max_iter=3, damping=damping,
                                                proj_fp32=1),
                                 z_guess=zg, quadrature=quad, progress=prog, exact_ic=exact_ic)
        row = {"quadrature": qn, "samples": ns, "projection": mn, "damping": damping,
               "initial_condition_fields": exact_ic,
               "latent_steps_per_s": round(1e3 / st["ms_per_step"], 1),
               "quadrature_points": st["n_quadrature_points"], "status": st["status"],
               "status_flags": B.flag_names(st["status"])}
        if tag:
            row["decoder"] = tag
        row.update(errs(x))
        del x
        torch.cuda.synchronize()
        runs.append(row)
        log("study:", json.dumps(row))

    run(B.QUAD_LAGRANGIAN, "lagrangian", s["P"], B.POS_VEL, "position-velocity")
    for qn, quad in (("lagrangian", B.QUAD_LAGRANGIAN), ("eulerian", B.QUAD_EULERIAN)):
        for ns in (10, 50, 100, 512):
            for mode, mn in ((B.POS_VEL, "position-velocity"), (B.VEL_ONLY, "velocity-only")):
                run(quad, qn, ns, mode, mn)
    for damping in (1e-5, 1e-6, 0.0):
        run(B.QUAD_LAGRANGIAN, "lagrangian", 512, B.POS_VEL, "position-velocity", damping=damping)
    run(B.QUAD_LAGRANGIAN, "lagrangian", 512, B.POS_VEL, "position-velocity", exact_ic=True)
    dec.close()
    # the same weights with fp32 hidden layers (the precision's share)
    dec32 = B.Decoder(Ws, bs, lo, hi, mean, std, B.OUT_DISPLACEMENT, B.PREC_FP32)
    run(B.QUAD_LAGRANGIAN, "lagrangian", 512, B.POS_VEL, "position-velocity", d=dec32,
        tag="same weights, fp32")
    dec32.close()
    # the linear-manifold baseline
    Wl, bl, Zl, norml = TR.train_linear(snap, r, train_steps, lam_F=lam_F, lam_v=lam_v)
    lo, hi, mean, std = norml
    ldec = B.Decoder(Wl, bl, lo, hi, mean, std, B.OUT_DISPLACEMENT, B.PREC_FP32)
    Zls = [Zl[min(2 * k, Zl.shape[0] - 1)] for k in range(len(fom_pic))]
    proj = EV.best_projection(ldec, s, fom_pic, Zls)
    out["linear_best_projection"] = errs(proj)
    del proj
    log("study: linear best projection", json.dumps(out["linear_best_projection"]))
    try:
        run(B.QUAD_LAGRANGIAN, "lagrangian", 512, B.POS_VEL, "position-velocity", d=ldec,
            zg=Zl[0], tag="linear, one layer")
    except Exception as exc:           # a diverging run is a result, not a crash
        runs.append({"decoder": "linear, one layer", "samples": 512, "failed": str(exc)})
    ldec.close()
    out["runs"] = runs
    return out


SHAPE_NAMES = ["1 point tile per wave", "2 point tiles per wave", "4 point tiles per wave",
               "units split over a block", "points split, activations in registers"]


def batched_study(B, scenes, s, n_inst=256, n_steps=400, record_every=20, train_steps=8000,
                  n_train=8, n_held=2, train_frames=200, every=5, n_eval=65536, r=16, width=128,
                  n_hidden=5, codes="encoder", quadratures=("lagrangian", "eulerian"),
                  trainings=("bf16", "fp32", "bf16_encoder")):
    """Training on several parameter instances and the batched reduced model
    judged per instance against the full-order model.

    Training data: n_train instances (E log-uniform in [1e4, 1e5], v0
    uniform in [-2, 2]^3, seeded) of the 2,097,152-particle scene, frames
    every `every` steps up to train_frames (65,536 particles each, PIC
    transfers); the decoder (bf16, then fp32, same initial weights and
    batches) is trained with Adam and judged by its final objective and by
    the best projection of n_held held-out instances' trajectories onto its
    manifold; a third training (bf16) takes its codes from the encoder
    network of Section 4.1 instead of free per-snapshot codes.  `codes`
    picks the bf16 decoder that drives the reduced runs ("free" or
    "encoder").  Then n_inst instances (E log-uniform in [1e3, 1e5], v0
    uniform in [-2, 2]^3, 256-1024 samples each, a second seed) start from
    the least-squares initial latents (position and velocity) and advance
    together, one HIP graph per batched step, with each quadrature; every
    instance is judged on n_eval particles every record_every steps against
    its own full-order run (PIC transfers, the reduced substep's scheme)."""
    import torch
    from paper_2109_12390_amd import evaluate as EV
    from paper_2109_12390_amd import train as TR
    dev = "cuda:0"
    P = s["P"]
    t_all = time.perf_counter()
    Et, vt = scenes.parameter_instances(n_train + n_held, 31, E_range=(1.0e4, 1.0e5))
    train_inst = [(float(Et[i]), tuple(float(c) for c in vt[i])) for i in range(n_train)]
    held = [(float(Et[i]), tuple(float(c) for c in vt[i])) for i in range(n_train, n_train + n_held)]
    n_fom = every * train_frames
    snap = TR.generate_snapshots(s, train_inst, n_steps=n_fom, every=every, n_sub=n_eval, seed=4,
                                 affine=False)
    torch.cuda.synchronize()
    log("batched study: %d training frames of %d instances (%.1f s)"
        % (snap.n_frames, n_train, time.perf_counter() - t_all))
    lam_F, lam_v = TR.balanced_penalties(snap)
    held_fom = [EV.fom_positions(s, E, v0, n_fom, 50, affine=False) for (E, v0) in held]
    fpi = n_fom // every + 1                               # frames per training instance
    sub_train = torch.tensor(snap.sub, device=dev).long()

    def as_frames(frs):
        """[d][P] frames -> concatenated positions of the training subset."""
        return torch.stack([f[:, sub_train].T.reshape(-1) for f in frs]).contiguous()

    decs, training = {}, {}
    # free codes train best from 1e-2; the encoder from the paper's 1e-3
    # (from 1e-2 its objective stalls at 4x that of free codes)
    for prec, pname, enc, lr0 in ((B.PREC_BF16, "bf16", False, 1e-2),
                                  (B.PREC_FP32, "fp32", False, 1e-2),
                                  (B.PREC_BF16, "bf16_encoder", True, 1e-3)):
        if pname not in trainings:
            continue
        t0 = time.perf_counter()
        out = TR.train(snap, width=width, n_hidden=n_hidden, r=r, steps=train_steps, n_groups=64,
                       rows_per_group=256, precision=prec, lr0=lr0, lr1=lr0 * 1e-2, lam_F=lam_F,
                       lam_v=lam_v, log_every=train_steps // 4, encoder=enc)
        Ws, bs, Z, norm, hist = out[:5]
        pe = torch.tensor(out[5], device=dev) if enc else None
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        dec = B.Decoder(Ws, bs, *norm, B.OUT_DISPLACEMENT, prec)
        enc_args = (r, 3, norm[0].astype(np.float32), norm[1].astype(np.float32))
        # held-out reconstruction: best projection of the held-out frames
        # (every 50 steps), each from the encoder's code of the frame, or
        # without an encoder from the training code that decodes closest
        rec = []
        for fr in held_fom:
            if enc:
                zg = TR.encode(pe, as_frames(fr), *enc_args).double().cpu().numpy()
            else:
                zg = EV.nearest_codes(dec, s, fr, Z)
            proj = EV.best_projection(dec, s, fr, zg)
            rec.append(round(EV.displacement_error(proj, fr, s["X"])[0], 4))
            del proj
        training[pname] = {"learning_rate": [lr0, lr0 * 1e-2],
                           "objective": [(int(a), float(b)) for a, b in hist],
                           "final_objective": float(hist[-1][1]), "seconds": round(t_train, 1),
                           "rows_per_s": round(train_steps * 64 * 256 / t_train),
                           "held_out_best_projection_error": rec}
        log("batched study: training", pname, json.dumps(training[pname]))
        decs[pname] = (dec, Z, pe, enc_args)
    snap_sub = snap.sub
    del snap
    use = "bf16_encoder" if codes == "encoder" else "bf16"
    for k in decs:
        if k != use:
            decs[k][0].close()
    dec, Z, pe, enc_args = decs[use]
    # the batched instances
    Es, v0s = scenes.parameter_instances(n_inst, 32)
    rng = np.random.default_rng(33)
    ns = rng.integers(256, 1025, size=n_inst).astype(np.int32)
    sub = np.sort(np.random.default_rng(34).choice(P, size=n_eval, replace=False))
    X = s["X"]
    Xg = torch.tensor(np.ascontiguousarray(X.T), device=dev)
    sub_t = torch.tensor(sub, device=dev).long()
    Xe = Xg[:, sub_t].contiguous()
    # initial latents: least squares from the encoder's code of the
    # reference configuration, or without an encoder from the training
    # instances' first codes, each instance at the one whose tangent space
    # fits its velocity
    if pe is not None:
        x_ref = torch.tensor(np.ascontiguousarray(X[snap_sub].reshape(1, -1)), device=dev)
        cand = TR.encode(pe, x_ref, *enc_args).double().cpu().numpy()
    else:
        cand = Z.reshape(n_train, fpi, r)[:, 0]
    z_init, v_init, choice = EV.rom_initial_states(dec, s, v0s, cand)
    log("batched study: initial codes chosen per candidate:",
        np.bincount(choice, minlength=len(cand)).tolist())
    # full-order reference per instance on the evaluation subset
    t0 = time.perf_counter()
    fom = []
    for b in range(n_inst):
        fr = EV.fom_positions(s, float(Es[b]), v0s[b], n_steps, record_every, affine=False)
        fom.append(np.stack([f[:, sub_t].cpu().numpy() for f in fr]))
        del fr
        if (b + 1) % 32 == 0:
            log("batched study: full-order reference %d / %d (%.0f s)"
                % (b + 1, n_inst, time.perf_counter() - t0))
    fom = np.stack(fom)                                   # [inst][frame][d][n_eval]
    Xs = X[sub].T.astype(np.float64)                      # [d][n_eval]
    grid = B.Grid(3, s["n"], s["dx"], s["bound"], s["floor_mode"], s["mu_f"], s["gravity"])
    legs = {}
    qmap = {"lagrangian": B.QUAD_LAGRANGIAN, "eulerian": B.QUAD_EULERIAN}
    for qn in quadratures:
        quad = qmap[qn]
        rom = B.Rom(dec, grid, Xg, torch.tensor(Es.astype(np.float32), device=dev),
                    torch.tensor(ns, device=dev),
                    B.gn_opts(mode=B.POS_VEL, max_iter=3, damping=1e-4, proj_fp32=1), seed=5,
                    rho0=float(s["rho"]),
                    m_uniform=float(s["m"]), autotune=True, quadrature=quad)
        z = z_init.clone()
        zp = z_init.clone()
        vh = v_init.clone()
        st = torch.zeros(n_inst, dtype=torch.int32, device=dev)
        xbuf = torch.zeros(n_inst, 3, n_eval, device=dev)
        B.rom_decode(dec, Xe, z, xbuf)
        rec = [xbuf.cpu().numpy()]
        times = []
        for i in range(n_steps):
            a = torch.cuda.Event(enable_timing=True)
            e = torch.cuda.Event(enable_timing=True)
            a.record()
            rom.step(1, i, s["dt"], z, zp, vh, status=st, use_graph=True)
            e.record()
            torch.cuda.synchronize()
            times.append(a.elapsed_time(e))
            if (i + 1) % record_every == 0:
                B.rom_decode(dec, Xe, z, xbuf)
                rec.append(xbuf.cpu().numpy())
            if (i + 1) % 50 == 0:
                log("batched study: %s step %d / %d, %.1f ms per batched step"
                    % (qn, i + 1, n_steps, float(np.mean(times[1:]))))
        rom.close()
        dz = (z - z_init).abs().max(1).values / (1.0 + z_init.abs().max(1).values)
        xr = np.stack(rec, axis=1)                        # [inst][frame][d][n_eval]
        e_u = np.empty(n_inst)
        for b in range(n_inst):
            fb = fom[b].astype(np.float64)
            num = ((xr[b].astype(np.float64) - fb) ** 2).sum()
            den = ((fb - Xs[None]) ** 2).sum()
            e_u[b] = np.sqrt(num / den)
        del xr
        flags = st.cpu().numpy()
        t = np.array(times[1:])                           # the first replay includes the capture
        soft = Es < 1.0e4

        def dist(v):
            return {"n": int(v.size), "mean": round(float(v.mean()), 4),
                    "p50": round(float(np.percentile(v, 50)), 4),
                    "p90": round(float(np.percentile(v, 90)), 4),
                    "max": round(float(v.max()), 4)} if v.size else None
        legs[qn] = {"latent_steps_per_s": round(n_inst * 1e3 / t.mean(), 1),
                    "ms_per_batched_step": round(float(t.mean()), 3),
                    "p50_ms": round(float(np.percentile(t, 50)), 3),
                    "p99_ms": round(float(np.percentile(t, 99)), 3),
                    "timed_steps": int(t.size),
                    "latent_change_p50": round(float(dz.median().item()), 4),
                    "e_u": dist(e_u), "e_u_E_below_1e4": dist(e_u[soft]),
                    "e_u_E_from_1e4": dist(e_u[~soft]),
                    "instances_with_flags": {"domain": int(((flags & B.FLAG_DOMAIN) != 0).sum()),
                                             "singular": int(((flags & B.FLAG_SINGULAR) != 0).sum()),
                                             "noconv": int(((flags & B.FLAG_NOCONV) != 0).sum()),
                                             "linesearch": int(((flags & B.FLAG_LINESEARCH) != 0).sum())},
                    "e_u_per_instance": [round(float(v), 4) for v in e_u]}
        log("batched study:", qn, json.dumps({k: v for k, v in legs[qn].items()
                                               if k != "e_u_per_instance"}))
    dec.close()
    return {"config": {"instances": n_inst, "particles": P, "samples": "256-1024 per instance",
                       "r": r, "decoder": "bf16 MLP %d x %d, trained on %d instances, %s codes"
                                          % (width, n_hidden, n_train, codes),
                       "E": "log-uniform [1e3, 1e5]", "v0": "uniform [-2, 2]^3",
                       "initial_latents": "least squares (position, then velocity) from the "
                                          + ("encoder's code of the reference configuration"
                                             if codes == "encoder" else
                                             "training instance's first code that fits v0 best"),
                       "projection": "position-velocity, 3 Gauss-Newton iterations, damping 1e-4, "
                                     "positions of the projection decoded in fp32",
                       "steps": n_steps, "judged_every": record_every, "eval_particles": n_eval,
                       "reference": "full-order model per instance, no affine transfer term",
                       "graph": "HIP graph of one step of all instances"},
            "training_data": {"instances": n_train, "E": "log-uniform [1e4, 1e5]",
                              "v0": "uniform [-2, 2]^3", "frames_per_instance": fpi,
                              "every": every, "particles": n_eval, "held_out_instances": n_held},
            "training": training, "legs": legs,
            "E": [round(float(e), 1) for e in Es], "v0": [[round(float(c), 3) for c in v] for v in v0s],
            "seconds": round(time.perf_counter() - t_all, 1)}


def decoder_shapes(dec, n_inst, P, n_samples):
    """Autotuned decoder launch shapes of a reduced-order step's launches."""
    return {"all particles (positions)": SHAPE_NAMES[dec.shape(1, n_inst, P)],
            "samples (latent Jacobian)": SHAPE_NAMES[dec.shape(9, n_inst, n_samples)],
            "line-search candidates": SHAPE_NAMES[dec.shape(1, n_inst * 9, n_samples)]}


def rom_batched_throughput(B, scenes, s, n_inst, steps, r=16, width=128, n_hidden=5):
    """Reduced-order steps of n_inst parameter instances of the same scene
    advanced together: Young's moduli log-uniform in [1e3, 1e5] and initial
    latent velocities from seeded draws, 256 to 1024 sample points per
    instance, the same bf16 decoder (random initialisation, throughput only),
    position-velocity projection with 3 Gauss-Newton iterations, every step
    of all instances replayed from one HIP graph.  Aggregate latent steps/s
    = instances x steps / time."""
    import torch
    dev = "cuda:0"
    X = s["X"]
    P = s["P"]
    Ws, bs = scenes.xavier_decoder(3, r, width, n_hidden, 11)
    lo, hi = X.min(0), X.max(0)
    dec = B.Decoder(Ws, bs, lo, hi, np.zeros(3, np.float32), np.full(3, 1e-3, np.float32),
                    B.OUT_DISPLACEMENT, B.PREC_BF16)
    grid = B.Grid(3, s["n"], s["dx"], s["bound"], s["floor_mode"], s["mu_f"], s["gravity"])
    Xg = torch.tensor(np.ascontiguousarray(X.T), device=dev)
    Es, _ = scenes.parameter_instances(n_inst, 21)
    rng = np.random.default_rng(22)
    ns = rng.integers(256, 1025, size=n_inst).astype(np.int32)
    E = torch.tensor(Es.astype(np.float32), device=dev)
    nst = torch.tensor(ns, device=dev)
    rom = B.Rom(dec, grid, Xg, E, nst, B.gn_opts(mode=B.POS_VEL, max_iter=3, damping=1e-4), seed=5,
                rho0=1000.0,
                m_uniform=float(s["m"]), autotune=True)
    shapes = decoder_shapes(dec, n_inst, P, int(ns.max()))
    z = torch.zeros(n_inst, r, dtype=torch.float64, device=dev)
    zp = z.clone()
    vh = torch.tensor(1e-2 * rng.standard_normal((n_inst, r)), device=dev)
    st = torch.zeros(n_inst, dtype=torch.int32, device=dev)
    rom.step(1, 0, s["dt"], z, zp, vh, status=st, use_graph=True)      # capture + warm-up
    torch.cuda.synchronize()
    times = []
    for i in range(steps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        rom.step(1, i + 1, s["dt"], z, zp, vh, status=st, use_graph=True)
        b.record()
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    q = [rom.last_counts(b)[0] for b in (0, n_inst // 2, n_inst - 1)]
    rom.close()
    dec.close()
    times = np.array(times)
    return {"metric": "ROM latent steps/s (all instances)", "value": float(n_inst * 1e3 / times.mean()),
            "decoder_shapes": shapes,
            "unit": "latent steps/s", "ms_per_batched_step": float(times.mean()),
            "p50_ms": float(np.percentile(times, 50)), "p99_ms": float(np.percentile(times, 99)),
            "steps": int(steps), "quadrature_points_sampled_instances": [int(v) for v in q],
            "config": {"instances": n_inst, "particles": P, "samples": "256-1024 per instance",
                       "r": r, "decoder": "bf16 MLP %d x %d, random init" % (width, n_hidden),
                       "E": "log-uniform [1e3, 1e5]",
                       "projection": "position-velocity, 3 Gauss-Newton iterations",
                       "graph": "HIP graph of one step of all instances"},
            "error_vs_full_order": None}


if __name__ == "__main__":
    main()
