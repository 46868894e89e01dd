"""The allocation-free projection entry point (rom_project_noalloc), called
through the C ABI, against rom_project with a caller workspace on the same
inputs: bit-identical latents, velocities and status on two calls in a row,
the second with fewer instances and samples (the fixed scratch keeps the
first call's contents), and MR_ESCRATCH for a call beyond its 16 MiB."""
import ctypes

import numpy as np
import pytest

from oracle import decoder as OD
from paper_2109_12390_amd import binding as B
from paper_2109_12390_amd import scenes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
dev = "cuda"


def _case(seed, Bn, ns, d=3, r=8, P=3000):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0.2, 0.8, size=(P, d)).astype(np.float32)
    Ws, bs = scenes.random_decoder(d, r, 32, 3, seed, scale=1.5, bias_scale=0.1)
    lo, hi = X.min(0), X.max(0)
    mean = np.zeros(d, np.float32)
    std = np.full(d, 0.1, np.float32)
    odec = OD.Decoder(Ws, bs, lo, hi, mean, std)
    gdec = B.Decoder(Ws, bs, lo, hi, mean, std, B.OUT_DISPLACEMENT, B.PREC_FP32)
    idx = np.sort(rng.choice(P, size=(Bn, ns), replace=True), axis=1).astype(np.int32)
    zn = 0.4 * rng.standard_normal((Bn, r))
    zp = zn - 0.01 * rng.standard_normal((Bn, r))
    dt = 1e-2
    xt = np.zeros((Bn, d, ns), np.float32)
    vt = rng.standard_normal((Bn, d, ns)).astype(np.float32)
    for b in range(Bn):
        xt[b] = (OD.decode(odec, X[idx[b]].astype(np.float64), zn[b] + dt * rng.standard_normal(r))
                 + 1e-4 * rng.standard_normal((ns, d))).T
    T = lambda a, dt_=torch.float32: torch.tensor(np.ascontiguousarray(a), dtype=dt_, device=dev)
    return dict(gdec=gdec, X=T(X.T), idx=T(idx, torch.int32), xt=T(xt), vt=T(vt),
                zn=T(zn, torch.float64), zp=T(zp, torch.float64), dt=dt, Bn=Bn, r=r)


def _noalloc(c, opts, z, v, it, st, res):
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    return B.load().rom_project_noalloc(
        c["gdec"].handle, c["Bn"], c["X"].shape[1], p(c["X"]), c["idx"].shape[1], p(c["idx"]),
        None, p(c["xt"]), p(c["vt"]), p(c["zn"]), p(c["zp"]), c["dt"], ctypes.byref(opts), p(z),
        p(v), p(it), p(res), p(st), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


@pytest.mark.parametrize("mode", [B.POS_VEL, B.VEL_ONLY])
def test_noalloc_projection_equals_workspace_projection(gpu, mode):
    opts = B.gn_opts(mode=mode, max_iter=3)
    for seed, Bn, ns in ((31, 4, 96), (32, 2, 40)):      # the second call is smaller
        c = _case(seed, Bn, ns)
        outs = {}
        for kind in ("workspace", "noalloc"):
            z = torch.zeros(Bn, c["r"], dtype=torch.float64, device=dev)
            v = torch.zeros_like(z)
            it = torch.zeros(Bn, dtype=torch.int32, device=dev)
            st = torch.zeros(Bn, dtype=torch.int32, device=dev)
            res = torch.zeros(Bn, dtype=torch.float64, device=dev)
            if kind == "workspace":
                B.rom_project(c["gdec"], c["X"], c["idx"], c["xt"], c["vt"], c["zn"], c["zp"],
                              c["dt"], opts, z, v, iters=it, resid=res, status=st)
            else:
                assert _noalloc(c, opts, z, v, it, st, res) == B.MR_OK
            torch.cuda.synchronize()
            outs[kind] = (z, v, it, st, res)
        for a, b in zip(outs["workspace"], outs["noalloc"]):
            assert torch.equal(a, b), (mode, seed)
        print("mode %d B %d ns %d: noalloc == workspace (|dz| %.2e)"
              % (mode, Bn, ns, float((outs["noalloc"][0] - c["zn"]).abs().max())))
        c["gdec"].close()


def test_noalloc_projection_rejects_oversized_calls(gpu):
    c = _case(33, 1, 8)
    opts = B.gn_opts(max_backtrack=30)
    big = 40000
    assert B.rom_project_workspace_bytes(c["gdec"], 1, big, opts) > (16 << 20)
    c["idx"] = torch.zeros(1, big, dtype=torch.int32, device=dev)
    c["xt"] = torch.zeros(1, 3, big, device=dev)
    c["vt"] = torch.zeros(1, 3, big, device=dev)
    z = torch.zeros(1, c["r"], dtype=torch.float64, device=dev)
    i32 = torch.zeros(1, dtype=torch.int32, device=dev)
    res = torch.zeros(1, dtype=torch.float64, device=dev)
    assert _noalloc(c, opts, z, z.clone(), i32, i32.clone(), res) == B.MR_ESCRATCH
    c["gdec"].close()
