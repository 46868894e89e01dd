"""Python binding of libmpmrom.so (the C ABI declared in include/mpmrom.h).

Argument marshalling only: every function below builds the plain descriptor
structs, takes raw device pointers of PyTorch tensors and the current HIP
stream, and calls the entry point of the same name.  All arithmetic runs in
the library's HIP kernels.  There is no fallback: if the library is missing
or fails to load, `load()` raises.
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpmrom.so")

MR_OK = 0
MR_EINVAL, MR_ENOMEM, MR_EDEVICE, MR_ESINGULAR, MR_ENOCONV, MR_EDOMAIN = -1, -2, -3, -4, -5, -6
MR_ESCRATCH = -7
FLAG_DOMAIN, FLAG_SINGULAR, FLAG_NOCONV, FLAG_LINESEARCH, FLAG_DRIFT = 1, 2, 4, 8, 16
FLOOR_STICKY, FLOOR_COULOMB = 0, 1
FIXED_COROTATED, NEO_HOOKEAN = 0, 1
NO_AFFINE, ACCUMULATE, TRIAL, NO_F_UPDATE, SORTED = 1, 2, 4, 8, 16
OUT_POSITION, OUT_DISPLACEMENT = 0, 1
PREC_FP32, PREC_BF16 = 0, 1
POS_VEL, VEL_ONLY = 0, 1

_ERRNAMES = {MR_EINVAL: "MR_EINVAL", MR_ENOMEM: "MR_ENOMEM", MR_EDEVICE: "MR_EDEVICE",
             MR_ESINGULAR: "MR_ESINGULAR", MR_ENOCONV: "MR_ENOCONV", MR_EDOMAIN: "MR_EDOMAIN",
             MR_ESCRATCH: "MR_ESCRATCH"}


class MrError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__("%s returned %s (%d)" % (fn, _ERRNAMES.get(code, "?"), code))
        self.code = code


class MrGrid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("dx", ctypes.c_float),
                ("bound", ctypes.c_int32), ("floor_mode", ctypes.c_int32),
                ("mu_friction", ctypes.c_float), ("gravity", ctypes.c_float * 3)]


class MrMaterial(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("E", ctypes.c_float), ("nu", ctypes.c_float)]


class MrParticles(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("x", ctypes.c_void_p), ("v", ctypes.c_void_p),
                ("C", ctypes.c_void_p), ("F", ctypes.c_void_p), ("m", ctypes.c_void_p),
                ("V0", ctypes.c_void_p), ("m_uniform", ctypes.c_float),
                ("V0_uniform", ctypes.c_float)]


class MrGnOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("max_backtrack", ctypes.c_int32), ("armijo_c", ctypes.c_double),
                ("damping", ctypes.c_double), ("tol_step", ctypes.c_double),
                ("proj_fp32", ctypes.c_int32)]


class MrRomConfig(ctypes.Structure):
    _fields_ = [("B", ctypes.c_int32), ("n_particles", ctypes.c_int64),
                ("n_samples_max", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("rho0", ctypes.c_float), ("m_uniform", ctypes.c_float),
                ("model", ctypes.c_int32), ("nu", ctypes.c_float),
                ("autotune", ctypes.c_int32), ("quadrature", ctypes.c_int32),
                ("quad_per_dim", ctypes.c_int32), ("newton_iters", ctypes.c_int32),
                ("newton_tol", ctypes.c_float)]


QUAD_LAGRANGIAN = 0
QUAD_EULERIAN = 1


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_f32 = ctypes.c_float
_f64 = ctypes.c_double

# name -> (restype, argtypes); must list every function of include/mpmrom.h
SIGNATURES = {
    "mpm_p2g": (_i32, [ctypes.POINTER(MrGrid), ctypes.POINTER(MrMaterial),
                       ctypes.POINTER(MrParticles), _vp, _i64, _f32, _vp, _i32, _vp, _vp, _vp]),
    "mpm_grid_update": (_i32, [ctypes.POINTER(MrGrid), _f32, _vp, _vp, _i64, _vp]),
    "mpm_g2p": (_i32, [ctypes.POINTER(MrGrid), ctypes.POINTER(MrParticles), _vp, _i64, _f32,
                       _vp, _i32, _vp, _vp, _vp, _vp]),
    "mpm_cell_sort": (_i32, [ctypes.POINTER(MrGrid), ctypes.POINTER(MrParticles), _vp, _vp,
                             _vp, _vp]),
    "mpm_cell_sort_ex": (_i32, [ctypes.POINTER(MrGrid), ctypes.POINTER(MrParticles), _vp, _vp,
                                _i32, _vp, _vp]),
    "mpm_workspace_bytes": (_i64, [ctypes.POINTER(MrGrid), _i64]),
    "mpm_cell_keys": (_i32, [ctypes.POINTER(MrGrid), ctypes.POINTER(MrParticles), _vp, _vp]),
    "mpm_step": (_i32, [ctypes.POINTER(MrGrid), ctypes.POINTER(MrMaterial),
                        ctypes.POINTER(MrParticles), _f32, _i32, _i32, _i32, _vp, _vp, _vp,
                        _vp, _vp, _vp]),
    "mpm_g2p2g": (_i32, [ctypes.POINTER(MrGrid), ctypes.POINTER(MrMaterial),
                         ctypes.POINTER(MrParticles), _f32, _vp, _vp, _i32, _vp, _vp, _vp]),
    "mr_timing_create": (_i32, [_i32, ctypes.POINTER(_vp)]),
    "mr_timing_destroy": (None, [_vp]),
    "mr_timing_reset": (_i32, [_vp]),
    "mr_timing_sample": (_i32, [_vp, ctypes.c_uint32, _i32]),
    "mr_timing_read": (_i32, [_vp, _i32, ctypes.POINTER(_i64), ctypes.POINTER(_f64)]),
    "mpm_step_workspace_bytes": (_i64, [ctypes.POINTER(MrGrid), _i64]),
    "rom_decoder_create": (_i32, [_i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _i32, _i32,
                                  ctypes.POINTER(_vp)]),
    "rom_decoder_destroy": (None, [_vp]),
    "rom_decoder_set_params": (_i32, [_vp, _vp, _i32, _vp]),
    "rom_decoder_autotune": (_i32, [_vp, _i32, _i64, _i32, _i32, _vp]),
    "rom_decoder_shape": (_i32, [_vp, _i32, _i32, _i64]),
    "rom_decoder_set_shape": (_i32, [_vp, _i32, _i32, _i64, _i32]),
    "mr_mfma_probe": (_i32, [_i32, _i32, _vp, _vp]),
    "rom_decode": (_i32, [_vp, _i32, _i64, _vp, _i64, _vp, _vp, _vp, _vp]),
    "rom_decode_jac": (_i32, [_vp, _i32, _i64, _vp, _i64, _vp, _i32, _vp, _vp, _vp, _vp, _vp,
                              _vp, _vp]),
    "rom_project": (_i32, [_vp, _i32, _i64, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _f64,
                           ctypes.POINTER(MrGnOpts), _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t,
                           _vp]),
    "rom_project_workspace_bytes": (_i64, [_vp, _i32, _i64, ctypes.POINTER(MrGnOpts)]),
    "rom_project_noalloc": (_i32, [_vp, _i32, _i64, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _f64,
                                   ctypes.POINTER(MrGnOpts), _vp, _vp, _vp, _vp, _vp, _vp]),
    "rom_create": (_i32, [_vp, ctypes.POINTER(MrGrid), ctypes.POINTER(MrRomConfig), _vp, _vp,
                          _vp, _vp, ctypes.POINTER(MrGnOpts), ctypes.POINTER(_vp)]),
    "rom_destroy": (None, [_vp]),
    "rom_step": (_i32, [_vp, _i32, _i64, _f64, _vp, _vp, _vp, _vp, _i32, _vp]),
    "rom_last_counts": (_i32, [_vp, _i32, ctypes.POINTER(_i64), ctypes.POINTER(_i64), _vp]),
    "rom_set_fields": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "rom_positions": (_i32, [_vp, _vp, _f64, _vp, _vp]),
    "rom_train_param_count": (_i64, [_i32, _i32, _i32, _i32]),
    "rom_trainer_create": (_i32, [_i32, _i32, _i32, _i32, _i32, _i64, _vp, _vp, _vp, _vp, _i32,
                                  ctypes.POINTER(_vp)]),
    "rom_trainer_destroy": (None, [_vp]),
    "rom_train_forward": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _i32, _i32, _f32, _vp, _vp, _vp,
                                 _vp]),
    "rom_train_backward": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "rom_train_loss": (_i32, [_i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _f32, _f32,
                              _vp, _vp, _vp, _vp, _vp]),
    "rom_adam_step": (_i32, [_i64, _vp, _vp, _vp, _vp, _f32, _f32, _f32, _f32, _i32, _vp]),
    "rom_encoder_layout": (_i32, [_i64, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i64),
                                  ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                                  ctypes.POINTER(_i64)]),
    "rom_encoder_forward": (_i32, [_i32, _i32, _i64, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                   _vp]),
    "rom_encoder_backward": (_i32, [_i32, _i32, _i64, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                    _vp, _vp, _i32, _vp]),
    "rom_trainer_set_deterministic": (_i32, [_vp, _i32]),
    "rom_train_gather": (_i32, [_i32, _i32, _i32, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                _vp, _vp, _vp]),
    "mr_sync_status": (_i32, [_vp, _vp, _i32, _vp]),
    "mr_version": (ctypes.c_char_p, []),
}

_lib = None


def load(path=LIB_PATH):
    """Loads libmpmrom.so and declares every entry point; raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libmpmrom.so is not built (expected at %s); "
                           "run __graft_entry__.build()" % path)
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(name, rc):
    if rc != MR_OK:
        raise MrError(name, rc)


def _ptr(t, dtype=None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError("expected dtype %s, got %s" % (dtype, t.dtype))
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Grid:
    def __init__(self, dim, n, dx, bound=3, floor_mode=FLOOR_STICKY, mu_friction=0.0,
                 gravity=(0.0, 0.0, 0.0)):
        self.dim, self.n, self.dx = dim, list(n), dx
        self.bound, self.floor_mode, self.mu_friction = bound, floor_mode, mu_friction
        self.gravity = list(gravity) + [0.0] * (3 - len(gravity))

    def c(self):
        n = self.n + [1] * (3 - len(self.n))
        return MrGrid(self.dim, (ctypes.c_int32 * 3)(*n), self.dx, self.bound, self.floor_mode,
                      self.mu_friction, (ctypes.c_float * 3)(*self.gravity))

    def nodes(self):
        k = 1
        for v in self.n:
            k *= v
        return k


class Particles:
    """Device SoA particle arrays: x, v (d, n); C, F (d*d, n); optional
    per-particle m, V0 (n,)."""

    def __init__(self, x, v=None, C=None, F=None, m=None, V0=None, m_uniform=0.0,
                 V0_uniform=0.0):
        self.x, self.v, self.C, self.F, self.m, self.V0 = x, v, C, F, m, V0
        self.m_uniform, self.V0_uniform = m_uniform, V0_uniform

    @property
    def n(self):
        return self.x.shape[-1]

    def c(self):
        f = torch.float32
        return MrParticles(self.n, _ptr(self.x, f), _ptr(self.v, f), _ptr(self.C, f),
                           _ptr(self.F, f), _ptr(self.m, f), _ptr(self.V0, f),
                           self.m_uniform, self.V0_uniform)


def workspace_bytes(grid, n):
    return int(load().mpm_workspace_bytes(ctypes.byref(grid.c()), n))


def new_workspace(grid, n, device="cuda"):
    return torch.empty(max(workspace_bytes(grid, n), 1), dtype=torch.uint8, device=device)


def mpm_p2g(grid, material, parts, grid_buf, dt, subset=None, flags=0, workspace=None,
            status=None, stream=None):
    lib = load()
    g, m, p = grid.c(), MrMaterial(*material), parts.c()
    ns = subset.numel() if subset is not None else parts.n
    _check("mpm_p2g", lib.mpm_p2g(ctypes.byref(g), ctypes.byref(m), ctypes.byref(p),
                                  _ptr(subset, torch.int32), ns, dt, _ptr(grid_buf, torch.float32),
                                  flags, _ptr(workspace), _ptr(status, torch.int32),
                                  _stream(stream)))


def mpm_grid_update(grid, dt, grid_buf, active=None, stream=None):
    lib = load()
    na = active.numel() if active is not None else 0
    _check("mpm_grid_update", lib.mpm_grid_update(ctypes.byref(grid.c()), dt,
                                                  _ptr(grid_buf, torch.float32),
                                                  _ptr(active, torch.int32), na, _stream(stream)))


def mpm_g2p(grid, parts, dt, grid_buf, subset=None, flags=0, x_trial=None, v_trial=None,
            status=None, stream=None):
    lib = load()
    p = parts.c()
    ns = subset.numel() if subset is not None else parts.n
    _check("mpm_g2p", lib.mpm_g2p(ctypes.byref(grid.c()), ctypes.byref(p),
                                  _ptr(subset, torch.int32), ns, dt,
                                  _ptr(grid_buf, torch.float32), flags,
                                  _ptr(x_trial, torch.float32), _ptr(v_trial, torch.float32),
                                  _ptr(status, torch.int32), _stream(stream)))


def mpm_cell_sort_ex(grid, parts, workspace, flags, perm_out=None, status=None, stream=None):
    lib = load()
    p = parts.c()
    _check("mpm_cell_sort_ex", lib.mpm_cell_sort_ex(ctypes.byref(grid.c()), ctypes.byref(p),
                                                    _ptr(perm_out, torch.int32), _ptr(workspace),
                                                    flags, _ptr(status, torch.int32),
                                                    _stream(stream)))


def mpm_cell_sort(grid, parts, workspace, perm_out=None, status=None, stream=None):
    lib = load()
    p = parts.c()
    _check("mpm_cell_sort", lib.mpm_cell_sort(ctypes.byref(grid.c()), ctypes.byref(p),
                                              _ptr(perm_out, torch.int32), _ptr(workspace),
                                              _ptr(status, torch.int32), _stream(stream)))


def mpm_cell_keys(grid, parts, keys_out, stream=None):
    lib = load()
    p = parts.c()
    _check("mpm_cell_keys", lib.mpm_cell_keys(ctypes.byref(grid.c()), ctypes.byref(p),
                                              _ptr(keys_out, torch.int32), _stream(stream)))


def mpm_step_workspace_bytes(grid, n):
    return int(load().mpm_step_workspace_bytes(ctypes.byref(grid.c()), n))


NO_VC_OUT = 32
DETERMINISTIC = 64
KC_NAMES = ["cell_sort", "p2g", "grid_update", "g2p", "g2p2g", "zero_grid"]


class Timing:
    """Launch timer (mr_timing_*): per-kernel-class launch counts and times."""

    def __init__(self, capacity=65536):
        h = ctypes.c_void_p()
        _check("mr_timing_create", load().mr_timing_create(capacity, ctypes.byref(h)))
        self.handle = h

    def reset(self):
        _check("mr_timing_reset", load().mr_timing_reset(self.handle))

    def sample(self, every, classes=None):
        """Record only every `every`-th launch of each class in `classes`
        (names from KC_NAMES; default all)."""
        names = KC_NAMES if classes is None else classes
        mask = 0
        for nm in names:
            mask |= 1 << KC_NAMES.index(nm)
        _check("mr_timing_sample", load().mr_timing_sample(self.handle, mask, every))

    def read(self):
        n = len(KC_NAMES)
        la = (_i64 * n)()
        ms = (_f64 * n)()
        _check("mr_timing_read", load().mr_timing_read(self.handle, n, la, ms))
        return {KC_NAMES[i]: (la[i], ms[i]) for i in range(n) if la[i] > 0}

    def close(self):
        if self.handle:
            load().mr_timing_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mpm_step(grid, material, parts, dt, n_steps, sort_every, flags, grid_buf, workspace,
             perm_accum=None, status=None, timing=None, stream=None):
    lib = load()
    p = parts.c()
    _check("mpm_step", lib.mpm_step(ctypes.byref(grid.c()), ctypes.byref(MrMaterial(*material)),
                                    ctypes.byref(p), dt, n_steps, sort_every, flags,
                                    _ptr(grid_buf, torch.float32), _ptr(workspace),
                                    _ptr(perm_accum, torch.int32), _ptr(status, torch.int32),
                                    timing.handle if timing is not None else None,
                                    _stream(stream)))


def mpm_g2p2g(grid, material, parts, dt, grid_in, grid_out, workspace, flags=0, status=None,
              stream=None):
    lib = load()
    p = parts.c()
    _check("mpm_g2p2g", lib.mpm_g2p2g(ctypes.byref(grid.c()), ctypes.byref(MrMaterial(*material)),
                                      ctypes.byref(p), dt, _ptr(grid_in, torch.float32),
                                      _ptr(grid_out, torch.float32), flags, _ptr(workspace),
                                      _ptr(status, torch.int32), _stream(stream)))


def flag_names(flags):
    """Names of the MR_FLAG_* bits set in an int (empty list for 0)."""
    names = [(FLAG_DOMAIN, "DOMAIN"), (FLAG_SINGULAR, "SINGULAR"), (FLAG_NOCONV, "NOCONV"),
             (FLAG_LINESEARCH, "LINESEARCH"), (FLAG_DRIFT, "DRIFT")]
    return [n for bit, n in names if int(flags) & bit]


def sync_status(flags_dev, stream=None):
    """Returns (code, host flags list) after synchronising the stream."""
    lib = load()
    n = flags_dev.numel()
    host = (ctypes.c_int32 * max(n, 1))()
    rc = lib.mr_sync_status(_stream(stream), _ptr(flags_dev, torch.int32), n, host)
    return rc, list(host)[:n]


def mfma_probe(blocks, iters, sink, stream=None):
    """Dense bf16 matrix-core loop (measurement aid): blocks x 4 x iters x 8
    x 16,384 FLOP; sink is a float32 device tensor of blocks x 256."""
    _check("mr_mfma_probe", load().mr_mfma_probe(blocks, iters, _ptr(sink, torch.float32),
                                                 _stream(stream)))


def version():
    return load().mr_version().decode()


def pack_params(weights, biases):
    """[W_0 (row-major), b_0, W_1, b_1, ...] as one float32 numpy array."""
    import numpy as np
    parts = []
    for W, b in zip(weights, biases):
        parts.append(np.asarray(W, dtype=np.float32).reshape(-1))
        parts.append(np.asarray(b, dtype=np.float32).reshape(-1))
    return np.ascontiguousarray(np.concatenate(parts))


class Decoder:
    """Owns an mr_decoder handle (rom_decoder_create / rom_decoder_destroy)."""

    def __init__(self, weights, biases, in_min, in_max, out_mean, out_std,
                 output_mode=OUT_DISPLACEMENT, precision=PREC_FP32):
        import numpy as np
        lib = load()
        self.d = int(np.asarray(out_mean).shape[0])
        self.width = int(np.asarray(weights[0]).shape[0])
        self.r = int(np.asarray(weights[0]).shape[1]) - self.d
        self.n_hidden = len(weights) - 1
        self.precision = precision
        params = pack_params(weights, biases)
        f = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.float32))
        self._keep = [params, f(in_min), f(in_max), f(out_mean), f(out_std)]
        h = ctypes.c_void_p()
        _check("rom_decoder_create", lib.rom_decoder_create(
            self.d, self.r, self.width, self.n_hidden,
            *[ctypes.c_void_p(a.ctypes.data) for a in self._keep],
            output_mode, precision, ctypes.byref(h)))
        self.handle = h

    def set_params(self, params, stream=None):
        """params: device float32 tensor in the packed layout."""
        _check("rom_decoder_set_params", load().rom_decoder_set_params(
            self.handle, _ptr(params, torch.float32), 1, _stream(stream)))

    def autotune(self, B, n, cfg_mask=7, reps=3, stream=None):
        """Times the decoder's launch shapes at B instances of n points
        (rom_decoder_autotune) and records the fastest in the decoder."""
        _check("rom_decoder_autotune", load().rom_decoder_autotune(self.handle, B, n, cfg_mask, reps,
                                                                   _stream(stream)))

    def shape(self, cfg, B, n):
        """Launch shape a configuration (1, 5 or 9) uses at B x n points."""
        return int(load().rom_decoder_shape(self.handle, cfg, B, n))

    def set_shape(self, cfg, B, n, shape):
        """Pins the launch shape of a configuration's size class
        (rom_decoder_set_shape)."""
        _check("rom_decoder_set_shape", load().rom_decoder_set_shape(self.handle, cfg, B, n, shape))

    def close(self):
        if self.handle:
            load().rom_decoder_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rom_decode(dec, X, xhat, x_out, idx=None, stream=None):
    """X: (d, n_ref) device float32; xhat: (B, r) float64; x_out (B, d, n)."""
    n = idx.numel() if idx is not None else X.shape[1]
    _check("rom_decode", load().rom_decode(dec.handle, xhat.shape[0], X.shape[1],
                                           _ptr(X, torch.float32), n, _ptr(idx, torch.int32),
                                           _ptr(xhat, torch.float64), _ptr(x_out, torch.float32),
                                           _stream(stream)))


def rom_decode_jac(dec, X, xhat, n=None, idx=None, idx_per_instance=0, vhat=None, x=None, F=None,
                   v=None, Jz=None, stream=None):
    if n is None:
        n = X.shape[1] if idx is None else idx.shape[-1]
    _check("rom_decode_jac", load().rom_decode_jac(
        dec.handle, xhat.shape[0], X.shape[1], _ptr(X, torch.float32), n, _ptr(idx, torch.int32),
        idx_per_instance, _ptr(xhat, torch.float64), _ptr(vhat, torch.float64),
        _ptr(x, torch.float32), _ptr(F, torch.float32), _ptr(v, torch.float32),
        _ptr(Jz, torch.float32), _stream(stream)))


def gn_opts(mode=POS_VEL, max_iter=3, max_backtrack=8, armijo_c=1e-4, damping=0.0, tol_step=0.0,
            proj_fp32=0):
    """proj_fp32: 0, 1 (positions in fp32) or 2 (positions and Jacobian)."""
    return MrGnOpts(mode, max_iter, max_backtrack, armijo_c, damping, tol_step, int(proj_fp32))


def rom_project_workspace_bytes(dec, B, ns, opts):
    n = load().rom_project_workspace_bytes(dec.handle, B, ns, ctypes.byref(opts))
    if n < 0:
        raise MrError("rom_project_workspace_bytes", n)
    return n


def rom_project(dec, X, sample_idx, x_trial, v_trial, xhat_n, xhat_prev, dt, opts, xhat_next,
                vhat_next, ns_per_instance=None, iters=None, resid=None, status=None,
                workspace=None, stream=None):
    """sample_idx (B, ns) int32; x_trial, v_trial (B, d, ns) float32;
    latents (B, r) float64; workspace: a uint8 device tensor of at least
    rom_project_workspace_bytes bytes (allocated here when None)."""
    B_, ns = sample_idx.shape
    if workspace is None:
        workspace = torch.empty(rom_project_workspace_bytes(dec, B_, ns, opts), dtype=torch.uint8,
                                device=sample_idx.device)
    _check("rom_project", load().rom_project(
        dec.handle, B_, X.shape[1], _ptr(X, torch.float32), ns, _ptr(sample_idx, torch.int32),
        _ptr(ns_per_instance, torch.int32), _ptr(x_trial, torch.float32),
        _ptr(v_trial, torch.float32), _ptr(xhat_n, torch.float64), _ptr(xhat_prev, torch.float64),
        dt, ctypes.byref(opts), _ptr(xhat_next, torch.float64), _ptr(vhat_next, torch.float64),
        _ptr(iters, torch.int32), _ptr(resid, torch.float64), _ptr(status, torch.int32),
        _ptr(workspace, torch.uint8), workspace.numel(), _stream(stream)))


def encoder_layout(in_len, r):
    """(n_conv, d_conv, n_params, act_floats, work_floats) of the encoder."""
    nc = _i32()
    dc, npar, act, work = _i64(), _i64(), _i64(), _i64()
    _check("rom_encoder_layout", load().rom_encoder_layout(
        in_len, r, ctypes.byref(nc), ctypes.byref(dc), ctypes.byref(npar), ctypes.byref(act),
        ctypes.byref(work)))
    return nc.value, dc.value, npar.value, act.value, work.value


def _host_f32(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    return a, ctypes.c_void_p(a.ctypes.data)


def encoder_forward(d, r, x, params, in_min, in_max, act, z, frame_idx=None, n=None,
                    stream=None):
    """x: device float32 [frames][in_len]; frame_idx: device int32 [n] or
    None (n = x.shape[0]); act: [n][act_floats]; z: [n][r]."""
    in_len = x.shape[-1]
    n = (frame_idx.numel() if frame_idx is not None else x.shape[0]) if n is None else n
    lo, plo = _host_f32(in_min)
    hi, phi = _host_f32(in_max)
    _check("rom_encoder_forward", load().rom_encoder_forward(
        d, r, in_len, n, _ptr(x, torch.float32), _ptr(frame_idx, torch.int32),
        _ptr(params, torch.float32), plo, phi, _ptr(act, torch.float32), _ptr(z, torch.float32),
        _stream(stream)))


def encoder_backward(d, r, x, params, in_min, in_max, act, dz, grad, work, frame_idx=None,
                     n=None, deterministic=False, stream=None):
    in_len = x.shape[-1]
    n = (frame_idx.numel() if frame_idx is not None else x.shape[0]) if n is None else n
    lo, plo = _host_f32(in_min)
    hi, phi = _host_f32(in_max)
    _check("rom_encoder_backward", load().rom_encoder_backward(
        d, r, in_len, n, _ptr(x, torch.float32), _ptr(frame_idx, torch.int32),
        _ptr(params, torch.float32), plo, phi, _ptr(act, torch.float32),
        _ptr(dz, torch.float32), _ptr(grad, torch.float32), _ptr(work, torch.float32),
        1 if deterministic else 0, _stream(stream)))


class Rom:
    """Owns an mr_rom handle (rom_create / rom_destroy)."""

    def __init__(self, dec, grid, X_all, E, n_samples, opts, seed, rho0, m_uniform=0.0,
                 m_all=None, model=NEO_HOOKEAN, nu=0.3, autotune=False,
                 quadrature=QUAD_LAGRANGIAN, quad_per_dim=0, newton_iters=0, newton_tol=0.0):
        lib = load()
        self.dec = dec
        self.B = E.numel()
        cfg = MrRomConfig(self.B, X_all.shape[1], int(n_samples.max().item()), seed, rho0,
                          m_uniform, model, nu, 1 if autotune else 0, quadrature, quad_per_dim,
                          newton_iters, newton_tol)
        self.opts = opts
        h = ctypes.c_void_p()
        _check("rom_create", lib.rom_create(dec.handle, ctypes.byref(grid.c()), ctypes.byref(cfg),
                                            _ptr(X_all, torch.float32), _ptr(m_all, torch.float32),
                                            _ptr(E, torch.float32), _ptr(n_samples, torch.int32),
                                            ctypes.byref(opts), ctypes.byref(h)))
        torch.cuda.synchronize()
        self.handle = h

    def step(self, n_steps, step0, dt, xhat, xhat_prev, vhat, status=None, use_graph=False,
             stream=None):
        _check("rom_step", load().rom_step(self.handle, n_steps, step0, dt,
                                           _ptr(xhat, torch.float64), _ptr(xhat_prev, torch.float64),
                                           _ptr(vhat, torch.float64), _ptr(status, torch.int32),
                                           1 if use_graph else 0, _stream(stream)))

    def set_fields(self, xhat0, vhat0, v0, stream=None):
        """Initial-condition correction fields (rom_set_fields); v0 is a
        (B, d) array of uniform initial velocities; xhat0=None turns them
        off."""
        if xhat0 is None:
            _check("rom_set_fields", load().rom_set_fields(self.handle, None, None, None,
                                                           _stream(stream)))
            return
        v = torch.as_tensor(np.asarray(v0, dtype=np.float32), device=xhat0.device).contiguous()
        _check("rom_set_fields", load().rom_set_fields(
            self.handle, _ptr(xhat0, torch.float64), _ptr(vhat0, torch.float64),
            _ptr(v, torch.float32), _stream(stream)))

    def positions(self, xhat, t, x_out, stream=None):
        """Every particle's position (caller order) at latents xhat, time t."""
        _check("rom_positions", load().rom_positions(self.handle, _ptr(xhat, torch.float64),
                                                     float(t), _ptr(x_out, torch.float32),
                                                     _stream(stream)))

    def last_counts(self, b=0, stream=None):
        q, a = ctypes.c_int64(), ctypes.c_int64()
        _check("rom_last_counts", load().rom_last_counts(self.handle, b, ctypes.byref(q),
                                                         ctypes.byref(a), _stream(stream)))
        return q.value, a.value

    def close(self):
        if self.handle:
            load().rom_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
