"""Python binding of the eleven-grid HIP library (argument marshalling only).

Every step of the computation runs in the gfx950 kernels of ``libmarfa.so``;
this module only converts arrays and tensors to the plain pointers of the C ABI
declared in ``include/marfa.h``.  PyTorch provides device memory and streams.
If the library has not been built this module raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# MARFA_LIB selects another build of the library (e.g. one with a different user line shape)
LIB_PATH = os.environ.get("MARFA_LIB") or os.path.join(_HERE, "libmarfa.so")

OK, E_INVALID, E_NOMEM, E_DEVICE, E_UNSUPPORTED, E_STATE, E_IO = 0, -1, -2, -3, -4, -5, -6
PTBIN_NT = 20481          # values per PT-table record (Appendix A)
PTBIN_TRUNCATE = 1
SHAPES = {"voigt": 0, "lorentz": 1, "doppler": 2, "user": 3}
EVALS = {"plain": 0, "surrogate": 1}
CHIS = {"none": 0, "tonkov": 1, "user": 2}
OUTS = {"sigma": 0, "k": 1}


class MarfaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class Lines(C.Structure):
    _fields_ = [("n", C.c_int64), ("nu0", C.c_void_p), ("S296", C.c_void_p), ("gamma_air", C.c_void_p),
                ("gamma_self", C.c_void_p), ("E_lower", C.c_void_p), ("n_air", C.c_void_p),
                ("mol_iso", C.c_void_p), ("delta_air", C.c_void_p), ("molar_mass_g", C.c_double)]


class Layer(C.Structure):
    _fields_ = [("p_atm", C.c_double), ("T_K", C.c_double), ("p_self_atm", C.c_double), ("q_ratio", C.c_double)]


class Request(C.Structure):
    _fields_ = [("nu_begin", C.c_double), ("nu_end", C.c_double), ("cutoff", C.c_double),
                ("shape", C.c_int32), ("chi", C.c_int32), ("out_kind", C.c_int32), ("eval", C.c_int32),
                ("prune_rel", C.c_double), ("R", C.c_double), ("level_table", C.c_int32),
                ("fp64", C.c_int32), ("stencil", C.c_int32), ("reserved", C.c_int32 * 3)]


class Stats(C.Structure):
    _fields_ = [("points_per_layer", C.c_int64), ("n_layers", C.c_int32), ("lines_total", C.c_int64),
                ("lines_kept", C.c_int64), ("pairs_level", C.c_int64 * 11), ("pairs_core", C.c_int64),
                ("pairs_wing", C.c_int64), ("pairs_band", C.c_int64), ("wing_terms", C.c_int64),
                ("level_nodes", C.c_int64), ("iters_level", C.c_int64 * 11),
                ("band_iters_level", C.c_int64 * 11), ("flops_per_eval", C.c_double),
                ("flops_per_core", C.c_double), ("flops_per_term", C.c_double), ("flops_per_band", C.c_double),
                ("flops_per_cascade", C.c_double), ("flops_level", C.c_double), ("flops_cascade", C.c_double),
                ("bytes_level", C.c_double), ("bytes_cascade", C.c_double)]


class Timing(C.Structure):
    _fields_ = [("prep_ms", C.c_float), ("level_ms", C.c_float), ("cascade_ms", C.c_float),
                ("total_ms", C.c_float)]


class Tiles(C.Structure):
    _fields_ = [("item_nodes", C.c_int32), ("blocks_per_cu", C.c_int32), ("tuned", C.c_int32),
                ("wave_nodes", C.c_int32 * 11), ("tune_ms", C.c_float)]


class SampleCfg(C.Structure):
    _fields_ = [("nu_lo", C.c_double), ("nu_hi", C.c_double), ("T_lo", C.c_double), ("T_hi", C.c_double),
                ("molar_mass_g", C.c_double)]


class TrainCfg(C.Structure):
    _fields_ = [("n_train", C.c_int64), ("n_val", C.c_int64), ("epochs", C.c_int32), ("batch", C.c_int32),
                ("lr_max", C.c_float), ("lr_min", C.c_float), ("seed", C.c_uint64), ("loss_power", C.c_int32),
                ("reserved", C.c_int32)]


class TrainReport(C.Structure):
    _fields_ = [("train_loss", C.c_float), ("val_loss", C.c_float), ("val_max_abs", C.c_float),
                ("val_mean_abs", C.c_float), ("ms", C.c_float), ("steps", C.c_int64), ("x_max", C.c_double)]


N_PARAMS = 12801
MLP_WIDTHS = (3, 64, 64, 64, 64, 1)

_lib = None


def lib():
    """Load libmarfa.so; raise if it is missing (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.marfa_plan_create.argtypes = [C.POINTER(vp), C.POINTER(Lines), C.POINTER(Layer), i32,
                                        C.POINTER(Request), i32]
        L.marfa_plan_points.argtypes = [vp, C.POINTER(i64)]
        L.marfa_execute.argtypes = [vp, vp, i64, vp]
        L.marfa_execute_layers.argtypes = [vp, i32, i32, vp, i64, vp]
        L.marfa_plan_count.argtypes = [vp, C.POINTER(Stats)]
        L.marfa_plan_tiles.argtypes = [vp, C.POINTER(Tiles)]
        L.marfa_plan_tune.argtypes = [vp, vp, i64, vp]
        L.marfa_plan_set_tiles.argtypes = [vp, C.POINTER(Tiles)]
        L.marfa_plan_set_tiles.restype = C.c_int32
        L.marfa_execute_timed.argtypes = [vp, vp, i64, vp, C.POINTER(Timing)]
        L.marfa_plan_destroy.argtypes = [vp]
        L.marfa_plan_destroy.restype = None
        L.marfa_status_string.argtypes = [i32]
        L.marfa_status_string.restype = C.c_char_p
        L.marfa_last_error.argtypes = [C.c_char_p, C.c_size_t]
        L.marfa_voigt_eval.argtypes = [i32, i64, vp, vp, vp, i32]
        u64, f32p = C.c_uint64, C.POINTER(C.c_float)
        L.marfa_surrogate_create.argtypes = [C.POINTER(vp), i32, C.c_double, u64, i32]
        L.marfa_surrogate_set_params.argtypes = [vp, vp, i64]
        L.marfa_surrogate_get_params.argtypes = [vp, vp, i64]
        L.marfa_surrogate_load.argtypes = [vp, vp, i64, C.c_double]
        L.marfa_surrogate_save.argtypes = [vp, vp, i64, C.POINTER(C.c_double)]
        L.marfa_surrogate_forward.argtypes = [vp, vp, i64, vp, vp]
        L.marfa_surrogate_loss_grad.argtypes = [vp, vp, vp, i64, f32p, vp]
        L.marfa_surrogate_loss_grad_noalloc.argtypes = [vp, vp, vp, i64, vp, vp]
        L.marfa_surrogate_make_samples.argtypes = [vp, C.POINTER(SampleCfg), u64, i64, vp, vp, vp]
        L.marfa_surrogate_train.argtypes = [vp, C.POINTER(SampleCfg), C.POINTER(TrainCfg), C.POINTER(TrainReport)]
        L.marfa_surrogate_destroy.argtypes = [vp]
        L.marfa_surrogate_destroy.restype = None
        L.marfa_plan_set_surrogate.argtypes = [vp, vp]
        L.marfa_plan_set_eval.argtypes = [vp, i32]
        L.marfa_ptbin_write.argtypes = [C.c_char_p, vp, i64, C.c_double, i32, vp, i32, C.POINTER(i32)]
        L.marfa_linedb_count.argtypes = [C.c_char_p, C.POINTER(i64)]
        L.marfa_linedb_read.argtypes = [C.c_char_p, i64, i64, vp, vp, vp, vp, vp, vp, vp, vp]
        L.marfa_linedb_write.argtypes = [C.c_char_p, C.POINTER(Lines)]
        for f in ("marfa_surrogate_create", "marfa_surrogate_set_params", "marfa_surrogate_get_params",
                  "marfa_surrogate_load", "marfa_surrogate_save",
                  "marfa_surrogate_forward", "marfa_surrogate_loss_grad", "marfa_surrogate_loss_grad_noalloc",
                  "marfa_surrogate_make_samples",
                  "marfa_surrogate_train", "marfa_plan_set_surrogate", "marfa_plan_set_eval"):
            getattr(L, f).restype = C.c_int32
        for f in ("marfa_plan_create", "marfa_plan_points", "marfa_execute", "marfa_execute_layers",
                  "marfa_plan_count", "marfa_plan_tiles", "marfa_execute_timed", "marfa_plan_tune", "marfa_last_error",
                  "marfa_voigt_eval", "marfa_ptbin_write", "marfa_linedb_count", "marfa_linedb_read",
                  "marfa_linedb_write"):
            getattr(L, f).restype = C.c_int32
        _lib = L
    return _lib


def _check(status):
    if status != OK:
        buf = C.create_string_buffer(512)
        lib().marfa_last_error(buf, 512)
        raise MarfaError(status, buf.value.decode(errors="replace") or lib().marfa_status_string(status).decode())


def _ptr(a):
    return C.c_void_p(a.ctypes.data) if a is not None else C.c_void_p(0)


def _stream_handle(stream, device):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return C.c_void_p(stream.cuda_stream)


class Plan:
    """A computation plan: line list + PT layers + request, resident on one GPU.

    lines: an object with arrays nu0 (f8), S296, gamma_air, gamma_self, E_lower,
    n_air, delta_air (f4), mol_iso (i4) and attribute molar_mass.
    layers: array [n, 4] of (p_atm, T_K, p_self_atm, q_ratio).
    """

    def __init__(self, lines, layers, *, nu_begin, nu_end, cutoff, shape="voigt", chi="none", out="sigma",
                 prune=0.0, R=48, level_table=0, fp64=False, stencil=3, eval="plain", device=0):
        L = lib()
        self._arrs = [np.ascontiguousarray(lines.nu0, np.float64),
                      np.ascontiguousarray(lines.S296, np.float32),
                      np.ascontiguousarray(lines.gamma_air, np.float32),
                      np.ascontiguousarray(lines.gamma_self, np.float32),
                      np.ascontiguousarray(lines.E_lower, np.float32),
                      np.ascontiguousarray(lines.n_air, np.float32),
                      np.ascontiguousarray(lines.mol_iso, np.int32),
                      np.ascontiguousarray(lines.delta_air, np.float32)]
        a = self._arrs
        n = int(a[0].shape[0])
        for x in a[1:]:
            if x.shape[0] != n:
                raise ValueError("line arrays differ in length")
        ls = Lines(n, *[_ptr(x) for x in a], float(lines.molar_mass))
        lay = np.ascontiguousarray(np.asarray(layers, np.float64).reshape(-1, 4))
        lays = (Layer * lay.shape[0])(*[Layer(*row) for row in lay])
        rq = Request(float(nu_begin), float(nu_end), float(cutoff), SHAPES.get(shape, shape),
                     CHIS.get(chi, chi), OUTS.get(out, out), EVALS.get(eval, eval), float(prune), float(R),
                     int(level_table),
                     1 if fp64 else 0, int(stencil), (C.c_int32 * 3)(0, 0, 0))
        h = C.c_void_p()
        _check(L.marfa_plan_create(C.byref(h), C.byref(ls), lays, lay.shape[0], C.byref(rq), int(device)))
        self._h = h
        self._arrs = None
        self.device = int(device)
        self.n_layers = int(lay.shape[0])
        self.fp64 = bool(fp64)
        p = C.c_int64()
        _check(L.marfa_plan_points(self._h, C.byref(p)))
        self.points = int(p.value)

    def _out(self, out, n_layers):
        import torch
        dt = torch.float64 if self.fp64 else torch.float32
        if out is None:
            out = torch.empty((n_layers, self.points), dtype=dt, device=f"cuda:{self.device}")
        if out.dtype != dt or out.dim() != 2 or out.shape[0] < n_layers or out.shape[1] < self.points:
            raise ValueError("output tensor has the wrong dtype or shape")
        if out.stride(1) != 1:
            raise ValueError("output rows must be contiguous")
        return out

    def execute(self, out=None, stream=None):
        """All layers into out [n_layers, >=points] (allocated if None); asynchronous."""
        out = self._out(out, self.n_layers)
        _check(lib().marfa_execute(self._h, C.c_void_p(out.data_ptr()), out.stride(0),
                                   _stream_handle(stream, self.device)))
        return out

    def execute_layers(self, first, count, out=None, stream=None):
        out = self._out(out, count)
        _check(lib().marfa_execute_layers(self._h, int(first), int(count), C.c_void_p(out.data_ptr()),
                                          out.stride(0), _stream_handle(stream, self.device)))
        return out

    def count(self):
        s = Stats()
        _check(lib().marfa_plan_count(self._h, C.byref(s)))
        return dict(points_per_layer=s.points_per_layer, n_layers=s.n_layers, lines_total=s.lines_total,
                    lines_kept=s.lines_kept, pairs_level=list(s.pairs_level), pairs_core=s.pairs_core,
                    pairs_wing=s.pairs_wing, pairs_band=s.pairs_band, wing_terms=s.wing_terms,
                    level_nodes=s.level_nodes, iters_level=list(s.iters_level),
                    band_iters_level=list(s.band_iters_level), flops_per_eval=s.flops_per_eval,
                    flops_per_core=s.flops_per_core, flops_per_term=s.flops_per_term,
                    flops_per_band=s.flops_per_band, flops_per_cascade=s.flops_per_cascade,
                    flops_level=s.flops_level, flops_cascade=s.flops_cascade, bytes_level=s.bytes_level,
                    bytes_cascade=s.bytes_cascade)

    def execute_timed(self, out=None, stream=None):
        """Run all layers as three stage graphs with HIP events between them on
        the launch stream; synchronous; returns (out, stage durations in ms)."""
        out = self._out(out, self.n_layers)
        t = Timing()
        _check(lib().marfa_execute_timed(self._h, C.c_void_p(out.data_ptr()), out.stride(0),
                                         _stream_handle(stream, self.device), C.byref(t)))
        return out, dict(prep_ms=t.prep_ms, level_ms=t.level_ms, cascade_ms=t.cascade_ms, total_ms=t.total_ms)

    def tiles(self):
        t = Tiles()
        _check(lib().marfa_plan_tiles(self._h, C.byref(t)))
        return dict(item_nodes=t.item_nodes, blocks_per_cu=t.blocks_per_cu, tuned=bool(t.tuned),
                    wave_nodes=list(t.wave_nodes), tune_ms=float(t.tune_ms))

    def set_tiles(self, tiles):
        """Use tile parameters from an earlier tune (dict as returned by tiles())."""
        t = Tiles(int(tiles["item_nodes"]), int(tiles["blocks_per_cu"]), 0,
                  (C.c_int32 * 11)(*[int(w) for w in tiles["wave_nodes"]]), 0.0)
        _check(lib().marfa_plan_set_tiles(self._h, C.byref(t)))
        return self.tiles()

    def tune(self, out=None, stream=None):
        """Autotune the level kernel's tiles on the device (synchronous);
        `out` is scratch output.  Returns the chosen tiles."""
        out = self._out(out, self.n_layers)
        _check(lib().marfa_plan_tune(self._h, C.c_void_p(out.data_ptr()), out.stride(0),
                                     _stream_handle(stream, self.device)))
        return self.tiles()

    def set_surrogate(self, surrogate):
        """Attach a trained Surrogate (None detaches); it evaluates the line
        shapes while the plan's eval is "surrogate" (see set_eval)."""
        _check(lib().marfa_plan_set_surrogate(self._h, surrogate._h if surrogate is not None else None))
        self._surrogate = surrogate

    def set_eval(self, eval):
        """Line-shape evaluation: "plain" or "surrogate" (the attached network)."""
        _check(lib().marfa_plan_set_eval(self._h, EVALS.get(eval, eval)))

    def close(self):
        if getattr(self, "_h", None):
            lib().marfa_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _sample_cfg(nu_lo, nu_hi, T_lo, T_hi, molar_mass=44.0):
    return SampleCfg(float(nu_lo), float(nu_hi), float(T_lo), float(T_hi), float(molar_mass))


class Surrogate:
    """The learned line shape (see marfa_surrogate_* in include/marfa.h).

    Features and targets are device tensors: X [n, 3] float32, T [n] float32.
    """

    def __init__(self, chi="tonkov", cutoff=125.0, seed=1, device=0):
        h = C.c_void_p()
        _check(lib().marfa_surrogate_create(C.byref(h), CHIS.get(chi, chi), float(cutoff), int(seed), int(device)))
        self._h = h
        self.device = int(device)
        self.chi = chi
        self.cutoff = float(cutoff)
        self.report = None

    def get_params(self):
        p = np.empty(N_PARAMS, np.float32)
        _check(lib().marfa_surrogate_get_params(self._h, _ptr(p), N_PARAMS))
        return p

    def set_params(self, params):
        """Replace the parameters; the library first waits for the device's
        queued work, so launches already enqueued use the old weights."""
        p = np.ascontiguousarray(params, np.float32)
        _check(lib().marfa_surrogate_set_params(self._h, _ptr(p), p.size))

    def save(self, path):
        """Write the trained network -- parameters, x_max (the largest |x| of
        its training distribution), chi and cut-off -- to an .npz file."""
        p = np.empty(N_PARAMS, np.float32)
        x_max = C.c_double()
        _check(lib().marfa_surrogate_save(self._h, _ptr(p), N_PARAMS, C.byref(x_max)))
        np.savez(path, params=p, x_max=np.float64(x_max.value), chi=np.int32(CHIS.get(self.chi, self.chi)),
                 cutoff=np.float64(self.cutoff))

    @classmethod
    def load(cls, path, device=0):
        """A network written by save(), ready to attach to plans."""
        with np.load(path) as z:
            s = cls(chi=int(z["chi"]), cutoff=float(z["cutoff"]), device=device)
            p = np.ascontiguousarray(z["params"], np.float32)
            _check(lib().marfa_surrogate_load(s._h, _ptr(p), p.size, float(z["x_max"])))
        return s

    def forward(self, X, stream=None):
        import torch
        X = X.contiguous()
        if X.dtype != torch.float32 or X.dim() != 2 or X.shape[1] != 3:
            raise ValueError("X must be float32 [n, 3]")
        out = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
        _check(lib().marfa_surrogate_forward(self._h, C.c_void_p(X.data_ptr()), X.shape[0],
                                             C.c_void_p(out.data_ptr()), _stream_handle(stream, self.device)))
        return out

    def loss_grad(self, X, T):
        import torch
        torch.cuda.synchronize(self.device)
        X, T = X.contiguous(), T.contiguous()
        g = np.empty(N_PARAMS, np.float32)
        loss = C.c_float()
        _check(lib().marfa_surrogate_loss_grad(self._h, C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()),
                                               X.shape[0], C.byref(loss), _ptr(g)))
        return float(loss.value), g

    def loss_grad_noalloc(self, X, T, out, stream=None):
        """Gradient and loss into the caller's device tensor out (float32,
        N_PARAMS + 1 values: the gradient, then the mean squared error);
        allocates nothing, asynchronous on `stream`; n <= 4096 samples."""
        if not (X.is_contiguous() and T.is_contiguous() and out.is_contiguous()):
            raise ValueError("X, T and out must be contiguous")
        if str(out.dtype) != "torch.float32" or out.numel() != N_PARAMS + 1:
            raise ValueError("out must be float32 with N_PARAMS + 1 elements")
        _check(lib().marfa_surrogate_loss_grad_noalloc(self._h, C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()),
                                                       X.shape[0], C.c_void_p(out.data_ptr()),
                                                       _stream_handle(stream, self.device)))
        return out

    def make_samples(self, n, seed, nu_lo=375.0, nu_hi=2625.0, T_lo=150.0, T_hi=740.0, molar_mass=44.0,
                     stream=None):
        import torch
        X = torch.empty((n, 3), dtype=torch.float32, device=f"cuda:{self.device}")
        T = torch.empty(n, dtype=torch.float32, device=f"cuda:{self.device}")
        cfg = _sample_cfg(nu_lo, nu_hi, T_lo, T_hi, molar_mass)
        _check(lib().marfa_surrogate_make_samples(self._h, C.byref(cfg), int(seed), int(n),
                                                  C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()),
                                                  _stream_handle(stream, self.device)))
        return X, T

    def train(self, n_train=10_000_000, n_val=1_000_000, epochs=20, batch=8192, lr_max=2e-3, lr_min=1e-6,
              seed=4, nu_lo=375.0, nu_hi=2625.0, T_lo=150.0, T_hi=740.0, molar_mass=44.0, loss_power=2):
        import torch
        torch.cuda.synchronize(self.device)
        sc = _sample_cfg(nu_lo, nu_hi, T_lo, T_hi, molar_mass)
        tc = TrainCfg(int(n_train), int(n_val), int(epochs), int(batch), float(lr_max), float(lr_min), int(seed),
                      int(loss_power), 0)
        r = TrainReport()
        _check(lib().marfa_surrogate_train(self._h, C.byref(sc), C.byref(tc), C.byref(r)))
        self.report = dict(train_loss=r.train_loss, val_loss=r.val_loss, val_max_abs=r.val_max_abs,
                           val_mean_abs=r.val_mean_abs, ms=r.ms, steps=r.steps, x_max=r.x_max)
        return self.report

    def fit(self, nu_lo, nu_hi, T_lo, T_hi, molar_mass=44.0, n_train=20_000_000, n_val=1_000_000, epochs=300,
            fine_epochs=100, batch=16384, lr=3e-3, seed=4):
        """Two-stage training: mean squared error, then a fourth-power stage
        at a tenth of the learning rate that weights the largest errors.
        20M samples by default: on the 100-layer tables the worst sampled
        nodes are 5.7e-4 (200k lines) and 9.1e-4 (2M lines) from the direct
        sum, against 8.3e-4 and 1.1-1.3e-3 with 10M."""
        rng = dict(nu_lo=nu_lo, nu_hi=nu_hi, T_lo=T_lo, T_hi=T_hi, molar_mass=molar_mass)
        r1 = self.train(n_train=n_train, n_val=n_val, epochs=epochs, batch=batch, lr_max=lr, lr_min=lr * 1e-3,
                        seed=seed, **rng)
        if fine_epochs <= 0:
            return r1
        r2 = self.train(n_train=n_train, n_val=n_val, epochs=fine_epochs, batch=batch, lr_max=lr / 10,
                        lr_min=lr * 1e-3, seed=seed, loss_power=4, **rng)
        r2 = dict(r2, ms=r1["ms"] + r2["ms"], steps=r1["steps"] + r2["steps"])
        self.report = r2
        return r2

    def close(self):
        if getattr(self, "_h", None):
            lib().marfa_surrogate_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def voigt_eval(x, y, fp64=False, device=0):
    """K(x, y) through the device line-shape code (tests)."""
    x = np.ascontiguousarray(x, np.float64).ravel()
    y = np.ascontiguousarray(np.broadcast_to(np.asarray(y, np.float64), x.shape)).ravel()
    out = np.empty_like(x)
    _check(lib().marfa_voigt_eval(int(device), x.shape[0], _ptr(x), _ptr(y), _ptr(out), 1 if fp64 else 0))
    return out


def record_number(nu: float) -> int:
    """Appendix A: the record holding wavenumber nu is int(nu/10)."""
    return int(nu / 10.0)


def write_ptbin(path, values, nu_begin, truncate=True, stream=None) -> int:
    """Write the PT-table records (Appendix A) covered by one layer's spectrum.

    values: a 1-D float32 torch tensor on a GPU (e.g. a row of Plan.execute's
    output) or a numpy float32 array, holding the spectrum at
    nu_begin + i / 2048 cm^-1.  Returns the number of records written.
    """
    n = C.c_int32(0)
    flags = PTBIN_TRUNCATE if truncate else 0
    if isinstance(values, np.ndarray):
        v = np.ascontiguousarray(values, np.float32).ravel()
        _check(lib().marfa_ptbin_write(os.fsencode(path), _ptr(v), v.shape[0], float(nu_begin), 0, None, flags,
                                       C.byref(n)))
    else:
        import torch
        if values.dtype != torch.float32 or not values.is_cuda or values.dim() != 1 or values.stride(0) != 1:
            raise ValueError("values must be a contiguous 1-D float32 GPU tensor or a numpy array")
        dev = values.device.index
        with torch.cuda.device(dev):
            _check(lib().marfa_ptbin_write(os.fsencode(path), C.c_void_p(values.data_ptr()), values.shape[0],
                                           float(nu_begin), 1, _stream_handle(stream, dev), flags, C.byref(n)))
    return n.value


def ptbin_name(layer_number: int) -> str:
    """Appendix A file name: the 1-based layer number padded with '_' to three characters."""
    return f"{layer_number:_<3d}.ptbin"


def write_pt_table(out, directory, nu_begin, stream=None) -> list:
    """One .ptbin file per layer (rows of out), named by 1-based layer number.
    Records hold single precision (Appendix A): a double-precision output is
    rounded to float32 on the device first."""
    os.makedirs(directory, exist_ok=True)
    paths = []
    for i in range(out.shape[0]):
        row = out[i]
        if not isinstance(row, np.ndarray):
            import torch
            row = row.to(torch.float32).contiguous()
        p = os.path.join(directory, ptbin_name(i + 1))
        write_ptbin(p, row, nu_begin, truncate=True, stream=stream)
        paths.append(p)
    return paths


def read_line_db(path, first=0, count=None, molar_mass=44.0):
    """Line records of an Appendix B database file, as a synth.LineList."""
    from .synth import LineList
    L = lib()
    n = C.c_int64(0)
    _check(L.marfa_linedb_count(os.fsencode(path), C.byref(n)))
    if count is None:
        count = n.value - first
    arrs = [np.empty(count, np.float64)] + [np.empty(count, np.float32) for _ in range(5)] + \
           [np.empty(count, np.int32), np.empty(count, np.float32)]
    _check(L.marfa_linedb_read(os.fsencode(path), int(first), int(count), *[_ptr(a) for a in arrs]))
    return LineList(*arrs, molar_mass=molar_mass)


def write_line_db(path, lines):
    """Write lines (any object with the LineList arrays) as Appendix B records."""
    a = [np.ascontiguousarray(lines.nu0, np.float64), np.ascontiguousarray(lines.S296, np.float32),
         np.ascontiguousarray(lines.gamma_air, np.float32), np.ascontiguousarray(lines.gamma_self, np.float32),
         np.ascontiguousarray(lines.E_lower, np.float32), np.ascontiguousarray(lines.n_air, np.float32),
         np.ascontiguousarray(lines.mol_iso, np.int32), np.ascontiguousarray(lines.delta_air, np.float32)]
    ls = Lines(int(a[0].shape[0]), *[_ptr(x) for x in a], float(getattr(lines, "molar_mass", 44.0)))
    _check(lib().marfa_linedb_write(os.fsencode(path), C.byref(ls)))
