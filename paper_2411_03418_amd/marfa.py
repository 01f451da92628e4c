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
LIB_PATH = os.path.join(_HERE, "libmarfa.so")

OK, E_INVALID, E_NOMEM, E_DEVICE, E_UNSUPPORTED, E_STATE = 0, -1, -2, -3, -4, -5
SHAPES = {"voigt": 0, "lorentz": 1, "doppler": 2}
CHIS = {"none": 0, "tonkov": 1}
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
                ("fp64", C.c_int32), ("reserved", C.c_int32 * 4)]


class Stats(C.Structure):
    _fields_ = [("points_per_layer", C.c_int64), ("n_layers", C.c_int32), ("lines_total", C.c_int64),
                ("lines_kept", C.c_int64), ("pairs_level", C.c_int64 * 11), ("pairs_core", C.c_int64),
                ("pairs_wing", C.c_int64), ("pairs_band", C.c_int64), ("wing_terms", C.c_int64),
                ("level_nodes", C.c_int64), ("iters_level", C.c_int64 * 11),
                ("band_iters_level", C.c_int64 * 11)]


class Timing(C.Structure):
    _fields_ = [("prep_ms", C.c_float), ("level_ms", C.c_float), ("cascade_ms", C.c_float),
                ("total_ms", C.c_float)]


class Tiles(C.Structure):
    _fields_ = [("item_nodes", C.c_int32), ("blocks_per_cu", C.c_int32), ("tuned", C.c_int32),
                ("wave_nodes", C.c_int32 * 11), ("tune_ms", C.c_float)]


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
        L.marfa_execute_timed.argtypes = [vp, vp, i64, vp, C.POINTER(Timing)]
        L.marfa_plan_destroy.argtypes = [vp]
        L.marfa_plan_destroy.restype = None
        L.marfa_status_string.argtypes = [i32]
        L.marfa_status_string.restype = C.c_char_p
        L.marfa_last_error.argtypes = [C.c_char_p, C.c_size_t]
        L.marfa_voigt_eval.argtypes = [i32, i64, vp, vp, vp, i32]
        for f in ("marfa_plan_create", "marfa_plan_points", "marfa_execute", "marfa_execute_layers",
                  "marfa_plan_count", "marfa_plan_tiles", "marfa_execute_timed", "marfa_plan_tune", "marfa_last_error",
                  "marfa_voigt_eval"):
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
                 prune=0.0, R=48, level_table=0, fp64=False, device=0):
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
                     CHIS.get(chi, chi), OUTS.get(out, out), 0, float(prune), float(R), int(level_table),
                     1 if fp64 else 0, (C.c_int32 * 4)(0, 0, 0, 0))
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
                    band_iters_level=list(s.band_iters_level))

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

    def tune(self, out=None, stream=None):
        """Autotune the level kernel's tiles on the device (synchronous);
        `out` is scratch output.  Returns the chosen tiles."""
        out = self._out(out, self.n_layers)
        _check(lib().marfa_plan_tune(self._h, C.c_void_p(out.data_ptr()), out.stride(0),
                                     _stream_handle(stream, self.device)))
        return self.tiles()

    def close(self):
        if getattr(self, "_h", None):
            lib().marfa_plan_destroy(self._h)
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
