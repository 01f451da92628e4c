"""ctypes loader for the FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke entry point and the benchmark's CPU-baseline leg may
import this.  It takes plain numpy arrays (from the shared input generator) and
shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "marfa_oracle.c")


_DEPS = [_SRC, os.path.join(_HERE, "marfa_oracle.h"), os.path.join(_HERE, "orc_user.h")]


def build() -> str:
    """Compile the oracle with gcc (IEEE double arithmetic, no fast-math).
    ORC_USER_HEADER=/abs/path.h substitutes the user line shape and chi."""
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-Wall", "-o", _SO, _SRC, "-lm", "-lpthread"]
    user = os.environ.get("ORC_USER_HEADER")
    if user:
        cmd.insert(1, f'-DORC_USER_HEADER="{user}"')
    subprocess.run(cmd, check=True)
    return _SO


class _Lines(C.Structure):
    _fields_ = [("n", C.c_int64), ("nu0", C.c_void_p), ("S296", C.c_void_p),
                ("gamma_air", C.c_void_p), ("gamma_self", C.c_void_p), ("E_lower", C.c_void_p),
                ("n_air", C.c_void_p), ("delta_air", C.c_void_p), ("molar_mass", C.c_double)]


class _Layer(C.Structure):
    _fields_ = [("p_atm", C.c_double), ("T_K", C.c_double), ("p_self_atm", C.c_double),
                ("q_ratio", C.c_double)]


class _Request(C.Structure):
    _fields_ = [("nu_begin", C.c_double), ("nu_end", C.c_double), ("cutoff", C.c_double),
                ("shape", C.c_int32), ("chi", C.c_int32), ("out_kind", C.c_int32),
                ("level_table", C.c_int32), ("prune_rel", C.c_double), ("R", C.c_double),
                ("stencil", C.c_int32)]


class _State(C.Structure):
    _fields_ = [("S", C.c_double), ("gamma_L", C.c_double), ("alpha_D", C.c_double),
                ("nu_t", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < max(os.path.getmtime(p) for p in _DEPS):
            build()
        L = C.CDLL(_SO)
        d, i64, i32, vp = C.c_double, C.c_int64, C.c_int32, C.c_void_p
        L.orc_dawson.restype = d
        L.orc_dawson.argtypes = [d]
        L.orc_voigt_K.restype = d
        L.orc_voigt_K.argtypes = [d, d]
        L.orc_voigt_K_vec.argtypes = [i64, vp, vp, vp]
        L.orc_chi.restype = d
        L.orc_chi.argtypes = [i32, d]
        L.orc_user_chi_breaks.restype = i32
        L.orc_user_chi_breaks.argtypes = [C.c_void_p, i32]
        L.orc_stencil_of.restype = i32
        L.orc_stencil_of.argtypes = [C.POINTER(_Request), i32, i64, vp, vp]
        L.orc_shape.restype = d
        L.orc_shape.argtypes = [i32, d, d, d]
        L.orc_line_state_of.argtypes = [C.POINTER(_Lines), C.POINTER(_Layer), i64, C.POINTER(_State)]
        L.orc_line_states.argtypes = [C.POINTER(_Lines), C.POINTER(_Layer), vp, vp, vp, vp]
        L.orc_number_density.restype = d
        L.orc_number_density.argtypes = [C.POINTER(_Layer)]
        L.orc_direct.argtypes = [C.POINTER(_Lines), C.POINTER(_Layer), C.POINTER(_Request), vp, i64,
                                 vp, i32]
        L.orc_grid.argtypes = [C.POINTER(_Lines), C.POINTER(_Layer), C.POINTER(_Request), vp, i32]
        L.orc_mlp_forward.argtypes = [i32, vp, vp, vp, i64, vp]
        L.orc_mlp_loss_grad.argtypes = [i32, vp, vp, vp, vp, i64, vp, vp]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


class _Keep:
    """Holds the arrays a ctypes struct points into."""

    def __init__(self, lines):
        self.arrs = [np.ascontiguousarray(lines.nu0, np.float64),
                     np.ascontiguousarray(lines.S296, np.float32),
                     np.ascontiguousarray(lines.gamma_air, np.float32),
                     np.ascontiguousarray(lines.gamma_self, np.float32),
                     np.ascontiguousarray(lines.E_lower, np.float32),
                     np.ascontiguousarray(lines.n_air, np.float32),
                     np.ascontiguousarray(lines.delta_air, np.float32)]
        a = self.arrs
        self.s = _Lines(lines.n, *[_ptr(x) for x in a], float(lines.molar_mass))


def _layer(lay):
    p, T, ps, q = (float(v) for v in lay)
    return _Layer(p, T, ps, q)


def _request(nu_begin, nu_end, cutoff, shape=0, chi=0, out_kind=0, level_table=0, prune=0.0,
             R=48.0, stencil=3):
    return _Request(float(nu_begin), float(nu_end), float(cutoff), int(shape), int(chi),
                    int(out_kind), int(level_table), float(prune), float(R), int(stencil))


def dawson(x: float) -> float:
    return lib().orc_dawson(float(x))


def voigt_K(x, y):
    x = np.ascontiguousarray(np.broadcast_to(np.asarray(x, np.float64), np.broadcast(x, y).shape))
    y = np.ascontiguousarray(np.broadcast_to(np.asarray(y, np.float64), x.shape))
    out = np.empty(x.shape, np.float64)
    rc = lib().orc_voigt_K_vec(x.size, _ptr(x), _ptr(y), _ptr(out))
    assert rc == 0
    return out


def chi(kind: int, absd: float) -> float:
    return lib().orc_chi(int(kind), float(absd))


def user_chi_breaks() -> list:
    """Ascending |d| [cm^-1] where the compiled-in user chi or its slope jumps."""
    buf = np.zeros(16, np.float64)
    n = lib().orc_user_chi_breaks(_ptr(buf), 16)
    if n < 0:
        raise RuntimeError("orc_user_chi_breaks failed")
    return [float(v) for v in buf[:n]]


def stencil_of(l: int, m: int, stencil: int = 3, level_table: int = 0):
    """Coarse node indices and weights interpolating level-l node m from level l+1."""
    rq = _request(0.0, 1.0, 25.0, level_table=level_table, stencil=stencil)
    k = np.zeros(5, np.int64)
    w = np.zeros(5, np.float64)
    n = lib().orc_stencil_of(C.byref(rq), int(l), int(m), _ptr(k), _ptr(w))
    if n < 0:
        raise ValueError("invalid stencil request")
    return k[:n].copy(), w[:n].copy()


def shape(kind: int, d: float, gamma_L: float, alpha_D: float) -> float:
    return lib().orc_shape(int(kind), float(d), float(gamma_L), float(alpha_D))


def line_state(lines, layer, j: int):
    k = _Keep(lines)
    st = _State()
    lay = _layer(layer)
    lib().orc_line_state_of(C.byref(k.s), C.byref(lay), int(j), C.byref(st))
    return dict(S=st.S, gamma_L=st.gamma_L, alpha_D=st.alpha_D, nu_t=st.nu_t)


def line_states(lines, layer):
    """line_state for every line: dict of arrays S, gamma_L, alpha_D, nu_t."""
    k = _Keep(lines)
    lay = _layer(layer)
    out = {f: np.empty(lines.n, np.float64) for f in ("S", "gamma_L", "alpha_D", "nu_t")}
    rc = lib().orc_line_states(C.byref(k.s), C.byref(lay), *[_ptr(out[f]) for f in ("S", "gamma_L", "alpha_D", "nu_t")])
    assert rc == 0
    return out


def number_density(layer) -> float:
    lay = _layer(layer)
    return lib().orc_number_density(C.byref(lay))


def direct(lines, layer, nodes, threads: int = 8, **req) -> np.ndarray:
    """Definition: sum of every kept line within the cut-off at nu = nodes * 2^-11."""
    k = _Keep(lines)
    lay = _layer(layer)
    rq = _request(**req)
    nodes = np.ascontiguousarray(nodes, np.int64)
    out = np.empty(nodes.shape[0], np.float64)
    rc = lib().orc_direct(C.byref(k.s), C.byref(lay), C.byref(rq), _ptr(nodes), nodes.shape[0],
                          _ptr(out), int(threads))
    if rc != 0:
        raise ValueError(f"orc_direct rejected its input ({rc})")
    return out


def grid(lines, layer, threads: int = 8, **req) -> np.ndarray:
    """Eleven-grid method over [nu_begin, nu_end] on the 2^-11 lattice."""
    k = _Keep(lines)
    lay = _layer(layer)
    rq = _request(**req)
    n = int(round((rq.nu_end - rq.nu_begin) * 2048)) + 1
    out = np.empty(n, np.float64)
    rc = lib().orc_grid(C.byref(k.s), C.byref(lay), C.byref(rq), _ptr(out), int(threads))
    if rc != 0:
        raise ValueError(f"orc_grid rejected its input ({rc})")
    return out


def mlp_forward(widths, params, X) -> np.ndarray:
    w = np.ascontiguousarray(widths, np.int32)
    P = np.ascontiguousarray(params, np.float64)
    X = np.ascontiguousarray(X, np.float64)
    Y = np.empty((X.shape[0], int(w[-1])), np.float64)
    rc = lib().orc_mlp_forward(len(w) - 1, _ptr(w), _ptr(P), _ptr(X), X.shape[0], _ptr(Y))
    assert rc == 0
    return Y


def mlp_loss_grad(widths, params, X, target):
    w = np.ascontiguousarray(widths, np.int32)
    P = np.ascontiguousarray(params, np.float64)
    X = np.ascontiguousarray(X, np.float64)
    t = np.ascontiguousarray(target, np.float64)
    g = np.empty_like(P)
    loss = C.c_double()
    rc = lib().orc_mlp_loss_grad(len(w) - 1, _ptr(w), _ptr(P), _ptr(X), _ptr(t), X.shape[0],
                                 C.byref(loss), _ptr(g))
    assert rc == 0
    return loss.value, g
