"""Host-side checks of the C ABI: the library loads, exports every declared
entry point, and rejects invalid input before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2411_03418_amd import marfa, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "marfa.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(marfa_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 10
    L = C.CDLL(marfa.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n


def test_status_strings():
    L = marfa.lib()
    assert L.marfa_status_string(0) == b"ok"
    assert L.marfa_status_string(-1) == b"invalid argument"
    assert L.marfa_status_string(-3) == b"device error"
    assert L.marfa_status_string(-6) == b"file error"


def _plan(**kw):
    lines = synth.make_lines(5, 995.0, 1015.0, 1)
    layers = kw.pop("layers", [[1.0, 296.0, 1.0, 0.0]])
    req = dict(nu_begin=1000.0, nu_end=1001.0, cutoff=25.0)
    req.update(kw)
    return marfa.Plan(lines, layers, **req)


@pytest.mark.parametrize("kw", [
    dict(nu_begin=1001.0, nu_end=1000.0),
    dict(nu_begin=1000.0001),
    dict(cutoff=0.0),
    dict(cutoff=float("nan")),
    dict(R=2.0),
    dict(R=47.5),
    dict(prune=1.0),
    dict(layers=[[1.0, 0.0, 1.0, 0.0]]),
    dict(layers=[[1.0, 296.0, 2.0, 0.0]]),
    dict(layers=[[float("inf"), 296.0, 1.0, 0.0]]),
    dict(level_table=3),
    dict(shape=7),
    dict(shape=4),
    dict(chi=3),
    dict(stencil=2),
    dict(stencil=6),
])
def test_invalid_requests(kw):
    with pytest.raises(marfa.MarfaError) as e:
        _plan(**kw)
    assert e.value.status == marfa.E_INVALID


def test_invalid_lines():
    lines = synth.make_lines(5, 995.0, 1015.0, 1)
    lines.gamma_air[2] = np.nan
    with pytest.raises(marfa.MarfaError) as e:
        marfa.Plan(lines, [[1.0, 296.0, 1.0, 0.0]], nu_begin=1000.0, nu_end=1001.0, cutoff=25.0)
    assert e.value.status == marfa.E_INVALID
    lines = synth.make_lines(5, 995.0, 1015.0, 1)
    lines.S296[0] = -1.0
    with pytest.raises(marfa.MarfaError):
        marfa.Plan(lines, [[1.0, 296.0, 1.0, 0.0]], nu_begin=1000.0, nu_end=1001.0, cutoff=25.0)


def test_line_count_limit():
    """Records are addressed by 32-bit byte offsets within a layer: 2^26 lines
    or more are refused before any array is read."""
    L = marfa.lib()
    one = np.zeros(1, np.float64)
    f = np.zeros(1, np.float32)
    p = lambda a: a.ctypes.data_as(C.c_void_p)
    lines = marfa.Lines(1 << 26, p(one), p(f), p(f), p(f), p(f), p(f), None, p(f), 44.0)
    lay = (marfa.Layer * 1)(marfa.Layer(1.0, 296.0, 1.0, 0.0))
    rq = marfa.Request(1000.0, 1001.0, 25.0, 0, 0, 0, 0, 0.0, 48.0, 0, 0, 3)
    h = C.c_void_p()
    assert L.marfa_plan_create(C.byref(h), C.byref(lines), lay, 1, C.byref(rq), 0) == marfa.E_INVALID
    assert not h.value


def test_voigt_eval_rejects_negative_y():
    with pytest.raises(marfa.MarfaError) as e:
        marfa.voigt_eval([1.0], [-1.0])
    assert e.value.status == marfa.E_INVALID


def _gpu_present():
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


@pytest.mark.skipif(_gpu_present(), reason="a device is present")
def test_no_device_reports_device_error():
    with pytest.raises(marfa.MarfaError) as e:
        _plan()
    assert e.value.status == marfa.E_DEVICE


def test_record_number_example():
    # Appendix A: 7564 cm^-1 is in record 756
    assert marfa.record_number(7564.0) == 756


@pytest.mark.parametrize("chi,cutoff", [(7, 125.0), (-1, 125.0), (1, 0.0), (1, -3.0), (1, float("nan"))])
def test_surrogate_create_rejects_bad_configuration(chi, cutoff):
    L = marfa.lib()
    h = C.c_void_p()
    st = L.marfa_surrogate_create(C.byref(h), chi, cutoff, 1, 0)
    assert st == marfa.E_INVALID
    assert not h.value


def test_surrogate_refuses_the_user_chi():
    L = marfa.lib()
    h = C.c_void_p()
    assert L.marfa_surrogate_create(C.byref(h), marfa.CHIS["user"], 125.0, 1, 0) == marfa.E_UNSUPPORTED
    assert not h.value


def test_null_handles_are_rejected():
    L = marfa.lib()
    t = marfa.Tiles()
    assert L.marfa_plan_set_tiles(None, C.byref(t)) == marfa.E_INVALID
    assert L.marfa_plan_set_surrogate(None, None) == marfa.E_INVALID
    assert L.marfa_plan_set_eval(None, 1) == marfa.E_INVALID
    assert L.marfa_surrogate_set_params(None, None, 0) == marfa.E_INVALID
    assert L.marfa_surrogate_train(None, None, None, None) == marfa.E_INVALID
    assert L.marfa_plan_tune(None, None, 0, None) == marfa.E_INVALID
    assert L.marfa_surrogate_loss_grad_noalloc(None, None, None, 1, None, None) == marfa.E_INVALID
    assert L.marfa_surrogate_load(None, None, 0, 1.0) == marfa.E_INVALID
    x_max = C.c_double()
    assert L.marfa_surrogate_save(None, None, 0, C.byref(x_max)) == marfa.E_INVALID
