"""PT-table record files (Appendix A of the paper).

The layout is read back here with numpy from its definition alone: record r
(r >= 1, r = int(nu / 10)) holds 20481 float32 values at nu = 10 r + i / 2048,
i = 0 .. 20480, at byte offset (r - 1) * 20481 * 4.  Byte work: compared
bit-exactly.  The host-memory form of the writer touches no GPU and runs on
the CPU; the device form is checked on the GPU against the plan's output.
"""
import os

import numpy as np
import pytest

from paper_2411_03418_amd import marfa as M

NT = 20481
STEP = 20480


def read_record(path, r):
    return np.fromfile(path, dtype="<f4", count=NT, offset=(r - 1) * NT * 4)


def spectrum(nu_begin, nu_end, seed=0):
    n = int(round((nu_end - nu_begin) * 2048)) + 1
    return np.random.default_rng(seed).random(n, dtype=np.float32)


def test_records_hold_their_ten_wavenumbers(tmp_path):
    v = spectrum(995.0, 1032.5)
    p = str(tmp_path / "1__.ptbin")
    assert M.write_ptbin(p, v, 995.0) == 3            # [1000,1010], [1010,1020], [1020,1030]
    assert os.path.getsize(p) == 102 * NT * 4
    m0 = 995 * 2048
    for r in (100, 101, 102):
        assert np.array_equal(read_record(p, r), v[r * STEP - m0:r * STEP - m0 + NT])
    # neighbouring records share their end value
    assert read_record(p, 100)[-1] == read_record(p, 101)[0]
    # records before the covered range are holes
    assert not read_record(p, 99).any()


def test_worked_example_7564():
    # Appendix A: 7564 cm^-1 is found in record 756
    assert M.record_number(7564.0) == 756


def test_lookup_by_record_number(tmp_path):
    v = spectrum(7550.0, 7580.0, seed=1)
    p = str(tmp_path / "65_.ptbin")
    assert M.write_ptbin(p, v, 7550.0) == 3           # records 755, 756 and 757
    rng = np.random.default_rng(2)
    m = rng.integers(7560 * 2048, 7580 * 2048, 200)
    for mm in m:
        nu = mm / 2048.0
        r = M.record_number(nu)
        i = mm - r * STEP
        assert read_record(p, r)[i] == v[mm - 7550 * 2048]
    nu = 7564.0
    assert read_record(p, 756)[(7564 - 7560) * 2048] == v[(7564 - 7550) * 2048]


def test_partial_intervals_and_record_zero(tmp_path):
    # [0, 10] would be record 0, which the 1-based file has no place for;
    # [20, 30] is only partly covered
    v = spectrum(0.0, 25.0, seed=3)
    p = str(tmp_path / "a.ptbin")
    assert M.write_ptbin(p, v, 0.0) == 1              # record 1 = [10, 20]
    assert np.array_equal(read_record(p, 1), v[STEP:STEP + NT])
    assert os.path.getsize(p) == NT * 4
    q = str(tmp_path / "b.ptbin")
    assert M.write_ptbin(q, spectrum(1001.0, 1009.0), 1001.0) == 0
    assert os.path.getsize(q) == 0
    assert M.write_ptbin(q, np.zeros(0, np.float32), 1000.0) == 0


def test_exact_interval_and_append_without_truncate(tmp_path):
    p = str(tmp_path / "c.ptbin")
    a = spectrum(1000.0, 1010.0, seed=4)              # exactly one interval, both ends
    assert M.write_ptbin(p, a, 1000.0) == 1
    b = spectrum(1020.0, 1030.0, seed=5)
    assert M.write_ptbin(p, b, 1020.0, truncate=False) == 1
    assert np.array_equal(read_record(p, 100), a)
    assert np.array_equal(read_record(p, 102), b)
    assert not read_record(p, 101).any()
    assert M.write_ptbin(p, b, 1020.0, truncate=True) == 1
    assert os.path.getsize(p) == 102 * NT * 4 and not read_record(p, 100).any()


def test_invalid_arguments(tmp_path):
    v = spectrum(1000.0, 1010.0)
    with pytest.raises(M.MarfaError) as e:
        M.write_ptbin(str(tmp_path / "x.ptbin"), v, 1000.0001)    # off the 2^-11 lattice
    assert e.value.status == M.E_INVALID
    with pytest.raises(M.MarfaError) as e:
        M.write_ptbin(str(tmp_path / "x.ptbin"), v, -10.0)
    assert e.value.status == M.E_INVALID
    with pytest.raises(M.MarfaError) as e:
        M.write_ptbin(str(tmp_path / "no" / "such" / "dir.ptbin"), v, 1000.0)
    assert e.value.status == M.E_IO
    L = M.lib()
    n = M.C.c_int32(7)
    assert L.marfa_ptbin_write(None, M._ptr(v), v.shape[0], 1000.0, 0, None, 1, M.C.byref(n)) == M.E_INVALID
    assert n.value == 0
    assert L.marfa_ptbin_write(b"/tmp/x", None, 5, 1000.0, 0, None, 1, None) == M.E_INVALID
    assert L.marfa_ptbin_write(b"/tmp/x", M._ptr(v), -1, 1000.0, 0, None, 1, None) == M.E_INVALID
    assert L.marfa_ptbin_write(str(tmp_path / "y").encode(), M._ptr(v), v.shape[0], 1000.0, 0, None, 4,
                               None) == M.E_INVALID


def test_file_names():
    assert [M.ptbin_name(i) for i in (1, 65, 100)] == ["1__.ptbin", "65_.ptbin", "100.ptbin"]


@pytest.mark.gpu
def test_device_output_written_per_layer(tmp_path):
    torch = pytest.importorskip("torch")
    from paper_2411_03418_amd import synth
    lines = synth.make_lines(400, 980.0, 1050.0, 41, shift=True)
    layers = synth.pt_table(3)
    plan = M.Plan(lines, layers, nu_begin=995.0, nu_end=1031.0, cutoff=25.0, chi="tonkov", device=0)
    out = plan.execute()
    torch.cuda.synchronize()
    host = out.cpu().numpy()
    paths = M.write_pt_table(out, str(tmp_path), 995.0)
    plan.close()
    assert [os.path.basename(p) for p in paths] == ["1__.ptbin", "2__.ptbin", "3__.ptbin"]
    m0 = 995 * 2048
    for i, p in enumerate(paths):
        assert os.path.getsize(p) == 102 * NT * 4
        for r in (100, 101, 102):
            assert np.array_equal(read_record(p, r), host[i, r * STEP - m0:r * STEP - m0 + NT])


# ------------------------------------------------------------------ line database (Appendix B)

def test_linedb_round_trip_and_layout(tmp_path):
    from paper_2411_03418_amd import synth
    lines = synth.make_lines(5000, 500.0, 600.0, 17, shift=True)
    lines.mol_iso[:] = np.arange(lines.n, dtype=np.int32) % 97 + 21
    p = str(tmp_path / "CO2.db")
    M.write_line_db(p, lines)
    assert os.path.getsize(p) == 36 * lines.n
    # layout read back with the independent struct codec
    ref = synth.unpack_records(open(p, "rb").read())
    back = M.read_line_db(p)
    for f in ("nu0", "S296", "gamma_air", "gamma_self", "E_lower", "n_air", "mol_iso", "delta_air"):
        assert np.array_equal(getattr(ref, f), getattr(lines, f)), f
        assert np.array_equal(getattr(back, f), getattr(lines, f)), f
    # and the writer's bytes equal the struct codec's for the first records
    assert open(p, "rb").read(36 * 50) == synth.pack_records(lines.subset(np.arange(50)))
    part = M.read_line_db(p, first=1234, count=100)
    assert np.array_equal(part.nu0, lines.nu0[1234:1334])


def test_linedb_errors(tmp_path):
    p = tmp_path / "bad.db"
    p.write_bytes(b"\0" * 35)
    with pytest.raises(M.MarfaError) as e:
        M.read_line_db(str(p))
    assert e.value.status == M.E_INVALID
    q = tmp_path / "empty.db"
    q.write_bytes(b"")
    assert M.read_line_db(str(q)).n == 0
    with pytest.raises(M.MarfaError) as e:
        M.read_line_db(str(tmp_path / "missing.db"))
    assert e.value.status == M.E_IO
    r = tmp_path / "two.db"
    r.write_bytes(b"\0" * 72)
    with pytest.raises(M.MarfaError) as e:
        M.read_line_db(str(r), first=1, count=2)
    assert e.value.status == M.E_INVALID


@pytest.mark.gpu
def test_double_precision_output_rounds_to_float32_records(tmp_path):
    torch = pytest.importorskip("torch")
    from paper_2411_03418_amd import synth
    lines = synth.make_lines(200, 990.0, 1030.0, 43)
    plan = M.Plan(lines, synth.pt_table(2), nu_begin=1000.0, nu_end=1010.0, cutoff=25.0, fp64=True, device=0)
    out = plan.execute()
    torch.cuda.synchronize()
    host = out.cpu().numpy()
    paths = M.write_pt_table(out, str(tmp_path), 1000.0)
    plan.close()
    for i, p in enumerate(paths):
        assert np.array_equal(read_record(p, 100), host[i].astype(np.float32))


@pytest.mark.gpu
def test_linedb_file_through_the_gpu_path(tmp_path):
    """Appendix B end to end: the 1,000-line single-layer workload written as a
    36-byte-record database file, read back by the library's reader, computed
    on the GPU, and compared with the oracle at every output node."""
    torch = pytest.importorskip("torch")
    import oracle as O
    from paper_2411_03418_amd import synth
    lines, layers, rq = synth.workload("single_1k")
    path = str(tmp_path / "lines.db")
    M.write_line_db(path, lines)
    assert os.path.getsize(path) == 36 * lines.n
    back = M.read_line_db(path, molar_mass=lines.molar_mass)
    for f in ("nu0", "S296", "gamma_air", "gamma_self", "E_lower", "n_air", "mol_iso", "delta_air"):
        assert np.array_equal(getattr(back, f), getattr(lines, f)), f
    req = dict(nu_begin=rq["nu_begin"], nu_end=rq["nu_end"], cutoff=rq["cutoff"])
    plan = M.Plan(back, layers, device=0, **req)
    got = plan.execute()
    torch.cuda.synchronize()
    got = got[0].double().cpu().numpy()
    plan.close()
    o = dict(req, chi=0, shape=0, prune=0.0)
    nodes = np.arange(int(req["nu_begin"] * 2048), int(req["nu_end"] * 2048) + 1)
    ref_d = O.direct(lines, layers[0], nodes, threads=8, **o)
    ref_g = O.grid(lines, layers[0], threads=8, **o)
    m = ref_d >= 1e-8 * ref_d.max()
    ed = float(np.max(np.abs(got[m] - ref_d[m]) / ref_d[m]))
    eg = float(np.max(np.abs(got[m] - ref_g[m]) / ref_g[m]))
    print(f"database file: vs direct {ed:.2e}, vs grid {eg:.2e} over {m.sum()} nodes")
    assert ed < 1e-4 and eg < 1e-5
