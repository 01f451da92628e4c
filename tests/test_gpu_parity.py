"""Parity of the HIP path with the FP64 oracle, element by element.

Gates (relative, on nodes where the direct sum is >= 1e-8 of the layer max):
GPU single precision vs the definition <= 1e-4; vs the oracle's eleven-grid
result <= FP32_VS_GRID = 1e-5 (implementation error only); GPU double
precision vs the oracle's eleven-grid result <= FP64_VS_GRID = 1e-12.

Two documented node classes have a bound of their own:

* Jump edges in single precision.  The device decides region membership, the
  chi piece and the cut-off on the single-precision distance to a line's
  centre; where a node lies within that distance's rounding of a jump of the
  line's part (|d| within 2^-22 |d| of the cut-off, a chi break or a region
  edge b_l, but not exactly on it), the pair can fall on the other side than
  in the oracle's double precision.  The node's error is then that line's jump there: its whole value
  at the cut-off, the relative step of chi at a break, at a region edge the
  difference of two valid decompositions (the scheme's interpolation error,
  taken as 1e-4 of the line's value), carried by the cascade to the fine
  nodes within reach of the coarsest level whose node the jump point is.
  edge_tolerance() finds these pairs from the oracle's double-precision line
  centres and adds the bound to the node's gate.
* FP64_VS_GRID_THIN = 1e-10, layers below 1e-4 atm: the double-precision
  device Voigt function takes K = Re w(z) from a rational approximation of
  the Faddeeva function w; for y << 1 and |x| of 5 to 8, Re w is smaller than
  |w| by about y / |x|, so rounding of w leaves K a relative error near
  |x| eps / y (7.8e-11 at y = 1e-5 on the device-K grid below).
"""
import os

import numpy as np
import pytest

import oracle as O
from paper_2411_03418_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)
FP32_VS_GRID = 1e-5
FP64_VS_GRID = 1e-12
FP64_VS_GRID_THIN = 1e-10
EDGE_REL = 2.0 ** -22     # relative reach of single-precision distance rounding


def fp64_gate(layer):
    return FP64_VS_GRID if layer[0] >= 1e-4 else FP64_VS_GRID_THIN


def _chi_breaks(kind):
    return {0: [], 1: [3.0, 150.0, 300.0], 2: O.user_chi_breaks()}[kind]


def edge_tolerance(lines, layer, req, nodes, ref):
    """Extra relative tolerance of each node for the single-precision jump-edge
    class (see the module docstring), from the oracle's line states.  A jump
    point that lies within rounding of a fine node m* coincides with the nodes
    of every level whose step divides m*; a pair there can change level or side
    on the coarsest of them, and the cascade carries the difference to the fine
    nodes within (stencil half-width + 1) coarser steps of m*."""
    o = _oreq(req)
    c = o["cutoff"]
    st = O.line_states(lines, layer)
    keep = st["S"] >= o["prune"] * st["S"].max() if o["prune"] > 0 else np.ones(lines.n, bool)
    idx = np.flatnonzero(keep)
    nu = st["nu_t"][idx]
    R, lt = o["R"], o["level_table"]
    steps = [1 << l for l in range(11)] if lt == 1 else [1] + [1 << (l + 1) for l in range(1, 11)]
    half = int(o["stencil"]) // 2 + 1
    jumps = [(c, "cut")] + [(R * steps[l + 1] / 2048.0, "edge") for l in range(10) if R * steps[l + 1] / 2048.0 < c]
    jumps += [(q, "chi") for q in _chi_breaks(o["chi"]) if q <= c]
    extra = np.zeros(nodes.size)
    n0 = int(nodes[0])
    for q, kind in jumps:
        for sgn in (1.0, -1.0):
            target = nu + sgn * q
            m = np.rint(target * 2048.0).astype(np.int64)
            # an exact coincidence (a centre on a node, a jump on the lattice)
            # leaves the single-precision distance exact: no flip there
            dist = np.abs(m / 2048.0 - target)
            near = (dist <= EDGE_REL * q) & (dist > 0)
            for j, mm in zip(idx[near], m[near]):
                top = max(l for l in range(11) if mm % steps[l] == 0)
                reach = half * steps[min(top + 1, 10)]
                lo, hi = max(int(mm) - reach, n0), min(int(mm) + reach, int(nodes[-1]))
                if lo > hi:
                    continue
                win = np.arange(lo, hi + 1, dtype=np.int64)
                # the line's own value on the window (beyond a cut-off: its
                # value just inside it, the size of the jump)
                g = O.direct(lines.subset([j]), layer, win, threads=1, **dict(o, prune=0.0, cutoff=c * (1 + 1e-6)))
                if kind == "cut":
                    f = 1.0
                elif kind == "chi":
                    f = abs(O.chi(o["chi"], q * (1 + 1e-9)) / O.chi(o["chi"], q) - 1.0)
                else:
                    f = 1e-4
                r = ref[win - n0]
                extra[win - n0] += np.where(r > 0, f * g / np.where(r > 0, r, 1.0), 0.0)
    return extra


def grid_check(got, ref_g, lines, layer, req, fp64):
    """Relative error against the oracle's eleven-grid result, asserted at the
    gate of the precision (single precision: plus the jump-edge allowance)."""
    m = ref_g >= 1e-8 * ref_g.max()
    err = np.zeros_like(ref_g)
    err[m] = np.abs(got[m] - ref_g[m]) / ref_g[m]
    if fp64:
        assert err.max() < fp64_gate(layer), err.max()
        return float(err.max())
    nodes = np.arange(int(round(req["nu_begin"] * 2048)), int(round(req["nu_end"] * 2048)) + 1)
    extra = edge_tolerance(lines, layer, req, nodes, ref_g)
    n_edge = int(np.count_nonzero(extra[m]))
    bad = err > FP32_VS_GRID + extra
    plain = float(err[m & (extra == 0)].max()) if np.any(m & (extra == 0)) else 0.0
    print(f"  vs grid: {plain:.2e} off the edge class; {n_edge} edge-class nodes, max {err[extra > 0].max() if n_edge else 0:.2e}")
    assert not np.any(bad & m), (np.flatnonzero(bad & m)[:10], err[bad & m][:10], extra[bad & m][:10])
    return float(err.max())


def marfa():
    from paper_2411_03418_amd import marfa as M
    return M


def run(lines, layers, fp64=False, **req):
    M = marfa()
    layers = np.asarray(layers, np.float64).reshape(-1, 4)
    print(f"[gpu] plan: {lines.n} lines, {layers.shape[0]} layers, {req}, fp64={fp64}", flush=True)
    plan = M.Plan(lines, layers, fp64=fp64, device=0, **req)
    out = plan.execute()
    torch.cuda.synchronize()
    res = out.double().cpu().numpy()
    plan.close()
    return res


def _oreq(req):
    o = dict(nu_begin=req["nu_begin"], nu_end=req["nu_end"], cutoff=req["cutoff"])
    o["chi"] = {"none": 0, "tonkov": 1, "user": 2}[req.get("chi", "none")]
    o["shape"] = {"voigt": 0, "lorentz": 1, "doppler": 2, "user": 3}[req.get("shape", "voigt")]
    o["prune"] = req.get("prune", 0.0)
    o["level_table"] = req.get("level_table", 0)
    o["out_kind"] = {"sigma": 0, "k": 1}[req.get("out", "sigma")]
    o["R"] = float(req.get("R", 48))
    o["stencil"] = int(req.get("stencil", 3))
    return o


def rel_err(got, ref):
    m = ref >= 1e-8 * ref.max()
    return float(np.max(np.abs(got[m] - ref[m]) / ref[m]))


def all_nodes(req):
    return np.arange(int(round(req["nu_begin"] * 2048)), int(round(req["nu_end"] * 2048)) + 1)


# ------------------------------------------------------------------ device Voigt

def test_device_voigt_single_and_double():
    M = marfa()
    xs = np.concatenate([np.linspace(0, 8, 81), np.geomspace(8, 1e7, 40)])
    ys = np.array([1e-4, 3e-4, 1e-3, 0.01, 0.1, 0.5, 1.0, 3.0, 5.9, 10.0, 100.0, 1e3])
    X, Y = np.meshgrid(xs, ys)
    X, Y = X.ravel(), Y.ravel()
    ref = O.voigt_K(X, Y)
    k32 = M.voigt_eval(X, Y, fp64=False)
    k64 = M.voigt_eval(X, Y, fp64=True)
    e32 = np.max(np.abs(k32 - ref) / ref)
    e64 = np.max(np.abs(k64 - ref) / ref)
    print(f"device K: fp32 {e32:.2e}, fp64 {e64:.2e}")
    assert e32 < 1e-5
    assert e64 < 1e-9


def test_device_voigt_branch_switch_continuous():
    M = marfa()
    # the single-precision path switches from the rational core to the wing
    # series at |z| = 6; both sides agree with each other and the oracle
    th = np.linspace(0.02, 1.5, 25)
    r = np.array([6.0 * (1 - 1e-6), 6.0 * (1 + 1e-6)])
    X = (r[:, None] * np.cos(th)[None, :]).ravel()
    Y = (r[:, None] * np.sin(th)[None, :]).ravel()
    k = M.voigt_eval(X, Y).reshape(2, -1)
    assert np.max(np.abs(k[0] - k[1]) / k[1]) < 1e-5


# ------------------------------------------------------------------ single lines

def _one(nu0, gamma, p=1.0, T=296.0, delta=0.0):
    L = synth.make_lines(1, 0, 1, 7)
    L.nu0[:] = nu0
    L.gamma_air[:] = gamma
    L.gamma_self[:] = gamma
    L.S296[:] = 1e-20
    L.E_lower[:] = 0.0
    L.delta_air[:] = delta
    return L, [p, T, p, 0.0]


ONE_LINE = [
    dict(nu0=1005.0, gamma=0.075),
    dict(nu0=1005.00013, gamma=0.075),
    dict(nu0=1005.3, gamma=0.075, chi="tonkov", c=125.0),
    dict(nu0=1002.1234, gamma=0.3, c=4.0, chi="tonkov"),
    dict(nu0=1007.7, gamma=0.09, p=10.0),
    dict(nu0=1003.0, gamma=0.09, p=30.0, c=125.0, chi="tonkov", nb=900.0, ne=1100.0),
    dict(nu0=1015.0, gamma=0.06, p=0.01),
    dict(nu0=1010.0, gamma=0.06, p=0.2),
    dict(nu0=1005.0, gamma=0.06, p=0.2, shape="lorentz"),
    dict(nu0=1005.0, gamma=0.06, p=0.2, shape="doppler"),
    dict(nu0=1004.2, gamma=0.06, p=0.4, lt=1),
    dict(nu0=1004.4, gamma=0.07, p=1e-4, T=150.0),
    # the compiled-in user shape and chi (Sections 2.2-2.3)
    dict(nu0=1005.00013, gamma=0.075, shape="user"),
    dict(nu0=1003.7, gamma=0.09, p=10.0, chi="user", c=60.0),
    dict(nu0=1001.9, gamma=0.3, chi="user", c=4.0),
    dict(nu0=1004.2, gamma=0.06, p=0.4, chi="user", shape="user", lt=1),
]


@pytest.mark.parametrize("case", ONE_LINE)
@pytest.mark.parametrize("fp64", [False, True])
def test_one_line_parity(case, fp64):
    L, lay = _one(case["nu0"], case["gamma"], p=case.get("p", 1.0), T=case.get("T", 296.0))
    req = dict(nu_begin=case.get("nb", 1000.0), nu_end=case.get("ne", 1010.0), cutoff=case.get("c", 25.0),
               chi=case.get("chi", "none"), shape=case.get("shape", "voigt"), level_table=case.get("lt", 0))
    got = run(L, [lay], fp64=fp64, **req)[0]
    o = _oreq(req)
    ref_g = O.grid(L, lay, threads=THREADS, **o)
    ref_d = O.direct(L, lay, all_nodes(req), threads=THREADS, **o)
    eg, ed = rel_err(got, ref_g), rel_err(got, ref_d)
    print(f"vs grid {eg:.2e}  vs direct {ed:.2e}")
    assert ed < 1e-4
    grid_check(got, ref_g, L, lay, req, fp64)


# ------------------------------------------------------------------ workloads

@pytest.mark.parametrize("fp64", [False, True])
def test_single_1k_workload(fp64):
    lines, layers, rq = synth.workload("single_1k")
    req = dict(nu_begin=rq["nu_begin"], nu_end=rq["nu_end"], cutoff=rq["cutoff"], chi="none")
    got = run(lines, layers, fp64=fp64, **req)[0]
    o = _oreq(req)
    ref_g = O.grid(lines, layers[0], threads=THREADS, **o)
    ref_d = O.direct(lines, layers[0], all_nodes(req), threads=THREADS, **o)
    eg, ed = rel_err(got, ref_g), rel_err(got, ref_d)
    print(f"single_1k fp64={fp64}: vs grid {eg:.2e} vs direct {ed:.2e}")
    assert ed < 1e-4
    grid_check(got, ref_g, lines, layers[0], req, fp64)


def test_multi_layer_pruned_ragged():
    # several tiles, a ragged tail, pruning with uneven kept counts per layer
    lines = synth.make_lines(3000, 930.0, 1090.0, 31, shift=True)
    layers = synth.pt_table(7)
    req = dict(nu_begin=1000.0, nu_end=1013.5, cutoff=60.0, chi="tonkov", prune=1e-6)
    got = run(lines, layers, **req)
    o = _oreq(req)
    for i in range(layers.shape[0]):
        ref_g = O.grid(lines, layers[i], threads=THREADS, **o)
        ref_d = O.direct(lines, layers[i], all_nodes(req), threads=THREADS, **o)
        eg, ed = rel_err(got[i], ref_g), rel_err(got[i], ref_d)
        print(f"layer {i}: vs grid {eg:.2e} vs direct {ed:.2e}")
        assert ed < 1e-4
        grid_check(got[i], ref_g, lines, layers[i], req, False)


@pytest.mark.parametrize("fp64", [False, True])
@pytest.mark.parametrize("stencil", [3, 4, 5])
def test_user_plugins_many_lines(fp64, stencil):
    # the compiled-in user shape and chi through every level, both band
    # passes and the learned-shape-free generic pair path, on several layers
    lines = synth.make_lines(2000, 940.0, 1080.0, 41, shift=True)
    layers = synth.pt_table(7)[[0, 3, 6]]
    req = dict(nu_begin=1000.0, nu_end=1012.0, cutoff=60.0, chi="user", shape="user", prune=1e-6,
               stencil=stencil, R={3: 48, 4: 24, 5: 12}[stencil])
    got = run(lines, layers, fp64=fp64, **req)
    o = _oreq(req)
    for i in range(layers.shape[0]):
        ref_g = O.grid(lines, layers[i], threads=THREADS, **o)
        ref_d = O.direct(lines, layers[i], all_nodes(req), threads=THREADS, **o)
        eg, ed = rel_err(got[i], ref_g), rel_err(got[i], ref_d)
        print(f"user plug-ins layer {i} fp64={fp64} stencil={stencil}: vs grid {eg:.2e} vs direct {ed:.2e}")
        assert ed < 1e-4
        grid_check(got[i], ref_g, lines, layers[i], req, fp64)


@pytest.mark.parametrize("fp64", [False, True])
def test_small_cutoff_node_major_band(fp64):
    # a cut-off below two coarsest steps: stencil hulls around a line centre
    # can hold the cut-off jump, so the top levels take the node-major band pass
    lines = synth.make_lines(500, 995.0, 1015.0, 35, shift=True)
    lay = [0.3, 260.0, 0.05, 0.0]
    req = dict(nu_begin=1000.0, nu_end=1010.0, cutoff=1.5)
    got = run(lines, [lay], fp64=fp64, **req)[0]
    o = _oreq(req)
    ref_d = O.direct(lines, lay, all_nodes(req), threads=THREADS, **o)
    ref_g = O.grid(lines, lay, threads=THREADS, **o)
    eg, ed = rel_err(got, ref_g), rel_err(got, ref_d)
    print(f"small cut-off fp64={fp64}: vs grid {eg:.2e} vs direct {ed:.2e}")
    assert ed < 1e-4
    grid_check(got, ref_g, lines, lay, req, fp64)


@pytest.mark.parametrize("fp64", [False, True])
def test_long_cutoff_all_tonkov_pieces(fp64):
    # cut-off 400 cm^-1: the 150 and 300 cm^-1 breaks of chi are jumps of the
    # coarse levels and windows span several chi pieces
    lines = synth.make_lines(1500, 600.0, 1400.0, 37, shift=True)
    lay = [2.0, 300.0, 2.0, 0.0]
    req = dict(nu_begin=995.0, nu_end=1005.0, cutoff=400.0, chi="tonkov")
    got = run(lines, [lay], fp64=fp64, **req)[0]
    o = _oreq(req)
    ref_d = O.direct(lines, lay, all_nodes(req), threads=THREADS, **o)
    ref_g = O.grid(lines, lay, threads=THREADS, **o)
    eg, ed = rel_err(got, ref_g), rel_err(got, ref_d)
    print(f"cut-off 400 fp64={fp64}: vs grid {eg:.2e} vs direct {ed:.2e}")
    assert ed < 1e-4
    grid_check(got, ref_g, lines, lay, req, fp64)


@pytest.mark.parametrize("fp64", [False, True])
def test_region_edge_next_to_chi_break(fp64):
    # R = 47 puts b_5 = 2.94 cm^-1 within one stencil hull of the 3 cm^-1 chi
    # break: a hull can straddle both jumps and only the smaller one corrects
    lines = synth.make_lines(800, 960.0, 1050.0, 38, shift=True)
    lay = [0.05, 220.0, 0.05, 0.0]
    req = dict(nu_begin=1000.0, nu_end=1010.0, cutoff=40.0, chi="tonkov", R=47)
    got = run(lines, [lay], fp64=fp64, **req)[0]
    o = _oreq(req)
    ref_d = O.direct(lines, lay, all_nodes(req), threads=THREADS, **o)
    ref_g = O.grid(lines, lay, threads=THREADS, **o)
    eg, ed = rel_err(got, ref_g), rel_err(got, ref_d)
    print(f"R=47 fp64={fp64}: vs grid {eg:.2e} vs direct {ed:.2e}")
    assert ed < 1e-4
    grid_check(got, ref_g, lines, lay, req, fp64)


# ------------------------------------------------------------------ rounding at region edges

@pytest.mark.parametrize("tiles", [None, {"item_nodes": 512, "blocks_per_cu": 8,
                                           "wave_nodes": [32, 32, 16, 8, 4, 2, 2, 2, 2, 2, 2]}])
def test_centres_within_rounding_of_a_node(tiles):
    # shifted centres 5.4e-5 of a fine step below / above a lattice node: the
    # single-precision distance to nodes one region radius away rounds onto
    # the region edge, so the region scan must take lines whose exact distance
    # is just outside its window (narrow wavefront tiles put a window edge
    # exactly there)
    L = synth.make_lines(2, 0, 1, 7)
    L.nu0[:] = [(19844672 - 5.4e-5) / 2048.0, (19834880 + 5.4e-5) / 2048.0]
    L.gamma_air[:] = 0.075
    L.gamma_self[:] = 0.075
    L.S296[:] = [1e-20, 3e-21]
    L.E_lower[:] = 0.0
    L.delta_air[:] = 0.0
    lay = [6.77, 645.0, 6.77, 0.0]
    req = dict(nu_begin=9679.0, nu_end=9699.0, cutoff=125.0)
    M = marfa()
    plan = M.Plan(L, np.array([lay]), device=0, **req)
    if tiles:
        plan.set_tiles(tiles)
    got = plan.execute()
    torch.cuda.synchronize()
    got = got[0].double().cpu().numpy()
    plan.close()
    o = _oreq(req)
    ref_g = O.grid(L, lay, threads=THREADS, **o)
    ref_d = O.direct(L, lay, all_nodes(req), threads=THREADS, **o)
    eg, ed = rel_err(got, ref_g), rel_err(got, ref_d)
    print(f"tiles {tiles}: vs grid {eg:.2e} vs direct {ed:.2e}")
    assert ed < 1e-4
    grid_check(got, ref_g, L, lay, req, False)


# ------------------------------------------------------------------ 5-point stencil

# R = 12 with the 5-point stencil: b_7 = 12 r_8 is exactly the 3 cm^-1 break of
# chi, so one merged jump carries both classes
FIVE = dict(stencil=5, R=12)


@pytest.mark.parametrize("case", ONE_LINE)
@pytest.mark.parametrize("fp64", [False, True])
def test_one_line_parity_5pt(case, fp64):
    L, lay = _one(case["nu0"], case["gamma"], p=case.get("p", 1.0), T=case.get("T", 296.0))
    req = dict(nu_begin=case.get("nb", 1000.0), nu_end=case.get("ne", 1010.0), cutoff=case.get("c", 25.0),
               chi=case.get("chi", "none"), shape=case.get("shape", "voigt"), level_table=case.get("lt", 0), **FIVE)
    got = run(L, [lay], fp64=fp64, **req)[0]
    o = _oreq(req)
    ref_g = O.grid(L, lay, threads=THREADS, **o)
    ref_d = O.direct(L, lay, all_nodes(req), threads=THREADS, **o)
    eg, ed = rel_err(got, ref_g), rel_err(got, ref_d)
    print(f"5-point: vs grid {eg:.2e}  vs direct {ed:.2e}")
    assert ed < 1e-4
    grid_check(got, ref_g, L, lay, req, fp64)


@pytest.mark.parametrize("fp64", [False, True])
def test_multi_layer_5pt(fp64):
    lines = synth.make_lines(3000, 930.0, 1090.0, 31, shift=True)
    layers = synth.pt_table(5)
    req = dict(nu_begin=1000.0, nu_end=1013.5, cutoff=60.0, chi="tonkov", prune=1e-6, **FIVE)
    got = run(lines, layers, fp64=fp64, **req)
    o = _oreq(req)
    for i in range(layers.shape[0]):
        ref_g = O.grid(lines, layers[i], threads=THREADS, **o)
        ref_d = O.direct(lines, layers[i], all_nodes(req), threads=THREADS, **o)
        eg, ed = rel_err(got[i], ref_g), rel_err(got[i], ref_d)
        print(f"5-point layer {i} fp64={fp64}: vs grid {eg:.2e} vs direct {ed:.2e}")
        assert ed < 1e-4
        grid_check(got[i], ref_g, lines, layers[i], req, fp64)


@pytest.mark.parametrize("fp64", [False, True])
def test_small_cutoff_node_major_band_5pt(fp64):
    # 5-point hulls span 4 r_(l+1): the cut-off jump falls inside hulls around
    # line centres from level 8 up, which take the node-major band pass
    lines = synth.make_lines(500, 995.0, 1015.0, 35, shift=True)
    lay = [0.3, 260.0, 0.05, 0.0]
    req = dict(nu_begin=1000.0, nu_end=1010.0, cutoff=1.5, **FIVE)
    got = run(lines, [lay], fp64=fp64, **req)[0]
    o = _oreq(req)
    ref_d = O.direct(lines, lay, all_nodes(req), threads=THREADS, **o)
    ref_g = O.grid(lines, lay, threads=THREADS, **o)
    eg, ed = rel_err(got, ref_g), rel_err(got, ref_d)
    print(f"5-point small cut-off fp64={fp64}: vs grid {eg:.2e} vs direct {ed:.2e}")
    assert ed < 1e-4
    grid_check(got, ref_g, lines, lay, req, fp64)


@pytest.mark.parametrize("fp64", [False, True])
def test_long_cutoff_5pt(fp64):
    lines = synth.make_lines(1500, 600.0, 1400.0, 37, shift=True)
    lay = [2.0, 300.0, 2.0, 0.0]
    req = dict(nu_begin=995.0, nu_end=1005.0, cutoff=400.0, chi="tonkov", **FIVE)
    got = run(lines, [lay], fp64=fp64, **req)[0]
    o = _oreq(req)
    ref_d = O.direct(lines, lay, all_nodes(req), threads=THREADS, **o)
    ref_g = O.grid(lines, lay, threads=THREADS, **o)
    eg, ed = rel_err(got, ref_g), rel_err(got, ref_d)
    print(f"5-point cut-off 400 fp64={fp64}: vs grid {eg:.2e} vs direct {ed:.2e}")
    assert ed < 1e-4
    grid_check(got, ref_g, lines, lay, req, fp64)


def test_autotune_keeps_parity_5pt():
    lines = synth.make_lines(3000, 930.0, 1090.0, 31, shift=True)
    layers = synth.pt_table(3)
    req = dict(nu_begin=1000.0, nu_end=1013.5, cutoff=60.0, chi="tonkov", prune=1e-6, stencil=5, R=24)
    M = marfa()
    plan = M.Plan(lines, layers, device=0, **req)
    out = torch.empty((plan.n_layers, plan.points), dtype=torch.float32, device="cuda:0")
    tiles = plan.tune(out=out)
    got = plan.execute(out=out)
    torch.cuda.synchronize()
    got = got.double().cpu().numpy()
    plan.close()
    o = _oreq(req)
    for i in range(layers.shape[0]):
        ref_g = O.grid(lines, layers[i], threads=THREADS, **o)
        eg = rel_err(got[i], ref_g)
        print(f"5-point tuned {tiles['wave_nodes']} layer {i}: vs grid {eg:.2e}")
        grid_check(got[i], ref_g, lines, layers[i], req, False)


# ------------------------------------------------------ 4-point midpoint rule

# the symmetric rule on the two coarse nodes on each side; its error falls
# like R^-4, so R = 24 keeps single lines within 1e-5 of the definition
FOUR = dict(stencil=4, R=24)


@pytest.mark.parametrize("case", ONE_LINE)
@pytest.mark.parametrize("fp64", [False, True])
def test_one_line_parity_4pt(case, fp64):
    L, lay = _one(case["nu0"], case["gamma"], p=case.get("p", 1.0), T=case.get("T", 296.0))
    req = dict(nu_begin=case.get("nb", 1000.0), nu_end=case.get("ne", 1010.0), cutoff=case.get("c", 25.0),
               chi=case.get("chi", "none"), shape=case.get("shape", "voigt"), level_table=case.get("lt", 0), **FOUR)
    got = run(L, [lay], fp64=fp64, **req)[0]
    o = _oreq(req)
    ref_g = O.grid(L, lay, threads=THREADS, **o)
    ref_d = O.direct(L, lay, all_nodes(req), threads=THREADS, **o)
    eg, ed = rel_err(got, ref_g), rel_err(got, ref_d)
    print(f"4-point: vs grid {eg:.2e}  vs direct {ed:.2e}")
    assert ed < 1e-4
    grid_check(got, ref_g, L, lay, req, fp64)


@pytest.mark.parametrize("fp64", [False, True])
def test_multi_layer_4pt(fp64):
    lines = synth.make_lines(3000, 930.0, 1090.0, 31, shift=True)
    layers = synth.pt_table(5)
    req = dict(nu_begin=1000.0, nu_end=1013.5, cutoff=60.0, chi="tonkov", prune=1e-6, **FOUR)
    got = run(lines, layers, fp64=fp64, **req)
    o = _oreq(req)
    for i in range(layers.shape[0]):
        ref_g = O.grid(lines, layers[i], threads=THREADS, **o)
        ref_d = O.direct(lines, layers[i], all_nodes(req), threads=THREADS, **o)
        eg, ed = rel_err(got[i], ref_g), rel_err(got[i], ref_d)
        print(f"4-point layer {i} fp64={fp64}: vs grid {eg:.2e} vs direct {ed:.2e}")
        assert ed < 1e-4
        grid_check(got[i], ref_g, lines, layers[i], req, fp64)


@pytest.mark.parametrize("fp64", [False, True])
def test_small_cutoff_node_major_band_4pt(fp64):
    lines = synth.make_lines(500, 995.0, 1015.0, 35, shift=True)
    lay = [0.3, 260.0, 0.05, 0.0]
    req = dict(nu_begin=1000.0, nu_end=1010.0, cutoff=1.5, **FOUR)
    got = run(lines, [lay], fp64=fp64, **req)[0]
    o = _oreq(req)
    ref_d = O.direct(lines, lay, all_nodes(req), threads=THREADS, **o)
    ref_g = O.grid(lines, lay, threads=THREADS, **o)
    eg, ed = rel_err(got, ref_g), rel_err(got, ref_d)
    print(f"4-point small cut-off fp64={fp64}: vs grid {eg:.2e} vs direct {ed:.2e}")
    assert ed < 1e-4
    grid_check(got, ref_g, lines, lay, req, fp64)


def test_autotune_keeps_parity_4pt():
    lines = synth.make_lines(3000, 930.0, 1090.0, 31, shift=True)
    layers = synth.pt_table(3)
    req = dict(nu_begin=1000.0, nu_end=1013.5, cutoff=60.0, chi="tonkov", prune=1e-6, **FOUR)
    M = marfa()
    plan = M.Plan(lines, layers, device=0, **req)
    out = torch.empty((plan.n_layers, plan.points), dtype=torch.float32, device="cuda:0")
    tiles = plan.tune(out=out)
    st = plan.count()
    got = plan.execute(out=out)
    torch.cuda.synchronize()
    got = got.double().cpu().numpy()
    plan.close()
    assert st["flops_per_band"] == 10 and st["pairs_band"] > 0
    o = _oreq(req)
    for i in range(layers.shape[0]):
        ref_g = O.grid(lines, layers[i], threads=THREADS, **o)
        eg = rel_err(got[i], ref_g)
        print(f"4-point tuned {tiles['wave_nodes']} layer {i}: vs grid {eg:.2e}")
        grid_check(got[i], ref_g, lines, layers[i], req, False)


def test_absorption_coefficient_output():
    lines = synth.make_lines(300, 980.0, 1030.0, 32)
    lay = [0.8, 280.0, 0.2, 0.0]
    req = dict(nu_begin=1000.0, nu_end=1002.0, cutoff=25.0)
    s = run(lines, [lay], **req)[0]
    k = run(lines, [lay], out="k", **req)[0]
    n = O.number_density(lay)
    assert np.allclose(k, s * n * 1e5, rtol=1e-6)


def test_empty_line_list_gives_zeros():
    lines = synth.make_lines(0, 0, 1, 1)
    got = run(lines, [[1.0, 296.0, 1.0, 0.0]], nu_begin=1000.0, nu_end=1001.0, cutoff=25.0)
    assert got.shape == (1, 2049) and not np.any(got)


def test_range_starting_at_zero():
    # coarse-level halos reach below 0 cm^-1; lines start at 0 (alpha_D -> 0)
    lines = synth.make_lines(400, 0.0, 40.0, 33, shift=True)
    lay = [0.5, 300.0, 0.5, 0.0]
    req = dict(nu_begin=0.0, nu_end=6.0, cutoff=25.0, chi="tonkov")
    got = run(lines, [lay], **req)[0]
    o = _oreq(req)
    ref_d = O.direct(lines, lay, all_nodes(req), threads=THREADS, **o)
    ref_g = O.grid(lines, lay, threads=THREADS, **o)
    assert rel_err(got, ref_d) < 1e-4
    grid_check(got, ref_g, lines, lay, req, False)


def test_deterministic_and_graph_replay():
    M = marfa()
    lines = synth.make_lines(5000, 970.0, 1040.0, 34, shift=True)
    layers = synth.pt_table(4)
    plan = M.Plan(lines, layers, nu_begin=1000.0, nu_end=1010.0, cutoff=25.0, chi="tonkov", device=0)
    a = plan.execute().clone()
    torch.cuda.synchronize()
    outs = []
    for _ in range(3):
        x = torch.randn(1000, device="cuda:0").sum()  # eager work between replays
        b = plan.execute()
        torch.cuda.synchronize()
        outs.append(b.clone())
        del x
    for b in outs:
        assert torch.equal(a, b)
    # explicit output buffer with a wider stride, then a subset of layers
    buf = torch.zeros((4, plan.points + 100), dtype=torch.float32, device="cuda:0")
    plan.execute(out=buf)
    torch.cuda.synchronize()
    assert torch.equal(buf[:, :plan.points], a)
    sub = plan.execute_layers(1, 2)
    torch.cuda.synchronize()
    assert torch.equal(sub, a[1:3])
    plan.close()


def test_autotune_keeps_parity():
    M = marfa()
    lines = synth.make_lines(3000, 930.0, 1090.0, 36, shift=True)
    layers = synth.pt_table(5)
    req = dict(nu_begin=1000.0, nu_end=1012.0, cutoff=60.0, chi="tonkov", prune=1e-6)
    plan = M.Plan(lines, layers, device=0, **req)
    before = plan.tiles()
    assert not before["tuned"]
    a = plan.execute().clone()
    t = plan.tune()
    print("tuned tiles", t)
    assert t["tuned"] and t["tune_ms"] > 0
    assert t["item_nodes"] in (128, 256, 512) and t["blocks_per_cu"] in (4, 8, 16)
    assert all(w in (1, 2, 4, 8, 16, 32, 64) for w in t["wave_nodes"])
    b = plan.execute()
    torch.cuda.synchronize()
    got = b.double().cpu().numpy()
    c = plan.execute().clone()   # replays of the re-captured graph are identical
    torch.cuda.synchronize()
    assert torch.equal(b, c)
    assert torch.allclose(a, b, rtol=1e-5, atol=0)
    plan.close()
    o = _oreq(req)
    for i in range(layers.shape[0]):
        ref_g = O.grid(lines, layers[i], threads=THREADS, **o)
        eg = rel_err(got[i], ref_g)
        print(f"tuned layer {i}: vs grid {eg:.2e}")
        grid_check(got[i], ref_g, lines, layers[i], req, False)


def test_single_200k_sampled():
    lines, layers, rq = synth.workload("single_200k")
    req = dict(nu_begin=rq["nu_begin"], nu_end=rq["nu_end"], cutoff=rq["cutoff"], chi="tonkov")
    got = run(lines, layers, **req)[0]
    rng = np.random.default_rng(7)
    nodes = np.unique(np.concatenate([
        rng.integers(int(req["nu_begin"] * 2048), int(req["nu_end"] * 2048) + 1, 3000),
        np.arange(1500 * 2048, 1500 * 2048 + 2049),          # one full 1 cm^-1 stretch
        np.arange(int(req["nu_begin"] * 2048), int(req["nu_begin"] * 2048) + 200),   # range start
        np.arange(int(req["nu_end"] * 2048) - 200, int(req["nu_end"] * 2048) + 1)]))  # range end
    ref = O.direct(lines, layers[0], nodes, threads=THREADS, **_oreq(req))
    g = got[nodes - int(req["nu_begin"] * 2048)]
    e = float(np.max(np.abs(g - ref) / ref))
    print(f"single_200k sampled ({nodes.size} nodes): max rel err {e:.2e}")
    assert e < 1e-4
