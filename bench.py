#!/usr/bin/env python3
"""Benchmark: spectral points per second on one MI355X for eleven-grid PT tables.

A step is one pass of the whole hot path (line preparation, level
accumulation, cascade) over every layer of the workload, replayed from the
plan's HIP graph with all inputs resident in HBM.  Prints one JSON line:

* the plain path on the large table (2M lines, 100 layers, 0-10000 cm^-1),
  tiles autotuned before timing;
* "surrogate": the learned line shape on the 100-layer 200k-line table
  (trained on the device first), its throughput, its speed relative to the
  plain path on the same table, and its deviation from the plain path;
* "roofline": counted algorithmic FP32 work of the level kernel per launch
  over its event-timed duration, against the FP32 vector peak;
* "cpu_baseline": the FP64 oracle's eleven-grid program on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VALU_TFLOPS = 157.3   # MI355X published FP32 vector peak
PEAK_BF16_MFMA_TFLOPS = 2500.0  # MI355X published dense BF16 matrix peak
# algorithmic flops of one network evaluation: 3->64 (2*3*64 + 64), three
# 64->64 layers (2*64*64 each), 64->1 (2*64); the split-BF16 activations run
# the hidden layers twice on the matrix cores, which is not counted here
FLOP_MLP = 2 * 3 * 64 + 64 + 3 * 2 * 64 * 64 + 2 * 64
STENCIL_R = {4: 24, 5: 24}   # R of the 4- and 5-point legs: about the 3-point R = 48 table's cost


def profiled_traffic(workload):
    """HBM bytes per k_level launch measured with rocprofv3 counters for this
    workload (profiles/k_level_f32_<workload>.md), or None when there is no such
    profile or the kernel sources changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"k_level_f32_{workload}.md")
    if not os.path.exists(path):
        return None
    rec = {}
    for ln in open(path):
        if ":" in ln and ln.split(":")[0] in ("traffic_bytes_per_launch", "kernel_source_sha256"):
            k, v = ln.split(":", 1)
            rec[k] = v.strip()
    h = hashlib.sha256()
    for src in ("marfa_level_f32.hip", "marfa_level.h", "marfa_device.h", "marfa_internal.h", "marfa_mlp.h",
                "marfa_user.h"):
        with open(os.path.join(ROOT, "paper_2411_03418_amd", "csrc", src), "rb") as f:
            h.update(f.read())
    if rec.get("kernel_source_sha256") != h.hexdigest():
        return None
    return float(rec["traffic_bytes_per_launch"])


def _cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(lines, layers, req, budget_s):
    """The FP64 oracle on bounded samples of the workload, on this host's cores:
    the eleven-grid program on every core available to the process and on one
    core, and the direct sum per sampled node.  The budget is split between the
    three legs; each leg grows its sample until it uses its share."""
    import oracle as O
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    L = layers[len(layers) // 2]
    o = dict(cutoff=req["cutoff"], chi=req["chi"], prune=req["prune"])
    mid = 0.5 * (req["nu_begin"] + req["nu_end"])

    def grid_rate(threads, share):
        width = 0.25
        while True:
            t0 = time.perf_counter()
            out = O.grid(lines, L, threads=threads, nu_begin=mid, nu_end=mid + width, **o)
            dt = time.perf_counter() - t0
            if dt > share / 3 or width >= 4096:
                return out.size, dt, width
            width *= 2 if dt > 0.2 * share / 3 else 4

    pts, dt, width = grid_rate(cores, 0.5 * budget_s)
    pts1, dt1, width1 = grid_rate(1, 0.25 * budget_s)
    n = 64
    m0 = int(round(mid * 2048))
    while True:
        nodes = m0 + np.arange(n, dtype=np.int64) * 97
        t0 = time.perf_counter()
        O.direct(lines, L, nodes, threads=cores, nu_begin=req["nu_begin"], nu_end=req["nu_end"], **o)
        dtd = time.perf_counter() - t0
        if dtd > 0.25 * budget_s / 3 or n >= 1 << 20:
            break
        n *= 4 if dtd < 0.05 * budget_s / 3 else 2
    lay = f"layer {len(layers) // 2} (p={L[0]:.3g} atm, T={L[1]:.0f} K)"
    return dict(value=pts / dt, unit="points/s", cores=cores, kind="oracle",
                sample=f"eleven-grid oracle (FP64), {lay}, {width:g} cm^-1 at {mid:g} cm^-1 = {pts} points "
                       f"in {dt:.2f} s on {cores} threads",
                grid_1core=dict(value=pts1 / dt1, unit="points/s", cores=1,
                                sample=f"{width1:g} cm^-1 = {pts1} points in {dt1:.2f} s"),
                direct=dict(value=n / dtd, unit="points/s", cores=cores,
                            sample=f"direct sum at {n} nodes (every 97th from {mid:g} cm^-1) in {dtd:.2f} s"),
                host=dict(nproc=os.cpu_count(), cpu_model=_cpu_model(), threads_available=cores))


def timed_steps(plan, out, steps, warmup):
    import torch
    for _ in range(warmup):
        plan.execute(out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.execute(out=out)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3


def rel_dev(a, b):
    """max over layers and nodes with a >= 1e-8 of the layer max of |b - a| / a
    (infinite when b holds a non-finite value)."""
    worst = 0.0
    for i in range(a.shape[0]):
        x, y = a[i].double(), b[i].double()
        if not bool(torch_isfinite_all(y)):
            return float("inf")
        m = x >= 1e-8 * x.max()
        worst = max(worst, float(((y[m] - x[m]).abs() / x[m]).max()))
    return worst


def torch_isfinite_all(t):
    import torch
    return torch.isfinite(t).all()


def stencil_leg(lines, layers, req, plain, steps, ns):
    """The same table with the 4- or 5-point interpolation stencil at a smaller R."""
    import torch
    from paper_2411_03418_amd import marfa
    R = STENCIL_R[ns]
    plan = marfa.Plan(lines, layers, device=0, stencil=ns, R=R, **req)
    out = torch.empty((plan.n_layers, plan.points), dtype=torch.float32, device="cuda:0")
    tiles = plan.tune(out=out)
    st = plan.count()
    ms = timed_steps(plan, out, steps, 1)
    lv = []
    for _ in range(steps):
        _, t = plan.execute_timed(out=out)
        lv.append(t["level_ms"])
    dev = rel_dev(plain, out)
    points = plan.points * plan.n_layers
    print(f"[bench] {ns}-point R={R}: {ms:.1f} ms/step, level {np.mean(lv):.1f} ms; max dev from 3-point "
          f"{dev:.2e}", file=sys.stderr, flush=True)
    plan.close()
    del out
    torch.cuda.empty_cache()
    return dict(value=points / (ms * 1e-3), unit="points/s", ms_per_step=ms, level_ms=float(np.mean(lv)),
                steps=steps, stencil=ns, R=R, pairs=int(sum(st["pairs_level"])),
                band_pairs=int(st["pairs_band"]), max_rel_dev_from_3point=dev, tiles=tiles)


def surrogate_table_leg(plan, out, lines, layers, chi, cutoff, workload):
    """The learned line shape on the benchmark's own table, trained for its
    line and temperature ranges; one timed step (the deviation from the plain
    output of the same plan is over every node of every layer)."""
    import torch
    from paper_2411_03418_amd import marfa
    S = marfa.Surrogate(chi=chi, cutoff=cutoff, seed=1)
    nu = lines.nu0[lines.nu0 > 0]
    n_train = 20_000_000
    rep = S.fit(nu_lo=float(nu.min()), nu_hi=float(nu.max()), T_lo=float(layers[:, 1].min()),
                T_hi=float(layers[:, 1].max()), n_train=n_train)
    print(f"[bench] {workload} surrogate trained: {rep}", file=sys.stderr, flush=True)
    plain = out.clone()
    plan.set_surrogate(S)
    plan.set_eval("surrogate")
    ms = timed_steps(plan, out, 1, 0)
    dev = rel_dev(plain, out)
    plan.set_eval("plain")
    out.copy_(plain)   # later legs compare against the plain output
    del plain
    torch.cuda.empty_cache()
    S.close()
    points = plan.points * plan.n_layers
    print(f"[bench] {workload} surrogate {ms:.1f} ms/step; max dev from plain {dev:.2e}", file=sys.stderr, flush=True)
    return dict(workload=workload, value=points / (ms * 1e-3), unit="points/s", ms_per_step=ms, steps=1, warmup=0,
                max_rel_dev_from_plain=dev, train_ms=rep["ms"], train_samples=n_train,
                val_max_abs_t=rep["val_max_abs"])


def surrogate_leg(args):
    import torch
    from paper_2411_03418_amd import marfa, synth
    lines, layers, rq = synth.workload("pt100_200k")
    req = dict(nu_begin=rq["nu_begin"], nu_end=rq["nu_end"], cutoff=rq["cutoff"], chi="tonkov", prune=rq["prune"])
    S = marfa.Surrogate(chi="tonkov", cutoff=rq["cutoff"], seed=1)
    rep = S.fit(nu_lo=float(lines.nu0.min()), nu_hi=float(lines.nu0.max()), T_lo=float(layers[:, 1].min()),
                T_hi=float(layers[:, 1].max()))
    print(f"[bench] surrogate trained: {rep}", file=sys.stderr, flush=True)
    plan = marfa.Plan(lines, layers, device=0, **req)
    out = torch.empty((plan.n_layers, plan.points), dtype=torch.float32, device="cuda:0")
    plan.tune(out=out)
    st = plan.count()
    evals = st["pairs_wing"] + st["pairs_core"]   # shape evaluations, region and band passes
    ms_plain = timed_steps(plan, out, 3, 1)
    plain = out.clone()
    plan.set_surrogate(S)
    plan.set_eval("surrogate")
    ms_surr = timed_steps(plan, out, args.surrogate_steps, 1)
    dev = rel_dev(plain, out)
    _, t = plan.execute_timed(out=out)
    points = plan.points * plan.n_layers
    print(f"[bench] surrogate {ms_surr:.1f} ms/step vs plain {ms_plain:.1f}; max dev from plain {dev:.2e}",
          file=sys.stderr, flush=True)
    plan.close()
    S.close()
    mfma_tflops = evals * FLOP_MLP / (t["level_ms"] * 1e-3) / 1e12
    return dict(workload="pt100_200k", value=points / (ms_surr * 1e-3), unit="points/s", ms_per_step=ms_surr,
                roofline={"bound": "mfma", "achieved": mfma_tflops, "peak": PEAK_BF16_MFMA_TFLOPS, "unit": "TFLOP/s",
                          "frac": mfma_tflops / PEAK_BF16_MFMA_TFLOPS, "kernel": "k_level (learned shape)",
                          "evaluations": int(evals), "flop_per_evaluation": FLOP_MLP,
                          "note": "VALU-bound in practice: each SiLU activation costs two transcendentals (3.3x an FP32 add each)"},
                steps=args.surrogate_steps, level_ms=t["level_ms"], plain_ms_per_step=ms_plain,
                speed_vs_plain=ms_plain / ms_surr, max_rel_dev_from_plain=dev,
                train=dict(ms=rep["ms"], steps=rep["steps"], val_max_abs_t=rep["val_max_abs"],
                           val_mean_abs_t=rep["val_mean_abs"], samples=20_000_000,
                           recipe="300 epochs mean-squared + 100 epochs fourth-power, batch 16384"),
                mfma="v_mfma_f32_16x16x32_bf16, BF16 weights, BF16 hi/lo activations, FP32 accumulate")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="pt100_2m")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true", help="skip every learned-shape leg")
    ap.add_argument("--surrogate-200k", action="store_true",
                    help="also time the learned shape on the 200k-line table (its own plan and training)")
    ap.add_argument("--no-surrogate-table", action="store_true",
                    help="skip the learned shape on the benchmark's own table (one step)")
    ap.add_argument("--no-stencil5", action="store_true", help="skip the 5-point stencil leg")
    ap.add_argument("--no-stencil4", action="store_true", help="skip the 4-point stencil leg")
    ap.add_argument("--surrogate-steps", type=int, default=2)
    ap.add_argument("--no-tune", action="store_true", help="keep the density-based tiles")
    ap.add_argument("--tiles", default=None, metavar="JSON",
                    help="tile parameters from an earlier run's \"tiles\" (skips tuning)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (layers shard across GPUs "
              "without communication; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2411_03418_amd import marfa, synth

    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n * 4}))
        return

    t0 = time.perf_counter()
    lines, layers, rq = synth.workload(args.workload)
    chi = "tonkov" if rq["chi"] else "none"
    req = dict(nu_begin=rq["nu_begin"], nu_end=rq["nu_end"], cutoff=rq["cutoff"], chi=chi, prune=rq["prune"])
    print(f"[bench] {args.workload}: {lines.n} lines, {len(layers)} layers, inputs {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    plan = marfa.Plan(lines, layers, device=0, **req)
    out = torch.empty((plan.n_layers, plan.points), dtype=torch.float32, device="cuda:0")
    if args.tiles:
        tiles = plan.set_tiles(json.loads(args.tiles))
    elif not args.no_tune:
        tiles = plan.tune(out=out)
    else:
        tiles = plan.tiles()
    print(f"[bench] tiles {tiles}", file=sys.stderr, flush=True)
    st = plan.count()
    flops = st["flops_level"]
    print(f"[bench] pairs {sum(st['pairs_level']):.3e}, core {st['pairs_core']:.3e}, band {st['pairs_band']:.3e}, "
          f"counted {flops:.3e} flop per level launch", file=sys.stderr, flush=True)
    ms = timed_steps(plan, out, args.steps, args.warmup)
    points = plan.points * plan.n_layers
    # dominant kernel: the level stage, timed by HIP events on the launch stream
    lv, tot, prep, cas = [], [], [], []
    for _ in range(args.steps):
        _, t = plan.execute_timed(out=out)
        lv.append(t["level_ms"]); tot.append(t["total_ms"]); prep.append(t["prep_ms"]); cas.append(t["cascade_ms"])
    level_ms = float(np.mean(lv))
    achieved = flops / (level_ms * 1e-3) / 1e12
    print(f"[bench] {ms:.2f} ms/step; level {level_ms:.2f} ms, prep {np.mean(prep):.2f} ms, "
          f"cascade {np.mean(cas):.2f} ms", file=sys.stderr, flush=True)
    s_big = None
    if not args.no_surrogate and not args.no_surrogate_table:
        s_big = surrogate_table_leg(plan, out, lines, layers, chi, req["cutoff"], args.workload)
        s_big["speed_vs_plain"] = ms / s_big["ms_per_step"]
    plan.close()
    s5 = s4 = None
    if not args.no_stencil5:
        s5 = stencil_leg(lines, layers, req, out, args.steps, 5)
    if not args.no_stencil4:
        s4 = stencil_leg(lines, layers, req, out, args.steps, 4)
    del out
    torch.cuda.empty_cache()

    line = {
        "metric": "spectral points/s/GPU (PT table), plain vs MLP-surrogate at 1e-4/1e-3 rel err",
        "value": points / (ms * 1e-3),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "lines": lines.n, "layers": len(layers),
                   "points_per_layer": int(points // len(layers)), "nu_begin": req["nu_begin"],
                   "nu_end": req["nu_end"], "cutoff": req["cutoff"], "chi": chi, "prune_rel": req["prune"], "R": 48,
                   "path": "plain", "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VALU_TFLOPS, "traffic": profiled_traffic(args.workload),
                     "kernel": "k_level_f32", "kernel_ms": level_ms, "counted_tflop_per_launch": flops / 1e12,
                     "flops_per_unit": {k: st[k] for k in ("flops_per_eval", "flops_per_core", "flops_per_term",
                                                           "flops_per_band")},
                     "algorithmic_bytes_per_launch": st["bytes_level"],
                     "algorithmic_gbs": st["bytes_level"] / (level_ms * 1e-3) / 1e9},
        "stages_ms": {"prep": float(np.mean(prep)), "level": level_ms, "cascade": float(np.mean(cas)),
                      "graph_total": float(np.mean(tot))},
        "pairs": {"total": int(sum(st["pairs_level"])), "core": int(st["pairs_core"]),
                  "wing": int(st["pairs_wing"]), "band": int(st["pairs_band"]),
                  "per_level": [int(v) for v in st["pairs_level"]],
                  "wave_iters_per_level": [int(v) for v in st["iters_level"]],
                  "band_iters_per_level": [int(v) for v in st["band_iters_level"]],
                  "wing_terms": int(st["wing_terms"])},
        "tiles": tiles,
    }
    if s5 is not None:
        line["stencil5"] = s5
    if s4 is not None:
        line["stencil4"] = s4
    if args.surrogate_200k and not args.no_surrogate:
        line["surrogate"] = surrogate_leg(args)
    if s_big is not None:
        line["surrogate_table"] = s_big
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(lines, layers, dict(req, chi=rq["chi"]), args.cpu_seconds)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
