"""Write the direct-sum references for the sampled checks of the two
100-layer tables (tests/test_gpu_tables.py).

Calls only the FP64 oracle (oracle/) and the seeded input generator.  For each
table: eight layers spread over the PT table, 65,536 random output nodes on
each, plus three whole 10 cm^-1 records (20,481 nodes each; one at the low,
middle and high end of the spectrum) on three of those layers.  Each layer's
maximum of the direct sum (the "band maximum" of the tolerance) is the largest
value over the sampled nodes, over windows of 17 nodes around the centres of
the layer's strongest line peaks (the 500 highest by each of three rankings),
and over the peaks reached uphill from the 50 best of those nodes.

    python tests/golden/make_table_refs.py [pt100_2m|pt100_200k ...]
"""
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2411_03418_amd import synth  # noqa: E402

LAYERS = [0, 14, 28, 42, 57, 71, 85, 99]
N_NODES = 65536
RECORDS = {"pt100_2m": [20.0, 5000.0, 9980.0], "pt100_200k": [500.0, 1500.0, 2490.0]}
RECORD_LAYERS = [14, 57, 85]
SEED = {"pt100_2m": 21, "pt100_200k": 22}


def peak_candidates(lines, layer, req, n_peaks=500, half=8):
    """Nodes within `half` steps of the centres of the layer's strongest line
    peaks, ranked by S(T) / max(gamma_L, alpha_D) (the peak height up to a
    factor of order one), and separately by S(T) / gamma_L and S(T) / alpha_D."""
    st = O.line_states(lines, layer)
    lo, hi = int(round(req["nu_begin"] * 2048)), int(round(req["nu_end"] * 2048))
    inside = (st["nu_t"] * 2048 >= lo - half) & (st["nu_t"] * 2048 <= hi + half)
    picks = []
    for w in (np.maximum(st["gamma_L"], st["alpha_D"]), st["gamma_L"], st["alpha_D"]):
        score = np.where(inside & (w > 0), st["S"] / np.maximum(w, 1e-300), 0.0)
        picks.append(np.argsort(-score)[:n_peaks])
    nodes = []
    for j in np.unique(np.concatenate(picks)):
        m = int(round(st["nu_t"][j] * 2048))
        nodes.extend(range(m - half, m + half + 1))
    return np.unique(np.clip(np.asarray(nodes, np.int64), lo, hi))


def climb(lines, layer, req, start, value, threads, half=16):
    """Largest direct sum reached from the 50 best candidate nodes: from each,
    step uphill with doubling steps until the value falls, search the
    bracketed peak by integer ternary search, and take the maximum over a
    window of 2 half + 1 nodes around the point found (broad peaks of
    overlapping pressure-broadened lines can lie thousands of nodes away)."""
    lo, hi = int(round(req["nu_begin"] * 2048)), int(round(req["nu_end"] * 2048))
    cache = {}

    def f(k):
        k = min(max(int(k), lo), hi)
        if k not in cache:
            cache[k] = float(O.direct(lines, layer, np.array([k], np.int64), threads=threads, **req)[0])
        return cache[k]

    best = float(value.max())
    for m in start[np.argsort(-value)[:50]]:
        m = int(m)
        left, right = f(m - 1), f(m + 1)
        if f(m) < max(left, right):
            step = 1 if right >= left else -1
            a, b = m, m + step
            while f(b) > f(a) and lo < b < hi:
                a, b = b, b + 2 * (b - a)
            x0, x1 = sorted((a - (b - a), b))
            x0, x1 = max(x0, lo), min(x1, hi)
            while x1 - x0 > 2:
                t0, t1 = x0 + (x1 - x0) // 3, x1 - (x1 - x0) // 3
                if f(t0) < f(t1):
                    x0 = t0 + 1
                else:
                    x1 = t1 - 1 if t1 > t0 else t1
            m = max(range(x0, x1 + 1), key=f)
        win = np.arange(max(m - half, lo), min(m + half, hi) + 1, dtype=np.int64)
        v = O.direct(lines, layer, win, threads=threads, **req)
        best = max(best, float(v.max()), max(cache.values()))
    return best


def make(workload, threads):
    lines, layers, rq = synth.workload(workload)
    req = dict(nu_begin=rq["nu_begin"], nu_end=rq["nu_end"], cutoff=rq["cutoff"], chi=rq["chi"], prune=rq["prune"])
    lo, hi = int(round(req["nu_begin"] * 2048)), int(round(req["nu_end"] * 2048))
    rng = np.random.default_rng(SEED[workload])
    out = {}
    for li in LAYERS:
        t0 = time.time()
        nodes = rng.integers(lo, hi + 1, N_NODES)
        if li in RECORD_LAYERS:
            r0 = RECORDS[workload][RECORD_LAYERS.index(li)]
            nodes = np.concatenate([nodes, np.arange(int(r0 * 2048), int(r0 * 2048) + 20481)])
        nodes = np.unique(nodes.astype(np.int64))
        ref = O.direct(lines, layers[li], nodes, threads=threads, **req)
        cand = peak_candidates(lines, layers[li], req)
        cref = O.direct(lines, layers[li], cand, threads=threads, **req)
        lay_max = max(float(ref.max()), climb(lines, layers[li], req, cand, cref, threads))
        out[f"nodes_{li}"] = nodes.astype(np.int32)
        out[f"ref_{li}"] = ref
        out[f"max_{li}"] = np.array([lay_max])
        print(f"{workload} layer {li}: {nodes.size} nodes, max {lay_max:.6e}, {time.time() - t0:.1f} s", flush=True)
    out["layers"] = np.asarray(LAYERS, np.int64)
    path = os.path.join(HERE, f"ref_{workload}.npz")
    np.savez_compressed(path, **out)
    print("wrote", path)


if __name__ == "__main__":
    threads = len(os.sched_getaffinity(0))
    for w in sys.argv[1:] or ["pt100_200k", "pt100_2m"]:
        make(w, threads)
