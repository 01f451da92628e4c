"""Build libmarfa.so for gfx950 with hipcc (in-tree, next to this file).

Every translation unit is compiled to an object file in parallel (the level
kernel's instantiations sit in units of their own), then linked into one
shared library.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["csrc/marfa_kernels.hip", "csrc/marfa_level_f32.hip", "csrc/marfa_level_f32_count.hip",
           "csrc/marfa_level_f32_surr.hip", "csrc/marfa_level_f32_user.hip", "csrc/marfa_level_f32_s4.hip",
           "csrc/marfa_level_f64.hip", "csrc/marfa_level_f64_count.hip", "csrc/marfa_level_f64_user.hip",
           "csrc/marfa_level_f64_s4.hip", "csrc/marfa_plan.hip", "csrc/marfa_surrogate.hip", "csrc/marfa_io.hip"]
OUT = os.path.join(HERE, "libmarfa.so")
OBJDIR = os.path.join(HERE, "_build")

FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
    # packed FP32 VALU forms stay disabled for every HIP source
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _compile(hipcc, src):
    obj = os.path.join(OBJDIR, os.path.basename(src).replace(".hip", ".o"))
    # MARFA_USER_HEADER=/abs/path.h compiles another user line shape and chi in
    user = os.environ.get("MARFA_USER_HEADER")
    extra = [f'-DMARFA_USER_HEADER="{user}"'] if user else []
    cmd = [hipcc, *FLAGS, *extra, "-c", "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
           "-o", obj, os.path.join(HERE, src)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n" + r.stderr[-4000:])
    return obj, r.stderr


def build(verbose: bool = False, jobs: int | None = None) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda s: _compile(hipcc, s), SOURCES))
    objs = [o for o, _ in results]
    if verbose:
        for _, err in results:
            if err:
                print(err[-2000:])
    tmp = OUT + ".tmp"
    r = subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr[-4000:])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
