"""Build libgapsim.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgapsim.so")
SOURCES = ["gs_kernels.hip", "gs_api.hip", "gs_mlp.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # binary32 particle arithmetic is a fixed sequence of IEEE operations
    "-ffp-contract=off",
    # no packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]
# gs_kernels.hip is compiled once for its main unit and once per set of push
# kernel instantiations (GS_PUSH_PART), so that the units build in parallel
PUSH_PARTS = 5


def _units():
    units = [(os.path.join(CSRC, "gs_kernels.hip"), [], "gs_kernels")]
    for k in range(PUSH_PARTS):
        units.append((os.path.join(CSRC, "gs_kernels.hip"), [f"-DGS_PUSH_PART={k}"], f"gs_push{k}"))
    for src in SOURCES[1:]:
        units.append((os.path.join(CSRC, src), [], os.path.splitext(src)[0]))
    return units


def build(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    jobs = []
    for src, defs, name in _units():
        obj = os.path.join(objdir, name + ".o")
        jobs.append(([HIPCC, *FLAGS, *defs, *inc, "-c", src, "-o", obj], obj))
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", "0")) or (os.cpu_count() or 1)))

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        return subprocess.run(cmd, capture_output=True, text=True)

    with ThreadPoolExecutor(max_workers=workers) as ex:
        results = list(ex.map(run, [c for c, _ in jobs]))
    for r in results:
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc failed building libgapsim.so")
    tmp = LIB + ".tmp"
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *[o for _, o in jobs], "-o", tmp]
    r = run(link)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("linking libgapsim.so failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
