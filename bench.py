"""Throughput of the circuit-coupled ES-PIC step on one MI355X.

Default workload: the weak-coupling beam gap (4096 cells, 2e7 H+ macroparticles in
binary32, 2e4 beam ions per step, coupled-LC circuit, SEE with exponential 3 eV
electrons), inputs resident in HBM before the timed region.  One step = circuit +
field solve, gather/push/walls/SEE/beam/deposit, and the periodic slot
compaction, for every particle.

Prints one JSON line: particle-steps/s, the push kernel against the HBM
roofline (HIP events on the library's stream over the timed region), and the
CPU oracle timed on a bounded sample on the host.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E
BYTES_PER_PUSH_F32 = 16  # read x, v and write x, v (binary32)

# HBM traffic of the push kernel, taken with rocprofv3 FETCH_SIZE / WRITE_SIZE
# runs of this script; it is reported only while the sources it was measured
# on are unchanged and the run is the one that was measured.
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "k_push_traffic_beam_gap_4096c_2e7p_weak.json")
KERNEL_SOURCES = ["paper_2603_24010_amd/csrc/gs_kernels.hip", "paper_2603_24010_amd/csrc/gs_api.hip",
                  "paper_2603_24010_amd/csrc/gs_internal.h"]

WORKLOADS = {
    # name: (config builder kwargs, initial H+ count, coupling)
    "beam_gap_4096c_2e7p_weak": dict(n_cells=4096, n0=20_000_000, beam=20_000, mode=1,
                                     load="uniform"),
    "beam_gap_16384c_2e8p_strict": dict(n_cells=16384, n0=200_000_000, beam=20_000, mode=0,
                                        load="gauss"),
    "beam_gap_16384c_2e8p_weak": dict(n_cells=16384, n0=200_000_000, beam=20_000, mode=1,
                                      load="gauss"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_sim(name, spec, total_steps):
    from paper_2603_24010_amd import gapsim, workloads as W
    cfg = W.config2(n_cells=spec["n_cells"], beam_per_step=spec["beam"])
    if spec["load"] == "uniform":
        loads = W.load_config2(n=spec["n0"], seed=2, d=cfg.d)
    else:
        loads = W.load_config3(n=spec["n0"], seed=3, d=cfg.d)
    n_ion = spec["n0"]
    # every beam ion may still be in flight at the end (slow ones cross in
    # thousands of steps); emitted electrons stay well below one per beam ion
    grow = (total_steps + 64) * spec["beam"]
    cap = ((1 << 22) + grow, n_ion + grow + (1 << 20))
    sim = gapsim.GapSim(cfg, particle_fp=32, capacity=cap)
    for sp, (x, v) in loads.items():
        sim.inject(0, sp, x, v)
    return sim, cfg, loads


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def recorded_traffic(workload, steps, warmup, compact_every, tuned):
    """Bytes per push launch from the committed counter record, or None."""
    try:
        with open(TRAFFIC_RECORD) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    run = rec.get("run", {})
    if (rec.get("source_sha256") != kernel_source_hash() or tuned
            or run != {"workload": workload, "steps": steps, "warmup": warmup, "compact_every": compact_every}):
        return None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


def _counter_rows(path, counter):
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter:
                yield int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])


def pmc_summary(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_mb, kernel, last_n):
    """Per-launch HBM bytes of `kernel` over its last `last_n` dispatches.

    FETCH_SIZE / WRITE_SIZE (KiB per dispatch) are scaled by what the same
    counter reads for a plain device copy of copy_mb MiB, so the result is in
    bytes that the copy itself moved.
    """
    copy_bytes = copy_mb * (1 << 20)
    factors = []
    for path, counter in ((copy_fetch_csv, "FETCH_SIZE"), (copy_write_csv, "WRITE_SIZE")):
        vals = [v for _, k, v in _counter_rows(path, counter) if "copyBuffer" in k]
        vals = [v for v in vals if v * 1024 > copy_bytes / 8]  # the 1 GiB copies, not small staging ones
        factors.append(copy_bytes / (sum(vals) / len(vals) * 1024))
    out = {}
    for (path, counter), fac, key in zip(((fetch_csv, "FETCH_SIZE"), (write_csv, "WRITE_SIZE")), factors,
                                         ("fetch", "write")):
        rows = sorted((d, v) for d, k, v in _counter_rows(path, counter) if k.startswith(kernel))
        rows = rows[-last_n:]
        out[f"{key}_bytes_per_launch"] = sum(v for _, v in rows) / len(rows) * 1024 * fac
        out[f"{key}_copy_factor"] = fac
        out[f"{key}_launches"] = len(rows)
    return out


def cpu_baseline(spec, steps: int):
    """The oracle (binary32 mode, one thread) on the workload's initial state."""
    import oracle
    from paper_2603_24010_amd import workloads as W
    cfg = W.config2(n_cells=spec["n_cells"], beam_per_step=spec["beam"])
    n = min(spec["n0"], 20_000_000)
    if spec["load"] == "uniform":
        loads = W.load_config2(n=n, seed=2, d=cfg.d)
    else:
        loads = W.load_config3(n=n, seed=3, d=cfg.d)
    s = oracle.OracleSim(cfg, fp32=True)
    for sp, (x, v) in loads.items():
        s.inject(sp, x, v)
    t0 = time.perf_counter()
    s.step(spec["mode"], steps)
    el = time.perf_counter() - t0
    d = s.diag()
    return {"value": d["pushed_cum"] / el, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} initial H+ of the same workload, {steps} steps, binary32 oracle mode, "
                      f"{d['pushed_cum']} particle-steps in {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="beam_gap_4096c_2e7p_weak", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-steps", type=int, default=30)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--compact-every", type=int, default=32)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--deposit", type=int, default=0, help="0 auto, 1 64-bit LDS cells, 2 32-bit")
    ap.add_argument("--graph", type=int, default=0)
    ap.add_argument("--ppt", type=int, default=0, help="16-byte particle vectors per thread (1, 2)")
    ap.add_argument("--copy-reference-mb", type=int, default=0,
                    help="only run a plain device copy of this many MiB (5 times): the "
                         "reference that scales rocprof's FETCH_SIZE / WRITE_SIZE to bytes")
    ap.add_argument("--pmc-summary", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="no GPU work: reduce rocprofv3 counter CSVs of a bench run (same --steps) and of a "
                         "--copy-reference-mb 1024 run to the push kernel's bytes per launch, and write the record "
                         "that later bench runs report as roofline.traffic")
    args = ap.parse_args()
    if args.pmc_summary:
        rec = pmc_summary(*args.pmc_summary, copy_mb=1024, kernel="k_push", last_n=args.steps)
        rec["source_sha256"] = kernel_source_hash()
        rec["run"] = {"workload": args.workload, "steps": args.steps, "warmup": args.warmup,
                      "compact_every": args.compact_every}
        with open(TRAFFIC_RECORD, "w") as f:
            json.dump(rec, f, indent=1)
        print(json.dumps(rec))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this method has no multi-GPU path in this build "
              "(independent gaps would shard across GPUs with no exchange)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2603_24010_amd import gapsim
    torch.cuda.set_device(0)
    if args.copy_reference_mb:
        n = args.copy_reference_mb * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_reference_bytes_per_launch": 4 * n, "launches": 5}), flush=True)
        return
    # achievable HBM rate: a plain 1 GiB device-to-device copy, timed with events
    ca = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    cb = torch.empty_like(ca)
    cb.copy_(ca)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        cb.copy_(ca)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 10 * 2 * ca.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del ca, cb
    spec = WORKLOADS[args.workload]
    log(f"[bench] building workload {args.workload}")
    sim, cfg, _ = make_sim(args.workload, spec, args.warmup + args.steps)
    sim.set_option(gapsim.OPT_COMPACT_EVERY, args.compact_every)
    if args.block:
        sim.set_option(gapsim.OPT_BLOCK, args.block)
    if args.tile:
        sim.set_option(gapsim.OPT_TILE, args.tile)
    if args.grid:
        sim.set_option(gapsim.OPT_GRID, args.grid)
    if args.deposit:
        sim.set_option(gapsim.OPT_DEPOSIT, args.deposit)
    if args.ppt:
        sim.set_option(gapsim.OPT_PPT, args.ppt)
    tuned = bool(args.block or args.tile or args.grid or args.deposit or args.ppt or args.graph)
    mode = spec["mode"]
    log(f"[bench] warmup {args.warmup} steps")
    sim.step(mode, args.warmup)
    d0 = sim.diag(0)
    if args.graph:
        sim.set_option(gapsim.OPT_GRAPH, 1)
    else:
        sim.set_option(gapsim.OPT_TIMING, 1)
    sim.timing(reset=True)
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} steps")
    t0 = time.perf_counter()
    chunk = 250
    done = 0
    while done < args.steps:
        k = min(chunk, args.steps - done)
        sim.step(mode, k)
        done += k
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    d1 = sim.diag(0)
    tm = sim.timing(reset=True)
    pushed = d1["pushed_cum"] - d0["pushed_cum"]
    value = pushed / el
    push_s = tm["push_ms"] * 1e-3
    achieved = BYTES_PER_PUSH_F32 * pushed / push_s / 1e9 if push_s > 0 else None
    traffic = recorded_traffic(args.workload, args.steps, args.warmup, args.compact_every, tuned)
    out = {
        "metric": "particle-steps/s",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "cells": cfg.n_cells, "initial_particles": spec["n0"],
                   "beam_per_step": cfg.beam_per_step, "coupling": "weak" if mode else "strict",
                   "particles": "binary32", "field_circuit": "binary64",
                   "live_particles_end": int(d1["n_live"].sum())},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS if achieved else None, "traffic": traffic,
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                     "kernel": "k_push", "bytes_per_particle_step": BYTES_PER_PUSH_F32,
                     "algorithmic_bytes_per_launch": BYTES_PER_PUSH_F32 * pushed / max(1, tm["push_launches"]),
                     "avg_launch_ms": tm["push_ms"] / max(1, tm["push_launches"]),
                     "copy_GBps": copy_gbs,
                     "launches": tm["push_launches"]},
        "timed_with": "hip graphs" if args.graph else "eager launches, HIP events recorded by each kernel's dispatch",
        "kernel_ms_per_step": {"push": tm["push_ms"] / args.steps, "field": tm["field_ms"] / args.steps,
                               "source": tm["source_ms"] / args.steps,
                               "compact": tm["compact_ms"] / args.steps},
    }
    sim.close()
    if not args.no_cpu_baseline:
        log(f"[bench] cpu baseline: oracle, {args.cpu_steps} steps")
        out["cpu_baseline"] = cpu_baseline(spec, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
