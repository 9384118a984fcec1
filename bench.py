"""Throughput of the circuit-coupled ES-PIC step on one MI355X.

Default workload: the largest single-gap configuration, strict coupling on a
16384-cell gap holding 2e8 H+ macroparticles in binary32 (a Gaussian load at
0.9 d), 2e4 beam ions per step, coupled-LC circuit, SEE with exponential 3 eV
electrons; inputs resident in HBM before the timed region.  One step = circuit
+ field solve, gather/push/walls/SEE/beam/deposit for every particle, and the
periodic slot compaction (or cell sort): the timed window always ends with one,
so at least its amortised share is inside the measurement.  The launch shape
and the compaction interval come from the library's autotuner, run before the
timed region.

Prints one JSON line: particle-steps/s, the push kernel against the HBM
roofline (HIP events on the library's stream over the timed region), and the
CPU oracle timed on a bounded sample on the host.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E
STRICT, WEAK = 0, 1  # coupling modes in the library's numbering (gs_autotune, GapSim.step)
BYTES_PER_PUSH_F32 = 16  # read x, v and write x, v (binary32)

# HBM traffic of the push kernel, taken with rocprofv3 FETCH_SIZE / WRITE_SIZE
# runs of this script; it is reported only while the sources it was measured
# on are unchanged and the run is the one that was measured.
def traffic_record_path(workload):
    return os.path.join(ROOT, "profiles", f"k_push_traffic_{workload}.json")


DEFAULT_WORKLOAD = "beam_gap_16384c_2e8p_strict"
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
    # the default gap with the paper's SEE laws (Alg. 2): a fifth-order yield fit
    # clipped at zero and lognormal electron energies; the coefficients and (mu,
    # sigma) are stand-ins (the paper shows its fits only as figures)
    "beam_gap_4096c_2e7p_weak_paper_see": dict(n_cells=4096, n0=20_000_000, beam=20_000, mode=1,
                                               load="uniform", see="paper"),
}


def workload_cfg(spec):
    from paper_2603_24010_amd import workloads as W
    cfg = W.config2(n_cells=spec["n_cells"], beam_per_step=spec["beam"])
    if spec.get("see") == "paper":
        cfg = cfg.replace(see_amp=1.0, see_yield=W.YIELD_POLY,
                          see_poly=np.array([0.05, 0.12, -2.0e-3, 2.0e-5, -1.0e-7, 2.0e-10]),
                          see_poly_Emax_eV=8e4, see_law=W.SEE_LOGNORMAL, see_ln_mu=math.log(8.0),
                          see_ln_sigma=0.7)
    return cfg


def _finite(d):
    """JSON has no infinity: a non-finite float (no circuit resonance) becomes null."""
    return {k: (None if isinstance(v, float) and not math.isfinite(v) else v) for k, v in d.items()}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_sim(name, spec, total_steps):
    from paper_2603_24010_amd import gapsim, workloads as W
    cfg = workload_cfg(spec)
    if spec["load"] == "uniform":
        loads = W.load_config2(n=spec["n0"], seed=2, d=cfg.d)
    else:
        loads = W.load_config3(n=spec["n0"], seed=3, d=cfg.d)
    n_ion = spec["n0"]
    # every beam ion may still be in flight at the end (slow ones cross in
    # thousands of steps); each absorbed ion, loaded or beam, emits at most
    # see_amp secondary electrons, and the loaded ions are absorbed within a few
    # hundred steps
    grow = (total_steps + 64) * spec["beam"]
    n_sec = int(math.ceil(cfg.see_amp * (n_ion + grow)))
    cap = ((1 << 22) + n_sec, n_ion + grow + (1 << 20))
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


def run_key(workload, steps, warmup, launch):
    return {"workload": workload, "steps": steps, "warmup": warmup, "launch": launch}


def recorded_traffic(key):
    """Bytes per push launch from the committed counter record of this exact run
    (workload, steps, warmup and launch shape) on the current kernel sources, or None."""
    try:
        with open(traffic_record_path(key["workload"])) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != kernel_source_hash() or rec.get("run") != key:
        return None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


def host_cpu():
    """Model name of the host CPU and the threads the process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


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


# ---------------------------------------------------------------------------
# batched gaps (independent gaps of uneven particle counts and circuits)
# ---------------------------------------------------------------------------
BATCHED = {"batched_512gaps_512c_strict": dict(gaps=512, cells=512, seed0=0)}
MLP_WORKLOAD = "mlp_guess_512gaps_strict"


def make_batched(gaps, cells, seed0, total_steps, np_lo=50_000, np_hi=500_000):
    from paper_2603_24010_amd import gapsim, workloads as W
    cfgs, loads, caps = [], [], []
    for g in range(seed0, seed0 + gaps):
        cfg, n_p, e_b = W.config4_gap(g, n_cells=cells, np_lo=np_lo, np_hi=np_hi)
        cfgs.append(cfg)
        loads.append(W.load_config4_gap(n_p, e_b, g))
        # the beam keeps about n_p ions resident; room for fluctuations and for
        # the ions in flight when the run ends
        caps.append((n_p // 2 + 65536, int(1.3 * n_p) + 64 * cfg.beam_per_step + 4096))
    sim = gapsim.GapSim(cfgs, particle_fp=32, capacity=caps)
    for g in range(gaps):
        for sp, (x, v) in loads[g].items():
            sim.inject(g, sp, x, v)
    return sim, cfgs, sum(len(loads[g][1][0]) for g in range(gaps))


def pushed_total(sim):
    return sum(sim.diag(g)["pushed_cum"] for g in range(sim.G))


def eager_kernel_pass(sim, step, steps):
    """Per-kernel times over an eager pass with dispatch-recorded events."""
    from paper_2603_24010_amd import gapsim
    sim.set_option(gapsim.OPT_GRAPH, 0)
    sim.set_option(gapsim.OPT_TIMING, 1)
    sim.timing(reset=True)
    p0 = pushed_total(sim)
    step(steps)
    tm = sim.timing(reset=True)
    sim.set_option(gapsim.OPT_TIMING, 0)
    return tm, pushed_total(sim) - p0


def run_batched(args, name, copy_gbs):
    import torch
    from paper_2603_24010_amd import gapsim
    spec = BATCHED[name]
    log(f"[bench] building {spec['gaps']} gaps")
    sim, cfgs, n0 = make_batched(spec["gaps"], spec["cells"], spec["seed0"], args.warmup + args.steps + 128)
    log(f"[bench] {n0} initial particles; warmup {args.warmup} steps")
    step = lambda n: sim.step_strict(n, gapsim.GUESS_DIRECT)
    step(args.warmup)
    tuning = sim.autotune(0, gapsim.GUESS_DIRECT, trial_steps=8)
    log(f"[bench] autotuned: {tuning}")
    if args.sort_bin >= 0:
        # compare one sort setting against the tuned shape
        sim.set_option(gapsim.OPT_SORT_BIN, args.sort_bin)
        tuning = dict(tuning, sort_bin=args.sort_bin, forced="sort_bin")
    sim.set_option(gapsim.OPT_GRAPH, 1)
    # two intervals untimed: the graph of one interval is captured and
    # instantiated before the timed window, not inside it
    step(2 * tuning["compact_every"])
    torch.cuda.synchronize()
    p0 = pushed_total(sim)
    t0 = time.perf_counter()
    step(args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    pushed = pushed_total(sim) - p0
    tm, kp = eager_kernel_pass(sim, step, 64)
    push_s = tm["push_ms"] * 1e-3
    achieved = BYTES_PER_PUSH_F32 * kp / push_s / 1e9 if push_s > 0 else None
    live = sum(int(sim.diag(g)["n_live"].sum()) for g in range(sim.G))
    sim.close()
    out = {
        "metric": "particle-steps/s", "value": pushed / el, "unit": "particle-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": el * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": name, "gaps": spec["gaps"], "cells": spec["cells"], "initial_particles": n0,
                   "coupling": "strict", "particles": "binary32", "field_circuit": "binary64",
                   "live_particles_end": live, "tuning": tuning},
        "timed_with": "hip graphs, one per compaction interval",
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS if achieved else None, "traffic": None,
                     "kernel": "k_push", "bytes_per_particle_step": BYTES_PER_PUSH_F32,
                     "avg_launch_ms": tm["push_ms"] / max(1, tm["push_launches"]), "copy_GBps": copy_gbs,
                     "measured_over": "64 eager steps after the timed region, HIP events recorded by each "
                                      "kernel's dispatch"},
        "kernel_ms_per_step": {k[:-3]: tm[k] / 64 for k in ("push_ms", "field_ms", "compact_ms", "emit_ms")},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batched(spec, 4 * args.cpu_steps)
    print(json.dumps(out), flush=True)


def run_mlp(args, copy_gbs):
    """Newton guess network on batched strict gaps: record (input, target) pairs
    from the direct strict solve of a training ensemble, train the network on
    the GPU, then run held-out gaps with the plain extrapolated guess, the
    trained network and the untrained network, and one gap alone."""
    import torch
    from paper_2603_24010_amd import gapsim
    G, cells, steps_train, steps_eval = args.mlp_gaps, 512, args.mlp_train_steps, args.mlp_eval_steps
    skip = 11  # levels whose 8-level history and extrapolation reach before level 0
    # 1. training data
    log(f"[bench] mlp: {G} training gaps, {steps_train} recorded strict steps")
    sim, _, n0 = make_batched(G, cells, 0, steps_train)
    xr = torch.zeros((G * steps_train, 48), dtype=torch.float32, device="cuda")
    yr = torch.zeros((G * steps_train, 3), dtype=torch.float32, device="cuda")
    sim.mlp_record(xr, yr)
    sim.set_option(gapsim.OPT_GRAPH, 1)
    t0 = time.perf_counter()
    sim.step_strict(steps_train, gapsim.GUESS_DIRECT)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    sim.mlp_record()
    sim.close()
    x = xr[skip * G:].double()
    y = yr[skip * G:].double()
    x_mean, x_sd = x.mean(0), x.std(0)
    x_sd = torch.maximum(x_sd, 1e-6 * x.abs().max(0).values)
    x_sd[x_sd == 0] = 1.0
    y_mean, y_sd = y.mean(0), y.std(0)
    y_sd[y_sd == 0] = 1.0
    norm = torch.cat([x_mean, x_sd, y_mean, y_sd]).cpu().numpy()
    xn_all = ((x - x_mean) / x_sd).float()
    yn_all = ((y - y_mean) / y_sd).float()
    # how much of the target any linear function of the inputs explains (least
    # squares on the normalised data): the ceiling of an affine guess
    rng = np.random.default_rng(5)
    perm = torch.from_numpy(rng.permutation(xn_all.shape[0])).cuda()
    n_val = xn_all.shape[0] // 10
    val, trn = perm[:n_val], perm[n_val:]
    A = torch.cat([xn_all.double(), torch.ones((xn_all.shape[0], 1), dtype=torch.float64, device="cuda")], 1)
    wls = torch.linalg.lstsq(A[trn].cpu(), yn_all[trn].double().cpu()).solution.cuda()
    r_lin = yn_all[val].double() - A[val] @ wls
    r2_lin = (1.0 - r_lin.var(0) / yn_all[val].double().var(0)).cpu().numpy()
    xn = xn_all[trn].contiguous()
    yn = yn_all[trn].contiguous()
    xv = xn_all[val].contiguous()
    yv = yn_all[val].contiguous()
    del xr, yr, x, y, A, xn_all, yn_all
    n = xn.shape[0]
    # 2. training (Adam, batch 1024), seeded shuffles
    parts = []
    for fi, fo in ((48, 128), (128, 128), (128, 128), (128, 3)):
        bound = 1.0 / np.sqrt(fi)
        parts += [rng.uniform(-bound, bound, fo * fi), rng.uniform(-bound, bound, fo)]
    theta0 = np.concatenate(parts).astype(np.float32)
    th = torch.from_numpy(theta0.copy()).cuda()
    m, v = torch.zeros_like(th), torch.zeros_like(th)
    order = torch.from_numpy(np.concatenate([rng.permutation(n) for _ in range(args.mlp_epochs)])
                             .astype(np.int32)).cuda()
    B = 1024
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses, _ = gapsim.mlp_train(xn, yn, order, B, th, m, v, lr=1e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    losses = losses.cpu().numpy()
    n_steps_opt = len(losses)
    per_epoch = max(1, n_steps_opt // args.mlp_epochs)
    theta = th.cpu().numpy()
    # validation error of the bfloat16 network (the evaluation the strict step uses)
    probe, _, _ = make_batched(1, cells, 0, 1, np_lo=1000, np_hi=1000)

    def val_mse(weights):
        probe.mlp_set_weights(weights, norm)
        return float(((probe.mlp_forward(xv) - yv) ** 2).mean())

    val = {"trained": val_mse(theta), "untrained": val_mse(theta0), "zero": float((yv ** 2).mean())}
    probe.close()
    log(f"[bench] trained on {n} samples, {args.mlp_epochs} epochs: mean batch loss first epoch "
        f"{losses[:per_epoch].mean():.4g}, last epoch {losses[-per_epoch:].mean():.4g}; validation MSE {val}; "
        f"linear R^2 {r2_lin}")

    # 3. held-out gaps
    def evaluate(guess, weights, gaps, seed0, label):
        s, _, _ = make_batched(gaps, cells, seed0, steps_eval)
        if weights is not None:
            s.mlp_set_weights(weights, norm)
        s.set_option(gapsim.OPT_GRAPH, 1)
        r0 = []
        el = 0.0
        chunk = 100
        done = 0
        while done < steps_eval:
            k = min(chunk, steps_eval - done)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            s.step_strict(k, guess)
            torch.cuda.synchronize()
            el += time.perf_counter() - t1
            done += k
            if done > skip:
                r0 += [s.diag(g)["newton_resid0"] for g in range(gaps)]
        ds = [s.diag(g) for g in range(gaps)]
        s.close()
        tot = sum(d["newton_total"] for d in ds)
        lev = sum(d["newton_levels"] for d in ds)
        r0 = np.array(r0)
        res = {"corrections_per_level": tot / max(1, lev), "max_corrections": max(d["newton_max"] for d in ds),
               "levels": lev, "fallbacks": sum(d["newton_fallbacks"] for d in ds),
               "initial_residual": {"median": float(np.median(r0)), "p90": float(np.quantile(r0, 0.9)),
                                    "max": float(r0.max()), "below_tol": float(np.mean(r0 <= 1e-10)),
                                    "samples": int(r0.size)},
               "ms_per_step": el * 1e3 / steps_eval, "us_per_gap_step": el * 1e6 / (steps_eval * gaps)}
        log(f"[bench] {label}: {res}")
        return res

    plain = evaluate(gapsim.GUESS_EXTRAP, None, G, 512, "batched plain")
    trained = evaluate(gapsim.GUESS_MLP, theta, G, 512, "batched + trained network")
    untrained = evaluate(gapsim.GUESS_MLP, theta0, G, 512, "batched + untrained network")
    single = evaluate(gapsim.GUESS_EXTRAP, None, 1, 512, "single gap plain")
    flop_per_sample = 2 * 3 * (48 * 128 + 2 * 128 * 128 + 128 * 3)
    out = {
        "metric": "strict-step Newton updates per level at 1e-10 residual, network vs plain",
        "value": trained["corrections_per_level"], "unit": "updates/level", "n_gpus": 1,
        "steps": steps_eval, "warmup": 0, "ms_per_step": trained["ms_per_step"], "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 particles, f64 field/circuit, bf16 network",
        "data": "synthetic",
        "config": {"workload": MLP_WORKLOAD, "gaps": G, "cells": cells, "train_gaps_seeds": [0, G - 1],
                   "eval_gaps_seeds": [512, 512 + G - 1], "initial_particles_train": n0},
        "plain": plain, "trained": trained, "untrained": untrained, "single_gap_plain": single,
        "training": {"samples": n, "recorded_steps": steps_train, "generation_s": t_gen, "epochs": args.mlp_epochs,
                     "batch": B, "optimizer_steps": n_steps_opt,
                     "loss_first_epoch": float(losses[:per_epoch].mean()),
                     "loss_last_epoch": float(losses[-per_epoch:].mean()),
                     "validation_mse_normalised": val, "linear_least_squares_R2": [float(v) for v in r2_lin],
                     "seconds": t_train,
                     "samples_per_s": n_steps_opt * B / t_train,
                     "TFLOPs": n_steps_opt * B * flop_per_sample / t_train / 1e12},
        "copy_GBps": copy_gbs,
    }
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------------------
# the binary64 gap: 256 cells, 1e5 particles, series RC driven at 1 MHz
# ---------------------------------------------------------------------------
FP64_WORKLOAD = "rc_gap_256c_1e5p_strict_fp64"


def run_fp64(args, copy_gbs):
    import torch
    from paper_2603_24010_amd import gapsim, workloads as W
    cfg = W.config1()
    loads = W.load_config1(n_per_species=50_000, seed=0)
    sim = gapsim.GapSim(cfg, particle_fp=64, capacity=(200_000, 200_000))
    for sp, (x, v) in loads.items():
        sim.inject(0, sp, x, v)
    sim.set_option(gapsim.OPT_GRAPH, 1)
    # two compaction intervals (32 steps) untimed: the graph is captured and
    # instantiated before the timed window
    warm = 64
    sim.step_strict(warm)
    torch.cuda.synchronize()
    p0 = sim.diag(0)["pushed_cum"]
    t0 = time.perf_counter()
    sim.step_strict(args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    d = sim.diag(0)
    tm, kp = eager_kernel_pass(sim, lambda n: sim.step_strict(n), 64)
    sim.close()
    push_s = tm["push_ms"] * 1e-3
    achieved = 32 * kp / push_s / 1e9 if push_s > 0 else None
    out = {
        "metric": "particle-steps/s", "value": (d["pushed_cum"] - p0) / el, "unit": "particle-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": warm, "ms_per_step": el * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": FP64_WORKLOAD, "cells": cfg.n_cells, "particles": 100_000, "coupling": "strict"},
        "timed_with": "hip graphs",
        "roofline": {"bound": "latency", "kernel": "k_push", "achieved": achieved, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS if achieved else None, "traffic": None,
                     "bytes_per_particle_step": 32, "avg_launch_ms": tm["push_ms"] / max(1, tm["push_launches"]),
                     "copy_GBps": copy_gbs,
                     "note": "1e5 particles move 3.2 MB per step: launch and latency bound, a parity configuration"},
        "kernel_ms_per_step": {k[:-3]: tm[k] / 64 for k in ("push_ms", "field_ms", "compact_ms")},
    }
    if not args.no_cpu_baseline:
        import oracle
        s = oracle.OracleSim(cfg, fp32=False)
        for sp, (x, v) in loads.items():
            s.inject(sp, x, v)
        t0 = time.perf_counter()
        s.step(oracle.STRICT, args.steps)
        elc = time.perf_counter() - t0
        pc = s.diag()["pushed_cum"]
        out["cpu_baseline"] = {"value": pc / elc, "unit": "particle-steps/s", "cores": 1, "cpu_model": host_cpu()[0], "kind": "oracle",
                               "sample": f"the whole run: {args.steps} strict steps, binary64, {pc} particle-steps "
                                         f"in {elc:.1f} s"}
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------------------
# strict and weak coupling on the same large gap: the divergence between them
# ---------------------------------------------------------------------------
DIVERGENCE = "strict_vs_weak_16384c_2e8p"


def run_divergence(args, copy_gbs):
    import torch
    from paper_2603_24010_amd import gapsim, workloads as W
    n0, every = args.div_particles, 10
    cfg = W.config3(beam_per_step=20000)
    log(f"[bench] loading {n0} particles (Gaussian at 0.9 d, sigma 0.05 d)")
    loads = W.load_config3(n=n0, seed=3, d=cfg.d)
    grow = (args.steps + 64) * cfg.beam_per_step
    # the load sits 0.1 d from the grounded electrode: nearly every ion reaches
    # it within a few hundred steps, each freeing about a / 2 electrons
    cap = (int(0.55 * (n0 + grow)) + (1 << 22), n0 + grow + (1 << 20))
    sims = []
    for mode in (0, 1):
        s = gapsim.GapSim(cfg, particle_fp=32, capacity=cap)
        for sp, (x, v) in loads.items():
            s.inject(0, sp, x, v)
        # the launch the autotuner picks for this gap and mode (cached per shape)
        s.autotune(mode, gapsim.GUESS_DIRECT, trial_steps=8, cache_path=args.tuning_cache or None)
        sims.append(s)
    del loads
    launches = [s.launch() for s in sims]
    rec = {0: [], 1: []}
    el = {0: 0.0, 1: 0.0}
    pushed = {0: 0, 1: 0}
    done = 0
    while done < args.steps:
        k = min(every, args.steps - done)
        for mode, s in enumerate(sims):
            p0 = s.diag(0)["pushed_cum"]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.step(mode, k)
            torch.cuda.synchronize()
            el[mode] += time.perf_counter() - t0
            d = s.diag(0)
            pushed[mode] += d["pushed_cum"] - p0
            rec[mode].append((d["step"], d["phi0"], d["sigma"]))
        done += k
        if done % 500 == 0:
            log(f"[bench] {done} steps")
    tm = {}
    for mode, s in enumerate(sims):
        t, _ = eager_kernel_pass(s, lambda n, s=s, m=mode: s.step(m, n), 32)
        tm[mode] = t["push_ms"] / max(1, t["push_launches"])
    live = [int(s.diag(0)["n_live"].sum()) for s in sims]
    for s in sims:
        s.close()
    S, Wk = np.array(rec[0]), np.array(rec[1])
    dv = np.abs(S[:, 1] - Wk[:, 1])
    ds = np.abs(S[:, 2] - Wk[:, 2])
    vscale, sscale = np.abs(S[:, 1]).max(), np.abs(S[:, 2]).max()
    out = {
        "metric": "strict-weak divergence of gap voltage and surface charge; particle-steps/s",
        "value": (pushed[0] + pushed[1]) / (el[0] + el[1]), "unit": "particle-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 0, "ms_per_step": (el[0] + el[1]) * 1e3 / (2 * args.steps),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": DIVERGENCE, "cells": cfg.n_cells, "initial_particles": n0,
                   "beam_per_step": cfg.beam_per_step, "live_particles_end": live},
        "strict": {"particle_steps_per_s": pushed[0] / el[0], "push_ms": tm[0], "launch": launches[0]},
        "weak": {"particle_steps_per_s": pushed[1] / el[1], "push_ms": tm[1], "launch": launches[1]},
        "divergence": {
            "sampled_every": every,
            "max_abs_dV": float(dv.max()), "max_rel_dV": float(dv.max() / vscale),
            "final_abs_dV": float(dv[-1]), "max_abs_dsigma": float(ds.max()),
            "max_rel_dsigma": float(ds.max() / sscale), "V_scale": float(vscale),
            "curve": [[int(S[i, 0]), float(S[i, 1]), float(Wk[i, 1]), float(S[i, 2]), float(Wk[i, 2])]
                      for i in range(0, len(S), max(1, len(S) // 40))],
        },
        "roofline": {"bound": "hbm", "kernel": "k_push", "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "achieved": None, "frac": None, "traffic": None, "copy_GBps": copy_gbs},
    }
    print(json.dumps(out), flush=True)


TESLA_WORKLOAD = "tesla_600c_ground_pulse"


def _collapse_metrics(V, dt):
    """Bottom of the negative swing the pulse rides on, the first step after it
    with V above -3 kV, and the next positive peak."""
    lo = 250 + int(np.argmin(V[250:400]))
    up = lo + int(np.argmax(V[lo:] > -3e3))
    return {"swing_bottom_kV": float(V[lo] / 1e3), "swing_bottom_us": lo * dt * 1e6,
            "above_minus3kV_us": up * dt * 1e6, "next_peak_kV": float(V[lo:].max() / 1e3)}


def run_tesla(args, copy_gbs):
    """The paper's integrated Tesla run (Sec. 4.2) with stand-in pulse, layer,
    entry energies and yield law: strict and weak, with and without ion-induced
    emission, the whole 575 steps each on the GPU; the oracle (binary32 mode)
    timed on the same runs."""
    import torch
    from paper_2603_24010_amd import gapsim, workloads as W
    from paper_2603_24010_amd.engines import RadauCircuitEngine
    ENGINE = -1
    cfg0 = W.config_tesla()
    steps = len(cfg0.beam_schedule)
    cases = [("strict_see", STRICT, cfg0), ("weak_see", WEAK, cfg0),
             ("strict_no_see", STRICT, cfg0.replace(see_amp=0.0)),
             ("weak_no_see", WEAK, cfg0.replace(see_amp=0.0))]
    # weak coupling with the circuit in an external stiff engine (Radau IIA), the
    # way the paper's weak mode hands the circuit to a SPICE engine
    cases.append(("weak_engine_see", ENGINE, cfg0))
    res, curves, el_all, pushed_all = {}, {}, 0.0, 0
    for name, mode, cfg in cases:
        s = gapsim.GapSim(cfg, particle_fp=32, capacity=(3_000_000, 4_000_000))
        eng = RadauCircuitEngine(cfg) if mode == ENGINE else None
        V = np.zeros(steps)
        # App. D's a posteriori check, outside the timed part of each step
        chk = {"omega_pe_max": 0.0, "alpha_max": 0.0, "v_e_max": 0.0, "beta_max": [0.0, 0.0], "eta_max": 0.0,
               "n_e_max": 0.0, "flagged_steps": 0}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        el = 0.0
        for n in range(steps):
            if eng is not None:
                s.step_weak_external(1, eng)
            else:
                s.step(mode, 1)
            torch.cuda.synchronize()
            el += time.perf_counter() - t0
            V[n] = s.diag(0)["phi0"]
            r = s.dt_check(0)
            chk["omega_pe_max"] = max(chk["omega_pe_max"], r["omega_pe"])
            chk["alpha_max"] = max(chk["alpha_max"], r["alpha"])
            chk["n_e_max"] = max(chk["n_e_max"], r["n_e_max"])
            chk["v_e_max"] = max(chk["v_e_max"], float(r["v_max"][0]))
            chk["beta_max"] = [max(a, float(b)) for a, b in zip(chk["beta_max"], r["beta"])]
            chk["eta_max"] = max(chk["eta_max"], r["eta"])
            chk["flagged_steps"] += int(r["flags"] != 0)
            chk["omega_max"], chk["n_omega"] = r["omega_max"], r["n_omega"]
            t0 = time.perf_counter()
        d = s.diag(0)
        s.close()
        el_all += el
        pushed_all += d["pushed_cum"]
        curves[name] = V
        res[name] = dict(_collapse_metrics(V, cfg.dt), particle_steps=int(d["pushed_cum"]),
                         wall_s=el, injected=int(d["inj_cum"]), emitted=int(d["emit_cum"].sum()),
                         absorbed=[int(x) for x in d["abs_cum"].ravel()], time_step_check=_finite(chk))
        log(f"[bench] {name}: {res[name]}")
    rmse = lambda a, b: float(np.sqrt(np.mean((curves[a] - curves[b]) ** 2)) / 1e3)
    # the circuit alone (no particles): the library's BDF2 levels (strict steps
    # of an empty gap) and a Radau IIA step at the same dt, each against Radau on
    # a 16 times finer grid
    vac_cfg = cfg0.replace(see_amp=0.0, beam_schedule=None)
    vs = gapsim.GapSim(vac_cfg, particle_fp=32, capacity=(64, 64))
    v_bdf2 = []
    for _ in range(steps):
        vs.step_strict(1)
        v_bdf2.append(vs.diag(0)["phi0"])
    vs.close()
    v_bdf2 = np.array(v_bdf2)
    fine = RadauCircuitEngine(vac_cfg.replace(dt=vac_cfg.dt / 16))
    p, ref = 0.0, []
    for k in range(16 * steps):
        p = fine(0, k, vac_cfg.dt / 16, p)
        if k % 16 == 15:
            ref.append(p)
    coarse = RadauCircuitEngine(vac_cfg)
    p, v_rad = 0.0, []
    for k in range(steps):
        p = coarse(0, k, vac_cfg.dt, p)
        v_rad.append(p)
    ref = np.array(ref)
    vac = {"bdf2": float(np.sqrt(np.mean((v_bdf2 - ref) ** 2)) / 1e3),
           "radau": float(np.sqrt(np.mean((np.array(v_rad) - ref) ** 2)) / 1e3),
           "note": "BDF2's constant-history start puts its waveform half a step behind"}
    out = {
        "metric": "Tesla-run waveform (collapse with vs without SEE, strict vs weak RMSE); particle-steps/s",
        "value": pushed_all / el_all, "unit": "particle-steps/s", "n_gpus": 1, "steps": steps, "warmup": 0,
        "ms_per_step": el_all * 1e3 / (len(cases) * steps), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": TESLA_WORKLOAD, "cells": cfg0.n_cells, "dt_ns": cfg0.dt * 1e9,
                   "beam": "Gaussian pulse at the grounded electrode, stand-in: peak 4e4 ions/step at 4.5 us, "
                           "width 50 steps, 2 mm layer, 10-50 eV; yield 3 E/(E + 20 keV)",
                   "injected": int(cfg0.beam_schedule.sum())},
        "cases": res,
        "strict_weak_rmse_kV": {"see": rmse("strict_see", "weak_see"), "no_see": rmse("strict_no_see", "weak_no_see"),
                                "strict_vs_weak_external_engine_see": rmse("strict_see", "weak_engine_see"),
                                "weak_vs_weak_external_engine_see": rmse("weak_see", "weak_engine_see"),
                                "paper_context_kV": 0.228},
        "vacuum_circuit_rmse_vs_converged_kV": vac,
        "curve_kV": [[round(n * cfg0.dt * 1e6, 3)] + [round(float(curves[c][n]) / 1e3, 3) for c, _, _ in cases]
                     for n in range(0, steps, 5)],
        "roofline": {"bound": "latency", "kernel": "k_push", "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "achieved": None, "frac": None, "traffic": None, "copy_GBps": copy_gbs,
                     "note": "at most ~1.3e6 live particles: each step is a few launches of short kernels"},
    }
    if not args.no_cpu_baseline:
        import oracle
        pc, elc = 0, 0.0
        for name, mode, cfg in cases:
            o = oracle.OracleSim(cfg, fp32=True)
            t0 = time.perf_counter()
            if mode == ENGINE:
                o.step_external(RadauCircuitEngine(cfg), steps)
            else:
                o.step(mode, steps)
            elc += time.perf_counter() - t0
            pc += o.diag()["pushed_cum"]
        out["cpu_baseline"] = {"value": pc / elc, "unit": "particle-steps/s", "cores": 1, "cpu_model": host_cpu()[0], "kind": "oracle",
                               "sample": f"the same {len(cases)} runs, {steps} steps each, binary32 oracle mode, "
                                         f"{pc} particle-steps in {elc:.1f} s"}
    print(json.dumps(out), flush=True)


EXTERNAL_WORKLOAD = "beam_gap_4096c_2e7p_external_engine"


def run_external(args, copy_gbs):
    """The default beam gap (4096 cells, 2e7 H+, coupled LC) in weak coupling with
    the circuit stepped by an external engine (the package's exact linear engine,
    in Python) through gs_step_weak_external, against the same run with the
    library's own weak circuit.  Both read the diagnostics every 25 steps; the
    external path also waits for the device once per step to exchange voltages."""
    import torch
    from paper_2603_24010_amd import gapsim
    from paper_2603_24010_amd.engines import LinearCircuitEngine
    spec = WORKLOADS["beam_gap_4096c_2e7p_weak"]
    K, Wm = args.steps, args.warmup
    res, series = {}, {}
    for case in ("internal", "external"):
        sim, cfg, _ = make_sim(case, spec, Wm + K)
        # the launch shape the autotuner picks for this gap (its cache shared with
        # the plain workloads), with the library's own weak circuit in the trials
        tuning = sim.autotune(1, gapsim.GUESS_DIRECT, trial_steps=8, cache_path=args.tuning_cache or None)
        sim.set_option(gapsim.OPT_COMPACT_EVERY, args.compact_every or tuning["compact_every"])
        eng = LinearCircuitEngine(cfg)
        in_engine = [0.0]

        def timed_engine(g, n, dt, p):
            t = time.perf_counter()
            v = eng(g, n, dt, p)
            in_engine[0] += time.perf_counter() - t
            return v

        def advance(k):
            if case == "internal":
                sim.step_weak(k)
            else:
                sim.step_weak_external(k, timed_engine)
        # the field solve's time from the warmup steps (events on every launch);
        # in the timed steps only the push launches carry events
        sim.set_option(gapsim.OPT_TIMING, 1)
        sim.timing(reset=True)
        advance(Wm)
        tw = sim.timing(reset=True)
        d0 = sim.diag(0)
        sim.set_option(gapsim.OPT_TIMING, 2)
        sim.timing(reset=True)
        in_engine[0] = 0.0
        V = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = 0
        while done < K:
            k = min(25, K - done)
            advance(k)
            done += k
            V.append(sim.diag(0)["phi0"])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        d1 = sim.diag(0)
        tm = sim.timing(reset=True)
        pushed = d1["pushed_cum"] - d0["pushed_cum"]
        res[case] = {"particle_steps_per_s": pushed / el, "ms_per_step": el * 1e3 / K,
                     "push_us": tm["push_ms"] * 1e3 / max(1, tm["push_launches"]),
                     "field_us": tw["field_ms"] * 1e3 / max(1, tw["field_launches"]),
                     "launch": sim.launch(),
                     "engine_us_per_step": in_engine[0] * 1e6 / K, "pushed": int(pushed),
                     "push_GBps": BYTES_PER_PUSH_F32 * pushed / (tm["push_ms"] * 1e-3) / 1e9}
        series[case] = np.array(V)
        log(f"[bench] {case}: {res[case]}")
        sim.close()
    ex, it = res["external"], res["internal"]
    dv = float(np.abs(series["external"] - series["internal"]).max() / np.abs(series["internal"]).max())
    out = {
        "metric": "particle-steps/s, weak coupling with an external circuit engine",
        "value": ex["particle_steps_per_s"], "unit": "particle-steps/s", "n_gpus": 1, "steps": K, "warmup": Wm,
        "ms_per_step": ex["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": EXTERNAL_WORKLOAD, "cells": 4096, "initial_particles": spec["n0"],
                   "beam_per_step": spec["beam"], "engine": "exact linear (expm) coupled-LC engine in Python",
                   "coupling": "weak, external circuit engine"},
        "cases": res,
        "overhead_us_per_step": (ex["ms_per_step"] - it["ms_per_step"]) * 1e3,
        "gap_voltage_max_rel_diff_vs_internal_weak": dv,
        "roofline": {"bound": "hbm", "kernel": "k_push", "achieved": ex["push_GBps"], "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": ex["push_GBps"] / PEAK_HBM_GBS, "traffic": None,
                     "avg_launch_ms": ex["push_us"] * 1e-3, "copy_GBps": copy_gbs,
                     "bytes_per_particle_step": BYTES_PER_PUSH_F32},
    }
    if not args.no_cpu_baseline:
        import oracle
        from paper_2603_24010_amd import workloads as W
        cfg = W.config2(n_cells=4096, beam_per_step=spec["beam"])
        n = spec["n0"]
        o = oracle.OracleSim(cfg, fp32=True)
        for sp, (x, v) in W.load_config2(n=n, seed=2, d=cfg.d).items():
            o.inject(sp, x, v)
        eng = LinearCircuitEngine(cfg)
        steps = max(4, args.cpu_steps)
        t0 = time.perf_counter()
        o.step_external(eng, steps)
        elc = time.perf_counter() - t0
        pc = o.diag()["pushed_cum"]
        out["cpu_baseline"] = {"value": pc / elc, "unit": "particle-steps/s", "cores": 1, "cpu_model": host_cpu()[0], "kind": "oracle",
                               "sample": f"{n} initial H+ of the same workload, {steps} external-engine steps, "
                                         f"binary32 oracle mode, {pc} particle-steps in {elc:.1f} s"}
    print(json.dumps(out), flush=True)


TESLA_FINE_WORKLOAD = "tesla_600c_ground_pulse_dt15ps"


def run_tesla_fine(args, copy_gbs):
    """The Tesla run at the time step App. D verifies (1.5e-11 s, 575000 steps for
    the same 8.62 us and the same physical pulse), where the stand-in run keeps
    the particle constraints: strict and weak with and without emission, and weak
    with the circuit in an external Radau engine; graphs replay the steps, the
    gap voltage is read every 100 steps and the time-step check every 1000."""
    import torch
    from paper_2603_24010_amd import gapsim, workloads as W
    from paper_2603_24010_amd.engines import RadauCircuitEngine
    ENGINE = -1
    cfg0 = W.config_tesla(dt=1.5e-11)
    steps, every, chk_every = len(cfg0.beam_schedule), 100, 1000
    cases = [("strict_see", STRICT, cfg0), ("weak_see", WEAK, cfg0),
             ("strict_no_see", STRICT, cfg0.replace(see_amp=0.0)),
             ("weak_no_see", WEAK, cfg0.replace(see_amp=0.0)), ("weak_engine_see", ENGINE, cfg0)]
    res, curves, el_all, pushed_all = {}, {}, 0.0, 0
    for name, mode, cfg in cases:
        s = gapsim.GapSim(cfg, particle_fp=32, capacity=(3_000_000, 4_000_000))
        s.set_option(gapsim.OPT_COMPACT_EVERY, 50)
        eng = RadauCircuitEngine(cfg) if mode == ENGINE else None
        if eng is None:
            s.set_option(gapsim.OPT_GRAPH, 1)
        V = []
        chk = {"omega_pe_max": 0.0, "alpha_max": 0.0, "v_e_max": 0.0, "beta_max": [0.0, 0.0], "eta_max": 0.0,
               "n_e_max": 0.0, "flagged_checks": 0, "checks": 0}
        el = 0.0
        for n0 in range(0, steps, every):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if eng is not None:
                s.step_weak_external(every, eng)
            else:
                s.step(mode, every)
            torch.cuda.synchronize()
            el += time.perf_counter() - t0
            V.append(s.diag(0)["phi0"])
            if (n0 + every) % chk_every == 0:
                r = s.dt_check(0)
                chk["omega_pe_max"] = max(chk["omega_pe_max"], r["omega_pe"])
                chk["alpha_max"] = max(chk["alpha_max"], r["alpha"])
                chk["n_e_max"] = max(chk["n_e_max"], r["n_e_max"])
                chk["v_e_max"] = max(chk["v_e_max"], float(r["v_max"][0]))
                chk["beta_max"] = [max(a, float(b)) for a, b in zip(chk["beta_max"], r["beta"])]
                chk["eta_max"] = max(chk["eta_max"], r["eta"])
                chk["flagged_checks"] += int(r["flags"] != 0)
                chk["checks"] += 1
                chk["n_omega"] = r["n_omega"]
        d = s.diag(0)
        s.close()
        V = np.array(V)
        el_all += el
        pushed_all += d["pushed_cum"]
        curves[name] = V
        dts = cfg.dt * every
        lo = int(np.argmin(V[int(4.0e-6 / dts):int(6.0e-6 / dts)])) + int(4.0e-6 / dts)
        up = lo + int(np.argmax(V[lo:] > -3e3))
        res[name] = {"swing_bottom_kV": float(V[lo] / 1e3), "swing_bottom_us": (lo + 1) * dts * 1e6,
                     "above_minus3kV_us": (up + 1) * dts * 1e6, "next_peak_kV": float(V[lo:].max() / 1e3),
                     "particle_steps": int(d["pushed_cum"]), "wall_s": el, "injected": int(d["inj_cum"]),
                     "emitted": int(d["emit_cum"].sum()), "absorbed": [int(x) for x in d["abs_cum"].ravel()],
                     "time_step_check": _finite(chk)}
        log(f"[bench] {name}: {res[name]}")
    rmse = lambda a, b: float(np.sqrt(np.mean((curves[a] - curves[b]) ** 2)) / 1e3)
    out = {
        "metric": "Tesla-run waveform at dt = 1.5e-11 s (collapse with vs without SEE, strict vs weak RMSE); "
                  "particle-steps/s",
        "value": pushed_all / el_all, "unit": "particle-steps/s", "n_gpus": 1, "steps": steps, "warmup": 0,
        "ms_per_step": el_all * 1e3 / (len(cases) * steps), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": TESLA_FINE_WORKLOAD, "cells": cfg0.n_cells, "dt_s": cfg0.dt,
                   "beam": "the 15 ns run's stand-in pulse in physical time: 40 ions per 15 ps step at 4.5 us, "
                           "0.75 us width, 2 mm layer, 10-50 eV; yield 3 E/(E + 20 keV)",
                   "injected": int(cfg0.beam_schedule.sum()), "timed_with": "hip graphs (engine case eager)"},
        "cases": res,
        "strict_weak_rmse_kV": {"see": rmse("strict_see", "weak_see"), "no_see": rmse("strict_no_see", "weak_no_see"),
                                "strict_vs_weak_external_engine_see": rmse("strict_see", "weak_engine_see"),
                                "paper_context_kV": 0.228},
        "curve_kV_every_5ns": [[round((k + 1) * cfg0.dt * every * 1e6, 4)] +
                               [round(float(curves[c][k]) / 1e3, 3) for c, _, _ in cases]
                               for k in range(0, len(curves["strict_see"]), 50)],
        "roofline": {"bound": "latency", "kernel": "k_push", "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "achieved": None, "frac": None, "traffic": None, "copy_GBps": copy_gbs,
                     "note": "at most ~1.3e6 live particles: each step is a few short launches"},
    }
    if not args.no_cpu_baseline:
        # the oracle from level 0 into the rise of the pulse (about 25 s on one core)
        import oracle
        o = oracle.OracleSim(cfg0, fp32=True)
        n = 245_000
        t0 = time.perf_counter()
        o.step(oracle.STRICT, n)
        elc = time.perf_counter() - t0
        pc = o.diag()["pushed_cum"]
        out["cpu_baseline"] = {"value": pc / elc, "unit": "particle-steps/s", "cores": 1, "cpu_model": host_cpu()[0], "kind": "oracle",
                               "sample": f"strict with SEE, levels 0..{n - 1} (the pulse's rise), binary32 "
                                         f"oracle mode, {pc} particle-steps in {elc:.1f} s"}
    print(json.dumps(out), flush=True)


def cpu_baseline_batched(spec, steps):
    import oracle
    from paper_2603_24010_amd import workloads as W
    gaps = 16
    pushed, el = 0, 0.0
    for g in range(spec["seed0"], spec["seed0"] + gaps):
        cfg, n_p, e_b = W.config4_gap(g, n_cells=spec["cells"])
        s = oracle.OracleSim(cfg, fp32=True)
        for sp, (x, v) in W.load_config4_gap(n_p, e_b, g).items():
            s.inject(sp, x, v)
        t0 = time.perf_counter()
        s.step(oracle.STRICT, steps)
        el += time.perf_counter() - t0
        pushed += s.diag()["pushed_cum"]
    return {"value": pushed / el, "unit": "particle-steps/s", "cores": 1, "cpu_model": host_cpu()[0], "kind": "oracle",
            "sample": f"the first {gaps} gaps of the ensemble, {steps} strict steps each, binary32 oracle mode, "
                      f"{pushed} particle-steps in {el:.1f} s"}


def cpu_baseline(spec, steps: int):
    """The oracle (binary32 mode, one thread) on the workload's initial state."""
    import oracle
    from paper_2603_24010_amd import workloads as W
    cfg = workload_cfg(spec)
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
    return {"value": d["pushed_cum"] / el, "unit": "particle-steps/s", "cores": 1, "cpu_model": host_cpu()[0], "kind": "oracle",
            "sample": f"{n} initial H+ of the same workload, {steps} steps, binary32 oracle mode, "
                      f"{d['pushed_cum']} particle-steps in {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD,
                    choices=sorted(WORKLOADS) + sorted(BATCHED) + [MLP_WORKLOAD, DIVERGENCE, FP64_WORKLOAD,
                                                                   TESLA_WORKLOAD, EXTERNAL_WORKLOAD,
                                                                   TESLA_FINE_WORKLOAD])
    ap.add_argument("--div-particles", type=int, default=200_000_000)
    ap.add_argument("--cpu-steps", type=int, default=60)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--compact-every", type=int, default=0,
                    help="steps between compactions (or cell sorts); 0: the autotuner's choice (32 without it)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="single-gap workloads: keep the default launch shape instead of the autotuner's")
    ap.add_argument("--tuning-cache", default=os.path.join(ROOT, "paper_2603_24010_amd", "tuning_cache.txt"),
                    help="the autotuner's cache of choices per workload shape and device ('' for none)")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--deposit", type=int, default=0, help="0 auto, 1 64-bit LDS cells, 2 32-bit")
    ap.add_argument("--graph", type=int, default=0)
    ap.add_argument("--ppt", type=int, default=0, help="16-byte particle vectors per thread (1, 2)")
    ap.add_argument("--stream", type=int, default=-1,
                    help="push particle stream bits: 1 round-robin tile order, 2 non-temporal (-1: tuned)")
    ap.add_argument("--sort-bin", type=int, default=-1,
                    help="cells per bin of the periodic cell sort (0: plain compaction; -1: the autotuner's or 0)")
    ap.add_argument("--mlp-gaps", type=int, default=512)
    ap.add_argument("--mlp-train-steps", type=int, default=2000)
    ap.add_argument("--mlp-eval-steps", type=int, default=500)
    ap.add_argument("--mlp-epochs", type=int, default=10)
    ap.add_argument("--copy-reference-mb", type=int, default=0,
                    help="only run a plain device copy of this many MiB (5 times): the "
                         "reference that scales rocprof's FETCH_SIZE / WRITE_SIZE to bytes")
    ap.add_argument("--pmc-summary", nargs=5,
                    metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV", "BENCH_JSON"),
                    help="no GPU work: reduce rocprofv3 counter CSVs of a bench run (its JSON line in BENCH_JSON) "
                         "and of a --copy-reference-mb 1024 run to the push kernel's bytes per launch, and write "
                         "the record that later runs of the same command report as roofline.traffic")
    args = ap.parse_args()
    if args.pmc_summary:
        with open(args.pmc_summary[4]) as f:
            run = json.loads([ln for ln in f if ln.startswith("{")][-1])
        rec = pmc_summary(*args.pmc_summary[:4], copy_mb=1024, kernel="k_push", last_n=run["roofline"]["launches"])
        rec["source_sha256"] = kernel_source_hash()
        rec["run"] = run["roofline"]["run_key"]
        rec["algorithmic_bytes_per_launch"] = run["roofline"]["algorithmic_bytes_per_launch"]
        with open(traffic_record_path(rec["run"]["workload"]), "w") as f:
            json.dump(rec, f, indent=1)
        print(json.dumps(rec))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
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
    if args.workload in BATCHED:
        return run_batched(args, args.workload, copy_gbs)
    if args.workload == MLP_WORKLOAD:
        return run_mlp(args, copy_gbs)
    if args.workload == DIVERGENCE:
        return run_divergence(args, copy_gbs)
    if args.workload == FP64_WORKLOAD:
        return run_fp64(args, copy_gbs)
    if args.workload == TESLA_WORKLOAD:
        return run_tesla(args, copy_gbs)
    if args.workload == EXTERNAL_WORKLOAD:
        return run_external(args, copy_gbs)
    if args.workload == TESLA_FINE_WORKLOAD:
        return run_tesla_fine(args, copy_gbs)
    spec = WORKLOADS[args.workload]
    log(f"[bench] building workload {args.workload}")
    sim, cfg, _ = make_sim(args.workload, spec, args.warmup + args.steps + 128)
    manual = bool(args.block or args.tile or args.grid or args.deposit or args.ppt or args.sort_bin >= 0
                  or args.stream >= 0)
    if args.sort_bin >= 0:
        sim.set_option(gapsim.OPT_SORT_BIN, args.sort_bin)
    if args.stream >= 0:
        sim.set_option(gapsim.OPT_STREAM, args.stream)
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
    mode = spec["mode"]
    tuning = None
    if not (manual or args.no_autotune):
        # the autotuner times candidate launch shapes and compaction intervals on
        # this state (which it restores); a cached choice for this shape is reused
        log("[bench] autotuning")
        tuning = sim.autotune(mode, gapsim.GUESS_DIRECT, trial_steps=8, cache_path=args.tuning_cache or None)
        log(f"[bench] tuning: {tuning}")
    interval = args.compact_every or (tuning["compact_every"] if tuning else 32)
    # a timed window shorter than the interval holds one compaction all the
    # same (it ends with one), which would charge the whole interval's
    # compaction to fewer steps: the interval is then the window's length
    if not args.compact_every and args.steps < interval:
        interval = args.steps
    sim.set_option(gapsim.OPT_COMPACT_EVERY, interval)
    launch = sim.launch()
    log(f"[bench] warmup {args.warmup} steps")
    sim.step(mode, args.warmup)
    # the timed window ends with a compaction: at least its amortised share is
    # inside the measurement (one per window when the window is shorter than the
    # interval).  The steps in between, at least one interval and so at least one
    # compaction, give the per-kernel breakdown with events on every launch (an
    # evented launch leaves the queue idle for some microseconds, so the timed
    # window puts events on the push alone).
    align = (-(args.warmup + args.steps)) % interval + interval
    sim.set_option(gapsim.OPT_TIMING, 1)
    sim.timing(reset=True)
    sim.step(mode, align)
    tb = sim.timing(reset=True)
    sim.set_option(gapsim.OPT_TIMING, 0)
    d0 = sim.diag(0)
    if args.graph:
        sim.set_option(gapsim.OPT_GRAPH, 1)
    else:
        sim.set_option(gapsim.OPT_TIMING, 2)
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
    dtc = sim.dt_check(0)  # App. D's constraints at the last step (after the timed region)
    pushed = d1["pushed_cum"] - d0["pushed_cum"]
    value = pushed / el
    push_s = tm["push_ms"] * 1e-3
    achieved = BYTES_PER_PUSH_F32 * pushed / push_s / 1e9 if push_s > 0 else None
    key = run_key(args.workload, args.steps, args.warmup, launch)
    traffic = None if args.graph else recorded_traffic(key)
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
                   "live_particles_end": int(d1["n_live"].sum()),
                   "see": ("paper laws: fifth-order yield (stand-in coefficients), lognormal energies "
                           "(mu ln 8 eV, sigma 0.7)") if spec.get("see") == "paper"
                   else "saturating yield 0.5 E/(E + 1 keV), Exp(3 eV)",
                   "emitted_in_timed_steps": int((d1["emit_cum"] - d0["emit_cum"]).sum()),
                   "launch": launch, "autotuned": tuning is not None,
                   "autotuned_compact_every": tuning["compact_every"] if tuning else None,
                   "untimed_steps_before": args.warmup + align,
                   "compactions_in_timed_steps": (args.warmup + align + args.steps) // interval
                   - (args.warmup + align) // interval},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS if achieved else None, "traffic": traffic,
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                     "kernel": "k_push", "bytes_per_particle_step": BYTES_PER_PUSH_F32,
                     "algorithmic_bytes_per_launch": BYTES_PER_PUSH_F32 * pushed / max(1, tm["push_launches"]),
                     "avg_launch_ms": tm["push_ms"] / max(1, tm["push_launches"]),
                     "copy_GBps": copy_gbs,
                     "launches": tm["push_launches"], "run_key": key},
        "timed_with": "hip graphs" if args.graph else
        "eager launches; HIP events recorded by the push launches' dispatches (the other launches carry none)",
        "kernel_ms_per_step": {"push": tb["push_ms"] / align, "field": tb["field_ms"] / align,
                               "compact": tb["compact_ms"] / align, "emit": tb["emit_ms"] / align},
        "kernel_ms_per_step_from": f"the {align} steps before the timed window, events on every launch",
        "time_step_check": _finite({k: (v.tolist() if hasattr(v, "tolist") else v) for k, v in dtc.items()}),
    }
    sim.close()
    if not args.no_cpu_baseline:
        log(f"[bench] cpu baseline: oracle, {args.cpu_steps} steps")
        out["cpu_baseline"] = cpu_baseline(spec, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
