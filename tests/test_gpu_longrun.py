"""Long runs compared statistically: beyond the parity horizon single trajectories
of the binary32 GPU path and the binary64 oracle part (particle noise amplifies
rounding differences), so their ensembles are compared instead.

The oracle ensemble (16 seeds, 20000 weak steps, tests/golden/longrun_oracle.json)
was written by tests/golden/make_longrun_oracle.py, which calls only the oracle.
The GPU runs the same 16 seeded gaps as one batched context.  Bars: at every
sampled step the ensemble means of the gap voltage differ by at most 4 combined
standard errors (40 samples: 4 sigma keeps the family-wise false-alarm rate near
0.3%), the same for the surface charge, and a two-sample Kolmogorov-Smirnov test
of the final voltages does not reject (p > 0.01).
"""
import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))


def test_long_run_ensemble_matches_oracle():
    from scipy import stats
    import make_longrun_oracle as M
    from paper_2603_24010_amd import gapsim
    with open(os.path.join(HERE, "golden", "longrun_oracle.json")) as f:
        gold = json.load(f)
    seeds = sorted(int(s) for s in gold["series"])
    every, steps = gold["sample_every"], gold["steps"]
    cfgs, loads = [], []
    for s in seeds:
        cfg, ld = M.scenario(s)
        cfgs.append(cfg)
        loads.append(ld)
    sim = gapsim.GapSim(cfgs, particle_fp=32, capacity=(2_000_000, 2_000_000))
    for g, ld in enumerate(loads):
        for sp, (x, v) in ld.items():
            sim.inject(g, sp, x, v)
    sim.set_option(gapsim.OPT_GRAPH, 1)
    gpu = {g: [] for g in range(len(seeds))}
    for _ in range(steps // every):
        sim.step_weak(every)
        for g in range(len(seeds)):
            d = sim.diag(g)
            gpu[g].append([d["step"], d["phi0"], d["sigma"]])
    sim.close()
    Vg = np.array([[r[1] for r in gpu[g]] for g in range(len(seeds))])
    Sg = np.array([[r[2] for r in gpu[g]] for g in range(len(seeds))])
    Vo = np.array([[r[1] for r in gold["series"][str(s)]] for s in seeds])
    So = np.array([[r[2] for r in gold["series"][str(s)]] for s in seeds])
    steps_g = [r[0] for r in gpu[0]]
    assert steps_g == [r[0] for r in gold["series"][str(seeds[0])]]
    n = len(seeds)
    for name, A, B in (("V", Vg, Vo), ("sigma", Sg, So)):
        se = np.sqrt(A.var(0, ddof=1) / n + B.var(0, ddof=1) / n)
        z = np.abs(A.mean(0) - B.mean(0)) / np.where(se > 0, se, np.inf)
        print(f"{name}: ensemble spread {B.std(0).mean() / np.abs(B.mean(0)).mean():.2e} (relative), "
              f"largest |mean difference| / SE = {z.max():.2f}")
        assert z.max() <= 4.0, (name, z.max())
    ks = stats.ks_2samp(Vg[:, -1], Vo[:, -1])
    print(f"final V: KS statistic {ks.statistic:.3f}, p = {ks.pvalue:.3f}")
    assert ks.pvalue > 0.01
