"""Write tests/golden/longrun_oracle.json: the oracle's ensemble for the long-run
statistical comparison (calls only oracle/ and the seeded input generators).

Scenario: the coupled-LC gap (L1 1 uH, C1 1 uF at 3 kV, L2 10 mH, C2 50 pF, k 0.6)
with 512 cells, SEE amplitude 1.0 with exponential 3 eV electrons, 1e5 H+ loaded
uniformly with energies uniform in 1..50 keV, a beam of 20 H+ per step, weak
coupling, binary64 particles; 16 seeds (load seed and random-stream seed
100 + s); 20000 steps; the gap voltage and surface charge every 500 steps.

    python3 tests/golden/make_longrun_oracle.py [--seeds 16] [--steps 20000]
"""
import argparse
import json
import multiprocessing as mp
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

SAMPLE_EVERY = 500


def scenario(seed):
    from paper_2603_24010_amd import workloads as W
    cfg = W.config2(n_cells=512, beam_per_step=20, seed=100 + seed).replace(see_amp=1.0)
    loads = W.load_config2(n=100_000, seed=100 + seed, d=cfg.d)
    return cfg, loads


def run_one(args):
    seed, steps = args
    import oracle
    cfg, loads = scenario(seed)
    s = oracle.OracleSim(cfg, fp32=False)
    for sp, (x, v) in loads.items():
        s.inject(sp, x, v)
    series = []
    for k in range(steps // SAMPLE_EVERY):
        s.step(oracle.WEAK, SAMPLE_EVERY)
        d = s.diag()
        series.append([int(d["step"]), float(d["phi0"]), float(d["sigma"]), int(d["n_live"].sum())])
    return seed, series


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--seeds", type=int, default=16)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--procs", type=int, default=8)
    a = ap.parse_args()
    import oracle
    oracle.build(force=False)
    with mp.Pool(a.procs) as pool:
        res = dict(pool.map(run_one, [(s, a.steps) for s in range(a.seeds)]))
    out = {"scenario": __doc__.split("\n\n")[1], "sample_every": SAMPLE_EVERY, "steps": a.steps,
           "mode": "weak", "precision": "binary64",
           "series": {str(s): res[s] for s in range(a.seeds)}}
    with open(os.path.join(HERE, "longrun_oracle.json"), "w") as f:
        json.dump(out, f)
    print("wrote", os.path.join(HERE, "longrun_oracle.json"))


if __name__ == "__main__":
    main()
