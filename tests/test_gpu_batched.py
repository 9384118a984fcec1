"""Batched gaps: the autotuner leaves the state untouched and its choice does not
change results; graph replay of a batched strict run equals eager stepping."""
import os

import numpy as np
import pytest

from paper_2603_24010_amd import workloads as W

pytestmark = pytest.mark.gpu


def _gs():
    from paper_2603_24010_amd import gapsim
    return gapsim


def _batched(G=8, np_lo=4000, np_hi=20000):
    gs = _gs()
    cfgs, loads = [], []
    for g in range(G):
        cfg, n_p, e_b = W.config4_gap(g, np_lo=np_lo, np_hi=np_hi)
        cfgs.append(cfg)
        loads.append(W.load_config4_gap(n_p, e_b, g))
    sim = gs.GapSim(cfgs, particle_fp=32, capacity=(100_000, 100_000))
    for g in range(G):
        for sp, (x, v) in loads[g].items():
            sim.inject(g, sp, x, v)
    return sim, cfgs


def _state(sim, G):
    out = []
    for g in range(G):
        d = sim.diag(g)
        _, E, rho = sim.fields(g)
        xi, u, ids = sim.particles(g, 1)
        o = np.lexsort((u, xi, ids))
        out.append((d["step"], d["phi0"], d["sigma"], tuple(d["abs_cum"].ravel()), E.copy(), rho.copy(),
                    xi[o].copy(), u[o].copy()))
    return out


def _same(a, b):
    for sa, sb in zip(a, b):
        assert sa[0] == sb[0] and sa[1] == sb[1] and sa[2] == sb[2] and sa[3] == sb[3]
        for k in range(4, 8):
            np.testing.assert_array_equal(sa[k], sb[k])


def test_autotune_keeps_state_and_results(tmp_path):
    gs = _gs()
    G = 8
    a, _ = _batched(G)
    b, _ = _batched(G)
    a.step_strict(10)
    b.step_strict(10)
    before = _state(a, G)
    cache = os.path.join(tmp_path, "tune.txt")
    choice = a.autotune(0, gs.GUESS_DIRECT, trial_steps=3, cache_path=cache)
    print("autotune choice", choice)
    assert choice["ms_per_step"] > 0 and choice["block"] in (256, 512) and choice["ppt"] in (1, 2)
    _same(_state(a, G), before)
    # the cached choice comes back without trials
    again = a.autotune(0, gs.GUESS_DIRECT, trial_steps=3, cache_path=cache)
    assert {k: again[k] for k in ("block", "tile", "grid", "ppt", "compact_every")} == \
        {k: choice[k] for k in ("block", "tile", "grid", "ppt", "compact_every")}
    _same(_state(a, G), before)
    # results after the tuned launch shape are those of the default one
    a.step_strict(20)
    b.step_strict(20)
    _same(_state(a, G), _state(b, G))
    a.close()
    b.close()


def test_batched_graph_replay_equals_eager():
    gs = _gs()
    G = 8
    a, _ = _batched(G)
    b, _ = _batched(G)
    for s in (a, b):
        s.set_option(gs.OPT_COMPACT_EVERY, 6)
    a.set_option(gs.OPT_GRAPH, 1)
    a.step_strict(25)
    b.step_strict(25)
    _same(_state(a, G), _state(b, G))
    a.close()
    b.close()
