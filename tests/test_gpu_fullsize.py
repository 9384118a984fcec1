"""The benchmark's beam-gap workloads at full size, in the launch shape the
benchmark times, checked where the oracle can follow one particle at a time and
through properties that hold at any size:
  - 4096 cells, 2e7 H+ uniform in the gap, weak coupling;
  - 16384 cells, 2e8 H+ in a Gaussian at 0.9 d, strict coupling (the deposit
    then runs in 32-bit cells with carries: the grid's 64-bit row does not fit
    in LDS beside the field table).
Both with a beam of 2e4 ions per step and compaction every 32 steps.  After 40
steps (one compaction on the way), one more step is checked:
  - a sample of ions pushed by the GPU equals the oracle's binary32 push of the
    same ions through the same field table, bit for bit (App. C gather,
    eq. vel_update_main and eq. pos_update_main); an ion the oracle's push puts
    on a wall is gone;
  - a sample of the step's beam ions equals the oracle's draws for their indices;
  - the level's space charge equals the charge of the particles it was deposited
    from, exactly (fixed-point weights sum to whole macroparticles);
  - live count after = live before + injected + emitted - absorbed.
"""
import numpy as np
import pytest

import oracle
from paper_2603_24010_amd import workloads as W

pytestmark = pytest.mark.gpu

CASES = {
    "4096c_2e7p_weak": dict(n_cells=4096, n0=20_000_000, load="uniform", mode=1),
    "16384c_2e8p_strict": dict(n_cells=16384, n0=200_000_000, load="gauss", mode=0),
}


@pytest.mark.parametrize("name", list(CASES))
def test_full_size_sampled_push_and_invariants(name):
    from paper_2603_24010_amd import gapsim as gs
    spec = CASES[name]
    beam, warm, n0 = 20_000, 40, spec["n0"]
    cfg = W.config2(n_cells=spec["n_cells"], beam_per_step=beam)
    grow = (warm + 8) * beam
    if spec["load"] == "uniform":
        loads = W.load_config2(n=n0, seed=2, d=cfg.d)
        cap = ((1 << 22) + grow, n0 + grow + (1 << 20))
    else:
        loads = W.load_config3(n=n0, seed=3, d=cfg.d)
        cap = (int(0.55 * (n0 + grow)) + (1 << 22), n0 + grow + (1 << 20))
    sim = gs.GapSim(cfg, particle_fp=32, capacity=cap)
    sim.set_option(gs.OPT_COMPACT_EVERY, 32)
    for sp, (x, v) in loads.items():
        sim.inject(0, sp, x, v)
    del loads
    print(f"{name}: {n0} H+ injected, {warm} steps", flush=True)
    sim.step(spec["mode"], warm)
    da = sim.diag(0)
    xa, ua, ida = sim.particles(0, 1)
    n_el_a = int(da["n_live"][0])
    assert da["n_live"][1] == len(xa)

    sim.step(spec["mode"], 1)  # solves level `warm` from these particles, then pushes them
    db = sim.diag(0)
    assert db["step"] == warm
    _, E, _ = sim.fields(0)
    xb, ub, idb = sim.particles(0, 1)
    print(f"{name}: states read ({len(xa)} / {len(xb)} ions)", flush=True)

    # bookkeeping of the step; electrons past a full event queue of the previous
    # push are emitted by this step's field solve, before it deposits
    inj = int(db["inj_step"])
    absorbed = db["abs_step"]
    em_total = int((db["emit_cum"] - da["emit_cum"]).sum())
    deferred = em_total - int(db["emit_step"].sum())
    assert inj == beam and deferred >= 0
    assert db["n_live"][1] == len(xa) + inj - absorbed[1].sum() == len(xb)
    assert db["n_live"][0] == n_el_a + em_total - absorbed[0].sum()

    # the level's space charge: the particles it was deposited from
    s0 = cfg.weight * cfg.q_unit
    expect = cfg.area * s0 * (cfg.Z[1] * len(xa) + cfg.Z[0] * (n_el_a + deferred))
    assert abs(db["q_space"] - expect) <= 1e-12 * abs(expect)

    # the field table the push gathered from: surface field, E_{k+1/2}, ground field
    ehat = np.concatenate([[db["sigma"] / cfg.eps0], E, [db["e_ground"]]]).astype(np.float32)
    orc = oracle.OracleSim(cfg, fp32=True)
    alpha = orc.alpha32(1)
    ob = np.argsort(idb)
    ids_b = idb[ob]

    def find(i):
        # a numpy scalar of the array's type: a Python int would make searchsorted
        # convert the whole array on every call
        k = np.searchsorted(ids_b, np.uint32(i))
        return ob[k] if k < len(ids_b) and ids_b[k] == i else -1

    rng = np.random.default_rng(2024)
    walls = 0
    for j in rng.integers(0, len(xa), size=20_000):
        x1, u1, wall = oracle.push32(ehat, alpha, xa[j], ua[j])
        k = find(ida[j])
        if wall == 0:
            assert k >= 0, ida[j]
            assert xb[k] == x1 and ub[k] == u1, (ida[j], xa[j], ua[j], xb[k], ub[k], x1, u1)
        else:
            assert k < 0, ida[j]
            walls += 1
    print(f"{name}: 20000 sampled pushes equal, {walls} of them absorbed", flush=True)

    # the step's beam: ids follow the initial load and the earlier levels' beams
    id0 = n0 + warm * beam
    for q in rng.integers(0, beam, size=5000):
        k = find(id0 + int(q))
        assert k >= 0
        bx, bu = orc.beam_ion32(warm, int(q))
        assert xb[k] == bx and ub[k] == bu, q
    sim.close()
