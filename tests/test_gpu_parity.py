"""GPU path (through the C ABI) against the CPU oracle on identical seeded inputs.

Bars: absorbed / emitted / injected counts bit-exact; binary64 particles: fields,
surface charge, gap voltage and loop currents within 1e-12 (norm-wise relative);
binary32 particles against the oracle's binary32 mode: the same quantities within
1e-5, particle states equal (compared as sorted multisets, their order in memory
being unspecified), and the error against the binary64 oracle stated.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2603_24010_amd import workloads as W

pytestmark = pytest.mark.gpu


def _gapsim():
    from paper_2603_24010_amd import gapsim
    return gapsim


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    s = np.abs(b).max()
    return float(np.abs(a - b).max() / s) if s > 0 else float(np.abs(a - b).max())


def _series_rel(xs, ys):
    xs, ys = np.array(xs), np.array(ys)
    scale = np.abs(ys).max()
    return float(np.abs(xs - ys).max() / scale) if scale > 0 else float(np.abs(xs - ys).max())


def run_pair(cfg, loads, mode, nsteps, fp32, capacity, opts=None, check_every=1):
    """Advance the oracle and the GPU side by side; return per-step records."""
    gs = _gapsim()
    sim = gs.GapSim(cfg, particle_fp=32 if fp32 else 64, capacity=capacity)
    for k, v in (opts or {}).items():
        sim.set_option(k, v)
    orc = oracle.OracleSim(cfg, fp32=fp32)
    for sp in sorted(loads):
        x, v = loads[sp]
        sim.inject(0, sp, x, v)
        orc.inject(sp, x, v)
    recs = []
    for n in range(nsteps):
        sim.step(mode, 1)
        orc.step(mode, 1)
        if (n + 1) % check_every == 0 or n == nsteps - 1:
            recs.append((sim.diag(0), orc.diag()))
    return sim, orc, recs


def assert_counts_equal(dg, do):
    np.testing.assert_array_equal(dg["abs_cum"], do["abs_cum"])
    np.testing.assert_array_equal(dg["emit_cum"], do["emit_cum"])
    assert dg["inj_cum"] == do["inj_cum"]
    np.testing.assert_array_equal(dg["n_live"], do["n_live"])
    assert dg["pushed_cum"] == do["pushed_cum"]


EPS64 = 2.0 ** -52


def loop_rounding_floor(cfg, recs, mode):
    """Per level and loop, a bound on how far two correct binary64 evaluations of
    the loop increments D^n = q^n - q^{n-1} can differ.

    The library forms D_j as a sum of products, T^-1 times the BDF2 right-hand
    side (L h / (4 dt^2) + R D^{n-1} / (2 dt) - S q^{n-1} + b V_s, with
    h = 15 D^{n-1} - 7 D^{n-2} + D^{n-3}), minus z_j phi0 in strict mode, where
    T = 9 L / (4 dt^2) + 3 R / (2 dt) + S (in weak mode with the gap capacitor on
    the gap loop's diagonal) and z = T^-1 e_gap.  Its rounding is at most a few
    ulps of the sum of the terms' magnitudes, (3M + 4) eps times
    |T^-1| (|L| |h| / (4 dt^2) + |R| |D^{n-1}| / (2 dt) + |S| |q^{n-1}|) + |T^-1 b| |V_s|
    + |z| |phi0|, and in strict mode the two sides' electrode potentials differ by
    the measured |dphi0|, which moves D by |z| |dphi0|.  A loop whose increment is
    a near-cancellation of much larger terms (a loop closed by a large resistor)
    can only be held to this floor; for the others it is far below tol.
    Returns (floor of I, floor of q) as arrays [level, loop]."""
    M, g, dt = cfg.n_mesh, cfg.gap_mesh, cfg.dt
    L, R, S = (np.abs(np.asarray(a, dtype=np.float64)).reshape(M, M) for a in (cfg.L, cfg.R, cfg.S))
    T = 9 * np.asarray(cfg.L, dtype=np.float64).reshape(M, M) / (4 * dt * dt) \
        + 3 * np.asarray(cfg.R, dtype=np.float64).reshape(M, M) / (2 * dt) + np.asarray(cfg.S, dtype=np.float64).reshape(M, M)
    if mode == oracle.WEAK:
        cg = cfg.eps0 * cfg.area / cfg.d + cfg.c_par
        T[g, g] += 1.0 / cg
        S = S.copy()
        S[g, g] += 1.0 / cg
    Ti = np.linalg.inv(T)
    Tia = np.abs(Ti)
    bz = np.abs(Ti @ np.asarray(cfg.src, dtype=np.float64).reshape(M))
    z = np.abs(Ti[:, g])
    q_prev = np.asarray(cfg.q0, dtype=np.float64).reshape(M).copy()
    Dh = [np.zeros(M), np.zeros(M), np.zeros(M)]  # D^{n-1}, D^{n-2}, D^{n-3}
    c = (3 * M + 4) * EPS64
    fD_prev = np.zeros(M)
    fq = np.zeros(M)
    fI_all, fq_all = [], []
    for dg, do in recs:
        t = do["t"]
        Vs = cfg.src_dc + cfg.src_amp * math.sin(2 * math.pi * cfg.src_freq * t + cfg.src_phase)
        h = 15 * Dh[0] - 7 * Dh[1] + Dh[2]
        mag = Tia @ (L @ np.abs(h) / (4 * dt * dt) + R @ np.abs(Dh[0]) / (2 * dt) + S @ np.abs(q_prev)) \
            + bz * abs(Vs) + z * abs(do["phi0"])
        fD = c * mag
        if mode == oracle.STRICT:
            fD = fD + z * abs(dg["phi0"] - do["phi0"])
        q = np.array([do["q"][j] for j in range(M)])
        I = np.array([do["I"][j] for j in range(M)])
        fI_all.append((3 * fD + fD_prev) / (2 * dt) + 4 * EPS64 * np.abs(I))
        fq = fq + fD + 2 * EPS64 * np.abs(q)
        fq_all.append(fq.copy())
        fD_prev = fD
        Dh = [q - q_prev, Dh[0], Dh[1]]
        q_prev = q
    return np.array(fI_all), np.array(fq_all)


def check_run(recs, tol, M, cfg=None, mode=None):
    for dg, do in recs:
        assert dg["step"] == do["step"]
        assert_counts_equal(dg, do)
    for key in ("phi0", "sigma", "qcirc", "qcirc_star", "q_space"):
        r = _series_rel([d[key] for d, _ in recs], [o[key] for _, o in recs])
        assert r <= tol, (key, r)
    # loop currents and charges, each loop against its own scale; a loop may
    # fall back on its derived binary64 rounding floor (consecutive levels only)
    floors = loop_rounding_floor(cfg, recs, mode) if cfg is not None else (None, None)
    for key, fl in (("I", floors[0]), ("q", floors[1])):
        g = np.array([[d[key][j] for j in range(M)] for d, _ in recs])
        o = np.array([[od[key][j] for j in range(M)] for _, od in recs])
        for j in range(M):
            err = np.abs(g[:, j] - o[:, j])
            scale = np.abs(o[:, j]).max()
            if err.max() <= tol * scale:
                continue
            assert fl is not None, (key, j, float(err.max()), float(scale))
            assert np.all(err <= tol * scale + fl[:, j]), \
                (key, j, float(err.max()), float(scale), float((err / (tol * scale + fl[:, j])).max()))
            print(f"loop {j} {key}: error {err.max():.3e} of scale {scale:.3e}, within the rounding floor "
                  f"(max floor {fl[:, j].max():.3e})")


def check_fields(sim, orc, tol):
    pg, Eg, rg = sim.fields(0)
    po, Eo, ro = orc.fields()
    assert rel(rg, ro) <= tol, ("rho", rel(rg, ro))
    assert rel(Eg, Eo) <= tol, ("E", rel(Eg, Eo))
    assert rel(pg, po) <= tol, ("phi", rel(pg, po))


def sorted_state(xi, u):
    order = np.lexsort((u, xi))
    return xi[order], u[order]


# ---------------------------------------------------------------------------
# binary64 particles (the FP64 configuration: 256 cells, 1e5 particles)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mode", [oracle.STRICT, oracle.WEAK])
def test_config1_fp64_parity(mode):
    cfg = W.config1()
    loads = W.load_config1(n_per_species=50000, seed=0)
    # hotter load so that walls and emission are exercised within 50 steps
    loads = {s: (x, v * 30.0) for s, (x, v) in loads.items()}
    sim, orc, recs = run_pair(cfg, loads, mode, 50, False, (150000, 150000))
    check_run(recs, 1e-12, cfg.n_mesh, cfg, mode)
    check_fields(sim, orc, 1e-12)
    d = recs[-1][0]
    assert d["abs_cum"].sum() > 100 and d["emit_cum"].sum() > 0
    # particle states, sorted by id (ions and loaded electrons) in grid units
    dx, dt = cfg.d / cfg.n_cells, cfg.dt
    for sp in (0, 1):
        xg, ug, idg = sim.particles(0, sp)
        xo, vo, ido = orc.particles(sp)
        assert len(xg) == len(xo)
        og, oo = np.lexsort((xg, idg)), np.lexsort((xo / dx, ido))
        np.testing.assert_array_equal(idg[og], ido[oo])
        np.testing.assert_allclose(xg[og], (xo / dx)[oo], rtol=0, atol=1e-12 * cfg.n_cells)
        np.testing.assert_allclose(ug[og], (vo * dt / dx)[oo], rtol=1e-11,
                                   atol=1e-12 * np.abs(vo * dt / dx).max())


def test_paper_worked_value_on_gpu():
    """App. F: strict Q_circ = -1.606712e-17 C when an ion appears at x = 0.016 m."""
    gs = _gapsim()
    cfg = W.config_paper_validation()
    for mode, want in ((oracle.STRICT, -1.606712e-17), (oracle.WEAK, 0.0)):
        sim = gs.GapSim(cfg, particle_fp=64, capacity=(16, 16))
        sim.step(mode, 1000)
        sim.inject(0, 1, np.array([0.016]), np.array([0.0]))
        sim.step(mode, 1)
        d = sim.diag(0)
        assert d["step"] == 1000
        if mode == oracle.STRICT:
            assert abs(d["qcirc"] - want) <= 0.5e-6 * abs(want)
        else:
            assert d["qcirc_star"] == 0.0
        sim.close()


@pytest.mark.parametrize("make", [lambda: W.config1(n_cells=64),
                                  lambda: W.config2(n_cells=64, beam_per_step=0),
                                  lambda: W.config_tesla(n_cells=64).replace(
                                      beam_schedule=np.zeros(0, dtype=np.int64))])
@pytest.mark.parametrize("mode", [oracle.STRICT, oracle.WEAK])
def test_vacuum_circuit_parity(make, mode):
    cfg = make()
    sim, orc, recs = run_pair(cfg, {}, mode, 300, False, (16, 16))
    check_run(recs, 1e-12, cfg.n_mesh, cfg, mode)


# ---------------------------------------------------------------------------
# binary32 particles against the oracle's binary32 mode
# ---------------------------------------------------------------------------
def cfg2_small(n_cells=4096, beam=2000):
    return W.config2(n_cells=n_cells, beam_per_step=beam)


@pytest.mark.parametrize("sort_bin", [0, 64])
@pytest.mark.parametrize("mode", [oracle.WEAK, oracle.STRICT])
@pytest.mark.parametrize("n_cells", [4096, 16384])
def test_fp32_beam_gap_parity(mode, n_cells, sort_bin):
    """With and without the periodic cell sort (bins of 64 cells): the sort only
    reorders particles, so the bars are the same."""
    cfg = cfg2_small(n_cells=n_cells)
    loads = W.load_config2(n=200_000, seed=11)
    gs = _gapsim()
    opts = {gs.OPT_COMPACT_EVERY: 7, gs.OPT_SORT_BIN: sort_bin}
    sim, orc, recs = run_pair(cfg, loads, mode, 50, True, (400_000, 600_000), opts=opts)
    check_run(recs, 1e-5, cfg.n_mesh, cfg, mode)
    check_fields(sim, orc, 1e-5)
    d = recs[-1][0]
    assert d["abs_cum"][1].sum() > 100 and d["emit_cum"].sum() > 10 and d["inj_cum"] == 100_000
    for sp in (0, 1):
        xg, ug, _ = sim.particles(0, sp)
        xo, uo, _ = orc.particles_f32(sp)
        assert len(xg) == len(xo)
        a, b = sorted_state(xg, ug), sorted_state(xo, uo)
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_array_equal(a[1], b[1])


@pytest.mark.parametrize("sort_bin", [0, 16])
@pytest.mark.parametrize("mode", [oracle.STRICT, oracle.WEAK])
@pytest.mark.parametrize("layer", [2e-3, 0.0])
def test_fp32_tesla_ground_pulse_parity(mode, layer, sort_bin):
    """The paper's integrated-run shape (Sec. 4.2): five-loop Tesla circuit, ions
    entering next to the grounded electrode by a Gaussian schedule (here early and
    short, so that 80 steps see it rise and fall), emission on."""
    # started within one step's flight of the electrode the ions of a step are
    # absorbed together, in the workgroup holding them: a smaller pulse keeps
    # them within the 1152 events a workgroup emits in the same step
    sched = W.gaussian_schedule(80, 3000.0 if layer > 0 else 500.0, 35.0, 10.0)
    cfg = W.config_tesla(layer=layer).replace(beam_schedule=sched, see_amp=30.0)
    gs = _gapsim()
    opts = {gs.OPT_COMPACT_EVERY: 9, gs.OPT_SORT_BIN: sort_bin}
    sim, orc, recs = run_pair(cfg, {}, mode, 80, True, (200_000, 200_000), opts=opts)
    check_run(recs, 1e-5, cfg.n_mesh, cfg, mode)
    check_fields(sim, orc, 1e-5)
    d = recs[-1][0]
    assert d["inj_cum"] == int(sched.sum())
    assert d["abs_cum"][1].sum() > 1000 and d["emit_cum"].sum() > 100, (d["abs_cum"], d["emit_cum"])
    for sp in (0, 1):
        xg, ug, _ = sim.particles(0, sp)
        xo, uo, _ = orc.particles_f32(sp)
        assert len(xg) == len(xo)
        a, b = sorted_state(xg, ug), sorted_state(xo, uo)
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_array_equal(a[1], b[1])
    sim.close()


@pytest.mark.parametrize("mode", [oracle.WEAK, oracle.STRICT])
def test_fp32_paper_see_laws_parity(mode):
    """The paper's SEE laws (Sec. 2.3, Alg. 2): the fifth-order yield clipped at
    zero and lognormal electron energies, on the beam gap."""
    cfg = cfg2_small().replace(see_amp=1.0, see_yield=W.YIELD_POLY,
                               see_poly=np.array([0.05, 0.12, -2.0e-3, 2.0e-5, -1.0e-7, 2.0e-10]),
                               see_poly_Emax_eV=8e4, see_law=W.SEE_LOGNORMAL,
                               see_ln_mu=math.log(8.0), see_ln_sigma=0.7)
    loads = W.load_config2(n=200_000, seed=12)
    opts = {_gapsim().OPT_COMPACT_EVERY: 7}
    sim, orc, recs = run_pair(cfg, loads, mode, 50, True, (400_000, 600_000), opts=opts)
    check_run(recs, 1e-5, cfg.n_mesh, cfg, mode)
    check_fields(sim, orc, 1e-5)
    d = recs[-1][0]
    assert d["abs_cum"][1].sum() > 100 and d["emit_cum"].sum() > 100, (d["abs_cum"], d["emit_cum"])
    for sp in (0, 1):
        xg, ug, _ = sim.particles(0, sp)
        xo, uo, _ = orc.particles_f32(sp)
        assert len(xg) == len(xo)
        a, b = sorted_state(xg, ug), sorted_state(xo, uo)
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_array_equal(a[1], b[1])
    sim.close()


@pytest.mark.parametrize("mode", [oracle.WEAK, oracle.STRICT])
@pytest.mark.parametrize("n_cells", [4096, 16384])
def test_fp32_error_against_fp64_oracle(mode, n_cells):
    """What binary32 particles cost against the binary64 oracle over the 50-step
    horizon: phi and E at the end, and V, sigma, Q_circ and every loop's current
    and charge at every level, within 1e-5 relative (each against its own scale);
    absorbed counts equal.  The nodal density is the deposit of positions held in
    binary32 (a position one ulp away moves weight between two nodes), so it is
    stated, not held to the bar: the bar is on what the field and the circuit see.
    2e6 ions: the field's rounding noise is an average over them.  Absorbed
    counts may differ by an ion grazing a wall (a few at most)."""
    cfg = cfg2_small(n_cells=n_cells, beam=2000)
    loads = W.load_config2(n=2_000_000, seed=12)
    gs = _gapsim()
    sim = gs.GapSim(cfg, particle_fp=32, capacity=(600_000, 2_400_000))
    sim.set_option(gs.OPT_COMPACT_EVERY, 16)
    orc = oracle.OracleSim(cfg, fp32=False)
    for sp, (x, v) in loads.items():
        sim.inject(0, sp, x, v)
        orc.inject(sp, x, v)
    recs = []
    for _ in range(50):
        sim.step(mode, 1)
        orc.step(mode, 1)
        recs.append((sim.diag(0), orc.diag()))
    pg, Eg, rg = sim.fields(0)
    po, Eo, ro = orc.fields()
    errs = {"phi": rel(pg, po), "E": rel(Eg, Eo)}
    for key in ("phi0", "sigma", "qcirc", "qcirc_star"):
        errs[key] = _series_rel([d[key] for d, _ in recs], [o[key] for _, o in recs])
    for key in ("I", "q"):
        for j in range(cfg.n_mesh):
            errs[f"{key}{j}"] = _series_rel([d[key][j] for d, _ in recs], [o[key][j] for _, o in recs])
    print(f"binary32 vs binary64, {n_cells} cells, {'weak' if mode else 'strict'}, 50 steps: "
          + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()) + f"; nodal rho {rel(rg, ro):.2e}")
    for k, v in errs.items():
        assert v <= 1e-5, (k, v)
    # absorbed counts: an ion that grazes a wall can be absorbed one step apart
    # in the two precisions (counts are bit-exact against the oracle's binary32
    # mode, the other parity tests); here they may differ by a few
    dmax = max(int(np.abs(dg["abs_cum"] - do["abs_cum"]).max()) for dg, do in recs)
    print(f"largest absorbed-count difference at one level: {dmax}")
    assert dmax <= 3
    assert recs[-1][0]["abs_cum"][1].sum() > 1000
    sim.close()


# ---------------------------------------------------------------------------
# several gaps in one context
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("sort_bin,steal,stream", [(0, 0, 0), (8, 0, 0), (0, 2, 0), (0, 0, 3)])
def test_batched_gaps_parity(sort_bin, steal, stream):
    """Six gaps in one context against six oracles.  With steal on and five
    push workgroups, half of every workgroup's tiles go to the pool, so pool
    tiles switch between gaps and species; with the round-robin stream and
    five workgroups, consecutive tiles of a workgroup do too."""
    gs = _gapsim()
    G = 6
    cfgs, loads = [], []
    for g in range(G):
        cfg, n_p, e_b = W.config4_gap(g, np_lo=5000, np_hi=30000)
        cfgs.append(cfg)
        loads.append(W.load_config4_gap(n_p, e_b, g))
    sim = gs.GapSim(cfgs, particle_fp=32, capacity=(200_000, 200_000))
    sim.set_option(gs.OPT_COMPACT_EVERY, 5)
    sim.set_option(gs.OPT_SORT_BIN, sort_bin)
    sim.set_option(gs.OPT_STEAL, steal)
    sim.set_option(gs.OPT_STREAM, stream)
    if steal or stream:
        sim.set_option(gs.OPT_GRID, 5)
    orcs = []
    for g in range(G):
        o = oracle.OracleSim(cfgs[g], fp32=True)
        for sp, (x, v) in loads[g].items():
            o.inject(sp, x, v)
            sim.inject(g, sp, x, v)
        orcs.append(o)
    recs = [[] for _ in range(G)]
    for n in range(30):
        sim.step_strict(1)
        for g in range(G):
            orcs[g].step(oracle.STRICT, 1)
            recs[g].append((sim.diag(g), orcs[g].diag()))
    for g in range(G):
        check_run(recs[g], 1e-5, cfgs[g].n_mesh, cfgs[g], oracle.STRICT)


@pytest.mark.parametrize("mode", [oracle.STRICT, oracle.WEAK])
def test_mixed_grid_sizes_parity(mode):
    """A 16384-cell gap and a 700-cell gap in one context: past 8192 cells the
    field solve runs as three kernels over chunks of 1024 nodes, and the small
    gap's chunks past its own last node have nothing to do.  Both gaps against
    their oracles, with the binary32 particles bit-equal.  (Weak mode runs
    with the round-robin, non-temporal particle stream.)"""
    gs = _gapsim()
    cfgs = [cfg2_small(n_cells=16384, beam=1500), cfg2_small(n_cells=700, beam=800)]
    loads = [W.load_config2(n=60_000, seed=31), W.load_config2(n=20_000, seed=32)]
    sim = gs.GapSim(cfgs, particle_fp=32, capacity=(200_000, 200_000))
    sim.set_option(gs.OPT_COMPACT_EVERY, 4)
    sim.set_option(gs.OPT_STREAM, 3 if mode == oracle.WEAK else 0)
    orcs = []
    for g in range(2):
        o = oracle.OracleSim(cfgs[g], fp32=True)
        for sp in sorted(loads[g]):
            x, v = loads[g][sp]
            sim.inject(g, sp, x, v)
            o.inject(sp, x, v)
        orcs.append(o)
    recs = [[], []]
    for n in range(20):
        sim.step(mode, 1)
        for g in range(2):
            orcs[g].step(mode, 1)
            recs[g].append((sim.diag(g), orcs[g].diag()))
    for g in range(2):
        check_run(recs[g], 1e-5, cfgs[g].n_mesh, cfgs[g], mode)
        for dg, do in recs[g]:
            assert_counts_equal(dg, do)
        pg, Eg, rg = sim.fields(g)
        po, Eo, ro = orcs[g].fields()
        for name, a, b in (("rho", rg, ro), ("E", Eg, Eo), ("phi", pg, po)):
            assert rel(a, b) <= 1e-5, (g, name, rel(a, b))
        for sp in (0, 1):
            xg, ug, _ = sim.particles(g, sp)
            xo, uo, _ = orcs[g].particles_f32(sp)
            assert len(xg) == len(xo)
            a, b = sorted_state(xg, ug), sorted_state(xo, uo)
            np.testing.assert_array_equal(a[0], b[0])
            np.testing.assert_array_equal(a[1], b[1])
    assert recs[0][-1][0]["abs_cum"][1].sum() > 0
    sim.close()


# ---------------------------------------------------------------------------
# launch configurations, graphs, determinism, edge cases
# ---------------------------------------------------------------------------
def _cfg2_state(opts, nsteps=24, mode=oracle.WEAK, seed=21):
    gs = _gapsim()
    cfg = cfg2_small(n_cells=1024, beam=1500)
    loads = W.load_config2(n=100_000, seed=seed)
    sim = gs.GapSim(cfg, particle_fp=32, capacity=(300_000, 300_000))
    for k, v in opts.items():
        sim.set_option(k, v)
    for sp, (x, v) in loads.items():
        sim.inject(0, sp, x, v)
    sim.step(mode, nsteps)
    d = sim.diag(0)
    phi, E, rho = sim.fields(0)
    xi, u, _ = sim.particles(0, 1)
    xe, ue, _ = sim.particles(0, 0)
    sim.close()
    return d, E, sorted_state(xi, u), sorted_state(xe, ue)


def test_launch_shapes_and_graph_agree():
    gs = _gapsim()
    base = _cfg2_state({gs.OPT_COMPACT_EVERY: 8})
    variants = [
        {gs.OPT_COMPACT_EVERY: 8, gs.OPT_GRAPH: 1},
        {gs.OPT_COMPACT_EVERY: 1},
        {gs.OPT_COMPACT_EVERY: 5, gs.OPT_BLOCK: 512, gs.OPT_TILE: 512 * 8, gs.OPT_DEPOSIT: 2},
        {gs.OPT_COMPACT_EVERY: 6, gs.OPT_PPT: 2, gs.OPT_TILE: 512 * 24},
        {gs.OPT_COMPACT_EVERY: 7, gs.OPT_PPT: 2, gs.OPT_DEPOSIT: 2, gs.OPT_BLOCK: 256},
        {gs.OPT_COMPACT_EVERY: 3, gs.OPT_BLOCK: 1024, gs.OPT_TILE: 1024 * 16, gs.OPT_GRID: 7,
         gs.OPT_DEPOSIT: 1},
        {gs.OPT_COMPACT_EVERY: 2, gs.OPT_BLOCK: 256, gs.OPT_TILE: 256 * 24, gs.OPT_DEPOSIT: 2,
         gs.OPT_COMPACT_GRID: 3},
        {gs.OPT_COMPACT_EVERY: 4, gs.OPT_GRAPH: 1, gs.OPT_DEPOSIT: 2, gs.OPT_GRID: 33},
        {gs.OPT_COMPACT_EVERY: 8, gs.OPT_SORT_BIN: 16},
        {gs.OPT_COMPACT_EVERY: 3, gs.OPT_SORT_BIN: 4, gs.OPT_BLOCK: 512, gs.OPT_COMPACT_GRID: 5},
        {gs.OPT_COMPACT_EVERY: 5, gs.OPT_SORT_BIN: 1024, gs.OPT_GRAPH: 1, gs.OPT_DEPOSIT: 2},
        {gs.OPT_COMPACT_EVERY: 1, gs.OPT_SORT_BIN: 64, gs.OPT_PPT: 2, gs.OPT_GRID: 13},
        # the tile pool: with a handful of workgroups, a half or a quarter of every
        # run goes to the pool (electron and ion tiles, segment switches)
        {gs.OPT_COMPACT_EVERY: 4, gs.OPT_GRID: 3, gs.OPT_STEAL: 2},
        {gs.OPT_COMPACT_EVERY: 6, gs.OPT_GRID: 5, gs.OPT_STEAL: 4, gs.OPT_DEPOSIT: 2, gs.OPT_SORT_BIN: 16},
        {gs.OPT_COMPACT_EVERY: 8, gs.OPT_GRID: 2, gs.OPT_STEAL: 2, gs.OPT_GRAPH: 1},
        {gs.OPT_COMPACT_EVERY: 8, gs.OPT_STEAL: 0},
        # the particle stream: round-robin tile order with a handful of
        # workgroups (each takes tiles of both species), non-temporal accesses
        {gs.OPT_COMPACT_EVERY: 4, gs.OPT_GRID: 3, gs.OPT_STREAM: 1},
        {gs.OPT_COMPACT_EVERY: 5, gs.OPT_BLOCK: 512, gs.OPT_TILE: 512 * 8, gs.OPT_GRID: 7, gs.OPT_STREAM: 3},
        {gs.OPT_COMPACT_EVERY: 6, gs.OPT_PPT: 2, gs.OPT_TILE: 512 * 24, gs.OPT_STREAM: 2},
        {gs.OPT_COMPACT_EVERY: 3, gs.OPT_GRID: 5, gs.OPT_STREAM: 1, gs.OPT_STEAL: 4, gs.OPT_SORT_BIN: 16},
        {gs.OPT_COMPACT_EVERY: 8, gs.OPT_STREAM: 3, gs.OPT_GRAPH: 1, gs.OPT_DEPOSIT: 2},
    ]
    for opts in variants:
        d, E, ions, els = _cfg2_state(opts)
        assert_counts_equal(d, base[0])
        np.testing.assert_array_equal(E, base[1])
        for a, b in ((ions, base[2]), (els, base[3])):
            np.testing.assert_array_equal(a[0], b[0])
            np.testing.assert_array_equal(a[1], b[1])


def test_run_to_run_bitwise_identical():
    gs = _gapsim()
    a = _cfg2_state({gs.OPT_COMPACT_EVERY: 4}, seed=5)
    b = _cfg2_state({gs.OPT_COMPACT_EVERY: 4}, seed=5)
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_array_equal(a[2][0], b[2][0])


@pytest.mark.parametrize("fp32", [True, False])
@pytest.mark.parametrize("sort_bin", [4, 16, 100])
def test_cell_sort_orders_by_bin(sort_bin, fp32):
    """Right after a sort every region holds its live particles in increasing
    bin (cells // sort_bin, the last bin taking the electrode node), none lost:
    the ids of the live set are those before the sort."""
    gs = _gapsim()
    cfg = cfg2_small(n_cells=1000, beam=700)
    loads = W.load_config2(n=60_000, seed=4)
    sim = gs.GapSim(cfg, particle_fp=32 if fp32 else 64, capacity=(100_000, 100_000))
    sim.set_option(gs.OPT_COMPACT_EVERY, 6)
    sim.set_option(gs.OPT_SORT_BIN, sort_bin)
    for sp, (x, v) in loads.items():
        sim.inject(0, sp, x, v)
    sim.step_weak(6)  # the sixth step ends with the sort
    nb = -(-cfg.n_cells // sort_bin)
    for sp in (0, 1):
        x, u, ids = sim.particles(0, sp)
        assert len(x) == sim.diag(0)["n_live"][sp]
        b = np.minimum(np.floor(x).astype(np.int64) // sort_bin, nb - 1)
        assert np.all(np.diff(b) >= 0), sp
        if sp == 1:
            assert len(np.unique(ids)) == len(ids) > 50_000
    sim.close()


@pytest.mark.parametrize("fp32", [True, False])
def test_compaction_leaves_no_holes(fp32):
    """Right after a compaction every region's slots are exactly its live
    particles (the in-place fill moved the live particles past the live count
    into the absorbed slots below it), with no particle lost or duplicated."""
    gs = _gapsim()
    cfg = W.config1(n_cells=64).replace(see_amp=3.0, beam_per_step=50, beam_Emin_eV=1e3, beam_Emax_eV=5e3)
    loads = W.load_config1(n_per_species=20_000, seed=6)
    sim = gs.GapSim(cfg, particle_fp=32 if fp32 else 64, capacity=(80_000, 80_000))
    sim.set_option(gs.OPT_COMPACT_EVERY, 7)
    sim.set_option(gs.OPT_TILE, 2048)
    for sp, (x, v) in loads.items():
        sim.inject(0, sp, x, v * 30.0)
    sim.step_strict(6)
    d = sim.diag(0)
    assert np.all(d["n_slots"] > d["n_live"])  # absorbed slots are waiting
    ions_before = np.sort(sim.particles(0, 1)[2])
    sim.step_strict(1)  # ends with the compaction
    d = sim.diag(0)
    np.testing.assert_array_equal(d["n_slots"], d["n_live"])
    ions = np.sort(sim.particles(0, 1)[2])
    assert len(np.unique(ions)) == len(ions) == d["n_live"][1]
    # the step's survivors are among the ions before it, plus its beam
    assert np.isin(ions, ions_before).sum() == len(ions) - d["inj_step"]
    sim.close()


def test_emission_kernel_emits_within_the_step():
    """With the cell sort on, the ions a push absorbs past its LDS queue (a
    wall's impacts concentrated in the workgroups holding its bins) are emitted
    by the emission kernel in the same step: the emitted counts equal the
    oracle's at every level, as do voltages and fields."""
    gs = _gapsim()
    sched = W.gaussian_schedule(60, 3000.0, 30.0, 8.0)
    cfg = W.config_tesla(layer=0.0).replace(beam_schedule=sched, see_amp=30.0)
    sim, orc, recs = run_pair(cfg, {}, oracle.STRICT, 60, True, (200_000, 200_000),
                              opts={gs.OPT_SORT_BIN: 8, gs.OPT_COMPACT_EVERY: 4})
    check_run(recs, 1e-5, cfg.n_mesh, cfg, oracle.STRICT)
    check_fields(sim, orc, 1e-5)
    assert recs[-1][0]["emit_cum"].sum() > 1000
    sim.close()


def test_empty_and_edge_particles():
    """No particles; particles exactly on either electrode; a tail shorter than a tile."""
    gs = _gapsim()
    cfg = W.config1(n_cells=32).replace(see_amp=3.0)
    for fp32 in (False, True):
        sim = gs.GapSim(cfg, particle_fp=32 if fp32 else 64, capacity=(64, 64))
        orc = oracle.OracleSim(cfg, fp32=fp32)
        sim.step_strict(3)
        orc.step(oracle.STRICT, 3)
        x = np.array([0.0, cfg.d, 0.5 * cfg.d, cfg.d / cfg.n_cells, 1e-12])
        v = np.array([-1e5, 1e5, 3e5, -2e6, 4e4])
        for sp in (0, 1):
            sim.inject(0, sp, x, v)
            orc.inject(sp, x, v)
        for _ in range(6):
            sim.step_strict(1)
            orc.step(oracle.STRICT, 1)
            assert_counts_equal(sim.diag(0), orc.diag())
        sim.close()


def test_capacity_overflow_is_reported():
    gs = _gapsim()
    cfg = cfg2_small(n_cells=256, beam=300)
    sim = gs.GapSim(cfg, particle_fp=32, capacity=(100, 500))
    with pytest.raises(gs.GapsimError) as e:
        sim.step_weak(3)
        sim.diag(0)
    assert e.value.status == gs.GS_ECAPACITY


def test_inject_rejects_outside_positions():
    gs = _gapsim()
    cfg = W.config1(n_cells=32)
    sim = gs.GapSim(cfg, particle_fp=64, capacity=(16, 16))
    with pytest.raises(gs.GapsimError) as e:
        sim.inject(0, 0, np.array([2 * cfg.d]), np.array([0.0]))
    assert e.value.status == gs.GS_EINVAL


def test_launch_options_reject_out_of_range_values():
    """gs_set_option refuses values outside each option's range (EINVAL) and
    leaves the launch in effect as it was."""
    gs = _gapsim()
    cfg = W.config1(n_cells=32)
    sim = gs.GapSim(cfg, particle_fp=32, capacity=(16, 16))
    before = sim.launch()
    for opt, bad in ((gs.OPT_STREAM, 4), (gs.OPT_STREAM, -1), (gs.OPT_STEAL, 1), (gs.OPT_STEAL, 65),
                     (gs.OPT_PPT, 3), (gs.OPT_TIMING, 3)):
        with pytest.raises(gs.GapsimError) as e:
            sim.set_option(opt, bad)
        assert e.value.status == gs.GS_EINVAL, (opt, bad)
    assert sim.launch() == before
    for v in range(4):
        sim.set_option(gs.OPT_STREAM, v)
        assert sim.launch()["stream"] == v
    sim.close()


def test_event_overflow_emitted_in_the_same_step():
    """Past 1152 absorbed ions in one workgroup and step the rest wait in the
    gap's list, and the push's last workgroup emits them before the push ends:
    the absorbed and emitted counts equal the oracle's at every level, as do
    the voltages and fields."""
    sched = W.gaussian_schedule(60, 3000.0, 30.0, 8.0)
    cfg = W.config_tesla(layer=0.0).replace(beam_schedule=sched, see_amp=30.0)
    sim, orc, recs = run_pair(cfg, {}, oracle.STRICT, 60, True, (200_000, 200_000))
    check_run(recs, 1e-5, cfg.n_mesh, cfg, oracle.STRICT)
    check_fields(sim, orc, 1e-5)
    assert recs[-1][0]["emit_cum"].sum() > 1000
    sim.close()


@pytest.mark.parametrize("stream", [0, 3])
def test_event_overflow_in_batched_gaps(stream):
    """Three gaps in one context: the first and last absorb thousands of beam
    ions a step at the grounded electrode, past their workgroups' queues, so
    those wait in the gaps' lists that the push's last workgroup emits; the
    middle one emits within its workgroups.  Every gap's counts, electrode
    potential, surface and circuit charges and loop currents equal its
    oracle's at every level, and the first gap's fields at the end (contiguous
    tile runs, and the round-robin non-temporal stream over five workgroups)."""
    gs = _gapsim()
    sched = W.gaussian_schedule(40, 3000.0, 20.0, 8.0)
    hot = W.config_tesla(layer=0.0).replace(beam_schedule=sched, see_amp=30.0)
    cfgs = [hot, cfg2_small(n_cells=700, beam=800), hot.replace(seed=6)]
    loads = [{}, W.load_config2(n=20_000, seed=32), {}]
    sim = gs.GapSim(cfgs, particle_fp=32, capacity=(200_000, 200_000))
    sim.set_option(gs.OPT_COMPACT_EVERY, 7)
    if stream:
        sim.set_option(gs.OPT_STREAM, stream)
        sim.set_option(gs.OPT_GRID, 5)
    orcs = []
    for g, cfg in enumerate(cfgs):
        o = oracle.OracleSim(cfg, fp32=True)
        for sp in sorted(loads[g]):
            x, v = loads[g][sp]
            o.inject(sp, x, v)
            sim.inject(g, sp, x, v)
        orcs.append(o)
    recs = [[] for _ in cfgs]
    for n in range(40):
        sim.step_strict(1)
        for g in range(len(cfgs)):
            orcs[g].step(oracle.STRICT, 1)
            recs[g].append((sim.diag(g), orcs[g].diag()))
    for g, cfg in enumerate(cfgs):
        check_run(recs[g], 1e-5, cfg.n_mesh, cfg, oracle.STRICT)
    check_fields(sim, orcs[0], 1e-5)
    for g in (0, 2):
        assert recs[g][-1][0]["emit_cum"].sum() > 1000
    sim.close()


def test_tesla_scenario_waveform_matches_oracle():
    """The whole stand-in Tesla run (575 steps, 5e6 ions injected, emission on)
    on the GPU against the oracle's binary32 mode.  Past the parity horizon single
    particles part ways, so the bar is on the gap-voltage waveform: its largest
    deviation stays within 1% of the swing, and the injected count is exact."""
    cfg = W.config_tesla()
    gs = _gapsim()
    sim = gs.GapSim(cfg, particle_fp=32, capacity=(3_000_000, 4_000_000))
    orc = oracle.OracleSim(cfg, fp32=True)
    Vg, Vo = [], []
    for _ in range(575):
        sim.step_strict(1)
        orc.step(oracle.STRICT, 1)
        Vg.append(sim.diag(0)["phi0"])
        Vo.append(orc.diag()["phi0"])
    Vg, Vo = np.array(Vg), np.array(Vo)
    dev = np.abs(Vg - Vo).max() / np.abs(Vo).max()
    print(f"largest |V_gpu - V_oracle| / max|V| = {dev:.2e}")
    assert dev < 1e-2
    assert sim.diag(0)["inj_cum"] == orc.diag()["inj_cum"] == int(cfg.beam_schedule.sum())
    sim.close()


@pytest.mark.parametrize("mode", [oracle.STRICT, oracle.WEAK])
def test_fp64_largest_grid_parity(mode):
    """The largest binary64 grid (8192 cells: the 64-bit accumulator and the
    binary64 table take 128 KiB of LDS), with a beam and emission.  Weak mode
    runs with the round-robin tile order over a few workgroups (the
    non-temporal bit is for binary32 particles and does nothing here)."""
    cfg = W.config2(n_cells=8192, beam_per_step=300, seed=9)
    loads = W.load_config2(n=60_000, seed=13)
    gs = _gapsim()
    opts = {gs.OPT_COMPACT_EVERY: 6}
    if mode == oracle.WEAK:
        opts.update({gs.OPT_STREAM: 3, gs.OPT_GRID: 6, gs.OPT_TILE: 2048})
    sim, orc, recs = run_pair(cfg, loads, mode, 25, False, (200_000, 200_000), opts=opts)
    for dg, do in recs:
        assert dg["step"] == do["step"]
        assert_counts_equal(dg, do)
    for key in ("phi0", "qcirc", "qcirc_star", "q_space"):
        assert _series_rel([d[key] for d, _ in recs], [o[key] for _, o in recs]) <= 1e-12, key
    # sigma is a sum whose terms can be five orders above it: in weak mode the
    # circuit's gap charge and the re-imposed C_gap phi0 nearly cancel (here
    # ~1e-9 against ~1e-14 C/m^2), so rounding is bounded relative to the terms
    A = cfg.area
    terms = max(max(abs(o["sigma"]), abs(o["qcirc_star"]) / A, abs(o["qcirc"]) / A) for _, o in recs)
    dsig = max(abs(d["sigma"] - o["sigma"]) for d, o in recs)
    assert dsig <= 1e-12 * terms, (dsig, terms)
    check_fields(sim, orc, 1e-12)
    d = recs[-1][0]
    assert d["inj_cum"] == 25 * 300 and d["abs_cum"][1].sum() > 10, d["abs_cum"]
    sim.close()


@pytest.mark.parametrize("fp32", [False, True])
def test_two_cell_gap_parity(fp32):
    """The smallest grid: two cells, three nodes (both electrode half cells meet
    in the middle), with particles crossing it every few steps, emission and a
    beam."""
    d_gap = 2e-4  # 200 um, so that the hot load reaches both walls within the run
    cfg = W.config1(n_cells=2).replace(d=d_gap, beam_per_step=3, beam_Emin_eV=100.0, beam_Emax_eV=500.0,
                                       see_amp=3.0)
    loads = W.load_config1(n_per_species=500, seed=17, d=d_gap)
    loads = {s: (x, v * 30.0) for s, (x, v) in loads.items()}
    sim, orc, recs = run_pair(cfg, loads, oracle.STRICT, 30, fp32, (20_000, 20_000))
    check_run(recs, 1e-5 if fp32 else 1e-12, cfg.n_mesh, cfg, oracle.STRICT)
    check_fields(sim, orc, 1e-5 if fp32 else 1e-12)
    d = recs[-1][0]
    assert d["abs_cum"][0].sum() > 100 and d["abs_cum"][1].sum() > 10 and d["inj_cum"] == 90, d["abs_cum"]
    sim.close()


def test_many_gaps_batched():
    """3000 gaps of 16 cells in one context (the push's per-workgroup prefix over
    gaps and its LDS): every gap's counts against its own oracle run, and the
    voltages within 1e-12 (binary64)."""
    gs = _gapsim()
    G = 3000
    cfgs = [W.config1(n_cells=16).replace(seed=g, beam_per_step=g % 3, beam_Emin_eV=1e3, beam_Emax_eV=5e3)
            for g in range(G)]
    rng = np.random.default_rng(3)
    sim = gs.GapSim(cfgs, particle_fp=64, capacity=(256, 256))
    orcs = []
    for g in range(G):
        n = int(rng.integers(0, 40))
        x = rng.uniform(0.0, cfgs[g].d, size=n)
        v = rng.normal(0.0, 3e5, size=n)
        o = oracle.OracleSim(cfgs[g])
        if n:
            sim.inject(g, 1, x, v)
            o.inject(1, x, v)
        orcs.append(o)
    sim.step_strict(8)
    for g in range(G):
        orcs[g].step(oracle.STRICT, 8)
        dg, do = sim.diag(g), orcs[g].diag()
        assert dg["step"] == do["step"] == 7
        assert_counts_equal(dg, do)
        assert abs(dg["phi0"] - do["phi0"]) <= 1e-12 * max(abs(do["phi0"]), 1.0), g
    sim.close()
