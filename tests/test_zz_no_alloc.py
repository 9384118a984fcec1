"""gs_inject_noalloc (the entry point for callers that cannot allocate device
memory) against gs_inject, through the C ABI: two calls in a row, the second
smaller, then a few steps; the particle states and diagnostics are the same."""
import ctypes as C

import numpy as np
import pytest

from paper_2603_24010_amd import workloads as W

pytestmark = pytest.mark.gpu


def _state(sim, sp):
    x, u, ids = sim.particles(0, sp)
    o = np.lexsort((u, x, ids))  # emitted electrons share one id
    return x[o], u[o], ids[o]


@pytest.mark.parametrize("fp", [32, 64])
def test_inject_noalloc_matches_inject(fp):
    from paper_2603_24010_amd import gapsim as gs
    L = gs.lib()
    cfg = W.config2(n_cells=1024, beam_per_step=300)
    rng = np.random.default_rng(8)
    batches = []
    # (binary64 particles: at most 2^19 per gap, the fixed-point deposit's range)
    for n in ((300_000, 1_000) if fp == 32 else (150_000, 1_000)):  # the second call smaller
        x = np.ascontiguousarray(rng.uniform(0.0, cfg.d, n))
        v = np.ascontiguousarray(rng.normal(0.0, 2e5, n))
        batches.append((x, v))
    cap = (400_000, 400_000) if fp == 32 else (200_000, 200_000)
    a = gs.GapSim(cfg, particle_fp=fp, capacity=cap)
    b = gs.GapSim(cfg, particle_fp=fp, capacity=cap)
    for k, (x, v) in enumerate(batches):
        sp = k % 2
        a.inject(0, sp, x, v)  # gs_inject, host arrays
        rc = L.gs_inject_noalloc(b._h, 0, sp, len(x), x.ctypes.data_as(C.c_void_p), v.ctypes.data_as(C.c_void_p))
        assert rc == gs.GS_OK, L.gs_last_error(b._h)
    for sp in (0, 1):
        for p, q in zip(_state(a, sp), _state(b, sp)):
            np.testing.assert_array_equal(p, q)
    a.step_weak(5)
    b.step_weak(5)
    da, db = a.diag(0), b.diag(0)
    np.testing.assert_array_equal(da["n_live"], db["n_live"])
    np.testing.assert_array_equal(da["abs_cum"], db["abs_cum"])
    np.testing.assert_array_equal(da["emit_cum"], db["emit_cum"])
    assert da["phi0"] == db["phi0"] and da["sigma"] == db["sigma"]
    for sp in (0, 1):
        for p, q in zip(_state(a, sp), _state(b, sp)):
            np.testing.assert_array_equal(p, q)
    a.close()
    b.close()


def test_inject_noalloc_rejects_too_many():
    from paper_2603_24010_amd import gapsim as gs
    L = gs.lib()
    cfg = W.config1(n_cells=32)
    sim = gs.GapSim(cfg, particle_fp=64, capacity=(16, 16))
    n = (1 << 19) + 1
    x = np.zeros(n)
    rc = L.gs_inject_noalloc(sim._h, 0, 0, n, x.ctypes.data_as(C.c_void_p), x.ctypes.data_as(C.c_void_p))
    assert rc == gs.GS_EINVAL
    assert b"at most" in L.gs_last_error(sim._h)
    sim.close()
