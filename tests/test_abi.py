"""The C-ABI library on the CPU: it loads, exports every entry point the header
declares, and its host-side parameter checks work without a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2603_24010_amd import gapsim, workloads as W

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                      "gapsim.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = gapsim.lib()
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(gapsim.EXPORTED)


def test_version_string():
    assert gapsim.lib().gs_version().startswith(b"gapsim")


@pytest.mark.parametrize("make,fp,cap", [
    (lambda: W.config1(), 64, (100000, 100000)),
    (lambda: W.config2(), 32, (30_000_000, 2_000_000)),
    (lambda: W.config3(), 32, (10_000_000, 300_000_000)),
    (lambda: W.config4_gap(3)[0], 32, (100_000, 700_000)),
    (lambda: W.config_paper_validation(), 64, (16, 16)),
    (lambda: W.config2(n_cells=600).replace(**W.circuit_tesla()), 32, (1000, 1000)),
    (lambda: W.config_tesla(), 32, (3_000_000, 4_000_000)),
    (lambda: W.config_tesla().replace(beam_schedule=np.zeros(0, dtype=np.int64)), 32, (10, 10)),
])
def test_valid_configs_pass(make, fp, cap):
    assert gapsim.validate(make(), fp, cap) is None


@pytest.mark.parametrize("change,fp,cap,needle", [
    (dict(n_cells=1), 32, (10, 10), "n_cells"),
    (dict(n_cells=20000), 32, (10, 10), "n_cells"),
    (dict(n_cells=9000), 64, (10, 10), "n_cells"),
    (dict(dt=0.0), 32, (10, 10), "dt"),
    (dict(d=float("nan")), 32, (10, 10), "d,"),
    (dict(Z=(0, 1)), 32, (10, 10), "Z"),
    (dict(see_law=7), 32, (10, 10), "see_law"),
    (dict(see_max=5000), 32, (10, 10), "see_max"),
    (dict(beam_per_step=10, beam_Emin_eV=5.0, beam_Emax_eV=1.0), 32, (10, 10), "beam"),
    (dict(v_ref=0.0), 32, (10, 10), "v_ref"),
    (dict(gap_mesh=3), 32, (10, 10), "gap_mesh"),
    (dict(), 16, (10, 10), "particle_fp"),
    (dict(), 64, (1 << 19, 1 << 19), "2^19"),
    (dict(), 32, (-1, 10), "capacity"),
    (dict(beam_side=2), 32, (10, 10), "beam_side"),
    (dict(see_yield=2), 32, (10, 10), "see_yield"),
    (dict(see_yield=1, see_poly_Emax_eV=0.0), 32, (10, 10), "see_poly_Emax_eV"),
    (dict(see_poly=np.array([0, 0, float("inf"), 0, 0, 0])), 32, (10, 10), "see_poly"),
    (dict(see_law=2, see_ln_sigma=-1.0), 32, (10, 10), "see_ln"),
    (dict(beam_layer=0.01), 32, (10, 10), "beam_layer"),
    (dict(beam_layer=-1e-3), 32, (10, 10), "beam_layer"),
    (dict(beam_schedule=np.array([3, -1])), 32, (10, 10), "beam_schedule"),
    (dict(beam_schedule=np.array([0, 5])), 32, (10, 10), "beam energies"),
])
def test_invalid_params_rejected(change, fp, cap, needle):
    cfg = W.config1(n_cells=64).replace(**change)
    msg = gapsim.validate(cfg, fp, cap)
    assert msg is not None and needle in msg


def test_init_rejects_bad_arguments_without_touching_a_device():
    lib = gapsim.lib()
    h = C.c_void_p()
    arr = (gapsim.GsGapParams * 1)()
    arr[0] = gapsim.params_from(W.config1(n_cells=1), 64, (10, 10))
    rc = lib.gs_init_gap(C.byref(h), 1, arr, None, None)
    assert rc == gapsim.GS_EINVAL and not h.value
    assert b"n_cells" in lib.gs_last_error(None)
    rc = lib.gs_init_gap(C.byref(h), 0, arr, None, None)
    assert rc == gapsim.GS_EINVAL
    mixed = (gapsim.GsGapParams * 2)()
    mixed[0] = gapsim.params_from(W.config1(), 64, (10, 10))
    mixed[1] = gapsim.params_from(W.config1(), 32, (10, 10))
    assert lib.gs_init_gap(C.byref(h), 2, mixed, None, None) == gapsim.GS_EINVAL
    assert b"particle_fp" in lib.gs_last_error(None)


def test_null_context_is_a_state_error():
    lib = gapsim.lib()
    assert lib.gs_step_weak(None, 1) == gapsim.GS_ESTATE
    assert lib.gs_step_strict(None, 1, 0) == gapsim.GS_ESTATE
    assert lib.gs_set_option(None, 1, 256) == gapsim.GS_ESTATE


def test_external_engine_and_dt_check_argument_errors_without_a_device():
    lib = gapsim.lib()
    fn = gapsim.CIRCUIT_FN(lambda *a: 0)
    assert lib.gs_step_weak_external(None, 1, fn, None) == gapsim.GS_ESTATE
    assert lib.gs_dt_check(None, 0, C.byref(gapsim.GsDtReport())) == gapsim.GS_ESTATE
    w = C.c_double(-1.0)
    assert lib.gs_circuit_resonance(None, C.byref(w)) == gapsim.GS_EINVAL
    bad = gapsim.params_from(W.config1(n_cells=1), 64, (10, 10))
    assert lib.gs_circuit_resonance(C.byref(bad), C.byref(w)) == gapsim.GS_EINVAL
    good = gapsim.params_from(W.config1(), 64, (10, 10))
    assert lib.gs_circuit_resonance(C.byref(good), None) == gapsim.GS_EINVAL
    assert lib.gs_circuit_resonance(C.byref(good), C.byref(w)) == gapsim.GS_OK and w.value == 0.0


def test_c_program_compiles_and_links_against_the_library(tmp_path):
    """The boundary is usable from plain C: tests/c/abi_run.c builds with gcc
    against include/gapsim.h and links libgapsim.so (run on the GPU by
    tests/test_gpu_c_abi.py)."""
    import c_abi
    exe = c_abi.build(str(tmp_path))
    assert os.path.exists(exe)
