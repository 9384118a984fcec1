"""The library driven from plain C (tests/c/abi_run.c, no Python or PyTorch in
that process: the default stream and the library's own allocator), against the
oracle on the same inputs: counts bit-exact, gap voltage and surface charge
within 1e-12 (binary64 particles)."""
import subprocess

import numpy as np
import pytest

import oracle
from paper_2603_24010_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", [oracle.STRICT, oracle.WEAK])
def test_c_program_matches_oracle(tmp_path, mode):
    import c_abi
    from paper_2603_24010_amd import gapsim
    cfg = W.config1(n_cells=64)
    loads = W.load_config1(n_per_species=3000, seed=4)
    loads = {s: (x, v * 30.0) for s, (x, v) in loads.items()}
    params = gapsim.params_from(cfg, 64, (20000, 20000))
    exe = c_abi.build(str(tmp_path))
    pp, qp = c_abi.write_inputs(str(tmp_path), params, loads)
    steps = 30
    run = subprocess.run([exe, pp, qp, str(mode), str(steps)], capture_output=True, text=True, timeout=120)
    assert run.returncode == 0, run.stderr
    rows = [line.split() for line in run.stdout.splitlines()]
    assert len(rows) == steps
    orc = oracle.OracleSim(cfg)
    for sp, (x, v) in loads.items():
        orc.inject(sp, x, v)
    V, Vo, S, So = [], [], [], []
    for n, r in enumerate(rows):
        orc.step(mode, 1)
        d = orc.diag()
        assert int(r[0]) == d["step"] == n
        counts = [int(c) for c in r[4:10]]
        assert counts == list(d["abs_cum"].ravel()) + list(d["emit_cum"])
        assert int(r[10]) == int(d["n_live"].sum())
        V.append(float(r[1]))
        Vo.append(d["phi0"])
        S.append(float(r[2]))
        So.append(d["sigma"])
    V, Vo, S, So = map(np.array, (V, Vo, S, So))
    assert np.abs(V - Vo).max() <= 1e-12 * np.abs(Vo).max()
    assert np.abs(S - So).max() <= 1e-12 * np.abs(So).max()
    assert sum(int(c) for c in rows[-1][4:8]) > 50
