"""Helpers for driving the library from plain C (tests/c/abi_run.c)."""
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "c", "abi_run.c")
PKG = os.path.join(ROOT, "paper_2603_24010_amd")


def build(out_dir: str) -> str:
    """Compile abi_run.c with gcc against include/gapsim.h and libgapsim.so."""
    exe = os.path.join(out_dir, "abi_run")
    subprocess.run(["gcc", "-O1", "-std=c11", "-Wall", "-Werror", "-o", exe, SRC, "-I", os.path.join(ROOT, "include"),
                    "-L", PKG, "-lgapsim", "-Wl,-rpath," + PKG], check=True)
    return exe


def write_inputs(out_dir: str, params, loads) -> tuple:
    """The parameters as the bytes of a gs_gap_params and the particles as the
    program reads them."""
    import ctypes as C
    pp = os.path.join(out_dir, "params.bin")
    with open(pp, "wb") as f:
        f.write(C.string_at(C.addressof(params), C.sizeof(params)))
    qp = os.path.join(out_dir, "particles.bin")
    with open(qp, "wb") as f:
        for sp in (0, 1):
            x, v = loads.get(sp, (np.zeros(0), np.zeros(0)))
            np.array([len(x)], dtype=np.int64).tofile(f)
            np.ascontiguousarray(x, dtype=np.float64).tofile(f)
            np.ascontiguousarray(v, dtype=np.float64).tofile(f)
    return pp, qp
