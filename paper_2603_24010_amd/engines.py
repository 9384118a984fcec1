"""Circuit engines for weak coupling with an external solver
(GapSim.step_weak_external / gs_step_weak_external).

The paper's weak mode hands the circuit to a black-box simulator (ngspice via
PySpice, Sec. 2.1 and Alg. 1): each step the simulator restarts from given
capacitor voltages and inductor currents, runs a transient over one step and
returns the new node voltages; the gap charge it implies enters the surface-charge
update (Sec. 2.4.3).  An engine here is any callable
    engine(gap, level, dt, phi0_prev) -> gap voltage at level `level`
that keeps its own circuit state.  Host code only; nothing here runs on the GPU.
"""
from __future__ import annotations

import math

import numpy as np


class LinearCircuitEngine:
    """Exact transient of a linear loop circuit with inductance in every loop.

    For each gap: L q'' + R q' + S' q = src Vs(t), S' = S plus the gap element's
    elastance 1 / (C_gap + c_par) in the gap mesh, Vs(t) = dc + amp sin(w t + phase).
    With the source's sine and cosine carried as two more state variables the
    system is z' = A z, z = (q, q', sin, cos, 1), so one step is z <- expm(A dt) z,
    exact up to rounding.  At each call the gap capacitor restarts from the
    electrode potential the field solve gave (q_gap = (C_gap + c_par) phi0_prev);
    the other loop charges and every current carry over, as when a circuit
    simulator restarts from given capacitor voltages and inductor currents.
    The state before level 0 is q0 with no current, at t = -dt.
    """

    def __init__(self, cfgs):
        from scipy.linalg import expm
        if not isinstance(cfgs, (list, tuple)):
            cfgs = [cfgs]
        self._g = []
        for cfg in cfgs:
            M, gm = cfg.n_mesh, cfg.gap_mesh
            L = np.asarray(cfg.L, dtype=np.float64)
            if np.linalg.matrix_rank(L) < M:
                raise ValueError("LinearCircuitEngine needs inductance in every loop (L nonsingular)")
            ct = cfg.eps0 * cfg.area / cfg.d + cfg.c_par
            S = np.array(cfg.S, dtype=np.float64)
            S[gm, gm] += 1.0 / ct
            Li = np.linalg.inv(L)
            w = 2.0 * math.pi * cfg.src_freq
            n = 2 * M + 3
            A = np.zeros((n, n))
            A[:M, M:2 * M] = np.eye(M)
            A[M:2 * M, :M] = -Li @ S
            A[M:2 * M, M:2 * M] = -Li @ np.asarray(cfg.R, dtype=np.float64)
            b = Li @ np.asarray(cfg.src, dtype=np.float64)
            A[M:2 * M, 2 * M] = cfg.src_amp * b       # sin(w t + phase)
            A[M:2 * M, 2 * M + 2] = cfg.src_dc * b    # 1
            A[2 * M, 2 * M + 1] = w                   # (sin)' = w cos
            A[2 * M + 1, 2 * M] = -w                  # (cos)' = -w sin
            z = np.zeros(n)
            z[:M] = cfg.q0
            t0 = -cfg.dt
            z[2 * M] = math.sin(w * t0 + cfg.src_phase)
            z[2 * M + 1] = math.cos(w * t0 + cfg.src_phase)
            z[2 * M + 2] = 1.0
            self._g.append(dict(E=expm(A * cfg.dt), z=z, M=M, gm=gm, ct=ct, dt=cfg.dt, next=0))

    def __call__(self, gap, level, dt, phi0_prev):
        g = self._g[gap]
        if level != g["next"] or dt != g["dt"]:
            raise ValueError(f"gap {gap}: expected level {g['next']} with dt {g['dt']}, got {level}, {dt}")
        z = g["z"]
        z[g["gm"]] = g["ct"] * phi0_prev
        g["z"] = z = g["E"] @ z
        g["next"] = level + 1
        return float(z[g["gm"]] / g["ct"])

    def state(self, gap: int = 0):
        """Loop charges and currents after the last call."""
        g = self._g[gap]
        return g["z"][:g["M"]].copy(), g["z"][g["M"]:2 * g["M"]].copy()
