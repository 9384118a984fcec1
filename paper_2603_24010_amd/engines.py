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
    The state before level 0 is q0 with no current, at t = -dt, so an engine
    drives a context from its first level (a call for another level raises).
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


class RadauCircuitEngine:
    """A stiff transient of a linear loop circuit in descriptor form, as a
    SPICE-like engine: with z = (q, i),
        blkdiag(I, L) z' = [[0, I], [-S', -R]] z + (0, src Vs(t)),
    stepped by the two-stage Radau IIA collocation method (order 3, L-stable and
    stiffly accurate; Hairer and Wanner, Solving ODEs II, Sec. IV.5), `substeps`
    internal steps per coupling step.  L may be singular (loops without
    inductance, as in the paper's Tesla circuit): such loops are algebraic, and
    the method puts their currents back on the constraint after each restart of
    the gap capacitor, where the trapezoidal rule would ring.  The gap capacitor
    restarts from phi0_prev at each call; the state before level 0 is q0 with no
    current, at t = -dt, so an engine drives a context from its first level."""

    C = (1.0 / 3.0, 1.0)
    A = ((5.0 / 12.0, -1.0 / 12.0), (3.0 / 4.0, 1.0 / 4.0))

    def __init__(self, cfgs, substeps: int = 1):
        if not isinstance(cfgs, (list, tuple)):
            cfgs = [cfgs]
        self.substeps = int(substeps)
        self._g = []
        for cfg in cfgs:
            M, gm = cfg.n_mesh, cfg.gap_mesh
            h = cfg.dt / self.substeps
            ct = cfg.eps0 * cfg.area / cfg.d + cfg.c_par
            S = np.array(cfg.S, dtype=np.float64)
            S[gm, gm] += 1.0 / ct
            n = 2 * M
            Mm = np.zeros((n, n))
            Mm[:M, :M] = np.eye(M)
            Mm[M:, M:] = np.asarray(cfg.L, dtype=np.float64)
            Am = np.zeros((n, n))
            Am[:M, M:] = np.eye(M)
            Am[M:, :M] = -S
            Am[M:, M:] = -np.asarray(cfg.R, dtype=np.float64)
            (a11, a12), (a21, a22) = self.A
            K = np.block([[Mm - h * a11 * Am, -h * a12 * Am], [-h * a21 * Am, Mm - h * a22 * Am]])
            if np.linalg.cond(K) > 1e15:
                raise ValueError("the Radau stage matrix is singular for this circuit and step")
            z = np.zeros(n)
            z[:M] = cfg.q0
            self._g.append(dict(Ki=np.linalg.inv(K), Mm=Mm, z=z, M=M, gm=gm, ct=ct, dt=cfg.dt, h=h, next=0,
                                src=np.asarray(cfg.src, dtype=np.float64), cfg=cfg))

    def _vs(self, cfg, t):
        return cfg.src_dc + cfg.src_amp * math.sin(2.0 * math.pi * cfg.src_freq * t + cfg.src_phase)

    def __call__(self, gap, level, dt, phi0_prev):
        g = self._g[gap]
        if level != g["next"] or dt != g["dt"]:
            raise ValueError(f"gap {gap}: expected level {g['next']} with dt {g['dt']}, got {level}, {dt}")
        M, h, cfg = g["M"], g["h"], g["cfg"]
        z = g["z"]
        z[g["gm"]] = g["ct"] * phi0_prev
        (a11, a12), (a21, a22) = self.A
        t0 = (level - 1) * dt
        for k in range(self.substeps):
            ts = t0 + k * h
            b1 = self._vs(cfg, ts + self.C[0] * h) * g["src"]
            b2 = self._vs(cfg, ts + self.C[1] * h) * g["src"]
            mz = g["Mm"] @ z
            rhs = np.concatenate([mz, mz])
            rhs[M:2 * M] += h * (a11 * b1 + a12 * b2)
            rhs[3 * M:] += h * (a21 * b1 + a22 * b2)
            z = (g["Ki"] @ rhs)[2 * M:]  # stiffly accurate: the new state is the last stage
        g["z"] = z
        g["next"] = level + 1
        return float(z[g["gm"]] / g["ct"])

    def state(self, gap: int = 0):
        g = self._g[gap]
        return g["z"][:g["M"]].copy(), g["z"][g["M"]:].copy()
