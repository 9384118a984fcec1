"""Small circuit engines that stand in for an external circuit simulator in the
weak-coupling tests (the role the paper gives ngspice through PySpice, Alg. 1).
Each is called as engine(gap, level, dt, phi0_prev) and returns the gap voltage
its circuit reaches at that level after restarting its gap capacitor from
phi0_prev.  They are test inputs: the same engine class drives the oracle and
the GPU library (one fresh instance each)."""
import math


class IdealSource:
    """An ideal voltage source across the gap: V* = dc + amp sin(w t_n)."""

    def __init__(self, amp: float, w: float, dc: float = 0.0):
        self.amp, self.w, self.dc = amp, w, dc

    def __call__(self, gap, level, dt, phi0_prev):
        return self.dc + self.amp * math.sin(self.w * level * dt)


class RCCharger:
    """A DC source V0 charging the gap capacitor through R, integrated exactly
    over the step from the restarted voltage: V* = V0 + (phi0_prev - V0) exp(-dt / (R C))."""

    def __init__(self, V0: float, R: float, C: float):
        self.V0, self.R, self.C = V0, R, C

    def __call__(self, gap, level, dt, phi0_prev):
        return self.V0 + (phi0_prev - self.V0) * math.exp(-dt / (self.R * self.C))


class SeriesRCBDF2:
    """One mesh (source, R, elastance S and the gap element C_gap in parallel with
    c_par), stepped with BDF2 in loop-charge increments the way the library's own
    weak mode steps it: the gap charge restarts from (C_gap + c_par) phi0_prev,
    the previous increment is kept, and
        R (3 D - D_1) / (2 dt) + (S + 1 / C_t) (q_prev + D) = src Vs(t_n),
    C_t = C_gap + c_par.  Returns (q_prev + D) / C_t."""

    def __init__(self, cfg):
        assert cfg.n_mesh == 1 and cfg.L[0, 0] == 0.0
        self.R, self.S = float(cfg.R[0, 0]), float(cfg.S[0, 0])
        self.ct = cfg.eps0 * cfg.area / cfg.d + cfg.c_par
        self.src = float(cfg.src[0])
        self.dc, self.amp = cfg.src_dc, cfg.src_amp
        self.w, self.ph = 2.0 * math.pi * cfg.src_freq, cfg.src_phase
        self.D1 = 0.0

    def __call__(self, gap, level, dt, phi0_prev):
        vs = self.dc + self.amp * math.sin(self.w * level * dt + self.ph)
        q_prev = self.ct * phi0_prev
        sp = self.S + 1.0 / self.ct
        D = (self.src * vs - sp * q_prev + self.R * self.D1 / (2.0 * dt)) / (3.0 * self.R / (2.0 * dt) + sp)
        self.D1 = D
        return (q_prev + D) / self.ct
