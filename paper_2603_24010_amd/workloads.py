"""Seeded synthetic workloads: gap/circuit parameter sets and initial particle loads.

This module only *describes* inputs (element values, mesh matrices of a circuit,
random initial particle arrays).  It holds none of the method's arithmetic (no
BDF2, no Poisson, no push), so both the GPU library's binding and the CPU oracle's
binding may read it.

Circuits are given in loop (mesh) form, the way the paper writes its Tesla circuit
(Sec. 2.1, eq. loop_1..loop_5):  L q'' + R q' + S q + g V_gap = b Vs(t), where q are
loop charges, S holds elastances (1/C), g selects the one mesh that runs through the
gap, and c_par is a capacitance in parallel with the gap inside that mesh.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

MAX_MESH = 8

# CODATA 2018
E_CHARGE = 1.602176634e-19
M_ELECTRON = 9.1093837015e-31
M_PROTON = 1.67262192369e-27
EPS0 = 8.8541878128e-12

# constants the paper's validation runs use (App. E, tab:validation_parameters)
PAPER_EPS0 = 8.85e-12
PAPER_Q = 1.6e-19
PAPER_M_TI = 7.95e-26
PAPER_M_E_SCALED = 9.1e-28

SEE_FIXED = 0
SEE_EXP = 1
SEE_LOGNORMAL = 2
YIELD_SATURATING = 0
YIELD_POLY = 1
BEAM_CIRCUIT = 0
BEAM_GROUND = 1


@dataclasses.dataclass
class GapConfig:
    n_cells: int
    d: float
    area: float
    eps0: float
    dt: float
    Z: tuple = (-1, 1)
    mass: tuple = (M_ELECTRON, M_PROTON)
    q_unit: float = E_CHARGE
    weight: float = 2.5e7
    ev: float = E_CHARGE
    n_mesh: int = 1
    gap_mesh: int = 0
    L: np.ndarray = None
    R: np.ndarray = None
    S: np.ndarray = None
    src: np.ndarray = None
    src_dc: float = 0.0
    src_amp: float = 0.0
    src_freq: float = 0.0
    src_phase: float = 0.0
    c_par: float = 0.0
    q0: np.ndarray = None
    see_amp: float = 0.0
    see_E0_eV: float = 1000.0
    see_law: int = SEE_FIXED
    see_max: int = 32
    see_E_eV: float = 2.0
    see_yield: int = 0                # YIELD_SATURATING or YIELD_POLY
    see_poly: np.ndarray = None       # YIELD_POLY: c_0..c_5 in powers of E / 1 keV
    see_poly_Emax_eV: float = 8e4     # YIELD_POLY: energy clamp (the fit's range)
    see_ln_mu: float = 0.0            # SEE_LOGNORMAL: ln E ~ N(mu, sigma^2), E in eV
    see_ln_sigma: float = 0.0
    beam_per_step: int = 0
    beam_Emin_eV: float = 0.0
    beam_Emax_eV: float = 0.0
    beam_side: int = 0          # BEAM_CIRCUIT (node 0) or BEAM_GROUND (node N)
    beam_layer: float = 0.0     # start layer width [m]; 0: one step of flight
    beam_schedule: np.ndarray = None  # ions per step by level (int64); None: beam_per_step
    seed: int = 0
    v_ref: float = 1.0  # voltage scale for residual norms

    def __post_init__(self):
        m = self.n_mesh
        for name in ("L", "R", "S"):
            if getattr(self, name) is None:
                setattr(self, name, np.zeros((m, m)))
            setattr(self, name, np.asarray(getattr(self, name), dtype=np.float64).reshape(m, m))
        for name in ("src", "q0"):
            if getattr(self, name) is None:
                setattr(self, name, np.zeros(m))
            setattr(self, name, np.asarray(getattr(self, name), dtype=np.float64).reshape(m))
        self.see_poly = (np.zeros(6) if self.see_poly is None
                         else np.asarray(self.see_poly, dtype=np.float64).reshape(6))
        if self.beam_schedule is not None:
            self.beam_schedule = np.ascontiguousarray(self.beam_schedule, dtype=np.int64).reshape(-1)

    def replace(self, **kw) -> "GapConfig":
        return dataclasses.replace(self, **kw)


# ---------------------------------------------------------------------------
# circuits (mesh descriptions)
# ---------------------------------------------------------------------------
def circuit_series_rc_source(R: float, C: float, amp: float, freq: float) -> dict:
    """One mesh: source, R, C and the gap in series."""
    return dict(n_mesh=1, gap_mesh=0, L=[[0.0]], R=[[R]], S=[[1.0 / C]], src=[1.0],
                src_amp=amp, src_freq=freq, c_par=0.0, q0=[0.0])


def circuit_r_gap(R: float) -> dict:
    """One mesh: a resistor across the gap capacitor (the paper's App. E RC case)."""
    return dict(n_mesh=1, gap_mesh=0, L=[[0.0]], R=[[R]], S=[[0.0]], src=[0.0], c_par=0.0,
                q0=[0.0])


def circuit_coupled_lc(L1: float, C1: float, L2: float, C2: float, k: float, V1: float,
                       R2: float = 0.0) -> dict:
    """Two inductively coupled loops.  Primary: L1 with C1 charged to V1.  Secondary:
    L2 (and R2) closing on C2, with the gap in parallel with C2."""
    M = k * math.sqrt(L1 * L2)
    return dict(n_mesh=2, gap_mesh=1,
                L=[[L1, M], [M, L2]],
                R=[[0.0, 0.0], [0.0, R2]],
                S=[[1.0 / C1, 0.0], [0.0, 0.0]],
                src=[0.0, 0.0], c_par=C2, q0=[C1 * V1, 0.0])


def circuit_tesla(R1=5.0, R2=5.0, R3=100e6, C1=3.8e-6, C2=2.8e-12, L1=47e-6, L2=0.13, k=0.37,
                  V1=3000.0) -> dict:
    """The paper's simplified Tesla transformer (Sec. 2.1, tab:circuit_parameters):
    five loops; C3 is the gap (loop 4)."""
    M = k * math.sqrt(L1 * L2)
    L = np.zeros((5, 5))
    L[1, 1] = L1; L[1, 2] = M; L[2, 1] = M; L[2, 2] = L2
    R = np.array([
        [R1, -R1, 0.0, 0.0, -R1],
        [-R1, R1 + R2, 0.0, 0.0, R1],
        [0.0, 0.0, R3, -R3, R3],
        [0.0, 0.0, -R3, R3, -R3],
        [-R1, R1, R3, -R3, R1 + R3],
    ])
    S = np.zeros((5, 5))
    S[0, 0] = 1.0 / C1
    S[4, 4] = 1.0 / C2
    return dict(n_mesh=5, gap_mesh=3, L=L, R=R, S=S, src=np.zeros(5), c_par=0.0,
                q0=[C1 * V1, 0.0, 0.0, 0.0, 0.0])


# ---------------------------------------------------------------------------
# gap configurations
# ---------------------------------------------------------------------------
def config_paper_validation() -> GapConfig:
    """App. E (tab:validation_parameters): 80 mm gap, 601 nodes, dt 1.5e-11 s, R1 across
    the gap capacitor, paper constants (eps0 = 8.85e-12, e = 1.6e-19, Ti mass)."""
    return GapConfig(n_cells=600, d=0.08, area=2.53e-2, eps0=PAPER_EPS0, dt=1.5e-11,
                     mass=(PAPER_M_E_SCALED, PAPER_M_TI), q_unit=PAPER_Q, weight=2.5e7,
                     ev=PAPER_Q, v_ref=1.0, **circuit_r_gap(1.8e4))


def config1(n_cells: int = 256) -> GapConfig:
    """Strict, FP64: 1 cm gap, 256 cells, series R = 50 ohm, C = 100 pF, 10 kV 1 MHz
    drive; SEE a = 0.5 with 2 eV electrons."""
    return GapConfig(n_cells=n_cells, d=0.01, area=2.53e-2, eps0=EPS0, dt=1e-12, weight=2.5e7,
                     see_amp=0.5, see_law=SEE_FIXED, see_E_eV=2.0, seed=0, v_ref=1e4,
                     **circuit_series_rc_source(50.0, 100e-12, 1e4, 1e6))


def config2(n_cells: int = 4096, beam_per_step: int = 20000, weight: float = 2.5e5,
            seed: int = 2) -> GapConfig:
    """Weak, FP32 particles: coupled LC (L1 1 uH, C1 1 uF charged to 3 kV, L2 10 mH,
    C2 50 pF, k 0.6) loaded by the gap; H+ beam at the circuit electrode, 1-50 keV;
    SEE a = 0.5 with exponential 3 eV electrons."""
    return GapConfig(n_cells=n_cells, d=0.01, area=2.53e-2, eps0=EPS0, dt=1e-12, weight=weight,
                     see_amp=0.5, see_law=SEE_EXP, see_E_eV=3.0, beam_per_step=beam_per_step,
                     beam_Emin_eV=1e3, beam_Emax_eV=50e3, seed=seed, v_ref=3e3,
                     **circuit_coupled_lc(1e-6, 1e-6, 1e-2, 50e-12, 0.6, 3e3))


M_TI = 7.95e-26             # ion mass of the paper's integrated run (tab:space_time_variable)
M_ELECTRON_X1000 = 9.1e-28  # its electron mass, raised 1000-fold (Sec. 4.2)


def gaussian_schedule(n_steps: int, peak: float, center: float, width: float) -> np.ndarray:
    """Ions per step of a Gaussian pulse: round(peak exp(-(n - center)^2 / (2 width^2)))
    for the step that solves level n = 0 .. n_steps - 1."""
    n = np.arange(n_steps, dtype=np.float64)
    return np.rint(peak * np.exp(-0.5 * ((n - center) / width) ** 2)).astype(np.int64)


def config_tesla(n_cells: int = 600, n_steps: int = 575, peak: float = 40000.0, center: float = 300.0,
                 width: float = 50.0, layer: float = 2e-3, see_amp: float = 3.0, see_E0_eV: float = 2e4,
                 E_lo: float = 10.0, E_hi: float = 50.0, seed: int = 5, dt: float = 15e-9) -> GapConfig:
    """The paper's integrated Tesla run (Sec. 4.2, tab:space_time_variable,
    tab:circuit_parameters): 80 mm gap of 2.53e-2 m^2 on 600 cells, dt 15 ns, 575
    steps (8.62 us), Ti+ ions and electrons of 1000 times their mass, superparticle
    ratio 2.5e7, the five-loop Tesla circuit with C1 at 3 kV.  Ions enter in a
    layer next to the grounded electrode with a Gaussian pulse in time.  The paper
    shows the pulse, the layer, the ions' entry energies and the yield curve only
    as figures; peak / center / width (ions per step, steps), layer [m], energies
    [eV] and the yield law's a and E0 here are stand-ins.  The pulse is centred on
    the first swing that drives the circuit electrode negative (it attracts the
    ions), at 4.5 us.  n_steps, peak (ions per step), center and width are given
    for 15 ns steps; another dt keeps the same physical pulse and run length
    (dt = 1.5e-11 s, the step the paper's App. D checks, gives 574667 steps of
    40 ions at the peak)."""
    f = 15e-9 / dt
    if f != 1.0:
        n_steps = int(round(n_steps * f))
        peak, center, width = peak / f, center * f, width * f
    return GapConfig(n_cells=n_cells, d=0.08, area=2.53e-2, eps0=EPS0, dt=dt,
                     mass=(M_ELECTRON_X1000, M_TI), weight=2.5e7,
                     see_amp=see_amp, see_E0_eV=see_E0_eV, see_law=SEE_EXP, see_E_eV=3.0,
                     beam_side=BEAM_GROUND, beam_layer=layer,
                     beam_schedule=gaussian_schedule(n_steps, peak, center, width),
                     beam_Emin_eV=E_lo, beam_Emax_eV=E_hi, seed=seed, v_ref=1e4,
                     **circuit_tesla())


def config3(n_cells: int = 16384, **kw) -> GapConfig:
    return config2(n_cells=n_cells, **kw)


def config4_gap(g: int, n_cells: int = 512, np_lo: int = 50000, np_hi: int = 500000,
                weight: float = 2.5e5) -> tuple:
    """One gap of the batched ensemble: returns (config, n_particles, beam energy eV).
    Draws: particle count, monoenergetic beam energy, R in the secondary, k, SEE amplitude."""
    rng = np.random.Generator(np.random.Philox(1_000_003 + g))
    n_p = int(rng.integers(np_lo, np_hi + 1))
    e_b = float(rng.uniform(1e3, 50e3))
    R2 = float(rng.uniform(10.0, 200.0))
    k = float(rng.uniform(0.3, 0.8))
    a = float(rng.uniform(0.1, 1.0))
    d, dt = 0.01, 1e-12
    v_b = math.sqrt(2.0 * e_b * E_CHARGE / M_PROTON)
    rate = int(round(n_p * v_b * dt / d))
    cfg = GapConfig(n_cells=n_cells, d=d, area=2.53e-2, eps0=EPS0, dt=dt, weight=weight,
                    see_amp=a, see_law=SEE_EXP, see_E_eV=3.0, beam_per_step=rate,
                    beam_Emin_eV=e_b, beam_Emax_eV=e_b, seed=g, v_ref=3e3,
                    **circuit_coupled_lc(1e-6, 1e-6, 1e-2, 50e-12, k, 3e3, R2=R2))
    return cfg, n_p, e_b


# ---------------------------------------------------------------------------
# initial particle loads (SI: x in m, v in m/s), numpy Philox-seeded
# ---------------------------------------------------------------------------
def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(seed))


def load_uniform_maxwellian(d: float, n: int, mass: float, kT_eV: float, seed: int):
    """x ~ U(0, d), v_x ~ N(0, kT/m)."""
    rng = _rng(seed)
    x = rng.uniform(0.0, d, n)
    v = rng.normal(0.0, math.sqrt(kT_eV * E_CHARGE / mass), n)
    return x, v


def load_beam_energies(n: int, mass: float, e_lo_eV: float, e_hi_eV: float,
                       rng: np.random.Generator):
    e = rng.uniform(e_lo_eV, e_hi_eV, n)
    return np.sqrt(2.0 * e * E_CHARGE / mass)


def load_uniform_beam(d: float, n: int, mass: float, e_lo_eV: float, e_hi_eV: float, seed: int):
    """x ~ U(0, d), moving towards the grounded electrode with E ~ U(e_lo, e_hi)."""
    rng = _rng(seed)
    x = rng.uniform(0.0, d, n)
    v = load_beam_energies(n, mass, e_lo_eV, e_hi_eV, rng)
    return x, v


def load_gaussian_beam(d: float, n: int, mass: float, centre: float, width: float,
                       e_lo_eV: float, e_hi_eV: float, seed: int):
    """x ~ N(centre, width^2) truncated to (0, d) by redrawing; beam energies as above."""
    rng = _rng(seed)
    x = rng.normal(centre, width, n)
    bad = (x <= 0.0) | (x >= d)
    while bad.any():
        x[bad] = rng.normal(centre, width, int(bad.sum()))
        bad = (x <= 0.0) | (x >= d)
    v = load_beam_energies(n, mass, e_lo_eV, e_hi_eV, rng)
    return x, v


def load_config1(n_per_species: int = 50000, seed: int = 0, d: float = 0.01):
    """Electrons and H+ uniform in the gap, Maxwellian at 2 eV (v_x only is dynamic)."""
    xe, ve = load_uniform_maxwellian(d, n_per_species, M_ELECTRON, 2.0, seed)
    xi, vi = load_uniform_maxwellian(d, n_per_species, M_PROTON, 2.0, seed + 1)
    return {0: (xe, ve), 1: (xi, vi)}


def load_config2(n: int = 20_000_000, seed: int = 2, d: float = 0.01):
    x, v = load_uniform_beam(d, n, M_PROTON, 1e3, 50e3, seed)
    return {1: (x, v)}


def load_config3(n: int = 200_000_000, seed: int = 3, d: float = 0.01):
    x, v = load_gaussian_beam(d, n, M_PROTON, 0.9 * d, 0.05 * d, 1e3, 50e3, seed)
    return {1: (x, v)}


def load_config4_gap(n_p: int, e_b: float, g: int, d: float = 0.01):
    rng = _rng(7_000_000 + g)
    x = rng.uniform(0.0, d, n_p)
    v = np.full(n_p, math.sqrt(2.0 * e_b * E_CHARGE / M_PROTON))
    return {1: (x, v)}
