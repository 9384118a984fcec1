"""ctypes binding of the CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY.  Imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark; never by the product path (the GPU package
does not import this module, and this module does not import the GPU binding).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
MAX_MESH = 8
STRICT, WEAK, WEAK_EXT = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile oracle.c and mlp.c with gcc (plain -O2, no FMA contraction, no fast-math)."""
    if force or not os.path.exists(LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-Wall", "-o", LIB_PATH + ".tmp", os.path.join(HERE, "oracle.c"),
               os.path.join(HERE, "mlp.c"), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


Mat = (C.c_double * MAX_MESH) * MAX_MESH


class OrParams(C.Structure):
    _fields_ = [
        ("n_cells", C.c_int32),
        ("d", C.c_double), ("area", C.c_double), ("eps0", C.c_double), ("dt", C.c_double),
        ("Z", C.c_int32 * 2),
        ("mass", C.c_double * 2),
        ("q_unit", C.c_double), ("weight", C.c_double),
        ("ev", C.c_double),
        ("n_mesh", C.c_int32), ("gap_mesh", C.c_int32),
        ("L", Mat), ("R", Mat), ("S", Mat),
        ("src", C.c_double * MAX_MESH),
        ("src_dc", C.c_double), ("src_amp", C.c_double), ("src_freq", C.c_double),
        ("src_phase", C.c_double),
        ("c_par", C.c_double),
        ("q0", C.c_double * MAX_MESH),
        ("see_amp", C.c_double), ("see_E0_eV", C.c_double),
        ("see_law", C.c_int32), ("see_max", C.c_int32),
        ("see_E_eV", C.c_double),
        ("see_yield", C.c_int32), ("see_poly", C.c_double * 6), ("see_poly_Emax_eV", C.c_double),
        ("see_ln_mu", C.c_double), ("see_ln_sigma", C.c_double),
        ("beam_per_step", C.c_int64),
        ("beam_Emin_eV", C.c_double), ("beam_Emax_eV", C.c_double),
        ("beam_side", C.c_int32), ("beam_layer", C.c_double),
        ("beam_schedule", C.POINTER(C.c_int64)), ("beam_schedule_len", C.c_int64),
        ("seed", C.c_uint64),
        ("fp32", C.c_int32),
    ]


class OrDiag(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("t", C.c_double), ("phi0", C.c_double), ("sigma", C.c_double),
        ("qcirc", C.c_double), ("qcirc_star", C.c_double), ("qconv", C.c_double),
        ("e_ground", C.c_double),
        ("q", C.c_double * MAX_MESH), ("I", C.c_double * MAX_MESH),
        ("n_live", C.c_int64 * 2),
        ("abs_step", (C.c_int64 * 2) * 2), ("emit_step", C.c_int64 * 2), ("inj_step", C.c_int64),
        ("abs_cum", (C.c_int64 * 2) * 2), ("emit_cum", C.c_int64 * 2), ("inj_cum", C.c_int64),
        ("pushed_cum", C.c_int64), ("qcirc_step", C.c_double), ("q_space", C.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        P, D = C.POINTER(C.c_double), C.POINTER(C.c_uint64)
        L.or_philox4x64.argtypes = [D, D, D]
        L.or_poisson_draw.argtypes = [C.c_double, C.c_double, C.c_int32]
        L.or_poisson_draw.restype = C.c_int32
        L.or_create.argtypes = [C.POINTER(OrParams)]
        L.or_create.restype = C.c_void_p
        L.or_destroy.argtypes = [C.c_void_p]
        L.or_inject.argtypes = [C.c_void_p, C.c_int32, C.c_int64, P, P]
        L.or_inject.restype = C.c_int32
        L.or_step.argtypes = [C.c_void_p, C.c_int32]
        L.or_step.restype = C.c_int32
        L.or_get_diag.argtypes = [C.c_void_p, C.POINTER(OrDiag)]
        L.or_step_external.argtypes = [C.c_void_p, C.c_double]
        L.or_step_external.restype = C.c_int32
        L.or_phi0_prev.argtypes = [C.c_void_p]
        L.or_phi0_prev.restype = C.c_double
        L.or_get_fields.argtypes = [C.c_void_p, P, P, P]
        L.or_count.argtypes = [C.c_void_p, C.c_int32]
        L.or_count.restype = C.c_int64
        L.or_get_particles.argtypes = [C.c_void_p, C.c_int32, P, P, C.POINTER(C.c_uint32)]
        L.or_get_particles.restype = C.c_int64
        L.or_get_particles_f32.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_float),
                                           C.POINTER(C.c_float), C.POINTER(C.c_uint32)]
        L.or_get_particles_f32.restype = C.c_int64
        L.or_poisson_gauss.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_double, P, P]
        L.or_gather64.argtypes = [C.c_int32, C.c_double, P, C.c_double, C.c_double, C.c_double]
        L.or_gather64.restype = C.c_double
        L.or_gather32.argtypes = [C.c_int32, C.POINTER(C.c_float), C.c_float]
        L.or_gather32.restype = C.c_float
        L.or_push32.argtypes = [C.c_int32, C.POINTER(C.c_float), C.c_float, C.c_float, C.c_float,
                                C.POINTER(C.c_float), C.POINTER(C.c_float)]
        L.or_push32.restype = C.c_int32
        L.or_deposit32.argtypes = [C.c_int32, C.c_int32, C.POINTER(C.c_float), C.c_int64, C.POINTER(C.c_int64)]
        L.or_alpha32.argtypes = [C.c_void_p, C.c_int32]
        L.or_alpha32.restype = C.c_float
        L.or_beam_ion32.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.POINTER(C.c_float), C.POINTER(C.c_float)]
        L.or_emit_sample.argtypes = [C.c_void_p, C.c_int64, C.c_uint32, C.c_double, C.c_int32,
                                     C.POINTER(C.c_float), C.POINTER(C.c_float), C.c_int32]
        L.or_emit_sample.restype = C.c_int32
        L.or_circuit_run.argtypes = [C.POINTER(OrParams), C.c_int64, P, P]
        L.or_circuit_run.restype = C.c_int32
        L.or_gelu.argtypes = [C.c_double]
        L.or_gelu.restype = C.c_double
        L.or_gelu_grad.argtypes = [C.c_double]
        L.or_gelu_grad.restype = C.c_double
        L.or_mlp_forward.argtypes = [P, P, C.c_int64, P]
        L.or_mlp_loss_grad.argtypes = [P, P, P, C.c_int64, P]
        L.or_mlp_loss_grad.restype = C.c_double
        L.or_adam_step.argtypes = [P, P, P, C.c_int64, P, C.c_int64, C.c_double, C.c_double, C.c_double,
                                   C.c_double]
        L.or_round_bf16.argtypes = [C.c_float]
        L.or_round_bf16.restype = C.c_float
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def params_from(cfg, fp32: bool = False) -> OrParams:
    p = OrParams()
    p.n_cells = cfg.n_cells
    p.d, p.area, p.eps0, p.dt = cfg.d, cfg.area, cfg.eps0, cfg.dt
    p.Z[0], p.Z[1] = int(cfg.Z[0]), int(cfg.Z[1])
    p.mass[0], p.mass[1] = float(cfg.mass[0]), float(cfg.mass[1])
    p.q_unit, p.weight, p.ev = cfg.q_unit, cfg.weight, cfg.ev
    p.n_mesh, p.gap_mesh = cfg.n_mesh, cfg.gap_mesh
    for i in range(cfg.n_mesh):
        for j in range(cfg.n_mesh):
            p.L[i][j] = float(cfg.L[i, j])
            p.R[i][j] = float(cfg.R[i, j])
            p.S[i][j] = float(cfg.S[i, j])
        p.src[i] = float(cfg.src[i])
        p.q0[i] = float(cfg.q0[i])
    p.src_dc, p.src_amp, p.src_freq, p.src_phase = cfg.src_dc, cfg.src_amp, cfg.src_freq, cfg.src_phase
    p.c_par = cfg.c_par
    p.see_amp, p.see_E0_eV, p.see_law, p.see_max = cfg.see_amp, cfg.see_E0_eV, cfg.see_law, cfg.see_max
    p.see_E_eV = cfg.see_E_eV
    p.see_yield = int(cfg.see_yield)
    for j in range(6):
        p.see_poly[j] = float(cfg.see_poly[j])
    p.see_poly_Emax_eV, p.see_ln_mu, p.see_ln_sigma = cfg.see_poly_Emax_eV, cfg.see_ln_mu, cfg.see_ln_sigma
    p.beam_per_step = cfg.beam_per_step
    p.beam_Emin_eV, p.beam_Emax_eV = cfg.beam_Emin_eV, cfg.beam_Emax_eV
    p.beam_side, p.beam_layer = int(cfg.beam_side), float(cfg.beam_layer)
    if cfg.beam_schedule is not None:
        # the config owns this int64 array, so the pointer outlives the call
        p.beam_schedule = cfg.beam_schedule.ctypes.data_as(C.POINTER(C.c_int64))
        p.beam_schedule_len = int(cfg.beam_schedule.size)
    p.seed = cfg.seed
    p.fp32 = 1 if fp32 else 0
    return p


def philox4x64(ctr, key):
    c = np.asarray(ctr, dtype=np.uint64)
    k = np.asarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    D = C.POINTER(C.c_uint64)
    lib().or_philox4x64(c.ctypes.data_as(D), k.ctypes.data_as(D), out.ctypes.data_as(D))
    return out


def poisson_draw(lam: float, u: float, kmax: int = 32) -> int:
    return int(lib().or_poisson_draw(lam, u, kmax))


def poisson_gauss(rho: np.ndarray, dx: float, eps0: float, sigma: float) -> np.ndarray:
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    n_cells = rho.size - 1
    phi = np.zeros(n_cells + 1)
    lib().or_poisson_gauss(n_cells, dx, eps0, sigma, _dp(rho), _dp(phi))
    return phi


def gather64(E_half, dx, e0_surf, e_ground, x) -> np.ndarray:
    E_half = np.ascontiguousarray(E_half, dtype=np.float64)
    N = E_half.size
    return np.array([lib().or_gather64(N, dx, _dp(E_half), e0_surf, e_ground, float(v)) for v in x])


def gather32(ehat, xi) -> np.ndarray:
    ehat = np.ascontiguousarray(ehat, dtype=np.float32)
    N = ehat.size - 2
    F = C.POINTER(C.c_float)
    return np.array([lib().or_gather32(N, ehat.ctypes.data_as(F), float(v)) for v in xi],
                    dtype=np.float32)


def push32(ehat, alpha: float, xi: float, u: float):
    """One binary32 push in grid units: (xi', u', wall) with wall 0 inside, 1 at the
    circuit electrode, 2 at the ground."""
    ehat = np.ascontiguousarray(ehat, dtype=np.float32)
    xo, uo = C.c_float(), C.c_float()
    w = lib().or_push32(ehat.size - 2, ehat.ctypes.data_as(C.POINTER(C.c_float)), float(alpha), float(xi),
                        float(u), C.byref(xo), C.byref(uo))
    return np.float32(xo.value), np.float32(uo.value), int(w)


def deposit32(n_cells: int, Z: int, xi, acc=None) -> np.ndarray:
    """The binary32 deposit of positions xi (cells) with charge number Z, added to
    the int64 node accumulator acc (units of 2^-24 of a macroparticle); returns it."""
    xi = np.ascontiguousarray(xi, dtype=np.float32)
    if acc is None:
        acc = np.zeros(n_cells + 1, dtype=np.int64)
    assert acc.dtype == np.int64 and acc.size == n_cells + 1 and acc.flags["C_CONTIGUOUS"]
    lib().or_deposit32(n_cells, Z, xi.ctypes.data_as(C.POINTER(C.c_float)), xi.size,
                       acc.ctypes.data_as(C.POINTER(C.c_int64)))
    return acc


def circuit_run(cfg, nsteps: int):
    p = params_from(cfg)
    q = np.zeros(nsteps * cfg.n_mesh)
    v = np.zeros(nsteps)
    rc = lib().or_circuit_run(C.byref(p), nsteps, _dp(q), _dp(v))
    if rc:
        raise RuntimeError(f"or_circuit_run failed: {rc}")
    return q.reshape(nsteps, cfg.n_mesh), v


# ---------------------------------------------------------------------------
# guess network (mlp.c)
# ---------------------------------------------------------------------------
MLP_IN, MLP_HIDDEN, MLP_OUT = 48, 128, 3
MLP_NPARAM = 39683
# (name, offset, shape) of each parameter block in the flat vector
MLP_LAYOUT = []
_o = 0
for _name, _shape in (("W1", (128, 48)), ("b1", (128,)), ("W2", (128, 128)), ("b2", (128,)),
                      ("W3", (128, 128)), ("b3", (128,)), ("W4", (3, 128)), ("b4", (3,))):
    MLP_LAYOUT.append((_name, _o, _shape))
    _o += int(np.prod(_shape))
assert _o == MLP_NPARAM


def gelu(z: float) -> float:
    return float(lib().or_gelu(float(z)))


def gelu_grad(z: float) -> float:
    return float(lib().or_gelu_grad(float(z)))


def mlp_forward(theta, x) -> np.ndarray:
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, MLP_IN)
    y = np.zeros((x.shape[0], MLP_OUT))
    lib().or_mlp_forward(_dp(theta), _dp(x), x.shape[0], _dp(y))
    return y


def mlp_loss_grad(theta, x, t):
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, MLP_IN)
    t = np.ascontiguousarray(t, dtype=np.float64).reshape(-1, MLP_OUT)
    g = np.zeros(MLP_NPARAM)
    loss = lib().or_mlp_loss_grad(_dp(theta), _dp(x), _dp(t), x.shape[0], _dp(g))
    return float(loss), g


def adam_step(theta, m, v, t: int, g, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """In place on float64 arrays theta, m, v."""
    for a in (theta, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = np.ascontiguousarray(g, dtype=np.float64)
    lib().or_adam_step(_dp(theta), _dp(m), _dp(v), int(t), _dp(g), theta.size, lr, beta1, beta2, eps)


def round_bf16(a) -> np.ndarray:
    a = np.asarray(a, dtype=np.float32)
    f = lib().or_round_bf16
    return np.array([f(float(v)) for v in a.ravel()], dtype=np.float32).reshape(a.shape)


def circuit_resonance(cfg) -> float:
    """Highest ringing angular frequency of a gap's circuit (App. D,
    circuit-resolution constraint): the largest |Im lambda| over the finite roots
    of det(lambda^2 L + lambda R + S') = 0, S' = S plus 1 / (C_gap + c_par) in the
    gap mesh.  With lambda = w0 mu, w0 = sqrt(|S'| / |L|) (largest entries), and
    the matrices divided by |S'|, the scaled roots mu are the finite generalized
    eigenvalues of the first-order pencil A z = mu B z, z = (q, q'),
    A = [[0, I], [-S~, -R~]], B = [[I, 0], [0, L~]] (LAPACK's QZ through scipy);
    an eigenvalue whose beta is below 1e-12 of its alpha is infinite.  0 when
    no root oscillates."""
    import scipy.linalg as sl
    M, g = cfg.n_mesh, cfg.gap_mesh
    S = np.array(cfg.S, dtype=np.float64).copy()
    S[g, g] += 1.0 / (cfg.eps0 * cfg.area / cfg.d + cfg.c_par)
    L = np.asarray(cfg.L, dtype=np.float64)
    R = np.asarray(cfg.R, dtype=np.float64)
    if np.abs(L).max() == 0.0:
        return 0.0
    s = np.abs(S).max()
    w0 = math.sqrt(s / np.abs(L).max())
    Z, I = np.zeros((M, M)), np.eye(M)
    A = np.block([[Z, I], [-S / s, -R * (w0 / s)]])
    B = np.block([[I, Z], [Z, L * (w0 * w0 / s)]])
    (a, b), _ = sl.eig(A, B, homogeneous_eigvals=True)
    fin = np.abs(b) > 1e-12 * np.abs(a)
    lam = w0 * (a[fin] / b[fin])
    return float(np.abs(lam.imag).max()) if lam.size else 0.0


class OracleSim:
    """One gap advanced by the oracle."""

    def __init__(self, cfg, fp32: bool = False):
        self.cfg = cfg
        self.fp32 = fp32
        self._p = params_from(cfg, fp32)
        self._h = lib().or_create(C.byref(self._p))
        self._stepped = False
        if not self._h:
            raise ValueError("oracle rejected the parameters")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().or_destroy(h)
            self._h = None

    def inject(self, species: int, x, v):
        x = np.ascontiguousarray(x, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        rc = lib().or_inject(self._h, species, x.size, _dp(x), _dp(v))
        if rc:
            raise ValueError(f"or_inject failed: {rc}")

    def step(self, mode: int = STRICT, n: int = 1):
        for _ in range(n):
            rc = lib().or_step(self._h, mode)
            if rc:
                raise RuntimeError(f"or_step failed: {rc}")
            self._stepped = True

    def diag(self) -> dict:
        D = OrDiag()
        lib().or_get_diag(self._h, C.byref(D))
        M = self.cfg.n_mesh
        return dict(step=D.step, t=D.t, phi0=D.phi0, sigma=D.sigma, qcirc=D.qcirc,
                    qcirc_star=D.qcirc_star, qconv=D.qconv,
                    e_ground=D.e_ground, q=np.array(D.q[:M]), I=np.array(D.I[:M]),
                    n_live=np.array(D.n_live[:]),
                    abs_step=np.array([[D.abs_step[a][b] for b in range(2)] for a in range(2)]),
                    emit_step=np.array(D.emit_step[:]), inj_step=D.inj_step,
                    abs_cum=np.array([[D.abs_cum[a][b] for b in range(2)] for a in range(2)]),
                    emit_cum=np.array(D.emit_cum[:]), inj_cum=D.inj_cum,
                    pushed_cum=D.pushed_cum, qcirc_step=D.qcirc_step, q_space=D.q_space)

    def alpha32(self, species: int) -> np.float32:
        return np.float32(lib().or_alpha32(self._h, species))

    def beam_ion32(self, step: int, k: int):
        """Beam ion k of the step that solves level `step`, in grid units."""
        xi, u = C.c_float(), C.c_float()
        lib().or_beam_ion32(self._h, step, k, C.byref(xi), C.byref(u))
        return np.float32(xi.value), np.float32(u.value)

    def emit_sample(self, step: int, ion_id: int, v_ion: float, wall: int):
        """The secondary electrons of one absorbed ion (wall 0 circuit, 1 ground) in the
        push after level `step`: (xi, u) arrays in grid units."""
        xi, u = np.zeros(1024, dtype=np.float32), np.zeros(1024, dtype=np.float32)
        F = C.POINTER(C.c_float)
        k = lib().or_emit_sample(self._h, step, int(ion_id), float(v_ion), wall, xi.ctypes.data_as(F),
                                 u.ctypes.data_as(F), 1024)
        return xi[:min(k, 1024)], u[:min(k, 1024)]

    def phi0_prev(self) -> float:
        return float(lib().or_phi0_prev(self._h))

    def step_external(self, engine, n: int = 1, gap: int = 0):
        """Weak steps with an external circuit engine (Alg. 1 coupled as in Sec. 2.4.3):
        engine(gap, level, dt, phi0_prev) returns the gap voltage V* its circuit reaches
        at that level after restarting the gap capacitor from phi0_prev."""
        for _ in range(n):
            level = self.diag()["step"] + 1 if self._stepped else 0
            v = float(engine(gap, level, self.cfg.dt, self.phi0_prev()))
            rc = lib().or_step_external(self._h, v)
            if rc:
                raise RuntimeError(f"or_step_external failed: {rc}")
            self._stepped = True

    def dt_report(self) -> dict:
        """The time-step constraints of App. D at the last completed level, from the
        oracle's own state: circuit_resonance below, the largest |v_x| dt / dx per
        species, the most live electrons in one cell (count * weight / dx), the plasma
        frequency that density gives, and the relative change of the circuit charge
        over the last step."""
        cfg = self.cfg
        dx = cfg.d / cfg.n_cells
        beta = np.zeros(2)
        cells = np.zeros(cfg.n_cells, dtype=np.int64)
        for sp in range(2):
            if self.fp32:
                xi, u, _ = self.particles_f32(sp)
                xi = xi.astype(np.float64)
                u = u.astype(np.float64)
            else:
                x, v, _ = self.particles(sp)
                xi, u = x / dx, v * cfg.dt / dx
            if u.size:
                beta[sp] = np.abs(u).max()
            if sp == 0 and xi.size:
                np.add.at(cells, np.minimum(np.floor(xi).astype(np.int64), cfg.n_cells - 1), 1)
        w = circuit_resonance(cfg)
        n_e = cells.max() * cfg.weight / dx
        qe = cfg.q_unit * abs(cfg.Z[0])
        w_pe = np.sqrt(n_e * qe * qe / (cfg.eps0 * cfg.mass[0]))
        D = self.diag()
        q_prev = D["qcirc_star"] - D["qcirc_step"]
        q_ref = max(abs(D["qcirc_star"]), abs(q_prev))
        eta = abs(D["qcirc_step"]) / q_ref if q_ref > 0 else 0.0
        n_omega = 1.0 / (w * cfg.dt) if w > 0 else np.inf
        alpha = w_pe * cfg.dt
        flags = ((n_omega < 20) * 1) | ((beta.max() > 0.5) * 2) | ((alpha > 0.2) * 4) | ((eta > 0.2) * 8)
        return dict(dt=cfg.dt, omega_max=w, n_omega=n_omega, beta=beta, v_max=beta * dx / cfg.dt,
                    n_e_max=n_e, omega_pe=w_pe, alpha=alpha, eta=eta, flags=int(flags))

    def fields(self):
        N = self.cfg.n_cells
        phi, E, rho = np.zeros(N + 1), np.zeros(N), np.zeros(N + 1)
        lib().or_get_fields(self._h, _dp(phi), _dp(E), _dp(rho))
        return phi, E, rho

    def count(self, species: int) -> int:
        return int(lib().or_count(self._h, species))

    def particles(self, species: int):
        n = self.count(species)
        x, v = np.zeros(n), np.zeros(n)
        ids = np.zeros(n, dtype=np.uint32)
        lib().or_get_particles(self._h, species, _dp(x), _dp(v),
                               ids.ctypes.data_as(C.POINTER(C.c_uint32)))
        return x, v, ids

    def particles_f32(self, species: int):
        n = self.count(species)
        xi, u = np.zeros(n, dtype=np.float32), np.zeros(n, dtype=np.float32)
        ids = np.zeros(n, dtype=np.uint32)
        F = C.POINTER(C.c_float)
        rc = lib().or_get_particles_f32(self._h, species, xi.ctypes.data_as(F), u.ctypes.data_as(F),
                                        ids.ctypes.data_as(C.POINTER(C.c_uint32)))
        if rc < 0:
            raise RuntimeError("not an fp32 oracle")
        return xi, u, ids
