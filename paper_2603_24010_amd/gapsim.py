"""Thin ctypes binding of libgapsim.so (the C ABI in include/gapsim.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch supplies device memory (its caching allocator, through the
library's allocator hook) and the stream.  There is no CPU fallback: if the
library is missing or no GPU is present, construction fails loudly.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref
from typing import Iterable, List, Optional, Sequence, Union

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgapsim.so")
MAX_MESH = 8

GS_OK, GS_EINVAL, GS_ENOMEM, GS_ECAPACITY, GS_EDEVICE, GS_ENOCONV, GS_ESTATE = 0, -1, -2, -3, -4, -5, -6
GS_ECALLBACK = -7
GUESS_DIRECT, GUESS_EXTRAP, GUESS_MLP = 0, 1, 2
OPT_BLOCK, OPT_TILE, OPT_GRID, OPT_COMPACT_EVERY, OPT_GRAPH, OPT_TIMING = 1, 2, 3, 4, 5, 6
OPT_NEWTON_TOL, OPT_NEWTON_MAXIT, OPT_DEPOSIT, OPT_COMPACT_GRID, OPT_PPT = 7, 8, 9, 10, 11
OPT_SORT_BIN = 12
OPT_STEAL = 13
OPT_STREAM = 14

EXPORTED = [
    "gs_init_gap", "gs_destroy", "gs_inject", "gs_step_strict", "gs_step_weak", "gs_read_diagnostics",
    "gs_read_particles", "gs_set_option", "gs_get_timing", "gs_validate_params", "gs_last_error",
    "gs_version", "gs_mlp_set_weights", "gs_mlp_forward", "gs_mlp_record", "gs_mlp_train_workspace",
    "gs_mlp_train", "gs_autotune", "gs_step_weak_external", "gs_circuit_resonance", "gs_dt_check",
    "gs_get_launch", "gs_inject_noalloc",
]
MLP_IN, MLP_OUT, MLP_NPARAM, MLP_NORM = 48, 3, 39683, 102

Mat = (C.c_double * MAX_MESH) * MAX_MESH


class GsGapParams(C.Structure):
    _fields_ = [
        ("n_cells", C.c_int32),
        ("d", C.c_double), ("area", C.c_double), ("eps0", C.c_double), ("dt", C.c_double),
        ("Z", C.c_int32 * 2),
        ("mass", C.c_double * 2),
        ("q_unit", C.c_double), ("weight", C.c_double), ("ev", C.c_double),
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
        ("particle_fp", C.c_int32),
        ("capacity", C.c_int64 * 2),
        ("v_ref", C.c_double),
    ]


class GsDiag(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("t", C.c_double), ("phi0", C.c_double), ("sigma", C.c_double),
        ("qcirc", C.c_double), ("qcirc_star", C.c_double), ("qconv", C.c_double),
        ("e_ground", C.c_double),
        ("q", C.c_double * MAX_MESH), ("I", C.c_double * MAX_MESH),
        ("n_live", C.c_int64 * 2), ("n_slots", C.c_int64 * 2),
        ("abs_step", (C.c_int64 * 2) * 2), ("emit_step", C.c_int64 * 2), ("inj_step", C.c_int64),
        ("abs_cum", (C.c_int64 * 2) * 2), ("emit_cum", C.c_int64 * 2), ("inj_cum", C.c_int64),
        ("pushed_cum", C.c_int64),
        ("newton_last", C.c_int32), ("newton_fallback_last", C.c_int32),
        ("newton_total", C.c_int64), ("newton_fallbacks", C.c_int64),
        ("newton_max", C.c_int32), ("newton_levels", C.c_int32),
        ("newton_resid0", C.c_double), ("newton_resid", C.c_double),
        ("newton_guess", C.c_double * (MAX_MESH + 1)),
        ("mlp_proposal", C.c_double * 3),
        ("qcirc_step", C.c_double),
        ("q_space", C.c_double),
    ]


class GsTiming(C.Structure):
    _fields_ = [
        ("push_ms", C.c_double), ("field_ms", C.c_double), ("compact_ms", C.c_double),
        ("push_launches", C.c_int64), ("field_launches", C.c_int64), ("compact_launches", C.c_int64),
        ("emit_ms", C.c_double), ("emit_launches", C.c_int64),
    ]


class GsTuning(C.Structure):
    _fields_ = [("block", C.c_int32), ("tile", C.c_int32), ("grid", C.c_int32), ("ppt", C.c_int32),
                ("deposit", C.c_int32), ("compact_every", C.c_int32), ("sort_bin", C.c_int32),
                ("steal", C.c_int32), ("stream", C.c_int32), ("ms_per_step", C.c_double)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


# gs_circuit_fn: (user, gap, level, dt, phi0_prev, v_gap out) -> status
CIRCUIT_FN = C.CFUNCTYPE(C.c_int32, C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_double,
                         C.POINTER(C.c_double))


class GsDtReport(C.Structure):
    _fields_ = [("dt", C.c_double), ("omega_max", C.c_double), ("n_omega", C.c_double),
                ("v_max", C.c_double * 2), ("beta", C.c_double * 2), ("n_e_max", C.c_double),
                ("omega_pe", C.c_double), ("alpha", C.c_double), ("eta", C.c_double),
                ("flags", C.c_int32)]


class GsAllocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("release", RELEASE_FN), ("user", C.c_void_p)]


_lib = None


def lib():
    """Load libgapsim.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2603_24010_amd/build.py")
        # torch carries its own HIP runtime beside the system one the library
        # links: torch's must have found the GPU before the library is loaded,
        # or the library's runtime finds none (no effect on a machine without one)
        import torch
        torch.cuda.is_available()
        L = C.CDLL(LIB_PATH)
        vp, P = C.c_void_p, C.POINTER(C.c_double)
        L.gs_init_gap.argtypes = [C.POINTER(vp), C.c_int32, C.POINTER(GsGapParams), C.POINTER(GsAllocator), vp]
        L.gs_init_gap.restype = C.c_int
        L.gs_destroy.argtypes = [vp]
        L.gs_inject.argtypes = [vp, C.c_int32, C.c_int32, C.c_int64, vp, vp, C.c_int32]
        L.gs_inject.restype = C.c_int
        L.gs_step_strict.argtypes = [vp, C.c_int32, C.c_int32]
        L.gs_step_strict.restype = C.c_int
        L.gs_step_weak.argtypes = [vp, C.c_int32]
        L.gs_step_weak.restype = C.c_int
        L.gs_read_diagnostics.argtypes = [vp, C.c_int32, C.POINTER(GsDiag), P, P, P]
        L.gs_read_diagnostics.restype = C.c_int
        L.gs_read_particles.argtypes = [vp, C.c_int32, C.c_int32, vp, vp, C.POINTER(C.c_uint32),
                                        C.c_int64, C.POINTER(C.c_int64)]
        L.gs_read_particles.restype = C.c_int
        L.gs_set_option.argtypes = [vp, C.c_int32, C.c_int64]
        L.gs_set_option.restype = C.c_int
        L.gs_get_timing.argtypes = [vp, C.POINTER(GsTiming), C.c_int32]
        L.gs_get_timing.restype = C.c_int
        L.gs_validate_params.argtypes = [C.POINTER(GsGapParams), C.c_char_p, C.c_size_t]
        L.gs_validate_params.restype = C.c_int
        L.gs_last_error.argtypes = [vp]
        L.gs_last_error.restype = C.c_char_p
        L.gs_version.restype = C.c_char_p
        L.gs_mlp_set_weights.argtypes = [vp, C.POINTER(C.c_float), C.c_int64, P]
        L.gs_mlp_set_weights.restype = C.c_int
        L.gs_mlp_forward.argtypes = [vp, vp, C.c_int64, vp]
        L.gs_mlp_forward.restype = C.c_int
        L.gs_mlp_record.argtypes = [vp, vp, vp, C.c_int64]
        L.gs_mlp_record.restype = C.c_int
        L.gs_mlp_train_workspace.argtypes = [C.c_int32]
        L.gs_mlp_train_workspace.restype = C.c_size_t
        L.gs_mlp_train.argtypes = [vp, vp, C.c_int64, vp, C.c_int64, C.c_int32, vp, vp, vp, C.c_int64,
                                   C.c_double, C.c_double, C.c_double, C.c_double, vp, vp, vp, C.c_size_t,
                                   vp]
        L.gs_mlp_train.restype = C.c_int
        L.gs_autotune.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.c_char_p, C.POINTER(GsTuning)]
        L.gs_autotune.restype = C.c_int
        L.gs_inject_noalloc.argtypes = [vp, C.c_int32, C.c_int32, C.c_int64, vp, vp]
        L.gs_inject_noalloc.restype = C.c_int
        L.gs_get_launch.argtypes = [vp, C.POINTER(GsTuning)]
        L.gs_get_launch.restype = C.c_int
        L.gs_step_weak_external.argtypes = [vp, C.c_int32, CIRCUIT_FN, vp]
        L.gs_step_weak_external.restype = C.c_int
        L.gs_circuit_resonance.argtypes = [C.POINTER(GsGapParams), P]
        L.gs_circuit_resonance.restype = C.c_int
        L.gs_dt_check.argtypes = [vp, C.c_int32, C.POINTER(GsDtReport)]
        L.gs_dt_check.restype = C.c_int
        _lib = L
    return _lib


def _tuning_dict(t) -> dict:
    return dict(block=t.block, tile=t.tile, grid=t.grid, ppt=t.ppt, deposit=t.deposit,
                compact_every=t.compact_every, sort_bin=t.sort_bin, steal=t.steal, stream=t.stream,
                ms_per_step=t.ms_per_step)


class GapsimError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"gapsim status {status}: {msg}")
        self.status = status


def params_from(cfg, particle_fp: int = 32, capacity=(1 << 20, 1 << 20)) -> GsGapParams:
    p = GsGapParams()
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
    p.particle_fp = particle_fp
    p.capacity[0], p.capacity[1] = int(capacity[0]), int(capacity[1])
    p.v_ref = cfg.v_ref
    return p


def validate(cfg, particle_fp: int = 32, capacity=(1 << 20, 1 << 20)) -> Optional[str]:
    """Host-only parameter check; returns None if valid, else the message."""
    p = params_from(cfg, particle_fp, capacity)
    buf = C.create_string_buffer(256)
    rc = lib().gs_validate_params(C.byref(p), buf, 256)
    return None if rc == GS_OK else buf.value.decode()


def circuit_resonance(cfg) -> float:
    """Highest ringing angular frequency of the gap's circuit [rad/s] (host only)."""
    p = params_from(cfg, 32, (1, 1))
    w = C.c_double()
    rc = lib().gs_circuit_resonance(C.byref(p), C.byref(w))
    if rc != GS_OK:
        raise GapsimError(rc, "gs_circuit_resonance failed")
    return w.value


_live = weakref.WeakSet()


@atexit.register
def _close_all():
    # release device memory while torch is still importable
    for sim in list(_live):
        try:
            sim.close()
        except Exception:
            pass


class GapSim:
    """Gaps advanced together on one GPU stream."""

    def __init__(self, cfgs, particle_fp: int = 32, capacity=(1 << 20, 1 << 20),
                 stream=None, torch_alloc: bool = True):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("gapsim needs a ROCm GPU; none is visible")
        if not isinstance(cfgs, (list, tuple)):
            cfgs = [cfgs]
        self.cfgs = list(cfgs)
        self.G = len(cfgs)
        self.fp64 = particle_fp == 64
        caps = capacity if (isinstance(capacity, (list, tuple)) and len(capacity) == self.G
                            and isinstance(capacity[0], (list, tuple))) else [capacity] * self.G
        arr = (GsGapParams * self.G)()
        for g, cfg in enumerate(cfgs):
            arr[g] = params_from(cfg, particle_fp, caps[g])
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._alloc = None
        alloc_p = None
        if torch_alloc:
            dev_index = self.device.index
            stream_handle = self.stream
            # bound now: at interpreter exit the torch module may already be gone
            alloc_fn = torch.cuda.caching_allocator_alloc
            delete_fn = torch.cuda.caching_allocator_delete

            def _a(nbytes, user):
                try:
                    return alloc_fn(int(nbytes), dev_index, stream_handle)
                except Exception:
                    return None

            def _r(ptr, user):
                try:
                    delete_fn(ptr)
                except Exception:
                    pass

            self._alloc = GsAllocator(ALLOC_FN(_a), RELEASE_FN(_r), None)
            alloc_p = C.byref(self._alloc)
        h = C.c_void_p()
        rc = lib().gs_init_gap(C.byref(h), self.G, arr, alloc_p, C.c_void_p(self.stream.cuda_stream))
        if rc != GS_OK:
            raise GapsimError(rc, lib().gs_last_error(None).decode())
        self._h = h
        _live.add(self)

    # -- helpers ----------------------------------------------------------
    def _chk(self, rc: int):
        if rc != GS_OK:
            raise GapsimError(rc, lib().gs_last_error(self._h).decode())

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().gs_destroy(h)
        self._h = None
        _live.discard(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the C ABI ----------------------------------------------------------
    def inject(self, gap: int, species: int, x, v):
        try:
            import torch
            is_dev = isinstance(x, torch.Tensor) and x.is_cuda
        except ImportError:  # pragma: no cover
            is_dev = False
        if is_dev:
            x = x.contiguous().to(dtype=torch.float64)
            v = v.contiguous().to(dtype=torch.float64)
            self._chk(lib().gs_inject(self._h, gap, species, x.numel(), C.c_void_p(x.data_ptr()),
                                      C.c_void_p(v.data_ptr()), 1))
        else:
            x = np.ascontiguousarray(x, dtype=np.float64)
            v = np.ascontiguousarray(v, dtype=np.float64)
            self._chk(lib().gs_inject(self._h, gap, species, x.size, x.ctypes.data_as(C.c_void_p),
                                      v.ctypes.data_as(C.c_void_p), 0))

    def step_strict(self, n: int = 1, guess: int = GUESS_DIRECT):
        self._chk(lib().gs_step_strict(self._h, n, guess))

    def step_weak(self, n: int = 1):
        self._chk(lib().gs_step_weak(self._h, n))

    def step_weak_external(self, n: int, engine):
        """Weak steps with an external circuit engine: engine(gap, level, dt, phi0_prev)
        returns the gap voltage its circuit reaches at that level.  An exception in the
        engine stops the call before that step's device work and is raised again here."""
        caught = []

        def _fn(user, gap, level, dt, phi0_prev, v_out):
            try:
                v_out[0] = float(engine(int(gap), int(level), float(dt), float(phi0_prev)))
                return 0
            except BaseException as e:  # noqa: BLE001 - handed back after the C call
                caught.append(e)
                return 1

        cb = CIRCUIT_FN(_fn)
        rc = lib().gs_step_weak_external(self._h, n, cb, None)
        if caught:
            raise caught[0]
        self._chk(rc)

    def dt_check(self, gap: int = 0) -> dict:
        """The time-step constraints of App. D at the last completed step."""
        R = GsDtReport()
        self._chk(lib().gs_dt_check(self._h, gap, C.byref(R)))
        return dict(dt=R.dt, omega_max=R.omega_max, n_omega=R.n_omega, v_max=np.array(R.v_max[:]),
                    beta=np.array(R.beta[:]), n_e_max=R.n_e_max, omega_pe=R.omega_pe, alpha=R.alpha,
                    eta=R.eta, flags=R.flags)

    def step(self, mode: int, n: int = 1, guess: int = GUESS_DIRECT):
        """mode 0 = strict, 1 = weak (the oracle's numbering)."""
        if mode == 0:
            self.step_strict(n, guess)
        else:
            self.step_weak(n)

    def set_option(self, option: int, value: int):
        self._chk(lib().gs_set_option(self._h, option, int(value)))

    def diag(self, gap: int = 0) -> dict:
        D = GsDiag()
        rc = lib().gs_read_diagnostics(self._h, gap, C.byref(D), None, None, None)
        # a missed Newton tolerance is reported once with the outputs filled
        converged = rc != GS_ENOCONV
        if converged:
            self._chk(rc)
        M = self.cfgs[gap].n_mesh
        return dict(step=D.step, t=D.t, phi0=D.phi0, sigma=D.sigma, qcirc=D.qcirc,
                    qcirc_star=D.qcirc_star, qconv=D.qconv, e_ground=D.e_ground,
                    q=np.array(D.q[:M]), I=np.array(D.I[:M]),
                    n_live=np.array(D.n_live[:]), n_slots=np.array(D.n_slots[:]),
                    abs_step=np.array([[D.abs_step[a][b] for b in range(2)] for a in range(2)]),
                    emit_step=np.array(D.emit_step[:]), inj_step=D.inj_step,
                    abs_cum=np.array([[D.abs_cum[a][b] for b in range(2)] for a in range(2)]),
                    emit_cum=np.array(D.emit_cum[:]), inj_cum=D.inj_cum, pushed_cum=D.pushed_cum,
                    newton_converged=converged,
                    newton_last=D.newton_last, newton_fallback_last=D.newton_fallback_last,
                    newton_total=D.newton_total, newton_fallbacks=D.newton_fallbacks,
                    newton_max=D.newton_max, newton_levels=D.newton_levels,
                    newton_resid0=D.newton_resid0, newton_resid=D.newton_resid,
                    newton_guess=np.array(D.newton_guess[:M + 1]),
                    mlp_proposal=np.array(D.mlp_proposal[:]), qcirc_step=D.qcirc_step, q_space=D.q_space)

    def autotune(self, mode: int, guess: int = GUESS_DIRECT, trial_steps: int = 8,
                 cache_path: Optional[str] = None) -> dict:
        """gs_autotune: pick launch shape and compaction interval on the current
        state (which it leaves unchanged); returns the choice."""
        t = GsTuning()
        self._chk(lib().gs_autotune(self._h, mode, guess, trial_steps,
                                    cache_path.encode() if cache_path else None, C.byref(t)))
        return _tuning_dict(t)

    def launch(self) -> dict:
        """gs_get_launch: the launch configuration in effect."""
        t = GsTuning()
        self._chk(lib().gs_get_launch(self._h, C.byref(t)))
        d = _tuning_dict(t)
        del d["ms_per_step"]
        return d

    # -- Newton guess network -------------------------------------------------
    def mlp_set_weights(self, theta, norm):
        theta = np.ascontiguousarray(theta, dtype=np.float32)
        norm = np.ascontiguousarray(norm, dtype=np.float64)
        if norm.size != MLP_NORM:
            raise ValueError(f"norm must hold {MLP_NORM} values")
        self._chk(lib().gs_mlp_set_weights(self._h, theta.ctypes.data_as(C.POINTER(C.c_float)), theta.size,
                                           norm.ctypes.data_as(C.POINTER(C.c_double))))

    def mlp_forward(self, x):
        """x: float32 device tensor [n, 48] (normalised); returns [n, 3]."""
        import torch
        x = x.contiguous()
        assert x.is_cuda and x.dtype == torch.float32 and x.shape[-1] == MLP_IN
        y = torch.empty((x.shape[0], MLP_OUT), dtype=torch.float32, device=x.device)
        self._chk(lib().gs_mlp_forward(self._h, C.c_void_p(x.data_ptr()), x.shape[0],
                                       C.c_void_p(y.data_ptr())))
        return y

    def mlp_record(self, x=None, y=None):
        """Record (raw input, raw target) samples of the following strict steps
        into float32 device tensors x [cap, 48], y [cap, 3]; no arguments stop it."""
        if x is None or y is None:
            self._rec = None
            self._chk(lib().gs_mlp_record(self._h, None, None, 0))
            return
        assert x.is_cuda and y.is_cuda and x.is_contiguous() and y.is_contiguous()
        assert x.shape[1] == MLP_IN and y.shape[1] == MLP_OUT and x.shape[0] == y.shape[0]
        self._rec = (x, y)  # keep the buffers alive while the library writes them
        self._chk(lib().gs_mlp_record(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                      x.shape[0]))

    def fields(self, gap: int = 0):
        N = self.cfgs[gap].n_cells
        phi, E, rho = np.zeros(N + 1), np.zeros(N), np.zeros(N + 1)
        D = GsDiag()
        P = C.POINTER(C.c_double)
        self._chk(lib().gs_read_diagnostics(self._h, gap, C.byref(D), phi.ctypes.data_as(P),
                                            E.ctypes.data_as(P), rho.ctypes.data_as(P)))
        return phi, E, rho

    def particles(self, gap: int, species: int):
        """Live particles in grid units (xi = x/dx, u = v dt/dx) and ids."""
        n = C.c_int64(0)
        self._chk(lib().gs_read_particles(self._h, gap, species, None, None, None, 0, C.byref(n)))
        dt = np.float64 if self.fp64 else np.float32
        xi, u = np.zeros(n.value, dtype=dt), np.zeros(n.value, dtype=dt)
        ids = np.zeros(n.value, dtype=np.uint32)
        m = C.c_int64(0)
        self._chk(lib().gs_read_particles(self._h, gap, species, xi.ctypes.data_as(C.c_void_p),
                                          u.ctypes.data_as(C.c_void_p),
                                          ids.ctypes.data_as(C.POINTER(C.c_uint32)), n.value,
                                          C.byref(m)))
        return xi[:m.value], u[:m.value], ids[:m.value]

    def timing(self, reset: bool = False) -> dict:
        T = GsTiming()
        self._chk(lib().gs_get_timing(self._h, C.byref(T), 1 if reset else 0))
        return dict(push_ms=T.push_ms, field_ms=T.field_ms, compact_ms=T.compact_ms,
                    push_launches=T.push_launches, field_launches=T.field_launches,
                    compact_launches=T.compact_launches, emit_ms=T.emit_ms, emit_launches=T.emit_launches)


def mlp_train(x, t, order, batch: int, theta, adam_m, adam_v, step0: int = 0, lr: float = 1e-3,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, want_grad: bool = False,
              stream=None):
    """Adam on the guess network, on the GPU (gs_mlp_train).  x [n, 48], t [n, 3],
    theta / adam_m / adam_v [39683]: float32 device tensors (the last three are
    updated in place); order: int32 device tensor of sample indices.  Returns
    (per-step losses, last gradient or None) as float32 device tensors."""
    import torch
    dev = x.device
    for a in (x, t, theta, adam_m, adam_v):
        assert a.is_cuda and a.dtype == torch.float32 and a.is_contiguous()
    assert order.is_cuda and order.dtype == torch.int32 and order.is_contiguous()
    steps = order.numel() // batch
    loss = torch.zeros(max(steps, 1), dtype=torch.float32, device=dev)
    grad = torch.zeros(MLP_NPARAM, dtype=torch.float32, device=dev) if want_grad else None
    nbytes = lib().gs_mlp_train_workspace(batch)
    work = torch.empty(max(nbytes, 4), dtype=torch.uint8, device=dev)
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    rc = lib().gs_mlp_train(C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()), x.shape[0],
                            C.c_void_p(order.data_ptr()), order.numel(), batch, C.c_void_p(theta.data_ptr()),
                            C.c_void_p(adam_m.data_ptr()), C.c_void_p(adam_v.data_ptr()), step0, lr, beta1,
                            beta2, eps, C.c_void_p(loss.data_ptr()),
                            C.c_void_p(grad.data_ptr()) if grad is not None else None,
                            C.c_void_p(work.data_ptr()), nbytes, C.c_void_p(st.cuda_stream))
    if rc != GS_OK:
        raise GapsimError(rc, "gs_mlp_train failed (bad arguments or an index outside [0, n))")
    return loss[:steps], grad
