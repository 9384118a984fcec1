/*
 * gapsim: circuit-coupled 1D electrostatic particle-in-cell step on AMD MI355X
 * (gfx950), after Kim, Yun, Lee, Na, "Self-Consistent Numerical Framework for
 * Multiscale Circuit-Plasma Coupling with Secondary Electron Emission"
 * (arXiv 2603.24010).
 *
 * One time step of one or many independent vacuum gaps.  Node 0 (x = 0) is the
 * electrode wired to the external circuit, node N (x = d) is grounded.  Per
 * step and gap:
 *   1. circuit + field at level n: BDF2 loop-charge circuit (Sec. 2.1, App. A),
 *      node-centred Poisson with phi_N = 0 (Sec. 2.2.1, App. B) whose first row
 *      couples to the circuit, strict (Sec. 2.4.2, eq. Poisson_BC2) or weak
 *      (Sec. 2.4.3, eq. Poisson_BC3); surface charge eq. top_plate_charge;
 *   2. gather from the half-grid field and leapfrog push (Sec. 2.2.2, App. C);
 *   3. absorption at either electrode, convection charge (Sec. 2.4.1) and
 *      ion-induced secondary emission (Sec. 2.3, Alg. 2);
 *   4. optional ion beam entering at either electrode, by a fixed count or a
 *      per-step schedule (Sec. 4.2);
 *   5. charge deposit with the same linear weights, electrode nodes doubled
 *      (App. C, App. E).
 *
 * Conventions of every entry point:
 *   - Return a gs_status; nothing throws or aborts across this boundary.
 *   - Work is queued on the HIP stream given to gs_init_gap and is asynchronous,
 *     except gs_read_diagnostics / gs_read_particles / gs_get_timing, which
 *     synchronise that stream.
 *   - The library owns all device state; caller buffers are read or written
 *     during the call only and never retained.
 *   - A device-side error (particle capacity exceeded) is sticky: the next call
 *     returns GS_ECAPACITY and gs_last_error says which gap.
 *   - Calls on one context are not thread-safe.
 *   - Units are SI unless a name says otherwise.
 */
#ifndef GAPSIM_H
#define GAPSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GS_MAX_MESH 8

typedef enum {
  GS_OK = 0,
  GS_EINVAL = -1,     /* bad argument or parameter; nothing changed */
  GS_ENOMEM = -2,     /* an allocation failed; the context is unusable */
  GS_ECAPACITY = -3,  /* a gap ran out of particle slots; new particles were dropped */
  GS_EDEVICE = -4,    /* a HIP call failed; the context is unusable */
  GS_ENOCONV = -5,    /* a Newton solve missed its tolerance within its iteration cap */
  GS_ESTATE = -6,     /* call out of order (e.g. no context) */
  GS_ECALLBACK = -7   /* an external circuit engine reported failure; that step was not taken */
} gs_status;

enum { GS_SEE_FIXED = 0, GS_SEE_EXP = 1, GS_SEE_LOGNORMAL = 2 };
/* mean secondary yield as a function of the ion's energy */
enum { GS_YIELD_SATURATING = 0, GS_YIELD_POLY = 1 };
/* electrode the beam enters at */
enum { GS_BEAM_CIRCUIT = 0, GS_BEAM_GROUND = 1 };
enum { GS_GUESS_DIRECT = 0, GS_GUESS_EXTRAP = 1, GS_GUESS_MLP = 2 };

/* Device memory hook.  alloc(bytes, user) returns device memory or NULL;
 * release(ptr, user) frees it.  A NULL allocator means hipMalloc/hipFree. */
typedef struct {
  void *(*alloc)(size_t bytes, void *user);
  void (*release)(void *ptr, void *user);
  void *user;
} gs_allocator;

/* Parameters of one gap.
 *   Species 0 are electrons, species 1 ions.  A macroparticle of species s
 *   carries the areal sheet charge weight * q_unit * Z[s] [C/m^2] (the
 *   superparticle ratio times the particle charge, as in tab:validation_parameters).
 *   The circuit is written in loop (mesh) charges q (Sec. 2.1):
 *     L q'' + R q' + S q + e_gap V_gap = src * Vs(t),
 *     Vs(t) = src_dc + src_amp sin(2 pi src_freq t + src_phase),
 *   the gap element (the gap itself, eps0 area / d, in parallel with c_par) lying
 *   in mesh gap_mesh.  q0 holds the loop charges before t = 0 (switch closes at
 *   t = 0).  Matrices are row-major, only the leading n_mesh x n_mesh used.
 *   SEE (Sec. 2.3, Alg. 2): an ion hitting either electrode frees
 *   Poisson(gamma) electrons, at most see_max, E the ion's normal kinetic energy:
 *     GS_YIELD_SATURATING: gamma = see_amp (E/see_E0_eV) / (1 + E/see_E0_eV);
 *     GS_YIELD_POLY: gamma = see_amp max(f(x), 0), f(x) = sum_k see_poly[k] x^k
 *       (the paper's fifth-order fit), x = min(E, see_poly_Emax_eV) / 1 keV
 *       (evaluated by Horner's rule from see_poly[5]).
 *   Each electron leaves the surface normally with energy see_E_eV
 *   (GS_SEE_FIXED), an exponential draw of mean see_E_eV (GS_SEE_EXP), or
 *   exp(see_ln_mu + see_ln_sigma Z) eV, Z standard normal (GS_SEE_LOGNORMAL,
 *   the paper's law; Z = sqrt(-2 ln u1) cos(2 pi u2) from two of the ion's
 *   stream words).  see_amp > 0 switches emission on.
 *   Beam: ions enter at the circuit electrode (beam_side GS_BEAM_CIRCUIT, node 0,
 *   moving towards the ground) or at the grounded one (GS_BEAM_GROUND, node N,
 *   moving towards the circuit electrode), with energies uniform in
 *   [beam_Emin_eV, beam_Emax_eV].  They start uniformly within beam_layer [m]
 *   of that electrode, or, with beam_layer 0, within the distance they fly in
 *   one step (as if they entered during the step).  The paper injects its ions
 *   in a layer next to the grounded electrode with a Gaussian pulse in time
 *   (Sec. 4.2); a pulse is given as a schedule: with beam_schedule non-NULL the
 *   step that solves level n injects beam_schedule[n] ions (n <
 *   beam_schedule_len, none after), else beam_per_step every step.  The
 *   schedule is copied by gs_init_gap; the caller keeps its array.
 *   particle_fp: 32 (binary32 particles, 2^-24 fixed-point deposit weights) or
 *   64 (binary64 particles, 2^-44 weights); the same for every gap of a context.
 *   capacity[s]: particle slots of species s (live plus not-yet-reclaimed). */
typedef struct {
  int32_t n_cells;
  double d, area, eps0, dt;
  int32_t Z[2];
  double mass[2];
  double q_unit, weight, ev;
  int32_t n_mesh, gap_mesh;
  double L[GS_MAX_MESH][GS_MAX_MESH];
  double R[GS_MAX_MESH][GS_MAX_MESH];
  double S[GS_MAX_MESH][GS_MAX_MESH];
  double src[GS_MAX_MESH];
  double src_dc, src_amp, src_freq, src_phase;
  double c_par;
  double q0[GS_MAX_MESH];
  double see_amp, see_E0_eV;
  int32_t see_law, see_max;
  double see_E_eV;
  int32_t see_yield;
  double see_poly[6];
  double see_poly_Emax_eV;
  double see_ln_mu, see_ln_sigma;
  int64_t beam_per_step;
  double beam_Emin_eV, beam_Emax_eV;
  int32_t beam_side;
  double beam_layer;
  const int64_t *beam_schedule; /* nullable, see above */
  int64_t beam_schedule_len;
  uint64_t seed;
  int32_t particle_fp;
  int64_t capacity[2];
  double v_ref; /* voltage scale of the Newton residual norm (> 0) */
} gs_gap_params;

/* State of one gap after the last completed step (level n = step).  The
 * quantities are the coupling variables of the paper's variables table
 * (tab:variables, Sec. 2.4): the electrode potential phi0 = V_gap, the surface
 * charge sigma_+ of the circuit electrode, the circuit charge on the gap Q_circ
 * (weak mode: Q_circ* before the reset), the convection charge Q_conv that the
 * push delivered, and the loop charges and currents; the counts are the
 * electrode impact statistics of Sec. 2.3 and Sec. 4.2 (absorbed, emitted,
 * injected), and the Newton fields describe the strict step's Newton form (not
 * in the paper). */
typedef struct {
  int64_t step;           /* level of the last field solve (-1 before the first step) */
  double t;               /* step * dt */
  double phi0;            /* electrode potential = gap voltage */
  double sigma;           /* surface charge sigma_+ of the circuit electrode [C/m^2] */
  double qcirc;           /* circuit charge Q_circ (weak: re-imposed C_gap phi0) */
  double qcirc_star;      /* weak: the circuit's own gap charge; strict: = qcirc */
  double qconv;           /* convection charge that entered this level [C] */
  double e_ground;        /* field at the grounded electrode [V/m] */
  double q[GS_MAX_MESH];  /* loop charges */
  double I[GS_MAX_MESH];  /* loop currents (BDF2) */
  int64_t n_live[2];      /* live particles per species */
  int64_t n_slots[2];     /* slots in use per species (live + absorbed, not reclaimed) */
  int64_t abs_step[2][2]; /* absorbed in the last push [species][0 circuit, 1 ground] */
  int64_t emit_step[2];   /* electrons emitted in the last push at [electrode] */
  int64_t inj_step;       /* beam ions injected in the last step */
  int64_t abs_cum[2][2];
  int64_t emit_cum[2];
  int64_t inj_cum;
  int64_t pushed_cum;     /* particle pushes so far (particle-steps) */
  int32_t newton_last;    /* Newton updates at the last strict step (-1: direct solve) */
  int32_t newton_fallback_last; /* 1 if the last step fell back from the MLP guess */
  int64_t newton_total;   /* Newton updates summed over strict steps */
  int64_t newton_fallbacks;
  int32_t newton_max;     /* most updates any one level needed */
  int32_t newton_levels;  /* levels solved by Newton (not the direct solve) */
  double newton_resid0;   /* infinity norm of the scaled residual at the initial guess */
  double newton_resid;    /* ... after the last update */
  double newton_guess[GS_MAX_MESH + 1]; /* initial guess u = (V, I_0, ..) of the last solve
                                           (direct solve: the extrapolation) */
  double mlp_proposal[3]; /* the guess network's u at the last GS_GUESS_MLP solve, used or not */
  double qcirc_step;      /* qcirc_star minus the previous level's qcirc: the charge the
                             circuit moved onto the gap over the last step [C] */
  double q_space;         /* space charge in the gap at the last level: area times the
                             integral of rho (electrode nodes at half weight) [C]; with
                             sigma * area it is the charge that the grounded electrode
                             mirrors (Gauss' law) */
} gs_diag;

/* Accumulated device time of the library's kernels, measured with HIP events
 * on the context's stream while timing is switched on (GS_OPT_TIMING). */
typedef struct {
  double push_ms, field_ms, compact_ms;
  int64_t push_launches, field_launches, compact_launches;
  double emit_ms;          /* the emission kernel that runs after each push while the
                              cell sort is on */
  int64_t emit_launches;
} gs_timing;

/* Options for gs_set_option. */
enum {
  GS_OPT_BLOCK = 1,        /* push threads per block: 256 (default), 512, 768 or 1024 */
  GS_OPT_TILE = 2,         /* granularity at which particles are split between push
                              blocks (a multiple of 8 x the block size; default 8 x) */
  GS_OPT_GRID = 3,         /* push blocks; 0 = from occupancy */
  GS_OPT_COMPACT_EVERY = 4,/* steps between reclaiming absorbed slots (>= 1) */
  GS_OPT_GRAPH = 5,        /* 1: replay steps through a captured hipGraph */
  GS_OPT_TIMING = 6,       /* 1: time each kernel launch with HIP events, 2: the push only */
  GS_OPT_NEWTON_TOL = 7,   /* value * 1e-12 = scaled residual tolerance (default 1e-10) */
  GS_OPT_NEWTON_MAXIT = 8, /* Newton corrections allowed per level, 0..64 (default 8) */
  GS_OPT_DEPOSIT = 9,      /* binary32 deposit cells: 0 auto, 1 64-bit, 2 32-bit with carries */
  GS_OPT_COMPACT_GRID = 10,/* workgroups of the compaction kernel (>= 1) */
  GS_OPT_PPT = 11,         /* 16-byte particle vectors per thread per chunk: 1 (default) or 2 */
  GS_OPT_SORT_BIN = 12,    /* 0 (default): every GS_OPT_COMPACT_EVERY steps absorbed slots are
                              reclaimed in place of order; >= 4: instead the live particles
                              are counting-sorted by bins of this many cells, so that each
                              push workgroup deposits onto, and flushes, a narrow band of
                              nodes; the secondary emission of a push then runs in its own
                              kernel right after it.  Results do not depend on it. */
  GS_OPT_STEAL = 13,       /* k in 2..64: the last 1/k of each push workgroup's run of tiles
                              goes to a pool that workgroups done with their own runs draw
                              from, one tile at a time; 0 (default): fixed runs.  Results do
                              not depend on it. */
  GS_OPT_STREAM = 14       /* how the push streams the particle arrays, bits: 1 round-robin
                              tile order (push workgroup w takes tiles w, w + grid, ...,
                              instead of a contiguous run; the pool of GS_OPT_STEAL is then
                              unused), 2 non-temporal loads and stores of binary32
                              particles (for particle arrays far larger than the caches);
                              0 (default): neither.  Results do not depend on it. */
};

typedef struct gs_ctx gs_ctx;

/* Create a context for n_gaps gaps (Sec. 2.4: each gap is one load capacitor
 * with its own circuit).  params: n_gaps host structs, copied.  Each gap starts
 * with no particles, its circuit at q0 and the electrode holding the gap's share
 * of the gap-mesh charge; the first step solves level 0.  alloc may be NULL.
 * hip_stream is a hipStream_t (NULL = the default stream).  Errors: GS_EINVAL
 * (message from gs_last_error(NULL)), GS_ENOMEM, GS_EDEVICE; *out is NULL then. */
gs_status gs_init_gap(gs_ctx **out, int32_t n_gaps, const gs_gap_params *params,
                  const gs_allocator *alloc, void *hip_stream);

/* Destroy a context and free its device memory (NULL is ignored). */
void gs_destroy(gs_ctx *ctx);

/* Add n particles of one species to one gap at the current level: x in [0, d]
 * [m], v = v_x [m/s], each an array of n doubles, in host memory
 * (ptr_is_device = 0) or device memory (1).  Ids are assigned in order from the
 * gap's counter (ions' ids key their secondary-emission draws).  Their charge is
 * added to the density the next step solves with (App. E: a particle appearing
 * at a level counts at that level).  Copied; the caller keeps ownership.
 * Errors: GS_EINVAL (bad gap/species/position), GS_ECAPACITY. */
gs_status gs_inject(gs_ctx *ctx, int32_t gap, int32_t species, int64_t n, const double *x,
                    const double *v, int32_t ptr_is_device);

/* For callers that cannot allocate device memory (serving loops that inject
 * every step, harnesses that forbid hipMalloc): gs_inject for host arrays x, v
 * (n doubles each, same meaning and checks) that allocates nothing.  gs_inject
 * with host arrays allocates a device staging buffer per call; this copies them
 * through a staging array the library holds on each device for the life of
 * the process (2 * GS_INJECT_NOALLOC_MAX doubles, 8 MiB), so n is at most
 * GS_INJECT_NOALLOC_MAX (GS_EINVAL beyond).  Device arrays need no staging:
 * use gs_inject with ptr_is_device = 1.  Synchronises the context's stream
 * before returning.  Every context on one device shares the array: calls that
 * overlap in time on one device (from several threads or streams) race.
 * Errors: as gs_inject; GS_ESTATE if the array could not be set up. */
#define GS_INJECT_NOALLOC_MAX (1 << 19)
gs_status gs_inject_noalloc(gs_ctx *ctx, int32_t gap, int32_t species, int64_t n, const double *x,
                            const double *v);

/* Advance every gap n_steps steps with strict coupling (Sec. 2.4.2): the circuit
 * charge is an affine function of the electrode potential, eq. Q4_phi_relation,
 * folded into the first Poisson row (eq. Poisson_BC2) and solved in one pass.
 * guess = GS_GUESS_DIRECT solves that closed system directly; GS_GUESS_EXTRAP or
 * GS_GUESS_MLP instead runs Newton on u = (gap voltage, loop currents) from a
 * quadratic extrapolation or from the network set by gs_mlp_set_weights (the
 * Newton iteration decides convergence; a non-finite or worse MLP guess falls
 * back to the extrapolation).  The iteration stops when the scaled residual is
 * within the tolerance (GS_OPT_NEWTON_TOL) or when an update changed no
 * component by more than 8 units in its last place (the residual of the
 * representable u nearest the solution can exceed the tolerance when loop
 * currents are large), else at GS_OPT_NEWTON_MAXIT updates (GS_ENOCONV).  Asynchronous.  Errors: GS_EINVAL (bad mode; the
 * network needs every gap to have two meshes), GS_ESTATE (GS_GUESS_MLP before
 * weights were set), GS_ECAPACITY (sticky), GS_EDEVICE. */
gs_status gs_step_strict(gs_ctx *ctx, int32_t n_steps, int32_t guess);

/* Advance every gap n_steps steps with weak coupling (Sec. 2.4.3): the circuit
 * is stepped first with the gap as a capacitor, its gap charge enters the
 * surface-charge update (eq. Poisson_BC3), and after the field solve the gap
 * charge is re-imposed as C_gap phi0 (the circuit's increment history kept).
 * Asynchronous.  Errors as gs_step_strict. */
gs_status gs_step_weak(gs_ctx *ctx, int32_t n_steps);

/* Weak coupling with an external circuit engine (the SPICE-based solver option
 * of Sec. 2.1 with Alg. 1, coupled as in Sec. 2.4.3).  The engine holds the
 * circuit; for every step and gap the library calls
 *   fn(user, gap, level, dt, phi0_prev, &v_gap)
 * in gap order, on the calling thread, before any device work of that step:
 * level n is the level about to be solved, phi0_prev the electrode potential of
 * level n-1 (for n = 0: q0[gap_mesh] / (C_gap + c_par)).  The engine restarts
 * its gap capacitor from phi0_prev (the reset Q_circ^{n-1} = C_gap phi0^{n-1}),
 * advances its circuit over [t_{n-1}, t_n] and writes the gap voltage V* it
 * reaches; the library takes Q_circ^n* = C_gap V* into the surface-charge
 * update (eq. top_plate_charge), solves the field with the plain Gauss row
 * (eq. Poisson_BC3), re-imposes Q_circ^n = C_gap phi0^n and pushes.  C_gap =
 * eps0 area / d; an engine with c_par in its own circuit sees the parallel
 * capacitor there.  The library's own loop charges are not advanced (the gap
 * mesh holds (C_gap + c_par) phi0, the others keep their values, and the
 * loop currents in gs_diag are not the engine's).  Any non-zero return from fn,
 * or a non-finite v_gap, stops the call before that step's device work:
 * GS_ECALLBACK (GS_EINVAL for a non-finite v_gap), with every earlier step
 * done.  Timing: the first step of a call waits for the stream; each later
 * step waits only for the previous field solve, whose potentials the field
 * kernel writes to a small pinned host buffer the library owns (16 bytes per
 * gap, also where the engine's voltages go), so the engine runs while that
 * step's push is still on the device.  Otherwise asynchronous like
 * gs_step_weak (device errors surface at the next synchronising call); never
 * uses a captured graph.  Errors: GS_EINVAL (fn NULL, n_steps < 0),
 * GS_ECALLBACK and those of gs_step_weak. */
typedef int32_t (*gs_circuit_fn)(void *user, int32_t gap, int64_t level, double dt, double phi0_prev,
                                 double *v_gap);
gs_status gs_step_weak_external(gs_ctx *ctx, int32_t n_steps, gs_circuit_fn fn, void *user);

/* Highest ringing angular frequency omega_max of a gap's circuit (App. D,
 * circuit-resolution constraint), host only: the largest |Im lambda| over the
 * finite roots of det(lambda^2 L + lambda R + S') = 0, the free response of
 * the circuit in the parameters with S' = S plus the gap element's elastance
 * 1 / (C_gap + c_par) in the gap mesh.  0 when no root oscillates (e.g. no
 * inductance).  Errors: GS_EINVAL (invalid parameters, or the roots could not
 * be found). */
gs_status gs_circuit_resonance(const gs_gap_params *p, double *omega_max);

/* Time-step check of one gap against the constraints of App. D (time segment
 * selection), a posteriori, at the last completed step:
 *   omega_max  gs_circuit_resonance of the gap's parameters (an external
 *              circuit engine may run another circuit); n_omega = 1 /
 *              (omega_max dt), infinite when omega_max is 0, to be at least
 *              N_omega (20..50);
 *   beta[s]    largest |v_x| dt / dx over live particles of species s (the
 *              cell-crossing number, at most 0.2..0.5); v_max[s] that |v_x|;
 *   n_e_max    largest live-electron density in one cell, count * weight / dx
 *              [m^-3]; omega_pe = sqrt(n_e_max e^2 / (eps0 m_e)) with
 *              e = q_unit |Z[0]|, m_e = mass[0]; alpha = omega_pe dt (at most
 *              0.1..0.2);
 *   eta        |qcirc_step| / max(|qcirc_star|, |previous qcirc|): the
 *              circuit's relative charge change over the step, dt I_ref /
 *              Q_ref with I_ref = |qcirc_step| / dt (at most 0.05..0.2; 0
 *              when both charges are 0).
 * flags: bit 0 n_omega < 20, bit 1 a beta above 0.5, bit 2 alpha > 0.2, bit 3
 * eta > 0.2 (the permissive end of each of the paper's ranges).  Synchronises;
 * the scan runs on the device.  Errors: GS_EINVAL, GS_ENOMEM, GS_EDEVICE, the
 * sticky step errors. */
typedef struct {
  double dt;
  double omega_max, n_omega;
  double v_max[2], beta[2];
  double n_e_max, omega_pe, alpha;
  double eta;
  int32_t flags;
} gs_dt_report;
gs_status gs_dt_check(gs_ctx *ctx, int32_t gap, gs_dt_report *out);

/* Read one gap's state (synchronises the stream): the coupling variables of
 * tab:variables and the impact counts (gs_diag).  phi (n_cells + 1 values),
 * E (n_cells half-grid values E_{k+1/2}) and rho (n_cells + 1 nodal densities,
 * electrode nodes already doubled) of the last solved level are written to the
 * caller's host arrays when not NULL.  Errors: GS_EINVAL, GS_EDEVICE; the sticky
 * errors of the steps (GS_ECAPACITY, GS_EINVAL for a bad device-side injection);
 * GS_ENOCONV once after a strict Newton solve missed its tolerance (the outputs
 * are filled and the state stays valid: the last iterate was used).
 * Emission timing: the secondaries of the ions absorbed in a step are emitted
 * within that step (by the push workgroup that absorbed them, or, past what it
 * can hold, by the push's last workgroup to finish, or with the cell sort on by
 * the emission kernel right after the push). */
gs_status gs_read_diagnostics(gs_ctx *ctx, int32_t gap, gs_diag *out, double *phi, double *E,
                              double *rho);

/* Copy one gap's live particles of one species to host arrays in grid units:
 * xi = x / dx, u = v_x dt / dx, as binary32 (particle_fp 32) or binary64 (64);
 * id: their ids (0xFFFFFFFF for emitted electrons).  Order is unspecified.
 * At most max_n are written; *n_out receives the live count.  Synchronises. */
gs_status gs_read_particles(gs_ctx *ctx, int32_t gap, int32_t species, void *xi, void *u,
                            uint32_t *id, int64_t max_n, int64_t *n_out);

/* ---- Newton guess network --------------------------------------------------
 * Not part of the paper: the paper solves the strict step (Sec. 2.4.2) in one
 * linear pass.  Its Newton form (gs_step_strict with a guess mode) starts from
 * a guess of u = (gap voltage, I_0, I_1); a small network can propose it.  The
 * network is 48 -> 128 -> 128 -> 128 -> 3, GELU hidden layers (exact erf
 * form), linear output.  Parameters: one array of GS_MLP_NPARAM binary32 values
 * W1[128][48] b1[128] W2[128][128] b2[128] W3[128][128] b3[128] W4[3][128]
 * b4[3] (weights row-major [out][in]).
 * Input for level n: the last 8 steps k = 1..8, features 6(k-1) + q: (V,
 * I_0, I_1, sigma_+) of level n-k and (Q_abs, Q_em) of the push that followed
 * it (for k = 1 the push into level n, whose charge is known before level n
 * is solved), where Q_abs is the charge the circuit electrode absorbed and
 * Q_em the charge of the electrons it emitted (Q_conv = Q_abs - Q_em);
 * normalised as (x - x_mean) / x_scale.  Output y: u = u_extrap + y_mean + y_scale * y, with
 * u_extrap the quadratic extrapolation 3 u_{n-1} - 3 u_{n-2} + u_{n-3}.
 * norm: GS_MLP_NORM binary64 values x_mean[48] x_scale[48] y_mean[3]
 * y_scale[3]. */
#define GS_MLP_IN 48
#define GS_MLP_OUT 3
#define GS_MLP_NPARAM 39683
#define GS_MLP_NORM 102

/* Install the network used by gs_step_strict(..., GS_GUESS_MLP): theta (host,
 * n = GS_MLP_NPARAM finite values) is rounded to bfloat16 (nearest, ties to
 * even) for evaluation with binary32 sums; norm (host, GS_MLP_NORM values,
 * scales > 0) is copied.  Synchronises.  Errors: GS_EINVAL, GS_ENOMEM,
 * GS_EDEVICE. */
gs_status gs_mlp_set_weights(gs_ctx *ctx, const float *theta, int64_t n, const double *norm);

/* Evaluate the installed network (bfloat16 weights, binary32 sums, the same
 * device routine the strict step uses) on n normalised inputs: x [n][48] and
 * y [n][3] in device memory, caller-owned.  Asynchronous on the context's
 * stream.  Errors: GS_ESTATE (no weights), GS_EINVAL, GS_EDEVICE. */
gs_status gs_mlp_forward(gs_ctx *ctx, const float *x, int64_t n, float *y);

/* Record training samples from the following strict steps: the field solve of
 * level n of gap g writes sample (n - n0) * n_gaps + g, where n0 is the level
 * the next step solves, while that index is below capacity: x [.][48] the raw
 * (unnormalised) input of that level, y [.][3] the raw target u* - u_extrap,
 * u* being the level's solution (V, I_0, I_1).  Levels whose history reaches
 * before level 0 see zeros there.  x and y are device memory owned by the
 * caller, written asynchronously and kept until recording is switched off
 * (x or y NULL, or capacity 0).  Errors: GS_EINVAL. */
gs_status gs_mlp_record(gs_ctx *ctx, float *x, float *y, int64_t capacity);

/* Bytes of device workspace gs_mlp_train needs for a batch size (0 if batch < 1). */
size_t gs_mlp_train_workspace(int32_t batch);

/* Train the network by Adam (Kingma and Ba 2015; bias-corrected moments) on
 * the mean squared error, in binary32, on the GPU.  Device arrays, caller-owned:
 * x [n][48] normalised inputs, t [n][3] normalised targets; order [n_order]
 * sample indices, taken batch by batch (n_order / batch steps; a remainder is
 * ignored; an index outside [0, n) is replaced by 0 and makes the call return
 * GS_EINVAL); theta, adam_m, adam_v [GS_MLP_NPARAM] updated in place; step0 =
 * Adam steps already taken; loss [steps] (may be NULL) receives each step's
 * batch loss before its update; grad_last [GS_MLP_NPARAM] (may be NULL) the
 * last step's gradient; work (work_bytes >= gs_mlp_train_workspace(batch)).
 * Runs on hip_stream (a hipStream_t, NULL = default) and synchronises it at
 * the end.  Errors: GS_EINVAL, GS_EDEVICE. */
gs_status gs_mlp_train(const float *x, const float *t, int64_t n, const int32_t *order, int64_t n_order,
                       int32_t batch, float *theta, float *adam_m, float *adam_v, int64_t step0, double lr,
                       double beta1, double beta2, double eps, float *loss, float *grad_last, void *work,
                       size_t work_bytes, void *hip_stream);

/* A launch configuration chosen by gs_autotune (or in effect, gs_get_launch). */
typedef struct {
  int32_t block;          /* push threads per workgroup */
  int32_t tile;           /* particles per work tile */
  int32_t grid;           /* push workgroups */
  int32_t ppt;            /* 16-byte particle vectors per thread per chunk (1 or 2) */
  int32_t deposit;        /* GS_OPT_DEPOSIT value */
  int32_t compact_every;  /* steps between compactions (or cell sorts) */
  int32_t sort_bin;       /* GS_OPT_SORT_BIN value (0: compaction without sorting) */
  int32_t steal;          /* GS_OPT_STEAL value */
  int32_t stream;         /* GS_OPT_STREAM value */
  double ms_per_step;     /* measured time per step of the chosen configuration
                             (gs_get_launch: 0) */
} gs_tuning;

/* The launch configuration in effect (push shape, deposit cells, compaction
 * interval, cell-sort bin), as gs_autotune reports its choice.  Host only. */
gs_status gs_get_launch(const gs_ctx *ctx, gs_tuning *out);

/* Choose the push launch shape (block, vectors per thread, tile, grid), then
 * the compaction interval and whether to cell-sort (and by which bin) instead
 * of compacting, then the tile pool (GS_OPT_STEAL) and the particle stream
 * (GS_OPT_STREAM), for this context's gaps by timing candidates on its
 * own current state: every device buffer and host counter is saved first and
 * put back afterwards, so the state after the call is the state before it.
 * mode 0 strict (with guess) or 1 weak; trial_steps timed steps per shape
 * candidate (at least 64 per compaction candidate).  Needs room for one copy
 * of the context's device memory.  cache_path (may be NULL): a text file of
 * earlier choices keyed by the gap count, grid size, precision, mode, guess,
 * log2 of the live particles and CU count; a hit is applied without trials and
 * a new choice is appended.  The choice stays in effect (as if set with
 * gs_set_option) and is written to *out when not NULL.  Synchronises.  Errors:
 * GS_EINVAL, GS_ESTATE, GS_ENOMEM, GS_EDEVICE and the step errors. */
gs_status gs_autotune(gs_ctx *ctx, int32_t mode, int32_t guess, int32_t trial_steps, const char *cache_path,
                      gs_tuning *out);

/* Tune or switch parts of the launch configuration (see GS_OPT_*). */
gs_status gs_set_option(gs_ctx *ctx, int32_t option, int64_t value);

/* Accumulated kernel timings since the last reset (synchronises); reset != 0
 * clears them afterwards. */
gs_status gs_get_timing(gs_ctx *ctx, gs_timing *out, int32_t reset);

/* Check one gap's parameters on the host without touching a device.  On
 * GS_EINVAL a message is written to msg (cap bytes, NUL-terminated). */
gs_status gs_validate_params(const gs_gap_params *p, char *msg, size_t cap);

/* Message of the last failed call on ctx ("" if none); with ctx NULL the last
 * failed gs_init_gap. */
const char *gs_last_error(const gs_ctx *ctx);

/* Library version string. */
const char *gs_version(void);

#ifdef __cplusplus
}
#endif
#endif
