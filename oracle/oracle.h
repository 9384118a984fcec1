/*
 * CPU oracle for the circuit-coupled 1D electrostatic PIC step of
 * Kim, Yun, Lee, Na, "Self-Consistent Numerical Framework for Multiscale
 * Circuit-Plasma Coupling with Secondary Electron Emission" (arXiv 2603.24010).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference that the
 * GPU path is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product path never does.
 * It shares no source with the GPU library (its own header, its own structs,
 * its own random-number generator written from the published definition).
 *
 * Two arithmetic modes:
 *   fp32 = 0  every quantity in binary64, particles in SI units (m, m/s), charge
 *             deposited in binary64.  This is the scheme as the paper writes it.
 *   fp32 = 1  particles held in binary32 in grid units (position in cells,
 *             velocity in cells per step), every binary32 operation written out
 *             in a fixed order, charge weights rounded to multiples of 2^-24 of
 *             a macroparticle and summed exactly in int64.  Field, surface
 *             charge and circuit stay binary64.  This is the reduced-precision
 *             variant of the same scheme; it exists so that integer outcomes
 *             (which particle reaches which wall, how many electrons it frees)
 *             can be compared bit for bit with a binary32 particle code.
 */
#ifndef GAPSIM_ORACLE_H
#define GAPSIM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_MAX_MESH 8

enum { OR_STRICT = 0, OR_WEAK = 1, OR_WEAK_EXT = 2 };
enum { OR_SEE_FIXED = 0, OR_SEE_EXP = 1, OR_SEE_LOGNORMAL = 2 };
enum { OR_YIELD_SATURATING = 0, OR_YIELD_POLY = 1 };

typedef struct {
  /* gap and grid, SI.  Node 0 (x = 0) is the circuit electrode, node N
   * (x = d) is grounded. */
  int32_t n_cells;
  double d, area, eps0, dt;
  /* species 0 = electrons, 1 = ions: integer charge number and mass.  A
   * macroparticle of species s carries the areal sheet charge
   * weight * q_unit * Z[s]  [C/m^2]. */
  int32_t Z[2];
  double mass[2];
  double q_unit, weight;
  double ev; /* joules per electron-volt */
  /* lumped circuit in loop (mesh) charges: L q'' + R q' + S q + g V_gap = b Vs(t).
   * The gap element sits in mesh gap_mesh, in parallel with c_par. */
  int32_t n_mesh, gap_mesh;
  double L[OR_MAX_MESH][OR_MAX_MESH];
  double R[OR_MAX_MESH][OR_MAX_MESH];
  double S[OR_MAX_MESH][OR_MAX_MESH];
  double src[OR_MAX_MESH];
  double src_dc, src_amp, src_freq, src_phase;
  double c_par;
  double q0[OR_MAX_MESH]; /* loop charges for t < 0 (switch closes at t = 0) */
  /* secondary emission by ions (Sec. 2.3, Alg. 2): Poisson count of mean
   * amp*(E/E0)/(1+E/E0) (saturating) or amp*max(poly(min(E, Emax)/1 keV), 0)
   * (the paper's fifth-order fit), capped at see_max per impact; emitted
   * energy fixed, exponential of mean see_E_eV, or lognormal exp(mu + sigma Z). */
  double see_amp, see_E0_eV;
  int32_t see_law, see_max;
  double see_E_eV;
  int32_t see_yield;
  double see_poly[6];
  double see_poly_Emax_eV;
  double see_ln_mu, see_ln_sigma;
  /* ion beam, energies uniform in [beam_Emin_eV, beam_Emax_eV], entering at
   * the circuit electrode (beam_side 0, moving towards the ground) or at the
   * grounded one (beam_side 1, moving towards the circuit electrode), started
   * uniformly within beam_layer [m] of it (0: within one step's flight).  The
   * ions per step are beam_schedule[n] for the step that solves level n (n <
   * beam_schedule_len, none after) when beam_schedule is non-NULL, else
   * beam_per_step.  The schedule is copied by or_create. */
  int64_t beam_per_step;
  double beam_Emin_eV, beam_Emax_eV;
  int32_t beam_side;
  double beam_layer;
  const int64_t *beam_schedule;
  int64_t beam_schedule_len;
  uint64_t seed;
  int32_t fp32;
} or_params;

typedef struct {
  int64_t step;          /* time level n of the last field solve */
  double t;              /* n * dt */
  double phi0;           /* electrode potential = gap voltage at level n */
  double sigma;          /* sigma_+^n */
  double qcirc;          /* Q_circ^n (weak mode: after the reset to C_gap phi0^n) */
  double qcirc_star;     /* weak mode: the circuit's own gap charge before the
                            field is known; strict mode: equal to qcirc */
  double qconv;          /* Q_conv^n that entered this solve */
  double e_ground;       /* field at the grounded electrode */
  double q[OR_MAX_MESH]; /* loop charges at level n */
  double I[OR_MAX_MESH]; /* loop currents (BDF2) at level n */
  int64_t n_live[2];
  int64_t abs_step[2][2]; /* [species][electrode 0=circuit,1=ground], last push */
  int64_t emit_step[2];   /* electrons emitted at [electrode], last push */
  int64_t inj_step;
  int64_t abs_cum[2][2];
  int64_t emit_cum[2];
  int64_t inj_cum;
  int64_t pushed_cum;     /* particle pushes so far (particle-steps) */
  double qcirc_step;      /* qcirc_star - Q_circ^{n-1} */
  double q_space;         /* A * integral of rho^n over the gap (trapezoid on the nodes) */
} or_diag;

typedef struct or_sim or_sim;

/* Philox4x64-10 block function (Salmon, Moraes, Dror, Shaw, SC'11). */
void or_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
/* smallest k with P(X <= k) >= u for X ~ Poisson(lam), by sequential inversion,
 * stopped at kmax */
int32_t or_poisson_draw(double lam, double u, int32_t kmax);

or_sim *or_create(const or_params *p);
void or_destroy(or_sim *s);
/* append n particles of a species (SI x in m, v in m/s); ids are assigned in order */
int32_t or_inject(or_sim *s, int32_t species, int64_t n, const double *x, const double *v);
/* one time step: solve level n (strict or weak), push to n+1 */
int32_t or_step(or_sim *s, int32_t mode);
/* One weak step with an external circuit engine (Alg. 1 coupled as in
 * Sec. 2.4.3): v_star is the gap voltage the engine reached at level n after
 * restarting its gap capacitor from or_phi0_prev.  Or_step with OR_WEAK_EXT
 * uses the value given last. */
int32_t or_step_external(or_sim *s, double v_star);
/* Electrode potential of the last solved level (before level 0: the gap mesh's
 * initial charge over C_gap + c_par). */
double or_phi0_prev(const or_sim *s);
void or_get_diag(const or_sim *s, or_diag *out);
/* level-n fields of the last solve: phi[N+1], E[N] (half-grid), rho[N+1] */
void or_get_fields(const or_sim *s, double *phi, double *E, double *rho);
int64_t or_count(const or_sim *s, int32_t species);
/* live particles of a species in SI units (both modes) */
int64_t or_get_particles(const or_sim *s, int32_t species, double *x, double *v, uint32_t *id);
/* live particles of a species in grid units, binary32 (fp32 mode only) */
int64_t or_get_particles_f32(const or_sim *s, int32_t species, float *xi, float *u, uint32_t *id);

/* Stand-alone pieces, used by the tests on their own. */
/* Poisson with the plain Gauss row at the circuit electrode (eq. Poisson_BC) */
void or_poisson_gauss(int32_t n_cells, double dx, double eps0, double sigma,
                      const double *rho, double *phi);
/* linear gather from the half grid (App. C); E[k] = E_{k+1/2}, surface fields at
 * the two electrodes close the electrode half cells */
double or_gather64(int32_t n_cells, double dx, const double *E, double e0_surf, double e_ground,
                   double x);
/* the same in binary32, grid units: ehat[0] = surface field at node 0,
 * ehat[k] = E_{k-1/2} (k = 1..N), ehat[N+1] = field at node N */
/* Binary32 deposit (App. C weights, in units of 2^-24 of a macroparticle):
 * adds Z times the two node shares of each of the n positions xi (cells) to
 * acc[0..n_cells]; the step's own deposit calls it. */
void or_deposit32(int32_t n_cells, int32_t Z, const float *xi, int64_t n, int64_t *acc);
float or_gather32(int32_t n_cells, const float *ehat, float xi);
/* one binary32 push in grid units with that gather and charge-to-mass factor
 * alpha = Z q dt^2 / (m dx): writes the new position and velocity; returns 0
 * inside the gap, 1 at the circuit electrode (x <= 0), 2 at the ground (x >= N) */
int32_t or_push32(int32_t n_cells, const float *ehat, float alpha, float xi, float u, float *xi_out, float *u_out);
/* the binary32 alpha of a species as the oracle's push uses it */
float or_alpha32(const or_sim *s, int32_t species);
/* beam ion k of the step that solves level `step`, in grid units (binary32) */
void or_beam_ion32(const or_sim *s, int64_t step, int64_t k, float *xi, float *u);
/* the secondary electrons of one ion absorbed at wall 0 (circuit) or 1 (ground)
 * in the push after level `step`, impact velocity v_ion [m/s] (Alg. 2): their
 * count; the first max_out (at most 1024) written as start and velocity in
 * grid units.  Or_step emits through the same routine. */
int32_t or_emit_sample(const or_sim *s, int64_t step, uint32_t ion_id, double v_ion, int32_t wall, float *xi,
                       float *u, int32_t max_out);
/* Circuit alone, the gap as a capacitor eps0*A/d (plus c_par): q_out[n*M+j],
 * v_out[n] = gap voltage, for levels 0..nsteps-1 */
int32_t or_circuit_run(const or_params *p, int64_t nsteps, double *q_out, double *v_out);

/* Guess network of the Newton form of the strict step (mlp.c): layer sizes,
 * flat parameter layout W1 b1 W2 b2 W3 b3 W4 b4 (weights row-major [out][in]),
 * GELU hidden layers, linear output. */
#define OR_MLP_IN 48
#define OR_MLP_HIDDEN 128
#define OR_MLP_OUT 3
#define OR_MLP_NPARAM 39683
double or_gelu(double z);
double or_gelu_grad(double z);
/* y[n][3] for x[n][48] */
void or_mlp_forward(const double *theta, const double *x, int64_t n, double *y);
/* mean squared error over n samples and 3 outputs; grad (may be NULL) receives
 * its gradient with respect to theta */
double or_mlp_loss_grad(const double *theta, const double *x, const double *t, int64_t n, double *grad);
/* one Adam update, step number t >= 1 */
void or_adam_step(double *theta, double *m, double *v, int64_t t, const double *g, int64_t np, double lr,
                  double beta1, double beta2, double eps);
/* binary32 rounded to bfloat16, returned as binary32 */
float or_round_bf16(float x);

#ifdef __cplusplus
}
#endif
#endif
