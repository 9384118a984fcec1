/*
 * CPU oracle for the circuit-coupled 1D ES-PIC step (arXiv 2603.24010).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the product path.
 *
 * Written to be read against the paper:
 *   Sec. 2.1 / App. A   loop equations eq:loop_1..5, BDF2 stencils, T Q = C
 *   Sec. 2.2 / App. B   node-centred Poisson eq:dt_Poisson_app, half-grid field
 *                       eq:dt_E-field, grounded node N, Gauss row eq:Poisson_BC
 *   App. C              linear (CIC) gather from the half-grid, same weights for
 *                       the deposit
 *   App. E              boundary node receives twice the weight (no charge lost)
 *   Sec. 2.3 / Alg. 2   SEE: E_ion = m v_x^2 / 2, Poisson count, energy law,
 *                       normal emission
 *   Sec. 2.4.1          convection charge, counted over one step
 *   Sec. 2.4.2          strict mode: sigma update eq:top_plate_charge, modified
 *                       circuit row, Q4 = K - [T'^-1]_44 phi0, eq:Poisson_BC2
 *   Sec. 2.4.3          weak mode: circuit first, eq:Poisson_BC3, reset
 *                       Q4^n = C3 phi0^n
 * No blocking, fusion or reordering beyond the paper's own order.
 *
 * Build with -ffp-contract=off so that a*b+c stays two roundings (the binary32
 * mode depends on it).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x64-10, from Salmon et al., "Parallel random numbers: as easy as 1, */
/* 2, 3" (SC'11): 10 rounds of two 64x64->128 multiplies with key bumps by   */
/* the Weyl constants.                                                       */
/* ------------------------------------------------------------------------ */
static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
  unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}

void or_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(M0, c0, &hi0, &lo0);
    mulhilo64(M1, c2, &hi1, &lo1);
    uint64_t n0 = hi1 ^ c1 ^ k0;
    uint64_t n1 = lo1;
    uint64_t n2 = hi0 ^ c3 ^ k1;
    uint64_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 64 random bits -> double strictly inside (0, 1) */
static double unit_open(uint64_t r) {
  return ((double)(r >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

/* Random streams.  Every draw is keyed by what it belongs to, never by the
 * order in which a program happens to visit particles:
 *   SEE of an ion:   counter (step, ion id, 1, block), key (seed, 0)
 *   beam particle k: counter (step, k, 2, 0),          key (seed, 0)      */
static void draw_block(uint64_t seed, uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                       uint64_t out[4]) {
  const uint64_t ctr[4] = {c0, c1, c2, c3};
  const uint64_t key[2] = {seed, 0};
  or_philox4x64(ctr, key, out);
}

int32_t or_poisson_draw(double lam, double u, int32_t kmax) {
  /* P(X = 0) = e^-lam, P(X = k) = P(X = k-1) * lam / k */
  double p = exp(-lam);
  double F = p;
  int32_t k = 0;
  while (u > F && k < kmax) {
    k += 1;
    p = p * lam / (double)k;
    F = F + p;
  }
  return k;
}

/* ------------------------------------------------------------------------ */
/* dense solve, Gaussian elimination with partial pivoting (n <= 8), carried  */
/* out in extended precision so the oracle's own rounding stays negligible    */
/* ------------------------------------------------------------------------ */
static int solve_dense(int n, const double A_in[OR_MAX_MESH][OR_MAX_MESH], const double *b_in,
                       double *x) {
  long double A[OR_MAX_MESH][OR_MAX_MESH + 1];
  long double xs[OR_MAX_MESH];
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) A[i][j] = A_in[i][j];
    A[i][n] = b_in[i];
  }
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (fabsl(A[r][c]) > fabsl(A[piv][c])) piv = r;
    if (A[piv][c] == 0.0L) return -1;
    if (piv != c)
      for (int j = 0; j <= n; ++j) {
        long double t = A[c][j];
        A[c][j] = A[piv][j];
        A[piv][j] = t;
      }
    for (int r = c + 1; r < n; ++r) {
      long double f = A[r][c] / A[c][c];
      for (int j = c; j <= n; ++j) A[r][j] -= f * A[c][j];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    long double s = A[i][n];
    for (int j = i + 1; j < n; ++j) s -= A[i][j] * xs[j];
    xs[i] = s / A[i][i];
  }
  for (int i = 0; i < n; ++i) x[i] = (double)xs[i];
  return 0;
}

/* ------------------------------------------------------------------------ */
/* simulation state                                                          */
/* ------------------------------------------------------------------------ */
struct or_sim {
  or_params p;
  double dx;
  int N;
  /* particles (struct of arrays); fp64 mode uses x,v (SI), fp32 mode xf,uf */
  int64_t n, cap;
  double *x, *v;
  float *xf, *uf;
  int8_t *sp;
  uint32_t *id;
  uint32_t next_id;
  /* level bookkeeping */
  int64_t step;           /* next level to solve */
  double sigma_prev;      /* sigma_+^{n-1} */
  double qcirc_prev;      /* Q_circ^{n-1} */
  double qconv_pending;   /* Q_conv^n, collected by the previous push */
  double qprev[OR_MAX_MESH];  /* loop charges q^{n-1} */
  double dq[3][OR_MAX_MESH];  /* increments q^{k} - q^{k-1} for k = n-1, n-2, n-3 */
  /* fields of the last solve */
  double *rho, *phi, *E;
  double e0_surf, e_ground;
  /* binary32 copies used by the push in fp32 mode: Ehat[0..N+1] */
  float *ehat;
  float alpha32[2];       /* q dt^2 / (m dx) in binary32 */
  int64_t *sched;         /* own copy of the beam schedule (p.beam_schedule points here) */
  double v_ext;           /* OR_WEAK_EXT: the external engine's gap voltage for the level */
  or_diag diag;
};

static const uint32_t NO_ID = 0xFFFFFFFFu;
static const double QSCALE24 = 16777216.0; /* 2^24 */

static int grow(or_sim *s, int64_t need) {
  if (need <= s->cap) return 0;
  int64_t nc = s->cap ? s->cap : 1024;
  while (nc < need) nc *= 2;
  if (s->p.fp32) {
    float *a = (float *)realloc(s->xf, (size_t)nc * sizeof(float));
    if (!a) return -1;
    s->xf = a;
    a = (float *)realloc(s->uf, (size_t)nc * sizeof(float));
    if (!a) return -1;
    s->uf = a;
  } else {
    double *a = (double *)realloc(s->x, (size_t)nc * sizeof(double));
    if (!a) return -1;
    s->x = a;
    a = (double *)realloc(s->v, (size_t)nc * sizeof(double));
    if (!a) return -1;
    s->v = a;
  }
  int8_t *b = (int8_t *)realloc(s->sp, (size_t)nc);
  if (!b) return -1;
  s->sp = b;
  uint32_t *c = (uint32_t *)realloc(s->id, (size_t)nc * sizeof(uint32_t));
  if (!c) return -1;
  s->id = c;
  s->cap = nc;
  return 0;
}

or_sim *or_create(const or_params *p) {
  if (p->n_cells < 2 || p->n_mesh < 1 || p->n_mesh > OR_MAX_MESH || p->gap_mesh < 0 ||
      p->gap_mesh >= p->n_mesh || !(p->d > 0) || !(p->area > 0) || !(p->dt > 0) ||
      !(p->eps0 > 0))
    return NULL;
  or_sim *s = (or_sim *)calloc(1, sizeof(or_sim));
  if (!s) return NULL;
  s->p = *p;
  if (p->beam_schedule) {
    size_t n = p->beam_schedule_len > 0 ? (size_t)p->beam_schedule_len : 1;
    s->sched = (int64_t *)calloc(n, sizeof(int64_t));
    if (!s->sched) {
      free(s);
      return NULL;
    }
    for (int64_t i = 0; i < p->beam_schedule_len; ++i) s->sched[i] = p->beam_schedule[i];
    s->p.beam_schedule = s->sched;
  }
  s->N = p->n_cells;
  s->dx = p->d / (double)p->n_cells;
  s->rho = (double *)calloc((size_t)s->N + 1, sizeof(double));
  s->phi = (double *)calloc((size_t)s->N + 1, sizeof(double));
  s->E = (double *)calloc((size_t)s->N, sizeof(double));
  s->ehat = (float *)calloc((size_t)s->N + 2, sizeof(float));
  /* constant history before t = 0: q^{-1} = q0, all increments zero */
  for (int j = 0; j < p->n_mesh; ++j) s->qprev[j] = p->q0[j];
  /* gap charge before t = 0 sits on the electrode: sigma = Q_gap / A */
  double cgap = p->eps0 * p->area / p->d;
  double qgap0 = p->q0[p->gap_mesh] * cgap / (cgap + p->c_par);
  s->qcirc_prev = qgap0;
  s->sigma_prev = qgap0 / p->area;
  for (int sp = 0; sp < 2; ++sp)
    s->alpha32[sp] = (float)(((double)p->Z[sp] * p->q_unit) * p->dt * p->dt / (p->mass[sp] * s->dx));
  return s;
}

void or_destroy(or_sim *s) {
  if (!s) return;
  free(s->x); free(s->v); free(s->xf); free(s->uf); free(s->sp); free(s->id);
  free(s->rho); free(s->phi); free(s->E); free(s->ehat);
  free(s->sched);
  free(s);
}

static void append(or_sim *s, int sp, double x_si, double v_si, float xi, float u, uint32_t id) {
  int64_t i = s->n;
  if (s->p.fp32) {
    s->xf[i] = xi;
    s->uf[i] = u;
  } else {
    s->x[i] = x_si;
    s->v[i] = v_si;
  }
  s->sp[i] = (int8_t)sp;
  s->id[i] = id;
  s->n = i + 1;
}

int32_t or_inject(or_sim *s, int32_t species, int64_t n, const double *x, const double *v) {
  if (species < 0 || species > 1 || n < 0) return -1;
  if (grow(s, s->n + n)) return -2;
  for (int64_t k = 0; k < n; ++k) {
    if (!(x[k] >= 0.0 && x[k] <= s->p.d)) return -1;
    float xi = (float)(x[k] / s->dx);
    float u = (float)((v[k] * s->p.dt) / s->dx);
    append(s, species, x[k], v[k], xi, u, s->next_id);
    s->next_id += 1;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* charge deposit (App. C, boundary rule of App. E)                          */
/* ------------------------------------------------------------------------ */
static double sheet_of(const or_sim *s, int sp) {
  return s->p.weight * s->p.q_unit * (double)s->p.Z[sp];
}

/* binary32 positions in cells: weights rounded to multiples of 2^-24 of a
 * macroparticle, so that the two node shares of one particle add up to exactly
 * one macroparticle; Z times them added to acc[0..N] */
void or_deposit32(int32_t N, int32_t Z, const float *xi, int64_t n, int64_t *acc) {
  for (int64_t k = 0; k < n; ++k) {
    float x = xi[k];
    int j = (int)x;
    if (j > N - 1) j = N - 1;
    float f = x - (float)j;
    float w1f = f * 16777216.0f;
    int64_t w1 = (int64_t)rintf(w1f);
    int64_t w0 = 16777216 - w1;
    acc[j] += (int64_t)Z * w0;
    acc[j + 1] += (int64_t)Z * w1;
  }
}

static void deposit(or_sim *s) {
  const int N = s->N;
  const double dx = s->dx;
  for (int i = 0; i <= N; ++i) s->rho[i] = 0.0;
  if (!s->p.fp32) {
    for (int64_t k = 0; k < s->n; ++k) {
      double h = s->x[k] / dx;
      int j = (int)floor(h);
      if (j > N - 1) j = N - 1;
      double f = h - (double)j;
      double q = sheet_of(s, s->sp[k]);
      s->rho[j] += q * (1.0 - f) / dx;
      s->rho[j + 1] += q * f / dx;
    }
  } else {
    int64_t *acc = (int64_t *)calloc((size_t)N + 1, sizeof(int64_t));
    for (int64_t k = 0; k < s->n; ++k) or_deposit32(N, s->p.Z[s->sp[k]], &s->xf[k], 1, acc);
    const double s0 = s->p.weight * s->p.q_unit;
    for (int i = 0; i <= N; ++i) s->rho[i] = s0 * ((double)acc[i] / QSCALE24) / dx;
    free(acc);
  }
  /* the electrode nodes own half a cell: twice the weight */
  s->rho[0] *= 2.0;
  s->rho[N] *= 2.0;
}

/* ------------------------------------------------------------------------ */
/* Poisson: rows 1..N-1 phi_{i-1} - 2 phi_i + phi_{i+1} = -dx^2 rho_i / eps0, */
/* phi_N = 0, row 0: a0 phi_0 - phi_1 = r0.  Thomas algorithm.               */
/* ------------------------------------------------------------------------ */
static void thomas_poisson(int N, double dx, double eps0, double a0, double r0, const double *rho,
                           double *phi) {
  /* unknowns phi_0..phi_{N-1}; sub/super diagonal entries are 1 except row 0
   * whose super-diagonal is -1.  Extended precision: the system's condition
   * number grows like N^2. */
  long double *cp = (long double *)malloc(sizeof(long double) * (size_t)N);
  long double *dp = (long double *)malloc(sizeof(long double) * (size_t)N);
  long double *ph = (long double *)malloc(sizeof(long double) * ((size_t)N + 1));
  const long double h2e = (long double)dx * (long double)dx / (long double)eps0;
  cp[0] = -1.0L / (long double)a0;
  dp[0] = (long double)r0 / (long double)a0;
  for (int i = 1; i < N; ++i) {
    long double b = -2.0L;
    long double a = 1.0L;
    long double c = (i < N - 1) ? 1.0L : 0.0L; /* phi_N = 0 drops out */
    long double r = -h2e * (long double)rho[i];
    long double m = b - a * cp[i - 1];
    cp[i] = c / m;
    dp[i] = (r - a * dp[i - 1]) / m;
  }
  ph[N] = 0.0L;
  ph[N - 1] = dp[N - 1];
  for (int i = N - 2; i >= 0; --i) ph[i] = dp[i] - cp[i] * ph[i + 1];
  for (int i = 0; i <= N; ++i) phi[i] = (double)ph[i];
  free(cp);
  free(dp);
  free(ph);
}

void or_poisson_gauss(int32_t n_cells, double dx, double eps0, double sigma, const double *rho,
                      double *phi) {
  /* eq. Poisson_BC: -phi_0 + phi_1 = -(dx^2/eps0)(sigma/dx + rho_0/2) */
  double r0 = dx * dx / eps0 * (sigma / dx + rho[0] / 2.0);
  thomas_poisson(n_cells, dx, eps0, 1.0, r0, rho, phi);
}

/* ------------------------------------------------------------------------ */
/* circuit: BDF2 in loop charges (App. A)                                    */
/* ------------------------------------------------------------------------ */
/* BDF2 (App. A):
 *   dQ/dt   ~ (3 q^n - 4 q^{n-1} + q^{n-2}) / (2 dt)
 *   d2Q/dt2 ~ (9 q^n - 24 q^{n-1} + 22 q^{n-2} - 8 q^{n-3} + q^{n-4}) / (4 dt^2)
 * Written with the increments D^k = q^k - q^{k-1} these are exactly
 *   (3 D^n - D^{n-1}) / (2 dt)  and  (9 D^n - 15 D^{n-1} + 7 D^{n-2} - D^{n-3}) / (4 dt^2),
 * and q^n = q^{n-1} + D^n.  The loop equations L q'' + R q' + S q = b Vs become
 *   T D^n = C,  T = 9 L / (4 dt^2) + 3 R / (2 dt) + S,
 *   C = b Vs(t_n) - S q^{n-1} + L (15 D^{n-1} - 7 D^{n-2} + D^{n-3}) / (4 dt^2)
 *       + R D^{n-1} / (2 dt),
 * the same T Q = C system solved for the step's increment instead of the charge
 * itself (at dt of picoseconds the charge form loses most digits of the current
 * to cancellation). */
static double source_at(const or_params *p, double t) {
  return p->src_dc + p->src_amp * sin(2.0 * M_PI * p->src_freq * t + p->src_phase);
}

/* S, plus the gap capacitor (in parallel with c_par) when the gap is a capacitor */
static double elastance(const or_params *p, int with_gap, int i, int j) {
  double s = p->S[i][j];
  if (with_gap && i == p->gap_mesh && j == p->gap_mesh) {
    double cgap = p->eps0 * p->area / p->d;
    s += 1.0 / (cgap + p->c_par);
  }
  return s;
}

static void circuit_matrix(const or_params *p, int with_gap, double T[OR_MAX_MESH][OR_MAX_MESH]) {
  const double dt = p->dt;
  for (int i = 0; i < p->n_mesh; ++i)
    for (int j = 0; j < p->n_mesh; ++j)
      T[i][j] = 9.0 * p->L[i][j] / (4.0 * dt * dt) + 3.0 * p->R[i][j] / (2.0 * dt) +
                elastance(p, with_gap, i, j);
}

static void circuit_rhs(const or_params *p, int with_gap, double t, const double *qprev,
                        const double dq[3][OR_MAX_MESH], double *C) {
  const double dt = p->dt;
  double vs = source_at(p, t);
  for (int i = 0; i < p->n_mesh; ++i) {
    double c = p->src[i] * vs;
    for (int j = 0; j < p->n_mesh; ++j) {
      double d2 = 15.0 * dq[0][j] - 7.0 * dq[1][j] + dq[2][j];
      c += p->L[i][j] * d2 / (4.0 * dt * dt) + p->R[i][j] * dq[0][j] / (2.0 * dt);
      c -= elastance(p, with_gap, i, j) * qprev[j];
    }
    C[i] = c;
  }
}

/* accept level n: charges q^n and the step's increments D^n (these differ from
 * q^n - q^{n-1} only where the weak mode re-imposed the gap charge) */
static void push_history(double *qprev, double dq[3][OR_MAX_MESH], const double *qn,
                         const double *Dn, int M) {
  for (int j = 0; j < M; ++j) {
    dq[2][j] = dq[1][j];
    dq[1][j] = dq[0][j];
    dq[0][j] = Dn[j];
    qprev[j] = qn[j];
  }
}

int32_t or_circuit_run(const or_params *p, int64_t nsteps, double *q_out, double *v_out) {
  const int M = p->n_mesh;
  double T[OR_MAX_MESH][OR_MAX_MESH];
  double qprev[OR_MAX_MESH], dq[3][OR_MAX_MESH];
  double C[OR_MAX_MESH], D[OR_MAX_MESH], q[OR_MAX_MESH];
  double cgap = p->eps0 * p->area / p->d;
  circuit_matrix(p, 1, T);
  for (int j = 0; j < M; ++j) {
    qprev[j] = p->q0[j];
    dq[0][j] = dq[1][j] = dq[2][j] = 0.0;
  }
  for (int64_t n = 0; n < nsteps; ++n) {
    circuit_rhs(p, 1, (double)n * p->dt, qprev, (const double(*)[OR_MAX_MESH])dq, C);
    if (solve_dense(M, (const double(*)[OR_MAX_MESH])T, C, D)) return -1;
    for (int j = 0; j < M; ++j) {
      q[j] = qprev[j] + D[j];
      q_out[n * M + j] = q[j];
    }
    v_out[n] = q[p->gap_mesh] / (cgap + p->c_par);
    push_history(qprev, dq, q, D, M);
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* field solve at level n, strict (Sec. 2.4.2) or weak (Sec. 2.4.3)          */
/* ------------------------------------------------------------------------ */
static int solve_level(or_sim *s, int mode) {
  const or_params *p = &s->p;
  const int N = s->N, M = p->n_mesh, g = p->gap_mesh;
  const double dx = s->dx, eps0 = p->eps0, A = p->area;
  const double cgap = eps0 * A / p->d;
  const double t = (double)s->step * p->dt;
  double T[OR_MAX_MESH][OR_MAX_MESH], C[OR_MAX_MESH], q[OR_MAX_MESH], Dn[OR_MAX_MESH];
  double sigma, qcirc, qstar;

  deposit(s);
  const double qconv = s->qconv_pending;

  if (mode == OR_STRICT) {
    /* gap row uses the electrode potential instead of a capacitor:
     * T' D = C - g phi0.  With y = T'^-1 C and z = T'^-1 g the gap charge is
     * q_g^{n-1} + y_g - z_g phi0, i.e. Q_gap = K - [T'^-1]_gg phi0
     * (eq. Q4_phi_relation, eq. K_def); the parallel capacitance holds c_par phi0. */
    double y[OR_MAX_MESH], z[OR_MAX_MESH], e[OR_MAX_MESH];
    circuit_matrix(p, 0, T);
    circuit_rhs(p, 0, t, s->qprev, (const double(*)[OR_MAX_MESH])s->dq, C);
    if (solve_dense(M, (const double(*)[OR_MAX_MESH])T, C, y)) return -3;
    for (int j = 0; j < M; ++j) e[j] = (j == g) ? 1.0 : 0.0;
    if (solve_dense(M, (const double(*)[OR_MAX_MESH])T, e, z)) return -3;
    const double K = s->qprev[g] + y[g];
    const double G = z[g] + p->c_par;
    /* eq. Poisson_BC2 as the first row of the Poisson system */
    const double a0 = 1.0 + G * dx / (eps0 * A);
    const double r0 = dx * dx / eps0 * ((s->sigma_prev + (qconv + K - s->qcirc_prev) / A) / dx + s->rho[0] / 2.0);
    thomas_poisson(N, dx, eps0, a0, r0, s->rho, s->phi);
    const double phi0 = s->phi[0];
    qcirc = K - G * phi0;
    qstar = qcirc;
    /* eq. sigma_update */
    sigma = s->sigma_prev + (qconv + qcirc - s->qcirc_prev) / A;
    for (int j = 0; j < M; ++j) {
      Dn[j] = y[j] - z[j] * phi0;
      q[j] = s->qprev[j] + Dn[j];
    }
  } else if (mode == OR_WEAK_EXT) {
    /* an external engine has stepped the circuit (Alg. 1) and handed over the
     * gap voltage it reached: Q_gap* = C3 V* enters eq. top_plate_charge */
    qstar = cgap * s->v_ext;
    sigma = s->sigma_prev + (qconv + qstar - s->qcirc_prev) / A;
    or_poisson_gauss(N, dx, eps0, sigma, s->rho, s->phi);
    const double phi0 = s->phi[0];
    /* the engine holds the circuit: the own loops stay where they are, only
     * the gap mesh carries the re-imposed charge Q4^n = C3 phi0^n */
    for (int j = 0; j < M; ++j) {
      q[j] = s->qprev[j];
      Dn[j] = 0.0;
    }
    q[g] = (cgap + p->c_par) * phi0;
    Dn[g] = q[g] - s->qprev[g];
    qcirc = cgap * phi0;
  } else {
    /* circuit first, with the gap as a capacitor: Q_gap* = C3 V_C3 */
    double D[OR_MAX_MESH] = {0}, qs[OR_MAX_MESH] = {0};
    circuit_matrix(p, 1, T);
    circuit_rhs(p, 1, t, s->qprev, (const double(*)[OR_MAX_MESH])s->dq, C);
    if (solve_dense(M, (const double(*)[OR_MAX_MESH])T, C, D)) return -3;
    for (int j = 0; j < M; ++j) qs[j] = s->qprev[j] + D[j];
    const double vstar = qs[g] / (cgap + p->c_par);
    qstar = cgap * vstar;
    sigma = s->sigma_prev + (qconv + qstar - s->qcirc_prev) / A;
    /* eq. Poisson_BC3: the plain Gauss row with that sigma */
    or_poisson_gauss(N, dx, eps0, sigma, s->rho, s->phi);
    const double phi0 = s->phi[0];
    /* The next circuit solve starts from the gap charge the field implies
     * (Q4^n = C3 phi0^n).  Only the charge level is re-imposed; the step's
     * increments, i.e. the circuit's own current history, are kept, as when a
     * circuit simulator restarts from given capacitor voltages and inductor
     * currents (Alg. 1). */
    for (int j = 0; j < M; ++j) {
      q[j] = qs[j];
      Dn[j] = D[j];
    }
    q[g] = (cgap + p->c_par) * phi0;
    qcirc = cgap * phi0;
  }

  /* eq. dt_E-field on the half grid; electrode-surface fields from Gauss' law */
  for (int k = 0; k < N; ++k) s->E[k] = (s->phi[k] - s->phi[k + 1]) / dx;
  s->e0_surf = sigma / eps0;
  s->e_ground = s->E[N - 1] + dx * s->rho[N] / (2.0 * eps0);

  /* diagnostics of level n */
  or_diag *D = &s->diag;
  D->step = s->step;
  D->t = t;
  D->phi0 = s->phi[0];
  D->sigma = sigma;
  D->qcirc = qcirc;
  D->qconv = qconv;
  D->e_ground = s->e_ground;
  for (int j = 0; j < OR_MAX_MESH; ++j) {
    D->q[j] = 0.0;
    D->I[j] = 0.0;
  }
  D->qcirc_star = qstar;
  D->qcirc_step = qstar - s->qcirc_prev;
  {
    double sp = 0.5 * (s->rho[0] + s->rho[N]);
    for (int k = 1; k < N; ++k) sp += s->rho[k];
    D->q_space = A * dx * sp;
  }
  for (int j = 0; j < M; ++j) {
    D->q[j] = q[j];
    D->I[j] = (3.0 * Dn[j] - s->dq[0][j]) / (2.0 * p->dt);
  }

  push_history(s->qprev, s->dq, q, Dn, M);
  s->sigma_prev = sigma;
  s->qcirc_prev = qcirc;
  s->qconv_pending = 0.0;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* gather (App. C).  Half-grid fields E_{k+1/2} sit at (k+1/2) dx; in the two */
/* electrode half cells the field is interpolated towards the surface field  */
/* given by Gauss' law.                                                      */
/* ------------------------------------------------------------------------ */
double or_gather64(int32_t N, double dx, const double *E, double e0_surf, double e_ground, double x) {
  double h = x / dx;
  if (h < 0.5) {
    double t = 2.0 * h;
    return (1.0 - t) * e0_surf + t * E[0];
  }
  if (h >= (double)N - 0.5) {
    double t = 2.0 * (h - ((double)N - 0.5));
    return (1.0 - t) * E[N - 1] + t * e_ground;
  }
  double hh = h - 0.5;
  int j = (int)floor(hh);
  double w1 = hh - (double)j;
  double w0 = 1.0 - w1;
  return w0 * E[j] + w1 * E[j + 1];
}

static double gather64(const or_sim *s, double x) {
  return or_gather64(s->N, s->dx, s->E, s->e0_surf, s->e_ground, x);
}

/* binary32 mode: position xi in cells, Ehat[0] = surface field at node 0,
 * Ehat[k] = E_{k-1/2} for k = 1..N, Ehat[N+1] = field at the grounded node */
float or_gather32(int32_t N, const float *ehat, float xi) {
  const float Nf = (float)N;
  int k;
  float t;
  if (xi < 0.5f) {
    k = 0;
    t = xi + xi;
  } else if (xi >= Nf - 0.5f) {
    k = N;
    t = xi - (Nf - 0.5f);
    t = t + t;
  } else {
    float h = xi - 0.5f;
    int j = (int)h;
    t = h - (float)j;
    k = j + 1;
  }
  float a = ehat[k];
  float b = ehat[k + 1];
  float dlt = b - a;
  float m = t * dlt;
  return a + m;
}

/* eq. vel_update_main and eq. pos_update_main for one binary32 particle in grid
 * units; the wall it reaches, if any (App. E: x <= 0 circuit, x >= N ground) */
int32_t or_push32(int32_t N, const float *ehat, float alpha, float xi, float u, float *xi_out, float *u_out) {
  const float Ep = or_gather32(N, ehat, xi);
  const float du = alpha * Ep;
  const float u1 = u + du;
  const float x1 = xi + u1;
  *xi_out = x1;
  *u_out = u1;
  if (x1 <= 0.0f) return 1;
  if (x1 >= (float)N) return 2;
  return 0;
}

float or_alpha32(const or_sim *s, int32_t species) { return s->alpha32[species & 1]; }

/* ------------------------------------------------------------------------ */
/* secondary emission for one absorbed ion (Alg. 2)                          */
/* ------------------------------------------------------------------------ */
/* The secondary electrons of one ion absorbed at `wall` (0 circuit, 1 ground)
 * in the push after level `step`, impact velocity v_ion [m/s] (Alg. 2): returns
 * their count and writes the first max_out of them (start and velocity, SI and
 * grid units). */
static int32_t see_draw(const or_sim *s, int64_t step, uint32_t ion_id, double v_ion, int wall, double *x_si,
                        double *v_si, float *xi, float *u, int32_t max_out) {
  const or_params *p = &s->p;
  if (p->see_amp <= 0.0) return 0;
  /* Alg. 2: the incident energy, the mean yield (clipped at zero), the count */
  double e_ion = 0.5 * p->mass[1] * v_ion * v_ion / p->ev; /* eV */
  double lam;
  if (p->see_yield == OR_YIELD_POLY) {
    double x = (e_ion < p->see_poly_Emax_eV ? e_ion : p->see_poly_Emax_eV) / 1000.0;
    double f = p->see_poly[5];
    for (int j = 4; j >= 0; --j) f = f * x + p->see_poly[j];
    lam = p->see_amp * (f > 0.0 ? f : 0.0);
  } else {
    double r = e_ion / p->see_E0_eV;
    lam = p->see_amp * r / (1.0 + r);
  }
  if (lam < 0.0) lam = 0.0;
  uint64_t blk[4];
  draw_block(p->seed, (uint64_t)step, (uint64_t)ion_id, 1, 0, blk);
  int32_t k = or_poisson_draw(lam, unit_open(blk[0]), p->see_max);
  /* the electrons' energies take the ion's stream words from 1 on, in order:
   * one per electron (fixed, exponential) or two (lognormal) */
  int32_t w = 1;
  for (int32_t e = 0; e < k && e < max_out; ++e) {
    double E_se;
    if (p->see_law == OR_SEE_LOGNORMAL) {
      if (w % 4 == 0) draw_block(p->seed, (uint64_t)step, (uint64_t)ion_id, 1, (uint64_t)(w / 4), blk);
      double u1 = unit_open(blk[w % 4]);
      w += 1;
      if (w % 4 == 0) draw_block(p->seed, (uint64_t)step, (uint64_t)ion_id, 1, (uint64_t)(w / 4), blk);
      double u2 = unit_open(blk[w % 4]);
      w += 1;
      double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
      E_se = exp(p->see_ln_mu + p->see_ln_sigma * z);
    } else {
      if (w % 4 == 0) draw_block(p->seed, (uint64_t)step, (uint64_t)ion_id, 1, (uint64_t)(w / 4), blk);
      double uu = unit_open(blk[w % 4]);
      w += 1;
      E_se = (p->see_law == OR_SEE_EXP) ? -p->see_E_eV * log(uu) : p->see_E_eV;
    }
    double v_se = sqrt(2.0 * E_se * p->ev / p->mass[0]);
    /* normal emission into the gap, starting on the surface */
    x_si[e] = wall == 0 ? 0.0 : p->d;
    v_si[e] = wall == 0 ? v_se : -v_se;
    xi[e] = wall == 0 ? 0.0f : (float)s->N;
    u[e] = (float)((v_si[e] * p->dt) / s->dx);
  }
  return k;
}

int32_t or_emit_sample(const or_sim *s, int64_t step, uint32_t ion_id, double v_ion, int32_t wall, float *xi,
                       float *u, int32_t max_out) {
  double xs[1024], vs[1024];
  if (max_out > 1024) max_out = 1024;
  return see_draw(s, step, ion_id, v_ion, wall, xs, vs, xi, u, max_out);
}

static void emit_electrons(or_sim *s, uint32_t ion_id, double v_ion, int wall, int64_t *n_emitted) {
  double xs[1024], vs[1024];
  float xi[1024], u[1024];
  const int32_t k = see_draw(s, s->step, ion_id, v_ion, wall, xs, vs, xi, u, 1024);
  for (int32_t e = 0; e < k && e < 1024; ++e) append(s, 0, xs[e], vs[e], xi[e], u[e], NO_ID);
  *n_emitted += k;
}

/* ------------------------------------------------------------------------ */
/* one time step                                                             */
/* ------------------------------------------------------------------------ */
/* beam ion k of the step that solves level `step` (Sec. 4.2 and the beam of
 * the workloads): energy uniform in [Emin, Emax] and depth below its entry
 * electrode from its own random block */
static void beam_ion(const or_params *p, double dx, int64_t step, int64_t k, double *x_out, double *v_out,
                     float *xi_out, float *u_out) {
  const double dt = p->dt;
  uint64_t blk[4];
  draw_block(p->seed, (uint64_t)step, (uint64_t)k, 2, 0, blk);
  double E = p->beam_Emin_eV + (p->beam_Emax_eV - p->beam_Emin_eV) * unit_open(blk[0]);
  double v = sqrt(2.0 * E * p->ev / p->mass[1]);
  double depth = unit_open(blk[1]) * (p->beam_layer > 0.0 ? p->beam_layer : v * dt);
  double x = (p->beam_side == 1) ? p->d - depth : depth;
  double uv = (v * dt) / dx;
  *x_out = x;
  *v_out = (p->beam_side == 1) ? -v : v;
  *xi_out = (float)(x / dx);
  *u_out = (float)((p->beam_side == 1) ? -uv : uv);
}

void or_beam_ion32(const or_sim *s, int64_t step, int64_t k, float *xi, float *u) {
  double x, v;
  beam_ion(&s->p, s->dx, step, k, &x, &v, xi, u);
}

int32_t or_step(or_sim *s, int32_t mode) {
  const or_params *p = &s->p;
  const int N = s->N;
  const double dx = s->dx, dt = p->dt;
  int rc = solve_level(s, mode);
  if (rc) return rc;

  if (p->fp32) {
    s->ehat[0] = (float)s->e0_surf;
    for (int k = 0; k < N; ++k) s->ehat[k + 1] = (float)s->E[k];
    s->ehat[N + 1] = (float)s->e_ground;
  }

  int64_t abs_n[2][2] = {{0, 0}, {0, 0}};
  int64_t emit_n[2] = {0, 0};
  /* absorbed ions that will emit, in storage order */
  int64_t n_old = s->n;
  uint32_t *hit_id = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n_old + 1));
  double *hit_v = (double *)malloc(sizeof(double) * (size_t)(n_old + 1));
  int *hit_wall = (int *)malloc(sizeof(int) * (size_t)(n_old + 1));
  int64_t n_hit = 0;

  int64_t w = 0; /* survivors are packed to the front, order kept */
  for (int64_t k = 0; k < n_old; ++k) {
    int sp = s->sp[k];
    int wall = -1;
    double v_new_si;
    if (!p->fp32) {
      /* eq. vel_update_main, eq. pos_update_main */
      double qm = (double)p->Z[sp] * p->q_unit / p->mass[sp];
      double Ep = gather64(s, s->x[k]);
      double v1 = s->v[k] + qm * dt * Ep;
      double x1 = s->x[k] + dt * v1;
      if (x1 <= 0.0) wall = 0;
      else if (x1 >= p->d) wall = 1;
      s->x[k] = x1;
      s->v[k] = v1;
      v_new_si = v1;
    } else {
      float x1, u1;
      wall = or_push32(N, s->ehat, s->alpha32[sp], s->xf[k], s->uf[k], &x1, &u1) - 1;
      s->xf[k] = x1;
      s->uf[k] = u1;
      v_new_si = (double)u1 * dx / dt;
    }
    if (wall >= 0) {
      abs_n[sp][wall] += 1;
      if (p->Z[sp] > 0) {
        hit_id[n_hit] = s->id[k];
        hit_v[n_hit] = v_new_si;
        hit_wall[n_hit] = wall;
        n_hit += 1;
      }
      continue;
    }
    if (w != k) {
      if (p->fp32) {
        s->xf[w] = s->xf[k];
        s->uf[w] = s->uf[k];
      } else {
        s->x[w] = s->x[k];
        s->v[w] = s->v[k];
      }
      s->sp[w] = s->sp[k];
      s->id[w] = s->id[k];
    }
    w += 1;
  }
  s->n = w;

  /* secondary electrons */
  for (int64_t h = 0; h < n_hit; ++h) {
    if (grow(s, s->n + p->see_max)) return -2;
    emit_electrons(s, hit_id[h], hit_v[h], hit_wall[h], &emit_n[hit_wall[h]]);
  }
  free(hit_id);
  free(hit_v);
  free(hit_wall);

  /* ion beam: the step's count, then each ion's energy and depth below its
   * entry electrode from its own random block */
  int64_t n_inj = p->beam_per_step;
  if (p->beam_schedule)
    n_inj = (s->step < p->beam_schedule_len) ? p->beam_schedule[s->step] : 0;
  if (n_inj > 0) {
    if (grow(s, s->n + n_inj)) return -2;
    for (int64_t k = 0; k < n_inj; ++k) {
      double x, vs;
      float xi, u;
      beam_ion(p, dx, s->step, k, &x, &vs, &xi, &u);
      append(s, 1, x, vs, xi, u, s->next_id);
      s->next_id += 1;
    }
  }

  /* convection charge at the circuit electrode over this step (Sec. 2.4.1):
   * charges that arrived, minus the charge the emitted electrons carried away */
  const double A = p->area;
  double qconv = 0.0;
  qconv += A * sheet_of(s, 1) * (double)abs_n[1][0];
  qconv += A * sheet_of(s, 0) * (double)abs_n[0][0];
  qconv -= A * sheet_of(s, 0) * (double)emit_n[0];
  s->qconv_pending = qconv;

  or_diag *D = &s->diag;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      D->abs_step[a][b] = abs_n[a][b];
      D->abs_cum[a][b] += abs_n[a][b];
    }
  for (int b = 0; b < 2; ++b) {
    D->emit_step[b] = emit_n[b];
    D->emit_cum[b] += emit_n[b];
  }
  D->inj_step = n_inj;
  D->inj_cum += n_inj;
  D->pushed_cum += n_old;
  s->step += 1;
  return 0;
}

int32_t or_step_external(or_sim *s, double v_star) {
  s->v_ext = v_star;
  return or_step(s, OR_WEAK_EXT);
}

double or_phi0_prev(const or_sim *s) {
  if (s->step == 0) {
    const double cgap = s->p.eps0 * s->p.area / s->p.d;
    return s->p.q0[s->p.gap_mesh] / (cgap + s->p.c_par);
  }
  return s->phi[0];
}

void or_get_diag(const or_sim *s, or_diag *out) {
  *out = s->diag;
  out->n_live[0] = or_count(s, 0);
  out->n_live[1] = or_count(s, 1);
}

void or_get_fields(const or_sim *s, double *phi, double *E, double *rho) {
  if (phi) memcpy(phi, s->phi, sizeof(double) * ((size_t)s->N + 1));
  if (E) memcpy(E, s->E, sizeof(double) * (size_t)s->N);
  if (rho) memcpy(rho, s->rho, sizeof(double) * ((size_t)s->N + 1));
}

int64_t or_count(const or_sim *s, int32_t species) {
  int64_t c = 0;
  for (int64_t k = 0; k < s->n; ++k) c += (s->sp[k] == species);
  return c;
}

int64_t or_get_particles(const or_sim *s, int32_t species, double *x, double *v, uint32_t *id) {
  int64_t c = 0;
  for (int64_t k = 0; k < s->n; ++k) {
    if (s->sp[k] != species) continue;
    if (s->p.fp32) {
      if (x) x[c] = (double)s->xf[k] * s->dx;
      if (v) v[c] = (double)s->uf[k] * s->dx / s->p.dt;
    } else {
      if (x) x[c] = s->x[k];
      if (v) v[c] = s->v[k];
    }
    if (id) id[c] = s->id[k];
    c += 1;
  }
  return c;
}

int64_t or_get_particles_f32(const or_sim *s, int32_t species, float *xi, float *u, uint32_t *id) {
  if (!s->p.fp32) return -1;
  int64_t c = 0;
  for (int64_t k = 0; k < s->n; ++k) {
    if (s->sp[k] != species) continue;
    if (xi) xi[c] = s->xf[k];
    if (u) u[c] = s->uf[k];
    if (id) id[c] = s->id[k];
    c += 1;
  }
  return c;
}
