// Host side of the C ABI (include/gapsim.h): parameter checks, the constant
// circuit matrices of each gap, device memory, launch orchestration, readback,
// the external circuit engine's step loop, the circuit's resonance (damped
// roots of the loop equations) and the time-step check, the autotuner.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "gs_internal.h"
#include "gs_mlp_dev.h"

using namespace gs;

static thread_local std::string g_init_error;

// Staging array of gs_inject_noalloc: x then v of at most GS_INJECT_NOALLOC_MAX
// particles, in binary64.  Every device the library runs on holds its own copy
// until the process ends; host code uses the address hipGetSymbolAddress gives
// for the current device (looked up once per device at context set-up), never
// the array's name.  All calls on one device share it.
static __device__ __align__(256) double scratch[2 * GS_INJECT_NOALLOC_MAX];
static std::mutex g_scratch_mu;
constexpr int SCRATCH_DEVS = 64;
static void *g_scratch_dev[SCRATCH_DEVS];

struct gs_ctx {
  int G = 0;
  int fp64 = 0;
  int nmax = 0;
  std::vector<gs_gap_params> params;
  std::vector<GapConst> hc;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;  // private stream graphs are captured on
  gs_allocator alloc{nullptr, nullptr, nullptr};
  std::vector<void *> blocks;
  std::vector<size_t> block_bytes;
  DevPtrs dp{};
  LaunchCfg lc{};
  int compact_every = 32;
  int since_compact = 0;
  int emits = 0;  // some gap has secondary emission
  int use_graph = 0;
  int timing = 0;
  double newton_tol = 1e-10;
  int newton_maxit = 8;
  int device = 0, ncu = 0;
  int deposit_opt = 0;  // 0 auto, 1 wide, 2 carry
  int grid_opt = 0;     // grid fixed by the caller
  int64_t steps_done = 0;
  int64_t epoch = 0;
  std::vector<int64_t> next_id;
  std::vector<std::vector<int64_t>> sched;  // per gap: copy of the beam schedule (empty: none)
  std::vector<int> sched_on;                // per gap: the schedule is in force
  double *ext_host = nullptr;               // pinned, mapped: [G] engine voltages, [G] field potentials,
                                            // then the lists' size the device last saw
  volatile unsigned long long *list_hint = nullptr;
  void *scratch = nullptr;                  // this device's staging array of gs_inject_noalloc
  hipEvent_t ext_ev = nullptr;              // recorded after each external-mode field solve
  std::string err;
  int sticky = 0;  // gs_status of a device error already seen
  // timing
  struct Pend {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Pend> pend;
  std::vector<hipEvent_t> pool;
  gs_timing tm{};
  // graph cache: one captured chunk of `compact_every` steps per (mode, guess)
  hipGraphExec_t gexec[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
  int gexec_len[2][3] = {{0, 0, 0}, {0, 0, 0}};
  // guess network
  uint16_t *mlp_w = nullptr;
  double *mlp_norm = nullptr;
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
static gs_status fail(gs_ctx *c, gs_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c)
    c->err = buf;
  else
    g_init_error = buf;
  return s;
}

#define HIPCHK(ctx, call)                                                                     \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return fail(ctx, GS_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));            \
  } while (0)

static void *dev_alloc(gs_ctx *c, size_t bytes) {
  if (bytes == 0) bytes = 16;
  void *p = nullptr;
  if (c->alloc.alloc) {
    p = c->alloc.alloc(bytes, c->alloc.user);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  if (p) {
    c->blocks.push_back(p);
    c->block_bytes.push_back(bytes);
  }
  return p;
}

static void dev_free_all(gs_ctx *c) {
  for (void *p : c->blocks) {
    if (c->alloc.release)
      c->alloc.release(p, c->alloc.user);
    else if (!c->alloc.alloc)
      (void)hipFree(p);
  }
  c->blocks.clear();
  c->block_bytes.clear();
}

// Gauss-Jordan inverse in extended precision; returns false if singular
static bool invert(int n, const long double *A, long double *Ainv) {
  long double a[(MAXM + 1) * 2 * (MAXM + 1)];
  const int w = 2 * n;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < w; ++j) a[i * w + j] = j < n ? A[i * n + j] : (j - n == i ? 1.0L : 0.0L);
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (fabsl(a[r * w + col]) > fabsl(a[piv * w + col])) piv = r;
    if (a[piv * w + col] == 0.0L || !std::isfinite((double)a[piv * w + col])) return false;
    if (piv != col)
      for (int j = 0; j < w; ++j) std::swap(a[col * w + j], a[piv * w + j]);
    long double d = a[col * w + col];
    for (int j = 0; j < w; ++j) a[col * w + j] /= d;
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      long double f = a[r * w + col];
      if (f == 0.0L) continue;
      for (int j = 0; j < w; ++j) a[r * w + j] -= f * a[col * w + j];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Ainv[i * n + j] = a[i * w + n + j];
  return true;
}

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

extern "C" gs_status gs_validate_params(const gs_gap_params *p, char *msg, size_t cap) {
  auto bad = [&](const char *m) {
    if (msg && cap) snprintf(msg, cap, "%s", m);
    return GS_EINVAL;
  };
  if (!p) return bad("params is NULL");
  if (p->particle_fp != 32 && p->particle_fp != 64) return bad("particle_fp must be 32 or 64");
  const int nlim = p->particle_fp == 32 ? 16384 : 8192;
  if (p->n_cells < 2 || p->n_cells > nlim) return bad("n_cells out of range (2..16384 fp32, 2..8192 fp64)");
  if (!finite_pos(p->d) || !finite_pos(p->area) || !finite_pos(p->eps0) || !finite_pos(p->dt))
    return bad("d, area, eps0 and dt must be finite and positive");
  for (int s = 0; s < 2; ++s) {
    if (p->Z[s] == 0 || p->Z[s] < -64 || p->Z[s] > 64) return bad("Z must be a nonzero integer in [-64, 64]");
    if (!finite_pos(p->mass[s])) return bad("masses must be finite and positive");
    if (p->capacity[s] < 0 || p->capacity[s] > (int64_t)0x7FFFFFFF) return bad("capacity out of range");
  }
  if (!finite_pos(p->q_unit) || !finite_pos(p->ev)) return bad("q_unit and ev must be positive");
  if (!std::isfinite(p->weight) || p->weight < 0) return bad("weight must be finite and >= 0");
  if (p->n_mesh < 1 || p->n_mesh > GS_MAX_MESH) return bad("n_mesh must be in 1..8");
  if (p->gap_mesh < 0 || p->gap_mesh >= p->n_mesh) return bad("gap_mesh out of range");
  if (!std::isfinite(p->c_par) || p->c_par < 0) return bad("c_par must be >= 0");
  for (int i = 0; i < p->n_mesh; ++i) {
    for (int j = 0; j < p->n_mesh; ++j)
      if (!std::isfinite(p->L[i][j]) || !std::isfinite(p->R[i][j]) || !std::isfinite(p->S[i][j]))
        return bad("circuit matrices must be finite");
    if (!std::isfinite(p->src[i]) || !std::isfinite(p->q0[i])) return bad("src and q0 must be finite");
  }
  if (!std::isfinite(p->src_dc) || !std::isfinite(p->src_amp) || !std::isfinite(p->src_freq) ||
      !std::isfinite(p->src_phase))
    return bad("source parameters must be finite");
  if (!std::isfinite(p->see_amp) || p->see_amp < 0) return bad("see_amp must be >= 0");
  if (!finite_pos(p->see_E0_eV)) return bad("see_E0_eV must be positive");
  if (p->see_law != GS_SEE_FIXED && p->see_law != GS_SEE_EXP && p->see_law != GS_SEE_LOGNORMAL)
    return bad("see_law must be FIXED, EXP or LOGNORMAL");
  if (p->see_yield != GS_YIELD_SATURATING && p->see_yield != GS_YIELD_POLY)
    return bad("see_yield must be SATURATING or POLY");
  for (int j = 0; j < 6; ++j)
    if (!std::isfinite(p->see_poly[j])) return bad("see_poly coefficients must be finite");
  if (p->see_yield == GS_YIELD_POLY && !finite_pos(p->see_poly_Emax_eV))
    return bad("see_poly_Emax_eV must be positive");
  if (p->see_law == GS_SEE_LOGNORMAL &&
      (!std::isfinite(p->see_ln_mu) || !std::isfinite(p->see_ln_sigma) || p->see_ln_sigma < 0))
    return bad("see_ln_mu must be finite and see_ln_sigma >= 0");
  if (p->see_max < 0 || p->see_max > 1024) return bad("see_max must be in 0..1024");
  if (!std::isfinite(p->see_E_eV) || p->see_E_eV < 0) return bad("see_E_eV must be >= 0");
  if (p->beam_per_step < 0 || p->beam_per_step > (int64_t)1 << 30) return bad("beam_per_step out of range");
  if (p->beam_side != GS_BEAM_CIRCUIT && p->beam_side != GS_BEAM_GROUND)
    return bad("beam_side must be GS_BEAM_CIRCUIT or GS_BEAM_GROUND");
  if (!std::isfinite(p->beam_layer) || p->beam_layer < 0 || !(p->beam_layer < p->d))
    return bad("beam_layer must be in [0, d)");
  bool any_beam = p->beam_per_step > 0;
  if (p->beam_schedule) {
    if (p->beam_schedule_len < 0 || p->beam_schedule_len > ((int64_t)1 << 26))
      return bad("beam_schedule_len out of range (0..2^26)");
    any_beam = false;
    for (int64_t i = 0; i < p->beam_schedule_len; ++i) {
      if (p->beam_schedule[i] < 0 || p->beam_schedule[i] > (int64_t)1 << 30)
        return bad("beam_schedule entries must be in 0..2^30");
      any_beam = any_beam || p->beam_schedule[i] > 0;
    }
  } else if (p->beam_schedule_len != 0) {
    return bad("beam_schedule is NULL but beam_schedule_len is not 0");
  }
  if (any_beam &&
      (!finite_pos(p->beam_Emin_eV) || !std::isfinite(p->beam_Emax_eV) || p->beam_Emax_eV < p->beam_Emin_eV))
    return bad("beam energies must satisfy 0 < Emin <= Emax");
  if (!finite_pos(p->v_ref)) return bad("v_ref must be positive");
  if (p->particle_fp == 64 && p->capacity[0] + p->capacity[1] > ((int64_t)1 << 19))
    return bad("particle_fp 64 holds at most 2^19 particles per gap (2^-44 weights in int64)");
  return GS_OK;
}

// constant per-gap data: grid, species, and the circuit matrices (extended precision)
static gs_status build_const(gs_ctx *ctx, int g, const gs_gap_params &p, GapConst &c) {
  memset(&c, 0, sizeof c);
  const int M = p.n_mesh;
  c.N = p.n_cells;
  c.M = M;
  c.g = p.gap_mesh;
  c.see_law = p.see_law;
  c.see_max = p.see_max;
  c.Z[0] = p.Z[0];
  c.Z[1] = p.Z[1];
  // with a schedule the per-step count is ignored (levels past it inject none)
  c.beam_n = p.beam_schedule ? 0 : p.beam_per_step;
  c.beam_side = p.beam_side;
  c.beam_layer = p.beam_layer;
  c.cap[0] = p.capacity[0];
  c.cap[1] = p.capacity[1];
  c.seed = p.seed;
  c.d = p.d;
  c.dx = p.d / (double)p.n_cells;
  c.A = p.area;
  c.eps0 = p.eps0;
  c.dt = p.dt;
  c.cgap = p.eps0 * p.area / p.d;
  c.c_par = p.c_par;
  c.s0 = p.weight * p.q_unit;
  for (int s = 0; s < 2; ++s) {
    // velocity change (cells per step) per V/m: Z q dt^2 / (m dx)
    c.alpha[s] = ((double)p.Z[s] * p.q_unit) * p.dt * p.dt / (p.mass[s] * c.dx);
    c.mass[s] = p.mass[s];
  }
  c.ev = p.ev;
  c.see_amp = p.see_amp;
  c.see_E0 = p.see_E0_eV;
  c.see_E = p.see_E_eV;
  c.see_yield = p.see_yield;
  for (int j = 0; j < 6; ++j) c.see_poly[j] = p.see_poly[j];
  c.see_pEmax = p.see_poly_Emax_eV;
  c.see_mu = p.see_ln_mu;
  c.see_sig = p.see_ln_sigma;
  c.beam_Emin = p.beam_Emin_eV;
  c.beam_Emax = p.beam_Emax_eV;
  c.v_ref = p.v_ref;
  c.src_dc = p.src_dc;
  c.src_amp = p.src_amp;
  c.src_w = 2.0 * M_PI * p.src_freq;
  c.src_phase = p.src_phase;

  // T' = 9 L / (4 dt^2) + 3 R / (2 dt) + S (gap row without the gap capacitor),
  // Tw = T' + e_g e_g^T / (C_gap + c_par) (gap as a capacitor, weak mode)
  const long double dt = p.dt;
  const long double cg = (long double)c.cgap + (long double)p.c_par;
  long double Tp[MAXM * MAXM], Tw[MAXM * MAXM], Ti[MAXM * MAXM], Twi[MAXM * MAXM];
  for (int i = 0; i < M; ++i)
    for (int j = 0; j < M; ++j) {
      Tp[i * M + j] = 9.0L * p.L[i][j] / (4.0L * dt * dt) + 3.0L * p.R[i][j] / (2.0L * dt) + p.S[i][j];
      Tw[i * M + j] = Tp[i * M + j] + ((i == c.g && j == c.g) ? 1.0L / cg : 0.0L);
    }
  if (!invert(M, Tp, Ti)) return fail(ctx, GS_EINVAL, "gap %d: strict circuit matrix is singular", g);
  if (!invert(M, Tw, Twi)) return fail(ctx, GS_EINVAL, "gap %d: circuit matrix is singular", g);
  for (int i = 0; i < M; ++i) {
    long double sb = 0, sz = 0, wb = 0;
    for (int j = 0; j < M; ++j) {
      long double aL = 0, aR = 0, aS = 0, bL = 0, bR = 0, bS = 0;
      for (int k = 0; k < M; ++k) {
        aL += Ti[i * M + k] * p.L[k][j];
        aR += Ti[i * M + k] * p.R[k][j];
        aS += Ti[i * M + k] * p.S[k][j];
        bL += Twi[i * M + k] * p.L[k][j];
        bR += Twi[i * M + k] * p.R[k][j];
        long double sw = p.S[k][j] + ((k == c.g && j == c.g) ? 1.0L / cg : 0.0L);
        bS += Twi[i * M + k] * sw;
      }
      c.sL[i * MAXM + j] = (double)(aL / (4.0L * dt * dt));
      c.sR[i * MAXM + j] = (double)(aR / (2.0L * dt));
      c.sS[i * MAXM + j] = (double)aS;
      c.wL[i * MAXM + j] = (double)(bL / (4.0L * dt * dt));
      c.wR[i * MAXM + j] = (double)(bR / (2.0L * dt));
      c.wS[i * MAXM + j] = (double)bS;
      c.Tp[i * MAXM + j] = (double)Tp[i * M + j];
      sb += Ti[i * M + j] * p.src[j];
      wb += Twi[i * M + j] * p.src[j];
    }
    sz = Ti[i * M + c.g];
    c.sb[i] = (double)sb;
    c.sz[i] = (double)sz;
    c.wb[i] = (double)wb;
  }
  // Newton Jacobian of r(u), u = (V, I_0..I_{M-1}) (see k_field)
  const int nu = M + 1;
  long double J[(MAXM + 1) * (MAXM + 1)], Ji[(MAXM + 1) * (MAXM + 1)];
  const long double vr = p.v_ref;
  const long double dfac = (long double)p.d / ((long double)p.eps0 * (long double)p.area);
  for (int i = 0; i < nu * nu; ++i) J[i] = 0;
  J[0] = (1.0L + dfac * p.c_par) / vr;
  J[0 * nu + 1 + c.g] = -dfac * (2.0L * dt / 3.0L) / vr;
  for (int i = 0; i < M; ++i) {
    J[(1 + i) * nu + 0] = (i == c.g ? 1.0L : 0.0L) / vr;
    for (int j = 0; j < M; ++j) J[(1 + i) * nu + 1 + j] = Tp[i * M + j] * (2.0L * dt / 3.0L) / vr;
  }
  if (!invert(nu, J, Ji)) return fail(ctx, GS_EINVAL, "gap %d: Newton Jacobian is singular", g);
  for (int i = 0; i < nu; ++i)
    for (int j = 0; j < nu; ++j) c.Jinv[i * (MAXM + 1) + j] = (double)Ji[i * nu + j];
  return GS_OK;
}

static void init_state(const gs_gap_params &p, const GapConst &c, GapState &s) {
  memset(&s, 0, sizeof s);
  s.level = -1;
  for (int j = 0; j < p.n_mesh; ++j) s.qprev[j] = p.q0[j];
  // the gap's share of the gap-mesh charge sits on the electrode
  const double qgap0 = p.q0[p.gap_mesh] * c.cgap / (c.cgap + p.c_par);
  s.qcirc_prev = qgap0;
  s.sigma_prev = qgap0 / p.area;
  const double v0 = p.q0[p.gap_mesh] / (c.cgap + p.c_par);
  for (int k = 0; k < 3; ++k) s.uh[k][0] = v0;
  s.newton_last = -1;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" const char *gs_version(void) { return "gapsim 0.1 (gfx950)"; }

extern "C" const char *gs_last_error(const gs_ctx *ctx) {
  return ctx ? ctx->err.c_str() : g_init_error.c_str();
}

static void choose_launch(gs_ctx *ctx);

static gs_status setup(gs_ctx *ctx) {
  const int G = ctx->G;
  ctx->hc.resize(G);
  size_t slots = 0, nodes = 0, etab = 0, events = 0, nsched = 0, bins = 0;
  ctx->nmax = 0;
  for (int g = 0; g < G; ++g) {
    gs_status st = build_const(ctx, g, ctx->params[g], ctx->hc[g]);
    if (st != GS_OK) return st;
    GapConst &c = ctx->hc[g];
    // regions start on 64-slot boundaries: the push moves particles with
    // 16-byte vector loads and stores
    auto pad = [](size_t v) { return (v + 63) / 64 * 64; };
    c.pbase[0] = (int64_t)slots;
    slots += pad((size_t)c.cap[0]);
    c.pbase[1] = (int64_t)slots;
    slots += pad((size_t)c.cap[1]);
    c.nbase = (int64_t)nodes;
    nodes += (size_t)c.N + 1;
    // absorbed-ion events of one push: up to an eighth of the ion slots
    c.evbase = (int64_t)events;
    c.evcap = (ctx->params[g].see_amp > 0.0) ? (int64_t)(c.cap[1] / 8 + 4096) : 0;
    events += (size_t)c.evcap;
    // field tables start on 16-byte boundaries (the push stages them with
    // 16-byte loads)
    c.ebase = (int64_t)etab;
    etab += ((size_t)c.N + 2 + 3) / 4 * 4;
    c.sched_base = (int64_t)nsched;
    c.sched_len = (int64_t)ctx->sched[g].size();
    nsched += ctx->sched[g].size();
    // cell-sort bin counters: room for the finest bin the option allows
    const size_t nbin = ((size_t)c.N + SORT_BIN_MIN - 1) / SORT_BIN_MIN;
    c.hbase[0] = (int64_t)bins;
    c.hbase[1] = (int64_t)(bins + nbin);
    bins += 2 * nbin;
    ctx->nmax = std::max(ctx->nmax, c.N);
  }
  const size_t ps = ctx->fp64 ? 8 : 4;
  DevPtrs &d = ctx->dp;
#define ALLOC(dst, type, count)                                                     \
  do {                                                                              \
    dst = (type)dev_alloc(ctx, (size_t)(count));                                    \
    if (!dst) return fail(ctx, GS_ENOMEM, "device allocation of %zu bytes failed", \
                          (size_t)(count));                                         \
  } while (0)
  for (int b = 0; b < 2; ++b) {
    ALLOC(d.X[b], void *, slots * ps);
    ALLOC(d.U[b], void *, slots * ps);
    ALLOC(d.ID[b], uint32_t *, slots * 4);
  }
  ALLOC(d.next_count, unsigned long long *, (size_t)G * 2 * 8);
  ALLOC(d.cursor, unsigned long long *, (size_t)G * 2 * 8);
  ALLOC(d.fill_h, unsigned long long *, (size_t)G * 2 * 8);
  // in-place compaction: a live bit per slot, and per-tile counters (a region
  // of cap slots has far fewer tiles of 65536 slots than words of 64), both
  // indexed from the region's pbase / 64
  ALLOC(d.tcnt, int *, (slots / 64 + 1) * 4);
  ALLOC(d.live, unsigned long long *, (slots / 64 + 1) * 8);
  ALLOC(d.wrank, int *, (slots / 64 + 1) * 4);
  ALLOC(d.tally, unsigned long long *, (size_t)G * T_N * 8);
  ALLOC(d.acc, unsigned long long *, nodes * 8);
  ALLOC(d.rho64, double *, nodes * 8);
  ALLOC(d.E64, double *, nodes * 8);
  ALLOC(d.phi64, double *, nodes * 8);
  ALLOC(d.fsl, double *, nodes * 8);
  ALLOC(d.fpart, double *, (size_t)G * NCHMAX * 2 * 8);
  ALLOC(d.foff, double *, (size_t)G * NCHMAX * 8);
  ALLOC(d.fsig, double *, (size_t)G * 8);
  ALLOC(d.ehat, void *, etab * ps);
  ALLOC(d.ev, Event *, events * sizeof(Event));
  ALLOC(d.ev_count, unsigned long long *, (size_t)G * 8);
  ALLOC(d.ev_done, unsigned long long *, (size_t)G * 8);
  ALLOC(d.hist, unsigned long long *, bins * 8);
  ALLOC(d.bcur, unsigned long long *, bins * 8);
  int64_t *sched_d = nullptr;
  ALLOC(sched_d, int64_t *, std::max<size_t>(nsched, 1) * 8);
  d.sched = sched_d;
  // exchange buffer of the external circuit engine: coherent pinned host memory
  // the field kernel reads and writes directly (16 bytes per gap), and the
  // word the push's tail or k_emit writes the lists' size to (16 bytes)
  {
    void *h = nullptr, *dptr = nullptr;
    const size_t nb = (size_t)G * 16 + 16;
    const hipError_t eh = hipHostMalloc(&h, nb, hipHostMallocMapped | hipHostMallocCoherent);
    if (eh != hipSuccess || !h)
      return fail(ctx, GS_ENOMEM, "pinned host allocation of %zu bytes failed: %s", nb, hipGetErrorString(eh));
    ctx->ext_host = (double *)h;
    memset(h, 0, nb);
    HIPCHK(ctx, hipHostGetDevicePointer(&dptr, h, 0));
    d.ext_v = (const double *)dptr;
    d.ext_phi = (double *)dptr + G;
    d.list_seen = (unsigned long long *)((char *)dptr + (size_t)G * 16);
    ctx->list_hint = (volatile unsigned long long *)((char *)h + (size_t)G * 16);
    HIPCHK(ctx, hipEventCreateWithFlags(&ctx->ext_ev, hipEventDisableTiming));
  }
  // overflow event regions for up to eight 256-thread push workgroups per CU
  // (the largest grid the autotuner tries), when any gap emits; each holds
  // 1/32768 of the emitting gaps' ion slots, within [OVQ_MIN, OVQ_MAX] (a
  // push that absorbs a few tenths of a percent of 2e8 ions stays within them)
  bool emits = false;
  int64_t ion_slots = 0;
  for (int g = 0; g < G; ++g)
    if (ctx->params[g].see_amp > 0.0) {
      emits = true;
      ion_slots += ctx->hc[g].cap[1];
    }
  {
    int dev = 0, ncu = 0;
    HIPCHK(ctx, hipGetDevice(&dev));
    HIPCHK(ctx, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    d.ovf_wgs = emits ? (int64_t)8 * std::max(ncu, 1) : 0;
    d.ovq = std::min<int64_t>(OVQ_MAX, std::max<int64_t>(OVQ_MIN, (ion_slots / 32768 + 255) / 256 * 256));
  }
  ctx->emits = emits ? 1 : 0;
  ALLOC(d.ovf, Event *, (size_t)std::max<int64_t>(d.ovf_wgs, 1) * (size_t)d.ovq * sizeof(Event));
  ALLOC(d.epoch, int64_t *, 8);
  ALLOC(d.err, unsigned int *, 8);
  ALLOC(d.steal, unsigned int *, 256);
  ALLOC(d.push_done, unsigned int *, 33 * 128);
  ALLOC(d.gc, const GapConst *, sizeof(GapConst) * (size_t)G);
  ALLOC(d.gs, GapState *, sizeof(GapState) * (size_t)G);
#undef ALLOC
  d.mlp_w = nullptr;
  d.mlp_norm = nullptr;
  d.rec_x = d.rec_y = nullptr;
  d.rec_cap = d.rec_level0 = 0;
  hipStream_t s = ctx->stream;
  std::vector<GapState> hs(G);
  for (int g = 0; g < G; ++g) init_state(ctx->params[g], ctx->hc[g], hs[g]);
  HIPCHK(ctx, hipMemcpyAsync((void *)d.gc, ctx->hc.data(), sizeof(GapConst) * G, hipMemcpyHostToDevice, s));
  HIPCHK(ctx, hipMemcpyAsync(d.gs, hs.data(), sizeof(GapState) * G, hipMemcpyHostToDevice, s));
  HIPCHK(ctx, hipMemsetAsync(d.next_count, 0, (size_t)G * 2 * 8, s));
  HIPCHK(ctx, hipMemsetAsync(d.cursor, 0, (size_t)G * 2 * 8, s));
  HIPCHK(ctx, hipMemsetAsync(d.tally, 0, (size_t)G * T_N * 8, s));
  HIPCHK(ctx, hipMemsetAsync(d.ev_count, 0, (size_t)G * 8, s));
  HIPCHK(ctx, hipMemsetAsync(d.ev_done, 0, (size_t)G * 8, s));
  HIPCHK(ctx, hipMemsetAsync(d.steal, 0, 256, s));
  HIPCHK(ctx, hipMemsetAsync(d.push_done, 0, 33 * 128, s));
  HIPCHK(ctx, hipMemsetAsync(d.hist, 0, bins * 8, s));
  HIPCHK(ctx, hipMemsetAsync(d.bcur, 0, bins * 8, s));
  for (int g = 0; g < G; ++g)
    if (!ctx->sched[g].empty())
      HIPCHK(ctx, hipMemcpyAsync(sched_d + ctx->hc[g].sched_base, ctx->sched[g].data(), ctx->sched[g].size() * 8,
                                 hipMemcpyHostToDevice, s));
  HIPCHK(ctx, hipMemsetAsync(d.acc, 0, nodes * 8, s));
  HIPCHK(ctx, hipMemsetAsync(d.rho64, 0, nodes * 8, s));
  HIPCHK(ctx, hipMemsetAsync(d.E64, 0, nodes * 8, s));
  HIPCHK(ctx, hipMemsetAsync(d.phi64, 0, nodes * 8, s));
  HIPCHK(ctx, hipMemsetAsync(d.epoch, 0, 8, s));
  const unsigned int err0[2] = {0u, 0xFFFFFFFFu};
  HIPCHK(ctx, hipMemcpyAsync(d.err, err0, 8, hipMemcpyHostToDevice, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  ctx->next_id.assign(G, 0);
  HIPCHK(ctx, hipGetDevice(&ctx->device));
  HIPCHK(ctx, hipDeviceGetAttribute(&ctx->ncu, hipDeviceAttributeMultiprocessorCount, ctx->device));
  ctx->lc.fp64 = ctx->fp64;
  ctx->lc.nmax = ctx->nmax;
  ctx->lc.block = 256;
  ctx->lc.tile = ctx->lc.block * 8;
  ctx->lc.wide = 1;
  ctx->lc.compact_grid = 4 * ctx->ncu;
  ctx->lc.ppt = ctx->fp64 ? 2 : 4;
  ctx->lc.sort_bin = 0;
  ctx->lc.steal = 0;
  ctx->lc.stream = 0;
  ctx->lc.masks = 0;
  ctx->lc.lists = 0;
  choose_launch(ctx);
  return GS_OK;
}

// LDS of one push workgroup (dynamic part plus the static prefix-scan buffer)
static size_t push_lds_total(const gs_ctx *ctx, int wide, int block) {
  return push_lds_bytes(ctx->nmax, ctx->fp64, ctx->G, wide) + (size_t)block * 4;
}

// the deposit-cell width (auto: 64-bit cells whenever the grid fits) and a
// persistent grid sized by LDS and thread occupancy
static void choose_launch(gs_ctx *ctx) {
  const size_t lds_cap = 163840;
  int wide = 1;
  if (!ctx->fp64) {
    if (ctx->deposit_opt == 2 || (ctx->deposit_opt == 0 && push_lds_total(ctx, 1, ctx->lc.block) > lds_cap))
      wide = 0;
  }
  ctx->lc.wide = wide;
  const size_t lds = push_lds_total(ctx, wide, ctx->lc.block);
  const int per_cu_lds = (int)std::max<size_t>(1, lds_cap / lds);
  const int per_cu_thr = std::max(1, 2048 / ctx->lc.block);
  if (!ctx->grid_opt) ctx->lc.grid = std::max(1, ctx->ncu * std::min(per_cu_lds, per_cu_thr));
}

static bool launch_fits(const gs_ctx *ctx) {
  return push_lds_total(ctx, ctx->lc.wide, ctx->lc.block) <= 163840;
}

// the staging array's address on the context's device (current during set-up)
static gs_status scratch_setup(gs_ctx *ctx) {
  if (ctx->device < 0 || ctx->device >= SCRATCH_DEVS)
    return fail(ctx, GS_EDEVICE, "device %d: no staging array slot", ctx->device);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[ctx->device]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(ctx, GS_EDEVICE, "hipGetSymbolAddress(staging array): %s", hipGetErrorString(e));
    g_scratch_dev[ctx->device] = ptr;
  }
  ctx->scratch = g_scratch_dev[ctx->device];
  return GS_OK;
}

extern "C" gs_status gs_init_gap(gs_ctx **out, int32_t n_gaps, const gs_gap_params *params,
                             const gs_allocator *alloc, void *hip_stream) {
  if (!out) return fail(nullptr, GS_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_gaps < 1 || n_gaps > 16384 || !params) return fail(nullptr, GS_EINVAL, "n_gaps must be in 1..16384");
  char msg[256];
  for (int g = 0; g < n_gaps; ++g) {
    if (gs_validate_params(&params[g], msg, sizeof msg) != GS_OK)
      return fail(nullptr, GS_EINVAL, "gap %d: %s", g, msg);
    if (params[g].particle_fp != params[0].particle_fp)
      return fail(nullptr, GS_EINVAL, "all gaps of a context share particle_fp");
  }
  if (alloc && (!alloc->alloc || !alloc->release))
    return fail(nullptr, GS_EINVAL, "allocator needs both alloc and release");
  gs_ctx *ctx = new (std::nothrow) gs_ctx();
  if (!ctx) return fail(nullptr, GS_ENOMEM, "out of host memory");
  ctx->G = n_gaps;
  ctx->fp64 = params[0].particle_fp == 64;
  ctx->params.assign(params, params + n_gaps);
  // the schedules are copied; the caller keeps its arrays
  ctx->sched.assign(n_gaps, std::vector<int64_t>());
  ctx->sched_on.assign(n_gaps, 0);
  for (int g = 0; g < n_gaps; ++g) {
    if (params[g].beam_schedule) {
      ctx->sched_on[g] = 1;
      ctx->sched[g].assign(params[g].beam_schedule, params[g].beam_schedule + params[g].beam_schedule_len);
    }
    ctx->params[g].beam_schedule = nullptr;
    ctx->params[g].beam_schedule_len = 0;
  }
  ctx->stream = (hipStream_t)hip_stream;
  if (alloc) ctx->alloc = *alloc;
  int nm = 0;
  for (int g = 0; g < n_gaps; ++g) nm = std::max(nm, params[g].n_cells);
  const size_t lds = push_lds_bytes(nm, ctx->fp64, n_gaps, ctx->fp64) + 256 * 4;
  if (lds > 163840) {
    delete ctx;
    return fail(nullptr, GS_EINVAL, "grid of %d cells with %d gaps exceeds the 160 KiB LDS budget", nm, n_gaps);
  }
  gs_status st = setup(ctx);
  if (st == GS_OK) st = scratch_setup(ctx);
  if (st != GS_OK) {
    g_init_error = ctx->err;
    if (ctx->ext_ev) (void)hipEventDestroy(ctx->ext_ev);
    if (ctx->ext_host) (void)hipHostFree(ctx->ext_host);
    dev_free_all(ctx);
    delete ctx;
    return st;
  }
  *out = ctx;
  return GS_OK;
}

extern "C" void gs_destroy(gs_ctx *ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  for (auto &pe : ctx->pend) {
    (void)hipEventDestroy(pe.a);
    (void)hipEventDestroy(pe.b);
  }
  for (hipEvent_t e : ctx->pool) (void)hipEventDestroy(e);
  for (int m = 0; m < 2; ++m)
    for (int k = 0; k < 3; ++k)
      if (ctx->gexec[m][k]) (void)hipGraphExecDestroy(ctx->gexec[m][k]);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  if (ctx->ext_ev) (void)hipEventDestroy(ctx->ext_ev);
  if (ctx->ext_host) (void)hipHostFree(ctx->ext_host);
  dev_free_all(ctx);
  delete ctx;
}

static gs_status check_sticky(gs_ctx *ctx, bool sync) {
  if (ctx->sticky) return (gs_status)ctx->sticky;
  if (!sync) return GS_OK;
  unsigned int e[2];
  HIPCHK(ctx, hipMemcpyAsync(e, ctx->dp.err, 8, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  if (e[0] & ERR_CAPACITY) {
    ctx->sticky = GS_ECAPACITY;
    return fail(ctx, GS_ECAPACITY, "gap %u ran out of particle slots", e[1]);
  }
  if (e[0] & ERR_BADINJECT) {
    ctx->sticky = GS_EINVAL;
    return fail(ctx, GS_EINVAL, "an injected position was outside [0, d]");
  }
  if (e[0] & ERR_NOCONV) {
    // reported once: the state stays valid (the last iterate was used)
    const unsigned int keep = e[0] & ~(unsigned int)ERR_NOCONV;
    HIPCHK(ctx, hipMemcpyAsync(ctx->dp.err, &keep, 4, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return fail(ctx, GS_ENOCONV, "a strict Newton solve missed its tolerance within its iteration cap");
  }
  return GS_OK;
}

extern "C" gs_status gs_inject(gs_ctx *ctx, int32_t gap, int32_t species, int64_t n, const double *x,
                               const double *v, int32_t ptr_is_device) {
  if (!ctx) return GS_ESTATE;
  if (gap < 0 || gap >= ctx->G || species < 0 || species > 1 || n < 0)
    return fail(ctx, GS_EINVAL, "bad gap, species or count");
  if (n == 0) return GS_OK;
  if (!x || !v) return fail(ctx, GS_EINVAL, "x and v must not be NULL");
  gs_status st = check_sticky(ctx, false);
  if (st != GS_OK) return st;
  const double d = ctx->params[gap].d;
  const double *xd = x, *vd = v;
  void *tmp = nullptr;
  if (!ptr_is_device) {
    for (int64_t i = 0; i < n; ++i)
      if (!(x[i] >= 0.0 && x[i] <= d) || !std::isfinite(v[i]))
        return fail(ctx, GS_EINVAL, "particle %lld: x outside [0, d] or v not finite", (long long)i);
    HIPCHK(ctx, hipMalloc(&tmp, (size_t)n * 16));
    HIPCHK(ctx, hipMemcpyAsync(tmp, x, (size_t)n * 8, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync((char *)tmp + (size_t)n * 8, v, (size_t)n * 8, hipMemcpyHostToDevice, ctx->stream));
    xd = (const double *)tmp;
    vd = (const double *)((char *)tmp + (size_t)n * 8);
  }
  hipError_t e = launch_inject(ctx->dp, gap, species, n, xd, vd, ctx->next_id[gap], ctx->fp64, ctx->stream);
  ctx->next_id[gap] += n;
  if (tmp) {
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(tmp);
  }
  if (e != hipSuccess) return fail(ctx, GS_EDEVICE, "inject launch: %s", hipGetErrorString(e));
  return check_sticky(ctx, true);
}

extern "C" gs_status gs_inject_noalloc(gs_ctx *ctx, int32_t gap, int32_t species, int64_t n, const double *x,
                                       const double *v) {
  if (!ctx) return GS_ESTATE;
  if (gap < 0 || gap >= ctx->G || species < 0 || species > 1 || n < 0)
    return fail(ctx, GS_EINVAL, "bad gap, species or count");
  if (n > GS_INJECT_NOALLOC_MAX)
    return fail(ctx, GS_EINVAL, "gs_inject_noalloc takes at most %d particles per call (got %lld)",
                GS_INJECT_NOALLOC_MAX, (long long)n);
  if (n == 0) return GS_OK;
  if (!x || !v) return fail(ctx, GS_EINVAL, "x and v must not be NULL");
  if (!ctx->scratch) return fail(ctx, GS_ESTATE, "no staging array on this context's device");
  gs_status st = check_sticky(ctx, false);
  if (st != GS_OK) return st;
  const double d = ctx->params[gap].d;
  for (int64_t i = 0; i < n; ++i)
    if (!(x[i] >= 0.0 && x[i] <= d) || !std::isfinite(v[i]))
      return fail(ctx, GS_EINVAL, "particle %lld: x outside [0, d] or v not finite", (long long)i);
  double *xs = (double *)ctx->scratch;
  double *vs = xs + n;
  HIPCHK(ctx, hipMemcpyAsync(xs, x, (size_t)n * 8, hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(ctx, hipMemcpyAsync(vs, v, (size_t)n * 8, hipMemcpyHostToDevice, ctx->stream));
  hipError_t e = launch_inject(ctx->dp, gap, species, n, xs, vs, ctx->next_id[gap], ctx->fp64, ctx->stream);
  ctx->next_id[gap] += n;
  if (e != hipSuccess) return fail(ctx, GS_EDEVICE, "inject launch: %s", hipGetErrorString(e));
  // synchronises: the staging array is free again when the call returns
  return check_sticky(ctx, true);
}

static hipEvent_t ev_get(gs_ctx *ctx) {
  if (!ctx->pool.empty()) {
    hipEvent_t e = ctx->pool.back();
    ctx->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

// Runs launch(t); when timing is on, t carries two events that the kernel's
// own dispatch packets record, so the elapsed time is the kernel's alone.
// Timing level 2 instruments the push only: an evented launch leaves the queue
// idle for some microseconds around it, which level 2 confines to one launch a
// step.
template <class F>
static hipError_t timed(gs_ctx *ctx, int kind, F &&launch) {
  if (!ctx->timing || (ctx->timing == 2 && kind != 0)) return launch(KTime{});
  KTime t;
  t.a = ev_get(ctx);
  t.b = ev_get(ctx);
  hipError_t e = launch(t);
  ctx->pend.push_back({kind, t.a, t.b});
  return e;
}

// beam ions of the step that solves level n (the host's copy of what the
// field kernel hands the push)
static int64_t beam_at(const gs_ctx *ctx, int g, int64_t n) {
  if (!ctx->sched_on[g]) return ctx->params[g].beam_per_step;
  const std::vector<int64_t> &s = ctx->sched[g];
  return n >= 0 && n < (int64_t)s.size() ? s[(size_t)n] : 0;
}

// The push, and the emission of every absorbed ion in the same step, so the
// emitted counts of a level never lag: the ions a push workgroup absorbs past
// what it can emit itself (its LDS queue and overflow region) wait in the
// gap's list.  The push's last workgroup emits the lists when the last push
// seen left none (the usual case: the overflow regions are sized for the
// step's impacts); when it left some (impacts concentrated in a few
// workgroups), k_emit emits them with many workgroups after the push, which
// costs less than the fences and the serial passes of one workgroup.  The
// size read here is a step or two old (the device writes it to host memory):
// either way every list is emitted within its step.  With the cell sort on, a
// wall's impacts sit in few workgroups: the push then keeps only its LDS
// queue, and k_emit emits the long lists.  (A captured graph keeps the choice
// made when it was captured.)
// masks: a compaction follows this push (the push then writes the live masks)
static hipError_t launch_push_emit(gs_ctx *ctx, hipStream_t s, bool timing, bool masks) {
  DevPtrs dp = ctx->dp;
  if (ctx->lc.sort_bin > 0) dp.ovf_wgs = 0;
  LaunchCfg lc = ctx->lc;
  lc.masks = masks && lc.sort_bin == 0;
  const bool listed = ctx->list_hint && *ctx->list_hint != 0ull;
  lc.lists = ctx->emits && lc.sort_bin == 0 && lc.grid < 65536 && !listed;
  auto push = [&](KTime t) { return launch_push(dp, ctx->G, lc, s, t); };
  hipError_t e = timing ? timed(ctx, 0, push) : push(KTime{});
  if (e != hipSuccess || !ctx->emits || lc.lists) return e;
  auto emit = [&](KTime t) { return launch_emit(ctx->dp, ctx->G, ctx->fp64, std::max(ctx->ncu, 1), s, t); };
  return timing ? timed(ctx, 3, emit) : emit(KTime{});
}

// the compaction (after a push that wrote the live masks), or the cell sort in
// its place
static hipError_t launch_reclaim(gs_ctx *ctx, hipStream_t s, KTime t) {
  LaunchCfg lc = ctx->lc;
  lc.masks = 1;
  return lc.sort_bin > 0 ? launch_sort(ctx->dp, ctx->G, lc, s, t) : launch_compact(ctx->dp, ctx->G, lc, s, t);
}

// after_field: an event to record between the field solve and the push
static gs_status one_step(gs_ctx *ctx, int mode, int guess, hipEvent_t after_field = nullptr) {
  hipError_t e = timed(ctx, 1, [&](KTime t) {
    return launch_field(ctx->dp, ctx->G, mode, guess, ctx->newton_tol, ctx->newton_maxit, ctx->fp64,
                        ctx->nmax, ctx->stream, t);
  });
  if (e != hipSuccess) return fail(ctx, GS_EDEVICE, "field launch: %s", hipGetErrorString(e));
  if (after_field && (e = hipEventRecord(after_field, ctx->stream)) != hipSuccess)
    return fail(ctx, GS_EDEVICE, "event record: %s", hipGetErrorString(e));
  e = launch_push_emit(ctx, ctx->stream, true, ctx->since_compact + 1 >= ctx->compact_every);
  if (e != hipSuccess) return fail(ctx, GS_EDEVICE, "push launch: %s", hipGetErrorString(e));
  ctx->since_compact += 1;
  if (ctx->since_compact >= ctx->compact_every) {
    e = timed(ctx, 2, [&](KTime t) { return launch_reclaim(ctx, ctx->stream, t); });
    if (e != hipSuccess) return fail(ctx, GS_EDEVICE, "compact launch: %s", hipGetErrorString(e));
    ctx->since_compact = 0;
    ctx->epoch += 1;
  }
  ctx->steps_done += 1;
  for (int g = 0; g < ctx->G; ++g) ctx->next_id[g] += beam_at(ctx, g, ctx->steps_done - 1);
  return GS_OK;
}

static gs_status run_steps(gs_ctx *ctx, int n_steps, int mode, int guess) {
  if (!ctx) return GS_ESTATE;
  if (n_steps < 0) return fail(ctx, GS_EINVAL, "n_steps < 0");
  gs_status st = check_sticky(ctx, false);
  if (st != GS_OK) return st;
  int left = n_steps;
  // graph replay: whole chunks that start right after a compaction
  if (ctx->use_graph && !ctx->timing) {
    while (left > 0 && ctx->since_compact != 0) {
      if ((st = one_step(ctx, mode, guess)) != GS_OK) return st;
      --left;
    }
    const int L = ctx->compact_every;
    while (left >= L) {
      hipGraphExec_t &ge = ctx->gexec[mode][guess];
      if (!ge || ctx->gexec_len[mode][guess] != L) {
        if (ge) (void)hipGraphExecDestroy(ge);
        ge = nullptr;
        // capture on a private stream (the caller's may be the legacy default
        // stream, which cannot be captured); replay on the caller's stream
        if (!ctx->cap_stream) HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
        hipStream_t cs = ctx->cap_stream;
        hipGraph_t graph = nullptr;
        HIPCHK(ctx, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        hipError_t e1 = hipSuccess, e2 = hipSuccess, e3 = hipSuccess;
        for (int k = 0; k < L && e1 == hipSuccess && e2 == hipSuccess; ++k) {
          e1 = launch_field(ctx->dp, ctx->G, mode, guess, ctx->newton_tol, ctx->newton_maxit, ctx->fp64,
                            ctx->nmax, cs);
          if (e1 == hipSuccess) e2 = launch_push_emit(ctx, cs, false, k == L - 1);
        }
        if (e1 == hipSuccess && e2 == hipSuccess) e3 = launch_reclaim(ctx, cs, KTime{});
        hipError_t ec = hipStreamEndCapture(cs, &graph);
        if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || ec != hipSuccess || !graph) {
          if (graph) (void)hipGraphDestroy(graph);
          return fail(ctx, GS_EDEVICE, "graph capture failed (%s)",
                      hipGetErrorString(e1 != hipSuccess ? e1 : e2 != hipSuccess ? e2 : e3 != hipSuccess ? e3 : ec));
        }
        hipError_t ei = hipGraphInstantiate(&ge, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) return fail(ctx, GS_EDEVICE, "graph instantiate: %s", hipGetErrorString(ei));
        ctx->gexec_len[mode][guess] = L;
      }
      HIPCHK(ctx, hipGraphLaunch(ge, ctx->stream));
      left -= L;
      ctx->steps_done += L;
      ctx->epoch += 1;
      for (int g = 0; g < ctx->G; ++g)
        for (int64_t n = ctx->steps_done - L; n < ctx->steps_done; ++n) ctx->next_id[g] += beam_at(ctx, g, n);
    }
  }
  while (left > 0) {
    if ((st = one_step(ctx, mode, guess)) != GS_OK) return st;
    --left;
  }
  return GS_OK;
}

extern "C" gs_status gs_step_strict(gs_ctx *ctx, int32_t n_steps, int32_t guess) {
  if (!ctx) return GS_ESTATE;
  if (guess < GS_GUESS_DIRECT || guess > GS_GUESS_MLP) return fail(ctx, GS_EINVAL, "bad guess mode");
  if (guess == GS_GUESS_MLP) {
    if (!ctx->mlp_w) return fail(ctx, GS_ESTATE, "no guess network weights (gs_mlp_set_weights)");
    for (int g = 0; g < ctx->G; ++g)
      if (ctx->hc[g].M != 2)
        return fail(ctx, GS_EINVAL, "gap %d: the guess network needs a two-mesh circuit (u = V, I_0, I_1)", g);
  }
  return run_steps(ctx, n_steps, 0, guess);
}

extern "C" gs_status gs_step_weak(gs_ctx *ctx, int32_t n_steps) {
  if (!ctx) return GS_ESTATE;
  return run_steps(ctx, n_steps, 1, GS_GUESS_DIRECT);
}

extern "C" gs_status gs_step_weak_external(gs_ctx *ctx, int32_t n_steps, gs_circuit_fn fn, void *user) {
  if (!ctx) return GS_ESTATE;
  if (!fn || n_steps < 0) return fail(ctx, GS_EINVAL, "fn is NULL or n_steps < 0");
  gs_status st = check_sticky(ctx, false);
  if (st != GS_OK) return st;
  const int G = ctx->G;
  double *vh = ctx->ext_host, *ph = ctx->ext_host + G;
  std::vector<double> phi((size_t)G);
  for (int k = 0; k < n_steps; ++k) {
    const int64_t n = ctx->steps_done;  // the level this step solves
    if (n == 0) {
      // before the first level the electrode holds the gap mesh's initial charge
      for (int g = 0; g < G; ++g) {
        const GapConst &c = ctx->hc[g];
        phi[g] = ctx->params[g].q0[c.g] / (c.cgap + c.c_par);
      }
      if ((st = check_sticky(ctx, true)) != GS_OK) return st;
    } else if (k == 0) {
      // the last level may come from any kind of step: read the gap states
      HIPCHK(ctx, hipMemcpy2DAsync(phi.data(), 8, &ctx->dp.gs[0].phi0, sizeof(GapState), 8, (size_t)G,
                                   hipMemcpyDeviceToHost, ctx->stream));
      if ((st = check_sticky(ctx, true)) != GS_OK) return st;
    } else {
      // the previous field solve wrote its potentials to the exchange buffer;
      // its push may still run while the engine works
      HIPCHK(ctx, hipEventSynchronize(ctx->ext_ev));
      for (int g = 0; g < G; ++g) phi[g] = ph[g];
    }
    // the field kernel that read vh last has finished (stream or event wait above)
    for (int g = 0; g < G; ++g) {
      double v = 0.0;
      const int32_t rc = fn(user, g, n, ctx->hc[g].dt, phi[g], &v);
      if (rc != 0)
        return fail(ctx, GS_ECALLBACK, "circuit engine returned %d for gap %d at level %lld; step not taken", rc, g,
                    (long long)n);
      if (!std::isfinite(v))
        return fail(ctx, GS_EINVAL, "circuit engine gave a non-finite gap voltage for gap %d at level %lld", g,
                    (long long)n);
      vh[g] = v;
    }
    if ((st = one_step(ctx, 2, GS_GUESS_DIRECT, ctx->ext_ev)) != GS_OK) return st;
  }
  return GS_OK;
}

// ---------------------------------------------------------------------------
// circuit resonance (App. D, circuit-resolution constraint)
// ---------------------------------------------------------------------------
typedef std::complex<double> cplx;

// Eigenvalues of a real n x n matrix (row-major, n <= 2 MAXM): diagonal
// balancing by powers of two (Parlett and Reinsch), Householder reduction to
// Hessenberg form, then single-shift complex QR steps with Givens rotations
// (Wilkinson shift from the trailing 2 x 2 block, an ad hoc shift after 10
// and 20 steps without deflation), deflating one eigenvalue at a time.
// Returns false when some eigenvalue did not converge in 60 steps.
static bool eigenvalues(int n, double *A, cplx *ev) {
  auto at = [&](int i, int j) -> double & { return A[i * n + j]; };
  for (bool changed = true; changed;) {
    changed = false;
    for (int i = 0; i < n; ++i) {
      double c = 0.0, r = 0.0;
      for (int j = 0; j < n; ++j)
        if (j != i) {
          c += std::fabs(at(j, i));
          r += std::fabs(at(i, j));
        }
      if (c == 0.0 || r == 0.0) continue;
      const double s0 = c + r;
      double f = 1.0;
      while (c < 0.5 * r) {
        c *= 2.0;
        r *= 0.5;
        f *= 2.0;
      }
      while (c >= 2.0 * r) {
        c *= 0.5;
        r *= 2.0;
        f *= 0.5;
      }
      if (c + r < 0.95 * s0) {
        changed = true;
        for (int j = 0; j < n; ++j) at(j, i) *= f;
        for (int j = 0; j < n; ++j) at(i, j) /= f;
      }
    }
  }
  // Hessenberg: reflect x = A[k+1.., k] onto a multiple of e_1
  double v[2 * MAXM];
  for (int k = 0; k + 2 < n; ++k) {
    double nx = 0.0;
    for (int i = k + 1; i < n; ++i) nx += at(i, k) * at(i, k);
    nx = std::sqrt(nx);
    if (nx == 0.0) continue;
    const double a0 = at(k + 1, k);
    for (int i = k + 1; i < n; ++i) v[i] = at(i, k);
    v[k + 1] = a0 + (a0 >= 0.0 ? nx : -nx);
    double vv = 0.0;
    for (int i = k + 1; i < n; ++i) vv += v[i] * v[i];
    for (int j = 0; j < n; ++j) {  // A <- (I - 2 v v^T / vv) A
      double d = 0.0;
      for (int i = k + 1; i < n; ++i) d += v[i] * at(i, j);
      d *= 2.0 / vv;
      for (int i = k + 1; i < n; ++i) at(i, j) -= d * v[i];
    }
    for (int i = 0; i < n; ++i) {  // A <- A (I - 2 v v^T / vv)
      double d = 0.0;
      for (int j = k + 1; j < n; ++j) d += at(i, j) * v[j];
      d *= 2.0 / vv;
      for (int j = k + 1; j < n; ++j) at(i, j) -= d * v[j];
    }
    for (int i = k + 2; i < n; ++i) at(i, k) = 0.0;
  }
  cplx H[2 * MAXM][2 * MAXM];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) H[i][j] = cplx(at(i, j), 0.0);
  const double eps = 2.220446049250313e-16;
  for (int m = n; m > 0;) {  // H[0..m) is the active block
    if (m == 1) {
      ev[0] = H[0][0];
      break;
    }
    int its = 0;
    for (;;) {
      if (std::abs(H[m - 1][m - 2]) <= eps * (std::abs(H[m - 1][m - 1]) + std::abs(H[m - 2][m - 2]))) break;
      if (its == 60) return false;
      // shift: the eigenvalue of the trailing 2 x 2 block nearer its last entry
      cplx mu;
      if (its == 10 || its == 20) {
        mu = H[m - 1][m - 1] + cplx(0.75 * std::abs(H[m - 1][m - 2]), 0.0);
      } else {
        const cplx a = H[m - 2][m - 2], b = H[m - 2][m - 1], c = H[m - 1][m - 2], d = H[m - 1][m - 1];
        const cplx hlf = 0.5 * (a - d), disc = std::sqrt(hlf * hlf + b * c);
        const cplx l1 = d + hlf + disc, l2 = d + hlf - disc;
        mu = std::abs(l1 - d) < std::abs(l2 - d) ? l1 : l2;
      }
      ++its;
      // H - mu I = Q R by Givens rotations on rows (k, k+1); then H = R Q + mu I
      cplx gc[2 * MAXM], gs[2 * MAXM];
      for (int i = 0; i < m; ++i) H[i][i] -= mu;
      for (int k = 0; k + 1 < m; ++k) {
        const cplx x = H[k][k], y = H[k + 1][k];
        const double r = std::sqrt(std::norm(x) + std::norm(y));
        cplx c(1.0, 0.0), s(0.0, 0.0);
        if (r > 0.0) {
          c = x / r;
          s = y / r;
        }
        gc[k] = c;
        gs[k] = s;
        for (int j = k; j < m; ++j) {  // [c* s*; -s c] applied to rows k, k+1
          const cplx p = H[k][j], q = H[k + 1][j];
          H[k][j] = std::conj(c) * p + std::conj(s) * q;
          H[k + 1][j] = -s * p + c * q;
        }
      }
      for (int k = 0; k + 1 < m; ++k) {  // columns k, k+1 times the adjoint rotation
        const cplx c = gc[k], s = gs[k];
        const int top = std::min(k + 2, m - 1);
        for (int i = 0; i <= top; ++i) {
          const cplx p = H[i][k], q = H[i][k + 1];
          H[i][k] = p * c + q * s;
          H[i][k + 1] = -p * std::conj(s) + q * std::conj(c);
        }
      }
      for (int i = 0; i < m; ++i) H[i][i] += mu;
    }
    ev[m - 1] = H[m - 1][m - 1];
    --m;
  }
  return true;
}

// Highest ringing angular frequency of a gap's circuit: the largest |Im lambda|
// over the finite roots of det(lambda^2 L + lambda R + S') = 0, S' = S plus the
// gap element's elastance 1 / (C_gap + c_par) in the gap mesh (the free
// response of L q'' + R q' + S' q = 0).  L, R and S' may all be singular, so
// the roots come from a shifted and inverted pencil: with a real shift s that
// is not a root, P(s + 1/mu) = 0 exactly when mu is an eigenvalue of the
// companion matrix [[0, I], [-P(s)^-1 L, -P(s)^-1 (2 s L + R)]]; mu = 0
// belongs to infinite roots (so do roots more than 1e6 times farther from s
// than the nearest one).  0 when no root oscillates.
static gs_status circuit_resonance(const gs_gap_params &p, double *omega) {
  const int M = p.n_mesh, n = 2 * M;
  const double cgap = p.eps0 * p.area / p.d;
  double S[MAXM][MAXM], Ln = 0.0, Rn = 0.0, Sn = 0.0;
  for (int i = 0; i < M; ++i)
    for (int j = 0; j < M; ++j) {
      S[i][j] = p.S[i][j];
      if (i == p.gap_mesh && j == p.gap_mesh) S[i][j] += 1.0 / (cgap + p.c_par);
      Ln = std::max(Ln, std::fabs(p.L[i][j]));
      Rn = std::max(Rn, std::fabs(p.R[i][j]));
      Sn = std::max(Sn, std::fabs(S[i][j]));
    }
  *omega = 0.0;
  // no inductance, or nothing for it to ring against: no oscillating root
  if (Ln == 0.0 || (Sn == 0.0 && Rn == 0.0)) return GS_OK;
  // shift of the size of the roots: the LC (else RL) rate of the largest entries
  const double s0 = Sn > 0.0 ? -std::sqrt(Sn / Ln) : -Rn / Ln;
  static const double tries[] = {1.0, 1.37, 0.61, 2.9, 0.23};
  for (double f : tries) {
    const double s = s0 * f;
    // P(s) and its LU factors with partial pivoting
    double P[MAXM][MAXM], Rs[MAXM][MAXM];
    int piv[MAXM];
    double pmax = 0.0;
    for (int i = 0; i < M; ++i)
      for (int j = 0; j < M; ++j) {
        P[i][j] = s * s * p.L[i][j] + s * p.R[i][j] + S[i][j];
        Rs[i][j] = 2.0 * s * p.L[i][j] + p.R[i][j];
        pmax = std::max(pmax, std::fabs(P[i][j]));
      }
    bool singular = false;
    for (int k = 0; k < M && !singular; ++k) {
      int r = k;
      for (int i = k + 1; i < M; ++i)
        if (std::fabs(P[i][k]) > std::fabs(P[r][k])) r = i;
      if (!(std::fabs(P[r][k]) > 1e-12 * pmax)) {
        singular = true;
        break;
      }
      piv[k] = r;
      if (r != k)
        for (int j = 0; j < M; ++j) std::swap(P[k][j], P[r][j]);
      for (int i = k + 1; i < M; ++i) {
        P[i][k] /= P[k][k];
        for (int j = k + 1; j < M; ++j) P[i][j] -= P[i][k] * P[k][j];
      }
    }
    if (singular) continue;
    auto solve = [&](double *b) {
      // whole rows (multipliers included) were swapped: permute b first
      for (int k = 0; k < M; ++k) std::swap(b[k], b[piv[k]]);
      for (int k = 0; k < M; ++k)
        for (int i = k + 1; i < M; ++i) b[i] -= P[i][k] * b[k];
      for (int k = M - 1; k >= 0; --k) {
        for (int j = k + 1; j < M; ++j) b[k] -= P[k][j] * b[j];
        b[k] /= P[k][k];
      }
    };
    double K[4 * MAXM * MAXM];
    for (int i = 0; i < n * n; ++i) K[i] = 0.0;
    for (int i = 0; i < M; ++i) K[i * n + M + i] = 1.0;
    for (int j = 0; j < M; ++j) {
      double a[MAXM], b[MAXM];
      for (int i = 0; i < M; ++i) {
        a[i] = p.L[i][j];
        b[i] = Rs[i][j];
      }
      solve(a);
      solve(b);
      for (int i = 0; i < M; ++i) {
        K[(M + i) * n + j] = -a[i];
        K[(M + i) * n + M + j] = -b[i];
      }
    }
    cplx mu[2 * MAXM];
    if (!eigenvalues(n, K, mu)) continue;
    double mmax = 0.0;
    for (int i = 0; i < n; ++i) mmax = std::max(mmax, std::abs(mu[i]));
    // mu = 0 (an infinite root) can sit in a Jordan block of size two (a loop
    // of capacitors without inductance), which rounding splits by about
    // sqrt(eps) of the spectrum: take |mu| below 1e-6 of the largest as infinite
    double w = 0.0;
    for (int i = 0; i < n; ++i)
      if (std::abs(mu[i]) > 1e-6 * mmax) w = std::max(w, std::fabs((1.0 / mu[i]).imag()));
    *omega = w;
    return GS_OK;
  }
  return GS_EINVAL;
}

extern "C" gs_status gs_circuit_resonance(const gs_gap_params *p, double *omega_max) {
  if (!p || !omega_max) return GS_EINVAL;
  char msg[256];
  if (gs_validate_params(p, msg, sizeof msg) != GS_OK) return GS_EINVAL;
  return circuit_resonance(*p, omega_max);
}

extern "C" gs_status gs_dt_check(gs_ctx *ctx, int32_t gap, gs_dt_report *out) {
  if (!ctx) return GS_ESTATE;
  if (gap < 0 || gap >= ctx->G || !out) return fail(ctx, GS_EINVAL, "bad gap or out is NULL");
  gs_status st = check_sticky(ctx, true);
  if (st != GS_OK) return st;
  const GapConst &c = ctx->hc[gap];
  const gs_gap_params &p = ctx->params[gap];
  const size_t bytes = 16 + (size_t)c.N * 4;
  void *buf = nullptr;
  if (hipMalloc(&buf, bytes) != hipSuccess) return fail(ctx, GS_ENOMEM, "time-step check: %zu bytes", bytes);
  unsigned long long um[2] = {0ull, 0ull};
  std::vector<unsigned int> cells((size_t)c.N);
  GapState s;
  hipError_t e = hipMemsetAsync(buf, 0, bytes, ctx->stream);
  if (e == hipSuccess)
    e = launch_dt_scan(ctx->dp, gap, c.N, ctx->fp64, (unsigned long long *)buf, (unsigned int *)((char *)buf + 16),
                       ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(um, buf, 16, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(cells.data(), (char *)buf + 16, (size_t)c.N * 4, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&s, ctx->dp.gs + gap, sizeof s, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  (void)hipFree(buf);
  if (e != hipSuccess) return fail(ctx, GS_EDEVICE, "time-step check: %s", hipGetErrorString(e));
  gs_dt_report r;
  memset(&r, 0, sizeof r);
  r.dt = p.dt;
  if (circuit_resonance(p, &r.omega_max) != GS_OK)
    return fail(ctx, GS_EINVAL, "gap %d: the circuit's roots could not be found", gap);
  r.n_omega = r.omega_max > 0.0 ? 1.0 / (r.omega_max * p.dt) : INFINITY;
  for (int sp = 0; sp < 2; ++sp) {
    double u;
    if (ctx->fp64) {
      memcpy(&u, &um[sp], 8);
    } else {
      const uint32_t b = (uint32_t)um[sp];
      float f;
      memcpy(&f, &b, 4);
      u = (double)f;
    }
    r.beta[sp] = u;
    r.v_max[sp] = u * c.dx / p.dt;
  }
  unsigned int cmax = 0;
  for (unsigned int k : cells) cmax = std::max(cmax, k);
  r.n_e_max = (double)cmax * p.weight / c.dx;
  const double qe = p.q_unit * std::fabs((double)p.Z[0]);
  r.omega_pe = std::sqrt(r.n_e_max * qe * qe / (p.eps0 * p.mass[0]));
  r.alpha = r.omega_pe * p.dt;
  const double qprev = s.qcirc_star - s.qcirc_step;
  const double qref = std::max(std::fabs(s.qcirc_star), std::fabs(qprev));
  r.eta = qref > 0.0 ? std::fabs(s.qcirc_step) / qref : 0.0;
  r.flags = (r.n_omega < 20.0 ? 1 : 0) | (r.beta[0] > 0.5 || r.beta[1] > 0.5 ? 2 : 0) | (r.alpha > 0.2 ? 4 : 0) |
            (r.eta > 0.2 ? 8 : 0);
  *out = r;
  return GS_OK;
}

extern "C" gs_status gs_read_diagnostics(gs_ctx *ctx, int32_t gap, gs_diag *out, double *phi, double *E,
                                         double *rho) {
  if (!ctx) return GS_ESTATE;
  if (gap < 0 || gap >= ctx->G || !out) return fail(ctx, GS_EINVAL, "bad gap or out is NULL");
  const GapConst &c = ctx->hc[gap];
  GapState s;
  unsigned long long tl[T_N], nc[2];
  hipStream_t st = ctx->stream;
  if (phi) {
    hipError_t e = launch_phi(ctx->dp, gap, st);
    if (e != hipSuccess) return fail(ctx, GS_EDEVICE, "phi launch: %s", hipGetErrorString(e));
  }
  HIPCHK(ctx, hipMemcpyAsync(&s, ctx->dp.gs + gap, sizeof s, hipMemcpyDeviceToHost, st));
  HIPCHK(ctx, hipMemcpyAsync(tl, ctx->dp.tally + (size_t)gap * T_N, sizeof tl, hipMemcpyDeviceToHost, st));
  HIPCHK(ctx, hipMemcpyAsync(nc, ctx->dp.next_count + gap * 2, sizeof nc, hipMemcpyDeviceToHost, st));
  const size_t nn = (size_t)c.N + 1;
  if (phi) HIPCHK(ctx, hipMemcpyAsync(phi, ctx->dp.phi64 + c.nbase, nn * 8, hipMemcpyDeviceToHost, st));
  if (E) HIPCHK(ctx, hipMemcpyAsync(E, ctx->dp.E64 + c.nbase, (nn - 1) * 8, hipMemcpyDeviceToHost, st));
  if (rho) HIPCHK(ctx, hipMemcpyAsync(rho, ctx->dp.rho64 + c.nbase, nn * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(ctx, hipStreamSynchronize(st));
  memset(out, 0, sizeof *out);
  out->step = s.level;
  out->t = s.t;
  out->phi0 = s.phi0;
  out->sigma = s.sigma;
  out->qcirc = s.qcirc;
  out->qcirc_star = s.qcirc_star;
  out->qconv = s.qconv;
  out->e_ground = s.e_ground;
  for (int j = 0; j < c.M; ++j) {
    out->q[j] = s.q[j];
    out->I[j] = s.I[j];
  }
  // the last push's tallies are folded into the state by the next field solve;
  // combine them here
  const long long ab[4] = {(long long)tl[T_ABS], (long long)tl[T_ABS + 1], (long long)tl[T_ABS + 2],
                           (long long)tl[T_ABS + 3]};
  const long long em[2] = {(long long)tl[T_EMIT], (long long)tl[T_EMIT + 1]};
  for (int sp = 0; sp < 2; ++sp)
    for (int w = 0; w < 2; ++w) {
      out->abs_step[sp][w] = ab[sp * 2 + w];
      out->abs_cum[sp][w] = s.abs_cum[sp * 2 + w] + ab[sp * 2 + w];
    }
  for (int w = 0; w < 2; ++w) {
    out->emit_step[w] = em[w];
    out->emit_cum[w] = s.emit_cum[w] + em[w];
  }
  out->inj_step = (long long)tl[T_INJ];
  out->inj_cum = s.inj_cum + (long long)tl[T_INJ];
  out->pushed_cum = s.pushed_cum + (long long)tl[T_PUSHED];
  out->n_live[0] = s.live[0] + em[0] + em[1] - ab[0] - ab[1];
  out->n_live[1] = s.live[1] + (long long)tl[T_INJ] - ab[2] - ab[3];
  out->n_slots[0] = (long long)nc[0];
  out->n_slots[1] = (long long)nc[1];
  out->newton_last = s.newton_last;
  out->newton_fallback_last = s.newton_fb_last;
  out->newton_total = s.newton_total;
  out->newton_fallbacks = s.newton_fallbacks;
  out->newton_max = s.newton_max;
  out->newton_levels = s.newton_levels;
  out->newton_resid0 = s.newton_r0;
  out->newton_resid = s.newton_r;
  for (int j = 0; j <= c.M; ++j) out->newton_guess[j] = s.guess[j];
  for (int j = 0; j < 3; ++j) out->mlp_proposal[j] = s.mlp_prop[j];
  out->qcirc_step = s.qcirc_step;
  out->q_space = s.q_space;
  return check_sticky(ctx, true);
}

extern "C" gs_status gs_read_particles(gs_ctx *ctx, int32_t gap, int32_t species, void *xi, void *u,
                                       uint32_t *id, int64_t max_n, int64_t *n_out) {
  if (!ctx) return GS_ESTATE;
  if (gap < 0 || gap >= ctx->G || species < 0 || species > 1 || max_n < 0)
    return fail(ctx, GS_EINVAL, "bad gap, species or max_n");
  const GapConst &c = ctx->hc[gap];
  unsigned long long nc = 0;
  int64_t ep = 0;
  HIPCHK(ctx, hipMemcpyAsync(&nc, ctx->dp.next_count + gap * 2 + species, 8, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipMemcpyAsync(&ep, ctx->dp.epoch, 8, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  const int sel = (int)(ep & 1);
  const size_t n = std::min<size_t>((size_t)nc, (size_t)c.cap[species]);
  const size_t ps = ctx->fp64 ? 8 : 4;
  std::vector<unsigned char> hx(n * ps), hu(n * ps);
  std::vector<uint32_t> hid(n);
  const size_t off = (size_t)c.pbase[species];
  if (n) {
    HIPCHK(ctx, hipMemcpy(hx.data(), (char *)ctx->dp.X[sel] + off * ps, n * ps, hipMemcpyDeviceToHost));
    HIPCHK(ctx, hipMemcpy(hu.data(), (char *)ctx->dp.U[sel] + off * ps, n * ps, hipMemcpyDeviceToHost));
    HIPCHK(ctx, hipMemcpy(hid.data(), ctx->dp.ID[sel] + off, n * 4, hipMemcpyDeviceToHost));
  }
  int64_t live = 0;
  for (size_t i = 0; i < n; ++i) {
    const bool alive = ctx->fp64 ? ((double *)hx.data())[i] >= 0.0 : ((float *)hx.data())[i] >= 0.0f;
    if (!alive) continue;
    if (live < max_n) {
      if (xi) memcpy((char *)xi + live * ps, hx.data() + i * ps, ps);
      if (u) memcpy((char *)u + live * ps, hu.data() + i * ps, ps);
      if (id) id[live] = hid[i];
    }
    ++live;
  }
  if (n_out) *n_out = live;
  return check_sticky(ctx, true);
}

// ---------------------------------------------------------------------------
// Newton guess network
// ---------------------------------------------------------------------------
// Captured graphs hold the device pointer block by value: drop them when it changes.
static void drop_graphs(gs_ctx *ctx) {
  for (int m = 0; m < 2; ++m)
    for (int k = 0; k < 3; ++k) {
      if (ctx->gexec[m][k]) (void)hipGraphExecDestroy(ctx->gexec[m][k]);
      ctx->gexec[m][k] = nullptr;
      ctx->gexec_len[m][k] = 0;
    }
}

// binary32 -> bfloat16 bits, round to nearest, ties to even (NaN kept quiet)
static uint16_t to_bf16(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

extern "C" gs_status gs_mlp_set_weights(gs_ctx *ctx, const float *theta, int64_t n, const double *norm) {
  if (!ctx) return GS_ESTATE;
  if (!theta || !norm || n != MLP_NPARAM)
    return fail(ctx, GS_EINVAL, "theta must hold %d values and norm %d", MLP_NPARAM, MLP_NORM);
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(theta[i])) return fail(ctx, GS_EINVAL, "theta[%lld] is not finite", (long long)i);
  for (int i = 0; i < MLP_NORM; ++i) {
    const bool scale = (i >= MLP_IN && i < 2 * MLP_IN) || i >= 2 * MLP_IN + MLP_OUT;
    if (!std::isfinite(norm[i]) || (scale && !(norm[i] > 0.0)))
      return fail(ctx, GS_EINVAL, "norm[%d] must be finite (and positive for a scale)", i);
  }
  std::vector<uint16_t> wb((size_t)n);
  for (int64_t i = 0; i < n; ++i) wb[(size_t)i] = to_bf16(theta[i]);
  if (!ctx->mlp_w) {
    ctx->mlp_w = (uint16_t *)dev_alloc(ctx, sizeof(uint16_t) * MLP_NPARAM);
    ctx->mlp_norm = (double *)dev_alloc(ctx, sizeof(double) * MLP_NORM);
    if (!ctx->mlp_w || !ctx->mlp_norm) return fail(ctx, GS_ENOMEM, "guess network weights");
  }
  HIPCHK(ctx, hipMemcpyAsync(ctx->mlp_w, wb.data(), sizeof(uint16_t) * MLP_NPARAM, hipMemcpyHostToDevice,
                             ctx->stream));
  HIPCHK(ctx, hipMemcpyAsync(ctx->mlp_norm, norm, sizeof(double) * MLP_NORM, hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  ctx->dp.mlp_w = ctx->mlp_w;
  ctx->dp.mlp_norm = ctx->mlp_norm;
  drop_graphs(ctx);
  return GS_OK;
}

extern "C" gs_status gs_mlp_forward(gs_ctx *ctx, const float *x, int64_t n, float *y) {
  if (!ctx) return GS_ESTATE;
  if (!ctx->mlp_w) return fail(ctx, GS_ESTATE, "no guess network weights (gs_mlp_set_weights)");
  if (n < 0 || (n > 0 && (!x || !y))) return fail(ctx, GS_EINVAL, "bad x, y or n");
  if (n == 0) return GS_OK;
  hipError_t e = launch_mlp_forward(ctx->mlp_w, x, n, y, ctx->stream);
  if (e != hipSuccess) return fail(ctx, GS_EDEVICE, "guess network launch: %s", hipGetErrorString(e));
  return GS_OK;
}

extern "C" gs_status gs_mlp_record(gs_ctx *ctx, float *x, float *y, int64_t capacity) {
  if (!ctx) return GS_ESTATE;
  if (capacity < 0) return fail(ctx, GS_EINVAL, "capacity < 0");
  if (!x || !y || capacity == 0) {
    ctx->dp.rec_x = ctx->dp.rec_y = nullptr;
    ctx->dp.rec_cap = 0;
  } else {
    ctx->dp.rec_x = x;
    ctx->dp.rec_y = y;
    ctx->dp.rec_cap = capacity;
    ctx->dp.rec_level0 = ctx->steps_done;
  }
  drop_graphs(ctx);
  return GS_OK;
}

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------
namespace {
struct HostCounters {
  int64_t epoch, steps_done;
  int since_compact;
  std::vector<int64_t> next_id;
};

std::string tune_key(const gs_ctx *ctx, int mode, int guess, long long live) {
  int lg = 0;
  while ((1ll << (lg + 1)) <= live) ++lg;
  std::ostringstream k;
  // (v2: lines carry the pool share after the sort bin)
  k << "v3,G=" << ctx->G << ",nmax=" << ctx->nmax << ",fp=" << (ctx->fp64 ? 64 : 32) << ",mode=" << mode
    << ",guess=" << guess << ",log2live=" << lg << ",cu=" << ctx->ncu;
  return k.str();
}
}  // namespace

static void apply_tuning(gs_ctx *ctx, const gs_tuning &t) {
  ctx->lc.block = t.block;
  ctx->lc.ppt = t.ppt * (ctx->fp64 ? 2 : 4);
  ctx->lc.tile = t.tile;
  ctx->deposit_opt = t.deposit;
  ctx->grid_opt = 1;
  ctx->lc.grid = t.grid;
  ctx->compact_every = t.compact_every;
  ctx->lc.sort_bin = t.sort_bin;
  ctx->lc.steal = t.steal;
  ctx->lc.stream = t.stream;
  choose_launch(ctx);
  ctx->lc.grid = t.grid;
  drop_graphs(ctx);
}

static gs_tuning current_tuning(const gs_ctx *ctx) {
  gs_tuning t{};
  t.block = ctx->lc.block;
  t.tile = ctx->lc.tile;
  t.grid = ctx->lc.grid;
  t.ppt = ctx->lc.ppt / (ctx->fp64 ? 2 : 4);
  t.deposit = ctx->deposit_opt;
  t.compact_every = ctx->compact_every;
  t.sort_bin = ctx->lc.sort_bin;
  t.steal = ctx->lc.steal;
  t.stream = ctx->lc.stream;
  return t;
}

extern "C" gs_status gs_get_launch(const gs_ctx *ctx, gs_tuning *out) {
  if (!ctx || !out) return GS_ESTATE;
  *out = current_tuning(ctx);
  return GS_OK;
}

extern "C" gs_status gs_autotune(gs_ctx *ctx, int32_t mode, int32_t guess, int32_t trial_steps,
                                 const char *cache_path, gs_tuning *out) {
  if (!ctx) return GS_ESTATE;
  if (mode != 0 && mode != 1) return fail(ctx, GS_EINVAL, "mode must be 0 (strict) or 1 (weak)");
  if (guess < GS_GUESS_DIRECT || guess > GS_GUESS_MLP || (mode == 1 && guess != GS_GUESS_DIRECT))
    return fail(ctx, GS_EINVAL, "bad guess mode");
  if (guess == GS_GUESS_MLP && !ctx->mlp_w) return fail(ctx, GS_ESTATE, "no guess network weights");
  if (trial_steps < 1 || trial_steps > 4096) return fail(ctx, GS_EINVAL, "trial_steps must be in 1..4096");
  gs_status st = check_sticky(ctx, true);
  if (st != GS_OK) return st;
  // live particles (for the cache key)
  long long live = 0;
  {
    std::vector<GapState> hs(ctx->G);
    HIPCHK(ctx, hipMemcpy(hs.data(), ctx->dp.gs, sizeof(GapState) * ctx->G, hipMemcpyDeviceToHost));
    for (const GapState &s : hs) live += s.live[0] + s.live[1];
  }
  const std::string key = tune_key(ctx, mode, guess, live);
  if (cache_path && *cache_path) {
    std::ifstream f(cache_path);
    std::string line;
    while (std::getline(f, line)) {
      const size_t bar = line.find('|');
      if (bar == std::string::npos || line.substr(0, bar) != key) continue;
      gs_tuning t{};
      std::istringstream v(line.substr(bar + 1));
      if (v >> t.block >> t.tile >> t.grid >> t.ppt >> t.deposit >> t.compact_every >> t.sort_bin >> t.steal >>
          t.stream >> t.ms_per_step) {
        const LaunchCfg keep = ctx->lc;
        apply_tuning(ctx, t);
        if (!launch_fits(ctx)) {
          ctx->lc = keep;
          continue;
        }
        if (out) *out = t;
        return GS_OK;
      }
    }
  }
  // snapshot every device block and the host counters; trials run on the
  // live state and it is put back afterwards
  std::vector<void *> backup(ctx->blocks.size(), nullptr);
  auto free_backup = [&]() {
    for (void *b : backup)
      if (b) (void)hipFree(b);
  };
  for (size_t i = 0; i < ctx->blocks.size(); ++i) {
    if (hipMalloc(&backup[i], ctx->block_bytes[i]) != hipSuccess) {
      backup[i] = nullptr;
      free_backup();
      return fail(ctx, GS_ENOMEM, "autotune: no device memory for a snapshot of the state");
    }
    if (hipMemcpyAsync(backup[i], ctx->blocks[i], ctx->block_bytes[i], hipMemcpyDeviceToDevice, ctx->stream) !=
        hipSuccess) {
      free_backup();
      return fail(ctx, GS_EDEVICE, "autotune: snapshot copy failed");
    }
  }
  const HostCounters hc0{ctx->epoch, ctx->steps_done, ctx->since_compact, ctx->next_id};
  const LaunchCfg lc0 = ctx->lc;
  const int dep0 = ctx->deposit_opt, grid_opt0 = ctx->grid_opt, ce0 = ctx->compact_every;
  const int sb0 = ctx->lc.sort_bin;
  const int graph0 = ctx->use_graph, timing0 = ctx->timing;
  float *rx = ctx->dp.rec_x, *ry = ctx->dp.rec_y;
  ctx->dp.rec_x = ctx->dp.rec_y = nullptr;  // trials record nothing
  ctx->use_graph = 0;
  ctx->timing = 0;
  auto restore = [&]() -> gs_status {
    for (size_t i = 0; i < ctx->blocks.size(); ++i)
      HIPCHK(ctx, hipMemcpyAsync(ctx->blocks[i], backup[i], ctx->block_bytes[i], hipMemcpyDeviceToDevice,
                                 ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    ctx->epoch = hc0.epoch;
    ctx->steps_done = hc0.steps_done;
    ctx->since_compact = hc0.since_compact;
    ctx->next_id = hc0.next_id;
    return GS_OK;
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  // time one candidate: warm-up steps, then `steps` timed steps, from the snapshot
  // (reclaim_first: the first warm-up step ends with a compaction or sort, so
  // that the timed steps see particles in the order that choice keeps)
  auto trial = [&](const gs_tuning &t, int steps, double *ms, bool reclaim_first) -> gs_status {
    gs_status r = restore();
    if (r != GS_OK) return r;
    apply_tuning(ctx, t);
    if (!launch_fits(ctx)) {
      *ms = 1e300;
      return GS_OK;
    }
    if (reclaim_first) ctx->since_compact = t.compact_every - 1;
    for (int k = 0; k < 2; ++k)
      if ((r = one_step(ctx, mode, guess)) != GS_OK) return r;
    HIPCHK(ctx, hipEventRecord(e0, ctx->stream));
    for (int k = 0; k < steps; ++k)
      if ((r = one_step(ctx, mode, guess)) != GS_OK) return r;
    HIPCHK(ctx, hipEventRecord(e1, ctx->stream));
    HIPCHK(ctx, hipEventSynchronize(e1));
    float f = 0.f;
    HIPCHK(ctx, hipEventElapsedTime(&f, e0, e1));
    *ms = f / steps;
    return check_sticky(ctx, true);
  };
  gs_tuning best{};
  best.ms_per_step = 1e300;
  const int vper = ctx->fp64 ? 2 : 4;
  gs_status r = GS_OK;
  // launch shape first, with each particle stream (the best shape depends on
  // it), at the current compaction interval and sort setting
  for (int block : {256, 512, 768, 1024})
    for (int ppt : {1, 2})
      for (int tmul : {8, 32})
        for (int per_cu : {1, 2, 3, 4, 8})  // 256-thread workgroups per CU
          for (int sm = 0; sm <= (ctx->fp64 ? 1 : 3); ++sm) {
            if (r != GS_OK) break;
            gs_tuning t{};
            t.block = block;
            t.ppt = ppt;
            t.tile = block * tmul;
            if (t.tile % (block * ppt * vper)) continue;
            // the same threads per CU at other block sizes
            if (per_cu * 256 < block) continue;
            t.deposit = dep0;
            t.grid = std::max(1, ctx->ncu * per_cu * 256 / block);
            t.compact_every = ce0;
            t.sort_bin = sb0;
            t.stream = sm;
            double ms = 0;
            if ((r = trial(t, trial_steps, &ms, false)) != GS_OK) break;
            t.ms_per_step = ms;
            if (ms < best.ms_per_step) best = t;
          }
  // then the compaction interval and the cell sort (off, or bins of 16, 64 or
  // 256 cells), over a span that holds several compactions or sorts: the
  // sort's cost is amortised over the interval and its gain shows in the
  // pushes that follow it
  if (r == GS_OK) {
    const gs_tuning base = best;
    best.ms_per_step = 1e300;
    for (int sb : {0, 16, 64, 256})
      for (int ce : {16, 32, 64}) {
        if (sb && sort_lds_bytes(ctx->G, ctx->nmax, sb) > 163840) continue;
        if (sb && (ctx->nmax + sb - 1) / sb < 2) continue;  // one bin: nothing to sort
        gs_tuning t = base;
        t.compact_every = ce;
        t.sort_bin = sb;
        double ms = 0;
        if ((r = trial(t, std::max(trial_steps, 2 * ce), &ms, true)) != GS_OK) break;
        t.ms_per_step = ms;
        if (ms < best.ms_per_step) best = t;
      }
  }
  // then the share of tiles that go to the push's pool (off, a quarter, an
  // eighth), over the same span
  if (r == GS_OK) {
    const gs_tuning base = best;
    best.ms_per_step = 1e300;
    for (int k : {0, 4, 8}) {
      gs_tuning t = base;
      t.steal = k;
      double ms = 0;
      if ((r = trial(t, std::max(trial_steps, 2 * t.compact_every), &ms, true)) != GS_OK) break;
      t.ms_per_step = ms;
      if (ms < best.ms_per_step) best = t;
    }
  }
  // then the particle stream: round-robin tile order (no pool with it) and
  // non-temporal accesses (binary32), at the two tile sizes of the shape stage.
  // These candidates differ by a few per cent, so each is timed twice (the
  // second pass in reverse order) and keeps its faster time
  if (r == GS_OK) {
    const gs_tuning base = best;
    std::vector<gs_tuning> cand;
    for (int sm = 0; sm <= (ctx->fp64 ? 1 : 3); ++sm)
      for (int tmul : {8, 32}) {
        gs_tuning t = base;
        t.stream = sm;
        if (sm & STREAM_RR) t.steal = 0;
        t.tile = t.block * tmul;
        if (t.tile % (t.block * t.ppt * vper)) continue;
        t.ms_per_step = 1e300;
        cand.push_back(t);
      }
    for (int pass = 0; pass < 2 && r == GS_OK; ++pass)
      for (size_t k = 0; k < cand.size(); ++k) {
        gs_tuning &t = cand[pass ? cand.size() - 1 - k : k];
        double ms = 0;
        if ((r = trial(t, std::max(trial_steps, 2 * t.compact_every), &ms, true)) != GS_OK) break;
        t.ms_per_step = std::min(t.ms_per_step, ms);
      }
    // (the shape stage's own choice is among the candidates, re-timed)
    if (r == GS_OK) {
      best.ms_per_step = 1e300;
      for (const gs_tuning &t : cand)
        if (t.ms_per_step < best.ms_per_step) best = t;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  gs_status rr = restore();
  free_backup();
  ctx->dp.rec_x = rx;
  ctx->dp.rec_y = ry;
  ctx->use_graph = graph0;
  ctx->timing = timing0;
  if (r != GS_OK || rr != GS_OK || best.ms_per_step >= 1e299) {
    ctx->lc = lc0;
    ctx->deposit_opt = dep0;
    ctx->grid_opt = grid_opt0;
    ctx->compact_every = ce0;
    ctx->lc.sort_bin = sb0;
    drop_graphs(ctx);
    if (r != GS_OK) return r;
    if (rr != GS_OK) return rr;
    return fail(ctx, GS_EINVAL, "autotune: no candidate launch fits");
  }
  apply_tuning(ctx, best);
  if (cache_path && *cache_path) {
    std::ofstream f(cache_path, std::ios::app);
    f << key << "|" << best.block << " " << best.tile << " " << best.grid << " " << best.ppt << " " << best.deposit
      << " " << best.compact_every << " " << best.sort_bin << " " << best.steal << " " << best.stream << " "
      << best.ms_per_step << "\n";
  }
  if (out) *out = best;
  return GS_OK;
}

extern "C" gs_status gs_set_option(gs_ctx *ctx, int32_t option, int64_t value) {
  if (!ctx) return GS_ESTATE;
  const LaunchCfg keep = ctx->lc;
  const int keep_dep = ctx->deposit_opt, keep_grid = ctx->grid_opt;
  switch (option) {
    case GS_OPT_BLOCK:
      if (value != 256 && value != 512 && value != 768 && value != 1024)
        return fail(ctx, GS_EINVAL, "block must be 256, 512, 768 or 1024");
      ctx->lc.block = (int)value;
      if (ctx->lc.tile % (8 * ctx->lc.block)) ctx->lc.tile = ctx->lc.block * 8;
      break;
    case GS_OPT_TILE:
      if (value < 8 * ctx->lc.block || value % (8 * ctx->lc.block) || value > (1 << 24))
        return fail(ctx, GS_EINVAL, "tile must be a positive multiple of 8 x the block size");
      ctx->lc.tile = (int)value;
      break;
    case GS_OPT_GRID:
      if (value < 0 || value > 1 << 20) return fail(ctx, GS_EINVAL, "grid out of range");
      ctx->grid_opt = value > 0;
      if (value > 0) ctx->lc.grid = (int)value;
      break;
    case GS_OPT_DEPOSIT:
      if (value < 0 || value > 2) return fail(ctx, GS_EINVAL, "deposit must be 0, 1 or 2");
      ctx->deposit_opt = (int)value;
      break;
    case GS_OPT_PPT:
      if (value != 1 && value != 2) return fail(ctx, GS_EINVAL, "vectors per thread must be 1 or 2");
      ctx->lc.ppt = (int)value * (ctx->fp64 ? 2 : 4);
      if (ctx->lc.tile % (ctx->lc.block * ctx->lc.ppt)) ctx->lc.tile = ctx->lc.block * ctx->lc.ppt * 4;
      break;
    case GS_OPT_SORT_BIN:
      if (value != 0 && (value < SORT_BIN_MIN || value > 1 << 20))
        return fail(ctx, GS_EINVAL, "sort bin must be 0 or at least %d cells", SORT_BIN_MIN);
      if (value != 0 && sort_lds_bytes(ctx->G, ctx->nmax, (int)value) > 163840)
        return fail(ctx, GS_EINVAL, "a sort bin of %lld cells needs more than 160 KiB of LDS for %d gaps",
                    (long long)value, ctx->G);
      ctx->lc.sort_bin = (int)value;
      break;
    case GS_OPT_STEAL:
      if (value != 0 && (value < 2 || value > 64)) return fail(ctx, GS_EINVAL, "steal must be 0 or 2..64");
      ctx->lc.steal = (int)value;
      break;
    case GS_OPT_STREAM:
      if (value < 0 || value > 3) return fail(ctx, GS_EINVAL, "stream must be 0..3");
      ctx->lc.stream = (int)value;
      break;
    case GS_OPT_COMPACT_GRID:
      if (value < 1 || value > 1 << 20) return fail(ctx, GS_EINVAL, "compact grid out of range");
      ctx->lc.compact_grid = (int)value;
      break;
    case GS_OPT_COMPACT_EVERY:
      if (value < 1 || value > 1 << 20) return fail(ctx, GS_EINVAL, "compact_every must be >= 1");
      ctx->compact_every = (int)value;
      return GS_OK;
    case GS_OPT_GRAPH:
      ctx->use_graph = value ? 1 : 0;
      return GS_OK;
    case GS_OPT_TIMING:
      if (value < 0 || value > 2) return fail(ctx, GS_EINVAL, "timing must be 0, 1 or 2");
      ctx->timing = (int)value;
      return GS_OK;
    case GS_OPT_NEWTON_TOL:
      if (value <= 0) return fail(ctx, GS_EINVAL, "tolerance must be positive");
      ctx->newton_tol = (double)value * 1e-12;
      return GS_OK;
    case GS_OPT_NEWTON_MAXIT:
      if (value < 0 || value > 64) return fail(ctx, GS_EINVAL, "maxit must be in 0..64");
      ctx->newton_maxit = (int)value;
      return GS_OK;
    default:
      return fail(ctx, GS_EINVAL, "unknown option %d", option);
  }
  choose_launch(ctx);
  if (!launch_fits(ctx)) {
    ctx->lc = keep;
    ctx->deposit_opt = keep_dep;
    ctx->grid_opt = keep_grid;
    return fail(ctx, GS_EINVAL, "that launch shape needs more than 160 KiB of LDS per workgroup");
  }
  // a new shape invalidates captured graphs
  for (int m = 0; m < 2; ++m)
    for (int k = 0; k < 3; ++k)
      if (ctx->gexec[m][k]) {
        (void)hipGraphExecDestroy(ctx->gexec[m][k]);
        ctx->gexec[m][k] = nullptr;
      }
  return GS_OK;
}

extern "C" gs_status gs_get_timing(gs_ctx *ctx, gs_timing *out, int32_t reset) {
  if (!ctx || !out) return GS_ESTATE;
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  for (auto &pe : ctx->pend) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, pe.a, pe.b);
    if (pe.kind == 0) {
      ctx->tm.push_ms += ms;
      ctx->tm.push_launches += 1;
    } else if (pe.kind == 1) {
      ctx->tm.field_ms += ms;
      ctx->tm.field_launches += 1;
    } else if (pe.kind == 3) {
      ctx->tm.emit_ms += ms;
      ctx->tm.emit_launches += 1;
    } else {
      ctx->tm.compact_ms += ms;
      ctx->tm.compact_launches += 1;
    }
    ctx->pool.push_back(pe.a);
    ctx->pool.push_back(pe.b);
  }
  ctx->pend.clear();
  *out = ctx->tm;
  if (reset) memset(&ctx->tm, 0, sizeof ctx->tm);
  return GS_OK;
}
