// Device side of the circuit-coupled 1D ES-PIC step for gfx950.
//
// Per step two kernels run on the context's stream:
//   k_field   one workgroup per gap: charge accumulator -> rho, prefix scans for
//             the half-grid field, the circuit/surface-charge update (strict or
//             weak), the binary32/64 field table the push gathers from.
//             With an external circuit engine (field mode 2) the engine's gap
//             voltage comes from, and the potential goes to, pinned host memory.
//   k_push    persistent workgroups over tiles of every gap's particles: gather,
//             leapfrog, wall test and the charge deposit, privatised in LDS per
//             workgroup; at the start of each of its ion segments a workgroup
//             injects its share of the beam, at the end it emits the secondary
//             electrons of the ions it absorbed.
// Every few steps k_compact reclaims the slots of absorbed particles.  On
// request k_dt_scan reads one gap's particles for the time-step check.
//
// Compiled with -ffp-contract=off: the binary32 particle arithmetic is a fixed
// sequence of IEEE operations (no fused multiply-adds).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <type_traits>

#include "gs_internal.h"
#include "gs_mlp_dev.h"

namespace gs {

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11)
// ---------------------------------------------------------------------------
__device__ inline void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  // kept rolled: it runs only at emission and injection, and the push
  // kernel's instruction footprint matters more than its speed
#pragma unroll 1
  for (int r = 0; r < 10; ++r) {
    const uint64_t lo0 = M0 * c[0], hi0 = __umul64hi(M0, c[0]);
    const uint64_t lo1 = M1 * c[2], hi1 = __umul64hi(M1, c[2]);
    const uint64_t n0 = hi1 ^ c[1] ^ k0;
    const uint64_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += W0;
    k1 += W1;
  }
}

__device__ inline double unit_open(uint64_t r) {
  return ((double)(r >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

// random streams: SEE of an ion (step, id, 1, block); beam particle k (step, k, 2, 0)
__device__ inline void rng_block(uint64_t seed, uint64_t a, uint64_t b, uint64_t c, uint64_t d,
                                 uint64_t out[4]) {
  out[0] = a;
  out[1] = b;
  out[2] = c;
  out[3] = d;
  philox4x64_10(out, seed, 0);
}

// (not inlined: the constants of the exponential would otherwise be held in
// registers across the whole push kernel)
__device__ __attribute__((noinline)) int poisson_inverse(double lam, double u, int kmax) {
  double p = exp(-lam);
  double F = p;
  int k = 0;
  while (u > F && k < kmax) {
    k += 1;
    p = p * lam / (double)k;
    F = F + p;
  }
  return k;
}

// ---------------------------------------------------------------------------
// workgroup helpers
// ---------------------------------------------------------------------------
template <class T>
__device__ inline T block_exclusive_scan(T v, T *sh, T *total) {
  const int tid = threadIdx.x, nt = blockDim.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < nt; off <<= 1) {
    T a = (tid >= off) ? sh[tid - off] : (T)0;
    __syncthreads();
    sh[tid] += a;
    __syncthreads();
  }
  T incl = sh[tid];
  *total = sh[nt - 1];
  __syncthreads();
  return incl - v;
}

__device__ inline double block_sum(double v, double *sh) {
  const int tid = threadIdx.x, nt = blockDim.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = nt / 2; off > 0; off >>= 1) {
    if (tid < off) sh[tid] += sh[tid + off];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// block-wide exclusive scan of doubles built from wave scans: two barriers
// (wsum: one slot per wave)
// The wave scan moves values between lanes with DPP (row shifts within rows of
// 16 lanes, then the row broadcasts of lanes 15 and 31), a double as two
// 32-bit halves; lanes a shift or a mask leaves out add zero.
template <int CTRL, int ROW_MASK, int BANK_MASK>
__device__ inline double dpp_d(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROW_MASK, BANK_MASK, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, BANK_MASK, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ inline double wave_incl_scan_d(double x) {
  double y = x + dpp_d<0x111, 0xf, 0xf>(x);  // + lane - 1 (row_shr:1)
  y += dpp_d<0x112, 0xf, 0xf>(x);            // + lane - 2
  y += dpp_d<0x113, 0xf, 0xf>(x);            // + lane - 3: four lanes summed
  y += dpp_d<0x114, 0xf, 0xe>(y);            // lanes 4..15 of each row: + lane - 4
  y += dpp_d<0x118, 0xf, 0xc>(y);            // lanes 8..15: + lane - 8, each row scanned
  y += dpp_d<0x142, 0xa, 0xf>(y);            // rows 1 and 3: + lane 15 of the row before
  y += dpp_d<0x143, 0xc, 0xf>(y);            // rows 2 and 3: + lane 31
  return y;
}

__device__ inline double block_exclusive_scan_w(double v, double *wsum, double *total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const double incl = wave_incl_scan_d(v);
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  double before = 0.0, all = 0.0;
  for (int q = 0; q < nw; ++q) {
    const double a = wsum[q];
    if (q < w) before += a;
    all += a;
  }
  *total = all;
  __syncthreads();
  return before + incl - v;
}

// block_exclusive_scan_w of v, and in the same two barriers the block sum of w
__device__ inline double block_exclusive_scan_sum_w(double v, double w, double *wsum, double *wsum2, double *total,
                                                    double *wtotal) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const double incl = wave_incl_scan_d(v);
  const double wincl = wave_incl_scan_d(w);
  if (lane == 63) {
    wsum[wv] = incl;
    wsum2[wv] = wincl;
  }
  __syncthreads();
  double before = 0.0, all = 0.0, wall = 0.0;
  for (int q = 0; q < nw; ++q) {
    const double a = wsum[q];
    if (q < wv) before += a;
    all += a;
    wall += wsum2[q];
  }
  *total = all;
  *wtotal = wall;
  __syncthreads();
  return before + incl - v;
}

__device__ inline double block_sum_w(double v, double *wsum) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if (lane == 0) wsum[w] = v;
  __syncthreads();
  double all = 0.0;
  for (int q = 0; q < nw; ++q) all += wsum[q];
  __syncthreads();
  return all;
}

// wave-wide inclusive prefix sum (64 lanes)
__device__ inline int wave_incl_scan(int v);

// block-wide exclusive scan of ints from wave scans: two barriers (wsum: one
// slot per wave)
__device__ inline int block_exclusive_scan_i(int v, int *wsum, int *total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int incl = wave_incl_scan(v);
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  int before = 0, all = 0;
  for (int q = 0; q < nw; ++q) {
    const int a = wsum[q];
    if (q < w) before += a;
    all += a;
  }
  *total = all;
  __syncthreads();
  return before + incl - v;
}

__device__ inline int wave_incl_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

__device__ inline unsigned int wave_sum(unsigned int a) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
  return a;
}

// Secondary emission (Alg. 2), in two parts.  see_count: an absorbed ion's
// energy E = m v^2 / 2 from its impact velocity, the mean yield (saturating
// a (E/E0) / (1 + E/E0), or a times the fifth-order fit clipped at zero) and
// the Poisson count by inversion, drawn from the stream keyed by (level, ion
// id); blk keeps the block for the energies.
__device__ inline int see_count(const GapConst &c, long long level, uint32_t ion_id, double u_imp, uint64_t blk[4]) {
  const double v_ion = (u_imp * c.dx) / c.dt;
  const double e_ion = 0.5 * c.mass[1] * v_ion * v_ion / c.ev;
  double lam;
  if (c.see_yield == GS_YIELD_POLY) {
    const double x = (e_ion < c.see_pEmax ? e_ion : c.see_pEmax) / 1000.0;
    double f = c.see_poly[5];
#pragma unroll
    for (int j = 4; j >= 0; --j) f = f * x + c.see_poly[j];
    lam = c.see_amp * (f > 0.0 ? f : 0.0);
  } else {
    const double rr = e_ion / c.see_E0;
    lam = c.see_amp * rr / (1.0 + rr);
  }
  if (lam < 0.0) lam = 0.0;
  rng_block(c.seed, (uint64_t)level, (uint64_t)ion_id, 1, 0, blk);
  return poisson_inverse(lam, unit_open(blk[0]), c.see_max);
}

// An emitted electron's energy [eV] from its one or two uniform draws: fixed,
// exponential of mean E, or lognormal exp(mu + sig Z) with the Box-Muller
// normal Z = sqrt(-2 ln u0) cos(2 pi u1), evaluated as cospi(2 u1), whose
// argument needs no general range reduction.  (Not inlined, as
// poisson_inverse.)
__device__ __attribute__((noinline)) double see_energy(int law, double E, double mu, double sig, double u0,
                                                       double u1) {
  const double L = log(u0);
  if (law == GS_SEE_EXP) return -E * L;
  if (law == GS_SEE_LOGNORMAL) return exp(mu + sig * (sqrt(-2.0 * L) * cospi(2.0 * u1)));
  return E;
}

// see_write: the ion's nk electrons, energies fixed, exponential or lognormal
// (from the ion's stream words 1, 2, .. in order: one per electron, two for the
// lognormal's normal draw), placed on the wall node with the inward speed of
// their energy, in slots base.. of the electron region; counts per wall added
// to n[0], n[1].
template <class P>
__device__ inline void see_write(const DevPtrs &p, const GapConst &c, long long level, int g, int sel,
                                 uint32_t ion_id, int wall, int nk, uint64_t blk[4], unsigned long long base,
                                 unsigned int n[2]) {
  P *X = (P *)p.X[sel] + c.pbase[0];
  P *U = (P *)p.U[sel] + c.pbase[0];
  uint32_t *ID = p.ID[sel] + c.pbase[0];
  const P xw = wall == 0 ? (P)0 : (P)c.N;
  // one copy of each draw and function (cold code: its size is what costs)
  const int nw = c.see_law == GS_SEE_LOGNORMAL ? 2 : 1;
  int w = 1;  // word 0 of block 0 drew the count
  for (int e = 0; e < nk; ++e) {
    double u[2] = {0.5, 0.5};
#pragma unroll 1
    for (int t = 0; t < nw; ++t) {
      if ((w & 3) == 0) rng_block(c.seed, (uint64_t)level, (uint64_t)ion_id, 1, (uint64_t)(w >> 2), blk);
      const double uw = unit_open(blk[w & 3]);
      u[0] = t == 0 ? uw : u[0];
      u[1] = t == 1 ? uw : u[1];
      w += 1;
    }
    const double E_se = see_energy(c.see_law, c.see_E, c.see_mu, c.see_sig, u[0], u[1]);
    const double v_se = sqrt(2.0 * E_se * c.ev / c.mass[0]);
    const double v_si = wall == 0 ? v_se : -v_se;
    const unsigned long long sl = base + (unsigned long long)e;
    if (sl >= (unsigned long long)c.cap[0]) {
      atomicOr(&p.err[0], ERR_CAPACITY);
      atomicCAS(&p.err[1], 0xFFFFFFFFu, (unsigned int)g);
      continue;
    }
    X[sl] = xw;
    U[sl] = (P)((v_si * c.dt) / c.dx);
    ID[sl] = NO_ID;
    n[wall] += 1;
  }
}

// Emission for ne events of gap g listed in evs (each carrying its ion's id),
// one event per thread and pass, slots in buffer sel from one reservation per
// pass; emitted counts per wall added to emit_cnt (LDS).  Every thread of the
// block calls it.
template <class P>
__device__ void see_emit(const DevPtrs &p, const GapConst &c, long long level, int g, int sel, const Event *evs,
                         int ne, int *wsum, unsigned long long *s_base, unsigned int *emit_cnt) {
  for (int r = 0; r < ne; r += blockDim.x) {
    const int k = r + threadIdx.x;
    int nk = 0, wall = 0;
    uint32_t ion_id = 0;
    uint64_t blk[4] = {0, 0, 0, 0};
    if (k < ne) {
      const Event ev = evs[k];
      ion_id = ev.ref;
      wall = (int)ev.wall;
      nk = see_count(c, level, ion_id, ev.u, blk);
    }
    int btot;
    const int excl = block_exclusive_scan_i(nk, wsum, &btot);
    if (btot == 0) continue;
    if (threadIdx.x == 0) *s_base = atomicAdd(&p.next_count[g * 2 + 0], (unsigned long long)btot);
    __syncthreads();
    const unsigned long long base = *s_base;
    __syncthreads();
    unsigned int n[2] = {0u, 0u};
    see_write<P>(p, c, level, g, sel, ion_id, wall, nk, blk, base + (unsigned long long)excl, n);
    const unsigned int a0 = wave_sum(n[0]), a1 = wave_sum(n[1]);
    if ((threadIdx.x & 63) == 0) {
      if (a0) atomicAdd(&emit_cnt[0], a0);
      if (a1) atomicAdd(&emit_cnt[1], a1);
    }
  }
}

// This file is compiled once for everything but the push kernel's
// instantiations, and once per GS_PUSH_PART for one set of them (the units
// build in parallel); the push units skip the other kernels and launchers.
#ifndef GS_PUSH_PART
// ---------------------------------------------------------------------------
// The field solve of level n, in three kernels: k_fdens (the nodal density and
// the prefix sums within chunks of FCN nodes, many workgroups), k_field (the
// chunks' offsets, the circuit and the surface charge: one workgroup per gap)
// and k_ftable (the half-grid field and the push's gather table, many
// workgroups).
// ---------------------------------------------------------------------------
constexpr int FBS = 1024;  // k_field threads
constexpr int FDB = 256;   // k_fdens / k_ftable threads, four nodes each
// Up to FIELD1_NMAX cells one workgroup per gap does all of it (k_field1): a
// kernel costs some microseconds of its own here, and at 4096 cells the one
// workgroup's serial path is shorter than three kernels'.  Its S_k live in LDS
// (padded), and each thread forms at most FNQ nodes.
constexpr int FIELD1_NMAX = 8192;
constexpr int FNQ = (FIELD1_NMAX + 1 + FBS - 1) / FBS;
__device__ inline double node_rho(double s0, double dx, unsigned long long a, int j, int N, int fp64) {
  const double scale = fp64 ? 5.684341886080801486968994140625e-14 /* 2^-44 */
                            : 5.9604644775390625e-08 /* 2^-24 */;
  double r = s0 * ((double)(long long)a * scale) / dx;
  if (j == 0 || j == N) r *= 2.0;
  return r;
}

// Circuit, surface charge and electrode potential of level n (thread 0, on LDS
// copies of the gap's constants and state).  P = (dx/eps0) sum_k S_k is the
// potential the space charge alone gives the electrode.
__device__ void solve_level(const DevPtrs &p, int g, const GapConst &c, GapState &st, double P,
                            int mode, int guess, double tol, int maxit, double *sigma_out,
                            double *wk, const unsigned long long *tl, const double *mlp_u,
                            const unsigned long long *next_count, long long nb) {
  const int M = c.M, gm = c.g;
  const double A = c.A, eps0 = c.eps0;
  const long long n = st.level + 1;
  const double t = (double)n * c.dt;
  // convection charge of the push that led to this level (Sec. 2.4.1); tl is
  // the gap's tally, already staged in LDS
  long long ab[4], em[2], inj, pushed;
  for (int i = 0; i < 4; ++i) ab[i] = (long long)tl[T_ABS + i];
  em[0] = (long long)tl[T_EMIT];
  em[1] = (long long)tl[T_EMIT + 1];
  inj = (long long)tl[T_INJ];
  pushed = (long long)tl[T_PUSHED];
  const double qsh_i = A * (c.s0 * (double)c.Z[1]);
  const double qsh_e = A * (c.s0 * (double)c.Z[0]);
  double qconv = 0.0;
  qconv += qsh_i * (double)ab[1 * 2 + 0];
  qconv += qsh_e * (double)ab[0 * 2 + 0];
  qconv -= qsh_e * (double)em[0];
  for (int i = 0; i < 4; ++i) {
    st.abs_last[i] = ab[i];
    st.abs_cum[i] += ab[i];
  }
  for (int i = 0; i < 2; ++i) {
    st.emit_last[i] = em[i];
    st.emit_cum[i] += em[i];
  }
  st.inj_last = inj;
  st.inj_cum += inj;
  st.pushed_last = pushed;
  st.pushed_cum += pushed;
  st.live[0] += em[0] + em[1] - ab[0] - ab[1];
  st.live[1] += inj - ab[2] - ab[3];

  // (no sine on this serial path when there is no AC source: dc + 0 sin = dc)
  const double Vs = c.src_amp != 0.0 ? c.src_dc + c.src_amp * sin(c.src_w * t + c.src_phase) : c.src_dc;
  // small work vectors live in LDS: indexed by the run-time mesh count they would
  // otherwise go to scratch memory
  double *h = wk, *q = wk + MAXM, *Dn = wk + 2 * MAXM, *y = wk + 3 * MAXM;
  double *u = wk + 4 * MAXM, *r = u + (MAXM + 1), *ue = r + (MAXM + 1), *rc = ue + (MAXM + 1);
  for (int j = 0; j < M; ++j) h[j] = 15.0 * st.dq[0][j] - 7.0 * st.dq[1][j] + st.dq[2][j];
  double sigma, qcirc, qstar, phi0;
  if (mode == 0) {
    // strict: D = y - z phi0, Q_gap = K - G phi0 (eq. Q4_phi_relation, eq. K_def)
    for (int i = 0; i < M; ++i) {
      double a = c.sb[i] * Vs;
      for (int j = 0; j < M; ++j)
        a += c.sL[i * MAXM + j] * h[j] + c.sR[i * MAXM + j] * st.dq[0][j] -
             c.sS[i * MAXM + j] * st.qprev[j];
      y[i] = a;
    }
    const double K = st.qprev[gm] + y[gm];
    const double G = c.sz[gm] + c.c_par;
    // eq. Poisson_BC2 closed over the interior rows:
    // phi0 = (d/eps0) sigma + P with sigma = sigma* - G phi0 / A
    const double sig_star = st.sigma_prev + (qconv + K - st.qcirc_prev) / A;
    phi0 = ((c.d / eps0) * sig_star + P) / (1.0 + G * c.d / (eps0 * A));
    int iters = -1, fb = 0;
    double r0n = 0.0, rn = 0.0;
    if (guess == GS_GUESS_DIRECT) {
      // the direct solve starts from nothing; report the extrapolation
      for (int i = 0; i <= M; ++i) st.guess[i] = 3.0 * st.uh[0][i] - 3.0 * st.uh[1][i] + st.uh[2][i];
    } else {
      // Newton on u = (V, I_0..I_{M-1}); the residual is affine in u
      const int nu = M + 1;
      auto residual = [&](const double *uu, double *rr) {
        // BDF2 increments from the currents: I = (3 D - D1) / (2 dt)
        for (int j = 0; j < M; ++j) rc[j] = (2.0 * c.dt * uu[1 + j] + st.dq[0][j]) / 3.0 - y[j];
        // loop equations in volts: T' D - C' + g V = T' (D - y) + g V
        for (int i = 0; i < M; ++i) {
          double a = (i == gm) ? uu[0] : 0.0;
          for (int j = 0; j < M; ++j) a += c.Tp[i * MAXM + j] * rc[j];
          rr[1 + i] = a / c.v_ref;
        }
        // closure: V equals the electrode potential the field gives
        const double qgap = st.qprev[gm] + (rc[gm] + y[gm]) - c.c_par * uu[0];
        const double sg = st.sigma_prev + (qconv + qgap - st.qcirc_prev) / A;
        rr[0] = (uu[0] - ((c.d / eps0) * sg + P)) / c.v_ref;
      };
      auto norm = [&](const double *rr) {
        double m = 0.0;
        for (int i = 0; i < nu; ++i) m = fmax(m, fabs(rr[i]));
        return m;
      };
      // plain guess: quadratic extrapolation of the last three levels
      for (int i = 0; i < nu; ++i) ue[i] = 3.0 * st.uh[0][i] - 3.0 * st.uh[1][i] + st.uh[2][i];
      residual(ue, r);
      const double rext = norm(r);
      bool use_mlp = false;
      if (guess == GS_GUESS_MLP && mlp_u) {
        for (int i = 0; i < nu; ++i) u[i] = mlp_u[i];
        for (int i = 0; i < 3; ++i) st.mlp_prop[i] = mlp_u[i];
        residual(u, r);
        const double rm = norm(r);
        use_mlp = (rm == rm) && (rm <= rext);
        if (!use_mlp) fb = 1;
      }
      if (!use_mlp) {
        for (int i = 0; i < nu; ++i) u[i] = ue[i];
        residual(u, r);
      }
      for (int i = 0; i < nu; ++i) st.guess[i] = u[i];
      r0n = norm(r);
      rn = r0n;
      iters = 0;
      // stop when the residual is within the tolerance, or when an update no
      // longer moves any component by more than a few units in its last place
      // (large loop currents can leave the representable u nearest the
      // solution with a scaled residual above the tolerance)
      bool at_roundoff = false;
      while (!(rn <= tol) && !at_roundoff && iters < maxit) {
        at_roundoff = true;
        for (int i = 0; i < nu; ++i) {
          double a = 0.0;
          for (int j = 0; j < nu; ++j) a += c.Jinv[i * (MAXM + 1) + j] * r[j];
          ue[i] = u[i] - a;
          if (!(fabs(a) <= 8.0 * 2.220446049250313e-16 * fabs(u[i]))) at_roundoff = false;
        }
        for (int i = 0; i < nu; ++i) u[i] = ue[i];
        residual(u, r);
        rn = norm(r);
        iters += 1;
      }
      if (!(rn <= tol) && !at_roundoff) atomicOr(p.err, ERR_NOCONV);
      phi0 = u[0];
    }
    qcirc = K - G * phi0;
    qstar = qcirc;
    sigma = st.sigma_prev + (qconv + qcirc - st.qcirc_prev) / A;  // eq. sigma_update
    for (int j = 0; j < M; ++j) {
      Dn[j] = y[j] - c.sz[j] * phi0;
      q[j] = st.qprev[j] + Dn[j];
    }
    st.newton_last = iters;
    st.newton_fb_last = fb;
    if (iters >= 0) {
      st.newton_total += iters;
      st.newton_fallbacks += fb;
      st.newton_max = max(st.newton_max, iters);
      st.newton_levels += 1;
    }
    st.newton_r0 = r0n;
    st.newton_r = rn;
  } else if (mode == 2) {
    // weak with an external circuit engine: its gap voltage V* for this level
    // gives Q_circ* = C_gap V* (Sec. 2.4.3); the library's own loops are not
    // advanced, only the gap mesh follows the re-imposed charge
    qstar = c.cgap * p.ext_v[g];
    sigma = st.sigma_prev + (qconv + qstar - st.qcirc_prev) / A;
    phi0 = (c.d / eps0) * sigma + P;
    for (int j = 0; j < M; ++j) {
      q[j] = st.qprev[j];
      Dn[j] = 0.0;
    }
    q[gm] = (c.cgap + c.c_par) * phi0;
    Dn[gm] = q[gm] - st.qprev[gm];
    qcirc = c.cgap * phi0;
    p.ext_phi[g] = phi0;  // for the engine's next call, read once this kernel is done
    st.newton_last = -1;
    st.newton_fb_last = 0;
  } else {
    // weak: the circuit alone with the gap as a capacitor, then the field
    for (int i = 0; i < M; ++i) {
      double a = c.wb[i] * Vs;
      for (int j = 0; j < M; ++j)
        a += c.wL[i * MAXM + j] * h[j] + c.wR[i * MAXM + j] * st.dq[0][j] -
             c.wS[i * MAXM + j] * st.qprev[j];
      y[i] = a;
    }
    for (int j = 0; j < M; ++j) {
      q[j] = st.qprev[j] + y[j];
      Dn[j] = y[j];
    }
    const double vstar = q[gm] / (c.cgap + c.c_par);
    qstar = c.cgap * vstar;
    sigma = st.sigma_prev + (qconv + qstar - st.qcirc_prev) / A;
    phi0 = (c.d / eps0) * sigma + P;
    // re-impose the gap charge the field implies; the increment history stays
    q[gm] = (c.cgap + c.c_par) * phi0;
    qcirc = c.cgap * phi0;
    st.newton_last = -1;
    st.newton_fb_last = 0;
  }
  for (int j = 0; j < M; ++j) {
    st.I[j] = (3.0 * Dn[j] - st.dq[0][j]) / (2.0 * c.dt);
    st.q[j] = q[j];
    st.dq[2][j] = st.dq[1][j];
    st.dq[1][j] = st.dq[0][j];
    st.dq[0][j] = Dn[j];
    st.qprev[j] = q[j];
  }
  for (int i = 0; i <= M; ++i) {
    st.uh[2][i] = st.uh[1][i];
    st.uh[1][i] = st.uh[0][i];
  }
  st.uh[0][0] = phi0;
  for (int j = 0; j < M; ++j) st.uh[0][1 + j] = st.I[j];
  {
    // the guess network's history: this level's voltage, first two loop
    // currents, surface charge and the absorbed / emitted charge behind Q_conv
    const int hh = st.hist_head;
    st.hist[hh][0] = phi0;
    st.hist[hh][1] = st.I[0];
    st.hist[hh][2] = M > 1 ? st.I[1] : 0.0;
    st.hist[hh][3] = sigma;
    st.hist[hh][4] = qsh_i * (double)ab[1 * 2 + 0] + qsh_e * (double)ab[0 * 2 + 0];
    st.hist[hh][5] = qsh_e * (double)em[0];
    st.hist_head = (hh + 1) & 7;
  }
  st.qcirc_step = qstar - st.qcirc_prev;
  st.sigma_prev = sigma;
  st.qcirc_prev = qcirc;
  st.level = n;
  st.t = t;
  st.phi0 = phi0;
  st.sigma = sigma;
  st.qcirc = qcirc;
  st.qcirc_star = qstar;
  st.qconv = qconv;
  // particles the coming push sweeps; the step's beam gets the slots right after
  // them (its ids and slots are fixed before the push)
  // (append counters can run past the capacity after an overflow, which was
  // flagged when it happened; never sweep past the region)
  // (next_count: the append counters as the push and the emission left them;
  // nb: the beam of the step that solves level n, its schedule entry or else
  // the fixed count; both read at the field kernel's start)
  for (int s = 0; s < 2; ++s) st.count[s] = min((long long)next_count[s], c.cap[s]);
  st.beam_now = nb;
  p.next_count[g * 2 + 1] = (unsigned long long)(st.count[1] + nb);
  p.ev_count[g] = 0ull;
  p.ev_done[g] = 0ull;
  st.beam_id0 = st.next_id;
  st.next_id += nb;
  *sigma_out = sigma;
}

// k_field1: level n of one gap per workgroup, for grids up to FIELD1_NMAX
// cells: the nodal density (the accumulator cleared for the next push), the
// prefix sums S_k, the circuit and the surface charge, the half-grid field and
// the push's gather table.
__global__ __launch_bounds__(FBS) void k_field1(DevPtrs p, int mode, int guess, double tol,
                                                int maxit, int fp64) {
  const int g = blockIdx.x, tid = threadIdx.x;
  extern __shared__ __align__(16) double Sk[];  // S_k, one per cell (padded, see the prefix sums)
  // the gap's constants, state and last push's tallies, staged as one block
  // and the append counters as the push and the emission left them
  struct Staged {
    GapConst c;
    GapState s;
    unsigned long long tally[T_N];
    unsigned long long next_count[2];
  };
  __shared__ Staged stg;
  GapConst &sc = stg.c;
  GapState &ss = stg.s;
  unsigned long long *s_tally = stg.tally;
  __shared__ double wsum[FBS / 64], wsum2[FBS / 64];
  __shared__ double s_sigma, s_rhoN;
  __shared__ double s_work[8 * MAXM + 8];
  __shared__ float s_x[MLP_IN], s_h0[MLP_H], s_h1[MLP_H], s_y[MLP_OUT];
  __shared__ double s_ue[MAXM + 1], s_mu[MAXM + 1];
  // the first FBS x AV0 nodes of the push's charge accumulator, loaded before
  // anything else (nothing in this kernel writes them before the density pass),
  // from clamped indices and masked afterwards: a guarded load would be waited
  // for before the next is issued
  // (secondary emission is complete when this kernel runs: the emission kernel
  // ran after the push)
  constexpr int AV0 = 5;
  unsigned long long av0[AV0];
  {
    const int n0 = p.gc[g].N;
    const unsigned long long *a0 = p.acc + p.gc[g].nbase;
#pragma unroll
    for (int q = 0; q < AV0; ++q) av0[q] = a0[min(tid + q * FBS, n0)];
#pragma unroll
    for (int q = 0; q < AV0; ++q)
      if (tid + q * FBS > n0) av0[q] = 0ull;
  }
  // the coming push's tile pool starts empty
  if (g == 0 && tid == 0) *p.steal = 0u;
  // stage the gap's constants, state and last push's tallies: word tid of
  // their concatenation per thread, one load and one LDS store with no branch;
  // the tallies are cleared at the kernel's end
  {
    constexpr int NC = (int)(sizeof(GapConst) / 8), NS = (int)(sizeof(GapState) / 8);
    constexpr int NW = (int)(sizeof(Staged) / 8);
    static_assert(sizeof(Staged) == sizeof(GapConst) + sizeof(GapState) + 8 * (T_N + 2) && NW <= FBS,
                  "one staged word per thread");
    const unsigned long long *src =
        tid < NC ? (const unsigned long long *)&p.gc[g] + tid
        : tid < NC + NS ? (const unsigned long long *)&p.gs[g] + (tid - NC)
        : tid < NC + NS + T_N ? p.tally + (size_t)g * T_N + (tid - NC - NS)
                              : p.next_count + (size_t)g * 2 + min(tid - NC - NS - T_N, 1);
    const unsigned long long v = *src;
    if (tid < NW) ((unsigned long long *)&stg)[tid] = v;
  }
  __syncthreads();
  long long nbeam;
  {
    const long long n = ss.level + 1;
    int lane0 = 0;
    asm volatile("" : "+v"(lane0));
    const long long ix = sc.sched_len > 0 ? sc.sched_base + min(n, sc.sched_len - 1) : 0;
    const long long v = (long long)p.sched[ix + lane0];
    nbeam = n < sc.sched_len ? v : sc.beam_n;
  }

  // 0. strict coupling: the guess network's input (the last 8 levels from the
  //    history ring), recorded for training and/or evaluated for the guess
  const bool want_mlp = mode == 0 && guess == GS_GUESS_MLP && p.mlp_w != nullptr;
  const bool want_rec = mode == 0 && p.rec_x != nullptr;
  const long long rec_idx = (ss.level + 1 - p.rec_level0) * (long long)gridDim.x + g;
  const bool rec_here = want_rec && rec_idx >= 0 && rec_idx < p.rec_cap;
  if (want_mlp || rec_here) {
    if (tid < MLP_IN) {
      // block k = 1..8: (V, I_0, I_1, sigma) of level n-k and the absorbed /
      // emitted charge of the push that followed it (for k = 1 the push whose
      // tallies this solve is about to fold in)
      const int kk = tid / 6 + 1, q = tid % 6;
      double raw;
      if (q < 4) {
        raw = ss.hist[(ss.hist_head - kk) & 7][q];
      } else if (kk > 1) {
        raw = ss.hist[(ss.hist_head - kk + 1) & 7][q];
      } else {
        const double qi = sc.A * (sc.s0 * (double)sc.Z[1]), qe = sc.A * (sc.s0 * (double)sc.Z[0]);
        raw = q == 4 ? qi * (double)(long long)s_tally[T_ABS + 2] + qe * (double)(long long)s_tally[T_ABS + 0]
                     : qe * (double)(long long)s_tally[T_EMIT + 0];
      }
      if (rec_here) p.rec_x[rec_idx * MLP_IN + tid] = (float)raw;
      if (want_mlp) s_x[tid] = (float)((raw - p.mlp_norm[tid]) / p.mlp_norm[MLP_IN + tid]);
    }
    if (tid == 0)
      for (int i = 0; i <= sc.M; ++i) s_ue[i] = 3.0 * ss.uh[0][i] - 3.0 * ss.uh[1][i] + ss.uh[2][i];
    if (want_mlp) {
      mlp_eval_block(p.mlp_w, s_x, s_h0, s_h1, s_y);
      if (tid == 0)
        for (int i = 0; i < MLP_OUT; ++i)
          s_mu[i] = s_ue[i] + p.mlp_norm[2 * MLP_IN + i] + p.mlp_norm[2 * MLP_IN + MLP_OUT + i] * (double)s_y[i];
    }
  }

  const int N = sc.N;
  const double dx = sc.dx, eps0 = sc.eps0, s0 = sc.s0;
  unsigned long long *acc = p.acc + sc.nbase;
  double *rho = p.rho64 + sc.nbase;
  double *E = p.E64 + sc.nbase;

  // 1. nodal density of level n (to global rho and, as the cell terms of the
  //    prefix sums, to LDS); the accumulator is cleared for the next push.
  //    The rest of the thread's nodes are loaded before any clearing store:
  //    loads and stores share one counter, so a load issued after a store would
  //    wait for it too.
  const int ch = (N + FBS - 1) / FBS;  // cells per thread in the prefix sums below
  // floor(k / ch) = (k * ceil(2^32 / ch)) >> 32 for every k here (k <= 16384 + FBS)
  const unsigned long long chm = (4294967296ull + (unsigned long long)ch - 1ull) / (unsigned long long)ch;
  auto pad = [&](int k) { return k + (int)(((unsigned long long)k * chm) >> 32); };
  // (the nodes past the first FBS x AV0 only when the grid has them: the
  // condition is the workgroup's, and a load nobody needs still costs a round
  // trip)
  unsigned long long av[FNQ];
#pragma unroll
  for (int q = 0; q < AV0; ++q) av[q] = av0[q];
  if (N >= AV0 * FBS) {
#pragma unroll
    for (int q = AV0; q < FNQ; ++q) av[q] = acc[min(tid + q * FBS, N)];
  }
#pragma unroll
  for (int q = 0; q < FNQ; ++q) {
    const int k = tid + q * FBS;
    if (k > N) break;
    const double r = node_rho(s0, dx, av[q], k, N, fp64);
    rho[k] = r;
    acc[k] = 0ull;
    if (k < N)
      Sk[pad(k)] = (k == 0) ? dx * r / 2.0 : dx * r;
    else
      s_rhoN = r;
  }
  __syncthreads();
  // prefix sums S_k = dx rho_0/2 + dx sum_{1..k} rho_j over contiguous chunks
  // of ch cells per thread (cell k at LDS index k + k / ch: a chunk's stride
  // of ch + 1 doubles spreads a wave's lanes over the LDS banks, where a
  // stride of ch would put them on one)
  // (the chunk's cells are held in registers between the two passes; cell
  // k0 + i of thread tid sits at LDS index k0 + i + tid)
  const int k0 = min(tid * ch, N), k1 = min(k0 + ch, N);
  const int nk = k1 - k0;
  double cv[FNQ];
#pragma unroll
  for (int i = 0; i < FNQ; ++i) cv[i] = i < nk ? Sk[k0 + i + tid] : 0.0;
  // with sum_k S_k = sum_j c_j (N - j) (c_j the cell terms) taken in the same
  // reduction as the scan's wave totals
  double loc = 0.0, wloc = 0.0;
#pragma unroll
  for (int i = 0; i < FNQ; ++i)
    if (i < nk) {
      loc += cv[i];
      wloc += cv[i] * (double)(N - (k0 + i));
    }
  double tot, sumS;
  double run = block_exclusive_scan_sum_w(loc, wloc, wsum, wsum2, &tot, &sumS);
#pragma unroll
  for (int i = 0; i < FNQ; ++i)
    if (i < nk) {
      run += cv[i];
      Sk[k0 + i + tid] = run;
    }
  const double P = sumS * dx / eps0;

  // 2. circuit and surface charge
  if (tid == 0) {
    double sg;
    // space charge: the cell terms (rho_0 at half weight) plus the half cell at node N
    ss.q_space = sc.A * (tot + 0.5 * dx * s_rhoN);
    solve_level(p, g, sc, ss, P, mode, guess, tol, maxit, &sg, s_work, s_tally, want_mlp ? s_mu : nullptr,
                stg.next_count, nbeam);
    s_sigma = sg;
    if (rec_here)
      for (int i = 0; i < MLP_OUT; ++i)
        p.rec_y[rec_idx * MLP_OUT + i] = i <= sc.M ? (float)(ss.uh[0][i] - s_ue[i]) : 0.0f;
  }
  __syncthreads();

  // 3. half-grid field E_{k+1/2} = (sigma + S_k) / eps0 and the gather table
  const double sigma = s_sigma;
  const double rhoN = s_rhoN;
  const size_t eb = (size_t)sc.ebase;
  for (int k = tid; k < N; k += FBS) {
    const double e = (sigma + Sk[pad(k)]) / eps0;
    E[k] = e;
    if (fp64)
      ((double *)p.ehat)[eb + k + 1] = e;
    else
      ((float *)p.ehat)[eb + k + 1] = (float)e;
    if (k == N - 1) {
      const double ed = e + dx * rhoN / (2.0 * eps0);
      ss.e_ground = ed;
      if (fp64)
        ((double *)p.ehat)[eb + N + 1] = ed;
      else
        ((float *)p.ehat)[eb + N + 1] = (float)ed;
    }
  }
  if (tid == 0) {
    const double e0 = sigma / eps0;
    if (fp64)
      ((double *)p.ehat)[eb] = e0;
    else
      ((float *)p.ehat)[eb] = (float)e0;
  }
  __syncthreads();
  {
    const unsigned long long *a = (const unsigned long long *)&ss;
    unsigned long long *b = (unsigned long long *)&p.gs[g];
    for (int i = tid; i < (int)(sizeof(GapState) / 8); i += FBS) b[i] = a[i];
  }
  if (tid < T_N) p.tally[(size_t)g * T_N + tid] = 0ull;
}


// k_fdens: chunk c (blockIdx.x) of gap g (blockIdx.y), nodes [c FCN, (c + 1)
// FCN) up to N.  Each node's density goes to rho and its accumulator word is
// cleared for the next push; the cell terms c_k (dx rho_0 / 2, then dx rho_k,
// k < N) are summed within the chunk: the inclusive prefix L_k to fsl, the
// chunk's total and sum_k c_k (N - k) to fpart.
__global__ __launch_bounds__(FDB) void k_fdens(DevPtrs p, int fp64) {
  const int g = blockIdx.y, c = blockIdx.x, tid = threadIdx.x;
  __shared__ double wsum[FDB / 64], wsum2[FDB / 64];
  const GapConst &gc = p.gc[g];
  const int N = gc.N;
  const int kb = c * FCN + 4 * tid;  // this thread's first node
  if (c * FCN > N) return;           // (the whole workgroup)
  unsigned long long *acc = p.acc + gc.nbase;
  double *rho = p.rho64 + gc.nbase;
  double *sl = p.fsl + gc.nbase;
  const double dx = gc.dx, s0 = gc.s0;
  // (loads from clamped indices, all issued before the first is used)
  unsigned long long a[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) a[i] = acc[min(kb + i, N)];
  double cv[4];
  double loc = 0.0, wloc = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int k = kb + i;
    const double r = node_rho(s0, dx, a[i], k, N, fp64);
    cv[i] = k < N ? (k == 0 ? dx * r / 2.0 : dx * r) : 0.0;
    loc += cv[i];
    wloc += cv[i] * (double)(N - k);
    if (k <= N) {
      rho[k] = r;
      acc[k] = 0ull;
    }
  }
  double tot, wtot;
  double run = block_exclusive_scan_sum_w(loc, wloc, wsum, wsum2, &tot, &wtot);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    run += cv[i];
    if (kb + i < N) sl[kb + i] = run;
  }
  if (tid == 0) {
    double *pt = p.fpart + ((size_t)g * NCHMAX + c) * 2;
    pt[0] = tot;
    pt[1] = wtot;
  }
}

// k_field: one workgroup per gap.  The chunks' totals give S_k's offsets, the
// potential P = (dx / eps0) sum_k S_k that the space charge alone gives the
// electrode and the space charge; thread 0 solves the circuit and the surface
// charge (solve_level); the offsets and sigma go to k_ftable.
__global__ __launch_bounds__(FBS) void k_field(DevPtrs p, int mode, int guess, double tol,
                                               int maxit, int fp64) {
  const int g = blockIdx.x, tid = threadIdx.x;
  // the gap's constants, state and last push's tallies, staged as one block
  // and the append counters as the push and the emission left them
  struct Staged {
    GapConst c;
    GapState s;
    unsigned long long tally[T_N];
    unsigned long long next_count[2];
  };
  __shared__ Staged stg;
  GapConst &sc = stg.c;
  GapState &ss = stg.s;
  unsigned long long *s_tally = stg.tally;
  __shared__ double s_work[8 * MAXM + 8];
  __shared__ float s_x[MLP_IN], s_h0[MLP_H], s_h1[MLP_H], s_y[MLP_OUT];
  __shared__ double s_ue[MAXM + 1], s_mu[MAXM + 1];
  // (secondary emission is complete when this kernel runs: the emission kernel
  // ran after the push)
  // the coming push's tile pool starts empty
  if (g == 0 && tid == 0) *p.steal = 0u;
  // the chunks' totals (lane c of wave 0) and rho_N, loaded before anything
  // else (they do not depend on the staged state)
  const int N0 = p.gc[g].N;
  const int nch = N0 / FCN + 1;
  double ptot = 0.0, pw = 0.0, rhoN = 0.0;
  if (tid < 64) {
    const double *pt = p.fpart + ((size_t)g * NCHMAX + min(tid, nch - 1)) * 2;
    ptot = pt[0];
    pw = pt[1];
    rhoN = p.rho64[p.gc[g].nbase + N0];
    if (tid >= nch) ptot = pw = 0.0;
  }
  // stage the gap's constants, state and last push's tallies: word tid of
  // their concatenation per thread, one load and one LDS store with no branch
  // (a guarded load is waited for inside its branch); the tallies are cleared at
  // the kernel's end
  {
    constexpr int NC = (int)(sizeof(GapConst) / 8), NS = (int)(sizeof(GapState) / 8);
    constexpr int NW = (int)(sizeof(Staged) / 8);
    static_assert(sizeof(Staged) == sizeof(GapConst) + sizeof(GapState) + 8 * (T_N + 2) && NW <= FBS,
                  "one staged word per thread");
    const unsigned long long *src =
        tid < NC ? (const unsigned long long *)&p.gc[g] + tid
        : tid < NC + NS ? (const unsigned long long *)&p.gs[g] + (tid - NC)
        : tid < NC + NS + T_N ? p.tally + (size_t)g * T_N + (tid - NC - NS)
                              : p.next_count + (size_t)g * 2 + min(tid - NC - NS - T_N, 1);
    const unsigned long long v = *src;
    if (tid < NW) ((unsigned long long *)&stg)[tid] = v;
  }
  __syncthreads();
  // the beam of the step that solves level n = level + 1: its schedule entry,
  // else the fixed count
  // (read from a clamped index and chosen afterwards, through an index the
  // compiler takes for a per-lane one: a load on each side of the choice would
  // become one flat load, and a uniform one a scalar load, either of which every
  // later barrier's wait on LDS would also wait for; the schedule array holds
  // at least one entry)
  long long nbeam;
  {
    const long long n = ss.level + 1;
    int lane0 = 0;
    asm volatile("" : "+v"(lane0));
    const long long ix = sc.sched_len > 0 ? sc.sched_base + min(n, sc.sched_len - 1) : 0;
    const long long v = (long long)p.sched[ix + lane0];
    nbeam = n < sc.sched_len ? v : sc.beam_n;
  }

  // 0. strict coupling: the guess network's input (the last 8 levels from the
  //    history ring), recorded for training and/or evaluated for the guess
  const bool want_mlp = mode == 0 && guess == GS_GUESS_MLP && p.mlp_w != nullptr;
  const bool want_rec = mode == 0 && p.rec_x != nullptr;
  const long long rec_idx = (ss.level + 1 - p.rec_level0) * (long long)gridDim.x + g;
  const bool rec_here = want_rec && rec_idx >= 0 && rec_idx < p.rec_cap;
  if (want_mlp || rec_here) {
    if (tid < MLP_IN) {
      // block k = 1..8: (V, I_0, I_1, sigma) of level n-k and the absorbed /
      // emitted charge of the push that followed it (for k = 1 the push whose
      // tallies this solve is about to fold in)
      const int kk = tid / 6 + 1, q = tid % 6;
      double raw;
      if (q < 4) {
        raw = ss.hist[(ss.hist_head - kk) & 7][q];
      } else if (kk > 1) {
        raw = ss.hist[(ss.hist_head - kk + 1) & 7][q];
      } else {
        const double qi = sc.A * (sc.s0 * (double)sc.Z[1]), qe = sc.A * (sc.s0 * (double)sc.Z[0]);
        raw = q == 4 ? qi * (double)(long long)s_tally[T_ABS + 2] + qe * (double)(long long)s_tally[T_ABS + 0]
                     : qe * (double)(long long)s_tally[T_EMIT + 0];
      }
      if (rec_here) p.rec_x[rec_idx * MLP_IN + tid] = (float)raw;
      if (want_mlp) s_x[tid] = (float)((raw - p.mlp_norm[tid]) / p.mlp_norm[MLP_IN + tid]);
    }
    if (tid == 0)
      for (int i = 0; i <= sc.M; ++i) s_ue[i] = 3.0 * ss.uh[0][i] - 3.0 * ss.uh[1][i] + ss.uh[2][i];
    if (want_mlp) {
      mlp_eval_block(p.mlp_w, s_x, s_h0, s_h1, s_y);
      if (tid == 0)
        for (int i = 0; i < MLP_OUT; ++i)
          s_mu[i] = s_ue[i] + p.mlp_norm[2 * MLP_IN + i] + p.mlp_norm[2 * MLP_IN + MLP_OUT + i] * (double)s_y[i];
    }
  }

  const int N = sc.N;
  const double dx = sc.dx, eps0 = sc.eps0, s0 = sc.s0;
  unsigned long long *acc = p.acc + sc.nbase;
  double *rho = p.rho64 + sc.nbase;
  double *E = p.E64 + sc.nbase;

  // 1. the chunks' offsets O_c (exclusive prefix of their totals) for
  //    k_ftable, the total S_{N-1} and sum_k S_k = sum_k c_k (N - k)
  if (tid < 64) {
    double run = ptot;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const double t = __shfl_up(run, o, 64);
      if (tid >= o) run += t;
    }
    double wsumall = pw;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) wsumall += __shfl_xor(wsumall, o, 64);
    const double tot = __shfl(run, 63, 64);
    if (tid < nch) p.foff[(size_t)g * NCHMAX + tid] = run - ptot;
    // 2. circuit and surface charge
    if (tid == 0) {
      const double dx = sc.dx, eps0 = sc.eps0;
      const double P = wsumall * dx / eps0;
      double sg;
      // space charge: the cell terms (rho_0 at half weight) plus the half cell at node N
      ss.q_space = sc.A * (tot + 0.5 * dx * rhoN);
      solve_level(p, g, sc, ss, P, mode, guess, tol, maxit, &sg, s_work, s_tally, want_mlp ? s_mu : nullptr,
                  stg.next_count, nbeam);
      p.fsig[g] = sg;
      const size_t eb = (size_t)sc.ebase;
      if (fp64)
        ((double *)p.ehat)[eb] = sg / eps0;
      else
        ((float *)p.ehat)[eb] = (float)(sg / eps0);
      if (rec_here)
        for (int i = 0; i < MLP_OUT; ++i)
          p.rec_y[rec_idx * MLP_OUT + i] = i <= sc.M ? (float)(ss.uh[0][i] - s_ue[i]) : 0.0f;
    }
  }
  __syncthreads();
  {
    const unsigned long long *a = (const unsigned long long *)&ss;
    unsigned long long *b = (unsigned long long *)&p.gs[g];
    for (int i = tid; i < (int)(sizeof(GapState) / 8); i += FBS) b[i] = a[i];
  }
  if (tid < T_N) p.tally[(size_t)g * T_N + tid] = 0ull;
}

// k_ftable: the half-grid field E_{k+1/2} = (sigma + S_k) / eps0, S_k = O_c +
// L_k, for the cells k < N of chunk c of gap g, and the push's gather table
// (E at the electrode, the half-grid values, and at node N the field the half
// cell's charge adds to the last value; that one is also the gap's e_ground).
__global__ __launch_bounds__(FDB) void k_ftable(DevPtrs p, int fp64) {
  const int g = blockIdx.y, c = blockIdx.x, tid = threadIdx.x;
  const GapConst &gc = p.gc[g];
  const int N = gc.N;
  if (c * FCN >= N) return;  // (the whole workgroup)
  const int kb = c * FCN + 4 * tid;
  const double *sl = p.fsl + gc.nbase;
  double *E = p.E64 + gc.nbase;
  const double off = p.foff[(size_t)g * NCHMAX + c], sigma = p.fsig[g];
  const double eps0 = gc.eps0, dx = gc.dx;
  const size_t eb = (size_t)gc.ebase;
  double L[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) L[i] = sl[min(kb + i, N - 1)];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int k = kb + i;
    if (k >= N) break;
    const double e = (sigma + (off + L[i])) / eps0;
    E[k] = e;
    if (fp64)
      ((double *)p.ehat)[eb + k + 1] = e;
    else
      ((float *)p.ehat)[eb + k + 1] = (float)e;
    if (k == N - 1) {
      const double ed = e + dx * p.rho64[gc.nbase + N] / (2.0 * eps0);
      p.gs[g].e_ground = ed;
      if (fp64)
        ((double *)p.ehat)[eb + N + 1] = ed;
      else
        ((float *)p.ehat)[eb + N + 1] = (float)ed;
    }
  }
}

#endif  // GS_PUSH_PART

// Launch with or without packet-recorded timing events.
template <typename K, typename... A>
static hipError_t launch_k(K kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s, hipEvent_t ea,
                           hipEvent_t eb, A... args) {
  if (ea || eb)
    hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)lds, s, ea, eb, 0u, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// k_push
// ---------------------------------------------------------------------------
// Charge accumulation in LDS, one cell per node.  The push deposits the
// unsigned CIC weights of one species (in units of 2^-24 or 2^-44 of a
// macroparticle); the species' charge number multiplies the sums when they are
// flushed to the gap's 64-bit node row.
//   Wide64  64-bit cells, non-returning adds (whenever the grid fits in LDS);
//   Carry32 32-bit cells (binary32 particles, largest grids); a cell that wraps
//           carries Z * 2^32 into the gap's row.
// Both give the exact integer sum, so the deposit is order independent.
struct Wide64 {
  typedef unsigned long long cell;
};
struct Carry32 {
  typedef unsigned int cell;
};

// 16-byte vectors of particle coordinates
template <class P>
struct Vec;
template <>
struct Vec<float> {
  typedef float4 type;
  static constexpr int n = 4;
  __device__ static inline float &at(float4 &v, int k) {
    return k == 0 ? v.x : k == 1 ? v.y : k == 2 ? v.z : v.w;
  }
};
template <>
struct Vec<double> {
  typedef double2 type;
  static constexpr int n = 2;
  __device__ static inline double &at(double2 &v, int k) { return k == 0 ? v.x : v.y; }
};

// Particle-stream loads and stores, with NT marked non-temporal: a stream far
// larger than the caches then does not evict what they hold, nor wait for
// allocations in them.  (A compile-time switch: a run-time one lets the
// compiler merge the two loads and drop the marking.)
template <class V>
struct NatV;
template <>
struct NatV<float4> {
  typedef float t __attribute__((ext_vector_type(4)));
};
template <>
struct NatV<double2> {
  typedef double t __attribute__((ext_vector_type(2)));
};
template <bool NT, class V>
__device__ inline V ld_stream(const V *a) {
  typedef typename NatV<V>::t N;
  V v;
  if (NT) {
    const N r = __builtin_nontemporal_load((const N *)a);
    __builtin_memcpy(&v, &r, sizeof(V));
  } else {
    v = *a;
  }
  return v;
}
template <bool NT, class V>
__device__ inline void st_stream(V *a, V v) {
  typedef typename NatV<V>::t N;
  if (NT) {
    N r;
    __builtin_memcpy(&r, &v, sizeof(V));
    __builtin_nontemporal_store(r, (N *)a);
  } else {
    *a = v;
  }
}

template <class P>
struct Prec;
template <>
struct Prec<float> {
  static constexpr float ONE_W = 16777216.0f;  // 2^24
  static constexpr long long W = 16777216ll;
  typedef unsigned int wt;
  __device__ static inline wt wq(float f) { return __float2uint_rn(f * ONE_W); }
};
template <>
struct Prec<double> {
  static constexpr double ONE_W = 17592186044416.0;  // 2^44
  static constexpr long long W = 17592186044416ll;
  typedef unsigned long long wt;
  __device__ static inline wt wq(double f) { return (unsigned long long)__double2ll_rn(f * ONE_W); }
};

// Linear gather from the extended half-grid table eh[0..N+1]:
// eh[0] = surface field at node 0, eh[k] = E_{k-1/2}, eh[N+1] = field at node N.
// All three cases are evaluated and one is selected (no divergent branches);
// each case is the same IEEE operation sequence as its branch form.
template <class P>
__device__ inline P gather(const P *eh, P xi, int N, P Nh) {
  const P h = xi - (P)0.5;
  const int j = (int)h;
  const P ti = h - (P)j;
  const P tl = xi + xi;
  P tr = xi - Nh;
  tr = tr + tr;
  const bool L = xi < (P)0.5, R = xi >= Nh;
  const int k = L ? 0 : (R ? N : j + 1);
  const P t = L ? tl : (R ? tr : ti);
  const P a = eh[k];
  const P b = eh[k + 1];
  const P dlt = b - a;
  const P m = t * dlt;
  return a + m;
}

template <class AC>
__device__ inline void acc_add(typename AC::cell *lds, unsigned long long *gacc, int j, unsigned long long w,
                               long long zhi);
template <>
__device__ inline void acc_add<Wide64>(unsigned long long *lds, unsigned long long *, int j,
                                       unsigned long long w, long long) {
  atomicAdd(&lds[j], w);
}
template <>
__device__ inline void acc_add<Carry32>(unsigned int *lds, unsigned long long *gacc, int j, unsigned long long w,
                                        long long zhi) {
  const unsigned int uw = (unsigned int)w;
  const unsigned int old = atomicAdd(&lds[j], uw);
  if (old + uw < old) atomicAdd(&gacc[j], (unsigned long long)zhi);
}

// Emission for the events [r0, r0 + nr) of gap g's list (every thread of the
// block): the electrons, their wall charge added to the gap's node row and
// their counts to its tallies, keyed by the gap's level as in the push that
// queued them.  s_base and s_emit are LDS scratch.
template <class P>
__device__ void emit_list(const DevPtrs &p, int g, int sel, long long r0, int nr, int *wsum,
                          unsigned long long *s_base, unsigned int *s_emit) {
  const GapConst &c = p.gc[g];
  const long long level = p.gs[g].level;
  if (threadIdx.x < 2) s_emit[threadIdx.x] = 0u;
  __syncthreads();
  see_emit<P>(p, c, level, g, sel, p.ev + c.evbase + r0, nr, wsum, s_base, s_emit);
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned int e0 = s_emit[0], e1 = s_emit[1];
    const long long ze = (long long)c.Z[0] * Prec<P>::W;
    unsigned long long *gacc = p.acc + c.nbase;
    if (e0) {
      atomicAdd(&gacc[0], (unsigned long long)(ze * (long long)e0));
      atomicAdd(&p.tally[(size_t)g * T_N + T_EMIT], (unsigned long long)e0);
    }
    if (e1) {
      atomicAdd(&gacc[c.N], (unsigned long long)(ze * (long long)e1));
      atomicAdd(&p.tally[(size_t)g * T_N + T_EMIT + 1], (unsigned long long)e1);
    }
    atomicAdd(&p.ev_done[g], (unsigned long long)nr);
  }
  __syncthreads();
}

constexpr int EVQ = 128;  // absorbed-ion events a push workgroup queues in LDS
// (more go to the workgroup's overflow region of a global buffer; both are
// emitted at the segment's flush, so a step's emission completes in its push)

template <class P, class AC>
struct PushShared {
  P *eh;
  typename AC::cell *acc;
  int *prefix;          // [G + 1]
  unsigned int *tally;  // [T_N]
  Event *evq;           // [EVQ]
  unsigned int *evq_n;
  int *wsum;            // [BS / 64] scan scratch
  unsigned int *listed; // the workgroup put absorbed ions in a gap's list (set
                        // when a segment is closed: its queue count passed the
                        // LDS queue and the overflow region)
  int masks;            // the launch writes the live masks
};

// push tiles of gap g: electrons, then ions (a gap with a beam has at least
// one ion tile: the workgroups holding its ion tiles inject the beam)
// (counts are below 2^31: 32-bit division, a fraction of the 64-bit code)
__device__ inline int tiles_of(long long count, int tile) {
  const unsigned int c = (unsigned int)count, t = (unsigned int)tile;
  const unsigned int q = c / t;
  return (int)(q + (c - q * t != 0u ? 1u : 0u));
}

__device__ inline void gap_tiles(const GapState &st, long long beam_n, int tile, int &te, int &ti) {
  te = tiles_of(st.count[0], tile);
  ti = tiles_of(st.count[1], tile);
  if (beam_n > 0 && ti == 0) ti = 1;
}


// Beam ions k0..k1-1 of gap g entering at the circuit electrode: energy
// uniform in [E_min, E_max], placed a random fraction of one step's flight into
// the gap, keyed by (level, k); slots count[1] + k and ids beam_id0 + k were
// set aside by the field solve.  Their charge goes to the ion segment's LDS
// accumulator.
template <class P, class AC>
__device__ void beam_inject(const DevPtrs &p, const GapConst &c, const GapState &st, int g, int sel, long long k0,
                            long long k1, typename AC::cell *acc, unsigned int *n_inj) {
  P *X = (P *)p.X[sel] + c.pbase[1];
  P *U = (P *)p.U[sel] + c.pbase[1];
  uint32_t *ID = p.ID[sel] + c.pbase[1];
  unsigned long long *gacc = p.acc + c.nbase;
  const int N = c.N;
  const long long zhi = (long long)c.Z[1] * 4294967296ll;
  unsigned int cnt = 0;
  for (long long k = k0 + threadIdx.x; k < k1; k += blockDim.x) {
    uint64_t blk[4];
    rng_block(c.seed, (uint64_t)st.level, (uint64_t)k, 2, 0, blk);
    const double E = c.beam_Emin + (c.beam_Emax - c.beam_Emin) * unit_open(blk[0]);
    const double v = sqrt(2.0 * E * c.ev / c.mass[1]);
    // depth below the entry electrode: within the layer, or within one step's flight
    const double depth = unit_open(blk[1]) * (c.beam_layer > 0.0 ? c.beam_layer : v * c.dt);
    const double x = c.beam_side == GS_BEAM_GROUND ? c.d - depth : depth;
    const P xi = (P)(x / c.dx);
    const double uv = (v * c.dt) / c.dx;
    const P u = (P)(c.beam_side == GS_BEAM_GROUND ? -uv : uv);
    const unsigned long long slot = (unsigned long long)st.count[1] + (unsigned long long)k;
    if (slot >= (unsigned long long)c.cap[1]) {
      atomicOr(&p.err[0], ERR_CAPACITY);
      atomicCAS(&p.err[1], 0xFFFFFFFFu, (unsigned int)g);
      continue;
    }
    X[slot] = xi;
    U[slot] = u;
    ID[slot] = (uint32_t)(st.beam_id0 + k);
    cnt += 1;
    int j = (int)xi;
    if (j > N - 1) j = N - 1;
    const P f = xi - (P)j;
    const typename Prec<P>::wt w1 = Prec<P>::wq(f);
    const typename Prec<P>::wt w0 = (typename Prec<P>::wt)Prec<P>::W - w1;
    acc_add<AC>(acc, gacc, j, (unsigned long long)w0, zhi);
    acc_add<AC>(acc, gacc, j + 1, (unsigned long long)w1, zhi);
  }
  const unsigned int a = wave_sum(cnt);
  if ((threadIdx.x & 63) == 0 && a) atomicAdd(n_inj, a);
}

// Emission for the events [r0, r0 + blockDim) of a segment's queue (the LDS
// queue, then the workgroup's overflow region): one per thread, counts drawn,
// one slot reservation for the electrons, which are written; returns the
// reservation's total.  The first round also flushes the node sums while its
// reservation is in flight.
template <class P, class AC>
__device__ inline int emit_round(const DevPtrs &p, const GapConst &c0, const GapState &st, int g, int s, int sel,
                                 PushShared<P, AC> &sh, const Event *ovf, int ne, int r0,
                                 unsigned long long *s_base) {
  // the emission's constants are read here, not at the kernel's start (held
  // in registers across the push they would spill)
  // (the pointer is the workgroup's: moved to scalar registers half by half,
  // which the empty asm then pins)
  const unsigned long long cu = (unsigned long long)&c0;
  const GapConst *cp = (const GapConst *)(((unsigned long long)(unsigned int)__builtin_amdgcn_readfirstlane(
                                               (int)(cu >> 32)) << 32) |
                                          (unsigned int)__builtin_amdgcn_readfirstlane((int)cu));
  asm volatile("" : "+s"(cp));
  const GapConst &c = *cp;
  const int i = r0 + (int)threadIdx.x;
  uint32_t ion_id = 0;
  int wall = 0, nk = 0;
  double u_imp = 0.0;
  if (i < ne) {
    const Event ev = i < EVQ ? sh.evq[i] : ovf[i - EVQ];
    ion_id = p.ID[sel][c.pbase[1] + ev.ref];
    wall = (int)ev.wall;
    u_imp = ev.u;
  }
  uint64_t blk[4] = {0, 0, 0, 0};
  if (i < ne) nk = see_count(c, st.level, ion_id, u_imp, blk);
  int btot = 0, excl = 0;
  if (r0 < ne)
    excl = block_exclusive_scan_i(nk, sh.wsum, &btot);
  else
    __syncthreads();
  unsigned long long base = 0;
  if (threadIdx.x == 0 && btot > 0) base = atomicAdd(&p.next_count[g * 2 + 0], (unsigned long long)btot);
  if (r0 == 0) {
    // node sums; each workgroup starts at its own node so that the workgroups
    // flushing at the same time add to different addresses
    unsigned long long *gacc = p.acc + c.nbase;
    const long long Z = (long long)c.Z[s];
    const int nn = c.N + 1;
    const int rot = (int)(((long long)blockIdx.x * 977) % nn);
    for (int q = threadIdx.x; q < nn; q += blockDim.x) {
      int j = q + rot;
      j = j >= nn ? j - nn : j;
      const unsigned long long v = (unsigned long long)sh.acc[j];
      if (v != 0ull) atomicAdd(&gacc[j], (unsigned long long)(Z * (long long)v));
    }
  }
  if (btot > 0) {
    if (threadIdx.x == 0) *s_base = base;
    __syncthreads();
    unsigned int n[2] = {0u, 0u};
    if (nk > 0) see_write<P>(p, c, st.level, g, sel, ion_id, wall, nk, blk, *s_base + (unsigned long long)excl, n);
    const unsigned int a0 = wave_sum(n[0]), a1 = wave_sum(n[1]);
    if ((threadIdx.x & 63) == 0) {
      if (a0) atomicAdd(&sh.tally[T_EMIT], a0);
      if (a1) atomicAdd(&sh.tally[T_EMIT + 1], a1);
    }
    __syncthreads();
  }
  return btot;
}

// Close one (gap, species) segment: for the ion segment emit the secondary
// electrons of the ions this workgroup absorbed, in rounds of one event per
// thread (the first round also hands the node sums times the charge number to
// the gap); then the emitted electrons' wall charge and the tallies.
template <class P, class AC>
__device__ void flush_seg(const DevPtrs &p, const GapConst &c, const GapState &st, int g, int s, int sel,
                          PushShared<P, AC> &sh) {
  __shared__ unsigned long long s_base;
  __syncthreads();
  const int ovq = (long long)blockIdx.x < p.ovf_wgs ? (int)p.ovq : 0;
  const int ne = s == 1 ? (int)min(*sh.evq_n, (unsigned int)(EVQ + ovq)) : 0;
  if (s == 1 && threadIdx.x == 0 && *sh.evq_n > (unsigned int)(EVQ + ovq)) *sh.listed = 1u;
  const Event *ovf = p.ovf + (size_t)blockIdx.x * (size_t)p.ovq;
  // one inlined copy of the round (the kernel's instruction footprint matters)
  int emitted = 0, r0 = 0;
  do {
    emitted += emit_round<P, AC>(p, c, st, g, s, sel, sh, ovf, ne, r0, &s_base);
    r0 += blockDim.x;
  } while (r0 < ne);
  if (emitted > 0 && threadIdx.x == 0) {
    // an emitted electron carries its full weight on its wall node
    unsigned long long *gacc = p.acc + c.nbase;
    const long long ze = (long long)c.Z[0] * Prec<P>::W;
    const unsigned int e0 = sh.tally[T_EMIT], e1 = sh.tally[T_EMIT + 1];
    if (e0) atomicAdd(&gacc[0], (unsigned long long)(ze * (long long)e0));
    if (e1) atomicAdd(&gacc[c.N], (unsigned long long)(ze * (long long)e1));
  }
  // the tallies, one per thread; the empty asm keeps the compiler from
  // computing the per-thread address once at the kernel's start and holding it
  // (spilled) across the push
  int t = (int)threadIdx.x;
  asm volatile("" : "+v"(t));
  if (t < T_N) {
    const unsigned int v = sh.tally[t];
    if (v) atomicAdd(&p.tally[(size_t)g * T_N + t], (unsigned long long)v);
  }
  __syncthreads();
}

// Stage one (gap, species) segment: clear the node accumulator and the
// tallies, inject this workgroup's share of the beam, and copy the gap's field
// table (16-byte aligned, N + 2 entries) into LDS with 16-byte loads, the
// first TQ per thread issued before anything else.  The table is the gap's,
// for either species: table is false when LDS already holds it (the previous
// segment was the gap's other species).
template <class P, class AC>
__device__ void load_seg(const DevPtrs &p, const GapConst &c, const GapState &st, int g, int sel,
                         PushShared<P, AC> &sh, long long kb0, long long kb1, bool table) {
  // the table moves as 16-byte vectors of a native vector type (arrays of it
  // stay in registers)
  typedef unsigned int V __attribute__((ext_vector_type(4)));
  constexpr int TQ = 5;  // table vectors per thread whose loads go out first
  const V *geh = (const V *)((const P *)p.ehat + c.ebase);
  V *leh = (V *)sh.eh;
  const int nv = (int)(((size_t)(c.N + 2) * sizeof(P) + 15) / 16);
  const int bs = blockDim.x;
  const int tid = threadIdx.x;
  // loads past the table repeat its last vector
  V t[TQ];
  if (table) {
#pragma unroll
    for (int q = 0; q < TQ; ++q) t[q] = geh[min(tid + q * bs, nv - 1)];
  }
  for (int j = tid; j <= c.N; j += bs) sh.acc[j] = 0;
  if (tid < T_N) sh.tally[tid] = 0u;
  if (tid == 0) *sh.evq_n = 0u;
  // the beam goes in while the table's loads are in flight (the beam's slots
  // lie past the swept range; its charge only has to reach the next density)
  if (kb1 > kb0) {
    __syncthreads();
    beam_inject<P, AC>(p, c, st, g, sel, kb0, kb1, sh.acc, &sh.tally[T_INJ]);
  }
  if (table) {
#pragma unroll
    for (int q = 0; q < TQ; ++q)
      if (tid + q * bs < nv) leh[tid + q * bs] = t[q];
    for (int j0 = tid + TQ * bs; j0 < nv; j0 += 4 * bs) {
      V r[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) r[q] = geh[min(j0 + q * bs, nv - 1)];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (j0 + q * bs < nv) leh[j0 + q * bs] = r[q];
    }
  }
  __syncthreads();
}

// Per-thread running counts of one segment.
struct SegCount {
  unsigned int pushed = 0, abs0 = 0, abs1 = 0;
};

// The gap constants one segment's push needs, held in registers (a reference
// into global memory would be re-read after every store).
struct SegK {
  int N;
  int g;
  int masks;  // write the live masks (a compaction follows this push)
  long long evbase, evcap;
  unsigned long long *gacc;
  const uint32_t *ids;        // the region's particle ids (overflowing events carry the id)
  unsigned long long *live;   // the region's live masks, one word per 64 slots
};

// Push one chunk of BS * PPT slots starting at slot r0 (relative to the region
// base): thread tid owns slots r0 + (v * BS + tid) * VN + kk.  FULL: every slot
// lies below n_here, so vectors are stored whole; otherwise slot by slot.
template <class P, class AC, int BS, int PPT, bool FULL, bool NT>
__device__ inline void push_chunk(const DevPtrs &p, const SegK &c, PushShared<P, AC> &sh, P *X, P *U,
                                  long long r0, long long n_here, typename Vec<P>::type *xv,
                                  typename Vec<P>::type *uv, P alpha, bool see, long long zhi, SegCount &cnt) {
  typedef typename Vec<P>::type V;
  constexpr int VN = Vec<P>::n;
  constexpr int NV = PPT / VN;
  const int tid = threadIdx.x;
  const int N = c.N;
  const int g = c.g;
  const P Nf = (P)N;
  const P Nh = Nf - (P)0.5;
  // slots that deposit nothing add zero at a node of their own (no
  // same-address LDS atomics within a wave)
  const int jdummy = (int)(threadIdx.x % (unsigned int)N);
  int jj[PPT];
  typename Prec<P>::wt w0[PPT], w1[PPT];
  unsigned int hit = 0;  // bit k: slot k is an absorbed ion (its wall in bit k+16)
  unsigned int alive = 0;  // bit k: slot k holds a particle after the push
  P u_hit[PPT];
  V xw[NV], uw[NV];
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int v = k / VN, kk = k % VN;
    const P xi = Vec<P>::at(xv[v], kk);
    const P u0 = Vec<P>::at(uv[v], kk);
    // empty slots and absorbed particles hold -1
    const bool live = xi >= (P)0;
    // gather, then the leapfrog (eq. vel_update_main, eq. pos_update_main)
    const P Ep = gather<P>(sh.eh, xi, N, Nh);
    const P du = alpha * Ep;
    const P u1 = u0 + du;
    const P x1 = xi + u1;
    const bool a0 = x1 <= (P)0;
    const bool a1 = !a0 && x1 >= Nf;
    const bool gone = live && (a0 || a1);
    const bool stay = live && !(a0 || a1);
    Vec<P>::at(xw[v], kk) = stay ? x1 : (P)-1;
    Vec<P>::at(uw[v], kk) = stay ? u1 : u0;
    alive |= (unsigned int)stay << k;
    cnt.pushed += live;
    cnt.abs0 += live && a0;
    cnt.abs1 += live && a1;
    hit |= ((unsigned int)gone << k) | ((unsigned int)(live && a1) << (k + 16));
    u_hit[k] = u1;
    // deposit with the gather's weights (App. C)
    const P xs = stay ? x1 : (P)0;
    int j = (int)xs;
    j = j > N - 1 ? N - 1 : j;
    j = stay ? j : jdummy;
    const P f = xs - (P)j;
    const typename Prec<P>::wt q1 = Prec<P>::wq(f);
    jj[k] = j;
    w1[k] = stay ? q1 : (typename Prec<P>::wt)0;
    w0[k] = stay ? (typename Prec<P>::wt)Prec<P>::W - q1 : (typename Prec<P>::wt)0;
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const long long i = r0 + (long long)(v * BS + tid) * VN;
    if (FULL) {
      st_stream<NT>((V *)(X + i), xw[v]);
      st_stream<NT>((V *)(U + i), uw[v]);
    } else {
#pragma unroll
      for (int k = 0; k < VN; ++k)
        if (i + k < n_here) {
          X[i + k] = Vec<P>::at(xw[v], k);
          U[i + k] = Vec<P>::at(uw[v], k);
        }
    }
  }
  if (c.masks) {
    // a compaction follows: the slots' liveness after this push, as whole
    // 64-slot words of the region's live masks (the lanes of a word gather
    // their bits; the compaction reads positions only for the words left)
    constexpr int LPW = 64 / VN;  // lanes per word
    const int lane = tid & 63;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      unsigned long long m = (unsigned long long)((alive >> (v * VN)) & ((1u << VN) - 1u))
                             << (VN * (lane % LPW));
#pragma unroll
      for (int o = 1; o < LPW; o <<= 1) m |= __shfl_xor(m, o, 64);
      const long long i = r0 + (long long)(v * BS + tid) * VN;
      if (lane % LPW == 0 && (FULL || i + 64 <= n_here)) c.live[i / 64] = m;
    }
  }
  // every slot adds (zero weights for slots that do not deposit): no branches
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    acc_add<AC>(sh.acc, c.gacc, jj[k], (unsigned long long)w0[k], zhi);
    acc_add<AC>(sh.acc, c.gacc, jj[k] + 1, (unsigned long long)w1[k], zhi);
  }
  // absorbed ions are queued for secondary emission: in LDS (emitted at the
  // segment's flush), then in the workgroup's overflow region, then in the
  // gap's list (emitted at the end of the push by its last workgroup, or by
  // k_emit after it).  The wave
  // takes its queue positions, and its share of the gap's list, with one atomic
  // each: a workgroup whose particles sit at a wall (sorted particles) absorbs
  // thousands of ions in one push, and an atomic per ion on the gap's counter
  // would serialise them.
  if (see) {
    const int nh = __popc(hit & 0xFFFFu);
    if (__ballot(nh != 0) != 0ull) {
      const int lane = tid & 63;
      const int incl = wave_incl_scan(nh);
      const unsigned int tot = (unsigned int)__shfl(incl, 63, 64);
      unsigned int q0 = 0;
      if (lane == 0) q0 = atomicAdd(sh.evq_n, tot);
      q0 = (unsigned int)__shfl((int)q0, 0, 64);
      const unsigned int lim = (unsigned int)EVQ + ((long long)blockIdx.x < p.ovf_wgs ? (unsigned int)p.ovq : 0u);
      const unsigned int over0 = q0 > lim ? q0 : lim;
      const unsigned int n_over = q0 + tot > lim ? q0 + tot - over0 : 0u;
      unsigned long long gb = 0;
      if (n_over && lane == 0) gb = atomicAdd(&p.ev_count[g], (unsigned long long)n_over);
      gb = __shfl(gb, 0, 64);
      unsigned int q = q0 + (unsigned int)(incl - nh);
      unsigned int rest = hit & 0xFFFFu;
      while (rest) {
        const int k = __ffs(rest) - 1;
        rest &= rest - 1u;
        Event ev;
        P uk = u_hit[0];
#pragma unroll
        for (int j = 1; j < PPT; ++j)
          if (j == k) uk = u_hit[j];
        ev.u = (double)uk;
        ev.ref = (uint32_t)(r0 + (long long)((k / VN) * BS + tid) * VN + k % VN);
        ev.wall = (hit >> (k + 16)) & 1u;
        if (q < (unsigned int)EVQ) {
          sh.evq[q] = ev;
        } else if (q < lim) {
          p.ovf[(size_t)blockIdx.x * (size_t)p.ovq + (q - EVQ)] = ev;
        } else {
          const unsigned long long e = gb + (unsigned long long)(q - over0);
          if (e < (unsigned long long)c.evcap) {
            ev.ref = c.ids[ev.ref];
            p.ev[c.evbase + e] = ev;
          } else {
            atomicOr(&p.err[0], ERR_CAPACITY);
            atomicCAS(&p.err[1], 0xFFFFFFFFu, (unsigned int)g);
          }
        }
        q += 1u;
      }
    }
  }
}

template <class P, int BS, int PPT, bool NT>
__device__ inline void load_chunk(const P *X, const P *U, long long r0, typename Vec<P>::type *xo,
                                  typename Vec<P>::type *uo) {
  typedef typename Vec<P>::type V;
  constexpr int VN = Vec<P>::n;
#pragma unroll
  for (int v = 0; v < PPT / VN; ++v) {
    const long long i = r0 + (long long)(v * BS + threadIdx.x) * VN;
    xo[v] = ld_stream<NT>((const V *)(X + i));
    uo[v] = ld_stream<NT>((const V *)(U + i));
  }
}

// Slots of one (gap, species) region as a stream of chunks: nrun runs of
// `run` slots (a multiple of the chunk), `step` slots apart, from slot a; the
// last run ends at b.  (One run: a contiguous range; several: the tiles a
// workgroup takes in round-robin order.)  Full chunks are software-pipelined,
// across runs too: the loads of the next chunk are in flight while this one is
// pushed.  Every load in the loop is unconditional (past the last full chunk
// it repeats that chunk's, whose data is dropped), so the waits count exactly.
// The remainder goes slot by slot: slots past b may be receiving appended
// particles.
template <class P, class AC, int BS, int PPT, bool NT>
__device__ void push_range(const DevPtrs &p, const GapConst &gc, const GapState &st, int g, int s, int sel,
                           PushShared<P, AC> &sh, long long a, long long b, long long run, long long step,
                           int nrun, long long kb0, long long kb1, bool stage, bool table, SegCount &cnt) {
  typedef typename Vec<P>::type V;
  constexpr int VN = Vec<P>::n;
  constexpr int NV = PPT / VN;
  constexpr int CH = BS * PPT;
  SegK c;
  c.N = gc.N;
  c.g = g;
  c.evbase = gc.evbase;
  c.evcap = gc.evcap;
  c.gacc = p.acc + gc.nbase;
  c.ids = p.ID[sel] + gc.pbase[s];
  c.masks = sh.masks;
  c.live = p.live + gc.pbase[s] / 64;
  P *X = (P *)p.X[sel] + gc.pbase[s];
  P *U = (P *)p.U[sel] + gc.pbase[s];
  const P alpha = (P)gc.alpha[s];
  const bool see = (s == 1) && (gc.see_amp > 0.0) && (gc.Z[1] > 0);
  const long long zhi = (long long)gc.Z[s] * 4294967296ll;
  // runs before the last are whole (a later tile of the region exists)
  const int cpr = (int)(run / CH);
  const long long last = a + (long long)(nrun - 1) * step;
  const long long nfull = (long long)(nrun - 1) * cpr + (b > last ? (b - last) / CH : 0);
  V xa[NV], ua[NV], xb[NV], ub[NV];
  // the first chunk's loads are in flight while the segment is staged (or,
  // when the segment is already open, while this range's beam goes in)
  if (nfull > 0) load_chunk<P, BS, PPT, NT>(X, U, a, xa, ua);
  if (stage)
    load_seg<P, AC>(p, gc, st, g, sel, sh, kb0, kb1, table);
  else if (kb1 > kb0)
    beam_inject<P, AC>(p, gc, st, g, sel, kb0, kb1, sh.acc, &sh.tally[T_INJ]);
  // one copy of the chunk body (the kernel's instruction footprint is what
  // limits it): the next chunk's loads go out before this chunk is pushed,
  // and the buffers are swapped by register moves
  long long rb = a;  // the run holding the chunk being pushed, and its index there
  int ci = 0;
  for (long long q = 0; q < nfull; ++q) {
    long long rbn = rb;
    int cin = ci + 1;
    if (cin == cpr) {
      cin = 0;
      rbn += step;
    }
    const long long cur = rb + (long long)ci * CH;
    load_chunk<P, BS, PPT, NT>(X, U, q + 1 < nfull ? rbn + (long long)cin * CH : cur, xb, ub);
    push_chunk<P, AC, BS, PPT, true, NT>(p, c, sh, X, U, cur, b, xa, ua, alpha, see, zhi, cnt);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      xa[v] = xb[v];
      ua[v] = ub[v];
    }
    rb = rbn;
    ci = cin;
  }
  const long long r0 = rb + (long long)ci * CH;
  if (r0 < b) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const long long i = r0 + (long long)(v * BS + threadIdx.x) * VN;
#pragma unroll
      for (int k = 0; k < VN; ++k) {
        Vec<P>::at(xa[v], k) = (i + k < b) ? X[i + k] : (P)-1;
        Vec<P>::at(ua[v], k) = (i + k < b) ? U[i + k] : (P)0;
      }
    }
    push_chunk<P, AC, BS, PPT, false, NT>(p, c, sh, X, U, r0, b, xa, ua, alpha, see, zhi, cnt);
  }
}

// A piece is a run of tiles within one (gap, species) segment.  A segment
// stays open in LDS (table, node sums, event queue, tallies) while the
// workgroup's pieces continue it, and is flushed when the next piece belongs to
// another segment, or at the end.  (og, os): the open segment, og < 0 for none.
// (Plain functions, not lambdas: a closure holding the kernel's argument block
// by address would copy it to the stack.)
template <class P, class AC>
__device__ __forceinline__ void close_seg(const DevPtrs &p, PushShared<P, AC> &sh, int sel, int og, int os) {
  // (workgroup-uniform; made scalars for the emission's scalar loads)
  const int g = __builtin_amdgcn_readfirstlane(og), s = __builtin_amdgcn_readfirstlane(os);
  flush_seg<P, AC>(p, p.gc[g], p.gs[g], g, s, sel, sh);
}

template <class P, class AC, int BS, int PPT, bool NT>
__device__ __forceinline__ void push_piece(const DevPtrs &p, PushShared<P, AC> &sh, int tile, int sel, int g,
                                           int s, int ls, int le, int stride, int &og, int &os) {
  g = __builtin_amdgcn_readfirstlane(g);
  s = __builtin_amdgcn_readfirstlane(s);
  ls = __builtin_amdgcn_readfirstlane(ls);
  le = __builtin_amdgcn_readfirstlane(le);
  stride = __builtin_amdgcn_readfirstlane(stride);
  const GapConst &c = p.gc[g];
  const GapState &st = p.gs[g];
  int te, ti;
  gap_tiles(st, st.beam_now, tile, te, ti);
  const bool stage = !(g == og && s == os);
  const bool table = og != g;  // (LDS holds the table of the last gap staged)
  if (stage && og >= 0) close_seg<P, AC>(p, sh, sel, og, os);
  SegCount cnt;
  // the local tiles ls, ls + stride, ... below le (stride 1: the run [ls, le))
  const int nrun = stride == 1 ? 1 : (le - ls + stride - 1) / stride;
  const int lt = stride == 1 ? le - 1 : ls + (nrun - 1) * stride;
  const long long a = (long long)ls * tile;
  const long long b = min((long long)(lt + 1) * tile, st.count[s]);
  const long long run = stride == 1 ? (long long)(le - ls) * tile : (long long)tile;
  const long long step = stride == 1 ? run : (long long)stride * tile;
  // the beam: over a run of tiles it is split by the gap's ion tiles, tile lt
  // taking ions [beam lt / ti, beam (lt + 1) / ti); a strided piece (the one
  // piece of its workgroup in this region, first tile ls < stride) takes share
  // ls of min(ti, stride) equal shares, so that each workgroup injects its
  // ions at once rather than a few per tile
  long long kb0 = 0, kb1 = 0;
  if (s == 1) {
    const int nb = stride == 1 ? ti : min(ti, stride);
    kb0 = st.beam_now * ls / nb;
    kb1 = st.beam_now * (stride == 1 ? le : ls + 1) / nb;
  }
  push_range<P, AC, BS, PPT, NT>(p, c, st, g, s, sel, sh, a, b, run, step, nrun, kb0, kb1, stage, table, cnt);
  // wave-level sums, then one LDS atomic per wave
  const unsigned int v0 = wave_sum(cnt.pushed), v1 = wave_sum(cnt.abs0), v2 = wave_sum(cnt.abs1);
  if ((threadIdx.x & 63) == 0) {
    if (v0) atomicAdd(&sh.tally[T_PUSHED], v0);
    if (v1) atomicAdd(&sh.tally[T_ABS + s * 2 + 0], v1);
    if (v2) atomicAdd(&sh.tally[T_ABS + s * 2 + 1], v2);
  }
  og = g;
  os = s;
}

// the pieces of the global tiles [ta, tb) of gap g, whose tiles start at t_g
template <class P, class AC, int BS, int PPT, bool NT>
__device__ __forceinline__ void push_tiles(const DevPtrs &p, PushShared<P, AC> &sh, int tile, int sel, int g,
                                           int t_g, int ta, int tb, int &og, int &os) {
  int te, ti;
  gap_tiles(p.gs[g], p.gs[g].beam_now, tile, te, ti);
  const int la = ta - t_g, lb = tb - t_g;
  if (la < te) push_piece<P, AC, BS, PPT, NT>(p, sh, tile, sel, g, 0, la, min(lb, te), 1, og, os);
  if (lb > te) push_piece<P, AC, BS, PPT, NT>(p, sh, tile, sel, g, 1, max(la, te) - te, lb - te, 1, og, os);
}

// The gaps' lists of absorbed ions (the events past the workgroups' own
// queues) are complete once every workgroup has pushed its particles.  Each
// workgroup counts itself, before its last flush (which the count's return
// then overlaps), in the counter of its group (blockIdx.x mod TICKET_GROUPS, a
// cache line each, so that a large grid does not queue on one address); the
// high half counts those that added to a list, after making their entries
// visible device-wide.  The workgroup that completes a group adds the group
// to the top counter, and the one that completes that is the last: when some
// workgroup added to a list, it emits the lists after its flush, as k_emit
// would after the push.  It leaves every counter at zero for the next launch,
// and the number of list events it emitted in the host word from which the
// host chooses who emits the next push's lists.  (The grid is below 2^16
// workgroups.)  push_ticket returns, in thread 0, 0 for a workgroup that is
// not the last, else 1 + the number of workgroups that added to a list.
constexpr int TICKET_LINE = 32;    // counter words per cache line
constexpr int TICKET_GROUPS = 32;  // group counters (see the allocation of push_done)
template <class P, class AC>
__device__ __forceinline__ unsigned int push_ticket(const DevPtrs &p, PushShared<P, AC> &sh, int os) {
  __syncthreads();
  const unsigned int lim = (unsigned int)EVQ + ((long long)blockIdx.x < p.ovf_wgs ? (unsigned int)p.ovq : 0u);
  const bool listed = *sh.listed != 0u || (os == 1 && *sh.evq_n > lim);
  if (listed) {
    __threadfence();
    __syncthreads();
  }
  unsigned int last = 0u;
  if (threadIdx.x == 0) {
    constexpr unsigned int NG = (unsigned int)TICKET_GROUPS;
    const unsigned int q = blockIdx.x % NG;
    const unsigned int nq = (gridDim.x - q + NG - 1u) / NG;  // workgroups in group q
    const unsigned int add = listed ? 0x10001u : 1u;
    const unsigned int gq = atomicAdd(&p.push_done[TICKET_LINE * (1u + q)], add) + add;
    if ((gq & 0xFFFFu) == nq) {
      if (gq >> 16) __threadfence();  // the group's list entries, on to the last one
      const unsigned int add2 = 1u + ((gq >> 16) << 16);
      const unsigned int t = atomicAdd(&p.push_done[0], add2) + add2;
      if ((t & 0xFFFFu) == min(gridDim.x, NG)) last = 1u + (t >> 16);
    }
  }
  return last;
}

constexpr int LIST_CH = 1 << 20;  // events per emission call
template <class P, class AC>
__device__ __forceinline__ void push_tail_emit(const DevPtrs &p, PushShared<P, AC> &sh, int G, int sel,
                                               unsigned int ticket) {
  __shared__ unsigned int s_last;
  __shared__ unsigned long long s_mask[16];
  __shared__ unsigned long long s_base;
  __shared__ unsigned int s_emit[2];
  if (threadIdx.x == 0) s_last = ticket;
  __syncthreads();
  const unsigned int last = s_last;
  if (last == 0u) return;
  if (threadIdx.x <= (unsigned int)TICKET_GROUPS) p.push_done[TICKET_LINE * threadIdx.x] = 0u;
  if (last == 1u) {
    if (threadIdx.x == 0) *p.list_seen = 0ull;
    return;
  }
  __threadfence();
  unsigned long long seen = 0;  // list events emitted (the same in every thread)
  // the gaps with a list, blockDim.x at a time, as bit masks per wave
  for (int g0 = 0; g0 < G; g0 += (int)blockDim.x) {
    const int g = g0 + (int)threadIdx.x;
    const unsigned long long m = __ballot(g < G && p.ev_count[g] != 0ull);
    if ((threadIdx.x & 63) == 0) s_mask[threadIdx.x >> 6] = m;
    __syncthreads();
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      unsigned long long mm = s_mask[w];
      while (mm != 0ull) {
        const int gg = g0 + w * 64 + (__ffsll((unsigned long long)mm) - 1);
        mm &= mm - 1ull;
        const long long ne = min((long long)p.ev_count[gg], p.gc[gg].evcap);
        seen += (unsigned long long)ne;
        for (long long r0 = 0; r0 < ne; r0 += LIST_CH)
          emit_list<P>(p, gg, sel, r0, (int)min((long long)LIST_CH, ne - r0), sh.wsum, &s_base, s_emit);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *p.list_seen = seen;
}

template <class P, class AC, int BS, int PPT, bool NT>
__global__ __launch_bounds__(BS, 3) void k_push(DevPtrs p, int G, int tile, int nmax, int steal, int rr,
                                                 int masks, int lists) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  typedef typename AC::cell cell;
  __shared__ int scan_sh[BS];
  __shared__ Event evq[EVQ];
  __shared__ unsigned int evq_n;
  __shared__ int wsum_sh[BS / 64];
  __shared__ unsigned int listed_sh;
  // layout: tally[T_N] | prefix[G+1] | eh[nmax+2] (P) | acc[nmax+1] (cell)
  PushShared<P, AC> sh;
  sh.evq = evq;
  sh.evq_n = &evq_n;
  sh.wsum = wsum_sh;
  sh.listed = &listed_sh;
  sh.masks = masks;
  sh.tally = (unsigned int *)lds_raw;
  sh.prefix = (int *)(lds_raw + 64);
  const size_t off = 64 + (((size_t)(G + 1) * 4 + 15) / 16) * 16;
  sh.eh = (P *)(lds_raw + off);
  sh.acc = (cell *)(lds_raw + off + ((((size_t)(nmax + 2) * sizeof(P)) + 15) / 16) * 16);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int sel = (int)(*p.epoch & 1);
  // (set before the first segment's staging barrier, read after the last flush)
  if (tid == 0) listed_sh = 0u;

  // tiles per gap and their prefix (each workgroup builds its own copy in LDS;
  // one gap needs no scan)
  int total1 = 0;
  if (G == 1) {
    int te, ti;
    gap_tiles(p.gs[0], p.gs[0].beam_now, tile, te, ti);
    total1 = te + ti;
  } else {
    const int per = (G + BS - 1) / BS;
    int mine = 0;
    for (int q = 0; q < per; ++q) {
      const int g = tid * per + q;
      if (g < G) {
        int te, ti;
        gap_tiles(p.gs[g], p.gs[g].beam_now, tile, te, ti);
        mine += te + ti;
      }
    }
    int tot_tiles;
    int run = block_exclusive_scan_i(mine, scan_sh, &tot_tiles);
    for (int q = 0; q < per; ++q) {
      const int g = tid * per + q;
      if (g < G) {
        sh.prefix[g] = run;
        int te, ti;
        gap_tiles(p.gs[g], p.gs[g].beam_now, tile, te, ti);
        run += te + ti;
      }
    }
    if (tid == 0) sh.prefix[G] = tot_tiles;
    __syncthreads();
  }

  auto prefix = [&](int i) { return G == 1 ? (i == 0 ? 0 : total1) : sh.prefix[i]; };

  const int total = prefix(G);
  const int nwg = (int)gridDim.x;
  int og = -1, os = 0;  // the open segment (gap, species), none yet
  if (rr) {
    // round robin: workgroup w takes the tiles w, w + nwg, w + 2 nwg, ...  At
    // any moment the workgroups then stream neighbouring tiles, one window of
    // memory, rather than nwg regions far apart.  Its tiles in one region are
    // one strided piece; t visits the workgroup's first tile of each region
    // it has tiles in (that tile's local index is below nwg)
    int g = 0;
    int t = (int)blockIdx.x;
    while (t < total) {
      while (prefix(g + 1) <= t) ++g;
      int te, ti;
      gap_tiles(p.gs[g], p.gs[g].beam_now, tile, te, ti);
      const int tg = prefix(g);
      const int s = t - tg < te ? 0 : 1;
      const int T0 = s ? tg + te : tg, T1 = s ? tg + te + ti : tg + te;
      push_piece<P, AC, BS, PPT, NT>(p, sh, tile, sel, g, s, t - T0, T1 - T0, nwg, og, os);
      t += ((T1 - t + nwg - 1) / nwg) * nwg;  // the first of its tiles past the region
    }
    const unsigned int ticket = lists ? push_ticket<P, AC>(p, sh, os) : 0u;
    if (og >= 0) close_seg<P, AC>(p, sh, sel, og, os);
    if (lists) push_tail_emit<P, AC>(p, sh, G, sel, ticket);
    return;
  }
  // the workgroup's contiguous run of tiles; with stealing on, the last R of
  // every run go to the pool instead (runs differ by at most one tile, so each
  // holds at least 8 R)
  const int R = p.steal != nullptr && steal > 0 ? (total / nwg) / steal : 0;
  const int t0 = (int)(((long long)blockIdx.x * total) / nwg);
  const int t1 = (int)(((long long)(blockIdx.x + 1) * total) / nwg) - R;
  {
    int g = 0, t = t0;
    while (t < t1) {
      while (prefix(g + 1) <= t) ++g;
      const int e = min(t1, prefix(g + 1));
      push_tiles<P, AC, BS, PPT, NT>(p, sh, tile, sel, g, prefix(g), t, e, og, os);
      t = e;
    }
  }
  if (R > 0) {
    // pool tile q is tile k = q / nwg of run w = q % nwg's reserved end: the
    // first reserved tile of every run goes out first
    // (the next index is taken while a tile is pushed: the counter is one
    // address for the whole device, and its atomics return slowly)
    __shared__ int s_q;
    const int npool = R * nwg;
    unsigned int qn = 0u;
    if (tid == 0) qn = atomicAdd(p.steal, 1u);
    for (;;) {
      __syncthreads();
      if (tid == 0) s_q = (int)qn;
      __syncthreads();
      // (the same for every thread: made a scalar, as the tile arithmetic is)
      const int q = __builtin_amdgcn_readfirstlane(s_q);
      if (q >= npool) break;
      if (tid == 0) qn = atomicAdd(p.steal, 1u);
      const int w = q % nwg, k = q / nwg;
      const int tt = (int)(((long long)(w + 1) * total) / nwg) - R + k;
      // the gap holding tile tt (binary search over the tile prefix)
      int g = 0;
      if (G > 1) {
        int lo = 0, hi = G - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (prefix(mid) <= tt)
            lo = mid;
          else
            hi = mid - 1;
        }
        g = lo;
      }
      push_tiles<P, AC, BS, PPT, NT>(p, sh, tile, sel, g, prefix(g), tt, tt + 1, og, os);
    }
  }
  const unsigned int ticket = lists ? push_ticket<P, AC>(p, sh, os) : 0u;
  if (og >= 0) close_seg<P, AC>(p, sh, sel, og, os);
  if (lists) push_tail_emit<P, AC>(p, sh, G, sel, ticket);
}

template <class P, class AC, int BS, int PPT, bool NT>
static hipError_t push_t(const DevPtrs &p, int G, const LaunchCfg &lc, hipStream_t s, KTime t) {
  const size_t lds = push_lds_bytes(lc.nmax, lc.fp64, G, sizeof(typename AC::cell) == 8);
  // opt in to more than 64 KiB of dynamic LDS (gfx950 has 160 KiB per CU)
  static size_t attr_set = 65536;
  if (lds > attr_set) {
    hipError_t e = hipFuncSetAttribute((const void *)k_push<P, AC, BS, PPT, NT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_set = lds;
  }
  return launch_k(k_push<P, AC, BS, PPT, NT>, dim3(lc.grid), dim3(BS), lds, s, t.a, t.b, p, G, lc.tile,
                  lc.nmax, lc.steal, (lc.stream & STREAM_RR) ? 1 : 0, lc.masks, lc.lists);
}

template <class P, class AC, int PPT, bool NT>
static hipError_t push_bs(const DevPtrs &p, int G, const LaunchCfg &lc, hipStream_t s, KTime t) {
  switch (lc.block) {
    case 256: return push_t<P, AC, 256, PPT, NT>(p, G, lc, s, t);
    case 512: return push_t<P, AC, 512, PPT, NT>(p, G, lc, s, t);
    case 768: return push_t<P, AC, 768, PPT, NT>(p, G, lc, s, t);
    default: return push_t<P, AC, 1024, PPT, NT>(p, G, lc, s, t);
  }
}

template <class P, class AC, bool NT>
static hipError_t push_b(const DevPtrs &p, int G, const LaunchCfg &lc, hipStream_t s, KTime t) {
  if (lc.ppt >= 2 * Vec<P>::n) return push_bs<P, AC, 2 * Vec<P>::n, NT>(p, G, lc, s, t);
  return push_bs<P, AC, Vec<P>::n, NT>(p, G, lc, s, t);
}
#ifdef GS_PUSH_PART
// one set of the push kernel's instantiations: particle precision, deposit
// cells, stream kind
#if GS_PUSH_PART == 0
hipError_t launch_push_f64(const DevPtrs &p, int G, const LaunchCfg &lc, hipStream_t s, KTime t) {
  return push_b<double, Wide64, false>(p, G, lc, s, t);
}
#elif GS_PUSH_PART == 1
hipError_t launch_push_f32w(const DevPtrs &p, int G, const LaunchCfg &lc, hipStream_t s, KTime t) {
  return push_b<float, Wide64, false>(p, G, lc, s, t);
}
#elif GS_PUSH_PART == 2
hipError_t launch_push_f32c(const DevPtrs &p, int G, const LaunchCfg &lc, hipStream_t s, KTime t) {
  return push_b<float, Carry32, false>(p, G, lc, s, t);
}
#elif GS_PUSH_PART == 3
hipError_t launch_push_f32w_nt(const DevPtrs &p, int G, const LaunchCfg &lc, hipStream_t s, KTime t) {
  return push_b<float, Wide64, true>(p, G, lc, s, t);
}
#elif GS_PUSH_PART == 4
hipError_t launch_push_f32c_nt(const DevPtrs &p, int G, const LaunchCfg &lc, hipStream_t s, KTime t) {
  return push_b<float, Carry32, true>(p, G, lc, s, t);
}
#else
#error "GS_PUSH_PART must be 0..4"
#endif
#else  // the other kernels and the launchers

// The regions' new slot counts after a sort (flip: its particles are in the
// other buffer now) or an in-place compaction.
__global__ void k_commit(DevPtrs p, int G, int flip) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 2 * G) {
    p.next_count[i] = p.cursor[i];
    p.cursor[i] = 0ull;
  }
  if (i == 0 && flip) *p.epoch += 1;
}

// ---------------------------------------------------------------------------
// Periodic cell sort: a counting sort of every (gap, species) region by bins of
// `bin` cells, in place of the compaction.  The live particles are written to
// the other buffer grouped by bin in increasing x, absorbed slots dropped; the
// order inside a bin is unspecified (no result depends on particle order).
// With sorted particles each push workgroup's run of tiles covers a narrow band
// of cells, so its deposit touches, and its flush adds, only that band.
//   k_sort_count    live particles per bin (hist)
//   k_sort_scan     bin offsets (bcur) and the region's live count (cursor)
//   k_sort_scatter  every particle to its bin's next slot
// then k_commit switches buffers as after a compaction.
// ---------------------------------------------------------------------------

// Adds one to cnt[bin] for every valid lane and returns each lane's rank among
// all additions to its bin so far.  Lanes of one bin share one LDS atomic (a
// sorted stream puts most of a wave in one or two bins, and separate atomics to
// one address would serialise); once the wave's leading bin holds fewer than 4
// lanes the remaining lanes add one by one.  Every lane of the wave calls it.
__device__ inline unsigned int wave_bin_rank(unsigned int *cnt, int bin, bool valid) {
  const int lane = threadIdx.x & 63;
  unsigned long long act = __ballot(valid);
  unsigned int rank = 0;
  while (act) {
    const int leader = __ffsll((long long)act) - 1;
    const int b0 = __shfl(bin, leader, 64);
    const unsigned long long m = __ballot(valid && bin == b0) & act;
    const int n = __popcll(m);
    if (n < 4) {
      if ((act >> lane) & 1ull) rank = atomicAdd(&cnt[bin], 1u);
      break;
    }
    unsigned int base = 0;
    if (lane == leader) base = atomicAdd(&cnt[b0], (unsigned int)n);
    base = __shfl(base, leader, 64);
    if ((m >> lane) & 1ull) rank = base + (unsigned int)__popcll(m & ((1ull << lane) - 1ull));
    act &= ~m;
  }
  return rank;
}

template <class P>
__device__ inline int bin_of(P x, int bin, int nb) {
  const int b = (int)x / bin;
  return b < nb - 1 ? b : nb - 1;
}

// The tile partition of k_compact over the regions' current slot counts:
// prefix[r] = first tile of region r (LDS, 2G + 1 entries).
template <int BS>
__device__ inline void region_tile_prefix(const DevPtrs &p, int G, int tile, int *prefix, int *scan_sh) {
  const int tid = threadIdx.x;
  const int R = 2 * G;
  const int per = (R + BS - 1) / BS;
  int mine = 0;
  for (int q = 0; q < per; ++q) {
    const int r = tid * per + q;
    if (r < R) mine += (int)((min((long long)p.next_count[r], p.gc[r >> 1].cap[r & 1]) + tile - 1) / tile);
  }
  int total_t;
  int run = block_exclusive_scan<int>(mine, scan_sh, &total_t);
  for (int q = 0; q < per; ++q) {
    const int r = tid * per + q;
    if (r < R) {
      prefix[r] = run;
      run += (int)((min((long long)p.next_count[r], p.gc[r >> 1].cap[r & 1]) + tile - 1) / tile);
    }
  }
  if (tid == 0) prefix[R] = total_t;
  __syncthreads();
}

// One vector of VN slots starting at slot j (below i_end, or masked past it):
// positions, velocities, ids; slots past i_end read as absorbed.
template <class P>
__device__ inline void load_vec(const P *X, const P *U, const uint32_t *I, long long j, long long i_end,
                                typename Vec<P>::type &xv, typename Vec<P>::type &uv, uint32_t *iv) {
  typedef typename Vec<P>::type PV;
  constexpr int VN = Vec<P>::n;
  typedef unsigned int IDV __attribute__((ext_vector_type(VN)));
  if (j + VN <= i_end) {
    xv = *(const PV *)(X + j);
    uv = *(const PV *)(U + j);
    const IDV t = *(const IDV *)(I + j);
#pragma unroll
    for (int k = 0; k < VN; ++k) iv[k] = t[k];
  } else {
#pragma unroll
    for (int k = 0; k < VN; ++k) {
      const bool in = j + k < i_end;
      Vec<P>::at(xv, k) = in ? X[j + k] : (P)-1;
      Vec<P>::at(uv, k) = in ? U[j + k] : (P)0;
      iv[k] = in ? I[j + k] : 0u;
    }
  }
}

template <class P, int BS>
__global__ __launch_bounds__(BS) void k_sort_count(DevPtrs p, int G, int tile, int bin, int nbmax) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  int *prefix = (int *)lds_raw;  // [2G + 1]
  unsigned int *cnt = (unsigned int *)(lds_raw + ((size_t)(2 * G + 1) * 4 + 15) / 16 * 16);  // [nbmax]
  __shared__ int scan_sh[BS];
  const int tid = threadIdx.x;
  const int src = (int)(*p.epoch & 1);
  region_tile_prefix<BS>(p, G, tile, prefix, scan_sh);
  const int total = prefix[2 * G];
  const int t0 = (int)(((long long)blockIdx.x * total) / gridDim.x);
  const int t1 = (int)(((long long)(blockIdx.x + 1) * total) / gridDim.x);
  constexpr int VN = Vec<P>::n;
  int r = 0;
  for (int t = t0; t < t1;) {
    while (prefix[r + 1] <= t) ++r;
    const int tend = min(t1, prefix[r + 1]);
    const int g = r >> 1, s = r & 1;
    const GapConst &c = p.gc[g];
    const int nb = (c.N + bin - 1) / bin;
    const long long n = min((long long)p.next_count[r], c.cap[s]);
    const long long i_beg = (long long)(t - prefix[r]) * tile;
    const long long i_end = min(n, (long long)(tend - prefix[r]) * tile);
    const P *X = (const P *)p.X[src] + c.pbase[s];
    for (int b = tid; b < nb; b += BS) cnt[b] = 0u;
    __syncthreads();
    for (long long i0 = i_beg; i0 < i_end; i0 += (long long)BS * VN) {
      const long long j = i0 + (long long)tid * VN;
      typename Vec<P>::type xv;
      if (j + VN <= i_end) {
        xv = *(const typename Vec<P>::type *)(X + j);
      } else {
#pragma unroll
        for (int k = 0; k < VN; ++k) Vec<P>::at(xv, k) = j + k < i_end ? X[j + k] : (P)-1;
      }
#pragma unroll
      for (int k = 0; k < VN; ++k) {
        const P x = Vec<P>::at(xv, k);
        const bool live = x >= (P)0;
        (void)wave_bin_rank(cnt, live ? bin_of<P>(x, bin, nb) : 0, live);
      }
    }
    __syncthreads();
    unsigned long long *h = p.hist + c.hbase[s];
    for (int b = tid; b < nb; b += BS)
      if (cnt[b]) atomicAdd(&h[b], (unsigned long long)cnt[b]);
    __syncthreads();
    t = tend;
  }
}

// one workgroup per region: exclusive scan of the bin counts into the bins'
// first slots, the region's live count for k_commit, counts cleared
constexpr int SSB = 256;
__global__ __launch_bounds__(SSB) void k_sort_scan(DevPtrs p, int bin) {
  __shared__ unsigned long long sh[SSB];
  const int r = blockIdx.x, g = r >> 1, s = r & 1;
  const GapConst &c = p.gc[g];
  const int nb = (c.N + bin - 1) / bin;
  unsigned long long *h = p.hist + c.hbase[s];
  unsigned long long *bc = p.bcur + c.hbase[s];
  unsigned long long run = 0;
  for (int b0 = 0; b0 < nb; b0 += SSB) {
    const int b = b0 + (int)threadIdx.x;
    const unsigned long long v = b < nb ? h[b] : 0ull;
    unsigned long long tot;
    const unsigned long long ex = block_exclusive_scan<unsigned long long>(v, sh, &tot);
    if (b < nb) {
      bc[b] = run + ex;
      h[b] = 0ull;
    }
    run += tot;
  }
  if (threadIdx.x == 0) p.cursor[r] = run;
}

template <class P, int BS>
__global__ __launch_bounds__(BS) void k_sort_scatter(DevPtrs p, int G, int tile, int bin, int nbmax) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  int *prefix = (int *)lds_raw;  // [2G + 1]
  const size_t o1 = ((size_t)(2 * G + 1) * 4 + 15) / 16 * 16;
  unsigned long long *base = (unsigned long long *)(lds_raw + o1);          // [nbmax]
  unsigned int *cnt = (unsigned int *)(lds_raw + o1 + (size_t)nbmax * 8);   // [nbmax]
  int *touched = (int *)(lds_raw + o1 + (size_t)nbmax * 12);                // [nbmax]
  __shared__ int scan_sh[BS];
  __shared__ int ntouched;
  const int tid = threadIdx.x;
  const int src = (int)(*p.epoch & 1), dst = src ^ 1;
  region_tile_prefix<BS>(p, G, tile, prefix, scan_sh);
  const int total = prefix[2 * G];
  const int t0 = (int)(((long long)blockIdx.x * total) / gridDim.x);
  const int t1 = (int)(((long long)(blockIdx.x + 1) * total) / gridDim.x);
  constexpr int VN = Vec<P>::n;
  int r = 0;
  for (int t = t0; t < t1;) {
    while (prefix[r + 1] <= t) ++r;
    const int tend = min(t1, prefix[r + 1]);
    const int g = r >> 1, s = r & 1;
    const GapConst &c = p.gc[g];
    const int nb = (c.N + bin - 1) / bin;
    const long long n = min((long long)p.next_count[r], c.cap[s]);
    const long long i_beg = (long long)(t - prefix[r]) * tile;
    const long long i_end = min(n, (long long)(tend - prefix[r]) * tile);
    const P *Xs = (const P *)p.X[src] + c.pbase[s];
    const P *Us = (const P *)p.U[src] + c.pbase[s];
    const uint32_t *Is = p.ID[src] + c.pbase[s];
    P *Xd = (P *)p.X[dst] + c.pbase[s];
    P *Ud = (P *)p.U[dst] + c.pbase[s];
    uint32_t *Id = p.ID[dst] + c.pbase[s];
    unsigned long long *bc = p.bcur + c.hbase[s];
    for (int b = tid; b < nb; b += BS) cnt[b] = 0u;
    if (tid == 0) ntouched = 0;
    __syncthreads();
    for (long long i0 = i_beg; i0 < i_end; i0 += (long long)BS * VN) {
      const long long j = i0 + (long long)tid * VN;
      typename Vec<P>::type xv, uv;
      uint32_t iv[VN];
      load_vec<P>(Xs, Us, Is, j, i_end, xv, uv, iv);
      int bk[VN];
      unsigned int rk[VN];
#pragma unroll
      for (int k = 0; k < VN; ++k) {
        const P x = Vec<P>::at(xv, k);
        const bool live = x >= (P)0;
        bk[k] = live ? bin_of<P>(x, bin, nb) : -1;
        rk[k] = wave_bin_rank(cnt, live ? bk[k] : 0, live);
        // the first particle of a bin in this chunk lists the bin
        if (live && rk[k] == 0u) touched[atomicAdd(&ntouched, 1)] = bk[k];
      }
      __syncthreads();
      // one slot reservation per bin the chunk touched
      const int nt = ntouched;
      for (int q = tid; q < nt; q += BS) {
        const int b = touched[q];
        base[b] = atomicAdd(&bc[b], (unsigned long long)cnt[b]);
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < VN; ++k)
        if (bk[k] >= 0) {
          const unsigned long long o = base[bk[k]] + rk[k];
          Xd[o] = Vec<P>::at(xv, k);
          Ud[o] = Vec<P>::at(uv, k);
          Id[o] = iv[k];
        }
      for (int q = tid; q < nt; q += BS) cnt[touched[q]] = 0u;
      __syncthreads();
      if (tid == 0) ntouched = 0;
      __syncthreads();
    }
    t = tend;
  }
}

// ---------------------------------------------------------------------------
// k_emit: secondary emission (Alg. 2) of the absorbed ions a push queued in the
// gaps' event lists, spread over many workgroups: chunks of EBS events, each
// with one slot reservation.  Keyed by the push's level, as in the push, so
// the electrons and their draws are the same; their wall charge goes to the
// node accumulator and their counts to the tallies the next field solve reads.
// Every event handled is counted in ev_done.  It runs when the push's last
// workgroup does not emit the lists itself (with the cell sort, whose lists
// are long).
// ---------------------------------------------------------------------------
constexpr int EBS = 256;
template <class P>
__global__ __launch_bounds__(EBS) void k_emit(DevPtrs p, int G) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  int *cpre = (int *)lds_raw;  // [G + 1]: first chunk of EBS events of gap g
  __shared__ int scan_sh[EBS];
  __shared__ int wsum[EBS / 64];
  __shared__ unsigned long long s_base;
  __shared__ unsigned int s_emit[2];
  const int tid = threadIdx.x;
  const int sel = (int)(*p.epoch & 1);
  // chunks of every gap's list, all counts loaded at once, and their prefix
  {
    const int per = (G + EBS - 1) / EBS;
    int mine = 0;
    for (int q = 0; q < per; ++q) {
      const int g = tid * per + q;
      if (g < G) mine += (int)((min((long long)p.ev_count[g], p.gc[g].evcap) + EBS - 1) / EBS);
    }
    int total;
    int run = block_exclusive_scan<int>(mine, scan_sh, &total);
    for (int q = 0; q < per; ++q) {
      const int g = tid * per + q;
      if (g < G) {
        cpre[g] = run;
        run += (int)((min((long long)p.ev_count[g], p.gc[g].evcap) + EBS - 1) / EBS);
      }
    }
    if (tid == 0) cpre[G] = total;
    __syncthreads();
  }
  const int total = cpre[G];
  // the lists' size for the host's next choice (whole chunks: an upper bound)
  if (blockIdx.x == 0 && tid == 0) *p.list_seen = (unsigned long long)total * EBS;
  int g = 0;
  for (int ch = blockIdx.x; ch < total; ch += gridDim.x) {
    // the gap holding chunk ch (chunks increase with g)
    int lo = 0, hi = G - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (cpre[mid] <= ch) lo = mid; else hi = mid - 1;
    }
    g = lo;
    const long long ne = min((long long)p.ev_count[g], p.gc[g].evcap);
    const long long r0 = (long long)(ch - cpre[g]) * EBS;
    emit_list<P>(p, g, sel, r0, (int)min((long long)EBS, ne - r0), wsum, &s_base, s_emit);
  }
}

// ---------------------------------------------------------------------------
// In-place compaction: the live particles of each (gap, species) region end in
// its first L slots, L its live count.  Only the live particles found at or past
// L move, each into one absorbed slot below L (as many of one as of the other);
// particles below L stay where they are, so a compaction reads the positions
// once and moves a few particles instead of copying the region.  Order is not
// kept (no result depends on it).  The region's slots are read in words of 64,
// their liveness kept as bit masks (live[pbase / 64 + word]), in tiles of
// CTW words; thread t of a tile takes words t, t + FW, t + 2 FW, t + 3 FW.
// Per-tile counts at tcnt[pbase / 64 + k] (tile k of the region):
//   k_fill_count  the live masks and each tile's live count
//   k_fill_plan   one workgroup per region: the tiles' exclusive live prefix, L
//   k_fill_holes  the absorbed slots below L, from the masks, listed in the
//                 region's part of the other particle buffer (spare between
//                 sorts), and H, their number
//   k_fill_rank   per word past L, the tail rank of its first live slot
//   k_fill_move   one thread per slot past L: a live one goes to the hole of
//                 its tail rank (the q-th listed hole for rank q)
// then k_commit sets each region's count to L.
// ---------------------------------------------------------------------------
constexpr int FW = 256;               // threads of the fill kernels
constexpr int WPT = 4;                // words per thread and tile
constexpr int CTW = FW * WPT;         // words per tile
constexpr long long CTS = CTW * 64ll;  // slots per tile

// bits of the slots [lo, hi) within the word starting at slot w0
__device__ inline unsigned long long slot_range_mask(long long w0, long long lo, long long hi) {
  const long long a = lo > w0 ? lo - w0 : 0, b = hi < w0 + 64 ? hi - w0 : 64;
  if (b <= a) return 0ull;
  const unsigned long long upto_b = b >= 64 ? ~0ull : ((1ull << b) - 1ull);
  const unsigned long long below_a = a <= 0 ? 0ull : ((1ull << a) - 1ull);
  return upto_b & ~below_a;
}

// The tile partition over every region's current slot count (prefix in LDS)
// and this workgroup's run of tiles.
#define FILL_TILE_RUN                                                        \
  extern __shared__ __align__(16) unsigned char lds_raw[];                   \
  int *prefix = (int *)lds_raw; /* [2G + 1] */                               \
  __shared__ int scan_sh[FW];                                                \
  __shared__ int wsum[FW / 64];                                              \
  const int tid = threadIdx.x;                                               \
  const int sel = (int)(*p.epoch & 1);                                       \
  region_tile_prefix<FW>(p, G, (int)CTS, prefix, scan_sh);                   \
  const int total = prefix[2 * G];                                           \
  const int t0 = (int)(((long long)blockIdx.x * total) / gridDim.x);         \
  const int t1 = (int)(((long long)(blockIdx.x + 1) * total) / gridDim.x);

// masks: the push before wrote the masks of the words below each region's
// count (its pushed range); only the other words are read from the positions
template <class P>
__global__ __launch_bounds__(FW) void k_fill_count(DevPtrs p, int G, int masks) {
  FILL_TILE_RUN
  typedef typename Vec<P>::type PV;
  constexpr int VN = Vec<P>::n;
  constexpr int NV = 64 / VN;  // vectors per word
  int r = 0;
  for (int t = t0; t < t1; ++t) {
    while (prefix[r + 1] <= t) ++r;
    const int s = r & 1, k = t - prefix[r];
    const GapConst &c = p.gc[r >> 1];
    const long long n = min((long long)p.next_count[r], c.cap[s]);
    const long long pushed = masks ? min((long long)p.gs[r >> 1].count[s], n) : 0;
    const long long i_beg = (long long)k * CTS, i_end = min(n, i_beg + CTS);
    const P *X = (const P *)p.X[sel] + c.pbase[s];
    unsigned long long *lm = p.live + c.pbase[s] / 64;
    int cnt = 0;
    for (int q = 0; q < WPT; ++q) {
      const long long w0 = i_beg + ((long long)q * FW + tid) * 64;
      if (w0 >= i_end) continue;
      if (w0 + 64 <= pushed) {
        cnt += __popcll(lm[w0 / 64]);
        continue;
      }
      // the word's loads all in flight before any is used
      PV xv[NV];
      if (w0 + 64 <= i_end) {
#pragma unroll
        for (int v = 0; v < NV; ++v) xv[v] = *(const PV *)(X + w0 + v * VN);
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
          for (int e = 0; e < VN; ++e) {
            const long long j = w0 + v * VN + e;
            Vec<P>::at(xv[v], e) = j < i_end ? X[j] : (P)-1;
          }
      }
      unsigned long long m = 0ull;
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int e = 0; e < VN; ++e) m |= (unsigned long long)(Vec<P>::at(xv[v], e) >= (P)0) << (v * VN + e);
      lm[w0 / 64] = m;
      cnt += __popcll(m);
    }
    int tot;
    (void)block_exclusive_scan_i(cnt, wsum, &tot);
    if (tid == 0) p.tcnt[c.pbase[s] / 64 + k] = tot;
  }
}

constexpr int FPB = 256;
__global__ __launch_bounds__(FPB) void k_fill_plan(DevPtrs p) {
  __shared__ int wsum[FPB / 64];
  const int r = blockIdx.x, s = r & 1;
  const GapConst &c = p.gc[r >> 1];
  const long long n = min((long long)p.next_count[r], c.cap[s]);
  const int ntiles = (int)((n + CTS - 1) / CTS);
  int *tc = p.tcnt + c.pbase[s] / 64;
  long long run = 0;
  for (int k0 = 0; k0 < ntiles; k0 += FPB) {
    const int k = k0 + (int)threadIdx.x;
    const int v = k < ntiles ? tc[k] : 0;
    int tot;
    const int ex = block_exclusive_scan_i(v, wsum, &tot);
    if (k < ntiles) tc[k] = (int)(run + ex);
    run += tot;
  }
  if (threadIdx.x == 0) {
    p.cursor[r] = (unsigned long long)run;
    p.fill_h[r] = 0ull;
  }
}

// live particles before tile k: the tile's exclusive prefix; in the tile: the
// next tile's prefix (or L after the last tile) minus it
template <class P>
__global__ __launch_bounds__(FW) void k_fill_holes(DevPtrs p, int G) {
  FILL_TILE_RUN
  int r = 0;
  for (int t = t0; t < t1; ++t) {
    while (prefix[r + 1] <= t) ++r;
    const int s = r & 1, k = t - prefix[r];
    const GapConst &c = p.gc[r >> 1];
    const long long n = min((long long)p.next_count[r], c.cap[s]);
    const long long L = (long long)p.cursor[r];
    const long long i_beg = (long long)k * CTS, i_end = min(n, i_beg + CTS);
    if (i_beg >= L) continue;
    const int *tc = p.tcnt + c.pbase[s] / 64;
    const long long live_before = tc[k];
    const long long live_tile = (k + 1 < prefix[r + 1] - prefix[r] ? (long long)tc[k + 1] : L) - live_before;
    const long long hi = min(i_end, L);
    long long holes = i_beg - live_before;  // absorbed slots before the tile (all below L)
    if (live_tile < i_end - i_beg) {
      const unsigned long long *lm = p.live + c.pbase[s] / 64;
      uint32_t *hl = (uint32_t *)p.X[sel ^ 1] + c.pbase[s];
      unsigned long long dead[WPT];
      int nd = 0;
#pragma unroll
      for (int q = 0; q < WPT; ++q) {
        const long long w0 = i_beg + ((long long)q * FW + tid) * 64;
        const unsigned long long rng = w0 < hi ? slot_range_mask(w0, i_beg, hi) : 0ull;
        dead[q] = rng ? ~lm[w0 / 64] & rng : 0ull;
        nd += __popcll(dead[q]);
      }
      int tot;
      const int ex = block_exclusive_scan_i(nd, wsum, &tot);
      long long o = holes + ex;
#pragma unroll
      for (int q = 0; q < WPT; ++q) {
        const long long w0 = i_beg + ((long long)q * FW + tid) * 64;
        unsigned long long d = dead[q];
        while (d) {
          const int b = __ffsll((long long)d) - 1;
          d &= d - 1ull;
          hl[o++] = (uint32_t)(w0 + b);
        }
      }
      holes += tot;
    }
    // the tile holding slot L - 1 knows how many holes lie below L
    if (tid == 0 && i_beg < L && L <= i_end) p.fill_h[r] = (unsigned long long)holes;
  }
}

// the tail rank of each word's first live slot at or past L (tiles past L)
template <class P>
__global__ __launch_bounds__(FW) void k_fill_rank(DevPtrs p, int G) {
  FILL_TILE_RUN
  (void)sel;
  int r = 0;
  for (int t = t0; t < t1; ++t) {
    while (prefix[r + 1] <= t) ++r;
    const int s = r & 1, k = t - prefix[r];
    const GapConst &c = p.gc[r >> 1];
    const long long n = min((long long)p.next_count[r], c.cap[s]);
    const long long L = (long long)p.cursor[r];
    const long long i_beg = (long long)k * CTS, i_end = min(n, i_beg + CTS);
    if (i_end <= L) continue;
    const long long H = (long long)p.fill_h[r];
    // tail rank of the tile's first slot at or past L: live ones in [L, lo)
    const long long lo = max(i_beg, L);
    const long long rank = i_beg >= L ? (long long)p.tcnt[c.pbase[s] / 64 + k] - (L - H) : 0;
    const unsigned long long *lm = p.live + c.pbase[s] / 64;
    int *wr = p.wrank + c.pbase[s] / 64;
    int cnt[WPT];
    int nl = 0;
#pragma unroll
    for (int q = 0; q < WPT; ++q) {
      const long long w0 = i_beg + ((long long)q * FW + tid) * 64;
      const unsigned long long rng = w0 < i_end ? slot_range_mask(w0, lo, i_end) : 0ull;
      cnt[q] = rng ? __popcll(lm[w0 / 64] & rng) : 0;
      nl += cnt[q];
    }
    int tot;
    const int ex = block_exclusive_scan_i(nl, wsum, &tot);
    long long q0 = rank + ex;
#pragma unroll
    for (int q = 0; q < WPT; ++q) {
      const long long w0 = i_beg + ((long long)q * FW + tid) * 64;
      if (w0 < i_end && w0 + 64 > lo) wr[w0 / 64] = (int)q0;
      q0 += cnt[q];
    }
  }
}

// every live slot at or past L, one thread each, to the hole of its tail rank
// (the word's rank plus the live slots before it in the word); grid-stride over
// the tails of all regions, whose lengths n - L are prefixed in LDS
template <class P>
__global__ __launch_bounds__(FW) void k_fill_move(DevPtrs p, int G) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  long long *tpre = (long long *)lds_raw;  // [2G + 1]: first flat index of region r's tail
  __shared__ long long scan_sh[FW];
  const int tid = threadIdx.x;
  const int sel = (int)(*p.epoch & 1);
  const int R = 2 * G;
  {
    const int per = (R + FW - 1) / FW;
    long long mine = 0;
    for (int q = 0; q < per; ++q) {
      const int r = tid * per + q;
      if (r < R) mine += min((long long)p.next_count[r], p.gc[r >> 1].cap[r & 1]) - (long long)p.cursor[r];
    }
    long long tot;
    long long run = block_exclusive_scan<long long>(mine, scan_sh, &tot);
    for (int q = 0; q < per; ++q) {
      const int r = tid * per + q;
      if (r < R) {
        tpre[r] = run;
        run += min((long long)p.next_count[r], p.gc[r >> 1].cap[r & 1]) - (long long)p.cursor[r];
      }
    }
    if (tid == 0) tpre[R] = tot;
    __syncthreads();
  }
  const long long total = tpre[R];
  int r = 0;
  for (long long f = (long long)blockIdx.x * FW + tid; f < total; f += (long long)gridDim.x * FW) {
    while (tpre[r + 1] <= f) ++r;
    const int s = r & 1;
    const GapConst &c = p.gc[r >> 1];
    const long long L = (long long)p.cursor[r];
    const long long j = L + (f - tpre[r]);
    const unsigned long long m = p.live[c.pbase[s] / 64 + j / 64];
    const int b = (int)(j & 63);
    if (!((m >> b) & 1ull)) continue;
    // live slots in this word before j and at or past L
    const long long w0 = j - b;
    const unsigned long long before = (b ? ((1ull << b) - 1ull) : 0ull) & slot_range_mask(w0, L, j + 1);
    const long long q = (long long)p.wrank[c.pbase[s] / 64 + j / 64] + __popcll(m & before);
    const uint32_t *hl = (const uint32_t *)p.X[sel ^ 1] + c.pbase[s];
    const long long dst = (long long)hl[q];
    P *X = (P *)p.X[sel] + c.pbase[s];
    P *U = (P *)p.U[sel] + c.pbase[s];
    uint32_t *I = p.ID[sel] + c.pbase[s];
    X[dst] = X[j];
    U[dst] = U[j];
    I[dst] = I[j];
  }
}

#undef FILL_TILE_RUN

// ---------------------------------------------------------------------------
// injection of caller particles (SI) into one gap
// ---------------------------------------------------------------------------
template <class P>
__global__ void k_inject(DevPtrs p, int gap, int species, long long n, const double *x,
                         const double *v, long long id0) {
  const GapConst &c = p.gc[gap];
  const int sel = (int)(*p.epoch & 1);
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i < n;
  // one slot reservation per wave
  const unsigned long long mask = __ballot(valid);
  if (mask == 0ull) return;
  const int lane = threadIdx.x & 63;
  const int first = __ffsll((long long)mask) - 1;
  unsigned long long base = 0;
  if (lane == first)
    base = atomicAdd(&p.next_count[gap * 2 + species], (unsigned long long)__popcll(mask));
  base = __shfl(base, first, 64);
  if (!valid) return;
  if (i == 0) {
    atomicAdd((unsigned long long *)&p.gs[gap].live[species], (unsigned long long)n);
    atomicAdd((unsigned long long *)&p.gs[gap].next_id, (unsigned long long)n);
  }
  const unsigned long long slot = base + (unsigned long long)__popcll(mask & ((1ull << lane) - 1ull));
  const double xs = x[i];
  if (!(xs >= 0.0 && xs <= c.d)) {
    atomicOr(&p.err[0], ERR_BADINJECT);
    return;
  }
  if (slot >= (unsigned long long)c.cap[species]) {
    atomicOr(&p.err[0], ERR_CAPACITY);
    atomicCAS(&p.err[1], 0xFFFFFFFFu, (unsigned int)gap);
    return;
  }
  const P xi = (P)(xs / c.dx);
  const P u = (P)((v[i] * c.dt) / c.dx);
  const size_t k = (size_t)c.pbase[species] + slot;
  ((P *)p.X[sel])[k] = xi;
  ((P *)p.U[sel])[k] = u;
  p.ID[sel][k] = (uint32_t)(id0 + i);
  int j = (int)xi;
  if (j > c.N - 1) j = c.N - 1;
  const P f = xi - (P)j;
  const long long w1 = Prec<P>::wq(f);
  const long long w0 = Prec<P>::W - w1;
  unsigned long long *gacc = p.acc + c.nbase;
  atomicAdd(&gacc[j], (unsigned long long)(c.Z[species] * w0));
  atomicAdd(&gacc[j + 1], (unsigned long long)(c.Z[species] * w1));
}

// phi_i = dx sum_{k >= i} E_{k+1/2}, phi_N = 0 (one gap, one workgroup)
constexpr int PBS = 256;
__global__ __launch_bounds__(PBS) void k_phi(DevPtrs p, int gap) {
  const GapConst &c = p.gc[gap];
  __shared__ double sh[PBS];
  const int N = c.N, tid = threadIdx.x;
  const double *E = p.E64 + c.nbase;
  double *phi = p.phi64 + c.nbase;
  const int chunk = (N + PBS - 1) / PBS;
  // thread t owns reversed positions k0..k1-1, i.e. nodes N-1-k counted from the ground
  const int k0 = tid * chunk, k1 = min(k0 + chunk, N);
  double loc = 0.0;
  for (int k = k0; k < k1; ++k) loc += c.dx * E[N - 1 - k];
  double tot;
  double run = block_exclusive_scan<double>(loc, sh, &tot);
  for (int k = k0; k < k1; ++k) {
    run += c.dx * E[N - 1 - k];
    phi[N - 1 - k] = run;
  }
  if (tid == 0) phi[N] = 0.0;
}

// ---------------------------------------------------------------------------
// time-step check of one gap (App. time segment selection): largest |u| of the
// live particles of each species and the live electrons in each cell
// ---------------------------------------------------------------------------
constexpr int DBS = 256;
template <class P>
__device__ inline unsigned long long nonneg_bits(P v);
template <>
__device__ inline unsigned long long nonneg_bits<float>(float v) {
  return (unsigned long long)__float_as_uint(v);
}
template <>
__device__ inline unsigned long long nonneg_bits<double>(double v) {
  return (unsigned long long)__double_as_longlong(v);
}

template <class P>
__global__ __launch_bounds__(DBS) void k_dt_scan(DevPtrs p, int gap, unsigned long long *umax,
                                                 unsigned int *cells) {
  extern __shared__ unsigned int hist[];  // [N]
  __shared__ P red[DBS / 64][2];
  const GapConst &c = p.gc[gap];
  const int N = c.N;
  const int sel = (int)(*p.epoch & 1);
  for (int k = threadIdx.x; k < N; k += DBS) hist[k] = 0u;
  __syncthreads();
  const P *X = (const P *)p.X[sel], *U = (const P *)p.U[sel];
  P m[2] = {(P)0, (P)0};
  const long long stride = (long long)gridDim.x * DBS;
  for (int s = 0; s < 2; ++s) {
    const long long n = min((long long)p.next_count[gap * 2 + s], (long long)c.cap[s]);
    const size_t b = (size_t)c.pbase[s];
    for (long long i = (long long)blockIdx.x * DBS + threadIdx.x; i < n; i += stride) {
      const P x = X[b + i];
      if (!(x >= (P)0)) continue;  // absorbed slot
      m[s] = fmax(m[s], fabs(U[b + i]));
      if (s == 0) atomicAdd(&hist[min((int)x, N - 1)], 1u);
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int s = 0; s < 2; ++s) {
    P v = m[s];
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    if (lane == 0) red[wave][s] = v;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    P v = red[0][threadIdx.x];
    for (int w = 1; w < DBS / 64; ++w) v = fmax(v, red[w][threadIdx.x]);
    atomicMax(&umax[threadIdx.x], nonneg_bits<P>(v));
  }
  for (int k = threadIdx.x; k < N; k += DBS)
    if (hist[k]) atomicAdd(&cells[k], hist[k]);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
size_t push_lds_bytes(int nmax, int fp64, int G, int wide) {
  const size_t ps = fp64 ? 8 : 4, cs = (fp64 || wide) ? 8 : 4;
  size_t off = 64 + (((size_t)(G + 1) * 4 + 15) / 16) * 16;
  off += (((size_t)(nmax + 2) * ps + 15) / 16) * 16;
  off += (size_t)(nmax + 1) * cs;
  return off;
}

hipError_t launch_field(const DevPtrs &p, int G, int mode, int guess, double tol, int maxit,
                        int fp64, int nmax, hipStream_t s, KTime t) {
  if (nmax <= FIELD1_NMAX) {
    // S_k of every cell, padded by one double per chunk of the prefix sums
    // (index k + k / ch < N + FBS)
    const size_t lds = ((size_t)nmax + (size_t)FBS + 1) * 8;
    static size_t attr_set = 32768;
    if (lds > attr_set) {
      hipError_t e = hipFuncSetAttribute((const void *)k_field1, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)lds);
      if (e != hipSuccess) return e;
      attr_set = lds;
    }
    return launch_k(k_field1, dim3(G), dim3(FBS), lds, s, t.a, t.b, p, mode, guess, tol, maxit, fp64);
  }
  // events (when timing) on the first and the last of the three launches
  const dim3 chunks((unsigned)(nmax / FCN + 1), (unsigned)G);
  hipError_t e = launch_k(k_fdens, chunks, dim3(FDB), 0, s, t.a, nullptr, p, fp64);
  if (e != hipSuccess) return e;
  e = launch_k(k_field, dim3(G), dim3(FBS), 0, s, nullptr, nullptr, p, mode, guess, tol, maxit, fp64);
  if (e != hipSuccess) return e;
  return launch_k(k_ftable, chunks, dim3(FDB), 0, s, nullptr, t.b, p, fp64);
}

hipError_t launch_push(const DevPtrs &p, int G, const LaunchCfg &lc, hipStream_t s, KTime t) {
  // (the non-temporal stream is for binary32 particles)
  const bool nt = (lc.stream & STREAM_NT) != 0;
  if (lc.fp64) return launch_push_f64(p, G, lc, s, t);
  if (lc.wide) return nt ? launch_push_f32w_nt(p, G, lc, s, t) : launch_push_f32w(p, G, lc, s, t);
  return nt ? launch_push_f32c_nt(p, G, lc, s, t) : launch_push_f32c(p, G, lc, s, t);
}

template <class P>
static hipError_t fill_t(const DevPtrs &p, int G, const LaunchCfg &lc, hipStream_t s, KTime t) {
  const int grid = lc.compact_grid > 0 ? lc.compact_grid : 1024;
  const size_t lds = ((size_t)(2 * G + 1) * 4 + 15) / 16 * 16;
  const size_t lds2 = (size_t)(2 * G + 1) * 8;  // the move's 64-bit tail prefix
  static size_t attr_set = 65536, attr_set2 = 65536;
  if (lds > attr_set) {
    for (const void *k : {(const void *)k_fill_count<P>, (const void *)k_fill_holes<P>, (const void *)k_fill_rank<P>}) {
      hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    attr_set = lds;
  }
  if (lds2 > attr_set2) {
    hipError_t e = hipFuncSetAttribute((const void *)k_fill_move<P>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds2);
    if (e != hipSuccess) return e;
    attr_set2 = lds2;
  }
  // the start event goes with the count pass, the end event with the commit
  hipError_t e = launch_k(k_fill_count<P>, dim3(grid), dim3(FW), lds, s, t.a, nullptr, p, G, lc.masks);
  if (e == hipSuccess) e = launch_k(k_fill_plan, dim3(2 * G), dim3(FPB), 0, s, nullptr, nullptr, p);
  if (e == hipSuccess) e = launch_k(k_fill_holes<P>, dim3(grid), dim3(FW), lds, s, nullptr, nullptr, p, G);
  if (e == hipSuccess) e = launch_k(k_fill_rank<P>, dim3(grid), dim3(FW), lds, s, nullptr, nullptr, p, G);
  if (e == hipSuccess) e = launch_k(k_fill_move<P>, dim3(grid), dim3(FW), lds2, s, nullptr, nullptr, p, G);
  if (e != hipSuccess) return e;
  return launch_k(k_commit, dim3((2 * G + 255) / 256), dim3(256), 0, s, nullptr, t.b, p, G, 0);
}

hipError_t launch_compact(const DevPtrs &p, int G, const LaunchCfg &lc, hipStream_t s, KTime t) {
  return lc.fp64 ? fill_t<double>(p, G, lc, s, t) : fill_t<float>(p, G, lc, s, t);
}

size_t sort_lds_bytes(int G, int nmax, int bin) {
  const int nbmax = (nmax + bin - 1) / bin;
  return ((size_t)(2 * G + 1) * 4 + 15) / 16 * 16 + (size_t)nbmax * 16;
}

template <class P>
static hipError_t sort_t(const DevPtrs &p, int G, const LaunchCfg &lc, hipStream_t s, KTime t) {
  const int bin = lc.sort_bin;
  const int nbmax = (lc.nmax + bin - 1) / bin;
  const size_t lds = sort_lds_bytes(G, lc.nmax, bin);
  static size_t attr_set = 65536;
  if (lds > attr_set) {
    hipError_t e = hipFuncSetAttribute((const void *)k_sort_count<P, 256>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void *)k_sort_scatter<P, 256>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    if (e != hipSuccess) return e;
    attr_set = lds;
  }
  const int grid = lc.compact_grid > 0 ? lc.compact_grid : 1024;
  // the start event goes with the count pass, the end event with the commit
  hipError_t e = launch_k(k_sort_count<P, 256>, dim3(grid), dim3(256), lds, s, t.a, nullptr, p, G, lc.tile, bin,
                          nbmax);
  if (e != hipSuccess) return e;
  e = launch_k(k_sort_scan, dim3(2 * G), dim3(SSB), 0, s, nullptr, nullptr, p, bin);
  if (e != hipSuccess) return e;
  e = launch_k(k_sort_scatter<P, 256>, dim3(grid), dim3(256), lds, s, nullptr, nullptr, p, G, lc.tile, bin, nbmax);
  if (e != hipSuccess) return e;
  return launch_k(k_commit, dim3((2 * G + 255) / 256), dim3(256), 0, s, nullptr, t.b, p, G, 1);
}

hipError_t launch_sort(const DevPtrs &p, int G, const LaunchCfg &lc, hipStream_t s, KTime t) {
  if (lc.sort_bin < SORT_BIN_MIN) return hipErrorInvalidValue;
  return lc.fp64 ? sort_t<double>(p, G, lc, s, t) : sort_t<float>(p, G, lc, s, t);
}

hipError_t launch_emit(const DevPtrs &p, int G, int fp64, int grid, hipStream_t s, KTime t) {
  const size_t lds = ((size_t)(G + 1) * 4 + 15) / 16 * 16;
  static size_t attr_set[2] = {65536, 65536};
  if (lds > attr_set[fp64 ? 1 : 0]) {
    const void *k = fp64 ? (const void *)k_emit<double> : (const void *)k_emit<float>;
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_set[fp64 ? 1 : 0] = lds;
  }
  return fp64 ? launch_k(k_emit<double>, dim3(grid), dim3(EBS), lds, s, t.a, t.b, p, G)
              : launch_k(k_emit<float>, dim3(grid), dim3(EBS), lds, s, t.a, t.b, p, G);
}

hipError_t launch_inject(const DevPtrs &p, int gap, int species, long long n, const double *x,
                         const double *v, long long id0, int fp64, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int bs = 256;
  const unsigned int grid = (unsigned int)((n + bs - 1) / bs);
  if (fp64)
    hipLaunchKernelGGL(k_inject<double>, dim3(grid), dim3(bs), 0, s, p, gap, species, n, x, v, id0);
  else
    hipLaunchKernelGGL(k_inject<float>, dim3(grid), dim3(bs), 0, s, p, gap, species, n, x, v, id0);
  return hipGetLastError();
}

hipError_t launch_dt_scan(const DevPtrs &p, int gap, int N, int fp64, unsigned long long *umax,
                          unsigned int *cells, hipStream_t s) {
  const size_t lds = (size_t)N * 4;
  static bool attr[2] = {false, false};
  const void *k = fp64 ? (const void *)k_dt_scan<double> : (const void *)k_dt_scan<float>;
  if (!attr[fp64]) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    if (e != hipSuccess) return e;
    attr[fp64] = true;
  }
  if (lds > 65536) return hipErrorInvalidValue;
  if (fp64)
    hipLaunchKernelGGL(k_dt_scan<double>, dim3(512), dim3(DBS), lds, s, p, gap, umax, cells);
  else
    hipLaunchKernelGGL(k_dt_scan<float>, dim3(512), dim3(DBS), lds, s, p, gap, umax, cells);
  return hipGetLastError();
}

hipError_t launch_phi(const DevPtrs &p, int gap, hipStream_t s) {
  hipLaunchKernelGGL(k_phi, dim3(1), dim3(PBS), 0, s, p, gap);
  return hipGetLastError();
}
#endif  // GS_PUSH_PART

}  // namespace gs
