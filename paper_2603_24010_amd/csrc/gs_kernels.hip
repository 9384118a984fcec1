// Device side of the circuit-coupled 1D ES-PIC step for gfx950.
//
// Per step two kernels run on the context's stream:
//   k_field  one workgroup per gap: charge accumulator -> rho, prefix scans for
//            the half-grid field, the circuit/surface-charge update (strict or
//            weak), the binary32/64 field table the push gathers from.
//   k_push   persistent workgroups over tiles of every gap's particles: gather,
//            leapfrog, wall test, secondary emission, beam injection and the
//            charge deposit, privatised in LDS per workgroup.
// Every few steps k_compact reclaims the slots of absorbed particles.
//
// Compiled with -ffp-contract=off: the binary32 particle arithmetic is a fixed
// sequence of IEEE operations (no fused multiply-adds).
#include <hip/hip_runtime.h>

#include "gs_internal.h"

namespace gs {

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11)
// ---------------------------------------------------------------------------
__device__ inline void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
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

__device__ inline int poisson_inverse(double lam, double u, int kmax) {
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
// helpers
// ---------------------------------------------------------------------------
// block-wide exclusive scan of one double per thread (blockDim.x <= 1024)
__device__ inline double block_exclusive_scan(double v, double *sh, double *total) {
  const int tid = threadIdx.x, nt = blockDim.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < nt; off <<= 1) {
    double a = (tid >= off) ? sh[tid - off] : 0.0;
    __syncthreads();
    sh[tid] += a;
    __syncthreads();
  }
  double incl = sh[tid];
  *total = sh[nt - 1];
  __syncthreads();
  return incl - v;
}

// block-wide exclusive scan of one int per thread
__device__ inline int block_exclusive_scan_int(int v, int *sh, int *total) {
  const int tid = threadIdx.x, nt = blockDim.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < nt; off <<= 1) {
    int a = (tid >= off) ? sh[tid - off] : 0;
    __syncthreads();
    sh[tid] += a;
    __syncthreads();
  }
  int incl = sh[tid];
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

__device__ inline double node_rho(const GapConst &c, const unsigned long long *acc, int j, int fp64) {
  const double scale = fp64 ? 5.684341886080801486968994140625e-14 /* 2^-44 */
                            : 5.9604644775390625e-08 /* 2^-24 */;
  double r = c.s0 * ((double)(long long)acc[j] * scale) / c.dx;
  if (j == 0 || j == c.N) r *= 2.0;
  return r;
}

// ---------------------------------------------------------------------------
// k_field: level n of one gap per workgroup
// ---------------------------------------------------------------------------
constexpr int FBS = 256;

__global__ __launch_bounds__(FBS) void k_field(DevPtrs p, int mode, int guess, double tol,
                                               int maxit, int fp64) {
  const int g = blockIdx.x, tid = threadIdx.x;
  const GapConst &c = p.gc[g];
  GapState &st = p.gs[g];
  const int N = c.N;
  const int M = c.M;
  const double dx = c.dx, eps0 = c.eps0, A = c.A;
  unsigned long long *acc = p.acc + c.nbase;
  double *rho = p.rho64 + c.nbase;
  double *E = p.E64 + c.nbase;

  __shared__ double sh[FBS];
  __shared__ double s_sigma, s_P, s_rhoN;

  // 1. nodal density of level n and prefix sums S_k = dx rho_0/2 + dx sum_{1..k} rho_j
  const int chunk = (N + FBS - 1) / FBS;
  const int k0 = tid * chunk;
  const int k1 = min(k0 + chunk, N);
  double loc = 0.0;
  for (int k = k0; k < k1; ++k) {
    double r = node_rho(c, acc, k, fp64);
    rho[k] = r;
    acc[k] = 0ull;
    loc += (k == 0) ? dx * r / 2.0 : dx * r;
  }
  if (tid == FBS - 1) {
    double r = node_rho(c, acc, N, fp64);
    rho[N] = r;
    acc[N] = 0ull;
    s_rhoN = r;
  }
  double tot;
  double run = block_exclusive_scan(loc, sh, &tot);
  double sumS = 0.0;
  for (int k = k0; k < k1; ++k) {
    double r = rho[k];
    run += (k == 0) ? dx * r / 2.0 : dx * r;
    E[k] = run;  // S_k for now
    sumS += run;
  }
  double P = block_sum(sumS, sh) * dx / eps0;

  // 2. circuit, surface charge and electrode potential (scalar work)
  if (tid == 0) {
    const long long n = st.level + 1;
    const double t = (double)n * c.dt;
    unsigned long long *tl = p.tally + (size_t)g * T_N;
    // convection charge of the push that led to this level (Sec. 2.4.1)
    long long ab[4], em[2], inj, pushed;
    for (int i = 0; i < 4; ++i) ab[i] = (long long)tl[T_ABS + i];
    em[0] = (long long)tl[T_EMIT];
    em[1] = (long long)tl[T_EMIT + 1];
    inj = (long long)tl[T_INJ];
    pushed = (long long)tl[T_PUSHED];
    for (int i = 0; i < T_N; ++i) tl[i] = 0ull;
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

    const double Vs = c.src_dc + c.src_amp * sin(c.src_w * t + c.src_phase);
    double h[MAXM], q[MAXM], Dn[MAXM];
    for (int j = 0; j < M; ++j) h[j] = 15.0 * st.dq[0][j] - 7.0 * st.dq[1][j] + st.dq[2][j];
    const int gm = c.g;
    double sigma, qcirc, qstar, phi0;
    if (mode == 0) {
      // strict: D = y - z phi0, Q_gap = K - G phi0 (eq. Q4_phi_relation)
      double y[MAXM];
      for (int i = 0; i < M; ++i) {
        double a = c.sb[i] * Vs;
        for (int j = 0; j < M; ++j)
          a += c.sL[i * MAXM + j] * h[j] + c.sR[i * MAXM + j] * st.dq[0][j] -
               c.sS[i * MAXM + j] * st.qprev[j];
        y[i] = a;
      }
      const double K = st.qprev[gm] + y[gm];
      const double G = c.sz[gm] + c.c_par;
      // phi0 from eq. Poisson_BC2 closed over the interior rows:
      // phi0 = (d/eps0) sigma + P, sigma = sigma* - G phi0 / A
      const double sig_star = st.sigma_prev + (qconv + K - st.qcirc_prev) / A;
      double u_sol0 = ((c.d / eps0) * sig_star + P) / (1.0 + G * c.d / (eps0 * A));
      int iters = -1, fb = 0;
      double r0n = 0.0, rn = 0.0;
      if (guess != GS_GUESS_DIRECT) {
        // Newton on u = (V, I_0..I_{M-1}) with the constant Jacobian J
        const int nu = M + 1;
        double u[MAXM + 1], r[MAXM + 1];
        auto residual = [&](const double *uu, double *rr) {
          // BDF2 increments from the currents: I = (3 D - D1) / (2 dt)
          double rho_c[MAXM];
          for (int j = 0; j < M; ++j)
            rho_c[j] = (2.0 * c.dt * uu[1 + j] + st.dq[0][j]) / 3.0 - y[j];
          // loop equations in volts: T' D - C' + g V = T' (D - y) + g V
          for (int i = 0; i < M; ++i) {
            double a = (i == gm) ? uu[0] : 0.0;
            for (int j = 0; j < M; ++j) a += c.Tp[i * MAXM + j] * rho_c[j];
            rr[1 + i] = a / c.v_ref;
          }
          // closure: V equals the electrode potential the field gives
          const double qgap = st.qprev[gm] + (rho_c[gm] + y[gm]) - c.c_par * uu[0];
          const double sg = st.sigma_prev + (qconv + qgap - st.qcirc_prev) / A;
          rr[0] = (uu[0] - ((c.d / eps0) * sg + P)) / c.v_ref;
        };
        auto norm = [&](const double *rr) {
          double m = 0.0;
          for (int i = 0; i < nu; ++i) m = fmax(m, fabs(rr[i]));
          return m;
        };
        // plain guess: quadratic extrapolation of the last three levels
        double ue[MAXM + 1];
        for (int i = 0; i < nu; ++i) ue[i] = 3.0 * st.uh[0][i] - 3.0 * st.uh[1][i] + st.uh[2][i];
        residual(ue, r);
        double rext = norm(r);
        bool use_mlp = false;
        if (guess == GS_GUESS_MLP && p.mlp_u) {
          for (int i = 0; i < nu; ++i) u[i] = p.mlp_u[(size_t)g * (MAXM + 1) + i];
          residual(u, r);
          double rm = norm(r);
          use_mlp = (rm == rm) && (rm <= rext);
          if (!use_mlp) fb = 1;
        }
        if (!use_mlp) {
          for (int i = 0; i < nu; ++i) u[i] = ue[i];
          residual(u, r);
        }
        r0n = norm(r);
        rn = r0n;
        iters = 0;
        while (!(rn <= tol) && iters < maxit) {
          for (int i = 0; i < nu; ++i) {
            double a = 0.0;
            for (int j = 0; j < nu; ++j) a += c.Jinv[i * (MAXM + 1) + j] * r[j];
            ue[i] = u[i] - a;
          }
          for (int i = 0; i < nu; ++i) u[i] = ue[i];
          residual(u, r);
          rn = norm(r);
          iters += 1;
        }
        if (!(rn <= tol)) atomicOr(p.err, ERR_NOCONV);
        u_sol0 = u[0];
      }
      phi0 = u_sol0;
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
      }
      st.newton_r0 = r0n;
      st.newton_r = rn;
    } else {
      // weak: the circuit alone with the gap as a capacitor, then the field
      double y[MAXM];
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
    // state of level n
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
    st.sigma_prev = sigma;
    st.qcirc_prev = qcirc;
    st.level = n;
    st.t = t;
    st.phi0 = phi0;
    st.sigma = sigma;
    st.qcirc = qcirc;
    st.qcirc_star = qstar;
    st.qconv = qconv;
    // particles the coming push sweeps; beam ids of this step
    for (int s = 0; s < 2; ++s) st.count[s] = (long long)p.next_count[g * 2 + s];
    st.beam_id0 = st.next_id;
    st.next_id += c.beam_n;
    s_sigma = sigma;
    s_P = P;
  }
  __syncthreads();

  // 3. half-grid field E_{k+1/2} = (sigma + S_k) / eps0 and the gather table
  const double sigma = s_sigma;
  for (int k = k0; k < k1; ++k) E[k] = (sigma + E[k]) / eps0;
  __syncthreads();
  if (fp64) {
    double *eh = (double *)p.ehat + c.ebase;
    for (int k = k0; k < k1; ++k) eh[k + 1] = E[k];
    if (tid == 0) {
      eh[0] = sigma / eps0;
      double ed = E[N - 1] + dx * s_rhoN / (2.0 * eps0);
      eh[N + 1] = ed;
      st.e_ground = ed;
    }
  } else {
    float *eh = (float *)p.ehat + c.ebase;
    for (int k = k0; k < k1; ++k) eh[k + 1] = (float)E[k];
    if (tid == 0) {
      eh[0] = (float)(sigma / eps0);
      double ed = E[N - 1] + dx * s_rhoN / (2.0 * eps0);
      eh[N + 1] = (float)ed;
      st.e_ground = ed;
    }
  }
}

// ---------------------------------------------------------------------------
// k_push
// ---------------------------------------------------------------------------
template <class P>
struct Acc;

// binary32 particles: 2^-24 weights, unsigned 32-bit LDS cells biased by 2^31;
// a wrap of a cell is carried into the gap's 64-bit accumulator at once
template <>
struct Acc<float> {
  typedef unsigned int cell;
  static constexpr unsigned int BIAS = 0x80000000u;
  __device__ static inline void add(cell *lds, unsigned long long *gacc, int j, long long c64) {
    const int c = (int)c64;
    const unsigned int uc = (unsigned int)c;
    const unsigned int old = atomicAdd(&lds[j], uc);
    long long carry = 0;
    if (c >= 0) {
      if (old + uc < old) carry = 1;
    } else {
      if (old < (unsigned int)(-c)) carry = -1;
    }
    if (carry) atomicAdd(&gacc[j], (unsigned long long)(carry * 4294967296ll));
  }
  __device__ static inline long long flush_value(cell v) {
    return (long long)v - (long long)BIAS;
  }
  __device__ static inline cell zero() { return BIAS; }
};

// binary64 particles: 2^-44 weights, 64-bit LDS cells
template <>
struct Acc<double> {
  typedef unsigned long long cell;
  __device__ static inline void add(cell *lds, unsigned long long *, int j, long long c) {
    atomicAdd(&lds[j], (unsigned long long)c);
  }
  __device__ static inline long long flush_value(cell v) { return (long long)v; }
  __device__ static inline cell zero() { return 0ull; }
};

template <class P>
struct Prec;
template <>
struct Prec<float> {
  static constexpr float ONE_W = 16777216.0f;  // 2^24
  static constexpr long long W = 16777216ll;
  __device__ static inline long long wq(float f) { return (long long)__float2uint_rn(f * ONE_W); }
};
template <>
struct Prec<double> {
  static constexpr double ONE_W = 17592186044416.0;  // 2^44
  static constexpr long long W = 17592186044416ll;
  __device__ static inline long long wq(double f) { return __double2ll_rn(f * ONE_W); }
};

// Linear gather from the extended half-grid table eh[0..N+1]:
// eh[0] = surface field at node 0, eh[k] = E_{k-1/2}, eh[N+1] = field at node N.
template <class P>
__device__ inline P gather(const P *eh, P xi, int N) {
  const P Nf = (P)N;
  int k;
  P t;
  if (xi < (P)0.5) {
    k = 0;
    t = xi + xi;
  } else if (xi >= Nf - (P)0.5) {
    k = N;
    t = xi - (Nf - (P)0.5);
    t = t + t;
  } else {
    P h = xi - (P)0.5;
    int j = (int)h;
    t = h - (P)j;
    k = j + 1;
  }
  P a = eh[k];
  P b = eh[k + 1];
  P dlt = b - a;
  P m = t * dlt;
  return a + m;
}

template <class P>
struct PushShared {
  P *eh;
  typename Acc<P>::cell *acc;
  int *prefix;          // [G + 1]
  unsigned int *tally;  // [T_N]
};

// tiles of gap g: electrons, then ions, then beam injections
__device__ inline void gap_tiles(const GapState &st, const GapConst &c, int tile, int &te, int &ti,
                                 int &tb) {
  te = (int)((st.count[0] + tile - 1) / tile);
  ti = (int)((st.count[1] + tile - 1) / tile);
  tb = (int)((c.beam_n + tile - 1) / tile);
}

template <class P>
__device__ void flush_gap(const DevPtrs &p, const GapConst &c, int g, PushShared<P> &sh) {
  __syncthreads();
  unsigned long long *gacc = p.acc + c.nbase;
  for (int j = threadIdx.x; j <= c.N; j += blockDim.x) {
    long long v = Acc<P>::flush_value(sh.acc[j]);
    if (v != 0) atomicAdd(&gacc[j], (unsigned long long)v);
  }
  if (threadIdx.x < T_N) {
    unsigned int v = sh.tally[threadIdx.x];
    if (v) atomicAdd(&p.tally[(size_t)g * T_N + threadIdx.x], (unsigned long long)v);
  }
  __syncthreads();
}

template <class P>
__device__ void load_gap(const DevPtrs &p, const GapConst &c, PushShared<P> &sh) {
  const P *geh = (const P *)p.ehat + c.ebase;
  for (int j = threadIdx.x; j <= c.N + 1; j += blockDim.x) sh.eh[j] = geh[j];
  for (int j = threadIdx.x; j <= c.N; j += blockDim.x) sh.acc[j] = Acc<P>::zero();
  if (threadIdx.x < T_N) sh.tally[threadIdx.x] = 0u;
  __syncthreads();
}

__device__ inline unsigned long long reserve(unsigned long long *counter, unsigned int n) {
  return atomicAdd(counter, (unsigned long long)n);
}

// secondary electrons of one absorbed ion (Alg. 2); returns how many were emitted
template <class P>
__device__ int emit_electrons(const DevPtrs &p, const GapConst &c, const GapState &st, int g,
                              int sel, uint32_t ion_id, P u_ion, int wall) {
  const double v_ion = ((double)u_ion * c.dx) / c.dt;
  const double e_ion = 0.5 * c.mass[1] * v_ion * v_ion / c.ev;
  const double rr = e_ion / c.see_E0;
  double lam = c.see_amp * rr / (1.0 + rr);
  if (lam < 0.0) lam = 0.0;
  uint64_t blk[4];
  rng_block(c.seed, (uint64_t)st.level, (uint64_t)ion_id, 1, 0, blk);
  const int k = poisson_inverse(lam, unit_open(blk[0]), c.see_max);
  if (k == 0) return 0;
  unsigned long long slot = reserve(&p.next_count[g * 2 + 0], (unsigned int)k);
  P *X = (P *)p.X[sel];
  P *U = (P *)p.U[sel];
  uint32_t *ID = p.ID[sel];
  const P xw = wall == 0 ? (P)0 : (P)c.N;
  int emitted = 0;
  for (int e = 0; e < k; ++e) {
    const int slotw = e + 1;
    if ((slotw & 3) == 0)
      rng_block(c.seed, (uint64_t)st.level, (uint64_t)ion_id, 1, (uint64_t)(slotw >> 2), blk);
    const double uu = unit_open(blk[slotw & 3]);
    const double E_se = (c.see_law == GS_SEE_EXP) ? -c.see_E * log(uu) : c.see_E;
    const double v_se = sqrt(2.0 * E_se * c.ev / c.mass[0]);
    const double v_si = wall == 0 ? v_se : -v_se;
    const P u_new = (P)((v_si * c.dt) / c.dx);
    const unsigned long long s = slot + (unsigned long long)e;
    if (s >= (unsigned long long)c.cap[0]) {
      atomicOr(&p.err[0], ERR_CAPACITY);
      atomicCAS(&p.err[1], 0xFFFFFFFFu, (unsigned int)g);
      continue;
    }
    const size_t i = (size_t)c.pbase[0] + s;
    X[i] = xw;
    U[i] = u_new;
    ID[i] = NO_ID;
    emitted += 1;
  }
  return emitted;
}

template <class P, int BS, int PPT>
__global__ __launch_bounds__(BS) void k_push(DevPtrs p, int G, int tile, int nmax) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  typedef typename Acc<P>::cell cell;
  __shared__ int scan_sh[BS];
  // layout: tally[T_N] | prefix[G+1] | eh[nmax+2] (P) | acc[nmax+1] (cell)
  PushShared<P> sh;
  sh.tally = (unsigned int *)lds_raw;
  sh.prefix = (int *)(lds_raw + 64);
  const size_t off = 64 + (((size_t)(G + 1) * 4 + 15) / 16) * 16;
  sh.eh = (P *)(lds_raw + off);
  sh.acc = (cell *)(lds_raw + off + ((((size_t)(nmax + 2) * sizeof(P)) + 15) / 16) * 16);
  const int tid = threadIdx.x;
  const int sel = (int)(*p.epoch & 1);

  // tiles per gap and their prefix (each workgroup builds its own copy in LDS)
  const int per = (G + BS - 1) / BS;
  int mine = 0;
  for (int q = 0; q < per; ++q) {
    const int g = tid * per + q;
    if (g < G) {
      int te, ti, tb;
      gap_tiles(p.gs[g], p.gc[g], tile, te, ti, tb);
      mine += te + ti + tb;
    }
  }
  int tot_tiles;
  int run = block_exclusive_scan_int(mine, scan_sh, &tot_tiles);
  for (int q = 0; q < per; ++q) {
    const int g = tid * per + q;
    if (g < G) {
      sh.prefix[g] = run;
      int te, ti, tb;
      gap_tiles(p.gs[g], p.gc[g], tile, te, ti, tb);
      run += te + ti + tb;
    }
  }
  if (tid == 0) sh.prefix[G] = tot_tiles;
  __syncthreads();

  const int total = sh.prefix[G];
  const int t0 = (int)(((long long)blockIdx.x * total) / gridDim.x);
  const int t1 = (int)(((long long)(blockIdx.x + 1) * total) / gridDim.x);
  int cur = -1;
  int g = 0;
  for (int t = t0; t < t1; ++t) {
    while (sh.prefix[g + 1] <= t) ++g;
    const GapConst &c = p.gc[g];
    const GapState &st = p.gs[g];
    if (g != cur) {
      if (cur >= 0) flush_gap<P>(p, p.gc[cur], cur, sh);
      load_gap<P>(p, c, sh);
      cur = g;
    }
    unsigned long long *gacc = p.acc + c.nbase;
    int te, ti, tb;
    gap_tiles(st, c, tile, te, ti, tb);
    int lt = t - sh.prefix[g];
    const int N = c.N;
    const P Nf = (P)N;
    if (lt < te + ti) {
      const int s = lt < te ? 0 : 1;
      if (s == 1) lt -= te;
      const long long cnt = st.count[s];
      P *X = (P *)p.X[sel] + c.pbase[s];
      P *U = (P *)p.U[sel] + c.pbase[s];
      const P alpha = (P)c.alpha[s];
      const int Z = c.Z[s];
      const bool see = (s == 1) && (c.see_amp > 0.0) && (Z > 0);
      const long long i0 = (long long)lt * tile;
      unsigned int n_pushed = 0, n_abs0 = 0, n_abs1 = 0, n_em0 = 0, n_em1 = 0;
      for (int r = 0; r < tile; r += BS * PPT) {
        P xv[PPT], uv[PPT];
        long long ii[PPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
          ii[k] = i0 + r + (long long)k * BS + tid;
          xv[k] = (P)-1;
          uv[k] = (P)0;
          if (ii[k] < cnt && ii[k] < i0 + tile) {
            xv[k] = X[ii[k]];
            uv[k] = U[ii[k]];
          }
        }
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
          P xi = xv[k];
          if (!(xi >= (P)0)) continue;  // empty slot or absorbed earlier
          n_pushed += 1;
          // gather, then the leapfrog (eq. vel_update_main, eq. pos_update_main)
          P Ep = gather<P>(sh.eh, xi, N);
          P du = alpha * Ep;
          P u1 = uv[k] + du;
          P x1 = xi + u1;
          int wall = -1;
          if (x1 <= (P)0) wall = 0;
          else if (x1 >= Nf) wall = 1;
          if (wall >= 0) {
            X[ii[k]] = (P)-1;
            if (wall == 0) n_abs0 += 1;
            else n_abs1 += 1;
            if (see) {
              const uint32_t id = p.ID[sel][c.pbase[s] + ii[k]];
              int ne = emit_electrons<P>(p, c, st, g, sel, id, u1, wall);
              if (ne) {
                // an electron on the wall node carries its full weight there
                const long long cw = (long long)c.Z[0] * Prec<P>::W;
                for (int e = 0; e < ne; ++e) Acc<P>::add(sh.acc, gacc, wall == 0 ? 0 : N, cw);
                if (wall == 0) n_em0 += ne;
                else n_em1 += ne;
              }
            }
            continue;
          }
          X[ii[k]] = x1;
          U[ii[k]] = u1;
          // deposit with the gather's weights (App. C)
          int j = (int)x1;
          if (j > N - 1) j = N - 1;
          P f = x1 - (P)j;
          long long w1 = Prec<P>::wq(f);
          long long w0 = Prec<P>::W - w1;
          Acc<P>::add(sh.acc, gacc, j, Z * w0);
          Acc<P>::add(sh.acc, gacc, j + 1, Z * w1);
        }
      }
      // wave-level sums, then one LDS atomic per wave
      unsigned int v[5] = {n_pushed, n_abs0, n_abs1, n_em0, n_em1};
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        unsigned int a = v[q];
        for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
        v[q] = a;
      }
      if ((tid & 63) == 0) {
        if (v[0]) atomicAdd(&sh.tally[T_PUSHED], v[0]);
        if (v[1]) atomicAdd(&sh.tally[T_ABS + s * 2 + 0], v[1]);
        if (v[2]) atomicAdd(&sh.tally[T_ABS + s * 2 + 1], v[2]);
        if (v[3]) atomicAdd(&sh.tally[T_EMIT + 0], v[3]);
        if (v[4]) atomicAdd(&sh.tally[T_EMIT + 1], v[4]);
      }
    } else {
      // beam ions entering at the circuit electrode
      lt -= te + ti;
      P *X = (P *)p.X[sel] + c.pbase[1];
      P *U = (P *)p.U[sel] + c.pbase[1];
      uint32_t *ID = p.ID[sel] + c.pbase[1];
      unsigned int n_inj = 0;
      for (int r = tid; r < tile; r += BS) {
        const long long k = (long long)lt * tile + r;
        const bool valid = k < c.beam_n;
        const unsigned long long mask = __ballot(valid);
        if (mask == 0ull) break;
        const int lane = tid & 63;
        const int first = __ffsll((long long)mask) - 1;
        const int rank = __popcll(mask & ((1ull << lane) - 1ull));
        unsigned long long base = 0;
        if (lane == first) base = reserve(&p.next_count[g * 2 + 1], (unsigned int)__popcll(mask));
        base = __shfl(base, first);
        if (!valid) continue;
        uint64_t blk[4];
        rng_block(c.seed, (uint64_t)st.level, (uint64_t)k, 2, 0, blk);
        const double E = c.beam_Emin + (c.beam_Emax - c.beam_Emin) * unit_open(blk[0]);
        const double v = sqrt(2.0 * E * c.ev / c.mass[1]);
        const double x = unit_open(blk[1]) * v * c.dt;
        const P xi = (P)(x / c.dx);
        const P u = (P)((v * c.dt) / c.dx);
        const unsigned long long slot = base + (unsigned long long)rank;
        if (slot >= (unsigned long long)c.cap[1]) {
          atomicOr(&p.err[0], ERR_CAPACITY);
          atomicCAS(&p.err[1], 0xFFFFFFFFu, (unsigned int)g);
          continue;
        }
        X[slot] = xi;
        U[slot] = u;
        ID[slot] = (uint32_t)(st.beam_id0 + k);
        n_inj += 1;
        int j = (int)xi;
        if (j > N - 1) j = N - 1;
        P f = xi - (P)j;
        long long w1 = Prec<P>::wq(f);
        long long w0 = Prec<P>::W - w1;
        Acc<P>::add(sh.acc, gacc, j, c.Z[1] * w0);
        Acc<P>::add(sh.acc, gacc, j + 1, c.Z[1] * w1);
      }
      unsigned int a = n_inj;
      for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
      if ((tid & 63) == 0 && a) atomicAdd(&sh.tally[T_INJ], a);
    }
  }
  if (cur >= 0) flush_gap<P>(p, p.gc[cur], cur, sh);
}

// ---------------------------------------------------------------------------
// k_compact: copy live slots of every (gap, species) region into the other
// buffer; order inside a region is not kept (nothing depends on it)
// ---------------------------------------------------------------------------
template <class P, int BS>
__global__ __launch_bounds__(BS) void k_compact(DevPtrs p, int G, int tile) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  int *prefix = (int *)lds_raw;  // [2G + 1]
  __shared__ int scan_sh[BS];
  __shared__ unsigned int wave_cnt[BS / 64];
  __shared__ unsigned long long blk_base;
  const int tid = threadIdx.x;
  const int src = (int)(*p.epoch & 1), dst = src ^ 1;
  const int R = 2 * G;
  const int per = (R + BS - 1) / BS;
  int mine = 0;
  for (int q = 0; q < per; ++q) {
    const int r = tid * per + q;
    if (r < R) mine += (int)(((long long)p.next_count[r] + tile - 1) / tile);
  }
  int total_t;
  int run = block_exclusive_scan_int(mine, scan_sh, &total_t);
  for (int q = 0; q < per; ++q) {
    const int r = tid * per + q;
    if (r < R) {
      prefix[r] = run;
      run += (int)(((long long)p.next_count[r] + tile - 1) / tile);
    }
  }
  if (tid == 0) prefix[R] = total_t;
  __syncthreads();
  const int total = prefix[2 * G];
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    int lo = 0, hi = 2 * G;  // find region r with prefix[r] <= t < prefix[r+1]
    while (hi - lo > 1) {
      int mid = (lo + hi) / 2;
      if (prefix[mid] <= t) lo = mid;
      else hi = mid;
    }
    const int r = lo;
    const int g = r >> 1, s = r & 1;
    const GapConst &c = p.gc[g];
    const long long n = (long long)p.next_count[g * 2 + s];
    const long long i0 = (long long)(t - prefix[r]) * tile;
    const P *Xs = (const P *)p.X[src] + c.pbase[s];
    const P *Us = (const P *)p.U[src] + c.pbase[s];
    const uint32_t *Is = p.ID[src] + c.pbase[s];
    P *Xd = (P *)p.X[dst] + c.pbase[s];
    P *Ud = (P *)p.U[dst] + c.pbase[s];
    uint32_t *Id = p.ID[dst] + c.pbase[s];
    for (int rr = 0; rr < tile; rr += BS) {
      const long long i = i0 + rr + tid;
      P x = (P)-1;
      if (i < n && rr + tid < tile) x = Xs[i];
      const bool live = x >= (P)0;
      const unsigned long long mask = __ballot(live);
      const int lane = tid & 63, w = tid >> 6;
      if (lane == 0) wave_cnt[w] = (unsigned int)__popcll(mask);
      __syncthreads();
      if (tid == 0) {
        unsigned int tot = 0;
        for (int q = 0; q < BS / 64; ++q) {
          unsigned int a = wave_cnt[q];
          wave_cnt[q] = tot;
          tot += a;
        }
        blk_base = tot ? atomicAdd(&p.cursor[g * 2 + s], (unsigned long long)tot) : 0ull;
      }
      __syncthreads();
      if (live) {
        const unsigned long long o =
            blk_base + wave_cnt[w] + (unsigned int)__popcll(mask & ((1ull << lane) - 1ull));
        Xd[o] = x;
        Ud[o] = Us[i];
        Id[o] = Is[i];
      }
      __syncthreads();
    }
  }
}

__global__ void k_commit(DevPtrs p, int G) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 2 * G) {
    p.next_count[i] = p.cursor[i];
    p.cursor[i] = 0ull;
  }
  if (i == 0) *p.epoch += 1;
}

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
  if (lane == first) base = atomicAdd(&p.next_count[gap * 2 + species], (unsigned long long)__popcll(mask));
  base = __shfl(base, first);
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
  P f = xi - (P)j;
  long long w1 = Prec<P>::wq(f);
  long long w0 = Prec<P>::W - w1;
  unsigned long long *gacc = p.acc + c.nbase;
  atomicAdd(&gacc[j], (unsigned long long)(c.Z[species] * w0));
  atomicAdd(&gacc[j + 1], (unsigned long long)(c.Z[species] * w1));
}

// phi_i = dx sum_{k >= i} E_{k+1/2}, phi_N = 0 (one gap, one workgroup)
__global__ __launch_bounds__(FBS) void k_phi(DevPtrs p, int gap) {
  const GapConst &c = p.gc[gap];
  __shared__ double sh[FBS];
  const int N = c.N, tid = threadIdx.x;
  const double *E = p.E64 + c.nbase;
  double *phi = p.phi64 + c.nbase;
  const int chunk = (N + FBS - 1) / FBS;
  // thread t owns the reversed range
  const int k0 = tid * chunk, k1 = min(k0 + chunk, N);
  double loc = 0.0;
  for (int k = k1 - 1; k >= k0; --k) loc += c.dx * E[N - 1 - k];
  double tot;
  double run = block_exclusive_scan(loc, sh, &tot);
  for (int k = k0; k < k1; ++k) {
    // reversed index m = N - 1 - k walks down from the grounded end
    run += c.dx * E[N - 1 - k];
    phi[N - 1 - k] = run;
  }
  (void)tot;
  if (tid == 0) phi[N] = 0.0;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
size_t push_lds_bytes(int nmax, int fp64, int G) {
  const size_t ps = fp64 ? 8 : 4, cs = fp64 ? 8 : 4;
  size_t off = 64 + (((size_t)(G + 1) * 4 + 15) / 16) * 16;
  off += (((size_t)(nmax + 2) * ps + 15) / 16) * 16;
  off += (size_t)(nmax + 1) * cs;
  return off;
}

hipError_t launch_field(const DevPtrs &p, int G, int mode, int guess, double tol, int maxit,
                        int fp64, hipStream_t s) {
  hipLaunchKernelGGL(k_field, dim3(G), dim3(FBS), 0, s, p, mode, guess, tol, maxit, fp64);
  return hipGetLastError();
}

template <class P, int BS, int PPT>
static hipError_t push_t(const DevPtrs &p, int G, const LaunchCfg &lc, hipStream_t s) {
  const size_t lds = push_lds_bytes(lc.nmax, lc.fp64, G);
  // opt in to more than 64 KiB of dynamic LDS (gfx950 has 160 KiB per CU)
  static size_t attr_set = 65536;
  if (lds > attr_set) {
    hipError_t e = hipFuncSetAttribute((const void *)k_push<P, BS, PPT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_set = lds;
  }
  hipLaunchKernelGGL((k_push<P, BS, PPT>), dim3(lc.grid), dim3(BS), lds, s, p, G, lc.tile, lc.nmax);
  return hipGetLastError();
}

hipError_t launch_push(const DevPtrs &p, int G, const LaunchCfg &lc, hipStream_t s) {
  if (lc.fp64) {
    switch (lc.block) {
      case 256: return push_t<double, 256, 2>(p, G, lc, s);
      case 512: return push_t<double, 512, 2>(p, G, lc, s);
      default: return push_t<double, 1024, 2>(p, G, lc, s);
    }
  }
  switch (lc.block) {
    case 256: return push_t<float, 256, 4>(p, G, lc, s);
    case 512: return push_t<float, 512, 4>(p, G, lc, s);
    default: return push_t<float, 1024, 4>(p, G, lc, s);
  }
}

hipError_t launch_compact(const DevPtrs &p, int G, const LaunchCfg &lc, hipStream_t s) {
  const int grid = lc.grid > 0 ? lc.grid * 2 : 1024;
  const size_t lds = ((size_t)(2 * G + 1) * 4 + 15) / 16 * 16;
  if (lc.fp64)
    hipLaunchKernelGGL((k_compact<double, 256>), dim3(grid), dim3(256), lds, s, p, G, lc.tile);
  else
    hipLaunchKernelGGL((k_compact<float, 256>), dim3(grid), dim3(256), lds, s, p, G, lc.tile);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_commit, dim3((2 * G + 255) / 256), dim3(256), 0, s, p, G);
  return hipGetLastError();
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

hipError_t launch_phi(const DevPtrs &p, int gap, hipStream_t s) {
  hipLaunchKernelGGL(k_phi, dim3(1), dim3(FBS), 0, s, p, gap);
  return hipGetLastError();
}

}  // namespace gs
