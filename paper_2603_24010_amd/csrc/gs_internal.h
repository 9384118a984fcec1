// Private definitions shared by the library's host and device sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gapsim.h"

namespace gs {

constexpr int MAXM = GS_MAX_MESH;
constexpr uint32_t NO_ID = 0xFFFFFFFFu;
// fixed-point charge weights: a macroparticle is 2^F units
constexpr int F32_BITS = 24;
constexpr int F64_BITS = 44;
// tallies per gap, filled by the push and folded into the state by the field solve
enum {
  T_ABS = 0,      // [s*2 + wall], 4 entries
  T_EMIT = 4,     // [wall], 2 entries
  T_INJ = 6,
  T_PUSHED = 7,   // live particles pushed
  T_N = 8
};

// Per-gap constants (read-only on the device).
struct GapConst {
  int32_t N;          // cells
  int32_t M, g;       // meshes, gap mesh
  int32_t see_law, see_max;
  int32_t see_yield, pad_y;
  int32_t Z[2];
  int32_t beam_side;  // GS_BEAM_CIRCUIT or GS_BEAM_GROUND
  int64_t beam_n;     // ions per step without a schedule
  int64_t sched_base, sched_len;  // the gap's beam schedule in DevPtrs::sched (len 0: none)
  int64_t cap[2];
  int64_t pbase[2];   // first particle slot of species s
  int64_t nbase;      // offset of the node arrays (N + 1 entries)
  int64_t evbase;     // first slot of the gap's absorbed-ion event list
  int64_t evcap;      // its capacity
  int64_t ebase;      // offset of the binary32/64 field table (N + 2 entries)
  int64_t hbase[2];   // first counter of species s in the cell-sort bin arrays
                      // (room for ceil(N / SORT_BIN_MIN) bins per species)
  uint64_t seed;
  double d, dx, A, eps0, dt, cgap, c_par;
  double s0;           // sheet charge per unit of Z: weight * q_unit [C/m^2]
  double alpha[2];     // Z q dt^2 / (m dx): velocity change in cells/step per V/m
  double mass[2], ev;
  double see_amp, see_E0, see_E;
  double see_poly[6], see_pEmax;  // GS_YIELD_POLY: coefficients in powers of E / 1 keV, E clamp [eV]
  double see_mu, see_sig;         // GS_SEE_LOGNORMAL: ln E ~ N(mu, sig^2), E in eV
  double beam_Emin, beam_Emax;
  double beam_layer;  // [m]; 0: one step of flight
  double v_ref;
  double src_dc, src_amp, src_w, src_phase;
  // strict: D = sL h + sR D1 - sS q1 + sb Vs - sz phi0     (h = 15 D1 - 7 D2 + D3)
  double sL[MAXM * MAXM], sR[MAXM * MAXM], sS[MAXM * MAXM], sb[MAXM], sz[MAXM];
  // weak: D* = wL h + wR D1 - wS q1 + wb Vs
  double wL[MAXM * MAXM], wR[MAXM * MAXM], wS[MAXM * MAXM], wb[MAXM];
  // T' itself (loop equations in volts for the Newton residual)
  double Tp[MAXM * MAXM];
  // Newton on u = (V, I_0..I_{M-1}): the residual is affine in u, so its
  // Jacobian J is constant; Jinv row-major (M+1)^2
  double Jinv[(MAXM + 1) * (MAXM + 1)];
};

// Per-gap mutable state (device).
struct GapState {
  int64_t level;        // last solved level (-1 before the first step)
  int64_t seen_epoch;   // compaction epoch already applied to this gap
  int64_t count[2];     // slots the current push sweeps, per species
  int64_t live[2];      // live particles after the last push, per species
  int64_t next_id;      // next particle id
  int64_t beam_id0;     // id of beam particle 0 of the current push
  int64_t beam_now;     // beam ions of the current push
  double qprev[MAXM];   // loop charges q^{n-1}
  double dq[3][MAXM];   // increments D^{n-1}, D^{n-2}, D^{n-3}
  double sigma_prev, qcirc_prev;
  // u = (V, I) history for the Newton guess
  double uh[3][MAXM + 1];
  // diagnostics of the last solved level
  double t, phi0, sigma, qcirc, qcirc_star, qconv, e_ground;
  double qcirc_step;    // Q_circ* of this level minus Q_circ of the one before
  double q_space;       // A times the integral of rho over the gap at this level
  double q[MAXM], I[MAXM];
  int64_t abs_last[4], emit_last[2], inj_last, pushed_last;
  int64_t abs_cum[4], emit_cum[2], inj_cum, pushed_cum;
  int32_t newton_last, newton_fb_last;
  int64_t newton_total, newton_fallbacks;
  int32_t newton_max, newton_levels;  // most corrections at one level; Newton levels solved
  double newton_r0, newton_r;
  double guess[MAXM + 1];  // the u the last Newton solve started from
  double mlp_prop[3];      // the guess network's proposal at the last solve (used or not)
  // ring of the last 8 levels' (V, I_0, I_1, sigma, Q_abs, Q_em): the guess
  // network's input; hist_head is the slot the next level goes to
  double hist[8][6];
  int32_t hist_head, pad1;
};

// An ion absorbed by an electrode, waiting for its secondary emission.
struct Event {
  double u;       // impact velocity in cells per step
  uint32_t ref;   // in a push workgroup's LDS queue: the ion's slot in its region;
                  // in the gap's overflow list: the ion's id (a compaction may move
                  // the slot before the field kernel emits).  The id keys the draws.
  uint32_t wall;
};

// Context-wide device pointers handed to kernels.
struct DevPtrs {
  const GapConst *gc;
  GapState *gs;
  // particle slots, two buffers selected by compaction epoch parity
  void *X[2], *U[2];
  uint32_t *ID[2];
  unsigned long long *next_count;  // [G][2] append cursor
  unsigned long long *cursor;      // [G][2] slot count after the compaction or sort in progress
  unsigned long long *tally;       // [G][T_N]
  unsigned long long *acc;         // node charge accumulators, int64 two's complement
  double *rho64, *E64, *phi64;     // node / half-grid / node arrays (nbase offsets; E uses nbase too)
  void *ehat;                      // field table for the push, binary32 or binary64
  int64_t *epoch;                  // compaction epoch (device)
  unsigned int *err;               // [0] flags, [1] gap of first error
  unsigned int *steal;             // the push's pool counter, cleared by the field solve
  unsigned int *push_done;         // push workgroups done: a top counter and 32 group
                                   // counters, 128 bytes apart (the last resets them)
  // the field solve's hand-offs between its kernels: the prefix sums of the
  // cell terms within chunks of FCN nodes (per node), the chunks' totals and
  // weighted sums [G][NCHMAX][2], their offsets [G][NCHMAX], sigma [G]
  double *fsl, *fpart, *foff, *fsig;
  Event *ev;                       // absorbed-ion events, per-gap lists
  unsigned long long *ev_count;    // [G]
  unsigned long long *ev_done;     // [G] events of the list already emitted by k_emit
  // periodic cell sort: live particles per bin, then per-bin write cursors
  unsigned long long *hist, *bcur;
  // in-place compaction: live particles per tile (then their prefix), at
  // tcnt[pbase / 64 + k] for tile k of a region; holes below the live count
  int *tcnt;
  unsigned long long *fill_h;  // [G][2]
  unsigned long long *live;    // a bit per slot, 64 per word from pbase / 64
  int *wrank;                  // per word past the live count: tail rank of its first live slot
  const int64_t *sched;            // beam schedules of all gaps (GapConst::sched_base)
  // exchange with an external circuit engine (field mode 2), in pinned host
  // memory the device maps: ext_v[g] the engine's gap voltage for the level
  // being solved (read), ext_phi[g] the electrode potential it gave (written)
  const double *ext_v;
  double *ext_phi;
  // mapped host word: the events the last push left in the gaps' lists (an
  // upper bound when k_emit wrote it), which the host reads to choose who
  // emits the next push's lists
  unsigned long long *list_seen;
  Event *ovf;                      // push workgroup b < ovf_wgs: events past its LDS queue,
  int64_t ovf_wgs;                 //   ovq of them from ovf + b * ovq
  int64_t ovq;
  // Newton guess network: bfloat16 weights (flat layout of gs_mlp_dev.h) and
  // the normalisation block; null until weights are set
  const uint16_t *mlp_w;
  const double *mlp_norm;
  // sample recording for training: level n of gap g goes to sample
  // (n - rec_level0) * G + g when that is below rec_cap
  float *rec_x;  // [rec_cap][48] raw features
  float *rec_y;  // [rec_cap][3] raw targets u* - u_extrapolated
  int64_t rec_cap, rec_level0;
};

enum { ERR_CAPACITY = 1u, ERR_BADINJECT = 2u, ERR_NOCONV = 4u };

// Nodes per chunk of the field solve's density and table kernels, and the
// chunks of the largest gap (16384 cells: nodes 0..16384).
constexpr int FCN = 1024;
constexpr int NCHMAX = 16384 / FCN + 1;

// Smallest cell-sort bin (cells per bin): bounds the bin arrays and the LDS of
// the sort kernels (16384 cells -> 4096 bins per species).
constexpr int SORT_BIN_MIN = 4;

// Absorbed-ion events a push workgroup keeps in its global overflow region
// (past these they go to the gap's list, emitted by k_emit after the push):
// from OVQ_MIN to OVQ_MAX, in proportion to the emitting gaps' ion slots.  A
// position in the gap's list costs each wave that needs one a returning atomic
// on the gap's counter, and at some 1e5 overflowing events a step those
// serialise; the regions are sized so that a push rarely needs the list.
constexpr int OVQ_MIN = 1024, OVQ_MAX = 8192;


struct LaunchCfg {
  int block;         // push block size
  int tile;          // particles per tile
  int grid;          // push blocks
  int nmax;          // largest n_cells of the context
  int fp64;          // particle precision
  int wide;          // binary32: 64-bit LDS deposit cells (else 32-bit cells with carries)
  int compact_grid;  // compaction blocks
  int ppt;           // particles per thread per chunk (one or two 16-byte vectors)
  int sort_bin;      // cells per bin of the periodic counting sort that replaces the
                     // compaction (0: plain compaction); with it the push queues no
                     // events past its LDS queue and k_emit emits them after the push
  int steal;         // the last 1/steal of each push workgroup's tiles go to a pool
                     // that workgroups done with their own draw from (0: none)
  int stream;        // push particle stream: STREAM_RR round-robin tile order,
                     // STREAM_NT non-temporal binary32 loads and stores
  int masks;         // per launch: the push writes the live masks of the words
                     // below each region's count, and the compaction that follows
                     // takes them instead of reading those positions
  int lists;         // per launch: the push's last workgroup emits the gaps'
                     // lists of absorbed ions (else k_emit does, after the push)
};
constexpr int STREAM_RR = 1, STREAM_NT = 2;

// launchers (gs_kernels.hip)
// Optional timing: when `a` is set, the start and end of the launched kernel(s)
// are recorded into these events by the dispatch packets themselves
// (hipExtLaunchKernel), so the elapsed time holds no launch latency.
struct KTime {
  hipEvent_t a = nullptr, b = nullptr;
};

hipError_t launch_field(const DevPtrs &p, int G, int mode, int guess, double newton_tol,
                        int newton_maxit, int fp64, int nmax, hipStream_t s, KTime t = {});
hipError_t launch_push(const DevPtrs &p, int G, const LaunchCfg &lc, hipStream_t s, KTime t = {});
// its instantiations, compiled in units of their own
hipError_t launch_push_f64(const DevPtrs &p, int G, const LaunchCfg &lc, hipStream_t s, KTime t);
hipError_t launch_push_f32w(const DevPtrs &p, int G, const LaunchCfg &lc, hipStream_t s, KTime t);
hipError_t launch_push_f32c(const DevPtrs &p, int G, const LaunchCfg &lc, hipStream_t s, KTime t);
hipError_t launch_push_f32w_nt(const DevPtrs &p, int G, const LaunchCfg &lc, hipStream_t s, KTime t);
hipError_t launch_push_f32c_nt(const DevPtrs &p, int G, const LaunchCfg &lc, hipStream_t s, KTime t);
hipError_t launch_compact(const DevPtrs &p, int G, const LaunchCfg &lc, hipStream_t s, KTime t = {});
// the cell sort (count, scan, scatter, commit), in place of launch_compact
hipError_t launch_sort(const DevPtrs &p, int G, const LaunchCfg &lc, hipStream_t s, KTime t = {});
// secondary emission of every gap's queued events, many workgroups (after a push)
hipError_t launch_emit(const DevPtrs &p, int G, int fp64, int grid, hipStream_t s, KTime t = {});
hipError_t launch_inject(const DevPtrs &p, int gap, int species, long long n, const double *x_dev,
                         const double *v_dev, long long id0, int fp64, hipStream_t s);
hipError_t launch_phi(const DevPtrs &p, int gap, hipStream_t s);
// time-step check: largest |u| per species (bit patterns of non-negative
// floats, max-reduced as unsigned integers) and electrons per cell of one gap
hipError_t launch_dt_scan(const DevPtrs &p, int gap, int N, int fp64, unsigned long long *umax,
                          unsigned int *cells, hipStream_t s);
// guess network (gs_mlp.hip): y[n][3] = net(x[n][48]) with bfloat16 weights W
hipError_t launch_mlp_forward(const uint16_t *W, const float *x, long long n, float *y, hipStream_t s);
size_t push_lds_bytes(int nmax, int fp64, int G, int wide);
size_t sort_lds_bytes(int G, int nmax, int bin);

}  // namespace gs
