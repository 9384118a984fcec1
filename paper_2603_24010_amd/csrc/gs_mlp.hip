// Training and batch evaluation of the Newton guess network on the GPU.
//
// Training is plain mini-batch gradient descent with Adam (Kingma and Ba,
// 2015) on the mean squared error, in binary32: forward and backward are
// strided GEMMs on the matrix cores with fused epilogues (bias, GELU, GELU'),
// the weight gradients split over the batch and summed in a fixed order, bias
// gradients are column sums; every reduction has a fixed order, so a run is
// bitwise repeatable.  Batch evaluation uses the same device routine as the
// strict step (bfloat16 weights, binary32 sums).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "gapsim.h"
#include "gs_internal.h"
#include "gs_mlp_dev.h"

namespace gs {

// ---------------------------------------------------------------------------
// C[m][n] = epilogue(sum_k A(m,k) B(k,n)),  A(m,k) = A[m sam + k sak],
// B(k,n) = B[k sbk + n sbn], C row-major with leading dimension ldc.
// On the matrix cores in binary32 (v_mfma_f32_16x16x4_f32: binary32 products,
// binary32 sums): 64 x 64 output tiles, 256 threads, each wave a 32 x 32
// quadrant as 2 x 2 blocks of 16 x 16; K in steps of 16 through LDS, the next
// step's operands loaded into registers while the current one is multiplied.
// blockIdx.z takes a slice of kslice of the K range (split-K): slice z writes
// C + z * slice_stride, and the slices are then summed in order z = 0, 1, ...
// (k_sum_slices).  Every sum has a fixed order, so a run is bitwise
// repeatable.
// Lane l of a wave gives the 16 x 4 A block's element (l % 16, l / 16) and the
// 4 x 16 B block's (l / 16, l % 16); its accumulator r holds D(4 (l / 16) + r,
// l % 16).
// ---------------------------------------------------------------------------
enum { EP_STORE = 0, EP_BIAS_GELU = 1, EP_BIAS = 2, EP_GELU_GRAD = 3 };

constexpr int GT = 64, GK = 16;
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ inline float gelu_grad_f32(float z) {
  const float Phi = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
  return Phi + z * (0.39894228040143268f * expf(-0.5f * z * z));
}

template <int EP>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, int kslice, const float *A, long sam, long sak,
                                              const float *B, long sbk, long sbn, float *C, long ldc,
                                              long slice_stride, const float *bias, float *Zout, const float *Zin) {
  __shared__ float As[GK][GT + 4];
  __shared__ float Bs[GK][GT + 4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  const int k_lo = blockIdx.z * kslice, k_hi = min(K, k_lo + kslice);
  const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;  // this wave's quadrant
  C += (long)blockIdx.z * slice_stride;
  // staging: element e = tid + 256 q of the 16 x 64 tile, q = 0..3
  float ra[4], rb[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q, kk = e / GT, mm = e % GT;
      const int k = k0 + kk, m = m0 + mm, n = n0 + mm;
      ra[q] = (m < M && k < k_hi) ? A[(long)m * sam + (long)k * sak] : 0.0f;
      rb[q] = (n < N && k < k_hi) ? B[(long)k * sbk + (long)n * sbn] : 0.0f;
    }
  };
  v4f acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (v4f){0.0f, 0.0f, 0.0f, 0.0f};
  if (k_lo < k_hi) load(k_lo);
  for (int k0 = k_lo; k0 < k_hi; k0 += GK) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      As[e / GT][e % GT] = ra[q];
      Bs[e / GT][e % GT] = rb[q];
    }
    __syncthreads();
    if (k0 + GK < k_hi) load(k0 + GK);
#pragma unroll
    for (int kk = 0; kk < GK; kk += 4) {
      const int kr = kk + (lane >> 4), c = lane & 15;
      const float a0 = As[kr][wm + c], a1 = As[kr][wm + 16 + c];
      const float b0 = Bs[kr][wn + c], b1 = Bs[kr][wn + 16 + c];
      acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + r, n = n0 + wn + 16 * j + (lane & 15);
        if (m >= M || n >= N) continue;
        const long o = (long)m * ldc + n;
        float v = acc[i][j][r];
        if (EP == EP_BIAS_GELU) {
          const float z = v + bias[n];
          Zout[o] = z;
          v = gelu_f32(z);
        } else if (EP == EP_BIAS) {
          v += bias[n];
        } else if (EP == EP_GELU_GRAD) {
          v *= gelu_grad_f32(Zin[o]);
        }
        C[o] = v;
      }
}

// C[i] = sum over z = 0..S-1 of P[z * stride + i], i < n, in that order
__global__ void k_sum_slices(const float *P, int S, long stride, long n, float *C) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.0f;
  for (int z = 0; z < S; ++z) s += P[(long)z * stride + i];
  C[i] = s;
}

template <int EP>
static hipError_t gemm(hipStream_t s, int M, int N, int K, const float *A, long sam, long sak, const float *B,
                       long sbk, long sbn, float *C, long ldc, const float *bias = nullptr,
                       float *Zout = nullptr, const float *Zin = nullptr) {
  dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT, 1);
  hipLaunchKernelGGL(k_gemm<EP>, grid, dim3(256), 0, s, M, N, K, K, A, sam, sak, B, sbk, sbn, C, ldc, 0L, bias,
                     Zout, Zin);
  return hipGetLastError();
}

// Up to SPLITK_MAX slices of the K range (each a whole number of K steps),
// for the weight gradients, whose K is the batch.
constexpr int SPLITK_MAX = 16;

static int splitk_slices(int K) {
  const int steps = (K + GK - 1) / GK;
  return steps < 4 ? 1 : (steps / 4 < SPLITK_MAX ? steps / 4 : SPLITK_MAX);
}

// C (M x N, contiguous rows) = A B with the K range split over slices, each
// slice's partial in P, then summed in slice order into C
static hipError_t gemm_splitk(hipStream_t s, int M, int N, int K, const float *A, long sam, long sak,
                              const float *B, long sbk, long sbn, float *C, float *P) {
  const int S = splitk_slices(K);
  const int kslice = ((K + S - 1) / S + GK - 1) / GK * GK;
  const int used = (K + kslice - 1) / kslice;
  const long n = (long)M * N;
  dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT, used);
  hipLaunchKernelGGL(k_gemm<EP_STORE>, grid, dim3(256), 0, s, M, N, K, kslice, A, sam, sak, B, sbk, sbn, P,
                     (long)N, n, nullptr, nullptr, nullptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_slices, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (const float *)P, used, n, n,
                     C);
  return hipGetLastError();
}

// batch rows selected by order[step * B + b]; an index outside [0, n) is
// replaced by 0 and counted in *bad
__global__ void k_gather(const float *x, const float *t, long long n, const int32_t *order, long long off, int B,
                         float *xb, float *tb, unsigned int *bad) {
  const int b = blockIdx.x;
  long long i = order[off + b];
  if (i < 0 || i >= n) {
    if (threadIdx.x == 0) atomicAdd(bad, 1u);
    i = 0;
  }
  for (int f = threadIdx.x; f < MLP_IN; f += blockDim.x) xb[(long)b * MLP_IN + f] = x[i * MLP_IN + f];
  if (threadIdx.x < MLP_OUT) tb[(long)b * MLP_OUT + threadIdx.x] = t[i * MLP_OUT + threadIdx.x];
}

// loss = mean (y - t)^2 over B x 3 values; dy = 2 (y - t) / (3 B)
__global__ __launch_bounds__(256) void k_loss(const float *y, const float *t, int B, float *dy, float *loss) {
  __shared__ float red[256];
  const int n = B * MLP_OUT;
  const float inv = 1.0f / (float)n;
  float s = 0.0f;
  for (int i = threadIdx.x; i < n; i += 256) {
    const float e = y[i] - t[i];
    s += e * e;
    dy[i] = 2.0f * e * inv;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) *loss = red[0] * inv;
}

// db[j] = sum_b dz[b][j]: 64 columns per workgroup and 16 row groups, group r
// summing rows r, r + 16, ... in order (eight loads in flight), then the 16
// partial sums of a column added in group order
constexpr int CS_COLS = 64, CS_GROUPS = 16;
__global__ __launch_bounds__(CS_COLS *CS_GROUPS) void k_colsum(const float *dz, int B, int N, float *db) {
  __shared__ float part[CS_GROUPS][CS_COLS];
  const int c = threadIdx.x % CS_COLS, r = threadIdx.x / CS_COLS;
  const int j = blockIdx.x * CS_COLS + c;
  const int jj = j < N ? j : N - 1;  // (columns past N read a valid one and are dropped)
  float s = 0.0f;
  int b = r;
  for (; b + 7 * CS_GROUPS < B; b += 8 * CS_GROUPS) {
    float v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = dz[(long)(b + q * CS_GROUPS) * N + jj];
#pragma unroll
    for (int q = 0; q < 8; ++q) s += v[q];
  }
  for (; b < B; b += CS_GROUPS) s += dz[(long)b * N + jj];
  part[r][c] = s;
  __syncthreads();
  if (r == 0 && j < N) {
    float t = 0.0f;
    for (int q = 0; q < CS_GROUPS; ++q) t += part[q][c];
    db[j] = t;
  }
}

__global__ void k_adam(float *th, float *m, float *v, const float *g, int np, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ __launch_bounds__(256) void k_mlp_forward(const uint16_t *W, const float *x, float *y) {
  __shared__ float s_x[MLP_IN], s_h0[MLP_H], s_h1[MLP_H], s_y[MLP_OUT];
  const long b = blockIdx.x;
  if (threadIdx.x < MLP_IN) s_x[threadIdx.x] = x[b * MLP_IN + threadIdx.x];
  mlp_eval_block(W, s_x, s_h0, s_h1, s_y);
  if (threadIdx.x < MLP_OUT) y[b * MLP_OUT + threadIdx.x] = s_y[threadIdx.x];
}

hipError_t launch_mlp_forward(const uint16_t *W, const float *x, long long n, float *y, hipStream_t s) {
  for (long long b0 = 0; b0 < n; b0 += (1 << 30)) {
    const long long nb = n - b0 < (1 << 30) ? n - b0 : (1 << 30);
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned int)nb), dim3(256), 0, s, W, x + b0 * MLP_IN,
                       y + b0 * MLP_OUT);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// workspace layout (floats) for batch B
struct TrainWs {
  float *xb, *tb, *z1, *a1, *z2, *a2, *z3, *a3, *y, *dy, *d0, *d1, *grad, *part;
  unsigned int *bad;
};

// the split-K partials of the largest weight gradient (H x H)
constexpr size_t PART_FLOATS = (size_t)SPLITK_MAX * MLP_H * MLP_H;

static size_t ws_floats(int B) {
  return (size_t)B * (MLP_IN + 2 * MLP_OUT + 6 * MLP_H + MLP_OUT + 2 * MLP_H) + MLP_NPARAM + PART_FLOATS + 64 * 16;
}

static TrainWs ws_map(void *work, int B) {
  TrainWs w;
  float *f = (float *)work;
  auto take = [&](size_t n) {
    float *r = f;
    f += (n + 63) / 64 * 64;
    return r;
  };
  w.bad = (unsigned int *)take(64);
  w.xb = take((size_t)B * MLP_IN);
  w.tb = take((size_t)B * MLP_OUT);
  w.z1 = take((size_t)B * MLP_H);
  w.a1 = take((size_t)B * MLP_H);
  w.z2 = take((size_t)B * MLP_H);
  w.a2 = take((size_t)B * MLP_H);
  w.z3 = take((size_t)B * MLP_H);
  w.a3 = take((size_t)B * MLP_H);
  w.y = take((size_t)B * MLP_OUT);
  w.dy = take((size_t)B * MLP_OUT);
  w.d0 = take((size_t)B * MLP_H);
  w.d1 = take((size_t)B * MLP_H);
  w.grad = take(MLP_NPARAM);
  w.part = take(PART_FLOATS);
  return w;
}

// one optimiser step on the batch at order[off .. off + B)
static hipError_t train_step(const float *x, const float *t, long long n, const int32_t *order, long long off,
                             int B, float *th, float *m, float *v, long long step, float lr, float b1, float b2,
                             float eps, float *loss, const TrainWs &w, hipStream_t s) {
  hipError_t e;
#define CK(x)                      \
  do {                             \
    if ((e = (x)) != hipSuccess) \
      return e;                    \
  } while (0)
  hipLaunchKernelGGL(k_gather, dim3(B), dim3(64), 0, s, x, t, n, order, off, B, w.xb, w.tb, w.bad);
  CK(hipGetLastError());
  const float *W1 = th + MLP_OFF_W1, *W2 = th + MLP_OFF_W2, *W3 = th + MLP_OFF_W3, *W4 = th + MLP_OFF_W4;
  float *g = w.grad;
  const int H = MLP_H, I = MLP_IN, O = MLP_OUT;
  // forward: z = a W^T + b, a' = GELU(z)
  CK(gemm<EP_BIAS_GELU>(s, B, H, I, w.xb, I, 1, W1, 1, I, w.a1, H, th + MLP_OFF_B1, w.z1));
  CK(gemm<EP_BIAS_GELU>(s, B, H, H, w.a1, H, 1, W2, 1, H, w.a2, H, th + MLP_OFF_B2, w.z2));
  CK(gemm<EP_BIAS_GELU>(s, B, H, H, w.a2, H, 1, W3, 1, H, w.a3, H, th + MLP_OFF_B3, w.z3));
  CK(gemm<EP_BIAS>(s, B, O, H, w.a3, H, 1, W4, 1, H, w.y, O, th + MLP_OFF_B4));
  hipLaunchKernelGGL(k_loss, dim3(1), dim3(256), 0, s, w.y, w.tb, B, w.dy, loss);
  CK(hipGetLastError());
  // backward: dW = dz^T a_prev, db = column sums of dz, dz_prev = (dz W) * GELU'(z_prev)
  CK(gemm_splitk(s, O, H, B, w.dy, 1, O, w.a3, H, 1, g + MLP_OFF_W4, w.part));
  hipLaunchKernelGGL(k_colsum, dim3(1), dim3(CS_COLS * CS_GROUPS), 0, s, w.dy, B, O, g + MLP_OFF_B4);
  CK(hipGetLastError());
  CK(gemm<EP_GELU_GRAD>(s, B, H, O, w.dy, O, 1, W4, H, 1, w.d0, H, nullptr, nullptr, w.z3));
  CK(gemm_splitk(s, H, H, B, w.d0, 1, H, w.a2, H, 1, g + MLP_OFF_W3, w.part));
  hipLaunchKernelGGL(k_colsum, dim3(H / CS_COLS), dim3(CS_COLS * CS_GROUPS), 0, s, w.d0, B, H, g + MLP_OFF_B3);
  CK(hipGetLastError());
  CK(gemm<EP_GELU_GRAD>(s, B, H, H, w.d0, H, 1, W3, H, 1, w.d1, H, nullptr, nullptr, w.z2));
  CK(gemm_splitk(s, H, H, B, w.d1, 1, H, w.a1, H, 1, g + MLP_OFF_W2, w.part));
  hipLaunchKernelGGL(k_colsum, dim3(H / CS_COLS), dim3(CS_COLS * CS_GROUPS), 0, s, w.d1, B, H, g + MLP_OFF_B2);
  CK(hipGetLastError());
  CK(gemm<EP_GELU_GRAD>(s, B, H, H, w.d1, H, 1, W2, H, 1, w.d0, H, nullptr, nullptr, w.z1));
  CK(gemm_splitk(s, H, I, B, w.d0, 1, H, w.xb, I, 1, g + MLP_OFF_W1, w.part));
  hipLaunchKernelGGL(k_colsum, dim3(H / CS_COLS), dim3(CS_COLS * CS_GROUPS), 0, s, w.d0, B, H, g + MLP_OFF_B1);
  CK(hipGetLastError());
  const double c1 = 1.0 - std::pow((double)b1, (double)step), c2 = 1.0 - std::pow((double)b2, (double)step);
  hipLaunchKernelGGL(k_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, th, m, v, (const float *)g,
                     MLP_NPARAM, lr, b1, b2, eps, (float)c1, (float)c2);
  CK(hipGetLastError());
#undef CK
  return hipSuccess;
}

}  // namespace gs

using namespace gs;

extern "C" size_t gs_mlp_train_workspace(int32_t batch) {
  if (batch < 1) return 0;
  return ws_floats(batch) * sizeof(float);
}

extern "C" gs_status gs_mlp_train(const float *x, const float *t, int64_t n, const int32_t *order, int64_t n_order,
                                  int32_t batch, float *theta, float *adam_m, float *adam_v, int64_t step0,
                                  double lr, double beta1, double beta2, double eps, float *loss, float *grad_last,
                                  void *work, size_t work_bytes, void *hip_stream) {
  if (!x || !t || !order || !theta || !adam_m || !adam_v || !work) return GS_EINVAL;
  if (n < 1 || n_order < 0 || batch < 1 || batch > (1 << 20) || step0 < 0) return GS_EINVAL;
  if (!(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0))
    return GS_EINVAL;
  if (work_bytes < gs_mlp_train_workspace(batch)) return GS_EINVAL;
  hipStream_t s = (hipStream_t)hip_stream;
  const TrainWs w = ws_map(work, batch);
  if (hipMemsetAsync(w.bad, 0, 4, s) != hipSuccess) return GS_EDEVICE;
  const long long steps = n_order / batch;
  for (long long k = 0; k < steps; ++k) {
    if (train_step(x, t, n, order, k * batch, batch, theta, adam_m, adam_v, step0 + k + 1, (float)lr,
                   (float)beta1, (float)beta2, (float)eps, loss ? loss + k : nullptr, w, s) != hipSuccess)
      return GS_EDEVICE;
  }
  if (grad_last && steps > 0 &&
      hipMemcpyAsync(grad_last, w.grad, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return GS_EDEVICE;
  unsigned int bad = 0;
  if (hipMemcpyAsync(&bad, w.bad, 4, hipMemcpyDeviceToHost, s) != hipSuccess) return GS_EDEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return GS_EDEVICE;
  return bad ? GS_EINVAL : GS_OK;
}
