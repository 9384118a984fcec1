// Device side of the Newton guess network: 48 -> 128 -> 128 -> 128 -> 3, GELU
// hidden layers, linear output; weights in bfloat16, products and sums in
// binary32.  One workgroup evaluates one input vector; every (output, part)
// partial sum has a fixed owner and a fixed order, and the eight parts of an
// output are combined by the same butterfly, so the result does not depend on
// the workgroup size.
#ifndef GS_MLP_DEV_H
#define GS_MLP_DEV_H

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gs {

constexpr int MLP_IN = 48;
constexpr int MLP_H = 128;
constexpr int MLP_OUT = 3;
constexpr int MLP_NPARAM = 39683;
// flat layout: W1[128][48] b1 W2[128][128] b2 W3[128][128] b3 W4[3][128] b4
constexpr int MLP_OFF_W1 = 0;
constexpr int MLP_OFF_B1 = MLP_OFF_W1 + MLP_H * MLP_IN;
constexpr int MLP_OFF_W2 = MLP_OFF_B1 + MLP_H;
constexpr int MLP_OFF_B2 = MLP_OFF_W2 + MLP_H * MLP_H;
constexpr int MLP_OFF_W3 = MLP_OFF_B2 + MLP_H;
constexpr int MLP_OFF_B3 = MLP_OFF_W3 + MLP_H * MLP_H;
constexpr int MLP_OFF_W4 = MLP_OFF_B3 + MLP_H;
constexpr int MLP_OFF_B4 = MLP_OFF_W4 + MLP_OUT * MLP_H;
static_assert(MLP_OFF_B4 + MLP_OUT == MLP_NPARAM, "layout");
// normalisation block (binary64): x_mean[48] x_scale[48] y_mean[3] y_scale[3]
constexpr int MLP_NORM = 2 * MLP_IN + 2 * MLP_OUT;

__device__ inline float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ inline float gelu_f32(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

// out[j] = act(b[j] + sum_i W[j][i] in[i]); in and out in LDS.  Eight parts per
// output, part p summing inputs [p n_in/8, (p+1) n_in/8) in order.
__device__ inline void mlp_layer(const uint16_t *W, const uint16_t *b, const float *in, int n_in, float *out,
                                 int n_out, bool act) {
  const int chunk = n_in / 8;
  for (int q = threadIdx.x; q < n_out * 8; q += blockDim.x) {
    const int j = q >> 3, part = q & 7;
    const uint16_t *w = W + (size_t)j * n_in + part * chunk;
    const float *x = in + part * chunk;
    float s = 0.0f;
    for (int i = 0; i < chunk; ++i) s += bf16_to_f32(w[i]) * x[i];
    s += __shfl_xor(s, 4, 64);
    s += __shfl_xor(s, 2, 64);
    s += __shfl_xor(s, 1, 64);
    if (part == 0) {
      const float z = s + bf16_to_f32(b[j]);
      out[j] = act ? gelu_f32(z) : z;
    }
  }
  __syncthreads();
}

// y = net(x): x[48] in LDS (already normalised), h0/h1 scratch of 128 floats
// in LDS, y[3] in LDS.  Every thread of the workgroup calls it.
__device__ inline void mlp_eval_block(const uint16_t *W, const float *x, float *h0, float *h1, float *y) {
  __syncthreads();
  mlp_layer(W + MLP_OFF_W1, W + MLP_OFF_B1, x, MLP_IN, h0, MLP_H, true);
  mlp_layer(W + MLP_OFF_W2, W + MLP_OFF_B2, h0, MLP_H, h1, MLP_H, true);
  mlp_layer(W + MLP_OFF_W3, W + MLP_OFF_B3, h1, MLP_H, h0, MLP_H, true);
  mlp_layer(W + MLP_OFF_W4, W + MLP_OFF_B4, h0, MLP_H, y, MLP_OUT, false);
}

}  // namespace gs
#endif
