/*
 * CPU oracle for the guess network of the strict-coupling Newton solve.
 *
 * TEST INFRASTRUCTURE ONLY (same rules as oracle.c: loaded by the tests, the
 * smoke check and the CPU-baseline leg of the benchmark, never by the product
 * path; no source shared with the GPU library).
 *
 * The paper solves the strict step directly; a learned initial guess for the
 * Newton form of that step (gap voltage and loop currents) is an extension of
 * this implementation, so nothing here is cited to the paper.  The pieces are
 * textbook definitions, written out plainly in binary64:
 *   - fully connected layers y = W x + b, W stored row-major [out][in];
 *   - GELU(z) = z * Phi(z) with Phi the standard normal distribution function
 *     (Hendrycks and Gimpel, 2016), exact (erf) form;
 *   - loss = mean over samples and outputs of (y - t)^2;
 *   - gradients by the chain rule, layer by layer (reverse mode);
 *   - Adam (Kingma and Ba, 2015, Algorithm 1) with bias-corrected moments;
 *   - rounding of binary32 to bfloat16 (the upper 16 bits), to nearest, ties
 *     to even.
 * Layer sizes 48 -> 128 -> 128 -> 128 -> 3; parameters in one flat array:
 *   W1[128][48] b1[128] W2[128][128] b2[128] W3[128][128] b3[128] W4[3][128] b4[3]
 * (39683 values).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define NI OR_MLP_IN
#define NH OR_MLP_HIDDEN
#define NO OR_MLP_OUT

static const int64_t OFF_W1 = 0;
static const int64_t OFF_B1 = (int64_t)NH * NI;
static const int64_t OFF_W2 = (int64_t)NH * NI + NH;
static const int64_t OFF_B2 = (int64_t)NH * NI + NH + (int64_t)NH * NH;
static const int64_t OFF_W3 = (int64_t)NH * NI + 2 * NH + (int64_t)NH * NH;
static const int64_t OFF_B3 = (int64_t)NH * NI + 2 * NH + 2 * (int64_t)NH * NH;
static const int64_t OFF_W4 = (int64_t)NH * NI + 3 * NH + 2 * (int64_t)NH * NH;
static const int64_t OFF_B4 = (int64_t)NH * NI + 3 * NH + 2 * (int64_t)NH * NH + (int64_t)NO * NH;

double or_gelu(double z) { return 0.5 * z * (1.0 + erf(z / sqrt(2.0))); }

/* d/dz [z Phi(z)] = Phi(z) + z phi(z) */
double or_gelu_grad(double z) {
  const double Phi = 0.5 * (1.0 + erf(z / sqrt(2.0)));
  const double phi = exp(-0.5 * z * z) / sqrt(2.0 * M_PI);
  return Phi + z * phi;
}

/* out[j] = b[j] + sum_i W[j][i] in[i] */
static void dense(const double *W, const double *b, const double *in, int n_in, int n_out, double *out) {
  for (int j = 0; j < n_out; ++j) {
    double s = b[j];
    for (int i = 0; i < n_in; ++i) s += W[(int64_t)j * n_in + i] * in[i];
    out[j] = s;
  }
}

/* forward pass of one sample, keeping pre-activations z1..z3 and activations a1..a3 */
static void forward1(const double *th, const double *x, double *z1, double *a1, double *z2, double *a2,
                     double *z3, double *a3, double *y) {
  dense(th + OFF_W1, th + OFF_B1, x, NI, NH, z1);
  for (int j = 0; j < NH; ++j) a1[j] = or_gelu(z1[j]);
  dense(th + OFF_W2, th + OFF_B2, a1, NH, NH, z2);
  for (int j = 0; j < NH; ++j) a2[j] = or_gelu(z2[j]);
  dense(th + OFF_W3, th + OFF_B3, a2, NH, NH, z3);
  for (int j = 0; j < NH; ++j) a3[j] = or_gelu(z3[j]);
  dense(th + OFF_W4, th + OFF_B4, a3, NH, NO, y);
}

void or_mlp_forward(const double *theta, const double *x, int64_t n, double *y) {
  double z1[NH], a1[NH], z2[NH], a2[NH], z3[NH], a3[NH];
  for (int64_t s = 0; s < n; ++s)
    forward1(theta, x + s * NI, z1, a1, z2, a2, z3, a3, y + s * NO);
}

/* Reverse mode through one dense layer: given dout = dL/dout, accumulate
 * dL/dW += dout (x) in, dL/db += dout, and return din = W^T dout. */
static void dense_back(const double *W, const double *in, const double *dout, int n_in, int n_out, double *dW,
                       double *db, double *din) {
  for (int j = 0; j < n_out; ++j) {
    db[j] += dout[j];
    for (int i = 0; i < n_in; ++i) dW[(int64_t)j * n_in + i] += dout[j] * in[i];
  }
  if (din) {
    for (int i = 0; i < n_in; ++i) {
      double s = 0.0;
      for (int j = 0; j < n_out; ++j) s += W[(int64_t)j * n_in + i] * dout[j];
      din[i] = s;
    }
  }
}

double or_mlp_loss_grad(const double *theta, const double *x, const double *t, int64_t n, double *grad) {
  double z1[NH], a1[NH], z2[NH], a2[NH], z3[NH], a3[NH], y[NO];
  double dy[NO], da3[NH], dz3[NH], da2[NH], dz2[NH], da1[NH], dz1[NH];
  if (grad) memset(grad, 0, sizeof(double) * OR_MLP_NPARAM);
  double loss = 0.0;
  const double inv = 1.0 / ((double)n * NO);
  for (int64_t s = 0; s < n; ++s) {
    const double *xs = x + s * NI;
    forward1(theta, xs, z1, a1, z2, a2, z3, a3, y);
    for (int o = 0; o < NO; ++o) {
      const double e = y[o] - t[s * NO + o];
      loss += e * e * inv;
      dy[o] = 2.0 * e * inv;
    }
    if (!grad) continue;
    dense_back(theta + OFF_W4, a3, dy, NH, NO, grad + OFF_W4, grad + OFF_B4, da3);
    for (int j = 0; j < NH; ++j) dz3[j] = da3[j] * or_gelu_grad(z3[j]);
    dense_back(theta + OFF_W3, a2, dz3, NH, NH, grad + OFF_W3, grad + OFF_B3, da2);
    for (int j = 0; j < NH; ++j) dz2[j] = da2[j] * or_gelu_grad(z2[j]);
    dense_back(theta + OFF_W2, a1, dz2, NH, NH, grad + OFF_W2, grad + OFF_B2, da1);
    for (int j = 0; j < NH; ++j) dz1[j] = da1[j] * or_gelu_grad(z1[j]);
    dense_back(theta + OFF_W1, xs, dz1, NI, NH, grad + OFF_W1, grad + OFF_B1, NULL);
  }
  return loss;
}

/* Adam, step number t >= 1 */
void or_adam_step(double *theta, double *m, double *v, int64_t t, const double *g, int64_t np, double lr,
                  double beta1, double beta2, double eps) {
  const double c1 = 1.0 - pow(beta1, (double)t), c2 = 1.0 - pow(beta2, (double)t);
  for (int64_t i = 0; i < np; ++i) {
    m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
    v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
    const double mh = m[i] / c1, vh = v[i] / c2;
    theta[i] -= lr * mh / (sqrt(vh) + eps);
  }
}

/* binary32 -> bfloat16 (kept in a binary32), round to nearest, ties to even */
float or_round_bf16(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) {
    u |= 0x00400000u; /* NaN stays NaN (quiet) */
  } else {
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
  }
  u &= 0xFFFF0000u;
  float r;
  memcpy(&r, &u, 4);
  return r;
}
