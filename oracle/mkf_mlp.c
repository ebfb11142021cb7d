/*
 * mkf_mlp.c -- TEST INFRASTRUCTURE ONLY: FP64 reference of the learned
 * propagation surrogate (a multilayer perceptron 8 -> 64 -> 64 -> 7 with
 * SiLU activations), its loss gradient and the Adam step.  Only the tests
 * use it; the GPU library has its own kernels.
 *
 * Parameters, in this order (5,191 values):
 *   W1[64][8], b1[64], W2[64][64], b2[64], W3[7][64], b3[7].
 * Forward: z1 = W1 x + b1, h1 = silu(z1), z2 = W2 h1 + b2, h2 = silu(z2),
 * y = W3 h2 + b3, with silu(z) = z / (1 + exp(-z)).
 * Loss over a batch of B samples: L = (1/B) sum_s sum_j w_j (y_sj - t_sj)^2.
 * Adam (Kingma & Ba 2015): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
 *
 * round_bf16 != 0 rounds x, h1 and h2 to bfloat16 (round to nearest even)
 * before each product, as the GPU's matrix cores consume them; everything
 * else stays FP64.
 */
#define _USE_MATH_DEFINES
#include <math.h>
#include <stdint.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define NI 8
#define NH 64
#define NO 7
#define NPARAM (NH * NI + NH + NH * NH + NH + NO * NH + NO)

static double silu(double z) { return z / (1.0 + exp(-z)); }
static double dsilu(double z) {
  double s = 1.0 / (1.0 + exp(-z));
  return s * (1.0 + z * (1.0 - s));
}

static double bf16(double v) {
  float f = (float)v;
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) != 0x7f800000u) {
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
  }
  u &= 0xffff0000u;
  memcpy(&f, &u, 4);
  return (double)f;
}

int orc_mlp_nparam(void) { return NPARAM; }

/* y[B][NO] for x[B][NI] */
void orc_mlp_forward(const double *p, int B, const double *x, int round_bf16, double *y) {
  const double *W1 = p, *b1 = W1 + NH * NI, *W2 = b1 + NH, *b2 = W2 + NH * NH;
  const double *W3 = b2 + NH, *b3 = W3 + NO * NH;
  for (int s = 0; s < B; ++s) {
    double xi[NI], h1[NH], h2[NH];
    for (int k = 0; k < NI; ++k) xi[k] = round_bf16 ? bf16(x[s * NI + k]) : x[s * NI + k];
    for (int i = 0; i < NH; ++i) {
      double z = b1[i];
      for (int k = 0; k < NI; ++k) z += W1[i * NI + k] * xi[k];
      h1[i] = round_bf16 ? bf16(silu(z)) : silu(z);
    }
    for (int i = 0; i < NH; ++i) {
      double z = b2[i];
      for (int k = 0; k < NH; ++k) z += W2[i * NH + k] * h1[k];
      h2[i] = round_bf16 ? bf16(silu(z)) : silu(z);
    }
    for (int j = 0; j < NO; ++j) {
      double z = b3[j];
      for (int k = 0; k < NH; ++k) z += W3[j * NH + k] * h2[k];
      y[s * NO + j] = z;
    }
  }
}

/* loss and its gradient g[NPARAM] (backpropagation, written out) */
double orc_mlp_grad(const double *p, int B, const double *x, const double *t,
                    const double *w, int round_bf16, double *g) {
  const double *W1 = p, *b1 = W1 + NH * NI, *W2 = b1 + NH, *b2 = W2 + NH * NH;
  const double *W3 = b2 + NH, *b3 = W3 + NO * NH;
  double *gW1 = g, *gb1 = gW1 + NH * NI, *gW2 = gb1 + NH, *gb2 = gW2 + NH * NH;
  double *gW3 = gb2 + NH, *gb3 = gW3 + NO * NH;
  memset(g, 0, sizeof(double) * NPARAM);
  double L = 0.0;
  for (int s = 0; s < B; ++s) {
    double xi[NI], z1[NH], h1[NH], z2[NH], h2[NH], y[NO], dy[NO], dh2[NH], dz2[NH], dh1[NH],
        dz1[NH];
    for (int k = 0; k < NI; ++k) xi[k] = round_bf16 ? bf16(x[s * NI + k]) : x[s * NI + k];
    for (int i = 0; i < NH; ++i) {
      z1[i] = b1[i];
      for (int k = 0; k < NI; ++k) z1[i] += W1[i * NI + k] * xi[k];
      h1[i] = round_bf16 ? bf16(silu(z1[i])) : silu(z1[i]);
    }
    for (int i = 0; i < NH; ++i) {
      z2[i] = b2[i];
      for (int k = 0; k < NH; ++k) z2[i] += W2[i * NH + k] * h1[k];
      h2[i] = round_bf16 ? bf16(silu(z2[i])) : silu(z2[i]);
    }
    for (int j = 0; j < NO; ++j) {
      y[j] = b3[j];
      for (int k = 0; k < NH; ++k) y[j] += W3[j * NH + k] * h2[k];
      const double d = y[j] - t[s * NO + j];
      L += w[j] * d * d / B;
      dy[j] = 2.0 * w[j] * d / B;
    }
    for (int k = 0; k < NH; ++k) {
      dh2[k] = 0.0;
      for (int j = 0; j < NO; ++j) {
        gW3[j * NH + k] += dy[j] * h2[k];
        dh2[k] += W3[j * NH + k] * dy[j];
      }
    }
    for (int j = 0; j < NO; ++j) gb3[j] += dy[j];
    for (int i = 0; i < NH; ++i) dz2[i] = dh2[i] * dsilu(z2[i]);
    for (int k = 0; k < NH; ++k) {
      dh1[k] = 0.0;
      for (int i = 0; i < NH; ++i) {
        gW2[i * NH + k] += dz2[i] * h1[k];
        dh1[k] += W2[i * NH + k] * dz2[i];
      }
    }
    for (int i = 0; i < NH; ++i) gb2[i] += dz2[i];
    for (int i = 0; i < NH; ++i) dz1[i] = dh1[i] * dsilu(z1[i]);
    for (int i = 0; i < NH; ++i) {
      for (int k = 0; k < NI; ++k) gW1[i * NI + k] += dz1[i] * xi[k];
      gb1[i] += dz1[i];
    }
  }
  return L;
}

void orc_adam(double *p, double *m, double *v, const double *g, int n, int t, double lr,
              double b1, double b2, double eps) {
  const double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
  for (int i = 0; i < n; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    p[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
  }
}

/* Step size of step s (0-based) of an n_steps-step training schedule: a
 * half cosine from lr at the first step down to lr_min = lr / 100 at the
 * last (lr for a one-step schedule).  The training recipe is a reading: the
 * paper does not train a network. */
double orc_lr_cosine(double lr, int n_steps, int s) {
  const double lr_min = 0.01 * lr;
  const double u = n_steps > 1 ? (double)s / (double)(n_steps - 1) : 0.0;
  return lr_min + 0.5 * (lr - lr_min) * (1.0 + cos(M_PI * u));
}
