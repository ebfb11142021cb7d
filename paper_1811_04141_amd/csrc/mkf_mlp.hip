// mkf_mlp.hip -- training data, training and inference kernels of the
// learned propagation surrogate (MLP 8 -> 64 -> 64 -> 7, SiLU, BF16 weights
// and activations on the matrix cores, FP32 accumulation and master
// weights).
//
// Training: each wavefront takes 64 samples, runs the forward pass, the
// backward pass (dH = W^T dZ on MFMA with transposed weight images) and the
// weight gradients (dW = dZ H^T on MFMA with samples as the reduction
// dimension, from unit-major LDS tiles), and writes its partial gradient.
// A second kernel sums the partials in a fixed order (deterministic) and
// applies Adam to the FP32 master weights, refreshing the BF16 images.
#include <hip/hip_runtime.h>

#include "mkf_kernels.hpp"
#include "mkf_mlp.hpp"

namespace mkf {

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  // SplitMix64 (Steele, Lea, Flood 2014), used as a counter-based generator
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}
__device__ __forceinline__ float uniform01(uint64_t seed, uint64_t ctr) {
  return (float)(splitmix64(seed ^ splitmix64(ctr)) >> 40) * (1.0f / 16777216.0f);
}

// ------------------------------------------------------------ training data
//
// States on barrel layer k (uniform over the layers that have a next one) of
// tracks from the beam line: pT log-uniform 0.3-10 GeV/c, |eta| < 2.4,
// both charges, vertex z in +-5 cm, direction spread by 3 mrad; target the
// next barrel layer.  The plain propagator gives the path length l and the
// state there.  Targets, in the frame of the initial transverse direction
// d (and its left normal n), scaled by 10 / l_line:
//   y0 = 10 (l / l_line - 1) / (omega R),
//   y1, y2 = the end point's offset from the straight line along d and n,
//   y3 = its offset in z from the straight line (zero for an exact helix),
//   y4, y5 = 10 (cos, sin of the turning angle omega l) - (10, 0),
//   y6 = 0 (theta is constant in a uniform field).
// A draw that cannot reach the target layer inside |z| <= 100, or meets it
// at a path more than 1.5 times the straight line's (nearly tangent), is
// redrawn (up to 32 times; the sample is flagged invalid after that).
__global__ __launch_bounds__(256) void k_mlp_datagen(FindParams P, int64_t n, uint64_t seed,
                                                     const float *radii, int n_radii, float *x,
                                                     float *t, float *valid) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float xin[8] = {}, tout[7] = {};
  float ok = 0.f;
  for (int attempt = 0; attempt < 32 && ok == 0.f; ++attempt) {
    const uint64_t c = ((uint64_t)i * 32 + attempt) * 8;
    const int k0 = min((int)(uniform01(seed, c) * (n_radii - 1)), n_radii - 2);
    const float R0 = radii[k0], R1 = radii[k0 + 1];
    const float pt = expf(logf(0.3f) + uniform01(seed, c + 1) * (logf(10.f) - logf(0.3f)));
    const float q = uniform01(seed, c + 2) < 0.5f ? -1.f : 1.f;
    const float eta = -2.4f + 4.8f * uniform01(seed, c + 3);
    const float theta = 2.f * atanf(expf(-eta));
    const float phi_pos = -kPi + kTwoPi * uniform01(seed, c + 4);
    const float w = P.cfg.mkb * q / pt;
    if (!(fabsf(w) * R1 < 2.f)) continue;  // turns back before the target
    const float h0 = asinf(0.5f * R0 * w);   // half the turning angle from the beam line
    const float phi_dir = phi_pos + h0 + 0.003f * (2.f * uniform01(seed, c + 5) - 1.f);
    const float l0 = 2.f * h0 / w;
    const float cot = cosf(theta) / sinf(theta);
    const float z0 = -5.f + 10.f * uniform01(seed, c + 6) + l0 * cot;
    if (fabsf(z0) > 100.f) continue;
    float p[6] = {R0 * cosf(phi_pos), R0 * sinf(phi_pos), z0, q / pt, wrap_phi(phi_dir), theta};
    DevLayer L{};
    L.kind = 0;
    L.pos = R1;
    PropT<float> pr;
    // in the loaded parameterised field, if any: the network then predicts
    // the stepped crossings the find makes there
    if (propagate<false, float>(p, nullptr, L, P.cfg.mkb, P.cfg.l_min, false, 0.f, pr, 0.f,
                                nullptr, nullptr, P.cfg.field.on ? &P.cfg.field : nullptr) != kOk)
      continue;
    if (fabsf(pr.p[2]) > 100.f) continue;
    const float ll = line_path(p, R1);
    if (!(ll > 0.f) || !(pr.l <= 1.5f * ll)) continue;
    mlp_inputs(p, R1, P.cfg.mkb, xin);
    float sphi, cphi;
    sincosf(p[4], &sphi, &cphi);
    const float dx = pr.p[0] - fmaf(pr.l, cphi, p[0]);
    const float dy = pr.p[1] - fmaf(pr.l, sphi, p[1]);
    const float inv = kOutL / ll;
    float st, ct;
    sincosf(w * pr.l, &st, &ct);
    tout[0] = (pr.l / ll - 1.f) * kOutL / (w * R1);
    tout[1] = fmaf(dx, cphi, dy * sphi) * inv;
    tout[2] = fmaf(dy, cphi, -dx * sphi) * inv;
    tout[3] = (pr.p[2] - fmaf(pr.l, cot, p[2])) * inv;
    tout[4] = (ct - 1.f) * kOutL;
    tout[5] = st * kOutL;
    tout[6] = 0.f;
    ok = 1.f;
  }
  for (int k = 0; k < 8; ++k) x[i * 8 + k] = ok ? xin[k] : 0.f;
  for (int k = 0; k < 7; ++k) t[i * 7 + k] = ok ? tout[k] : 0.f;
  valid[i] = ok;
}

// ------------------------------------------------------------ gradients

struct GradParams {
  MlpWeights w;
  const float *x, *t, *valid;
  int64_t n;       // samples available
  int64_t begin;   // first sample of this batch (wraps modulo n)
  float loss_w[7];
  float inv_batch;
  float *partial;  // [waves][kNParam + 1]
};

constexpr int kLdU = 72;  // unit-major tiles: [unit][64 samples + 8]

// acc[mt][nt] = A (MT*32 x 64, unit-major LDS) . B^T (NT*32 x 64 unit-major):
// products summed over the 64 samples of the wave.
template <int MT, int NT>
__device__ __forceinline__ void gemm_uu(const __bf16 *A, const __bf16 *B, f32x16 (&acc)[MT][NT]) {
  const int lane = threadIdx.x & 63, r = lane & 31, h = lane >> 5;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[mt][nt][i] = 0.f;
#pragma unroll
  for (int kc = 0; kc < 4; ++kc) {
    bf16x8 a[MT], b[NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
      a[mt] = *reinterpret_cast<const bf16x8 *>(A + (32 * mt + r) * kLdU + 16 * kc + 8 * h);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
      b[nt] = *reinterpret_cast<const bf16x8 *>(B + (32 * nt + r) * kLdU + 16 * kc + 8 * h);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        acc[mt][nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[mt], b[nt], acc[mt][nt], 0, 0, 0);
  }
}

// write an accumulator tile set into a unit-major [unit][sample] LDS tile
template <int MT>
__device__ __forceinline__ void store_unit_major(const f32x16 (&acc)[MT][2], __bf16 *out) {
  const int lane = threadIdx.x & 63, r = lane & 31, h = lane >> 5;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int i = 0; i < 16; ++i)
        out[(32 * mt + acc_row(i, h)) * kLdU + 32 * nt + r] = (__bf16)acc[mt][nt][i];
}

__global__ __launch_bounds__(64) void k_mlp_grad(GradParams G) {
  __shared__ __attribute__((aligned(16))) __bf16 sX[64 * kLdX];
  __shared__ __attribute__((aligned(16))) __bf16 sXu[32 * kLdU];
  __shared__ __attribute__((aligned(16))) __bf16 sH1[64 * kLdH], sH1u[64 * kLdU], sH2[64 * kLdH], sH2u[64 * kLdU];
  __shared__ __attribute__((aligned(16))) __bf16 sDY[64 * kLdY], sDYu[32 * kLdU];
  __shared__ __attribute__((aligned(16))) __bf16 sDZ2[64 * kLdH], sDZ2u[64 * kLdU], sDZ1u[64 * kLdU];
  const int lane = threadIdx.x, r = lane & 31, h = lane >> 5;
  const int64_t base = G.begin + (int64_t)blockIdx.x * 64;
  const int64_t s = (base + lane) % G.n;
  // inputs, both layouts
  for (int k = 0; k < 16; ++k) sX[lane * kLdX + k] = (__bf16)(k < 8 ? G.x[s * 8 + k] : 0.f);
  for (int k = 0; k < 32; ++k) sXu[k * kLdU + lane] = (__bf16)(k < 8 ? G.x[s * 8 + k] : 0.f);
  wave_sync();
  f32x16 z1[2][2], z2[2][2];
  gemm_w_act<2, 1>(G.w.W1p, kLdW1, sX, kLdX, G.w.b1, z1);
  {
    f32x16 a[2][2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int i = 0; i < 16; ++i) a[mt][nt][i] = silu(z1[mt][nt][i]);
    store_act<2, false>(a, sH1, kLdH);
    store_unit_major<2>(a, sH1u);
  }
  wave_sync();
  gemm_w_act<2, 4>(G.w.W2p, kLdW2, sH1, kLdH, G.w.b2, z2);
  {
    f32x16 a[2][2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int i = 0; i < 16; ++i) a[mt][nt][i] = silu(z2[mt][nt][i]);
    store_act<2, false>(a, sH2, kLdH);
    store_unit_major<2>(a, sH2u);
  }
  wave_sync();
  f32x16 y[1][2];
  gemm_w_act<1, 4>(G.w.W3p, kLdW3, sH2, kLdH, G.w.b3, y);
  // output error: dL/dy = 2 w_j (y - t) / B for valid samples
  float loss = 0.f;
  f32x16 dy[1][2];
#pragma unroll
  for (int nt = 0; nt < 2; ++nt)
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int j = acc_row(i, h);
      float d = 0.f;
      if (j < kNO) {
        const int64_t sj = (base + 32 * nt + r) % G.n;
        const float vv = G.valid[sj];
        const float e = y[0][nt][i] - G.t[sj * 7 + j];
        loss += vv * G.loss_w[j] * e * e;
        d = 2.f * vv * G.loss_w[j] * e * G.inv_batch;
      }
      dy[0][nt][i] = d;
    }
  store_act<1, false>(dy, sDY, kLdY);
  store_unit_major<1>(dy, sDYu);
  wave_sync();
  // dZ2 = (W3^T dY) * silu'(z2)
  {
    f32x16 g[2][2];
    gemm_w_act<2, 2>(G.w.W3T, kLdW3T, sDY, kLdY, nullptr, g);
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int i = 0; i < 16; ++i) g[mt][nt][i] *= dsilu(z2[mt][nt][i]);
    store_act<2, false>(g, sDZ2, kLdH);
    store_unit_major<2>(g, sDZ2u);
  }
  wave_sync();
  // dZ1 = (W2^T dZ2) * silu'(z1)
  {
    f32x16 g[2][2];
    gemm_w_act<2, 4>(G.w.W2T, kLdW2, sDZ2, kLdH, nullptr, g);
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int i = 0; i < 16; ++i) g[mt][nt][i] *= dsilu(z1[mt][nt][i]);
    store_unit_major<2>(g, sDZ1u);
  }
  wave_sync();
  float *out = G.partial + (size_t)blockIdx.x * (kNParam + 1);
  // weight gradients, summed over the wave's samples on the matrix cores
  {
    f32x16 g3[1][2];
    gemm_uu<1, 2>(sDYu, sH2u, g3);
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int j = acc_row(i, h), k = 32 * nt + r;
        if (j < kNO) out[kOffW3 + j * kNH + k] = g3[0][nt][i];
      }
  }
  {
    f32x16 g2[2][2];
    gemm_uu<2, 2>(sDZ2u, sH1u, g2);
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int i = 0; i < 16; ++i)
          out[kOffW2 + (32 * mt + acc_row(i, h)) * kNH + 32 * nt + r] = g2[mt][nt][i];
  }
  {
    f32x16 g1[2][1];
    gemm_uu<2, 1>(sDZ1u, sXu, g1);
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int i = 0; i < 16; ++i)
        if (r < kNI) out[kOffW1 + (32 * mt + acc_row(i, h)) * kNI + r] = g1[mt][0][i];
  }
  // bias gradients: sums over the samples of the unit-major tiles
  {
    float b1 = 0.f, b2 = 0.f, b3 = 0.f;
    for (int q = 0; q < 64; ++q) {
      b1 += (float)sDZ1u[lane * kLdU + q];
      b2 += (float)sDZ2u[lane * kLdU + q];
      if (lane < kNO) b3 += (float)sDYu[lane * kLdU + q];
    }
    out[kOffB1 + lane] = b1;
    out[kOffB2 + lane] = b2;
    if (lane < kNO) out[kOffB3 + lane] = b3;
  }
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) loss += __shfl_xor(loss, m);
  if (lane == 0) out[kNParam] = loss * G.inv_batch;
}

// Sum the partial gradients in wave order; then either write the gradient
// (adam == 0) or take an Adam step on the FP32 master weights and refresh
// the BF16 operand images.
struct AdamParams {
  float *param, *m, *v;
  const float *partial;
  int n_waves;
  int step;  // 1-based
  float lr, b1, b2, eps;
  int adam;
  float *grad_out;  // when adam == 0
  float *loss_out;  // one float
  __bf16 *W1p, *W2p, *W3p, *W2T, *W3T;
  float *b1v, *b2v, *b3v;
};

__device__ __forceinline__ void write_images(const AdamParams &A, int p, float val) {
  const __bf16 b = (__bf16)val;
  if (p < kOffB1) {
    const int i = p / kNI, k = p % kNI;
    A.W1p[i * kLdW1 + k] = b;
  } else if (p < kOffW2) {
    A.b1v[p - kOffB1] = val;
  } else if (p < kOffB2) {
    const int i = (p - kOffW2) / kNH, k = (p - kOffW2) % kNH;
    A.W2p[i * kLdW2 + k] = b;
    A.W2T[k * kLdW2 + i] = b;
  } else if (p < kOffW3) {
    A.b2v[p - kOffB2] = val;
  } else if (p < kOffB3) {
    const int j = (p - kOffW3) / kNH, k = (p - kOffW3) % kNH;
    A.W3p[j * kLdW3 + k] = b;
    A.W3T[k * kLdW3T + j] = b;
  } else {
    A.b3v[p - kOffB3] = val;
  }
}

__global__ __launch_bounds__(256) void k_mlp_reduce(AdamParams A) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kNParam) return;
  float g = 0.f;
  for (int w = 0; w < A.n_waves; ++w) g += A.partial[(size_t)w * (kNParam + 1) + p];
  if (p == kNParam) {
    *A.loss_out = g;
    return;
  }
  if (!A.adam) {
    A.grad_out[p] = g;
    return;
  }
  const float m = A.b1 * A.m[p] + (1.f - A.b1) * g;
  const float v = A.b2 * A.v[p] + (1.f - A.b2) * g * g;
  A.m[p] = m;
  A.v[p] = v;
  const float c1 = 1.f - powf(A.b1, (float)A.step), c2 = 1.f - powf(A.b2, (float)A.step);
  const float np = A.param[p] - A.lr * (m / c1) / (sqrtf(v / c2) + A.eps);
  A.param[p] = np;
  write_images(A, p, np);
}

// First level of the partial-gradient sum for large batches: row g of out
// is the sum of partial rows g * group .. g * group + group - 1 (in order).
__global__ __launch_bounds__(256) void k_mlp_partial_sum(const float *in, int n_in, int group,
                                                         float *out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kNParam) return;
  const int g = blockIdx.y;
  const int w1 = min(n_in, (g + 1) * group);
  float acc = 0.f;
  for (int w = g * group; w < w1; ++w) acc += in[(size_t)w * (kNParam + 1) + p];
  out[(size_t)g * (kNParam + 1) + p] = acc;
}

// BF16 images of the given master weights (padding stays zero).
__global__ __launch_bounds__(256) void k_mlp_images(AdamParams A) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kNParam) return;
  write_images(A, p, A.param[p]);
}

// ------------------------------------------------------------ inference

// Forward pass of the wave's 64 samples on 32 x 32 tiles (the training
// layout): X is the sample-major input tile [64][kLdX] (k 0..7 inputs,
// 8..15 zero), H a separate [64][kLdH] scratch tile (not overlaying X).
// out[j] receives output j of the lane's own sample.
__device__ __forceinline__ void mlp_forward64(const MlpWeights &w, const __bf16 *X, __bf16 *H,
                                              float *out) {
  const int lane = threadIdx.x & 63;
  f32x16 y[1][2];
  {
    f32x16 acc[2][2];
    gemm_w_act<2, 1>(w.W1p, kLdW1, X, kLdX, w.b1, acc);
    store_act<2, true>(acc, H, kLdH);
  }
  wave_sync();
  {
    f32x16 acc[2][2];
    gemm_w_act<2, 4>(w.W2p, kLdW2, H, kLdH, w.b2, acc);
    wave_sync();  // every lane has read h1 before h2 overwrites it
    store_act<2, true>(acc, H, kLdH);
  }
  wave_sync();
  gemm_w_act<1, 4>(w.W3p, kLdW3, H, kLdH, w.b3, y);
  // output j of sample s: column s % 32 of tile s / 32, row j (rows 0..3 in
  // the lower half of the lanes, 4..6 in the upper)
#pragma unroll
  for (int j = 0; j < kNO; ++j) {
    const int src = (lane & 31) + (j < 4 ? 0 : 32);
    const float v0 = __shfl(y[0][0][j & 3], src);
    const float v1 = __shfl(y[0][1][j & 3], src);
    out[j] = lane >= 32 ? v1 : v0;
  }
}


// Inference of n samples.  Calls of at most kInferNarrow samples run 16
// samples per wavefront, four wavefronts per block, on the find's own
// inference code (mlp_forward16): less padding for small calls, and the
// entry point's tests check that code.  Larger calls run 64 samples per
// wavefront on the training layout (mlp_forward64), which loads each weight
// operand once per 64 samples.  The two accumulate in different orders, so
// their outputs may differ in the last bits.
constexpr int64_t kInferNarrow = 16384;

__global__ __launch_bounds__(256) void k_mlp_infer16(MlpWeights w, int64_t n, const float *x,
                                                     float *y) {
  __shared__ __attribute__((aligned(16))) __bf16 sH[4][16 * kLdH];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t s0 = ((int64_t)blockIdx.x * 4 + wv) * 16;  // the wave's first sample
  __bf16 *H = sH[wv];
  __bf16 *X = H;  // the input tile overlays the activation tile
  {
    // 16 samples x 8 inputs, two consecutive inputs per lane
    const int r = lane >> 2, k = 2 * (lane & 3);
    const int64_t s = s0 + r;
    const float a = s < n ? x[s * 8 + k] : 0.f;
    const float b = s < n ? x[s * 8 + k + 1] : 0.f;
    X[r * kLdX + k] = (__bf16)a;
    X[r * kLdX + k + 1] = (__bf16)b;
  }
  wave_sync();
  f32x4 yt;
  mlp_forward16(w, X, H, yt);
  // lane (h, r) holds outputs 4h .. 4h + 3 of sample r
  const int r = lane & 15, h = lane >> 4;
  const int64_t s = s0 + r;
  if (h < 2 && s < n)
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (4 * h + i < kNO) y[s * 7 + 4 * h + i] = yt[i];
}

__global__ __launch_bounds__(256) void k_mlp_infer64(MlpWeights w, int64_t n, const float *x,
                                                     float *y) {
  __shared__ __attribute__((aligned(16))) __bf16 sX[4][64 * kLdX];
  __shared__ __attribute__((aligned(16))) __bf16 sH[4][64 * kLdH];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool valid = s < n;
  for (int k = 0; k < 16; ++k)
    sX[wv][lane * kLdX + k] = (__bf16)((valid && k < 8) ? x[s * 8 + k] : 0.f);
  wave_sync();
  float out[kNO];
  mlp_forward64(w, sX[wv], sH[wv], out);
  if (valid)
    for (int j = 0; j < kNO; ++j) y[s * 7 + j] = out[j];
}

// ------------------------------------------------------------ launchers

void launch_mlp_datagen(hipStream_t s, const FindParams &P, int64_t n, uint64_t seed,
                        const float *radii, int n_radii, float *x, float *t, float *valid) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_mlp_datagen, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, P, n, seed,
                     radii, n_radii, x, t, valid);
}

void launch_mlp_grad(hipStream_t s, const MlpWeights &w, const float *x, const float *t,
                     const float *valid, int64_t n, int64_t begin, int batch, const float *loss_w,
                     float *partial) {
  GradParams G{};
  G.w = w;
  G.x = x;
  G.t = t;
  G.valid = valid;
  G.n = n;
  G.begin = begin;
  for (int j = 0; j < 7; ++j) G.loss_w[j] = loss_w[j];
  G.inv_batch = 1.f / (float)batch;
  G.partial = partial;
  hipLaunchKernelGGL(k_mlp_grad, dim3(batch / 64), dim3(64), 0, s, G);
}

void launch_mlp_reduce(hipStream_t s, const MlpBuffers &B, const float *partial, int n_waves,
                       int step, float lr, int adam, float *grad_out, float *loss_out,
                       float *scratch) {
  if (n_waves > kReduceGroup) {  // two levels, both in a fixed order
    const int n1 = (n_waves + kReduceGroup - 1) / kReduceGroup;
    hipLaunchKernelGGL(k_mlp_partial_sum, dim3((kNParam + 1 + 255) / 256, n1), dim3(256), 0, s,
                       partial, n_waves, kReduceGroup, scratch);
    partial = scratch;
    n_waves = n1;
  }
  AdamParams A{};
  A.param = B.param;
  A.m = B.m;
  A.v = B.v;
  A.partial = partial;
  A.n_waves = n_waves;
  A.step = step;
  A.lr = lr;
  A.b1 = 0.9f;
  A.b2 = 0.999f;
  A.eps = 1e-8f;
  A.adam = adam;
  A.grad_out = grad_out;
  A.loss_out = loss_out;
  A.W1p = B.W1p;
  A.W2p = B.W2p;
  A.W3p = B.W3p;
  A.W2T = B.W2T;
  A.W3T = B.W3T;
  A.b1v = B.b1;
  A.b2v = B.b2;
  A.b3v = B.b3;
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kNParam + 1 + 255) / 256), dim3(256), 0, s, A);
}

void launch_mlp_images(hipStream_t s, const MlpBuffers &B) {
  AdamParams A{};
  A.param = B.param;
  A.W1p = B.W1p;
  A.W2p = B.W2p;
  A.W3p = B.W3p;
  A.W2T = B.W2T;
  A.W3T = B.W3T;
  A.b1v = B.b1;
  A.b2v = B.b2;
  A.b3v = B.b3;
  hipLaunchKernelGGL(k_mlp_images, dim3((kNParam + 255) / 256), dim3(256), 0, s, A);
}

void launch_mlp_infer(hipStream_t s, const MlpWeights &w, int64_t n, const float *x, float *y) {
  if (n == 0) return;
  if (n <= kInferNarrow)
    hipLaunchKernelGGL(k_mlp_infer16, dim3((unsigned)((n + 63) / 64)), dim3(256), 0, s, w, n, x,
                       y);
  else
    hipLaunchKernelGGL(k_mlp_infer64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, n,
                       x, y);
}

}  // namespace mkf
