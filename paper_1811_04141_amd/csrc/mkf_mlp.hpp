// mkf_mlp.hpp -- wave-level BF16 matrix-core (MFMA) kernels of the learned
// propagation surrogate: a multilayer perceptron 8 -> 64 -> 64 -> 7 with
// SiLU activations, BF16 weights and activations, FP32 accumulation.
//
// A wavefront evaluates 64 samples at once.  Activations are staged in the
// wave's own LDS tile, sample-major ([sample][unit], rows padded by 8
// elements); each layer is a chain of v_mfma_f32_32x32x16_bf16 over
// 32 x 32 output tiles.  Operand layout of that instruction (lane l,
// r = l % 32, h = l / 32): A holds row r, k = 8h .. 8h + 7 of the 32 x 16 tile;
// B holds column r, k = 8h .. 8h + 7 of the 16 x 32 tile; accumulator
// register i holds row 8 (i / 4) + 4 h + i % 4, column r of the 32 x 32 tile.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mkf {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int kNI = 8, kNH = 64, kNO = 7;
constexpr int kNParam = kNH * kNI + kNH + kNH * kNH + kNH + kNO * kNH + kNO;  // 5191
// parameter offsets (row-major, as in the host-side parameter vector)
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kNH * kNI, kOffW2 = kOffB1 + kNH;
constexpr int kOffB2 = kOffW2 + kNH * kNH, kOffW3 = kOffB2 + kNH, kOffB3 = kOffW3 + kNO * kNH;

// padded BF16 operand images of the weights (rows x row length)
constexpr int kLdW1 = 16;   // W1p [64][16], columns 8..15 zero
constexpr int kLdW2 = 64;   // W2p [64][64] and W2T [64][64]
constexpr int kLdW3 = 64;   // W3p [32][64], rows 7..31 zero
constexpr int kLdW3T = 32;  // W3T [64][32], columns 7..31 zero
// LDS row strides (elements) of the activation tiles
constexpr int kLdX = 24;    // [64][16 + 8]
constexpr int kLdH = 72;    // [64][64 + 8]
constexpr int kLdY = 40;    // [64][32 + 8]

struct MlpWeights {
  const __bf16 *W1p, *W2p, *W3p, *W2T, *W3T;
  const float *b1, *b2, *b3;  // 64, 64, 32 (b3 zero beyond 7)
};

// input and target standardisation of the surrogate (fixed constants)
constexpr float kInR = 1.f / 70.f;  // target radius / 70 cm
constexpr float kInZ = 0.01f;       // z / 100 cm
constexpr float kInCot = 0.2f;      // cot(theta) / 5
constexpr float kInIpt = 0.3f;      // (q/pT) * 0.3 (c/GeV)^-1
constexpr float kOutL = 10.f;       // y0 = 10 (l / l_line - 1) / (omega R)

// Inputs of the surrogate for a state p = (x, y, z, q/pT, phi, theta) heading
// to the cylinder of radius R.  The transverse crossing is invariant under
// rotations about z and under scaling, so it is described by r0 / R, the
// angle alpha between the direction and the radial direction at the start
// (cos, sin) and omega R (omega = the signed curvature); R, cot(theta), z
// and q/pT complete the state for the longitudinal outputs.
__device__ __forceinline__ void mlp_inputs(const float *p, float R, float mkb, float *x) {
  float sphi, cphi;
  sincosf(p[4], &sphi, &cphi);
  float sth, cth;
  sincosf(p[5], &sth, &cth);
  const float r0 = sqrtf(fmaf(p[0], p[0], p[1] * p[1]));
  const float ir0 = r0 > 0.f ? 1.f / r0 : 0.f;
  x[0] = r0 / R;
  x[1] = r0 > 0.f ? fmaf(p[0], cphi, p[1] * sphi) * ir0 : 1.f;
  x[2] = fmaf(p[0], sphi, -p[1] * cphi) * ir0;
  x[3] = mkb * p[3] * R;
  x[4] = R * kInR;
  x[5] = cth / sth * kInCot;
  x[6] = p[2] * kInZ;
  x[7] = p[3] * kInIpt;
}

// straight-line transverse path from (x, y) along phi to the cylinder R
// (the baseline of the surrogate's relative correction)
__device__ __forceinline__ float line_path(const float *p, float R) {
  float sphi, cphi;
  sincosf(p[4], &sphi, &cphi);
  const float a = fmaf(p[0], cphi, p[1] * sphi);
  const float g0 = fmaf(p[0], p[0], fmaf(p[1], p[1], -R * R));
  return -a + sqrtf(fmaxf(fmaf(a, a, -g0), 0.f));
}

// path length predicted from the surrogate's first output: the helix path
// differs from the straight line by a relative amount of first order in
// omega R, which the network predicts divided by omega R
__device__ __forceinline__ float surrogate_path(const float *p, float R, float mkb, float y0) {
  return line_path(p, R) * fmaf(y0 * (1.f / kOutL), mkb * p[3] * R, 1.f);
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// The activations are stored as bfloat16 (8 significant bits), so the
// logistic uses the hardware exponential and reciprocal.
__device__ __forceinline__ float sigmoid(float z) {
  return __builtin_amdgcn_rcpf(1.f + __expf(-z));
}
__device__ __forceinline__ float silu(float z) { return z * sigmoid(z); }
__device__ __forceinline__ float dsilu(float z) {
  const float s = sigmoid(z);
  return s * (1.f + z * (1.f - s));
}

__device__ __forceinline__ int acc_row(int i, int h) { return 8 * (i / 4) + 4 * h + (i % 4); }

// acc[mt][nt] = bias + W (MT*32 x KC*16, row-major, ld) . act^T, where act is
// the sample-major LDS tile [32 NT][lda] (columns = units, k).
template <int MT, int KC, int NT = 2>
__device__ __forceinline__ void gemm_w_act(const __bf16 *W, int ldw, const __bf16 *act, int lda,
                                           const float *bias, f32x16 (&acc)[MT][NT]) {
  const int lane = threadIdx.x & 63, r = lane & 31, h = lane >> 5;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[mt][nt][i] = bias ? bias[32 * mt + acc_row(i, h)] : 0.f;
#pragma unroll
  for (int kc = 0; kc < KC; ++kc) {
    bf16x8 a[MT], b[NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
      a[mt] = *reinterpret_cast<const bf16x8 *>(W + (32 * mt + r) * ldw + 16 * kc + 8 * h);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
      b[nt] = *reinterpret_cast<const bf16x8 *>(act + (32 * nt + r) * lda + 16 * kc + 8 * h);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        acc[mt][nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[mt], b[nt], acc[mt][nt], 0, 0, 0);
  }
}

// Store silu(acc) (or acc itself) as BF16 into a sample-major LDS tile.
// Accumulator registers 4q .. 4q + 3 hold four consecutive units of one
// sample, written as one 8-byte store.
template <int MT, bool kSilu, int NT = 2>
__device__ __forceinline__ void store_act(const f32x16 (&acc)[MT][NT], __bf16 *out, int ldo) {
  const int lane = threadIdx.x & 63, r = lane & 31, h = lane >> 5;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        bf16x4 v;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float a = acc[mt][nt][4 * q + e];
          v[e] = (__bf16)(kSilu ? silu(a) : a);
        }
        *reinterpret_cast<bf16x4 *>(out + (32 * nt + r) * ldo + 32 * mt + acc_row(4 * q, h)) = v;
      }
}

// Forward pass of the first 32 NT samples of the wave's tiles; X is the
// sample-major input tile (k 0..7 inputs, 8..15 zero), H a [64][kLdH]
// scratch tile (X may lie inside H).  y receives the output layer's accumulators: output j of
// sample s is column s % 32 of tile s / 32, row j (see mlp_output).
template <int NT>
__device__ __forceinline__ void mlp_forward_tiles(const MlpWeights &w, const __bf16 *X, __bf16 *H,
                                                  f32x16 (&y)[1][NT]) {
  {
    f32x16 acc[2][NT];
    gemm_w_act<2, 1, NT>(w.W1p, kLdW1, X, kLdX, w.b1, acc);
    wave_sync();  // X may overlay H: every lane has read it before h1 is stored
    store_act<2, true, NT>(acc, H, kLdH);
  }
  wave_sync();
  {
    f32x16 acc[2][NT];
    gemm_w_act<2, 4, NT>(w.W2p, kLdW2, H, kLdH, w.b2, acc);
    wave_sync();  // every lane has read h1 before h2 overwrites it
    store_act<2, true, NT>(acc, H, kLdH);
  }
  wave_sync();
  gemm_w_act<1, 4, NT>(w.W3p, kLdW3, H, kLdH, w.b3, y);
}

// Output j of sample s (any lane may ask for any sample): row j < 4 is in
// half 0, register j; rows 4..6 in half 1, register j - 4.
template <int NT>
__device__ __forceinline__ float mlp_output(const f32x16 (&y)[1][NT], int s, int j) {
  const int reg = j & 3;
  const int src = (s & 31) + (j < 4 ? 0 : 32);
  float v = __shfl(y[0][0][reg], src);
  if (NT == 2) {
    const float v1 = __shfl(y[0][NT - 1][reg], src);
    v = s >= 32 ? v1 : v;
  }
  return v;
}

// Forward pass of the wave's 64 samples (sample = lane); returns the first
// output (y0) of the lane's own sample; all 7 outputs go to y_all[7] if not
// null.
__device__ __forceinline__ float mlp_forward_wave(const MlpWeights &w, const __bf16 *X, __bf16 *H,
                                                  float *y_all) {
  const int lane = threadIdx.x & 63;
  f32x16 y[1][2];
  mlp_forward_tiles<2>(w, X, H, y);
  float own[kNO];
#pragma unroll
  for (int j = 0; j < kNO; ++j) own[j] = mlp_output<2>(y, lane, j);
  if (y_all)
#pragma unroll
    for (int j = 0; j < kNO; ++j) y_all[j] = own[j];
  return own[0];
}

}  // namespace mkf
