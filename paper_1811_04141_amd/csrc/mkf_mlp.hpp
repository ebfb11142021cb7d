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

__device__ __forceinline__ float silu(float z) { return z / (1.f + __expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
  const float s = 1.f / (1.f + __expf(-z));
  return s * (1.f + z * (1.f - s));
}

__device__ __forceinline__ int acc_row(int i, int h) { return 8 * (i / 4) + 4 * h + (i % 4); }

// acc[mt][nt] = bias + W (MT*32 x KC*16, row-major, ld) . act^T, where act is
// the sample-major LDS tile [64][lda] (columns = units, k).
template <int MT, int KC>
__device__ __forceinline__ void gemm_w_act(const __bf16 *W, int ldw, const __bf16 *act, int lda,
                                           const float *bias, f32x16 (&acc)[MT][2]) {
  const int lane = threadIdx.x & 63, r = lane & 31, h = lane >> 5;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[mt][nt][i] = bias ? bias[32 * mt + acc_row(i, h)] : 0.f;
#pragma unroll
  for (int kc = 0; kc < KC; ++kc) {
    bf16x8 a[MT], b[2];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
      a[mt] = *reinterpret_cast<const bf16x8 *>(W + (32 * mt + r) * ldw + 16 * kc + 8 * h);
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
      b[nt] = *reinterpret_cast<const bf16x8 *>(act + (32 * nt + r) * lda + 16 * kc + 8 * h);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
        acc[mt][nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[mt], b[nt], acc[mt][nt], 0, 0, 0);
  }
}

// Store silu(acc) (or acc itself) as BF16 into a sample-major LDS tile.
template <int MT, bool kSilu>
__device__ __forceinline__ void store_act(const f32x16 (&acc)[MT][2], __bf16 *out, int ldo) {
  const int lane = threadIdx.x & 63, r = lane & 31, h = lane >> 5;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const float v = kSilu ? silu(acc[mt][nt][i]) : acc[mt][nt][i];
        out[(32 * nt + r) * ldo + 32 * mt + acc_row(i, h)] = (__bf16)v;
      }
}

// Forward pass of the wave's 64 samples; X is the sample-major input tile
// (k 0..7 inputs, 8..15 zero), H a [64][kLdH] scratch tile.  Returns the
// first output (y0) of the lane's own sample; all 7 outputs go to y[7] if
// not null (this lane's sample).
__device__ __forceinline__ float mlp_forward_wave(const MlpWeights &w, const __bf16 *X, __bf16 *H,
                                                  float *y_all) {
  const int lane = threadIdx.x & 63, h = lane >> 5;
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
  f32x16 acc[1][2];
  gemm_w_act<1, 4>(w.W3p, kLdW3, H, kLdH, w.b3, acc);
  // row j < 4: half 0, register j; rows 4..6: half 1, register j - 4.
  // This lane's sample (lane) is column lane % 32 of sample tile lane / 32.
  float own[kNO];
#pragma unroll
  for (int j = 0; j < kNO; ++j) {
    const int reg = j & 3;
    const int src = (lane & 31) + (j < 4 ? 0 : 32);
    const float t0 = __shfl(acc[0][0][reg], src);
    const float t1 = __shfl(acc[0][1][reg], src);
    own[j] = h ? t1 : t0;
  }
  if (y_all)
#pragma unroll
    for (int j = 0; j < kNO; ++j) y_all[j] = own[j];
  return own[0];
}

}  // namespace mkf
