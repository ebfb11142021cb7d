// mkf_mlp.hpp -- wave-level BF16 matrix-core (MFMA) kernels of the learned
// propagation surrogate: a multilayer perceptron 8 -> 64 -> 64 -> 7 with
// SiLU activations, BF16 weights and activations, FP32 accumulation.
//
// Activations are staged in the wave's own LDS tile, sample-major
// ([sample][unit], rows padded by 8 elements).
//
// Training (64 samples per wavefront) chains v_mfma_f32_32x32x16_bf16 over
// 32 x 32 output tiles.  Operand layout of that instruction (lane l,
// r = l % 32, h = l / 32): A holds row r, k = 8h .. 8h + 7 of the 32 x 16 tile;
// B holds column r, k = 8h .. 8h + 7 of the 16 x 32 tile; accumulator
// register i holds row 8 (i / 4) + 4 h + i % 4, column r of the 32 x 32 tile.
//
// Inference runs on 16-sample tiles of v_mfma_f32_16x16x32_bf16 (lane l,
// r = l % 16, h = l / 16): A holds row r, k = 8h .. 8h + 7 of the 16 x 32
// tile; B holds column r, the same k; accumulator register i holds row
// 4h + i, column r.  The find asks for at most 10 samples per wavefront at
// a time, so the narrower tile halves the activations each lane evaluates.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mkf {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

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
// trig: sin phi, cos phi, sin theta, cos theta of p, already at hand.
__device__ __forceinline__ void mlp_inputs(const float *p, const float *trig, float R, float mkb,
                                           float *x) {
  const float sphi = trig[0], cphi = trig[1], sth = trig[2], cth = trig[3];
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

__device__ __forceinline__ void mlp_inputs(const float *p, float R, float mkb, float *x) {
  float trig[4];
  sincosf(p[4], &trig[0], &trig[1]);
  sincosf(p[5], &trig[2], &trig[3]);
  mlp_inputs(p, trig, R, mkb, x);
}

// straight-line transverse path from (x, y) along phi to the cylinder R
// (the baseline of the surrogate's relative correction)
__device__ __forceinline__ float line_path(const float *p, float sphi, float cphi, float R) {
  const float a = fmaf(p[0], cphi, p[1] * sphi);
  const float g0 = fmaf(p[0], p[0], fmaf(p[1], p[1], -R * R));
  return -a + sqrtf(fmaxf(fmaf(a, a, -g0), 0.f));
}
__device__ __forceinline__ float line_path(const float *p, float R) {
  float sphi, cphi;
  sincosf(p[4], &sphi, &cphi);
  return line_path(p, sphi, cphi, R);
}

// path length predicted from the surrogate's first output: the helix path
// differs from the straight line by a relative amount of first order in
// omega R, which the network predicts divided by omega R (trig as in
// mlp_inputs)
__device__ __forceinline__ float surrogate_path(const float *p, const float *trig, float R,
                                                float mkb, float y0) {
  return line_path(p, trig[0], trig[1], R) * fmaf(y0 * (1.f / kOutL), mkb * p[3] * R, 1.f);
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
// the sample-major LDS tile [64][lda] (columns = units, k).
template <int MT, int KC>
__device__ __forceinline__ void gemm_w_act(const __bf16 *W, int ldw, const __bf16 *act, int lda,
                                           const float *bias, f32x16 (&acc)[MT][2]) {
  constexpr int NT = 2;
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
template <int MT, bool kSilu>
__device__ __forceinline__ void store_act(const f32x16 (&acc)[MT][2], __bf16 *out, int ldo) {
  constexpr int NT = 2;
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

// bias + W . act^T for the four 16-unit row tiles of a 64-unit layer with
// K = 32 KC (16-sample tile, layout above).
template <int KC>
__device__ __forceinline__ void gemm16(const __bf16 *W, int ldw, const __bf16 *act, int lda,
                                       const float *bias, f32x4 (&acc)[4]) {
  const int lane = threadIdx.x & 63, r = lane & 15, h = lane >> 4;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[mt][i] = bias[16 * mt + 4 * h + i];
#pragma unroll
  for (int kc = 0; kc < KC; ++kc) {
    const bf16x8 b = *reinterpret_cast<const bf16x8 *>(act + r * lda + 32 * kc + 8 * h);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      const bf16x8 a = *reinterpret_cast<const bf16x8 *>(W + (16 * mt + r) * ldw + 32 * kc + 8 * h);
      acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[mt], 0, 0, 0);
    }
  }
}

// silu(acc) as BF16 into the sample-major tile: registers 0..3 of a lane
// are four consecutive units of one sample, one 8-byte store per row tile.
__device__ __forceinline__ void store16_silu(const f32x4 (&acc)[4], __bf16 *out, int ldo) {
  const int lane = threadIdx.x & 63, r = lane & 15, h = lane >> 4;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    bf16x4 v;
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = (__bf16)silu(acc[mt][e]);
    *reinterpret_cast<bf16x4 *>(out + r * ldo + 16 * mt + 4 * h) = v;
  }
}

// Forward pass of 16 samples: X is the sample-major input tile [16][kLdX]
// (k 0..7 the inputs), H a [16][kLdH] scratch tile (X may lie inside H).
// Sample columns are independent, so rows of X that hold no sample may hold
// anything.  y: output j of sample s is register j % 4 of lane s + 16 (j / 4)
// (mlp_output16).
__device__ __forceinline__ void mlp_forward16(const MlpWeights &w, const __bf16 *X, __bf16 *H,
                                              f32x4 &y) {
  const int lane = threadIdx.x & 63, r = lane & 15, h = lane >> 4;
  {
    // first layer: K = 8 inputs, padded to the instruction's 32 with zeros
    // in the lanes of k >= 8 (both operands, so padding cannot meet a NaN)
    f32x4 acc[4];
    const bf16x8 zero = {};
    const bf16x8 b = h == 0 ? *reinterpret_cast<const bf16x8 *>(X + r * kLdX) : zero;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[mt][i] = w.b1[16 * mt + 4 * h + i];
      const bf16x8 a =
          h == 0 ? *reinterpret_cast<const bf16x8 *>(w.W1p + (16 * mt + r) * kLdW1) : zero;
      acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[mt], 0, 0, 0);
    }
    wave_sync();  // X may overlay H: every lane has read it before h1 is stored
    store16_silu(acc, H, kLdH);
  }
  wave_sync();
  {
    f32x4 acc[4];
    gemm16<2>(w.W2p, kLdW2, H, kLdH, w.b2, acc);
    wave_sync();  // every lane has read h1 before h2 overwrites it
    store16_silu(acc, H, kLdH);
  }
  wave_sync();
  // output layer: rows 0..15 of the padded W3p (7 outputs, the rest zero)
#pragma unroll
  for (int i = 0; i < 4; ++i) y[i] = w.b3[4 * h + i];
#pragma unroll
  for (int kc = 0; kc < 2; ++kc) {
    const bf16x8 b = *reinterpret_cast<const bf16x8 *>(H + r * kLdH + 32 * kc + 8 * h);
    const bf16x8 a = *reinterpret_cast<const bf16x8 *>(w.W3p + r * kLdW3 + 32 * kc + 8 * h);
    y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, y, 0, 0, 0);
  }
}

// Output j of sample s of mlp_forward16 (any lane may ask for any sample).
__device__ __forceinline__ float mlp_output16(const f32x4 &y, int s, int j) {
  return __shfl(y[j & 3], (s & 15) + 16 * (j >> 2));
}

}  // namespace mkf
