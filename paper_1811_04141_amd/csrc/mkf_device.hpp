// mkf_device.hpp -- per-lane track-state algebra for gfx950 (FP32 for the
// find and the fit, FP64 for the seed fit).
//
// One candidate per lane: the 6-parameter helix state p = (x, y, z, q/pT,
// phi, theta) and the 21 upper-triangle entries of its covariance live in
// VGPRs.  None of this is a dense contraction (6x6 with a sparse Jacobian,
// 2x2 measurement algebra), so it is written as straight-line VALU code with
// the sparsity unrolled by hand; MFMA would waste its tiles here.
//
// Method (arXiv:1811.04141): barrel and endcap propagation and KF update
// (Introduction, the paragraph on realistic geometries), constant field and
// scattering material (Section 2.1), the Kalman filter of the Introduction.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mkf {

constexpr float kPi = 3.14159265358979f;
constexpr float kTwoPi = 6.28318530717959f;
constexpr int kMaxLayers = 32;
constexpr int kMaxPlan = 32;
constexpr int kGroup = 8;  // lanes per seed (candidate slots)

enum : int { kOk = 0, kNoCrossing = 1, kOutOfExtent = 2 };

// Layer as the kernels see it (staged in LDS).
struct DevLayer {
  int kind;         // 0 barrel, 1 disk
  float pos;        // R or Z
  float lo, hi;     // extent (z for barrel, r for disk)
  float vu_max, vv_max;
  int nphi, nq;
  int bin_base;     // first bin of this layer within one event's bins
  float q_lo;       // q bin = floor((q - q_lo) * q_scale)
  float q_scale;
  float phi_scale;  // nphi / (2 pi)
  float cs, sn;     // cos, sin of the stereo angle
  float hole_lo, hole_hi;  // no sensors for hole_lo < q < hole_hi
};

// Material map in r-z: per bin (x/X0, xi in g/cm^2) at normal incidence.
struct DevMat {
  const float2 *tab;  // [nz][nr]; nullptr: constant scattering angle
  int nr, nz;
  float r_scale;      // nr / r_max
  float z_max;
  float z_scale;      // nz / (2 z_max)
  float mass;
  float k_max;
};

// Parameterised axial field: omega = kb0 (1 + c_r2 r^2 + c_z2 z^2 +
// c_z4 z^4) (q/pT), kb0 = -kappa b0; Runge-Kutta steps of at most h_max.
struct DevField {
  int on;
  float kb0, c_r2, c_z2, c_z4;
  float h_max;
};

struct DevCfg {
  float mkb;        // -kappa * B: omega = mkb * (q/pT)
  float chi2_cut;
  float ms_var;     // ms_sigma^2
  float edge_margin;
  float l_min;
  int n_cand;
  int max_holes;
  float init_var[6];
  DevMat mat;
  DevField field;
};


// scalar helpers overloaded for FP32 (the find) and FP64 (seed fitting)
__device__ __forceinline__ void sincos_t(float x, float *s, float *c) { sincosf(x, s, c); }
__device__ __forceinline__ void sincos_t(double x, double *s, double *c) { sincos(x, s, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float sqrt_t(float a) { return sqrtf(a); }
__device__ __forceinline__ double sqrt_t(double a) { return sqrt(a); }
__device__ __forceinline__ float rsqrt_t(float a) { return rsqrtf(a); }
__device__ __forceinline__ double rsqrt_t(double a) { return 1.0 / sqrt(a); }
__device__ __forceinline__ float atan_t(float a) { return atanf(a); }
__device__ __forceinline__ double atan_t(double a) { return atan(a); }
__device__ __forceinline__ float log_t(float a) { return logf(a); }
__device__ __forceinline__ double log_t(double a) { return log(a); }
// for the material corrections (a relative error of ~1e-6 in a correction
// of ~1e-3 is far below the FP32 state's rounding): hardware reciprocal,
// logarithm and sine/cosine in FP32, the exact forms in FP64
__device__ __forceinline__ float div_fast(float a, float b) {
  return a * __builtin_amdgcn_rcpf(b);
}
__device__ __forceinline__ double div_fast(double a, double b) { return a / b; }
__device__ __forceinline__ float log_fast(float a) { return __logf(a); }
__device__ __forceinline__ double log_fast(double a) { return log(a); }
__device__ __forceinline__ void sincos_fast(float x, float *s, float *c) { __sincosf(x, s, c); }
__device__ __forceinline__ void sincos_fast(double x, double *s, double *c) { sincos(x, s, c); }
__device__ __forceinline__ float abs_t(float a) { return fabsf(a); }
__device__ __forceinline__ double abs_t(double a) { return fabs(a); }
__device__ __forceinline__ float copysign_t(float a, float b) { return copysignf(a, b); }
__device__ __forceinline__ double copysign_t(double a, double b) { return copysign(a, b); }

template <typename T> struct Consts;
template <> struct Consts<float> {
  static __device__ __forceinline__ float pi() { return kPi; }
  static __device__ __forceinline__ float two_pi() { return kTwoPi; }
};
template <> struct Consts<double> {
  static __device__ __forceinline__ double pi() { return 3.14159265358979323846; }
  static __device__ __forceinline__ double two_pi() { return 6.28318530717958647692; }
};

// index of (i, j), i <= j, in the packed upper triangle
__host__ __device__ constexpr int tri(int i, int j) {
  return i * 6 - (i * (i - 1)) / 2 + (j - i);
}

template <typename T>
__device__ __forceinline__ T wrap_phi(T a) {
  if (a > Consts<T>::pi()) a -= Consts<T>::two_pi();
  else if (a <= -Consts<T>::pi()) a += Consts<T>::two_pi();
  return a;
}

// sinc(h) = sin h / h
template <typename T>
__device__ __forceinline__ T sinc_from(T h, T sh) {
  return h == T(0) ? T(1) : sh / h;
}

// d sinc / dh: Taylor series below |h| < 0.5 (the closed form cancels)
template <typename T>
__device__ __forceinline__ T dsinc(T h, T sh, T ch) {
  if (abs_t(h) < T(0.5)) {
    const T h2 = h * h;
    return h * (T(-1) / T(3) +
                h2 * (T(1) / T(30) +
                      h2 * (T(-1) / T(840) + h2 * (T(1) / T(45360) - h2 * (T(1) / T(3991680))))));
  }
  return (h * ch - sh) / (h * h);
}

// transverse path for the quadratic's root tau: l = (2/w) atan(w tau / 2)
template <typename T>
__device__ __forceinline__ T tau_to_l(T tau, T w) {
  const T zz = T(0.5) * w * tau;
  // atan(z)/z; below |z| < 1e-3 the series 1 - z^2/3 is exact to FP64 rounding
  const T f = abs_t(zz) < T(1e-3) ? T(1) - zz * zz * (T(1) / T(3)) * (T(1) - T(0.6) * zz * zz)
                                  : atan_t(zz) / zz;
  return tau * f;
}

// Smallest transverse path l > l_min, inside the first half turn, at which
// the helix reaches the cylinder r = R.  Closed form: with
// a = x cos phi + y sin phi, c = y cos phi - x sin phi, g0 = x^2 + y^2 - R^2,
// tau = (2/w) tan(w l / 2) solves (1 + c w + g0 w^2/4) tau^2 + 2 a tau + g0 = 0;
// every real root is a crossing with |w l| < pi.  l grows with tau (dl/dtau
// = 1 / (1 + (w tau / 2)^2)), so the smaller root is converted first and the
// larger one only if the smaller lies below l_min: one arctangent per
// crossing in the usual case.
template <typename T>
__device__ __forceinline__ bool path_barrel(T x, T y, T cphi, T sphi, T w, T R, T l_min,
                                            T &l_out) {
  const T a = fma_t(x, cphi, y * sphi);
  const T c = fma_t(y, cphi, -x * sphi);
  const T g0 = fma_t(x, x, fma_t(y, y, -R * R));
  const T alpha = T(1) + c * w + T(0.25) * g0 * w * w;
  const T disc = fma_t(a, a, -alpha * g0);
  if (!(disc >= T(0))) return false;
  const T sq = sqrt_t(disc);
  const T qq = -(a + copysign_t(sq, a));
  // qq == 0: a == 0 and disc == 0, a double root at tau = 0 <= l_min
  if (qq == T(0)) return false;
  const T t1 = g0 / qq;
  const bool two = alpha != T(0);
  const T t2 = two ? qq / alpha : t1;
  const T ta = two && t2 < t1 ? t2 : t1, tb = two && t2 < t1 ? t1 : t2;
  T l = tau_to_l(ta, w);
  if (!(l > l_min)) {
    if (!two) return false;
    l = tau_to_l(tb, w);
    if (!(l > l_min)) return false;
  }
  l_out = l;
  return true;
}

// Result of a propagation.
template <typename T>
struct PropT {
  T p[6];
  T c[21];
  T l;
  T sth, cth;  // sin, cos of theta (unchanged by the transport)
  int status;
};
using Prop = PropT<float>;

// -kappa Bz at (x, y, z) of the parameterised field
template <typename T>
__device__ __forceinline__ T field_mkb(const DevField &f, T x, T y, T z) {
  // contraction within each expression only: the same rounding in every
  // kernel that inlines this
#pragma clang fp contract(on)
  const T r2 = x * x + y * y, z2 = z * z;
  return T(f.kb0) * (T(1) + T(f.c_r2) * r2 + T(f.c_z2) * z2 + T(f.c_z4) * z2 * z2);
}

// The increment d of one classical Runge-Kutta step of transverse length h
// of (x, y, z, phi) in the axial field (pT and theta constant; phi turns at
// the local curvature).
template <typename T>
__device__ __forceinline__ void rk4_field(const DevField &f, T ipt, T cot, const T *y, T h,
                                          T *d) {
#pragma clang fp contract(on)
  T k[4][4], t[4];
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const T a = st == 0 ? T(0) : (st == 3 ? h : T(0.5) * h);
#pragma unroll
    for (int i = 0; i < 4; ++i) t[i] = st == 0 ? y[i] : fma_t(a, k[st - 1][i], y[i]);
    T sp, cp;
    sincos_t(t[3], &sp, &cp);
    k[st][0] = cp;
    k[st][1] = sp;
    k[st][2] = cot;
    k[st][3] = field_mkb(f, t[0], t[1], t[2]) * ipt;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
    d[i] = h / T(6) * (k[0][i] + T(2) * k[1][i] + T(2) * k[2][i] + k[3][i]);
}

// Compensated (Kahan) accumulation of the steps: y holds the sum rounded,
// cmp the part rounded away (the sum is y - cmp), so that many short steps
// in FP32 do not accumulate the position's rounding.
template <typename T>
__device__ __forceinline__ void rk_accumulate(T *y, T *cmp, const T *d) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const T t = d[i] - cmp[i];
    const T s = y[i] + t;
    cmp[i] = (s - y[i]) - t;
    y[i] = s;
  }
}

constexpr float kFieldMaxPath = 1000.f;  // cm of transverse path searched

// Crossing of layer L in the parameterised field: on a disk, equal steps to
// the exact path (Z - z) tan(theta); on a barrel, steps of h_max until
// r^2 - R^2 changes sign, then three Newton iterations on the last step's length.
// The turning stays below half a turn, the path below kFieldMaxPath.
// y: the end point (x, y, z, phi unwrapped).
// cnt (if given): cnt[0] += Runge-Kutta steps taken, cnt[1] += Newton
// iterations.
template <typename T>
__device__ __forceinline__ bool field_crossing(const DevField &f, const T *p, T sth, T cth,
                                               const DevLayer &L, T l_min, T &l, T *y,
                                               int *cnt = nullptr) {
#pragma clang fp contract(on)
  const T cot = cth / sth;
  y[0] = p[0];
  y[1] = p[1];
  y[2] = p[2];
  y[3] = p[4];
  const T pos = T(L.pos);
  const T h_max = T(f.h_max);
  if (L.kind == 1) {
    if (cth == T(0)) return false;
    const T lt = (pos - p[2]) * sth / cth;
    if (!(lt > l_min) || lt > T(kFieldMaxPath)) return false;
    const int n = (int)ceil(lt / h_max);
    const T h = lt / T(n);
    if (cnt) cnt[0] += n;
    T cmp[4] = {T(0), T(0), T(0), T(0)}, d[4];
    for (int k = 0; k < n; ++k) {
      rk4_field(f, p[3], cot, y, h, d);
      rk_accumulate(y, cmp, d);
      if (abs_t(y[3] - p[4]) >= Consts<T>::pi()) return false;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) y[i] -= cmp[i];
    y[2] = pos;
    l = lt;
    return true;
  }
  const T R2 = pos * pos;
  T g = y[0] * y[0] + y[1] * y[1] - R2, lacc = T(0);
  T cmp[4] = {T(0), T(0), T(0), T(0)}, d[4];
  int nstep = 0;
  for (;;) {
    T yn[4], cn[4];
    if (cnt) ++cnt[0];
    rk4_field(f, p[3], cot, y, h_max, d);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      yn[i] = y[i];
      cn[i] = cmp[i];
    }
    rk_accumulate(yn, cn, d);
    const T gn = yn[0] * yn[0] + yn[1] * yn[1] - R2;
    if ((g < T(0)) != (gn < T(0)) || gn == T(0)) {
      T s = g == gn ? h_max : h_max * g / (g - gn), ys[4];
      for (int it = 0; it < 3; ++it) {
        if (cnt) {
          ++cnt[0];
          ++cnt[1];
        }
        rk4_field(f, p[3], cot, y, s, d);
#pragma unroll
        for (int i = 0; i < 4; ++i) ys[i] = y[i] + (d[i] - cmp[i]);
        T sp, cp;
        sincos_t(ys[3], &sp, &cp);
        const T gs = ys[0] * ys[0] + ys[1] * ys[1] - R2;
        const T gp = T(2) * (ys[0] * cp + ys[1] * sp);
        if (gp == T(0)) break;
        s -= gs / gp;
      }
      if (cnt) ++cnt[0];
      rk4_field(f, p[3], cot, y, s, d);
#pragma unroll
      for (int i = 0; i < 4; ++i) ys[i] = y[i] + (d[i] - cmp[i]);
      if (lacc + s > l_min && abs_t(ys[3] - p[4]) < Consts<T>::pi()) {
        l = lacc + s;
#pragma unroll
        for (int i = 0; i < 4; ++i) y[i] = ys[i];
        return true;
      }
    }
    if (abs_t(yn[3] - p[4]) >= Consts<T>::pi()) return false;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      y[i] = yn[i];
      cmp[i] = cn[i];
    }
    g = gn;
    lacc = T(++nstep) * h_max;  // the path so far, without accumulated rounding
    if (lacc > T(kFieldMaxPath)) return false;
  }
}

// Barrel crossing in the parameterised field from a predicted path l_hint
// (the learned surrogate's): equal Runge-Kutta steps of at most h_max to
// l_hint, then one Newton step on g = r^2 - R^2 there, taken as one
// Runge-Kutta step of the correction's length.  Kept under the checks of
// the uniform-field hint (correction at most 1e-4 l1, the Newton error bound
// 3 dl^2 / |g'| at most 1e-7 l1, g' of the sign that marks the first
// crossing, l1 > l_min, turning below half a turn); otherwise false, and the
// caller takes field_crossing.  y: the end point (x, y, z, phi unwrapped).
template <typename T>
__device__ __forceinline__ bool field_crossing_hinted(const DevField &f, const T *p, T sth, T cth,
                                                      const DevLayer &L, T l_min, T l_hint, T &l,
                                                      T *y, int *cnt = nullptr) {
#pragma clang fp contract(on)
  const T cot = cth / sth;
  const T pos = T(L.pos);
  const T h_max = T(f.h_max);
  if (!(l_hint > l_min) || !(l_hint <= T(kFieldMaxPath))) return false;
  const int n = max(1, (int)ceil(l_hint / h_max));
  const T h = l_hint / T(n);
  if (cnt) cnt[0] += n;
  y[0] = p[0];
  y[1] = p[1];
  y[2] = p[2];
  y[3] = p[4];
  T cmp[4] = {T(0), T(0), T(0), T(0)}, d[4];
  for (int k = 0; k < n; ++k) {
    rk4_field(f, p[3], cot, y, h, d);
    rk_accumulate(y, cmp, d);
    if (abs_t(y[3] - p[4]) >= Consts<T>::pi()) return false;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) y[i] -= cmp[i];
  T sp, cp;
  sincos_t(y[3], &sp, &cp);
  const T R2 = pos * pos;
  const T g = y[0] * y[0] + y[1] * y[1] - R2;
  const T gp = T(2) * (y[0] * cp + y[1] * sp);
  const T g0 = p[0] * p[0] + p[1] * p[1] - R2;
  if (!(gp * g0 < T(0))) return false;
  const T dl = -g / gp;
  const T l1 = l_hint + dl;
  if (!(l1 > l_min) || !(abs_t(dl) <= T(1e-4) * l1) ||
      !(T(3) * dl * dl <= T(1e-7) * l1 * abs_t(gp)))
    return false;
  if (cnt) {
    ++cnt[0];
    ++cnt[1];
  }
  rk4_field(f, p[3], cot, y, dl, d);
#pragma unroll
  for (int i = 0; i < 4; ++i) y[i] += d[i];
  if (abs_t(y[3] - p[4]) >= Consts<T>::pi()) return false;
  l = l1;
  return true;
}

// Exact helix transport by l, surface polish, extent test, and the
// surface-constrained covariance transport C' = F C F^T with
// F = (I - t n^T / (n^T t)) D (D: d p'/d p at fixed l; t = d p'/dl; n: the
// surface gradient).  With k = n^T D / (n^T t), F = D - t k^T and
//   C' = D C D^T - t g^T - g t^T + (k^T C k) t t^T,   g = D C k.
// kWantCov = false skips the covariance (plans).  check_extent widens the
// extent by edge_margin.
//
// l_hint > 0 (barrel only) is a predicted path length, e.g. the learned
// surrogate's: one exact Newton step on g(l) = r(l)^2 - R^2 refines it to
// l1, which is kept if the correction is at most 1e-4 l1, the Newton error
// bound left after it is at most 1e-7 l1 (near FP32 rounding), and g' at l1
// marks the first crossing; otherwise the closed form below is used, so the
// result never depends on the quality of the hint.  *sur (if given)
// receives 1 if the hint was kept, 2 if not.
//
// kWantFC: fc receives F C, 6x6 row-major (the cross-covariance of the
// start and end states, which smoothing needs).
//
// fld (if given and on): the parameterised field.  The crossing and the end
// point come from Runge-Kutta steps (field_crossing); the Jacobian is the
// helix's with the path's mean curvature (the turning over the path), whose
// end direction is the stepped one.
//
// trig (if given): sin phi, cos phi, sin theta, cos theta of p, computed by
// the caller (the same values the propagation would compute).
//
// cnt (if given): the field crossing's Runge-Kutta steps and Newton
// iterations are added to cnt[0] and cnt[1].
template <bool kWantCov, typename T, bool kWantFC = false>
__device__ __forceinline__ int propagate(const T *__restrict__ p, const T *__restrict__ c,
                                         const DevLayer &L, T mkb, T l_min, bool check_extent,
                                         T edge_margin, PropT<T> &o, T l_hint = T(0),
                                         int *sur = nullptr, T *fc = nullptr,
                                         const DevField *fld = nullptr,
                                         const T *trig = nullptr, int *cnt = nullptr) {
  T w = mkb * p[3];
  T sphi, cphi, sth, cth;
  if (trig) {
    sphi = trig[0];
    cphi = trig[1];
    sth = trig[2];
    cth = trig[3];
  } else {
    sincos_t(p[4], &sphi, &cphi);
    sincos_t(p[5], &sth, &cth);
  }
  const T cot = cth / sth;
  const T pos = T(L.pos);
  T l;
  bool hinted = false;
  const bool stepped = fld != nullptr && fld->on;
  T yf[4];
  if (stepped) {
    if (L.kind == 0 && l_hint > T(0)) {
      hinted = field_crossing_hinted(*fld, p, sth, cth, L, l_min, l_hint, l, yf, cnt);
      if (sur) *sur = hinted ? 1 : 2;
    }
    if (!hinted && !field_crossing(*fld, p, sth, cth, L, l_min, l, yf, cnt)) return kNoCrossing;
    w = (yf[3] - p[4]) / l;
    mkb = p[3] != T(0) ? w / p[3] : mkb;
  } else if (L.kind == 0) {
    if (l_hint > T(0)) {
      T hs, hc;
      const T hh = T(0.5) * w * l_hint;
      sincos_t(hh, &hs, &hc);
      const T Lh = l_hint * sinc_from(hh, hs);
      const T cps = cphi * hc - sphi * hs, sps = sphi * hc + cphi * hs;
      const T cp1 = cps * hc - sps * hs, sp1 = sps * hc + cps * hs;
      const T xh = fma_t(Lh, cps, p[0]), yh = fma_t(Lh, sps, p[1]);
      const T gh = fma_t(xh, xh, fma_t(yh, yh, -pos * pos));
      const T gph = T(2) * fma_t(xh, cp1, yh * sp1);
      // g(0) = r0^2 - R^2: the first crossing is the root where g changes
      // sign away from g(0), so g' there has the opposite sign
      const T g0 = fma_t(p[0], p[0], fma_t(p[1], p[1], -pos * pos));
      if (gph * g0 < T(0)) {
        const T dl = -gh / gph;
        const T l1 = l_hint + dl;
        // |g''| <= 6 for a track that reaches R, so the error left after
        // the step is at most 3 dl^2 / |g'|: keep it below 1e-7 l1
        hinted = l1 > l_min && abs_t(w) * l1 < Consts<T>::pi() &&
                 abs_t(dl) <= T(1e-4) * l1 && T(3) * dl * dl <= T(1e-7) * l1 * abs_t(gph);
        if (hinted) l = l1;
      }
      if (sur) *sur = hinted ? 1 : 2;
    }
    if (!hinted && !path_barrel(p[0], p[1], cphi, sphi, w, pos, l_min, l)) return kNoCrossing;
  } else {
    if (cth == T(0)) return kNoCrossing;
    l = (pos - p[2]) * sth / cth;
    if (!(l > l_min) || abs_t(w) * l >= Consts<T>::pi()) return kNoCrossing;
  }
  const T h = T(0.5) * w * l;
  T sh, ch;
  sincos_t(h, &sh, &ch);
  const T Lc = l * sinc_from(h, sh);  // chord length
  const T cpsi = cphi * ch - sphi * sh;  // direction of the chord
  const T spsi = sphi * ch + cphi * sh;
  const T cphi1 = cpsi * ch - spsi * sh;  // direction at the end
  const T sphi1 = spsi * ch + cpsi * sh;
  T x1 = fma_t(Lc, cpsi, p[0]);
  T y1 = fma_t(Lc, spsi, p[1]);
  T z1 = fma_t(l, cot, p[2]);
  if (stepped) {  // the stepped end point, on the mean-curvature helix's end direction
    x1 = yf[0];
    y1 = yf[1];
    z1 = yf[2];
  }
  // one Newton step along the track removes the rounding of the closed form
  // (a kept surrogate path has had its Newton step already)
  if (L.kind == 0 && !hinted) {
    const T g = fma_t(x1, x1, fma_t(y1, y1, -pos * pos));
    const T gp = T(2) * fma_t(x1, cphi1, y1 * sphi1);
    if (gp != T(0)) {
      const T dl = -g / gp;
      x1 = fma_t(dl, cphi1, x1);
      y1 = fma_t(dl, sphi1, y1);
      z1 = fma_t(dl, cot, z1);
      l += dl;
    }
  } else if (L.kind == 1) {
    const T dl = (pos - z1) * sth / cth;
    x1 = fma_t(dl, cphi1, x1);
    y1 = fma_t(dl, sphi1, y1);
    z1 = pos;
    l += dl;
  }
  if (check_extent) {
    const T q = L.kind == 0 ? z1 : sqrt_t(fma_t(x1, x1, y1 * y1));
    if (q < T(L.lo) - edge_margin || q > T(L.hi) + edge_margin) return kOutOfExtent;
    // a hole (shrunk by the same margin) has no sensors
    if (q > T(L.hole_lo) + edge_margin && q < T(L.hole_hi) - edge_margin) return kOutOfExtent;
  }
  o.p[0] = x1;
  o.p[1] = y1;
  o.p[2] = z1;
  o.p[3] = p[3];
  o.p[4] = wrap_phi(fma_t(w, l, p[4]));
  o.p[5] = p[5];
  o.l = l;
  o.sth = sth;
  o.cth = cth;
  o.status = kOk;
  if (!kWantCov) return kOk;

  // ---- Jacobian D (identity + E), fixed l
  const T dw = mkb;  // d w / d(q/pT)
  const T dLdw = l * dsinc(h, sh, ch) * T(0.5) * l;
  const T E03 = (dLdw * cpsi - Lc * spsi * T(0.5) * l) * dw;
  const T E04 = -Lc * spsi;
  const T E13 = (dLdw * spsi + Lc * cpsi * T(0.5) * l) * dw;
  const T E14 = Lc * cpsi;
  const T E25 = -l / (sth * sth);
  const T E43 = l * dw;
  // t = d p'/dl = (cphi1, sphi1, cot, 0, w, 0);  k = n^T D / (n^T t)
  T k0, k1, k2, k3, k4, k5;
  if (L.kind == 0) {
    const T inv = T(1) / fma_t(x1, cphi1, y1 * sphi1);
    k0 = x1 * inv;
    k1 = y1 * inv;
    k2 = T(0);
    k3 = fma_t(x1, E03, y1 * E13) * inv;
    k4 = fma_t(x1, E04, y1 * E14) * inv;
    k5 = T(0);
  } else {
    const T inv = T(1) / cot;
    k0 = T(0);
    k1 = T(0);
    k2 = inv;
    k3 = T(0);
    k4 = T(0);
    k5 = E25 * inv;
  }
  T C[6][6];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = i; j < 6; ++j) {
      C[i][j] = c[tri(i, j)];
      C[j][i] = C[i][j];
    }
  // hk = C k, s = k^T C k, g = D hk
  T hk[6];
#pragma unroll
  for (int i = 0; i < 6; ++i)
    hk[i] = C[i][0] * k0 + C[i][1] * k1 + C[i][2] * k2 + C[i][3] * k3 + C[i][4] * k4 +
            C[i][5] * k5;
  const T s = k0 * hk[0] + k1 * hk[1] + k2 * hk[2] + k3 * hk[3] + k4 * hk[4] + k5 * hk[5];
  T g[6];
  g[0] = fma_t(E03, hk[3], fma_t(E04, hk[4], hk[0]));
  g[1] = fma_t(E13, hk[3], fma_t(E14, hk[4], hk[1]));
  g[2] = fma_t(E25, hk[5], hk[2]);
  g[3] = hk[3];
  g[4] = fma_t(E43, hk[3], hk[4]);
  g[5] = hk[5];
  const T t[6] = {cphi1, sphi1, cot, T(0), w, T(0)};
  // C' = B D^T - t g^T - g t^T + s t t^T (upper triangle), with B = D C
  // formed one row at a time to keep register pressure down
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    T Bi[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      T v = C[i][j];
      if (i == 0) v = fma_t(E03, C[3][j], fma_t(E04, C[4][j], v));
      if (i == 1) v = fma_t(E13, C[3][j], fma_t(E14, C[4][j], v));
      if (i == 2) v = fma_t(E25, C[5][j], v);
      if (i == 4) v = fma_t(E43, C[3][j], v);
      Bi[j] = v;
    }
    T Ai[6];
    Ai[0] = fma_t(E03, Bi[3], fma_t(E04, Bi[4], Bi[0]));
    Ai[1] = fma_t(E13, Bi[3], fma_t(E14, Bi[4], Bi[1]));
    Ai[2] = fma_t(E25, Bi[5], Bi[2]);
    Ai[3] = Bi[3];
    Ai[4] = fma_t(E43, Bi[3], Bi[4]);
    Ai[5] = Bi[5];
#pragma unroll
    for (int j = i; j < 6; ++j) o.c[tri(i, j)] = Ai[j] - t[i] * g[j] - g[i] * t[j] + s * t[i] * t[j];
    if constexpr (kWantFC) {
      // F C = D C - t (C k)^T; on a disk the z row vanishes identically
#pragma unroll
      for (int j = 0; j < 6; ++j) fc[i * 6 + j] = (L.kind == 1 && i == 2) ? T(0) : Bi[j] - t[i] * hk[j];
    }
  }
  if (L.kind == 1) {
    // on a disk z is exact: its row and column vanish identically, so drop
    // the rounding residue instead of carrying it to the next step
#pragma unroll
    for (int j = 0; j < 6; ++j) o.c[j < 2 ? tri(j, 2) : tri(2, j)] = T(0);
  }
  return kOk;
}

// The wide diagonal prior diag(init_var) of a state that lies on a layer
// (a seed's first hit, a backward fit's first surface), less its extent
// along the layer's normal n at p: a state on a surface has no freedom
// there.  P D P^T with P = 1 - n n^T on the position block (the other
// blocks of the diagonal prior are unchanged).
template <typename T>
__device__ __forceinline__ void surface_prior(const DevCfg &cfg, const T *p, int kind, T *c) {
#pragma unroll
  for (int k = 0; k < 21; ++k) c[k] = T(0);
#pragma unroll
  for (int k = 0; k < 6; ++k) c[tri(k, k)] = T(cfg.init_var[k]);
  T nv[3] = {T(0), T(0), T(1)};
  if (kind == 0) {
    const T r = sqrt_t(p[0] * p[0] + p[1] * p[1]);
    nv[0] = p[0] / r;
    nv[1] = p[1] / r;
    nv[2] = T(0);
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) {
      T a = T(0);
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const T pim = (i == m ? T(1) : T(0)) - nv[i] * nv[m];
        const T pjm = (j == m ? T(1) : T(0)) - nv[j] * nv[m];
        a += pim * T(cfg.init_var[m]) * pjm;
      }
      c[tri(i, j)] = a;
    }
}

// Scattering noise of one crossed layer, added to the (q/pT, phi, theta)
// block: two independent deflections of variance sigma^2 perpendicular to
// the momentum with |p| fixed.
// (sth, cth: sin and cos of theta, where the caller has them)
template <typename T>
__device__ __forceinline__ void add_ms(const T *p, T ms_var, T *c, T sth, T cth) {
  if (ms_var == T(0)) return;
  const T is = T(1) / sth;
  const T a = p[3] * cth * is;
  c[tri(3, 3)] += a * a * ms_var;
  c[tri(3, 5)] -= a * ms_var;
  c[tri(4, 4)] += ms_var * (is * is);
  c[tri(5, 5)] += ms_var;
}

template <typename T>
__device__ __forceinline__ void add_ms(const T *p, T ms_var, T *c) {
  if (ms_var == T(0)) return;
  T sth, cth;
  sincos_t(p[5], &sth, &cth);
  add_ms(p, ms_var, c, sth, cth);
}

// Mean ionisation loss rate in silicon (Bethe, no density or shell
// correction), GeV cm^2/g, at (beta gamma)^2 = bg2 for a particle of mass m.
template <typename T>
__device__ __forceinline__ T si_loss_rate(T bg2, T m) {
  // contraction within each expression only: the same rounding in every
  // kernel that inlines this
#pragma clang fp contract(on)
  const T me = T(0.51099895e-3), r = div_fast(me, m);
  const T b2 = div_fast(bg2, T(1) + bg2), g = sqrt_t(T(1) + bg2);
  const T wmax = div_fast(T(2) * me * bg2, T(1) + T(2) * g * r + r * r);
  // K Z/A with K = 0.307075e-3 GeV cm^2/mol, Z/A = 0.49848; I = 173 eV
  return div_fast(T(0.307075e-3 * 0.49848), b2) *
         (T(0.5) * log_fast(T(2) * me * bg2 * wmax * T(1.0 / (173e-9 * 173e-9))) - b2);
}

// Effects of one crossed layer's material on the state at the crossing.
// Without a map: the constant scattering angle.  With one (the paper's r-z
// radiation and interaction length arrays, Section 2.1): the bin at the
// crossing gives the thickness at normal incidence, scaled by the path
// factor 1/|cos| of the incidence (at most k_max); the Highland angle of
// those radiation lengths at the momentum before the loss scatters the
// track; then the mean ionisation loss dp = dE / beta (at most half of |p|)
// changes |p| by -dir * dp (dir = -1 regains it on the way back).  The loss
// maps q/pT -> q/pT |p|/|p'| with dp held fixed; its Jacobian (identity but
// the q/pT row: j33 on q/pT, j35 on theta) multiplies the covariance on both
// sides and is returned in *j33, *j35.  tab: the map's table where the
// caller staged it (nullptr: the map's own).
template <typename T>
__device__ __forceinline__ void material(const DevCfg &cfg, int kind, T *p, T *c, T dir,
                                         T *j33 = nullptr, T *j35 = nullptr,
                                         const float2 *tab = nullptr) {
#pragma clang fp contract(on)
  if (j33) *j33 = T(1);
  if (j35) *j35 = T(0);
  const DevMat &M = cfg.mat;
  if (M.tab == nullptr) {
    add_ms(p, T(cfg.ms_var), c);
    return;
  }
  const T r = sqrt_t(p[0] * p[0] + p[1] * p[1]);
  int ir = (int)floor(r * T(M.r_scale));
  int iz = (int)floor((p[2] + T(M.z_max)) * T(M.z_scale));
  ir = ir < 0 ? 0 : (ir >= M.nr ? M.nr - 1 : ir);
  iz = iz < 0 ? 0 : (iz >= M.nz ? M.nz - 1 : iz);
  const float2 tb = (tab ? tab : M.tab)[iz * M.nr + ir];
  T sth, cth;
  sincos_t(p[5], &sth, &cth);
  T cosa = cth;
  if (kind == 0) {
    T sph, cph;
    sincos_fast(p[4], &sph, &cph);
    cosa = div_fast(sth * (cph * p[0] + sph * p[1]), r);
  }
  const T k = abs_t(cosa) * T(M.k_max) > T(1) ? div_fast(T(1), abs_t(cosa)) : T(M.k_max);
  const T pm = div_fast(T(1), abs_t(p[3]) * sth);
  const T m = T(M.mass);
  const T e = sqrt_t(pm * pm + m * m);
  const T beta = div_fast(pm, e);
  const T t = T(tb.x) * k;
  if (t > T(0)) {
    T f = T(1) + T(0.038) * log_fast(t);
    f = f < T(0) ? T(0) : f;
    const T th0 = div_fast(T(0.0136), beta * pm) * sqrt_t(t) * f;
    add_ms(p, th0 * th0, c);
  }
  const T x = T(tb.y) * k;
  if (x > T(0)) {
    const T im = div_fast(T(1), m);
    T dp = div_fast(x * si_loss_rate(pm * pm * im * im, m), beta);
    dp = dp > T(0.5) * pm ? T(0.5) * pm : dp;
    const T ratio = div_fast(T(1), T(1) - dir * div_fast(dp, pm));
    const T a = ratio * ratio;
    const T b = dir * dp * p[3] * abs_t(p[3]) * cth * a;
    p[3] *= ratio;
    // C <- J C J^T, J = I but row 3 = (0, 0, 0, a, 0, b)
    const T c33 = c[tri(3, 3)], c35 = c[tri(3, 5)], c55 = c[tri(5, 5)];
    // (tri takes its row index first: the smaller of the two)
#pragma unroll
    for (int mm = 0; mm < 6; ++mm) {
      if (mm == 3) continue;
      const int i3 = mm < 3 ? tri(mm, 3) : tri(3, mm);
      const int i5 = mm < 5 ? tri(mm, 5) : tri(5, mm);
      c[i3] = a * c[i3] + b * c[i5];
    }
    c[tri(3, 5)] = a * c35 + b * c55;
    c[tri(3, 3)] = a * a * c33 + T(2) * a * b * c35 + b * b * c55;
    if (j33) *j33 = a;
    if (j35) *j35 = b;
  }
}

// Local frame at the predicted point and the 2x2 predicted covariance
// H C H^T.  u = t.(x_h - x'), t = (-y', x')/r'; v = z_h - z' (barrel) or
// rh.(x_h - x'), rh = (x', y')/r' (disk).
template <typename T>
struct FrameT {
  T tx, ty, rx, ry;
  T suu, suv, svv;
};
using Frame = FrameT<float>;

template <typename T>
__device__ __forceinline__ void make_frame(const T *p, const T *c, int kind, FrameT<T> &f) {
  const T inv_r = rsqrt_t(fma_t(p[0], p[0], p[1] * p[1]));
  f.tx = -p[1] * inv_r;
  f.ty = p[0] * inv_r;
  f.rx = p[0] * inv_r;
  f.ry = p[1] * inv_r;
  const T c00 = c[tri(0, 0)], c01 = c[tri(0, 1)], c11 = c[tri(1, 1)];
  f.suu = f.tx * f.tx * c00 + T(2) * f.tx * f.ty * c01 + f.ty * f.ty * c11;
  if (kind == 0) {
    f.suv = f.tx * c[tri(0, 2)] + f.ty * c[tri(1, 2)];
    f.svv = c[tri(2, 2)];
  } else {
    f.suv = f.tx * f.rx * c00 + (f.tx * f.ry + f.ty * f.rx) * c01 + f.ty * f.ry * c11;
    f.svv = f.rx * f.rx * c00 + T(2) * f.rx * f.ry * c01 + f.ry * f.ry * c11;
  }
}

// Residual of a hit; false for a barrel hit in the opposite half.
template <typename T>
__device__ __forceinline__ bool residual(const T *p, const FrameT<T> &f, int kind, T hx, T hy,
                                         T hz, T &u, T &v) {
  const T dx = hx - p[0], dy = hy - p[1];
  u = fma_t(f.tx, dx, f.ty * dy);
  if (kind == 0) {
    if (fma_t(p[0], hx, p[1] * hy) <= T(0)) return false;
    v = hz - p[2];
  } else {
    v = fma_t(f.rx, dx, f.ry * dy);
  }
  return true;
}

// Hit covariance in the local (u, v) frame from the variances along and
// across the strips of a layer whose strips measure in a direction turned by
// the stereo angle (cos cs, sin sn) from u: V = R^T diag(vw, vp) R.
template <typename T>
__device__ __forceinline__ void hit_cov(T cs, T sn, T vw, T vp, T &vuu, T &vvv, T &vuv) {
  vuu = fma_t(cs * cs, vw, sn * sn * vp);
  vvv = fma_t(sn * sn, vw, cs * cs * vp);
  vuv = cs * sn * (vw - vp);
}

template <typename T>
__device__ __forceinline__ T chi2_of(const FrameT<T> &f, T vu, T vv, T vuv, T u, T v) {
  const T suu = f.suu + vu, svv = f.svv + vv, suv = f.suv + vuv;
  const T det = fma_t(suu, svv, -suv * suv);
  return (svv * u * u - T(2) * suv * u * v + suu * v * v) / det;
}

// Kalman update with the hit (u, v residual, covariance vu, vv, vuv): K = C H^T
// S^-1, p += K r, and the covariance in Joseph form,
//   C' = (I - K H) C (I - K H)^T + K V K^T = C - K (CH^T)^T - B K^T,
// with B = C H^T - K (H C H^T + V), which is zero in exact arithmetic and
// in FP32 carries the first-order effect of the rounding of K.  The plain
// gain form C - K (C H^T)^T loses the covariance where the prediction is
// much wider than the hit (tracks that meet a layer nearly tangentially),
// because its result is a small difference of large terms.
template <typename T>
__device__ __forceinline__ void kf_update(T *p, T *c, const FrameT<T> &f, int kind, T vu, T vv,
                                          T vuv, T u, T v) {
  T PHu[6], PHv[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const T ci0 = c[i <= 0 ? tri(i, 0) : tri(0, i)];
    const T ci1 = c[i <= 1 ? tri(i, 1) : tri(1, i)];
    PHu[i] = fma_t(f.tx, ci0, f.ty * ci1);
    PHv[i] = kind == 0 ? c[i <= 2 ? tri(i, 2) : tri(2, i)] : fma_t(f.rx, ci0, f.ry * ci1);
  }
  const T suu = f.suu + vu, svv = f.svv + vv, suv = f.suv + vuv;
  const T inv_det = T(1) / fma_t(suu, svv, -suv * suv);
  const T iuu = svv * inv_det, ivv = suu * inv_det, iuv = -suv * inv_det;
  T Ku[6], Kv[6], Bu[6], Bv[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    Ku[i] = fma_t(PHu[i], iuu, PHv[i] * iuv);
    Kv[i] = fma_t(PHu[i], iuv, PHv[i] * ivv);
    p[i] = fma_t(Ku[i], u, fma_t(Kv[i], v, p[i]));
    Bu[i] = PHu[i] - fma_t(Ku[i], suu, Kv[i] * suv);
    Bv[i] = PHv[i] - fma_t(Ku[i], suv, Kv[i] * svv);
  }
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = i; j < 6; ++j)
      c[tri(i, j)] -= fma_t(Ku[i], PHu[j], fma_t(Kv[i], PHv[j], fma_t(Bu[i], Ku[j], Bv[i] * Kv[j])));
  p[4] = wrap_phi(p[4]);
}

}  // namespace mkf
