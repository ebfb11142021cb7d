// mkf_kernels.hip -- gfx950 kernels of the Kalman-filter track finding and
// fitting hot path (arXiv:1811.04141).
//
//  hit index   : per (event, layer) phi x q bins, CSR over 32-byte records
//  seeding     : triplet helix, 3-hit Kalman fit, per-seed layer plan
//  find        : the clone engine (Introduction): every candidate of a seed
//                is propagated to the next plan layer, all its window hits
//                are scored by chi2, the seed's best extensions are chosen
//                across its lane group, and only the kept ones are updated.
//                One lane per candidate slot, a group of 6 lanes per seed
//                (10 seeds per wavefront) for budgets up to 6, else 8.
//                Two forms share the step code: one launch per layer step
//                with the state in HBM, or one persistent launch that keeps
//                the state in VGPRs across all steps of a seed tile.
//  finalize    : best candidate per seed, hit history from back-pointers
//  propagate / fit : unit propagation and search-free Kalman fitting.
#include <hip/hip_runtime.h>

#include "mkf_kernels.hpp"

namespace mkf {

typedef unsigned long long u64;
constexpr u64 kKeyMax = ~0ull;
constexpr unsigned kOrderNone = 0x7FFFFFu;  // misses and skips sort after every hit

// Ranking key of an extension: more hits first, then smaller accumulated
// chi2, then parent rank, then hit index (miss/skip last).  A total order:
// ties cannot occur between different extensions.
//   bits 58..63: 63 - n_hits   bits 26..57: chi2 (non-negative float bits)
//   bits 23..25: parent slot   bits 0..22 : hit index or kOrderNone
__device__ __forceinline__ u64 ext_key(int nh, float chi2, int parent, unsigned order) {
  return ((u64)(63 - nh) << 58) | ((u64)__float_as_uint(chi2) << 26) | ((u64)parent << 23) |
         (u64)order;
}
// Key of a finished candidate when the seed's result is chosen: final
// candidates (by slot) come before retired ones (by step, then slot) on
// equal hits and chi2.
__device__ __forceinline__ u64 final_key(int nh, float chi2, int retired, int step, int slot) {
  return ((u64)(63 - nh) << 58) | ((u64)__float_as_uint(chi2) << 26) | ((u64)retired << 25) |
         ((u64)step << 19) | ((u64)slot << 16);
}
__device__ __forceinline__ int fkey_step(u64 k) { return (int)((k >> 19) & 63); }
__device__ __forceinline__ int fkey_slot(u64 k) { return (int)((k >> 16) & 7); }

__device__ __forceinline__ u64 shfl_xor_u64(u64 v, int m) {
  unsigned lo = (unsigned)v, hi = (unsigned)(v >> 32);
  lo = __shfl_xor(lo, m);
  hi = __shfl_xor(hi, m);
  return ((u64)hi << 32) | lo;
}
// lane i <- lane i ^ 1 and i ^ 2 within quads, by DPP (no trip through the
// LDS crossbar)
template <int kCtrl>
__device__ __forceinline__ u64 dpp_u64(u64 v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)v, kCtrl, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(v >> 32), kCtrl, 0xF, 0xF, true);
  return ((u64)(unsigned)hi << 32) | (u64)(unsigned)lo;
}
constexpr int kDppXor1 = 0xB1;  // quad_perm(1, 0, 3, 2)
constexpr int kDppXor2 = 0x4E;  // quad_perm(2, 3, 0, 1)

__device__ __forceinline__ u64 shfl_u64(u64 v, int src) {
  unsigned lo = (unsigned)v, hi = (unsigned)(v >> 32);
  lo = __shfl(lo, src);
  hi = __shfl(hi, src);
  return ((u64)hi << 32) | lo;
}

// Lane groups of a seed: G consecutive lanes of a wavefront, one per
// candidate slot.  G = 8 (8 seeds per wave, any candidate budget) reduces
// with xor butterflies; G = 6 (10 seeds per wave, lanes 60-63 idle, for
// budgets up to 6) reduces over the three lane pairs by rotation.
template <int G> struct Grp;
template <> struct Grp<8> {
  static constexpr int kSeeds = 8;
  __device__ static int slot(int lane) { return lane & 7; }
  __device__ static int base(int lane) { return lane & ~7; }
  __device__ static u64 min(u64 v, int lane) {
    u64 o = dpp_u64<kDppXor1>(v);
    v = o < v ? o : v;
    o = dpp_u64<kDppXor2>(v);
    v = o < v ? o : v;
    o = shfl_xor_u64(v, 4);
    return o < v ? o : v;
  }
};
template <> struct Grp<6> {
  static constexpr int kSeeds = 10;
  __device__ static int slot(int lane) { return lane % 6; }
  __device__ static int base(int lane) { return lane - lane % 6; }
  // pairs (0,1) (2,3) (4,5); then the next pair's minimum, then the one
  // after (whose value already includes the first pair)
  __device__ static u64 min(u64 v, int lane) {
    const int sl = lane % 6, b = lane - sl;
    u64 o = dpp_u64<kDppXor1>(v);
    v = o < v ? o : v;
    o = shfl_u64(v, b + (sl < 4 ? sl + 2 : sl - 4));
    v = o < v ? o : v;
    o = shfl_u64(v, b + (sl < 2 ? sl + 4 : sl - 2));
    return o < v ? o : v;
  }
};

// Sorted insertion into a register list (compile-time indices only; keys
// are distinct, empty entries hold kKeyMax).  All comparisons with k come
// first; then entry i keeps its key if that is smaller than k, else takes k
// (where entry i - 1 is smaller) or entry i - 1's key (shifted up).  One
// compare per entry, none of them next to the selects that read it.
template <int N>
__device__ __forceinline__ void insert_sorted(u64 (&lst)[N], u64 k) {
  // the comparisons read a copy of k that the compiler cannot see through
  // (an empty statement, no instruction), so that it keeps one compare per
  // entry for both selects instead of forming a minimum and a maximum
  u64 kc = k;
  asm("" : "+v"(kc));
  bool below[N];
#pragma unroll
  for (int i = 0; i < N; ++i) below[i] = lst[i] < kc;
#pragma unroll
  for (int i = N - 1; i > 0; --i) lst[i] = below[i] ? lst[i] : (below[i - 1] ? k : lst[i - 1]);
  lst[0] = below[0] ? lst[0] : k;
}
// k into position n of a sorted list whose first n entries are all smaller
// than k and whose others are empty (nothing when n >= N): the insertion of
// a key that ranks after every key in the list, without comparisons
template <int N>
__device__ __forceinline__ void put_at(u64 (&lst)[N], int n, u64 k) {
#pragma unroll
  for (int i = 0; i < N; ++i) lst[i] = i == n ? k : lst[i];
}
template <int N>
__device__ __forceinline__ void pop_front(u64 (&lst)[N]) {
#pragma unroll
  for (int i = 0; i < N - 1; ++i) lst[i] = lst[i + 1];
  lst[N - 1] = kKeyMax;
}

__device__ __forceinline__ void stage_layers(const FindParams &P, DevLayer *sl) {
  for (int i = threadIdx.x; i < P.n_layers; i += blockDim.x) sl[i] = P.layers[i];
}

// Adds a wavefront's value of find counter k (every lane of the wave must
// call this; lanes with nothing to count pass 0).  Skipped when the whole
// wave has nothing.
__device__ __forceinline__ void add_counter(const FindParams &P, int k, int v) {
  if (__ballot(v != 0) == 0ull) return;
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) v += __shfl_xor(v, m);
  if ((threadIdx.x & 63) == 0)
    atomicAdd(&P.counters[k * kCounterSlots + blockIdx.x % kCounterSlots],
              (unsigned long long)v);
}

struct Cand {
  float p[6];
  float c[21];
  float chi2;
  int nh, nm;
  bool active;
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// ------------------------------------------------------------ records
//
// Per-seed records a find keeps besides the candidates: the back-pointers
// of every step and the best retired candidate.  The layer-synchronous form
// keeps them in HBM by position; the persistent form keeps them in the
// wavefront's LDS for the seed tile it is working on.
struct GlobalRec {
  const FindParams *P;
  int64_t pos;
  __device__ void put_bp(int step, int slot, int v) const {
    P->bp[((size_t)step * (size_t)P->n_seeds + pos) * P->slots + slot] = v;
  }
  __device__ int get_bp(int step, int slot) const {
    return P->bp[((size_t)step * (size_t)P->n_seeds + pos) * P->slots + slot];
  }
  __device__ void put_fin(const Cand &cd) const {
    const size_t N = (size_t)P->n_seeds;
#pragma unroll
    for (int i = 0; i < 6; ++i) P->fin_rec[i * N + pos] = cd.p[i];
#pragma unroll
    for (int i = 0; i < 21; ++i) P->fin_rec[(6 + i) * N + pos] = cd.c[i];
    P->fin_rec[27 * N + pos] = cd.chi2;
    P->fin_meta[pos] = cd.nh | (cd.nm << 8);
  }
  __device__ void get_fin(float *p, float *c, float &chi2, int &meta) const {
    const size_t N = (size_t)P->n_seeds;
    for (int i = 0; i < 6; ++i) p[i] = P->fin_rec[i * N + pos];
    for (int i = 0; i < 21; ++i) c[i] = P->fin_rec[(6 + i) * N + pos];
    chi2 = P->fin_rec[27 * N + pos];
    meta = P->fin_meta[pos];
  }
};

struct LdsRec {
  int *bp;       // this seed's back-pointers: step s, slot j at bp[s * stride + j]
  int stride;
  float *fin;    // this seed's best retired candidate [kFinWords]
  __device__ void put_bp(int step, int slot, int v) const { bp[step * stride + slot] = v; }
  __device__ int get_bp(int step, int slot) const { return bp[step * stride + slot]; }
  __device__ void put_fin(const Cand &cd) const {
#pragma unroll
    for (int i = 0; i < 6; ++i) fin[i] = cd.p[i];
#pragma unroll
    for (int i = 0; i < 21; ++i) fin[6 + i] = cd.c[i];
    fin[27] = cd.chi2;
    fin[28] = __int_as_float(cd.nh | (cd.nm << 8));
  }
  __device__ void get_fin(float *p, float *c, float &chi2, int &meta) const {
    for (int i = 0; i < 6; ++i) p[i] = fin[i];
    for (int i = 0; i < 21; ++i) c[i] = fin[6 + i];
    chi2 = fin[27];
    meta = __float_as_int(fin[28]);
  }
};

// ---------------------------------------------------------------- window
//
// Bounding box of the chi2 < cut ellipse of every hit on the layer: with
// S_hit <= H C H^T + diag(var_max), |u| <= sqrt(cut S_uu) and |v| <= sqrt(cut
// S_vv).  Barrel: u = R_h sin(dphi) (hits in the same half), v = dz, so
// |dphi| <= asin(s) <= s / sqrt(1 - s^2) with s = du / R.  Disk: the hit is at
// (r' + v) rh + u t, so its radius lies in [r' - dv, sqrt((r' + dv)^2 +
// du^2)] and its azimuth within atan(du / (r' - dv)) <= du / (r' - dv).  The
// box only has to contain the ellipse (the chi2 test decides), so these
// cheaper upper bounds replace asin and atan; a small margin absorbs FP32
// rounding of the bin assignment.  Hits are read four at a time from one
// base address (the sorted array is padded past its end) so that their
// loads overlap.
// Azimuth of (x, y) for the window centre only, within 1e-6 rad (the
// window adds that to its margin): octant reduction, then atan(a) = a P(a^2)
// on [0, 1] with a degree-7 polynomial fitted to atan (largest error 1.3e-7
// rad including FP32 evaluation), the ratio taken with the hardware
// reciprocal.
__device__ __forceinline__ float window_azimuth(float y, float x) {
  const float ax = fabsf(x), ay = fabsf(y);
  const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
  const float a = mx > 0.f ? mn * __builtin_amdgcn_rcpf(mx) : 0.f;
  const float s = a * a;
  float r = -0.004054667f;
  r = fmaf(r, s, 0.021863315f);
  r = fmaf(r, s, -0.055912834f);
  r = fmaf(r, s, 0.096422337f);
  r = fmaf(r, s, -0.139086440f);
  r = fmaf(r, s, 0.199465677f);
  r = fmaf(r, s, -0.333298624f);
  r = fmaf(r, s, 0.999999344f);
  r *= a;
  if (ay > ax) r = 0.5f * kPi - r;
  if (x < 0.f) r = kPi - r;
  return copysignf(r, y);
}

// chi2 of a window hit, with the hardware reciprocal (1 ulp) in place of a
// correctly rounded division; both forms of the find score hits with it
__device__ __forceinline__ float chi2_hit(const Frame &f, float vu, float vv, float vuv, float u,
                                          float v) {
  const float suu = f.suu + vu, svv = f.svv + vv, suv = f.suv + vuv;
  const float det = fmaf(suu, svv, -suv * suv);
  return (svv * u * u - 2.f * suv * u * v + suu * v * v) * __builtin_amdgcn_rcpf(det);
}

// The window's bins: q rows qlo..qhi of the event's layer (base: the index
// of its first bin) and up to two azimuth segments per row, [seg[0],
// seg[1]] and [seg[2], seg[3]] (the second empty unless the window wraps).
__device__ __forceinline__ void window_bins(const FindParams &P, const DevLayer &L, int ev,
                                            const Prop &pr, const Frame &f, int &base, int &qlo,
                                            int &qhi, int (&seg)[4]) {
  const float cut = P.cfg.chi2_cut;
  // (hardware square roots, 1 ulp: the 0.1% widening covers them)
  const float du = __builtin_amdgcn_sqrtf(cut * (f.suu + L.vu_max)) * 1.001f + 1e-5f;
  const float dv = __builtin_amdgcn_sqrtf(cut * (f.svv + L.vv_max)) * 1.001f + 1e-5f;
  const float phic = window_azimuth(pr.p[1], pr.p[0]);
  float dphi, qmin, qmax;
  if (L.kind == 0) {
    // (hardware reciprocals below: the 1e-5 and 1e-4 widenings cover their ulp)
    const float s = du * __builtin_amdgcn_rcpf(L.pos * 0.99999f);
    dphi = s >= 0.99f ? kPi : s * rsqrtf(fmaf(-s, s, 1.f)) * 1.0001f;
    qmin = pr.p[2] - dv;
    qmax = pr.p[2] + dv;
  } else {
    const float r = __builtin_amdgcn_sqrtf(fmaf(pr.p[0], pr.p[0], pr.p[1] * pr.p[1]));
    const float rl = r - dv;
    qmin = rl;
    qmax = __builtin_amdgcn_sqrtf(fmaf(r + dv, r + dv, du * du));
    dphi = rl > 0.f ? fminf(du * __builtin_amdgcn_rcpf(rl) * 1.0001f, kPi) : kPi;
  }
  dphi += 6e-6f;
  qmin -= 1e-4f;
  qmax += 1e-4f;
  const int nphi = L.nphi;
  qlo = clampi((int)floorf((qmin - L.q_lo) * L.q_scale), 0, L.nq - 1);
  qhi = clampi((int)floorf((qmax - L.q_lo) * L.q_scale), 0, L.nq - 1);
  seg[0] = 0;
  seg[1] = nphi - 1;
  seg[2] = 1;
  seg[3] = 0;
  if (dphi < kPi) {
    const int blo = (int)floorf((phic - dphi + kPi) * L.phi_scale);
    const int bhi = (int)floorf((phic + dphi + kPi) * L.phi_scale);
    if (bhi - blo + 1 < nphi) {
      if (blo < 0) {
        seg[0] = blo + nphi; seg[1] = nphi - 1; seg[2] = 0; seg[3] = bhi;
      } else if (bhi >= nphi) {
        seg[0] = blo; seg[1] = nphi - 1; seg[2] = 0; seg[3] = bhi - nphi;
      } else {
        seg[0] = blo; seg[1] = bhi;
      }
    }
  }
  base = ev * P.bins_per_event + L.bin_base;
}

// One window hit against a candidate's prediction (point p, frame f): its
// chi2 (>= 0), or a negative value for a hit on the other half of a barrel.
__device__ __forceinline__ float hit_chi2(const float *p, const Frame &f, int kind,
                                          const float4 &a, const float4 &b) {
  float u, v;
  if (!residual(p, f, kind, a.x, a.y, a.z, u, v)) return -1.f;
  return fmaxf(chi2_hit(f, a.w, b.x, b.z, u, v), 0.f);
}

// A hit's chi2 within this band of the cut is a decision that rounding may
// take either way (the band of the parity checks: 1e-3 relative + 1e-2).
__device__ __forceinline__ float near_cut_band(float cut) { return fmaf(1e-3f, cut, 1e-2f); }

// One lane's window scan: every hit of the window's bins, four at a time.
// n_near counts the hits whose chi2 lies within near_cut_band of the cut.
template <int N>
__device__ __forceinline__ void scan_window(const FindParams &P, const DevLayer &L, int ev,
                                            const Prop &pr, const Frame &f, float chi2_base,
                                            int nh, int slot, u64 (&lst)[N], int &n_ext,
                                            int &n_near) {
  const float cut = P.cfg.chi2_cut;
  const float band = near_cut_band(cut);
  int base, qlo, qhi, seg[4];
  window_bins(P, L, ev, pr, f, base, qlo, qhi, seg);
  for (int qb = qlo; qb <= qhi; ++qb) {
    const int row = base + qb * L.nphi;
#pragma unroll
    for (int sg = 0; sg < 2; ++sg) {
      const int lo = seg[2 * sg], hi = seg[2 * sg + 1];
      if (lo > hi) continue;
      const int h0 = P.bin_start[row + lo];
      const int h1 = P.bin_start[row + hi + 1];
      const float4 *hits = reinterpret_cast<const float4 *>(P.sorted);
      for (int k = h0; k < h1; k += 4) {
        // records k .. k + 3 from one base address: past the bin's last
        // hit they are the next bin's hits or the array's padding records
        // (kHitPad), read and not used
        const float4 *hk = hits + 2 * (size_t)k;
        float4 a[4];
        float4 b[4];  // (var_v, index, covariance uv, -)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          a[j] = hk[2 * j];
          b[j] = hk[2 * j + 1];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (k + j >= h1) break;
          const float c2 = hit_chi2(pr.p, f, L.kind, a[j], b[j]);
          n_near += fabsf(c2 - cut) <= band ? 1 : 0;
          if (c2 >= 0.f && c2 < cut) {
            insert_sorted(lst, ext_key(nh + 1, chi2_base + c2, slot,
                                       (unsigned)__float_as_int(b[j].y)));
            ++n_ext;
          }
        }
      }
    }
  }
}

// ------------------------------------------------------------ one step
//
// One layer step of one seed, executed by its G-lane group.  On entry each
// lane holds one candidate (or none); on exit it holds the candidate of its
// rank among the kept extensions.  pos indexes the seed's find buffers.
// cnt: the lane's counters, cnt[0] near-cut chi2 decisions, and with kMat
// cnt[1] Runge-Kutta steps and cnt[2] Newton iterations of field crossings.
template <int G, bool kMat, class Rec>
__device__ __forceinline__ void group_step(const FindParams &P, const DevLayer *sl, Cand &cd,
                                           int lane, int slot, const Rec &rec, int ev,
                                           int64_t ev_base, int step, int lid, u64 &fin_key,
                                           int *cnt, float l_hint = 0.f,
                                           int *sur = nullptr, const float2 *mtab = nullptr,
                                           const float *trig = nullptr) {
  const DevLayer &L = sl[lid];
  Prop pr;
  int st = kNoCrossing;
  if (cd.active)
    st = propagate<true, float>(cd.p, cd.c, L, P.cfg.mkb, P.cfg.l_min, true, P.cfg.edge_margin, pr,
                                l_hint, sur, nullptr, kMat ? &P.cfg.field : nullptr, trig,
                                kMat ? cnt + 1 : nullptr);
  const bool ok = cd.active && st == kOk;
  // kMat: the material map's effects and the parameterised field (a separate
  // instantiation, so that the constant-angle uniform-field form keeps its
  // register allocation)
  if (ok) {
    if constexpr (kMat) material<float>(P.cfg, L.kind, pr.p, pr.c, 1.f, nullptr, nullptr, mtab);
    else add_ms(pr.p, P.cfg.ms_var, pr.c, pr.sth, pr.cth);
  }

  u64 lst[G];  // this lane's best extensions (G >= n_cand)
#pragma unroll
  for (int i = 0; i < G; ++i) lst[i] = kKeyMax;
  int n_ext = 0;
  if (cd.active) {
    if (!ok) {
      lst[0] = ext_key(cd.nh, cd.chi2, slot, kOrderNone);  // skip (the list is empty)
      n_ext = 1;
    } else {
      Frame f;
      make_frame(pr.p, pr.c, L.kind, f);
      scan_window(P, L, ev, pr, f, cd.chi2, cd.nh, slot, lst, n_ext, cnt[0]);
      if (cd.nm < P.cfg.max_holes) {
        // a miss has one hit fewer than each of the n_ext hit extensions, so
        // it ranks after all of them
        put_at(lst, n_ext, ext_key(cd.nh, cd.chi2, slot, kOrderNone));
        ++n_ext;
      }
    }
  }

  // a candidate without any extension stops; keep the seed's best such one
  // (the group reductions below are skipped, wave-uniformly, once no lane
  // of the wavefront has anything left to contribute)
  const bool retire = cd.active && n_ext == 0;
  if (__ballot(retire) != 0ull) {
    const u64 rkey = retire ? final_key(cd.nh, cd.chi2, 1, step, slot) : kKeyMax;
    const u64 rmin = Grp<G>::min(rkey, lane);
    if (rmin < fin_key) {
      if (rkey == rmin) rec.put_fin(cd);
      fin_key = rmin;
    }
  }

  // the seed's best n_cand extensions, rank r goes to slot r (the last
  // round's winner stays on its list, which is not read again)
  u64 mine = kKeyMax;
  const int n_cand = P.cfg.n_cand;
  for (int r = 0; r < n_cand; ++r) {
    if (__ballot(lst[0] != kKeyMax) == 0ull) break;
    const u64 m = Grp<G>::min(lst[0], lane);
    if (slot == r) mine = m;
    if (r + 1 == n_cand) break;
    if (m != kKeyMax && lst[0] == m) pop_front(lst);
  }

  // the kept hit's record is requested first, so that its latency overlaps
  // the state exchange below
  const unsigned order = mine != kKeyMax ? (unsigned)(mine & 0x7FFFFFu) : kOrderNone;
  float4 ha = make_float4(0.f, 0.f, 0.f, 0.f), hb = ha;
  if (order != kOrderNone) {
    const float4 *hr = reinterpret_cast<const float4 *>(P.byorig + ev_base + order);
    ha = hr[0];
    hb = hr[1];  // (vv, index, vuv, -)
  }

  // children read their parent's propagated state (or, for a skip, its
  // unpropagated state) across the group
  // (a candidate whose propagation failed hands on its unpropagated state;
  // the selects are skipped, wave-uniformly, when no lane has one: lanes
  // without a candidate are never chosen as parents)
  float src[27];
#pragma unroll
  for (int i = 0; i < 6; ++i) src[i] = pr.p[i];
#pragma unroll
  for (int i = 0; i < 21; ++i) src[6 + i] = pr.c[i];
  if (__ballot(cd.active && !ok) != 0ull) {
#pragma unroll
    for (int i = 0; i < 6; ++i) src[i] = ok ? pr.p[i] : cd.p[i];
#pragma unroll
    for (int i = 0; i < 21; ++i) src[6 + i] = ok ? pr.c[i] : cd.c[i];
  }
  const int src_meta = cd.nh | (cd.nm << 8) | (ok ? (1 << 16) : 0);
  const int parent = mine == kKeyMax ? slot : (int)((mine >> 23) & 7);
  const int src_lane = Grp<G>::base(lane) + parent;
  float np[27];
#pragma unroll
  for (int i = 0; i < 27; ++i) np[i] = __shfl(src[i], src_lane);
  const int pmeta = __shfl(src_meta, src_lane);

  int bpv = -1;
  if (mine != kKeyMax) {
    int nh = pmeta & 0xFF, nm = (pmeta >> 8) & 0xFF;
    const bool pok = (pmeta >> 16) & 1;
    int hitcode;
    if (order != kOrderNone) {
      const float hx = ha.x, hy = ha.y, hz = ha.z, vu = ha.w, vv = hb.x, vuv = hb.z;
      Frame f;
      make_frame(np, np + 6, L.kind, f);
      float u, v;
      residual(np, f, L.kind, hx, hy, hz, u, v);
      kf_update(np, np + 6, f, L.kind, vu, vv, vuv, u, v);
      ++nh;
      hitcode = (int)order;
    } else if (pok) {
      ++nm;
      hitcode = -1;
    } else {
      hitcode = -2;
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) cd.p[i] = np[i];
#pragma unroll
    for (int i = 0; i < 21; ++i) cd.c[i] = np[6 + i];
    cd.chi2 = __uint_as_float((unsigned)(mine >> 26));
    cd.nh = nh;
    cd.nm = nm;
    cd.active = true;
    bpv = ((hitcode + 2) << 3) | parent;
  } else {
    cd.active = false;
  }
  rec.put_bp(step, slot, bpv);
}

// A seed's state; its record's last word, the index of its event's first
// hit, is returned.
__device__ __forceinline__ int load_seed(const FindParams &P, int64_t pos, Cand &cd) {
  // one seed's 28 words are contiguous: seven 16-byte loads
  const float4 *src = reinterpret_cast<const float4 *>(P.pstate + (size_t)pos * kSeedWords);
  float w[28];
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    const float4 v = src[k];
    w[4 * k] = v.x;
    w[4 * k + 1] = v.y;
    w[4 * k + 2] = v.z;
    w[4 * k + 3] = v.w;
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) cd.p[i] = w[i];
#pragma unroll
  for (int i = 0; i < 21; ++i) cd.c[i] = w[6 + i];
  cd.chi2 = 0.f;
  cd.nh = 3;
  cd.nm = 0;
  return __float_as_int(w[27]);
}

// A candidate slot's state and its meta word (hits, misses, active) as
// stored by store_cand.  The state words are requested together with the
// meta word, not after it, so that their latencies overlap (an empty
// slot's words are read and not used); the meta word is returned raw and
// unpacked by set_meta where it is first needed.
__device__ __forceinline__ int load_cand_raw(const FindParams &P, size_t idx, Cand &cd) {
  const size_t NS = (size_t)P.n_seeds * P.slots;
  const int meta = __float_as_int(P.cand[28 * NS + idx]);
#pragma unroll
  for (int i = 0; i < 6; ++i) cd.p[i] = P.cand[i * NS + idx];
#pragma unroll
  for (int i = 0; i < 21; ++i) cd.c[i] = P.cand[(6 + i) * NS + idx];
  cd.chi2 = P.cand[27 * NS + idx];
  return meta;
}
__device__ __forceinline__ void set_meta(Cand &cd, int meta) {
  cd.active = (meta >> 16) & 1;
  cd.nh = meta & 0xFF;
  cd.nm = (meta >> 8) & 0xFF;
}
__device__ __forceinline__ void load_cand(const FindParams &P, size_t idx, Cand &cd) {
  set_meta(cd, load_cand_raw(P, idx, cd));
}

__device__ __forceinline__ void store_cand(const FindParams &P, size_t idx, const Cand &cd) {
  const size_t NS = (size_t)P.n_seeds * P.slots;
  const int meta = cd.nh | (cd.nm << 8) | (cd.active ? (1 << 16) : 0);
  P.cand[28 * NS + idx] = __int_as_float(meta);
  if (cd.active) {
#pragma unroll
    for (int i = 0; i < 6; ++i) P.cand[i * NS + idx] = cd.p[i];
#pragma unroll
    for (int i = 0; i < 21; ++i) P.cand[(6 + i) * NS + idx] = cd.c[i];
    P.cand[27 * NS + idx] = cd.chi2;
  }
}

// The chosen candidate of a seed: state and counts, and its hit history
// followed back through the per-step back-pointers from (best_step,
// best_slot).  Plan steps after the candidate stopped read MKF_HIT_NONE.
template <class Rec>
__device__ __forceinline__ void write_result(const FindParams &P, int64_t pos, const Rec &rec,
                                             const float *p, const float *c, float chi2, int nh,
                                             int nm, int best_step, int best_slot, int plen) {
  float *out = P.out + (size_t)pos * kOutWords;
  float w[kOutHit];
#pragma unroll
  for (int i = 0; i < 6; ++i) w[kOutPar + i] = p[i];
#pragma unroll
  for (int i = 0; i < 21; ++i) w[kOutCov + i] = c[i];
  w[kOutChi2] = chi2;
  w[kOutMeta] = __int_as_float(nh | (nm << 8));
#pragma unroll
  for (int i = kOutMeta + 1; i < kOutHit; ++i) w[i] = 0.f;
#pragma unroll
  for (int k = 0; k < kOutHit / 4; ++k)
    reinterpret_cast<float4 *>(out)[k] = make_float4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]);
  int *hit = reinterpret_cast<int *>(out + kOutHit);
  for (int s = plen - 1; s > best_step; --s) hit[s] = MKF_HIT_NONE;
  int sl = best_slot;
  for (int s = best_step; s >= 0; --s) {
    const int v = rec.get_bp(s, sl);
    hit[s] = (v >> 3) - 2;
    sl = v & 7;
  }
}

template <class Rec>
__device__ __forceinline__ void write_retired(const FindParams &P, int64_t pos, const Rec &rec,
                                              u64 fin, int plen) {
  float p[6], c[21], chi2;
  int fm;
  rec.get_fin(p, c, chi2, fm);
  write_result(P, pos, rec, p, c, chi2, fm & 0xFF, (fm >> 8) & 0xFF, fkey_step(fin) - 1,
               fkey_slot(fin), plen);
}

template <class Rec>
__device__ __forceinline__ void write_empty(const FindParams &P, int64_t pos, const Rec &rec) {
  const float z[21] = {};
  write_result(P, pos, rec, z, z, 0.f, 0, 0, -1, 0, 0);
}

// --------------------------------------------------- layer-synchronous form

__global__ __launch_bounds__(256) void k_find_init(FindParams P) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t pos = gid / P.slots;
  const int slot = (int)(gid % P.slots);
  if (pos >= P.n_seeds) return;
  Cand cd;
  cd.active = slot == 0 && ((P.pinfo[pos] >> 8) & 1);
  cd.nh = 3;
  cd.nm = 0;
  cd.chi2 = 0.f;
  if (cd.active) load_seed(P, pos, cd);
  store_cand(P, (size_t)pos * P.slots + slot, cd);
  if (slot == 0) P.fin_key[pos] = kKeyMax;
}

// One layer step of the layer-synchronous form: G-lane seed groups,
// Grp<G>::kSeeds seeds per wavefront (lanes 60-63 idle for G = 6).
// (the uniform-field form is compiled for four waves per SIMD, which its
// load latency needs; the extended form would spill far more there)
template <bool kMat, int G>
__global__ __launch_bounds__(256, kMat ? 1 : 4) void k_find_step(FindParams P, int step,
                                                                 int64_t n_active) {
  __shared__ DevLayer sl[kMaxLayers];
  // XCD x (blocks x, x + 8, ...) takes the x-th contiguous share of the
  // positions, so that an XCD's L2 serves a few events' hits
  // (the grid is a multiple of kQueues blocks, so this is a permutation)
  const int64_t per = gridDim.x / kQueues;
  const int64_t b = (int64_t)(blockIdx.x % kQueues) * per + blockIdx.x / kQueues;
  const int lane = threadIdx.x & 63;
  const int grp = lane / G;
  const int64_t pos = (b * 4 + (threadIdx.x >> 6)) * Grp<G>::kSeeds + grp;
  const int slot = Grp<G>::slot(lane);
  // a seed group takes part while the step is in its plan (the whole group
  // leaves together); the wave stays to add its counters.  The positions
  // below n_active are the seeds whose plans are longer than step (the
  // host orders the seeds longest plan first), so every word the step
  // starts from is requested at once, without waiting for the plan length,
  // and before the block stages the layer table.
  const bool in_range = grp < Grp<G>::kSeeds && pos < n_active;
  // (the plan length is the low byte of the seed's info word, read as a
  // byte so that nothing waits on it before the barrier)
  int meta = 0, plen = 0, lid = 0, ev = 0;
  u64 fin_key = kKeyMax;
  Cand cd;
  if (in_range) {
    meta = load_cand_raw(P, (size_t)pos * G + slot, cd);
    fin_key = P.fin_key[pos];
    plen = reinterpret_cast<const unsigned char *>(P.pinfo)[4 * pos];
    lid = P.pplan[(size_t)pos * kMaxPlan + step];
    ev = P.pevent[pos];
  }
  stage_layers(P, sl);
  __syncthreads();
  if (__ballot(in_range) == 0ull) return;
  set_meta(cd, meta);
  const bool live = in_range && step < plen;
  int cnt[3] = {0, 0, 0};
  if (live) {
    const u64 fk0 = fin_key;
    group_step<G, kMat>(P, sl, cd, lane, slot, GlobalRec{&P, pos}, ev, P.ev_off[ev], step, lid,
                        fin_key, cnt);
    store_cand(P, (size_t)pos * G + slot, cd);
    if (slot == 0 && fin_key != fk0) P.fin_key[pos] = fin_key;
  }
  add_counter(P, kCntNearCut, cnt[0]);
  if constexpr (kMat) {
    add_counter(P, kCntRk, cnt[1]);
    add_counter(P, kCntNewton, cnt[2]);
  }
}

// Best of the final and the retired candidates of each seed (more hits,
// then smaller chi2) and the count of candidate-layer steps (1 for the seed
// at step 0, then every kept extension carried into the next step).  One
// lane per seed.
__global__ __launch_bounds__(256) void k_finalize(FindParams P) {
  __shared__ unsigned long long block_steps;
  if (threadIdx.x == 0) block_steps = 0;
  __syncthreads();
  const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pos < P.n_seeds) {
    const int info = P.pinfo[pos];
    const int plen = info & 0xFF;
    const bool ok = (info >> 8) & 1;
    const size_t N = (size_t)P.n_seeds;
    const int G = P.slots;
    const size_t NS = N * G;
    int cnt = (ok && plen > 0) ? 1 : 0;
    for (int s = 0; s + 1 < plen; ++s)
      for (int j = 0; j < G; ++j) cnt += P.bp[((size_t)s * N + pos) * G + j] >= 0;
    if (cnt) atomicAdd(&block_steps, (unsigned long long)cnt);
    u64 m = kKeyMax;
    int best = 0;
    if (ok)
      for (int j = 0; j < G; ++j) {
        const int meta = __float_as_int(P.cand[28 * NS + pos * G + j]);
        if (!((meta >> 16) & 1)) continue;
        const u64 fk = final_key(meta & 0xFF, P.cand[27 * NS + pos * G + j], 0, 0, j);
        if (fk < m) {
          m = fk;
          best = j;
        }
      }
    const u64 fin = ok ? P.fin_key[pos] : kKeyMax;
    const GlobalRec rec{&P, pos};
    if (m != kKeyMax && m < fin) {
      Cand cd;
      load_cand(P, (size_t)pos * G + best, cd);
      write_result(P, pos, rec, cd.p, cd.c, cd.chi2, cd.nh, cd.nm, plen - 1, best, plen);
    } else if (fin != kKeyMax) {
      write_retired(P, pos, rec, fin, plen);
    } else {
      write_empty(P, pos, rec);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && block_steps) atomicAdd(P.n_steps, block_steps);
}

// ----------------------------------------------------- persistent form
//
// Each wavefront claims tiles of 8 seeds from a counter and carries them
// through all their layer steps with the candidates in VGPRs; the seed's
// result is chosen in registers at the end.  Only the hit index, the
// back-pointers and the results touch memory.

// kWaves: the occupancy the register allocation targets (waves per SIMD);
// more waves hide more latency but spill part of the state to scratch.
// The autotuner picks the instantiation.
// kSurr: barrel propagations start from the learned surrogate's path length
// (one wave-wide matrix-core inference per layer step, then one exact Newton
// step per lane, falling back to the closed form when it does not converge).
// G: lanes per seed (8, or 6 for candidate budgets up to 6).
// kMat: with the material map and/or the parameterised field (constant
// scattering angle and uniform field otherwise).
template <int kWaves, bool kSurr, int G, bool kMat>
__device__ __forceinline__ void find_persistent(const FindParams &P) {
  __shared__ DevLayer sl[kMaxLayers];
  __shared__ unsigned long long block_steps;
  // surrogate: the network's BF16 weight images and biases, shared by the
  // block, and one activation tile per wave (the input tile overlays it)
  constexpr int kW1n = 64 * kLdW1, kW2n = 64 * kLdW2, kW3n = 32 * kLdW3;
  __shared__ __attribute__((aligned(16))) __bf16 sMW[kSurr ? kW1n + kW2n + kW3n : 8];
  __shared__ __attribute__((aligned(16))) float sMB[kSurr ? 64 + 64 + 32 : 4];
  // (one sample row per seed: at most 10 rows, one 16-sample tile per wave)
  __shared__ __attribute__((aligned(16))) __bf16 sMH[kSurr ? 4 * 16 * kLdH : 8];
  // material: a table of up to kMatLds bins is read from LDS
  constexpr int kMatLds = 1024;
  __shared__ float2 sMat[kMat ? kMatLds : 1];
  const float2 *mtab = nullptr;
  if constexpr (kMat) {
    const int nb = P.cfg.mat.nr * P.cfg.mat.nz;
    if (P.cfg.mat.tab && nb <= kMatLds) {
      for (int i = threadIdx.x; i < nb; i += blockDim.x) sMat[i] = P.cfg.mat.tab[i];
      mtab = sMat;
    }
  }
  stage_layers(P, sl);
  MlpWeights mw{};
  if constexpr (kSurr) {
    const int4 *g1 = reinterpret_cast<const int4 *>(P.mlp.W1p);
    const int4 *g2 = reinterpret_cast<const int4 *>(P.mlp.W2p);
    const int4 *g3 = reinterpret_cast<const int4 *>(P.mlp.W3p);
    int4 *d = reinterpret_cast<int4 *>(sMW);
    for (int i = threadIdx.x; i < kW1n / 8; i += blockDim.x) d[i] = g1[i];
    for (int i = threadIdx.x; i < kW2n / 8; i += blockDim.x) d[kW1n / 8 + i] = g2[i];
    for (int i = threadIdx.x; i < kW3n / 8; i += blockDim.x) d[(kW1n + kW2n) / 8 + i] = g3[i];
    for (int i = threadIdx.x; i < 64; i += blockDim.x) {
      sMB[i] = P.mlp.b1[i];
      sMB[64 + i] = P.mlp.b2[i];
      if (i < 32) sMB[128 + i] = P.mlp.b3[i];
    }
    mw = MlpWeights{sMW, sMW + kW1n, sMW + kW1n + kW2n, nullptr, nullptr, sMB, sMB + 64, sMB + 128};
  }
  if (threadIdx.x == 0) {
    block_steps = 0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int slot = Grp<G>::slot(lane);
  const int grp = lane / G;  // G = 6: lanes 60-63 form no seed group
  const int wv = threadIdx.x >> 6;
  // this wave's records in dynamic LDS: back-pointers [max_plan][kSeeds][G],
  // then the retired records [kSeeds][kFinWords]
  extern __shared__ int s_rec[];
  constexpr int kS = Grp<G>::kSeeds;
  int *wrec = s_rec + wv * persistent_rec_words(P.max_plan, G, kS);
  const int gi = grp < kS ? grp : 0;
  const LdsRec rec{wrec + gi * G, kS * G,
                   reinterpret_cast<float *>(wrec + P.max_plan * kS * G) + gi * kFinWords};
  int my_steps = 0, my_acc = 0, my_fb = 0;
  int cnt[3] = {0, 0, 0};  // near-cut decisions, field Runge-Kutta steps, Newton iterations
  int q = blockIdx.x % kQueues;  // this block's XCD
  int64_t q_lo = P.q_off[q], q_hi = P.q_off[q + 1];  // queue q's positions
  int tried = 0;
  // the next tile of queue q is claimed one tile ahead, so that the atomic's
  // latency overlaps the current tile's work (lane 0 holds it; -1: none)
  int ahead = -1;
  for (;;) {
    // (ahead is wave-uniform: a tile claimed ahead needs no wait here, so
    // the previous tile's result stores drain while this one starts)
    int tile;
    if (ahead >= 0) {
      tile = ahead;
    } else {
      int t = 0;
      if (lane == 0) t = atomicAdd(&P.tile_counter[q], 1);
      tile = __builtin_amdgcn_readfirstlane(__shfl(t, 0));
    }
    ahead = -1;
    const int64_t start = q_lo + (int64_t)tile * Grp<G>::kSeeds;
    const int64_t end = q_hi;
    if (start >= end) {
      // queue exhausted: help the next one; stop after all were tried
      if (++tried >= kQueues) break;
      q = (q + 1) % kQueues;
      q_lo = P.q_off[q];
      q_hi = P.q_off[q + 1];
      continue;
    }
    if (lane == 0 && start + Grp<G>::kSeeds < end) ahead = atomicAdd(&P.tile_counter[q], 1);
    const int64_t pos = start + grp;
    const bool valid = grp < Grp<G>::kSeeds && pos < end;
    // Every lane reads the words of an existing seed (lanes past the tile
    // read its last one and use none of it), without branches, so that the
    // seed's info word, event, state and first plan words are all requested
    // before the first wait; a seed without a fit has its state read and
    // not used.
    const int64_t pc = valid ? pos : end - 1;
    const int info_w = P.pinfo[pc];
    const int ev_w = P.pevent[pc];
    Cand cd;
    const int ev_base_w = load_seed(P, pc, cd);
    // the plan is read four layer ids at a time, one word ahead
    const int *plan_w = reinterpret_cast<const int *>(P.pplan) + (size_t)pc * (kMaxPlan / 4);
    int w_cur = plan_w[0];
    int w_next = plan_w[1];
    const int info = valid ? info_w : 0;
    const int ev = valid ? ev_w : 0;
    const int64_t ev_base = valid ? (int64_t)ev_base_w : 0;
    const int plen = info & 0xFF;
    cd.active = valid && slot == 0 && ((info >> 8) & 1);
    cd.nh = 3;
    cd.nm = 0;
    cd.chi2 = 0.f;
    u64 fin_key = kKeyMax;
    // the tile's longest plan (at most kMaxPlan = 32 steps), by a binary
    // search over ballots: no round trips through the LDS crossbar.  At
    // least one step is taken (a step beyond every plan does nothing), so
    // that the loads above are not deferred behind a test for an empty
    // tile.
    int maxlen = 1;
#pragma unroll
    for (int b = 32; b >= 1; b >>= 1)
      if (__ballot(plen >= maxlen + b) != 0ull) maxlen += b;
    // the tile claimed ahead is read now: its atomic was issued before this
    // tile's loads, so it has returned with the info word
    ahead = __builtin_amdgcn_readfirstlane(__shfl(ahead, 0));
    for (int step = 0; step < maxlen; ++step) {
      const bool in_plan = step < plen;
      if (step > 0 && (step & 3) == 0) {
        w_cur = w_next;
        w_next = step + 4 < plen ? plan_w[step / 4 + 1] : 0;
      }
      const int lid = in_plan ? (w_cur >> (8 * (step & 3))) & 0xFF : 0;
      float l_hint = 0.f;
      float trig[4];  // sin, cos of phi and theta, shared by the inputs and the propagation
      if constexpr (kSurr) {
        // The candidates of a seed all head to the same layer from nearby
        // states: the network predicts the path of the seed's leading
        // candidate (slot 0), one sample row per seed, and every candidate
        // applies that relative correction to its own straight-line path
        // and checks it with its own Newton step (falling back to the
        // closed form when the check fails).
        // (the sines and cosines are taken for every candidate that steps,
        // barrel or disk, and always handed to the propagation: a pointer
        // chosen per lane would keep the array in scratch memory)
        const bool want = in_plan && cd.active && sl[lid].kind == 0;
        const bool lead = want && slot == 0;
        float xin[kNI];
        if (in_plan && cd.active) {
          sincosf(cd.p[4], &trig[0], &trig[1]);
          sincosf(cd.p[5], &trig[2], &trig[3]);
        }
        if (lead) {
          mlp_inputs(cd.p, trig, sl[lid].pos, P.cfg.mkb, xin);
        } else {
#pragma unroll
          for (int k = 0; k < kNI; ++k) xin[k] = 0.f;
        }
        // the leading candidates write their inputs to consecutive sample
        // rows (at most 10 per wavefront: one 16-sample tile); no inference
        // at all when none heads to a barrel layer
        const unsigned long long m = __ballot(lead);
        if (m != 0ull) {
          const int base = Grp<G>::base(lane);
          const unsigned long long below = base ? (m & ((1ull << base) - 1ull)) : 0ull;
          const int row = __popcll(below);  // this seed's sample row
          __bf16 *H = sMH + wv * 16 * kLdH;
          __bf16 *X = H;  // the input tile overlays the activation tile
          if (lead) {
            bf16x8 xv;
#pragma unroll
            for (int k = 0; k < kNI; ++k) xv[k] = (__bf16)xin[k];
            *reinterpret_cast<bf16x8 *>(X + row * kLdX) = xv;
          }
          wave_sync();
          f32x4 y;
          mlp_forward16(mw, X, H, y);
          const float y0 = mlp_output16(y, row, 0);
          wave_sync();  // the tiles are rewritten at the next step
          if (want) l_hint = surrogate_path(cd.p, trig, sl[lid].pos, P.cfg.mkb, y0);
        }
      }
      if (in_plan) {
        my_steps += cd.active ? 1 : 0;
        int sur = 0;
        group_step<G, kMat>(P, sl, cd, lane, slot, rec, ev, ev_base, step, lid, fin_key, cnt,
                            l_hint, &sur, mtab, kSurr ? trig : nullptr);
        my_acc += sur == 1;
        my_fb += sur == 2;
      }
    }
    wave_sync();  // the group's records were written by its other lanes
    if (valid) {
      const u64 fk = cd.active ? final_key(cd.nh, cd.chi2, 0, 0, slot) : kKeyMax;
      const u64 m = Grp<G>::min(fk, lane);
      if (m != kKeyMax && m < fin_key) {
        if (fk == m)
          write_result(P, pos, rec, cd.p, cd.c, cd.chi2, cd.nh, cd.nm, plen - 1, slot, plen);
      } else if (slot == 0) {
        if (fin_key != kKeyMax) write_retired(P, pos, rec, fin_key, plen);
        else write_empty(P, pos, rec);
      }
    }
    wave_sync();  // read before the next tile overwrites them
  }
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) my_steps += __shfl_xor(my_steps, m);
  if (lane == 0 && my_steps) atomicAdd(&block_steps, (unsigned long long)my_steps);
  if constexpr (kSurr) {
    add_counter(P, kCntSurKept, my_acc);
    add_counter(P, kCntSurRejected, my_fb);
  }
  add_counter(P, kCntNearCut, cnt[0]);
  if constexpr (kMat) {
    add_counter(P, kCntRk, cnt[1]);
    add_counter(P, kCntNewton, cnt[2]);
  }
  __syncthreads();
  if (threadIdx.x == 0 && block_steps) atomicAdd(P.n_steps, block_steps);
}

template <int kWaves, bool kSurr, int G>
__global__ __launch_bounds__(256, kWaves) void k_find_persistent(FindParams P) {
  find_persistent<kWaves, kSurr, G, false>(P);
}

template <int kWaves, bool kSurr, int G>
__global__ __launch_bounds__(256, kWaves) void k_find_persistent_mat(FindParams P) {
  find_persistent<kWaves, kSurr, G, true>(P);
}

// Gather the seed results into processing order (untimed preparation), so
// that every read of the find is by position.
__global__ __launch_bounds__(256) void k_permute_seeds(FindParams P, float *pstate, int *pinfo,
                                                       int *pevent, int8_t *pplan) {
  const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pos >= P.n_seeds) return;
  const size_t N = (size_t)P.n_seeds;
  const int seed = P.order[pos];
  for (int i = 0; i < 27; ++i) pstate[(size_t)pos * kSeedWords + i] = P.seed_state[i * N + seed];
  // the last word: the index of the event's first hit (below 2^31), read
  // with the state so that the find need not look it up
  pstate[(size_t)pos * kSeedWords + 27] = __int_as_float((int)P.ev_off[P.seed_event[seed]]);
  pinfo[pos] = P.plan_len[seed] | (P.seed_ok[seed] << 8);
  pevent[pos] = P.seed_event[seed];
  for (int s = 0; s < kMaxPlan; ++s)
    pplan[(size_t)pos * kMaxPlan + s] = P.plan[(size_t)seed * kMaxPlan + s];
}

// --------------------------------------------------------------- seeding
//
// Seeds come from outside (Section 2.2).  The circle through the three
// transverse points gives the centre and radius, the turning sense the
// charge, the tangent at the first hit phi, and the z rise over the arc
// theta.  A wide diagonal prior at the first hit is filtered through the
// three hits.  The layer plan is the paper's per-region list of layers to
// traverse (Section 2.1): with region steering, the list of the region that
// holds the seed's pseudorapidity, less the seed layers; without, it is built
// per seed: every other layer the seed helix crosses inside its widened
// extent, by increasing path length.

__global__ __launch_bounds__(256) void k_seed(FindParams P, const int *seed_hits,
                                              float *seed_state, int *seed_ok, int *plan_len,
                                              int8_t *plan, double *plan_l, float *seed_chi2,
                                              const DevRegion *regions, int n_regions) {
  __shared__ DevLayer sl[kMaxLayers];
  stage_layers(P, sl);
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.n_seeds) return;
  const size_t N = (size_t)P.n_seeds;
  const int ev = P.seed_event[i];
  const int64_t e0 = P.ev_off[ev];
  // FP64: three updates shrink the wide prior by ~5 decades, more than FP32
  // keeps in C - K S K^T; the result is rounded to FP32 for the find
  double hx[3], hy[3], hz[3], hvu[3], hvv[3];
  int hl[3];
  for (int k = 0; k < 3; ++k) {
    const int64_t g = e0 + seed_hits[3 * i + k];
    hx[k] = P.hx[g];
    hy[k] = P.hy[g];
    hz[k] = P.hz[g];
    hvu[k] = P.hvu[g];
    hvv[k] = P.hvv[g];
    hl[k] = P.hlayer[g];
  }
  const double mkb = P.cfg.mkb, l_min = P.cfg.l_min, edge = P.cfg.edge_margin;
  int ok = 0;
  int n = 0;
  double p[6], c[21], chi2 = 0.0;
  do {
    const double ax = hx[1] - hx[0], ay = hy[1] - hy[0];
    const double bx = hx[2] - hx[0], by = hy[2] - hy[0];
    const double d = 2.0 * (ax * by - ay * bx);
    if (d == 0.0 || mkb == 0.0) break;
    const double a2 = ax * ax + ay * ay, b2 = bx * bx + by * by;
    const double ux = (by * a2 - ay * b2) / d;
    const double uy = (ax * b2 - bx * a2) / d;
    const double cx = hx[0] + ux, cy = hy[0] + uy;
    const double rho = sqrt(ux * ux + uy * uy);
    const double turn = (hx[1] - hx[0]) * (hy[2] - hy[1]) - (hy[1] - hy[0]) * (hx[2] - hx[1]);
    const bool ccw = turn > 0.0;  // omega > 0
    // omega = mkb * ipt and |omega| = 1/rho; a parameterised field is taken
    // at the middle hit
    const double mkb_s = P.cfg.field.on ? field_mkb(P.cfg.field, hx[1], hy[1], hz[1]) : mkb;
    if (mkb_s == 0.0) break;
    const double ipt = (ccw ? 1.0 : -1.0) / (mkb_s * rho);
    const double r1x = hx[0] - cx, r1y = hy[0] - cy;
    const double dirx = ccw ? -r1y : r1y, diry = ccw ? r1x : -r1x;
    const double phi1 = atan2(diry, dirx);
    const double r3x = hx[2] - cx, r3y = hy[2] - cy;
    const double dpsi = atan2(r1x * r3y - r1y * r3x, r1x * r3x + r1y * r3y);
    const double theta = atan2(rho * fabs(dpsi), hz[2] - hz[0]);
    p[0] = hx[0]; p[1] = hy[0]; p[2] = hz[0]; p[3] = ipt; p[4] = phi1; p[5] = theta;
    surface_prior(P.cfg, p, sl[hl[0]].kind, c);
    chi2 = 0.0;
    bool good = true;
    for (int k = 0; k < 3 && good; ++k) {
      const DevLayer &L = sl[hl[k]];
      if (k > 0) {
        PropT<double> pr;
        if (propagate<true, double>(p, c, L, mkb, l_min, false, 0.0, pr, 0.0, nullptr, nullptr,
                                    &P.cfg.field) != kOk) {
          good = false;
          break;
        }
        for (int q = 0; q < 6; ++q) p[q] = pr.p[q];
        for (int q = 0; q < 21; ++q) c[q] = pr.c[q];
      }
      material<double>(P.cfg, L.kind, p, c, 1.0);
      FrameT<double> f;
      make_frame(p, c, L.kind, f);
      double u, v;
      if (!residual(p, f, L.kind, hx[k], hy[k], hz[k], u, v)) {
        good = false;
        break;
      }
      double vuu, vvv, vuv;
      hit_cov((double)L.cs, (double)L.sn, hvu[k], hvv[k], vuu, vvv, vuv);
      chi2 += chi2_of(f, vuu, vvv, vuv, u, v);
      kf_update(p, c, f, L.kind, vuu, vvv, vuv, u, v);
    }
    if (!good) break;
    ok = 1;
    if (n_regions > 0) {
      const double eta = -log(tan(0.5 * p[5]));
      int r = 0;
      while (r < n_regions && !(eta >= regions[r].eta_lo && eta < regions[r].eta_hi)) ++r;
      if (r < n_regions) {
        const DevRegion &g = regions[r];
        for (int k = 0; k < g.n && n < kMaxPlan; ++k) {
          const int L = g.layers[k];
          if (L == hl[0] || L == hl[1] || L == hl[2]) continue;
          plan[i * kMaxPlan + n++] = (int8_t)L;
        }
      }
      break;
    }
    // plan: insertion by path length (ties by layer id) into global scratch
    for (int L = 0; L < P.n_layers; ++L) {
      if (L == hl[0] || L == hl[1] || L == hl[2]) continue;
      PropT<double> pr;
      if (propagate<false, double>(p, nullptr, sl[L], mkb, l_min, true, edge, pr, 0.0, nullptr,
                                   nullptr, &P.cfg.field) != kOk)
        continue;
      if (n >= kMaxPlan) break;
      const double lf = pr.l;
      int j = n;
      while (j > 0 && plan_l[i * kMaxPlan + j - 1] > lf) {
        plan_l[i * kMaxPlan + j] = plan_l[i * kMaxPlan + j - 1];
        plan[i * kMaxPlan + j] = plan[i * kMaxPlan + j - 1];
        --j;
      }
      plan_l[i * kMaxPlan + j] = lf;
      plan[i * kMaxPlan + j] = (int8_t)L;
      ++n;
    }
  } while (false);
  seed_ok[i] = ok;
  seed_chi2[i] = ok ? (float)chi2 : 0.f;
  plan_len[i] = ok ? n : 0;
  for (int k = 0; k < 6; ++k) seed_state[k * N + i] = ok ? (float)p[k] : 0.f;
  for (int k = 0; k < 21; ++k) seed_state[(6 + k) * N + i] = ok ? (float)c[k] : 0.f;
}

// ------------------------------------------------------------- hit index

__device__ __forceinline__ int event_of(const int64_t *ev_off, int n_events, int64_t i) {
  int lo = 0, hi = n_events;  // ev_off[lo] <= i < ev_off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (ev_off[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int bin_of(const DevLayer &L, float x, float y, float z) {
  const float phi = atan2f(y, x);
  const int pb = clampi((int)floorf((phi + kPi) * L.phi_scale), 0, L.nphi - 1);
  const float q = L.kind == 0 ? z : sqrtf(fmaf(x, x, y * y));
  const int qb = clampi((int)floorf((q - L.q_lo) * L.q_scale), 0, L.nq - 1);
  return L.bin_base + qb * L.nphi + pb;
}

// ------------------------------------------------------ triplet seeding
//
// The paper takes seeds from outside (Section 2.2); this builds them from
// the hits.  A seed is a triplet of hits a, b, c on three barrel layers
// (innermost first) whose helix is a plausible track from the beam line:
// with the circle through the three transverse points (centre c0, radius
// rho), pT = kappa |B| rho >= pt_min; the circle passes within d0_max of the
// beam line; a, b, c follow each other in the turning sense within half a
// turn; b lies within dz_max of the s-z line through a and c; and that line
// has |z| <= z0_max at the point of closest approach to the beam line, which
// precedes a within half a turn.  The cuts are evaluated in FP64.
//
// One thread per hit of the first layer walks the second layer's hits in an
// azimuth window (every z bin), drops pairs whose straight-line z at the beam
// line is far outside z0_max, and walks the third layer's hits in an azimuth
// and z window around the pair's extrapolation.  The windows only bound the
// search (their margins cover curvature, d0 and dz); the cuts decide.

// exact cuts of one triplet (FP64)
__device__ __forceinline__ bool triplet_passes(const DevCfg &cfg, const DevSeeding &sc, double ax,
                                               double ay, double az, double bx, double by,
                                               double bz, double cx, double cy, double cz) {
  const double ux0 = bx - ax, uy0 = by - ay, vx0 = cx - ax, vy0 = cy - ay;
  const double cr = ux0 * vy0 - uy0 * vx0;
  if (cr == 0.0) return false;
  const double u2 = ux0 * ux0 + uy0 * uy0, v2 = vx0 * vx0 + vy0 * vy0;
  const double ox = ax + (vy0 * u2 - uy0 * v2) / (2.0 * cr);
  const double oy = ay + (ux0 * v2 - vx0 * u2) / (2.0 * cr);
  const double rho = sqrt((ox - ax) * (ox - ax) + (oy - ay) * (oy - ay));
  // kappa |B| = |mkb|
  if (fabs((double)cfg.mkb) * rho < (double)sc.pt_min) return false;
  const double dist = sqrt(ox * ox + oy * oy);
  if (dist == 0.0 || fabs(dist - rho) > (double)sc.d0_max) return false;
  const double sg = cr > 0.0 ? 1.0 : -1.0;
  const double two_pi = 6.283185307179586;
  const double qa = atan2(ay - oy, ax - ox), qb = atan2(by - oy, bx - ox);
  const double qc = atan2(cy - oy, cx - ox), q0 = atan2(-oy, -ox);
  auto turn = [&](double from, double to) {
    double t = sg * (to - from);
    if (t < 0.0) t += two_pi;
    if (t < 0.0) t += two_pi;
    return t;
  };
  const double pab = turn(qa, qb), pac = turn(qa, qc), p0a = turn(q0, qa);
  const double pi = 3.141592653589793;
  if (!(pab > 0.0 && pac > pab && pac < pi && p0a < pi)) return false;
  const double slope = (cz - az) / (rho * pac);
  const double dz = bz - (az + slope * rho * pab);
  if (fabs(dz) > (double)sc.dz_max) return false;
  const double z0 = az - slope * rho * p0a;
  return fabs(z0) <= (double)sc.z0_max;
}

// the bin rows [qlo, qhi] x azimuth window [phi - dphi, phi + dphi] of one
// layer (two azimuth segments where it wraps); fn(hit record) per hit
template <class Fn>
__device__ __forceinline__ void walk_window(const FindParams &P, const DevLayer &L, int ev, float phi,
                                            float dphi, int qlo, int qhi, Fn fn) {
  const int nphi = L.nphi;
  int s0lo = 0, s0hi = nphi - 1, s1lo = 1, s1hi = 0;
  if (dphi < kPi) {
    const int blo = (int)floorf((phi - dphi + kPi) * L.phi_scale);
    const int bhi = (int)floorf((phi + dphi + kPi) * L.phi_scale);
    if (bhi - blo + 1 < nphi) {
      if (blo < 0) {
        s0lo = blo + nphi; s1lo = 0; s1hi = bhi;
      } else if (bhi >= nphi) {
        s0lo = blo; s1lo = 0; s1hi = bhi - nphi;
      } else {
        s0lo = blo; s0hi = bhi;
      }
    }
  }
  const int base = ev * P.bins_per_event + L.bin_base;
  for (int qb = qlo; qb <= qhi; ++qb) {
    const int row = base + qb * nphi;
    for (int sg = 0; sg < 2; ++sg) {
      const int lo = sg == 0 ? s0lo : s1lo, hi = sg == 0 ? s0hi : s1hi;
      if (lo > hi) continue;
      const int h0 = P.bin_start[row + lo], h1 = P.bin_start[row + hi + 1];
      for (int k = h0; k < h1; ++k) fn(P.sorted[k]);
    }
  }
}

// azimuth change between radii r0 < r1 of a circle of radius >= rho_min
// passing within d0 of the beam line, with room for rounding
__device__ __forceinline__ float bend_window(float r0, float r1, float rho_min, float d0) {
  const float s0 = fminf(1.f, r0 / (2.f * rho_min)), s1 = fminf(1.f, r1 / (2.f * rho_min));
  return asinf(s1) - asinf(s0) + d0 / r0 + d0 / r1 + 2e-3f;
}

// One thread per first-layer hit, taken in the hit index's order within
// its event (blockIdx.y), so that neighbouring lanes walk neighbouring
// windows; counts and offsets are indexed by that sorted position.
template <bool kWrite>
__global__ __launch_bounds__(256) void k_triplets(FindParams P, DevSeeding sc, int *counts,
                                                  const int *offsets, int *out_event,
                                                  int *out_hits) {
  __shared__ DevLayer sl[kMaxLayers];
  stage_layers(P, sl);
  __syncthreads();
  const int e = blockIdx.y;
  const DevLayer &L0 = sl[sc.layer[0]], &L1 = sl[sc.layer[1]], &L2 = sl[sc.layer[2]];
  const int first = e * P.bins_per_event + L0.bin_base;
  const int idx = P.bin_start[first] + blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= P.bin_start[first + L0.nq * L0.nphi]) return;
  const HitRec ha = P.sorted[idx];
  const float ax = ha.x, ay = ha.y, az = ha.z;
  const float ra = sqrtf(fmaf(ax, ax, ay * ay));
  const float rho_min = sc.pt_min / fabsf(P.cfg.mkb);
  const float R0 = L0.pos, R1 = L1.pos, R2 = L2.pos;
  const float dphi1 = bend_window(R0, R1, rho_min, sc.d0_max);
  const float dphi2 = bend_window(R1, R2, rho_min, sc.d0_max);
  const int pos = kWrite ? offsets[idx] : 0;
  int n = 0;
  walk_window(P, L1, e, atan2f(ay, ax), dphi1, 0, L1.nq - 1, [&](const HitRec &hb) {
    const float rb = sqrtf(fmaf(hb.x, hb.x, hb.y * hb.y));
    const float Z = hb.z - az;
    const float lever = ra / (rb - ra);
    // straight-line z at the beam line, against z0_max with room for the
    // arc-versus-radius differences (d0, bending) and dz
    const float z0e = az - Z * lever;
    if (fabsf(z0e) > sc.z0_max + 1.f + (0.1f * fabsf(Z) + sc.dz_max) * (lever + 1.f)) return;
    const float k = (R2 - ra) / (rb - ra);
    const float zp = az + Z * k;
    const float hw = (0.1f * fabsf(Z) + 2.f * sc.dz_max) * k + 0.5f;
    const int qlo = clampi((int)floorf((zp - hw - L2.q_lo) * L2.q_scale), 0, L2.nq - 1);
    const int qhi = clampi((int)floorf((zp + hw - L2.q_lo) * L2.q_scale), 0, L2.nq - 1);
    walk_window(P, L2, e, atan2f(hb.y, hb.x), dphi2, qlo, qhi, [&](const HitRec &hc) {
      if (!triplet_passes(P.cfg, sc, ax, ay, az, hb.x, hb.y, hb.z, hc.x, hc.y, hc.z)) return;
      if (kWrite) {
        out_event[pos + n] = e;
        out_hits[3 * (size_t)(pos + n)] = ha.orig;
        out_hits[3 * (size_t)(pos + n) + 1] = hb.orig;
        out_hits[3 * (size_t)(pos + n) + 2] = hc.orig;
      }
      ++n;
    });
  });
  if (!kWrite) counts[idx] = n;
}

// ---------------------------------------------------- duplicate removal
//
// Removal of duplicate tracks (the paper lists it as not yet done,
// Introduction and Section 3).  The hits of a track are its three seed hits
// and its found hits.  Track u ranks before t if it has more hits; with as
// many, a smaller chi2; with the same chi2, a lexicographically smaller seed
// triplet.  t is a duplicate if a track ranking before it shares at least
// frac of the hits of the shorter of the two.  Tracks that share a hit are
// found through a hit -> tracks table (CSR over all hits of all events).

// per track: its hits as global indices, sorted, and their use counts
__global__ __launch_bounds__(256) void k_dup_prep(FindParams P, const int *seed_hits, int *hbuf,
                                                  int *hn, int *cnt) {
  const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pos >= P.n_seeds) return;
  const int info = P.pinfo[pos];
  int n = 0;
  if ((info >> 8) & 1) {
    const int plen = info & 0xFF;
    const int *hit = reinterpret_cast<const int *>(P.out + (size_t)pos * kOutWords + kOutHit);
    const int64_t base = P.ev_off[P.pevent[pos]];
    const int *sh = seed_hits + (size_t)P.order[pos] * 3;
    int *h = hbuf + (size_t)pos * kDupStride;
    auto insert = [&](int v) {  // insertion into the sorted prefix
      int j = n;
      while (j > 0 && h[j - 1] > v) {
        h[j] = h[j - 1];
        --j;
      }
      h[j] = v;
      ++n;
    };
    for (int k = 0; k < 3; ++k) insert((int)(base + sh[k]));
    for (int s = 0; s < plen; ++s)
      if (hit[s] >= 0) insert((int)(base + hit[s]));
    for (int k = 0; k < n; ++k) atomicAdd(&cnt[h[k]], 1);
  }
  hn[pos] = n;
}

__global__ __launch_bounds__(256) void k_dup_fill(FindParams P, const int *hbuf, const int *hn,
                                                  const int *off, int *fill, int *list) {
  const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pos >= P.n_seeds) return;
  const int *h = hbuf + (size_t)pos * kDupStride;
  for (int k = 0; k < hn[pos]; ++k) list[off[h[k]] + atomicAdd(&fill[h[k]], 1)] = (int)pos;
}

__global__ __launch_bounds__(256) void k_dup_decide(FindParams P, const int *seed_hits,
                                                    const int *hbuf, const int *hn, const int *off,
                                                    const int *list, float frac, int *out_dup,
                                                    int *n_dup) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= P.n_seeds) return;
  const int nt = hn[t];
  const int seed_t = P.order[t];
  bool dup = false;
  if (nt > 0) {
    const int *ht = hbuf + (size_t)t * kDupStride;
    const float chi_t = P.out[(size_t)t * kOutWords + kOutChi2];
    const int *st = seed_hits + (size_t)seed_t * 3;
    for (int k = 0; k < nt && !dup; ++k) {
      const int g = ht[k];
      for (int j = off[g]; j < off[g + 1] && !dup; ++j) {
        const int u = list[j];
        if (u == t) continue;
        // shared hits, and the first of them in t's list: each partner is
        // weighed once, at the first hit the two share
        const int *hu = hbuf + (size_t)u * kDupStride;
        const int nu = hn[u];
        int a = 0, b = 0, shared = 0, first = -1;
        while (a < nt && b < nu) {
          const int x = ht[a], y = hu[b];
          if (x == y) {
            if (first < 0) first = a;
            ++shared;
            ++a;
            ++b;
          } else if (x < y) {
            ++a;
          } else {
            ++b;
          }
        }
        if (first != k) continue;
        const int mn = nt < nu ? nt : nu;
        if ((double)shared < (double)frac * (double)mn) continue;
        bool before;
        if (nu != nt) {
          before = nu > nt;
        } else {
          const float chi_u = P.out[(size_t)u * kOutWords + kOutChi2];
          if (chi_u != chi_t) {
            before = chi_u < chi_t;
          } else {
            const int *su = seed_hits + (size_t)P.order[u] * 3;
            int q = 0;
            while (q < 3 && su[q] == st[q]) ++q;
            before = q < 3 && su[q] < st[q];
          }
        }
        dup = before;
      }
    }
  }
  out_dup[seed_t] = dup ? 1 : 0;
  if (dup) atomicAdd(n_dup, 1);
}

// -------------------------------------------------------- seed cleaning
//
// Seed cleaning (Section 2.2: seeds built from hits of the same outgoing
// particle are reduced to one, using the identity of their hits and their
// fitted pT, eta and phi).  Seeds sharing a hit are instances of one
// particle if their fitted q/pT agree within tol_ipt (relative to the
// larger), eta within tol_eta and phi within tol_phi.  Seed u ranks before t
// if its fit chi2 is smaller; with the same chi2, if its hit triplet is
// lexicographically smaller.  t is kept if its fit succeeded and no seed
// ranking before it is an instance of the same particle.  Seeds sharing a
// hit are found through a hit -> seeds table, as for duplicate tracks.

__global__ __launch_bounds__(256) void k_clean_prep(FindParams P, const int *seed_hits, int *hbuf,
                                                    int *cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.n_seeds) return;
  int h[3] = {-1, -1, -1};
  if (P.seed_ok[i]) {
    const int64_t base = P.ev_off[P.seed_event[i]];
#pragma unroll
    for (int k = 0; k < 3; ++k) h[k] = (int)(base + seed_hits[3 * i + k]);
    // sort three
    if (h[0] > h[1]) { const int t = h[0]; h[0] = h[1]; h[1] = t; }
    if (h[1] > h[2]) { const int t = h[1]; h[1] = h[2]; h[2] = t; }
    if (h[0] > h[1]) { const int t = h[0]; h[0] = h[1]; h[1] = t; }
#pragma unroll
    for (int k = 0; k < 3; ++k) atomicAdd(&cnt[h[k]], 1);
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) hbuf[3 * i + k] = h[k];
}

__global__ __launch_bounds__(256) void k_clean_fill(FindParams P, const int *hbuf, const int *off,
                                                    int *fill, int *list) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.n_seeds || hbuf[3 * i] < 0) return;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int g = hbuf[3 * i + k];
    list[off[g] + atomicAdd(&fill[g], 1)] = (int)i;
  }
}

__device__ __forceinline__ float eta_of(float theta) { return -logf(tanf(0.5f * theta)); }

__global__ __launch_bounds__(256) void k_clean_decide(FindParams P, const int *seed_hits,
                                                      const float *seed_chi2, const int *hbuf,
                                                      const int *off, const int *list,
                                                      DevCleaning cc, int *out_keep,
                                                      int *n_keep) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= P.n_seeds) return;
  bool keep = P.seed_ok[t] != 0;
  if (keep) {
    const size_t N = (size_t)P.n_seeds;
    const float ipt_t = P.seed_state[3 * N + t], phi_t = P.seed_state[4 * N + t];
    const float eta_t = eta_of(P.seed_state[5 * N + t]);
    const float chi_t = seed_chi2[t];
    const int *ht = hbuf + 3 * t;
    for (int k = 0; k < 3 && keep; ++k) {
      const int g = ht[k];
      for (int j = off[g]; j < off[g + 1] && keep; ++j) {
        const int u = list[j];
        if (u == t) continue;
        // weigh each partner once, at the first hit the two share
        const int *hu = hbuf + 3 * (size_t)u;
        int first = -1;
        for (int a = 0; a < 3 && first < 0; ++a)
          if (ht[a] == hu[0] || ht[a] == hu[1] || ht[a] == hu[2]) first = a;
        if (first != k) continue;
        const float ipt_u = P.seed_state[3 * N + u];
        if (fabsf(ipt_t - ipt_u) > cc.tol_ipt * fmaxf(fabsf(ipt_t), fabsf(ipt_u))) continue;
        if (fabsf(eta_t - eta_of(P.seed_state[5 * N + u])) > cc.tol_eta) continue;
        if (fabsf(wrap_phi(phi_t - P.seed_state[4 * N + u])) > cc.tol_phi) continue;
        const float chi_u = seed_chi2[u];
        bool before;
        if (chi_u != chi_t) {
          before = chi_u < chi_t;
        } else {
          const int *su = seed_hits + 3 * (size_t)u, *st = seed_hits + 3 * t;
          int q = 0;
          while (q < 3 && su[q] == st[q]) ++q;
          before = q < 3 && su[q] < st[q];
        }
        if (before) keep = false;
      }
    }
  }
  out_keep[t] = keep ? 1 : 0;
  if (keep) atomicAdd(n_keep, 1);
}

__global__ __launch_bounds__(256) void k_hit_bins(FindParams P, int n_events, int64_t n_hits,
                                                  const int *layer, int *hit_bin, int *counts) {
  __shared__ DevLayer sl[kMaxLayers];
  stage_layers(P, sl);
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_hits) return;
  const int e = event_of(P.ev_off, n_events, i);
  const int b = e * P.bins_per_event + bin_of(sl[layer[i]], P.hx[i], P.hy[i], P.hz[i]);
  hit_bin[i] = b;
  atomicAdd(&counts[b], 1);
}

__global__ __launch_bounds__(256) void k_hit_scatter(FindParams P, int n_events, int64_t n_hits,
                                                     const int *hit_bin, int *fill,
                                                     HitRec *sorted, HitRec *byorig) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_hits) return;
  const int e = event_of(P.ev_off, n_events, i);
  const int b = hit_bin[i];
  const int slot = P.bin_start[b] + atomicAdd(&fill[b], 1);
  HitRec h;
  h.x = P.hx[i];
  h.y = P.hy[i];
  h.z = P.hz[i];
  const DevLayer &L = P.layers[P.hlayer[i]];
  hit_cov(L.cs, L.sn, P.hvu[i], P.hvv[i], h.vu, h.vv, h.vuv);
  h.orig = (int)(i - P.ev_off[e]);
  h.pad1 = 0;
  sorted[slot] = h;
  byorig[i] = h;
}

// exclusive scan, 2048 items per 256-thread block
constexpr int kScanItems = 8;
constexpr int kScanBlock = 256 * kScanItems;

__global__ __launch_bounds__(256) void k_block_scan(const int *in, int *out, int64_t n,
                                                    int *block_sums) {
  __shared__ int wsum[4];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
  int v[kScanItems];
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = base + k < n ? in[base + k] : 0;
    s += v[k];
  }
  // inclusive scan of s over the block
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int incl = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o);
    if (lane >= o) incl += t;
  }
  if (lane == 63) wsum[wid] = incl;
  __syncthreads();
  int woff = 0;
  for (int w = 0; w < wid; ++w) woff += wsum[w];
  int run = woff + incl - s;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == 255) block_sums[blockIdx.x] = woff + incl;
}

__global__ __launch_bounds__(256) void k_add_offsets(int *out, int64_t n, const int *offs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] += offs[i / kScanBlock];
}

__global__ void k_set_total(int *out, int64_t n, const int *block_sums, const int *scanned,
                            int64_t nb) {
  out[n] = nb == 1 ? block_sums[0] : scanned[nb];
}

// --------------------------------------------------------- unit kernels

__global__ __launch_bounds__(256) void k_propagate(FindParams P, int64_t n, const float *par,
                                                   const float *cov, const int *layer,
                                                   float *out_par, float *out_cov, float *out_l,
                                                   int *out_status) {
  __shared__ DevLayer sl[kMaxLayers];
  stage_layers(P, sl);
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float p[6], c[21];
  for (int k = 0; k < 6; ++k) p[k] = par[i * 6 + k];
  for (int k = 0; k < 21; ++k) c[k] = cov[i * 21 + k];
  const int lid = layer[i];
  Prop pr;
  const int st = (lid < 0 || lid >= P.n_layers)
                     ? 3
                     : propagate<true, float>(p, c, sl[lid], P.cfg.mkb, P.cfg.l_min, true,
                                       P.cfg.edge_margin, pr, 0.f, nullptr, nullptr,
                                       &P.cfg.field);
  out_status[i] = st;
  for (int k = 0; k < 6; ++k) out_par[i * 6 + k] = st == kOk ? pr.p[k] : 0.f;
  for (int k = 0; k < 21; ++k) out_cov[i * 21 + k] = st == kOk ? pr.c[k] : 0.f;
  out_l[i] = st == kOk ? pr.l : 0.f;
}

// Search-free Kalman fit: one lane per track, the hit loop in registers;
// the per-step inputs are step-major so each step is a coalesced read.
__global__ __launch_bounds__(256) void k_fit(DevCfg cfg, int64_t n, int n_steps,
                                             const int8_t *kind, const float *pos,
                                             const float *x, const float *y, const float *z,
                                             const float *vu, const float *vv, const int *len,
                                             const float *init_par, const float *init_cov,
                                             float *out_par, float *out_cov, float *out_chi2,
                                             int *out_status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float p[6], c[21];
#pragma unroll
  for (int k = 0; k < 6; ++k) p[k] = init_par[i * 6 + k];
#pragma unroll
  for (int k = 0; k < 21; ++k) c[k] = init_cov[i * 21 + k];
  float chi2 = 0.f;
  int status = 0;
  const int m = min(len[i], n_steps);
  // a step's surface and hit are requested one step ahead, while the step
  // before computes (the last step's words are requested twice, so that
  // every step issues the same loads)
  int nk = 0;
  float npos = 0.f, nx = 0.f, ny = 0.f, nz = 0.f, nvu = 0.f, nvv = 0.f;
  auto fetch = [&](int s) {
    const size_t j = (size_t)s * (size_t)n + i;
    nk = kind[j];
    npos = pos[j];
    nx = x[j];
    ny = y[j];
    nz = z[j];
    nvu = vu[j];
    nvv = vv[j];
  };
  if (m > 0) fetch(0);
  for (int s = 0; s < m; ++s) {
    DevLayer L;
    L.kind = nk;
    L.pos = npos;
    L.lo = 0.f;
    L.hi = 0.f;
    const float hx = nx, hy = ny, hz = nz, hvu = nvu, hvv = nvv;
    fetch(min(s + 1, m - 1));
    Prop pr;
    if (propagate<true, float>(p, c, L, cfg.mkb, cfg.l_min, false, 0.f, pr, 0.f, nullptr, nullptr,
                        &cfg.field) != kOk) {
      status = s + 1;
      break;
    }
    material(cfg, L.kind, pr.p, pr.c, 1.f);
    Frame f;
    make_frame(pr.p, pr.c, L.kind, f);
    float u, v;
    if (!residual(pr.p, f, L.kind, hx, hy, hz, u, v)) {
      status = s + 1;
      break;
    }
    chi2 += fmaxf(chi2_of(f, hvu, hvv, 0.f, u, v), 0.f);
    kf_update(pr.p, pr.c, f, L.kind, hvu, hvv, 0.f, u, v);
#pragma unroll
    for (int k = 0; k < 6; ++k) p[k] = pr.p[k];
#pragma unroll
    for (int k = 0; k < 21; ++k) c[k] = pr.c[k];
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) out_par[i * 6 + k] = p[k];
#pragma unroll
  for (int k = 0; k < 21; ++k) out_cov[i * 21 + k] = c[k];
  out_chi2[i] = chi2;
  out_status[i] = status;
}

// ---------------------------------------------------------- backward fit
//
// The layer plan's steering marks layers used only when a track is fitted
// backwards (Section 2.1).  A found track is fitted backwards by the same
// Kalman filter (Introduction) run over its hits in the reverse order: its
// crossed plan layers from the last to the first, then its three seed
// layers from the third to the first.  The filter starts at the first of
// these surfaces from the track's final state, with the seed prior less its
// extent along that surface's normal, and on every surface it propagates
// (from the second on), adds the layer's scattering and takes the hit if
// the surface has one.  Backward propagation is forward propagation of the
// reversed helix (opposite charge, opposite direction).

// q/pT -> -q/pT, phi -> phi + pi, theta -> pi - theta; the covariance
// becomes D C D with D = diag(1, 1, 1, -1, 1, -1)
template <typename T>
__device__ __forceinline__ void flip_state(T *p, T *c) {
  p[3] = -p[3];
  p[4] = p[4] > T(0) ? p[4] - Consts<T>::pi() : p[4] + Consts<T>::pi();
  p[5] = Consts<T>::pi() - p[5];
  c[tri(0, 3)] = -c[tri(0, 3)];
  c[tri(1, 3)] = -c[tri(1, 3)];
  c[tri(2, 3)] = -c[tri(2, 3)];
  c[tri(3, 4)] = -c[tri(3, 4)];
  c[tri(0, 5)] = -c[tri(0, 5)];
  c[tri(1, 5)] = -c[tri(1, 5)];
  c[tri(2, 5)] = -c[tri(2, 5)];
  c[tri(4, 5)] = -c[tri(4, 5)];
}

// One surface of the backward fit: propagate the reversed helix to it
// (except on the first), add its scattering, take its hit (code >= 0).
// Returns false if the surface is not reached or the hit lies in the
// other half of the layer.
template <typename T>
__device__ __forceinline__ bool backfit_surface(const FindParams &P, const DevLayer &L,
                                                bool first, int code, int64_t ev_base, T *p,
                                                T *c, float &chi2) {
  if (first) {
    surface_prior(P.cfg, p, L.kind, c);
  } else {
    flip_state(p, c);
    PropT<T> pr;
    if (propagate<true, T>(p, c, L, T(P.cfg.mkb), T(P.cfg.l_min), false, T(0), pr, T(0), nullptr,
                           nullptr, &P.cfg.field) != kOk)
      return false;
#pragma unroll
    for (int m = 0; m < 6; ++m) p[m] = pr.p[m];
#pragma unroll
    for (int m = 0; m < 21; ++m) c[m] = pr.c[m];
    flip_state(p, c);
  }
  // on the way back the track regains the layer's loss
  material<T>(P.cfg, L.kind, p, c, T(-1));
  if (code >= 0) {
    const HitRec h = P.byorig[ev_base + code];
    FrameT<T> f;
    make_frame(p, c, L.kind, f);
    T u, v;
    if (!residual(p, f, L.kind, T(h.x), T(h.y), T(h.z), u, v)) return false;
    chi2 += fmaxf((float)chi2_of(f, T(h.vu), T(h.vv), T(h.vuv), u, v), 0.f);
    kf_update(p, c, f, L.kind, T(h.vu), T(h.vv), T(h.vuv), u, v);
  }
  return true;
}

// Surface t of a track's backward sequence: plan step t - 3 for t >= 3,
// seed hit t below.  False for a plan step the track did not cross.
__device__ __forceinline__ bool backfit_seq(const FindParams &P, const int *hit,
                                            const int8_t *plan, const int *sh, int64_t ev_base,
                                            int t, int &lid, int &code) {
  if (t >= 3) {
    code = hit[t - 3];
    lid = plan[t - 3];
    return code >= MKF_HIT_MISS;  // not crossed, or after the track ended
  }
  code = sh[t];
  lid = P.hlayer[ev_base + code];
  return true;
}

// Carried from the FP64 head to the FP32 tail, per processing position:
// state and covariance (27 words), chi2, then status, surfaces done and the
// next sequence index as integers.
constexpr int kBfWords = 32;

// Head, one lane per seed: as in the seed fit, the wide prior is filtered
// through the track's first three hits in FP64 (they shrink it by ~5
// decades, more than FP32 keeps in the covariance update).
__global__ __launch_bounds__(256) void k_backfit_head(FindParams P, const int *seed_hits,
                                                      float *tmp) {
  __shared__ DevLayer sl[kMaxLayers];
  stage_layers(P, sl);
  __syncthreads();
  const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pos >= P.n_seeds) return;
  const int info = P.pinfo[pos];
  const int plen = info & 0xFF;
  double pd[6], cd[21];
#pragma unroll
  for (int k = 0; k < 6; ++k) pd[k] = 0.0;
#pragma unroll
  for (int k = 0; k < 21; ++k) cd[k] = 0.0;
  float chi2 = 0.f;
  int status = 0, k = 0, t = -1;
  if ((info >> 8) & 1) {
    const float *row = P.out + (size_t)pos * kOutWords;
    const int *hit = reinterpret_cast<const int *>(row + kOutHit);
    const int8_t *plan = P.pplan + (size_t)pos * kMaxPlan;
    const int64_t ev_base = P.ev_off[P.pevent[pos]];
    const int64_t ev_hits = P.ev_off[P.pevent[pos] + 1] - ev_base;
    const int *sh = seed_hits + (size_t)P.order[pos] * 3;
#pragma unroll
    for (int m = 0; m < 6; ++m) pd[m] = row[kOutPar + m];
    status = 1;
    int taken = 0;
    for (t = plen + 2; t >= 0 && taken < 3; --t) {
      int lid, code;
      if (!backfit_seq(P, hit, plan, sh, ev_base, t, lid, code)) continue;
      if (lid < 0 || lid >= P.n_layers || code >= ev_hits ||
          !backfit_surface<double>(P, sl[lid], k == 0, code, ev_base, pd, cd, chi2)) {
        status = -(k + 1);
        break;
      }
      taken += code >= 0;
      ++k;
    }
  }
  float w[kBfWords];
#pragma unroll
  for (int m = 0; m < 6; ++m) w[m] = (float)pd[m];
#pragma unroll
  for (int m = 0; m < 21; ++m) w[6 + m] = (float)cd[m];
  w[27] = chi2;
  w[28] = __int_as_float(status);
  w[29] = __int_as_float(k);
  w[30] = __int_as_float(t);
  w[31] = 0.f;
  float4 *dst = reinterpret_cast<float4 *>(tmp + (size_t)pos * kBfWords);
#pragma unroll
  for (int q = 0; q < kBfWords / 4; ++q)
    dst[q] = make_float4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
}

// Tail, one lane per seed: the rest of the sequence in FP32; results by
// seed id (a failed fit reports zeros).
__global__ __launch_bounds__(256) void k_backfit_tail(FindParams P, const int *seed_hits,
                                                      const float *tmp, float *out_par,
                                                      float *out_cov, float *out_chi2,
                                                      int *out_status) {
  __shared__ DevLayer sl[kMaxLayers];
  stage_layers(P, sl);
  __syncthreads();
  const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pos >= P.n_seeds) return;
  const int seed = P.order[pos];
  float w[kBfWords];
  const float4 *src = reinterpret_cast<const float4 *>(tmp + (size_t)pos * kBfWords);
#pragma unroll
  for (int q = 0; q < kBfWords / 4; ++q) {
    const float4 v = src[q];
    w[4 * q] = v.x;
    w[4 * q + 1] = v.y;
    w[4 * q + 2] = v.z;
    w[4 * q + 3] = v.w;
  }
  float p[6], c[21];
#pragma unroll
  for (int m = 0; m < 6; ++m) p[m] = w[m];
#pragma unroll
  for (int m = 0; m < 21; ++m) c[m] = w[6 + m];
  float chi2 = w[27];
  int status = __float_as_int(w[28]);
  int k = __float_as_int(w[29]);
  int t = __float_as_int(w[30]);
  if (status == 1) {
    const float *row = P.out + (size_t)pos * kOutWords;
    const int *hit = reinterpret_cast<const int *>(row + kOutHit);
    const int8_t *plan = P.pplan + (size_t)pos * kMaxPlan;
    const int64_t ev_base = P.ev_off[P.pevent[pos]];
    const int64_t ev_hits = P.ev_off[P.pevent[pos] + 1] - ev_base;
    const int *sh = seed_hits + (size_t)seed * 3;
    for (; t >= 0; --t) {
      int lid, code;
      if (!backfit_seq(P, hit, plan, sh, ev_base, t, lid, code)) continue;
      if (lid < 0 || lid >= P.n_layers || code >= ev_hits ||
          !backfit_surface<float>(P, sl[lid], k == 0, code, ev_base, p, c, chi2)) {
        status = -(k + 1);
        break;
      }
      ++k;
    }
  }
  if (status != 1) {
#pragma unroll
    for (int m = 0; m < 6; ++m) p[m] = 0.f;
#pragma unroll
    for (int m = 0; m < 21; ++m) c[m] = 0.f;
    chi2 = 0.f;
  }
#pragma unroll
  for (int m = 0; m < 6; ++m) out_par[(size_t)seed * 6 + m] = p[m];
#pragma unroll
  for (int m = 0; m < 21; ++m) out_cov[(size_t)seed * 21 + m] = c[m];
  out_chi2[seed] = chi2;
  out_status[seed] = status;
}

// ------------------------------------------------------------- smoothing
//
// Rauch-Tung-Striebel smoothing of the found tracks (the backward pass the
// layer plan's steering provides for, Section 2.1, applied to the Kalman
// filter of the Introduction): on the seed's third layer and on every plan
// layer a track crossed, its state given all its hits.
// * Forward (k_smooth_fwd, FP32): the find's filter along the track from the
//   seed state (propagate, add the layer's scattering, update with the hit
//   if there is one), keeping per surface the filtered state x, C, the
//   predicted state xp, Cp after scattering and F C (F: the transport from
//   the previous surface, C: the filtered covariance there).
// * Backward (k_smooth_bwd, FP32): from the last surface, where the smoothed
//   state is the filtered one,
//     xs(k) = x(k) + A (xs(k+1) - xp(k+1)),
//     Cs(k) = C(k) + A (Cs(k+1) - Cp(k+1)) A^T,   A = C(k) F^T Cp(k+1)^-1.
//   Cp(k+1) has no extent along its surface's normal and every vector it
//   meets lies in the surface, so the inverse is taken in the surface's five
//   free coordinates J: A = (J F C)^T (J Cp J^T)^-1 J, with a Cholesky
//   factor of J Cp J^T.

// per surface, SoA over positions: filtered 27, predicted 27, F C 36, layer
constexpr int kSmFields = 91;
constexpr int kSmFilt = 0, kSmPred = 27, kSmFC = 54, kSmLayer = 90;

__global__ __launch_bounds__(256) void k_smooth_fwd(FindParams P, const int *seed_hits,
                                                    float *wk, int *n_surf) {
  __shared__ DevLayer sl[kMaxLayers];
  stage_layers(P, sl);
  __syncthreads();
  const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pos >= P.n_seeds) return;
  const size_t N = (size_t)P.n_seeds;
  auto at = [&](int j, int f) -> float & { return wk[((size_t)j * kSmFields + f) * N + pos]; };
  const int info = P.pinfo[pos];
  const int plen = info & 0xFF;
  int n = 0;
  if ((info >> 8) & 1) {
    const float *row = P.out + (size_t)pos * kOutWords;
    const int *hit = reinterpret_cast<const int *>(row + kOutHit);
    const int8_t *plan = P.pplan + (size_t)pos * kMaxPlan;
    const int64_t ev_base = P.ev_off[P.pevent[pos]];
    const int64_t ev_hits = P.ev_off[P.pevent[pos] + 1] - ev_base;
    const int *sh = seed_hits + (size_t)P.order[pos] * 3;
    float p[6], c[21];
    const float *st = P.pstate + (size_t)pos * kSeedWords;
#pragma unroll
    for (int m = 0; m < 6; ++m) p[m] = st[m];
#pragma unroll
    for (int m = 0; m < 21; ++m) c[m] = st[6 + m];
#pragma unroll
    for (int m = 0; m < 6; ++m) at(0, kSmFilt + m) = p[m];
#pragma unroll
    for (int m = 0; m < 21; ++m) at(0, kSmFilt + 6 + m) = c[m];
    at(0, kSmLayer) = __int_as_float(P.hlayer[ev_base + sh[2]]);
    n = 1;
    for (int s = 0; s < plen; ++s) {
      const int code = hit[s];
      if (code < MKF_HIT_MISS) continue;  // not crossed, or after the track ended
      const int lid = plan[s];
      if (lid < 0 || lid >= P.n_layers || code >= ev_hits) {
        n = -1;
        break;
      }
      const DevLayer &L = sl[lid];
      Prop pr;
      float fc[36];
      if (propagate<true, float, true>(p, c, L, P.cfg.mkb, P.cfg.l_min, false, 0.f, pr, 0.f,
                                       nullptr, fc, &P.cfg.field) != kOk) {
        n = -1;
        break;
      }
      float j33, j35;
      material(P.cfg, L.kind, pr.p, pr.c, 1.f, &j33, &j35);
      // the transport to the prediction includes the loss's Jacobian
#pragma unroll
      for (int m = 0; m < 6; ++m) fc[18 + m] = j33 * fc[18 + m] + j35 * fc[30 + m];
#pragma unroll
      for (int m = 0; m < 6; ++m) at(n, kSmPred + m) = pr.p[m];
#pragma unroll
      for (int m = 0; m < 21; ++m) at(n, kSmPred + 6 + m) = pr.c[m];
#pragma unroll
      for (int m = 0; m < 36; ++m) at(n, kSmFC + m) = fc[m];
      if (code >= 0) {
        const HitRec h = P.byorig[ev_base + code];
        Frame f;
        make_frame(pr.p, pr.c, L.kind, f);
        float u, v;
        if (!residual(pr.p, f, L.kind, h.x, h.y, h.z, u, v)) {
          n = -1;
          break;
        }
        kf_update(pr.p, pr.c, f, L.kind, h.vu, h.vv, h.vuv, u, v);
      }
#pragma unroll
      for (int m = 0; m < 6; ++m) p[m] = pr.p[m];
#pragma unroll
      for (int m = 0; m < 21; ++m) c[m] = pr.c[m];
#pragma unroll
      for (int m = 0; m < 6; ++m) at(n, kSmFilt + m) = p[m];
#pragma unroll
      for (int m = 0; m < 21; ++m) at(n, kSmFilt + 6 + m) = c[m];
      at(n, kSmLayer) = __int_as_float(lid);
      ++n;
    }
  }
  n_surf[pos] = n;
}

// the surface's five free coordinates: u0 = a0 v0 + a1 v1 (barrel: along
// the azimuth; disk: x), u1 = b0 v0 + b1 v1 + b2 v2 (barrel: z; disk: y),
// u2..u4 = q/pT, phi, theta
struct FreeCoords {
  float a0, a1, b0, b1, b2;
  __device__ void apply(const float *v, float *u) const {
    u[0] = fmaf(a0, v[0], a1 * v[1]);
    u[1] = fmaf(b0, v[0], fmaf(b1, v[1], b2 * v[2]));
    u[2] = v[3];
    u[3] = v[4];
    u[4] = v[5];
  }
  // row a of J as a 6-vector
  __device__ void row(int a, float *r) const {
#pragma unroll
    for (int i = 0; i < 6; ++i) r[i] = 0.f;
    if (a == 0) {
      r[0] = a0;
      r[1] = a1;
    } else if (a == 1) {
      r[0] = b0;
      r[1] = b1;
      r[2] = b2;
    } else {
      r[a + 1] = 1.f;
    }
  }
};

// J M J^T (5 x 5, lower triangle packed by rows) of a symmetric 6 x 6 M
// (upper triangle packed)
__device__ __forceinline__ void sandwich5(const FreeCoords &J, const float *M, float *out) {
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    float r[6], v[6];
    J.row(b, r);
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      float a = 0.f;
#pragma unroll
      for (int j = 0; j < 6; ++j) a = fmaf(M[i <= j ? tri(i, j) : tri(j, i)], r[j], a);
      v[i] = a;
    }
    float u[5];
    J.apply(v, u);
#pragma unroll
    for (int a = b; a < 5; ++a) out[a * (a + 1) / 2 + b] = u[a];
  }
}

// solve (L L^T) x = b in place, L lower-triangular 5x5 packed by rows
__device__ __forceinline__ void chol_solve5(const float *Lp, float *b) {
  float y[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    float a = b[i];
#pragma unroll
    for (int k = 0; k < i; ++k) a = fmaf(-Lp[i * (i + 1) / 2 + k], y[k], a);
    y[i] = a / Lp[i * (i + 1) / 2 + i];
  }
#pragma unroll
  for (int i = 4; i >= 0; --i) {
    float a = y[i];
#pragma unroll
    for (int k = i + 1; k < 5; ++k) a = fmaf(-Lp[k * (k + 1) / 2 + i], b[k], a);
    b[i] = a / Lp[i * (i + 1) / 2 + i];
  }
}

// Backward pass, FP32: the 5 x 5 systems are well conditioned once scaled
// by their diagonal (condition numbers of the correlation matrices up to
// ~500 on the benchmark's tracks), which a Cholesky solve respects.
__global__ __launch_bounds__(256) void k_smooth_bwd(FindParams P, const float *wk,
                                                    const int *n_surf, float *out_par,
                                                    float *out_cov, int *out_n) {
  const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pos >= P.n_seeds) return;
  const size_t N = (size_t)P.n_seeds;
  auto at = [&](int j, int f) { return wk[((size_t)j * kSmFields + f) * N + pos]; };
  const int seed = P.order[pos];
  int n = n_surf[pos];
  float *op = out_par + (size_t)seed * (kMaxPlan + 1) * 6;
  float *oc = out_cov + (size_t)seed * (kMaxPlan + 1) * 21;
  if (n > 0) {
    float xs[6], Cs[21];
#pragma unroll
    for (int m = 0; m < 6; ++m) xs[m] = at(n - 1, kSmFilt + m);
#pragma unroll
    for (int m = 0; m < 21; ++m) Cs[m] = at(n - 1, kSmFilt + 6 + m);
#pragma unroll
    for (int m = 0; m < 6; ++m) op[(n - 1) * 6 + m] = xs[m];
#pragma unroll
    for (int m = 0; m < 21; ++m) oc[(n - 1) * 21 + m] = Cs[m];
    for (int k = n - 2; k >= 0; --k) {
      // surface k+1: its free coordinates at the predicted point
      float xp[6];
#pragma unroll
      for (int m = 0; m < 6; ++m) xp[m] = at(k + 1, kSmPred + m);
      const int lid = __float_as_int(at(k + 1, kSmLayer));
      FreeCoords J;
      if (P.layers[lid].kind == 0) {
        const float ir = rsqrtf(fmaf(xp[0], xp[0], xp[1] * xp[1]));
        J = FreeCoords{-xp[1] * ir, xp[0] * ir, 0.f, 0.f, 1.f};
      } else {
        J = FreeCoords{1.f, 0.f, 0.f, 1.f, 0.f};
      }
      // Sr = J Cp J^T, then dPr = J (Cs - Cp) J^T
      float Sr[15], dPr[15];
      {
        float Cp[21];
#pragma unroll
        for (int m = 0; m < 21; ++m) Cp[m] = at(k + 1, kSmPred + 6 + m);
        sandwich5(J, Cp, Sr);
#pragma unroll
        for (int m = 0; m < 21; ++m) Cs[m] -= Cp[m];
        sandwich5(J, Cs, dPr);
      }
      // Cholesky factor of Sr in place
      bool pd = true;
#pragma unroll
      for (int i = 0; i < 5; ++i) {
#pragma unroll
        for (int j = 0; j <= i; ++j) {
          float a = Sr[i * (i + 1) / 2 + j];
#pragma unroll
          for (int q = 0; q < j; ++q) a = fmaf(-Sr[i * (i + 1) / 2 + q], Sr[j * (j + 1) / 2 + q], a);
          if (i == j) {
            pd = pd && a > 0.f;
            Sr[i * (i + 1) / 2 + i] = sqrtf(a > 0.f ? a : 1.f);
          } else {
            Sr[i * (i + 1) / 2 + j] = a / Sr[j * (j + 1) / 2 + j];
          }
        }
      }
      if (!pd) {
        n = -2;
        break;
      }
      // u = Sr^-1 J (xs - xp)
      float d[6], u[5];
#pragma unroll
      for (int m = 0; m < 6; ++m) d[m] = xs[m] - xp[m];
      d[4] = wrap_phi(d[4]);
      J.apply(d, u);
      chol_solve5(Sr, u);
      // M = J F C (5 x 6), one column at a time: xs(k) = x(k) + M^T u and
      // W = Sr^-1 M
      float W[5][6];
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        float col[6], w[5];
#pragma unroll
        for (int i = 0; i < 6; ++i) col[i] = at(k + 1, kSmFC + i * 6 + j);
        J.apply(col, w);
        float a = at(k, kSmFilt + j);
#pragma unroll
        for (int q = 0; q < 5; ++q) a = fmaf(w[q], u[q], a);
        xs[j] = a;
        chol_solve5(Sr, w);
#pragma unroll
        for (int q = 0; q < 5; ++q) W[q][j] = w[q];
      }
      xs[4] = wrap_phi(xs[4]);
      // Cs(k) = C(k) + W^T dPr W
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        float t[5];
#pragma unroll
        for (int a = 0; a < 5; ++a) {
          float v = 0.f;
#pragma unroll
          for (int b = 0; b < 5; ++b)
            v = fmaf(dPr[a >= b ? a * (a + 1) / 2 + b : b * (b + 1) / 2 + a], W[b][i], v);
          t[a] = v;
        }
#pragma unroll
        for (int j = i; j < 6; ++j) {
          float v = at(k, kSmFilt + 6 + tri(i, j));
#pragma unroll
          for (int a = 0; a < 5; ++a) v = fmaf(t[a], W[a][j], v);
          Cs[tri(i, j)] = v;
        }
      }
#pragma unroll
      for (int m = 0; m < 6; ++m) op[k * 6 + m] = xs[m];
#pragma unroll
      for (int m = 0; m < 21; ++m) oc[k * 21 + m] = Cs[m];
    }
  }
  out_n[seed] = n;
}

__global__ __launch_bounds__(256) void k_validate_hits(int64_t n, const float *x, const float *y,
                                                       const float *z, const float *vu,
                                                       const float *vv, const int *layer,
                                                       int n_layers, int *bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bool good = isfinite(x[i]) && isfinite(y[i]) && isfinite(z[i]) && isfinite(vu[i]) &&
                    isfinite(vv[i]) && vu[i] > 0.f && vv[i] > 0.f && layer[i] >= 0 &&
                    layer[i] < n_layers;
  if (!good) atomicOr(bad, 1);
}

__global__ void k_fill_u64(unsigned long long *p, int64_t n, unsigned long long v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_i32(int *p, int64_t n, int v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// The checked find's invariants of one seed's result record: a seed whose
// fit failed has no hits; otherwise each plan step holds a hit of the
// seed's event on that step's layer, a miss, a skip, or (once the candidate
// stopped, and from then on) none; the hit count is the three seed hits
// plus the hits taken, the miss count the misses; chi2 and the parameters
// are finite; the variances of q/pT, phi and theta are positive, those of
// the position at least -1e-5 of their (positive) sum.
__global__ __launch_bounds__(256) void k_check_results(FindParams P) {
  const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int bad = 0;
  if (pos < P.n_seeds) {
    const float *rec = P.out + (size_t)pos * kOutWords;
    const int *hit = reinterpret_cast<const int *>(rec + kOutHit);
    const int meta = __float_as_int(rec[kOutMeta]);
    const int nh = meta & 0xFF, nm = (meta >> 8) & 0xFF;
    const int info = P.pinfo[pos];
    const int plen = info & 0xFF;
    if (!((info >> 8) & 1)) {
      bad = nh != 0 || nm != 0;
    } else {
      const int ev = P.pevent[pos];
      const int64_t base = P.ev_off[ev], nev = P.ev_off[ev + 1] - base;
      int found = 0, miss = 0;
      bool stopped = false;
      for (int s = 0; s < plen; ++s) {
        const int h = hit[s];
        const int lid = P.pplan[(size_t)pos * kMaxPlan + s];
        if (h >= 0) {
          if (stopped || h >= nev) bad = 1;
          else if (P.hlayer[base + h] != lid) bad = 1;
          ++found;
        } else if (h == MKF_HIT_MISS) {
          bad |= stopped;
          ++miss;
        } else if (h == MKF_HIT_SKIP) {
          bad |= stopped;
        } else if (h == MKF_HIT_NONE) {
          stopped = true;
        } else {
          bad = 1;
        }
      }
      bad |= nh != 3 + found || nm != miss;
      const float c2 = rec[kOutChi2];
      bad |= !(c2 >= 0.f) || !isfinite(c2);
      // (the state lies on its last surface: the variance along the
      // surface's normal is zero up to rounding, so a position variance
      // may be a rounding below zero; their sum must be positive)
      const float tp = rec[kOutCov + tri(0, 0)] + rec[kOutCov + tri(1, 1)] +
                       rec[kOutCov + tri(2, 2)];
      bad |= !(tp > 0.f) || !isfinite(tp);
      for (int i = 0; i < 6; ++i) {
        bad |= !isfinite(rec[kOutPar + i]);
        const float d = rec[kOutCov + tri(i, i)];
        bad |= !isfinite(d) || (i < 3 ? d < -1e-5f * tp : !(d > 0.f));
      }
    }
  }
  add_counter(P, kCntCheckFailed, bad);
}

// ------------------------------------------------------------- launchers

static inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

void launch_hit_bins(hipStream_t s, const FindParams &P, int64_t n_hits, const int *layer,
                     int *hit_bin, int *counts) {
  if (n_hits == 0) return;
  hipLaunchKernelGGL(k_hit_bins, dim3(blocks_for(n_hits, 256)), dim3(256), 0, s, P, P.n_events,
                     n_hits, layer, hit_bin, counts);
}

void launch_scatter(hipStream_t s, const FindParams &P, int64_t n_hits, const int *hit_bin,
                    int *fill, HitRec *sorted, HitRec *byorig) {
  if (n_hits == 0) return;
  hipLaunchKernelGGL(k_hit_scatter, dim3(blocks_for(n_hits, 256)), dim3(256), 0, s, P,
                     P.n_events, n_hits, hit_bin, fill, sorted, byorig);
}

static void scan_rec(hipStream_t s, const int *in, int *out, int64_t n, int *scratch) {
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  int *sums = scratch;
  int *scanned = scratch + nb;
  hipLaunchKernelGGL(k_block_scan, dim3((unsigned)nb), dim3(256), 0, s, in, out, n, sums);
  if (nb > 1) {
    scan_rec(s, sums, scanned, nb, scratch + 2 * nb + 1);
    hipLaunchKernelGGL(k_add_offsets, dim3(blocks_for(n, 256)), dim3(256), 0, s, out, n,
                       scanned);
  }
  hipLaunchKernelGGL(k_set_total, dim3(1), dim3(1), 0, s, out, n, sums, scanned, nb);
}

void launch_scan(hipStream_t s, const int *in, int *out, int64_t n, int *tmp_a, int *tmp_b) {
  (void)tmp_b;
  if (n == 0) {
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(1), 0, s, out, (int64_t)1, 0);
    return;
  }
  scan_rec(s, in, out, n, tmp_a);
}

void launch_seed(hipStream_t s, const FindParams &P, const int *seed_hits, float *seed_state,
                 int *seed_ok, int *plan_len, int8_t *plan, double *plan_l, float *seed_chi2,
                 const DevRegion *regions, int n_regions) {
  if (P.n_seeds == 0) return;
  hipLaunchKernelGGL(k_seed, dim3(blocks_for(P.n_seeds, 256)), dim3(256), 0, s, P, seed_hits,
                     seed_state, seed_ok, plan_len, plan, plan_l, seed_chi2, regions, n_regions);
}

void launch_find_init(hipStream_t s, const FindParams &P) {
  if (P.n_seeds == 0) return;
  hipLaunchKernelGGL(k_find_init, dim3(blocks_for(P.n_seeds * P.slots, 256)), dim3(256), 0, s, P);
}

template <int G>
static void launch_find_step_g(hipStream_t s, const FindParams &P, int step, int64_t n_active) {
  const unsigned nb = blocks_for(n_active, 4 * Grp<G>::kSeeds);
  const unsigned grid = (nb + kQueues - 1) / kQueues * kQueues;  // whole XCD shares
  if (P.cfg.mat.tab || P.cfg.field.on)
    hipLaunchKernelGGL((k_find_step<true, G>), dim3(grid), dim3(256), 0, s, P, step, n_active);
  else hipLaunchKernelGGL((k_find_step<false, G>), dim3(grid), dim3(256), 0, s, P, step, n_active);
}

void launch_find_step(hipStream_t s, const FindParams &P, int step, int64_t n_active) {
  if (n_active == 0) return;
  if (P.slots == 6) launch_find_step_g<6>(s, P, step, n_active);
  else launch_find_step_g<8>(s, P, step, n_active);
}

template <int G, bool kSurr, bool kMat>
static void launch_persistent_g(hipStream_t s, const FindParams &P, int grid, int waves) {
  const size_t lds = 4 * sizeof(int) * persistent_rec_words(P.max_plan, G, Grp<G>::kSeeds);
  if constexpr (kMat) {
    switch (waves) {
      case 1: hipLaunchKernelGGL((k_find_persistent_mat<1, kSurr, G>), dim3(grid), dim3(256), lds, s, P); break;
      case 3: hipLaunchKernelGGL((k_find_persistent_mat<3, kSurr, G>), dim3(grid), dim3(256), lds, s, P); break;
      case 4: hipLaunchKernelGGL((k_find_persistent_mat<4, kSurr, G>), dim3(grid), dim3(256), lds, s, P); break;
      default: hipLaunchKernelGGL((k_find_persistent_mat<2, kSurr, G>), dim3(grid), dim3(256), lds, s, P); break;
    }
  } else {
    switch (waves) {
      case 1: hipLaunchKernelGGL((k_find_persistent<1, kSurr, G>), dim3(grid), dim3(256), lds, s, P); break;
      case 3: hipLaunchKernelGGL((k_find_persistent<3, kSurr, G>), dim3(grid), dim3(256), lds, s, P); break;
      case 4: hipLaunchKernelGGL((k_find_persistent<4, kSurr, G>), dim3(grid), dim3(256), lds, s, P); break;
      default: hipLaunchKernelGGL((k_find_persistent<2, kSurr, G>), dim3(grid), dim3(256), lds, s, P); break;
    }
  }
}

template <bool kSurr, bool kMat>
static void launch_persistent_k(hipStream_t s, const FindParams &P, int grid, int waves,
                                int group) {
  // 6-lane groups only hold budgets up to 6 candidates
  if (group == 8 || P.cfg.n_cand > 6) launch_persistent_g<8, kSurr, kMat>(s, P, grid, waves);
  else launch_persistent_g<6, kSurr, kMat>(s, P, grid, waves);
}

void launch_find_persistent(hipStream_t s, const FindParams &P, int grid_blocks, int waves,
                            bool surrogate, int group) {
  if (P.n_seeds == 0) return;
  if (P.cfg.mat.tab || P.cfg.field.on) {
    if (surrogate) launch_persistent_k<true, true>(s, P, grid_blocks, waves, group);
    else launch_persistent_k<false, true>(s, P, grid_blocks, waves, group);
  } else if (surrogate) launch_persistent_k<true, false>(s, P, grid_blocks, waves, group);
  else launch_persistent_k<false, false>(s, P, grid_blocks, waves, group);
}

void launch_finalize(hipStream_t s, const FindParams &P) {
  if (P.n_seeds == 0) return;
  hipLaunchKernelGGL(k_finalize, dim3(blocks_for(P.n_seeds, 256)), dim3(256), 0, s, P);
}
void launch_check_results(hipStream_t s, const FindParams &P) {
  if (P.n_seeds == 0) return;
  hipLaunchKernelGGL(k_check_results, dim3(blocks_for(P.n_seeds, 256)), dim3(256), 0, s, P);
}

void launch_permute_seeds(hipStream_t s, const FindParams &P, float *pstate, int *pinfo,
                          int *pevent, int8_t *pplan) {
  if (P.n_seeds == 0) return;
  hipLaunchKernelGGL(k_permute_seeds, dim3(blocks_for(P.n_seeds, 256)), dim3(256), 0, s, P,
                     pstate, pinfo, pevent, pplan);
}

void launch_propagate(hipStream_t s, const FindParams &P, int64_t n, const float *par,
                      const float *cov, const int *layer, float *out_par, float *out_cov,
                      float *out_l, int *out_status) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_propagate, dim3(blocks_for(n, 256)), dim3(256), 0, s, P, n, par, cov,
                     layer, out_par, out_cov, out_l, out_status);
}

void launch_fit(hipStream_t s, const DevCfg &cfg, int64_t n, int n_steps, const int8_t *kind,
                const float *pos, const float *x, const float *y, const float *z,
                const float *vu, const float *vv, const int *len, const float *init_par,
                const float *init_cov, float *out_par, float *out_cov, float *out_chi2,
                int *out_status) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_fit, dim3(blocks_for(n, 256)), dim3(256), 0, s, cfg, n, n_steps, kind, pos,
                     x, y, z, vu, vv, len, init_par, init_cov, out_par, out_cov, out_chi2,
                     out_status);
}

void launch_backfit(hipStream_t s, const FindParams &P, const int *seed_hits, float *tmp,
                    float *out_par, float *out_cov, float *out_chi2, int *out_status) {
  if (P.n_seeds == 0) return;
  hipLaunchKernelGGL(k_backfit_head, dim3(blocks_for(P.n_seeds, 256)), dim3(256), 0, s, P,
                     seed_hits, tmp);
  hipLaunchKernelGGL(k_backfit_tail, dim3(blocks_for(P.n_seeds, 256)), dim3(256), 0, s, P,
                     seed_hits, tmp, out_par, out_cov, out_chi2, out_status);
}

void launch_smooth(hipStream_t s, const FindParams &P, const int *seed_hits, float *wk,
                   int *n_surf, float *out_par, float *out_cov, int *out_n) {
  if (P.n_seeds == 0) return;
  hipLaunchKernelGGL(k_smooth_fwd, dim3(blocks_for(P.n_seeds, 256)), dim3(256), 0, s, P,
                     seed_hits, wk, n_surf);
  hipLaunchKernelGGL(k_smooth_bwd, dim3(blocks_for(P.n_seeds, 256)), dim3(256), 0, s, P, wk,
                     n_surf, out_par, out_cov, out_n);
}

void launch_triplets(hipStream_t s, const FindParams &P, const DevSeeding &sc,
                     int64_t max_event_hits, bool write, int *counts, const int *offsets,
                     int *out_event, int *out_hits) {
  if (max_event_hits == 0 || P.n_events == 0) return;
  const dim3 grid(blocks_for(max_event_hits, 256), (unsigned)P.n_events);
  if (write)
    hipLaunchKernelGGL(k_triplets<true>, grid, dim3(256), 0, s, P, sc, counts, offsets, out_event,
                       out_hits);
  else
    hipLaunchKernelGGL(k_triplets<false>, grid, dim3(256), 0, s, P, sc, counts, offsets,
                       out_event, out_hits);
}

void launch_dup_prep(hipStream_t s, const FindParams &P, const int *seed_hits, int *hbuf, int *hn,
                     int *cnt) {
  if (P.n_seeds == 0) return;
  hipLaunchKernelGGL(k_dup_prep, dim3(blocks_for(P.n_seeds, 256)), dim3(256), 0, s, P, seed_hits,
                     hbuf, hn, cnt);
}

void launch_dup_fill(hipStream_t s, const FindParams &P, const int *hbuf, const int *hn,
                     const int *off, int *fill, int *list) {
  if (P.n_seeds == 0) return;
  hipLaunchKernelGGL(k_dup_fill, dim3(blocks_for(P.n_seeds, 256)), dim3(256), 0, s, P, hbuf, hn,
                     off, fill, list);
}

void launch_dup_decide(hipStream_t s, const FindParams &P, const int *seed_hits, const int *hbuf,
                       const int *hn, const int *off, const int *list, float frac, int *out_dup,
                       int *n_dup) {
  if (P.n_seeds == 0) return;
  hipLaunchKernelGGL(k_dup_decide, dim3(blocks_for(P.n_seeds, 256)), dim3(256), 0, s, P,
                     seed_hits, hbuf, hn, off, list, frac, out_dup, n_dup);
}

void launch_clean_prep(hipStream_t s, const FindParams &P, const int *seed_hits, int *hbuf,
                       int *cnt) {
  if (P.n_seeds == 0) return;
  hipLaunchKernelGGL(k_clean_prep, dim3(blocks_for(P.n_seeds, 256)), dim3(256), 0, s, P,
                     seed_hits, hbuf, cnt);
}

void launch_clean_fill(hipStream_t s, const FindParams &P, const int *hbuf, const int *off,
                       int *fill, int *list) {
  if (P.n_seeds == 0) return;
  hipLaunchKernelGGL(k_clean_fill, dim3(blocks_for(P.n_seeds, 256)), dim3(256), 0, s, P, hbuf,
                     off, fill, list);
}

void launch_clean_decide(hipStream_t s, const FindParams &P, const int *seed_hits,
                         const float *seed_chi2, const int *hbuf, const int *off,
                         const int *list, const DevCleaning &cc, int *out_keep, int *n_keep) {
  if (P.n_seeds == 0) return;
  hipLaunchKernelGGL(k_clean_decide, dim3(blocks_for(P.n_seeds, 256)), dim3(256), 0, s, P,
                     seed_hits, seed_chi2, hbuf, off, list, cc, out_keep, n_keep);
}

void launch_validate_hits(hipStream_t s, int64_t n, const float *x, const float *y,
                          const float *z, const float *vu, const float *vv, const int *layer,
                          int n_layers, int *bad) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_validate_hits, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, x, y, z, vu,
                     vv, layer, n_layers, bad);
}

void launch_fill_u64(hipStream_t s, unsigned long long *p, int64_t n, unsigned long long v) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n, v);
}
void launch_fill_i32(hipStream_t s, int *p, int64_t n, int v) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n, v);
}

}  // namespace mkf
