// mkf_capi.hip -- host runtime behind the C ABI declared in include/mkf.h:
// argument validation, device buffers owned by the context, stream
// ordering, and the drivers of the two find forms.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/mkf.h"
#include "mkf_kernels.hpp"

using namespace mkf;

namespace {

// grow-only device buffer
struct DevBuf {
  void *ptr = nullptr;
  size_t bytes = 0;
  hipError_t ensure(size_t n) {
    if (n <= bytes && ptr) return hipSuccess;
    if (ptr) {
      hipError_t e = hipFree(ptr);
      if (e != hipSuccess) return e;
      ptr = nullptr;
      bytes = 0;
    }
    size_t alloc = n ? n : 256;
    hipError_t e = hipMalloc(&ptr, alloc);
    if (e == hipSuccess) bytes = alloc;
    return e;
  }
  void release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
  }
  template <class T> T *as() const { return static_cast<T *>(ptr); }
};

enum Stage { kCreated = 0, kGeometry = 1, kHits = 2, kSeeds = 3, kFound = 4 };

}  // namespace

// Scratch of mkf_surrogate_grad_noalloc, for callers that cannot allocate:
// the per-wave partial gradient rows of up to kNoAllocMaxSamples samples,
// their first-level sums and the per-sample weights.  Each GPU holds one
// copy (5.5 MB) for the life of the process; host code reaches it only
// through the address hipGetSymbolAddress gives on that device.
constexpr int kNoAllocMaxSamples = MKF_NOALLOC_MAX_SAMPLES;
constexpr int kNoAllocMaxWaves = kNoAllocMaxSamples / 64;
constexpr size_t kNoAllocPartial = (size_t)kNoAllocMaxWaves * (kNParam + 1);
constexpr size_t kNoAllocPartial2 = (size_t)(kNoAllocMaxWaves / kReduceGroup + 1) * (kNParam + 1);
constexpr size_t kNoAllocFloats = kNoAllocPartial + kNoAllocPartial2 + kNoAllocMaxSamples;
static __device__ __align__(256) float scratch[kNoAllocFloats];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch[kMaxDevices] = {};  // device address of scratch, per device

// Resolves scratch's device address on the current device, once per device.
hipError_t resolve_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[dev]) return hipSuccess;
  void *ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch[dev] = static_cast<float *>(ptr);
  return hipSuccess;
}

float *scratch_on(int dev) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return dev >= 0 && dev < kMaxDevices ? g_scratch[dev] : nullptr;
}

}  // namespace

struct mkf_ctx {
  mkf_config cfg{};
  hipStream_t stream = nullptr;
  std::string err;
  int stage = kCreated;

  int n_layers = 0;
  mkf_layer user_layers[kMaxLayers]{};  // as loaded (bin counts before the tuning's shifts)
  DevLayer layers[kMaxLayers]{};
  int bins_per_event = 0;
  DevBuf d_layers;
  int n_regions = 0;  // region steering (0: plans from each seed's helix)
  DevBuf d_regions;
  DevMat mat{};       // material map (mat.tab == nullptr: constant angle)
  DevBuf d_mat;
  DevField field{};   // parameterised field (field.on == 0: uniform bz)

  // hits
  int n_events = 0;
  int64_t n_hits = 0;
  std::vector<int64_t> ev_off;
  DevBuf d_ev_off, d_x, d_y, d_z, d_vu, d_vv, d_layer;
  DevBuf d_hit_bin, d_counts, d_fill, d_bin_start, d_scan_tmp, d_sorted, d_byorig, d_bad;

  // seeds
  int64_t n_seeds = 0;
  DevBuf d_seed_event, d_seed_hits, d_seed_state, d_seed_ok, d_plan_len, d_plan, d_plan_l;
  DevBuf d_seed_chi2;
  DevBuf d_order, d_pstate, d_pinfo, d_pevent, d_pplan;
  DevBuf d_bf_tmp;  // backward fit: state between its FP64 and FP32 parts
  DevBuf d_sm_wk, d_sm_n;  // smoothing: forward-pass states per surface, surface counts
  DevBuf d_tr_cnt, d_tr_off, d_tr_tmp;  // triplet seeding: counts, offsets, scan scratch
  DevBuf d_dup_h, d_dup_n, d_dup_cnt, d_dup_off, d_dup_fill, d_dup_list, d_dup_tmp, d_dup_total;
  std::vector<int32_t> h_order, h_plen, h_ok;
  std::vector<int64_t> active_at_step;  // seeds (in processing order) with plan_len > step
  int max_plan_len = 0;
  int64_t n_seeds_ok = 0;

  // find
  DevBuf d_cand, d_fin_key, d_fin_rec, d_fin_meta, d_bp, d_steps, d_tiles, d_qoff;
  DevBuf d_out;  // result rows (kOut*), n_seeds words each
  hipEvent_t ev_a = nullptr, ev_b = nullptr, ev_m0 = nullptr, ev_m1 = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  int graph_launches = 0;
  mkf_stats stats{};
  // pinned host words the find's step count and counters are read back
  // into: [0] steps, then kCounters x kCounterSlots
  unsigned long long *h_cnt = nullptr;
  int n_cu = 0;
  int device = 0;  // the device current at mkf_create
  std::string arch;
  mkf_tuning tuning{2, 8, 0, 0, 0};

  // learned surrogate: master weights, Adam moments, BF16 images, counters
  DevBuf d_mlp_param, d_mlp_m, d_mlp_v, d_W1p, d_W2p, d_W3p, d_W2T, d_W3T, d_mb1, d_mb2, d_mb3;
  DevBuf d_cnt, d_radii, d_tx, d_tt, d_tvalid, d_partial, d_partial2, d_loss, d_grad;
  int mlp_step = 0;  // Adam steps taken

  // fit scratch (host-side inputs are staged here)
  ~mkf_ctx() {
    DevBuf *all[] = {&d_layers, &d_regions, &d_mat, &d_ev_off, &d_x, &d_y, &d_z, &d_vu, &d_vv, &d_layer,
                     &d_hit_bin, &d_counts, &d_fill, &d_bin_start, &d_scan_tmp, &d_sorted,
                     &d_byorig, &d_bad, &d_seed_event, &d_seed_hits, &d_seed_state, &d_seed_ok,
                     &d_plan_len, &d_plan, &d_plan_l, &d_order, &d_pstate, &d_pinfo,
                     &d_pevent, &d_pplan, &d_cand, &d_fin_key, &d_fin_rec, &d_fin_meta,
                     &d_bp, &d_steps, &d_tiles, &d_qoff, &d_out, &d_mlp_param, &d_mlp_m, &d_mlp_v, &d_W1p,
                     &d_W2p, &d_W3p, &d_W2T, &d_W3T, &d_mb1, &d_mb2, &d_mb3, &d_cnt, &d_radii,
                     &d_tx, &d_tt, &d_tvalid, &d_partial, &d_partial2, &d_loss, &d_grad, &d_bf_tmp, &d_sm_wk, &d_sm_n, &d_tr_cnt, &d_tr_off, &d_tr_tmp, &d_dup_h, &d_dup_n, &d_dup_cnt, &d_dup_off,
                     &d_dup_fill, &d_dup_list, &d_dup_tmp, &d_dup_total, &d_seed_chi2};
    for (DevBuf *b : all) b->release();
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (ev_a) (void)hipEventDestroy(ev_a);
    if (ev_b) (void)hipEventDestroy(ev_b);
    if (ev_m0) (void)hipEventDestroy(ev_m0);
    if (ev_m1) (void)hipEventDestroy(ev_m1);
    if (h_cnt) (void)hipHostFree(h_cnt);
  }
};

namespace {

std::string g_create_error = "no error";

mkf_status fail(mkf_ctx *c, mkf_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  else g_create_error = buf;
  return st;
}

#define HIP_TRY(c, expr)                                                                 \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail((c), MKF_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));         \
  } while (0)

DevCfg dev_cfg(const mkf_config &c) {
  DevCfg d{};
  d.mkb = -c.kappa * c.bz;
  d.chi2_cut = c.chi2_cut;
  d.ms_var = c.ms_sigma * c.ms_sigma;
  d.edge_margin = c.edge_margin;
  d.l_min = c.l_min;
  d.n_cand = c.n_cand;
  d.max_holes = c.max_holes;
  for (int i = 0; i < 6; ++i) d.init_var[i] = c.init_var[i];
  return d;
}

FindParams params(mkf_ctx *c) {
  FindParams P{};
  P.layers = c->d_layers.as<DevLayer>();
  P.n_layers = c->n_layers;
  P.cfg = dev_cfg(c->cfg);
  P.cfg.mat = c->mat;
  P.cfg.field = c->field;
  P.n_events = c->n_events;
  P.ev_off = c->d_ev_off.as<int64_t>();
  P.hx = c->d_x.as<float>();
  P.hy = c->d_y.as<float>();
  P.hz = c->d_z.as<float>();
  P.hvu = c->d_vu.as<float>();
  P.hvv = c->d_vv.as<float>();
  P.hlayer = c->d_layer.as<int>();
  P.sorted = c->d_sorted.as<HitRec>();
  P.byorig = c->d_byorig.as<HitRec>();
  P.bin_start = c->d_bin_start.as<int>();
  P.bins_per_event = c->bins_per_event;
  P.n_seeds = c->n_seeds;
  P.seed_event = c->d_seed_event.as<int>();
  P.seed_state = c->d_seed_state.as<float>();
  P.seed_ok = c->d_seed_ok.as<int>();
  P.plan_len = c->d_plan_len.as<int>();
  P.plan = c->d_plan.as<int8_t>();
  P.order = c->d_order.as<int>();
  P.pstate = c->d_pstate.as<float>();
  P.pinfo = c->d_pinfo.as<int>();
  P.pevent = c->d_pevent.as<int>();
  P.pplan = c->d_pplan.as<int8_t>();
  P.out = c->d_out.as<float>();
  // the layer-synchronous form's lane groups: 6 lanes hold budgets up to 6
  P.slots = c->cfg.n_cand <= 6 ? 6 : 8;
  P.cand = c->d_cand.as<float>();
  P.fin_key = c->d_fin_key.as<unsigned long long>();
  P.fin_rec = c->d_fin_rec.as<float>();
  P.fin_meta = c->d_fin_meta.as<int>();
  P.bp = c->d_bp.as<int>();
  P.tile_counter = c->d_tiles.as<int>();
  P.q_off = c->d_qoff.as<int64_t>();
  P.max_plan = c->max_plan_len;
  P.n_steps = c->d_steps.as<unsigned long long>();
  P.mlp = MlpWeights{c->d_W1p.as<__bf16>(), c->d_W2p.as<__bf16>(), c->d_W3p.as<__bf16>(),
                     c->d_W2T.as<__bf16>(), c->d_W3T.as<__bf16>(), c->d_mb1.as<float>(),
                     c->d_mb2.as<float>(), c->d_mb3.as<float>()};
  P.counters = c->d_cnt.as<unsigned long long>();
  return P;
}

bool finite_f(float v) { return std::isfinite(v); }

MlpBuffers mlp_buffers(mkf_ctx *c) {
  MlpBuffers B{};
  B.param = c->d_mlp_param.as<float>();
  B.m = c->d_mlp_m.as<float>();
  B.v = c->d_mlp_v.as<float>();
  B.W1p = c->d_W1p.as<__bf16>();
  B.W2p = c->d_W2p.as<__bf16>();
  B.W3p = c->d_W3p.as<__bf16>();
  B.W2T = c->d_W2T.as<__bf16>();
  B.W3T = c->d_W3T.as<__bf16>();
  B.b1 = c->d_mb1.as<float>();
  B.b2 = c->d_mb2.as<float>();
  B.b3 = c->d_mb3.as<float>();
  return B;
}

// Surrogate buffers and the initial weights: Glorot-uniform from a fixed
// seed (reproducible), zero biases and Adam moments, zero image padding.
hipError_t mlp_setup(mkf_ctx *c) {
  const size_t bf = sizeof(__bf16);
  hipError_t e = hipSuccess;
  DevBuf *f32[] = {&c->d_mlp_param, &c->d_mlp_m, &c->d_mlp_v};
  for (DevBuf *b : f32)
    if (e == hipSuccess) e = b->ensure(sizeof(float) * kNParam);
  if (e == hipSuccess) e = c->d_W1p.ensure(bf * 64 * kLdW1);
  if (e == hipSuccess) e = c->d_W2p.ensure(bf * 64 * kLdW2);
  if (e == hipSuccess) e = c->d_W3p.ensure(bf * 32 * kLdW3);
  if (e == hipSuccess) e = c->d_W2T.ensure(bf * 64 * kLdW2);
  if (e == hipSuccess) e = c->d_W3T.ensure(bf * 64 * kLdW3T);
  if (e == hipSuccess) e = c->d_mb1.ensure(sizeof(float) * 64);
  if (e == hipSuccess) e = c->d_mb2.ensure(sizeof(float) * 64);
  if (e == hipSuccess) e = c->d_mb3.ensure(sizeof(float) * 32);
  if (e == hipSuccess) e = c->d_cnt.ensure(sizeof(unsigned long long) * kCounters * kCounterSlots);
  if (e != hipSuccess) return e;
  DevBuf *zero[] = {&c->d_mlp_m, &c->d_mlp_v, &c->d_W1p, &c->d_W2p, &c->d_W3p, &c->d_W2T,
                    &c->d_W3T, &c->d_mb1, &c->d_mb2, &c->d_mb3, &c->d_cnt};
  for (DevBuf *b : zero)
    if (e == hipSuccess) e = hipMemsetAsync(b->ptr, 0, b->bytes, c->stream);
  std::vector<float> p(kNParam, 0.f);
  uint64_t st = 0x5EEDF00Dull;
  auto uni = [&]() {  // SplitMix64 stream
    st += 0x9E3779B97F4A7C15ull;
    uint64_t z = st;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
  };
  auto fill = [&](int off, int fan_out, int fan_in) {
    const double a = std::sqrt(6.0 / (fan_in + fan_out));
    for (int i = 0; i < fan_out * fan_in; ++i) p[off + i] = (float)((2.0 * uni() - 1.0) * a);
  };
  fill(kOffW1, kNH, kNI);
  fill(kOffW2, kNH, kNH);
  fill(kOffW3, kNO, kNH);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->d_mlp_param.ptr, p.data(), sizeof(float) * kNParam,
                       hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) {
    launch_mlp_images(c->stream, mlp_buffers(c));
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  c->mlp_step = 0;
  return e;
}

void drop_graph(mkf_ctx *c) {
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->graph_exec = nullptr;
  c->graph = nullptr;
}

// copy a caller array (host or device) into a context buffer
mkf_status stage_in(mkf_ctx *c, DevBuf &dst, const void *src, size_t bytes, int mem) {
  HIP_TRY(c, dst.ensure(bytes));
  if (bytes == 0) return MKF_OK;
  HIP_TRY(c, hipMemcpyAsync(dst.ptr, src, bytes,
                            mem == MKF_MEM_DEVICE ? hipMemcpyDeviceToDevice
                                                  : hipMemcpyHostToDevice,
                            c->stream));
  return MKF_OK;
}

}  // namespace

extern "C" {

mkf_status mkf_create(const mkf_config *cfg, void *stream, mkf_ctx **out) {
  if (!out) return fail(nullptr, MKF_E_ARG, "out is NULL");
  *out = nullptr;
  if (!cfg) return fail(nullptr, MKF_E_ARG, "cfg is NULL");
  if (!(cfg->n_cand >= 1 && cfg->n_cand <= MKF_MAX_CAND))
    return fail(nullptr, MKF_E_ARG, "n_cand must be in 1..%d", MKF_MAX_CAND);
  if (cfg->max_holes < 0 || cfg->max_holes > 32)
    return fail(nullptr, MKF_E_ARG, "max_holes must be in 0..32");
  const float fv[] = {cfg->bz, cfg->kappa, cfg->chi2_cut, cfg->ms_sigma, cfg->edge_margin,
                      cfg->l_min};
  for (float v : fv)
    if (!finite_f(v)) return fail(nullptr, MKF_E_ARG, "non-finite setting");
  if (!(cfg->chi2_cut > 0.f) || cfg->ms_sigma < 0.f || cfg->edge_margin < 0.f ||
      !(cfg->l_min > 0.f) || !(cfg->kappa > 0.f))
    return fail(nullptr, MKF_E_ARG, "chi2_cut, kappa, l_min must be > 0; ms_sigma, edge_margin >= 0");
  for (int i = 0; i < 6; ++i)
    if (!(cfg->init_var[i] > 0.f) || !finite_f(cfg->init_var[i]))
      return fail(nullptr, MKF_E_ARG, "init_var must be finite and > 0");
  if (cfg->flags & ~(MKF_F_BATCHED | MKF_F_GRAPH | MKF_F_SURROGATE | MKF_F_CHECKED))
    return fail(nullptr, MKF_E_ARG, "unknown flag bits 0x%x", (unsigned)cfg->flags);
  mkf_ctx *c = new (std::nothrow) mkf_ctx();
  if (!c) return fail(nullptr, MKF_E_CAPACITY, "out of host memory");
  c->cfg = *cfg;
  c->stream = static_cast<hipStream_t>(stream);
  hipError_t e = hipEventCreate(&c->ev_a);
  if (e == hipSuccess) e = hipEventCreate(&c->ev_b);
  if (e == hipSuccess) e = hipEventCreate(&c->ev_m0);
  if (e == hipSuccess) e = hipEventCreate(&c->ev_m1);
  if (e == hipSuccess) e = c->d_steps.ensure(sizeof(unsigned long long));
  if (e == hipSuccess) e = c->d_tiles.ensure(sizeof(int) * kQueues);
  if (e == hipSuccess) e = c->d_bad.ensure(sizeof(int));
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void **>(&c->h_cnt),
                      sizeof(unsigned long long) * (1 + kCounters * kCounterSlots),
                      hipHostMallocDefault);
  if (e != hipSuccess) {
    delete c;
    return fail(nullptr, MKF_E_HIP, "HIP setup failed: %s", hipGetErrorString(e));
  }
  int dev = 0, n_cu = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  c->n_cu = std::max(1, n_cu);
  c->device = dev;
  if (hipError_t es = resolve_scratch(dev)) {
    delete c;
    return fail(nullptr, MKF_E_HIP, "scratch address on device %d: %s", dev,
                hipGetErrorString(es));
  }
  if (hipError_t em = mlp_setup(c)) {
    delete c;
    return fail(nullptr, MKF_E_HIP, "surrogate setup failed: %s", hipGetErrorString(em));
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) c->arch = prop.gcnArchName;
  for (char &ch : c->arch)
    if (ch == ' ' || ch == ':') ch = '_';
  c->err = "no error";
  *out = c;
  return MKF_OK;
}

void mkf_destroy(mkf_ctx *ctx) {
  if (!ctx) return;
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  else (void)hipDeviceSynchronize();
  delete ctx;
}

const char *mkf_last_error(const mkf_ctx *ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

}  // extern "C"

namespace {

int shifted_bins(int n, int shift, int max) {
  const int64_t v = shift >= 0 ? (int64_t)n << shift : (int64_t)n >> -shift;
  return (int)std::min<int64_t>(std::max<int64_t>(v, 1), max);
}

// Device layer records from the loaded layers and the tuning's bin shifts.
mkf_status upload_layers(mkf_ctx *c) {
  int base = 0;
  DevLayer dl[kMaxLayers]{};
  for (int i = 0; i < c->n_layers; ++i) {
    const mkf_layer &L = c->user_layers[i];
    const int nphi = shifted_bins(L.n_phi_bins, c->tuning.phi_bin_shift, 4096);
    const int nq = shifted_bins(L.n_q_bins, c->tuning.q_bin_shift, 1024);
    DevLayer &d = dl[i];
    d.kind = L.kind;
    d.pos = L.pos;
    d.lo = L.ext_lo;
    d.hi = L.ext_hi;
    d.vu_max = L.var_u_max;
    d.vv_max = L.var_v_max;
    d.nphi = nphi;
    d.nq = nq;
    d.bin_base = base;
    d.q_lo = L.ext_lo;
    d.q_scale = (float)nq / (L.ext_hi - L.ext_lo);
    d.phi_scale = (float)nphi / kTwoPi;
    d.cs = L.stereo == 0.f ? 1.f : std::cos(L.stereo);
    d.sn = L.stereo == 0.f ? 0.f : std::sin(L.stereo);
    d.hole_lo = L.hole_lo < L.hole_hi ? L.hole_lo : 0.f;
    d.hole_hi = L.hole_lo < L.hole_hi ? L.hole_hi : 0.f;
    base += nphi * nq;
  }
  HIP_TRY(c, c->d_layers.ensure(sizeof(DevLayer) * kMaxLayers));
  HIP_TRY(c, hipMemcpyAsync(c->d_layers.ptr, dl, sizeof(dl), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  std::memcpy(c->layers, dl, sizeof(dl));
  c->bins_per_event = base;
  return MKF_OK;
}

// The binned hit index of the loaded hits (count, scan, scatter), for the
// current layer records.
mkf_status build_index(mkf_ctx *c) {
  const int64_t n_hits = c->n_hits;
  const int64_t total_bins = (int64_t)c->n_events * c->bins_per_event;
  if (total_bins >= ((int64_t)1 << 31) - 1)
    return fail(c, MKF_E_CAPACITY, "events x bins exceed the index size");
  HIP_TRY(c, c->d_hit_bin.ensure(sizeof(int) * (size_t)std::max<int64_t>(n_hits, 1)));
  HIP_TRY(c, c->d_counts.ensure(sizeof(int) * (size_t)std::max<int64_t>(total_bins, 1)));
  HIP_TRY(c, c->d_fill.ensure(sizeof(int) * (size_t)std::max<int64_t>(total_bins, 1)));
  HIP_TRY(c, c->d_bin_start.ensure(sizeof(int) * (size_t)(total_bins + 1)));
  HIP_TRY(c, c->d_scan_tmp.ensure(sizeof(int) * (size_t)(4 * (total_bins / 2048 + 4) + 64)));
  HIP_TRY(c, c->d_sorted.ensure(sizeof(HitRec) * (size_t)(std::max<int64_t>(n_hits, 1) + kHitPad)));
  HIP_TRY(c, c->d_byorig.ensure(sizeof(HitRec) * (size_t)std::max<int64_t>(n_hits, 1)));
  HIP_TRY(c, hipEventRecord(c->ev_a, c->stream));
  launch_fill_i32(c->stream, c->d_counts.as<int>(), total_bins, 0);
  launch_fill_i32(c->stream, c->d_fill.as<int>(), total_bins, 0);
  FindParams P = params(c);
  launch_hit_bins(c->stream, P, n_hits, c->d_layer.as<int>(), c->d_hit_bin.as<int>(),
                  c->d_counts.as<int>());
  launch_scan(c->stream, c->d_counts.as<int>(), c->d_bin_start.as<int>(), total_bins,
              c->d_scan_tmp.as<int>(), nullptr);
  launch_scatter(c->stream, P, n_hits, c->d_hit_bin.as<int>(), c->d_fill.as<int>(),
                 c->d_sorted.as<HitRec>(), c->d_byorig.as<HitRec>());
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipEventRecord(c->ev_b, c->stream));
  HIP_TRY(c, hipEventSynchronize(c->ev_b));
  float ms = 0.f;
  HIP_TRY(c, hipEventElapsedTime(&ms, c->ev_a, c->ev_b));
  c->stats.index_ms = ms;
  return MKF_OK;
}

}  // namespace

extern "C" {

mkf_status mkf_load_geometry(mkf_ctx *c, const mkf_layer *layers, int32_t n_layers) {
  if (!c) return MKF_E_ARG;
  if (!layers || n_layers <= 0 || n_layers > MKF_MAX_LAYERS)
    return fail(c, MKF_E_ARG, "need 1..%d layers", MKF_MAX_LAYERS);
  for (int i = 0; i < n_layers; ++i) {
    const mkf_layer &L = layers[i];
    if (L.kind != MKF_BARREL && L.kind != MKF_DISK)
      return fail(c, MKF_E_GEOMETRY, "layer %d: bad kind %d", i, L.kind);
    if (!finite_f(L.pos) || !finite_f(L.ext_lo) || !finite_f(L.ext_hi) ||
        !(L.ext_lo < L.ext_hi))
      return fail(c, MKF_E_GEOMETRY, "layer %d: bad position or extent", i);
    if (L.kind == MKF_BARREL && !(L.pos > 0.f))
      return fail(c, MKF_E_GEOMETRY, "layer %d: barrel radius must be > 0", i);
    if (L.kind == MKF_DISK && !(L.ext_lo >= 0.f))
      return fail(c, MKF_E_GEOMETRY, "layer %d: disk inner radius must be >= 0", i);
    if (!(L.var_u_max > 0.f) || !(L.var_v_max > 0.f) || !finite_f(L.var_u_max) ||
        !finite_f(L.var_v_max))
      return fail(c, MKF_E_GEOMETRY, "layer %d: variance bounds must be > 0", i);
    if (L.n_phi_bins < 1 || L.n_phi_bins > 4096 || L.n_q_bins < 1 || L.n_q_bins > 1024)
      return fail(c, MKF_E_GEOMETRY, "layer %d: bin counts out of range", i);
    if (!finite_f(L.stereo) || !(std::fabs(L.stereo) < 1.5707f))
      return fail(c, MKF_E_GEOMETRY, "layer %d: stereo angle must lie in (-pi/2, pi/2)", i);
    if (!finite_f(L.hole_lo) || !finite_f(L.hole_hi))
      return fail(c, MKF_E_GEOMETRY, "layer %d: bad hole", i);
  }
  std::memcpy(c->user_layers, layers, sizeof(mkf_layer) * n_layers);
  c->n_layers = n_layers;
  mkf_status st = upload_layers(c);
  if (st != MKF_OK) return st;
  c->n_regions = 0;
  c->stage = kGeometry;
  return MKF_OK;
}

mkf_status mkf_load_material(mkf_ctx *c, const mkf_material_info *info, const float *x_x0,
                             const float *xi) {
  if (!c) return MKF_E_ARG;
  if (!info) {
    c->mat = DevMat{};
    drop_graph(c);
    return MKF_OK;
  }
  if (info->n_r < 1 || info->n_z < 1 || info->n_r > 4096 || info->n_z > 4096 ||
      (int64_t)info->n_r * info->n_z > (1 << 22))
    return fail(c, MKF_E_ARG, "material map: need 1..4096 bins per axis, at most 2^22 in all");
  if (!finite_f(info->r_max) || !(info->r_max > 0.f) || !finite_f(info->z_max) ||
      !(info->z_max > 0.f))
    return fail(c, MKF_E_ARG, "material map: r_max and z_max must be finite and > 0");
  if (!finite_f(info->mass) || !(info->mass > 0.f) || !finite_f(info->k_max) ||
      !(info->k_max >= 1.f))
    return fail(c, MKF_E_ARG, "material map: need mass > 0 and k_max >= 1");
  if (!x_x0 || !xi) return fail(c, MKF_E_ARG, "material map: NULL table");
  const size_t n = (size_t)info->n_r * (size_t)info->n_z;
  std::vector<float2> tab(n);
  for (size_t i = 0; i < n; ++i) {
    if (!finite_f(x_x0[i]) || !(x_x0[i] >= 0.f) || !(x_x0[i] <= 1.f) || !finite_f(xi[i]) ||
        !(xi[i] >= 0.f) || !(xi[i] <= 100.f))
      return fail(c, MKF_E_ARG, "material map: bin %zu out of range (0 <= x/X0 <= 1, 0 <= xi <= 100)",
                  i);
    tab[i] = make_float2(x_x0[i], xi[i]);
  }
  HIP_TRY(c, c->d_mat.ensure(sizeof(float2) * n));
  HIP_TRY(c, hipMemcpyAsync(c->d_mat.ptr, tab.data(), sizeof(float2) * n, hipMemcpyHostToDevice,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  DevMat m{};
  m.tab = c->d_mat.as<float2>();
  m.nr = info->n_r;
  m.nz = info->n_z;
  m.r_scale = (float)info->n_r / info->r_max;
  m.z_max = info->z_max;
  m.z_scale = (float)info->n_z / (2.f * info->z_max);
  m.mass = info->mass;
  m.k_max = info->k_max;
  c->mat = m;
  drop_graph(c);
  return MKF_OK;
}

mkf_status mkf_load_field(mkf_ctx *c, const mkf_field *f) {
  if (!c) return MKF_E_ARG;
  if (!f) {
    c->field = DevField{};
    drop_graph(c);
    return MKF_OK;
  }
  if (!finite_f(f->b0) || f->b0 == 0.f || !finite_f(f->c_r2) || !finite_f(f->c_z2) ||
      !finite_f(f->c_z4))
    return fail(c, MKF_E_ARG, "field: coefficients must be finite and b0 != 0");
  if (!finite_f(f->h_max) || !(f->h_max >= 0.01f) || !(f->h_max <= 100.f))
    return fail(c, MKF_E_ARG, "field: h_max must lie in [0.01, 100] cm");
  DevField d{};
  d.on = 1;
  d.kb0 = -c->cfg.kappa * f->b0;
  d.c_r2 = f->c_r2;
  d.c_z2 = f->c_z2;
  d.c_z4 = f->c_z4;
  d.h_max = f->h_max;
  c->field = d;
  drop_graph(c);
  return MKF_OK;
}

mkf_status mkf_load_steering(mkf_ctx *c, const mkf_region *regions, int32_t n_regions) {
  if (!c) return MKF_E_ARG;
  if (c->stage < kGeometry) return fail(c, MKF_E_ORDER, "load_geometry first");
  if (n_regions < 0 || n_regions > MKF_MAX_REGIONS || (n_regions > 0 && !regions))
    return fail(c, MKF_E_ARG, "need 0..%d regions", MKF_MAX_REGIONS);
  DevRegion dr[kMaxRegions]{};
  for (int r = 0; r < n_regions; ++r) {
    const mkf_region &g = regions[r];
    if (std::isnan(g.eta_lo) || std::isnan(g.eta_hi) || !(g.eta_lo < g.eta_hi))
      return fail(c, MKF_E_ARG, "region %d: need eta_lo < eta_hi", r);
    if (g.n_layers < 0 || g.n_layers > MKF_MAX_PLAN)
      return fail(c, MKF_E_ARG, "region %d: need 0..%d layers", r, MKF_MAX_PLAN);
    bool seen[kMaxLayers] = {};
    for (int k = 0; k < g.n_layers; ++k) {
      const int L = g.layers[k];
      if (L < 0 || L >= c->n_layers)
        return fail(c, MKF_E_ARG, "region %d: layer id %d not in the geometry", r, L);
      if (seen[L]) return fail(c, MKF_E_ARG, "region %d: layer %d listed twice", r, L);
      seen[L] = true;
      dr[r].layers[k] = (int8_t)L;
    }
    dr[r].eta_lo = g.eta_lo;
    dr[r].eta_hi = g.eta_hi;
    dr[r].n = g.n_layers;
  }
  HIP_TRY(c, c->d_regions.ensure(sizeof(dr)));
  HIP_TRY(c, hipMemcpyAsync(c->d_regions.ptr, dr, sizeof(dr), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->n_regions = n_regions;
  return MKF_OK;
}

mkf_status mkf_load_hits(mkf_ctx *c, int32_t n_events, const int64_t *ev_off, const float *x,
                         const float *y, const float *z, const float *var_u,
                         const float *var_v, const int32_t *layer, int32_t mem) {
  if (!c) return MKF_E_ARG;
  if (c->stage < kGeometry) return fail(c, MKF_E_ORDER, "load_geometry first");
  if (n_events < 0 || !ev_off) return fail(c, MKF_E_ARG, "bad event offsets");
  if (mem != MKF_MEM_HOST && mem != MKF_MEM_DEVICE) return fail(c, MKF_E_ARG, "bad mem");
  if (ev_off[0] != 0) return fail(c, MKF_E_ARG, "ev_off[0] must be 0");
  for (int e = 0; e < n_events; ++e) {
    const int64_t n = ev_off[e + 1] - ev_off[e];
    if (n < 0) return fail(c, MKF_E_ARG, "event offsets must not decrease");
    if (n >= (int64_t)0x7FFFFF) return fail(c, MKF_E_CAPACITY, "event %d has too many hits", e);
  }
  const int64_t n_hits = ev_off[n_events];
  if (n_hits > 0 && (!x || !y || !z || !var_u || !var_v || !layer))
    return fail(c, MKF_E_ARG, "hit array is NULL");
  if (n_hits >= ((int64_t)1 << 31)) return fail(c, MKF_E_CAPACITY, "too many hits");
  const int64_t total_bins = (int64_t)n_events * c->bins_per_event;
  if (total_bins >= ((int64_t)1 << 31) - 1)
    return fail(c, MKF_E_CAPACITY, "events x bins exceed the index size");
  if (mem == MKF_MEM_HOST) {
    for (int64_t i = 0; i < n_hits; ++i) {
      if (!finite_f(x[i]) || !finite_f(y[i]) || !finite_f(z[i]) || !finite_f(var_u[i]) ||
          !finite_f(var_v[i]) || !(var_u[i] > 0.f) || !(var_v[i] > 0.f))
        return fail(c, MKF_E_ARG, "hit %lld: non-finite value or variance <= 0", (long long)i);
      if (layer[i] < 0 || layer[i] >= c->n_layers)
        return fail(c, MKF_E_ARG, "hit %lld: layer %d out of range", (long long)i, layer[i]);
    }
  }
  c->stage = kGeometry;
  drop_graph(c);
  const size_t fb = sizeof(float) * (size_t)n_hits;
  mkf_status st;
  if ((st = stage_in(c, c->d_ev_off, ev_off, sizeof(int64_t) * (n_events + 1), MKF_MEM_HOST))) return st;
  if ((st = stage_in(c, c->d_x, x, fb, mem))) return st;
  if ((st = stage_in(c, c->d_y, y, fb, mem))) return st;
  if ((st = stage_in(c, c->d_z, z, fb, mem))) return st;
  if ((st = stage_in(c, c->d_vu, var_u, fb, mem))) return st;
  if ((st = stage_in(c, c->d_vv, var_v, fb, mem))) return st;
  if ((st = stage_in(c, c->d_layer, layer, sizeof(int) * (size_t)n_hits, mem))) return st;
  if (mem == MKF_MEM_DEVICE && n_hits > 0) {
    HIP_TRY(c, hipMemsetAsync(c->d_bad.ptr, 0, sizeof(int), c->stream));
    launch_validate_hits(c->stream, n_hits, c->d_x.as<float>(), c->d_y.as<float>(),
                         c->d_z.as<float>(), c->d_vu.as<float>(), c->d_vv.as<float>(),
                         c->d_layer.as<int>(), c->n_layers, c->d_bad.as<int>());
    int bad = 0;
    HIP_TRY(c, hipMemcpyAsync(&bad, c->d_bad.ptr, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (bad) return fail(c, MKF_E_ARG, "hits: non-finite value, variance <= 0 or bad layer");
  }
  c->n_events = n_events;
  c->n_hits = n_hits;
  c->ev_off.assign(ev_off, ev_off + n_events + 1);
  if ((st = build_index(c))) return st;
  c->stage = kHits;
  c->n_seeds = 0;
  return MKF_OK;
}

mkf_status mkf_seed(mkf_ctx *c, int64_t n_seeds, const int32_t *seed_event,
                    const int32_t *seed_hits, int32_t mem) {
  if (!c) return MKF_E_ARG;
  if (c->stage < kHits) return fail(c, MKF_E_ORDER, "load_hits first");
  if (n_seeds < 0 || n_seeds >= ((int64_t)1 << 28)) return fail(c, MKF_E_ARG, "bad seed count");
  if (n_seeds > 0 && (!seed_event || !seed_hits)) return fail(c, MKF_E_ARG, "seed array is NULL");
  if (mem != MKF_MEM_HOST && mem != MKF_MEM_DEVICE) return fail(c, MKF_E_ARG, "bad mem");
  std::vector<int32_t> h_ev, h_hits;
  const int32_t *sev = seed_event, *sh = seed_hits;
  if (mem == MKF_MEM_DEVICE && n_seeds > 0) {
    // seeds are small: validate on the host
    h_ev.resize(n_seeds);
    h_hits.resize(3 * n_seeds);
    HIP_TRY(c, hipMemcpyAsync(h_ev.data(), seed_event, 4 * n_seeds, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(h_hits.data(), seed_hits, 12 * n_seeds, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    sev = h_ev.data();
    sh = h_hits.data();
  }
  for (int64_t i = 0; i < n_seeds; ++i) {
    if (sev[i] < 0 || sev[i] >= c->n_events)
      return fail(c, MKF_E_ARG, "seed %lld: event %d out of range", (long long)i, sev[i]);
    const int64_t nh = c->ev_off[sev[i] + 1] - c->ev_off[sev[i]];
    for (int k = 0; k < 3; ++k)
      if (sh[3 * i + k] < 0 || sh[3 * i + k] >= nh)
        return fail(c, MKF_E_ARG, "seed %lld: hit index out of range", (long long)i);
  }
  c->stage = kHits;
  drop_graph(c);
  const size_t N = (size_t)std::max<int64_t>(n_seeds, 1);
  mkf_status st;
  if ((st = stage_in(c, c->d_seed_event, sev, 4 * (size_t)n_seeds, MKF_MEM_HOST))) return st;
  if ((st = stage_in(c, c->d_seed_hits, sh, 12 * (size_t)n_seeds, MKF_MEM_HOST))) return st;
  HIP_TRY(c, c->d_seed_event.ensure(4 * N));
  HIP_TRY(c, c->d_seed_state.ensure(sizeof(float) * 27 * N));
  HIP_TRY(c, c->d_seed_ok.ensure(4 * N));
  HIP_TRY(c, c->d_plan_len.ensure(4 * N));
  HIP_TRY(c, c->d_plan.ensure(kMaxPlan * N));
  HIP_TRY(c, c->d_plan_l.ensure(sizeof(double) * kMaxPlan * N));
  HIP_TRY(c, c->d_order.ensure(4 * N));
  HIP_TRY(c, c->d_seed_chi2.ensure(4 * N));
  c->n_seeds = n_seeds;
  FindParams P = params(c);
  HIP_TRY(c, hipEventRecord(c->ev_a, c->stream));
  launch_seed(c->stream, P, c->d_seed_hits.as<int>(), c->d_seed_state.as<float>(),
              c->d_seed_ok.as<int>(), c->d_plan_len.as<int>(), c->d_plan.as<int8_t>(),
              c->d_plan_l.as<double>(), c->d_seed_chi2.as<float>(),
              c->n_regions > 0 ? c->d_regions.as<DevRegion>() : nullptr, c->n_regions);
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipEventRecord(c->ev_b, c->stream));
  // processing order: longest plans first (the persistent form takes tiles
  // in this order, so the longest work starts first), then by event and
  // direction so that a wavefront's seeds search nearby hits
  std::vector<int32_t> plen(n_seeds), ok(n_seeds), ev(sev, sev + n_seeds);
  std::vector<float> phi(n_seeds), theta(n_seeds);
  if (n_seeds > 0) {
    HIP_TRY(c, hipMemcpyAsync(plen.data(), c->d_plan_len.ptr, 4 * n_seeds, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(ok.data(), c->d_seed_ok.ptr, 4 * n_seeds, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(phi.data(), c->d_seed_state.as<float>() + 4 * N, 4 * n_seeds,
                              hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(theta.data(), c->d_seed_state.as<float>() + 5 * N, 4 * n_seeds,
                              hipMemcpyDeviceToHost, c->stream));
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  float ms = 0.f;
  HIP_TRY(c, hipEventElapsedTime(&ms, c->ev_a, c->ev_b));
  c->stats.seed_ms = ms;
  std::vector<int32_t> order(n_seeds);
  std::iota(order.begin(), order.end(), 0);
  int64_t q_off[kQueues + 1] = {};
  if (c->cfg.flags & MKF_F_BATCHED) {
    // whole events to the kQueues tile queues (one per XCD), balanced by
    // their summed plan lengths (longest first to the least loaded queue);
    // inside a queue event by event, longest plans first, then direction
    std::vector<int64_t> cost(c->n_events, 0);
    for (int64_t i = 0; i < n_seeds; ++i) cost[ev[i]] += plen[i] + 1;
    std::vector<int> evs(c->n_events), ev_q(c->n_events, 0);
    std::iota(evs.begin(), evs.end(), 0);
    std::stable_sort(evs.begin(), evs.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    int64_t load[kQueues] = {};
    for (int e : evs) {
      int q = 0;
      for (int k = 1; k < kQueues; ++k)
        if (load[k] < load[q]) q = k;
      ev_q[e] = q;
      load[q] += cost[e];
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      if (ev_q[ev[a]] != ev_q[ev[b]]) return ev_q[ev[a]] < ev_q[ev[b]];
      if (ev[a] != ev[b]) return ev[a] < ev[b];
      if (plen[a] != plen[b]) return plen[a] > plen[b];
      const int ta = (int)(theta[a] * 8.f), tb = (int)(theta[b] * 8.f);
      if (ta != tb) return ta < tb;
      return phi[a] < phi[b];
    });
    for (int64_t p = 0; p < n_seeds; ++p) q_off[ev_q[ev[order[p]]] + 1]++;
    for (int q = 0; q < kQueues; ++q) q_off[q + 1] += q_off[q];
  } else {
    // longest plans first, so the seeds still active at a step form a prefix
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      if (plen[a] != plen[b]) return plen[a] > plen[b];
      if (ev[a] != ev[b]) return ev[a] < ev[b];
      const int ta = (int)(theta[a] * 8.f), tb = (int)(theta[b] * 8.f);
      if (ta != tb) return ta < tb;
      return phi[a] < phi[b];
    });
    for (int q = 1; q <= kQueues; ++q) q_off[q] = n_seeds;
  }
  HIP_TRY(c, c->d_qoff.ensure(sizeof(q_off)));
  HIP_TRY(c, hipMemcpyAsync(c->d_qoff.ptr, q_off, sizeof(q_off), hipMemcpyHostToDevice, c->stream));
  if (n_seeds > 0)
    HIP_TRY(c, hipMemcpyAsync(c->d_order.ptr, order.data(), 4 * n_seeds, hipMemcpyHostToDevice, c->stream));
  c->max_plan_len = 0;
  c->n_seeds_ok = 0;
  for (int64_t i = 0; i < n_seeds; ++i) {
    c->max_plan_len = std::max(c->max_plan_len, plen[i]);
    c->n_seeds_ok += ok[i] ? 1 : 0;
  }
  c->active_at_step.assign(kMaxPlan, 0);
  for (int s = 0; s < kMaxPlan; ++s) {
    // the layer-synchronous form keeps the longest plans first: the seeds
    // still active at step s form a prefix of the positions
    int64_t n = 0;
    for (int64_t i = 0; i < n_seeds; ++i) n += plen[i] > s ? 1 : 0;
    c->active_at_step[s] = (c->cfg.flags & MKF_F_BATCHED) ? n_seeds : n;
  }
  // find buffers
  HIP_TRY(c, c->d_cand.ensure(sizeof(float) * kCandFields * kGroup * N));
  HIP_TRY(c, c->d_fin_key.ensure(8 * N));
  HIP_TRY(c, c->d_fin_rec.ensure(sizeof(float) * 28 * N));
  HIP_TRY(c, c->d_fin_meta.ensure(4 * N));
  HIP_TRY(c, c->d_bp.ensure(4 * (size_t)kMaxPlan * kGroup * N));
  HIP_TRY(c, c->d_pstate.ensure(sizeof(float) * kSeedWords * N));
  HIP_TRY(c, c->d_pinfo.ensure(4 * N));
  HIP_TRY(c, c->d_pevent.ensure(4 * N));
  HIP_TRY(c, c->d_pplan.ensure(kMaxPlan * N));
  HIP_TRY(c, c->d_out.ensure(sizeof(float) * kOutWords * N));
  {
    FindParams Q = params(c);
    launch_permute_seeds(c->stream, Q, c->d_pstate.as<float>(), c->d_pinfo.as<int>(),
                         c->d_pevent.as<int>(), c->d_pplan.as<int8_t>());
    HIP_TRY(c, hipGetLastError());
  }
  c->h_order = order;
  c->h_plen = plen;
  c->h_ok = ok;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->stats.n_seeds = n_seeds;
  c->stats.n_seeds_ok = c->n_seeds_ok;
  c->stats.max_plan_len = c->max_plan_len;
  c->stage = kSeeds;
  return MKF_OK;
}

mkf_status mkf_get_seed_states(mkf_ctx *c, float *par, float *cov, int32_t *ok,
                               int32_t *plan_len, int8_t *plan, float *chi2) {
  if (!c) return MKF_E_ARG;
  if (c->stage < kSeeds) return fail(c, MKF_E_ORDER, "seed first");
  const size_t n = (size_t)c->n_seeds, N = std::max<size_t>(n, 1);
  if (n == 0) return MKF_OK;
  std::vector<float> st(27 * N);
  HIP_TRY(c, hipMemcpyAsync(st.data(), c->d_seed_state.ptr, sizeof(float) * 27 * N,
                            hipMemcpyDeviceToHost, c->stream));
  if (ok) HIP_TRY(c, hipMemcpyAsync(ok, c->d_seed_ok.ptr, 4 * n, hipMemcpyDeviceToHost, c->stream));
  if (plan_len)
    HIP_TRY(c, hipMemcpyAsync(plan_len, c->d_plan_len.ptr, 4 * n, hipMemcpyDeviceToHost, c->stream));
  if (plan)
    HIP_TRY(c, hipMemcpyAsync(plan, c->d_plan.ptr, kMaxPlan * n, hipMemcpyDeviceToHost, c->stream));
  if (chi2)
    HIP_TRY(c, hipMemcpyAsync(chi2, c->d_seed_chi2.ptr, 4 * n, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (size_t i = 0; i < n; ++i) {
    if (par)
      for (int k = 0; k < 6; ++k) par[6 * i + k] = st[k * N + i];
    if (cov)
      for (int k = 0; k < 21; ++k) cov[21 * i + k] = st[(6 + k) * N + i];
  }
  return MKF_OK;
}

// Queue the whole find on the context stream.  main_a/main_b (may be
// null) bracket the layer-step kernels.
static int enqueue_find(mkf_ctx *c, const FindParams &P, hipEvent_t main_a, hipEvent_t main_b) {
  int launches = 0;
  launch_fill_u64(c->stream, c->d_steps.as<unsigned long long>(), 1, 0ull);
  launch_fill_u64(c->stream, c->d_cnt.as<unsigned long long>(), kCounters * kCounterSlots, 0ull);
  ++launches;
  if (c->cfg.flags & MKF_F_BATCHED) {
    launch_fill_i32(c->stream, c->d_tiles.as<int>(), kQueues, 0);
    ++launches;
    if (main_a) (void)hipEventRecord(main_a, c->stream);
    launch_find_persistent(c->stream, P, c->tuning.blocks_per_cu * c->n_cu,
                           c->tuning.waves_per_simd, (c->cfg.flags & MKF_F_SURROGATE) != 0,
                           c->tuning.lane_group);
    ++launches;
    c->stats.main_launches = 1;
  } else {
    launch_find_init(c->stream, P);
    ++launches;
    if (main_a) (void)hipEventRecord(main_a, c->stream);
    int n = 0;
    for (int s = 0; s < c->max_plan_len; ++s) {
      launch_find_step(c->stream, P, s, c->active_at_step[s]);
      ++n;
    }
    launches += n;
    c->stats.main_launches = n;
  }
  if (main_b) (void)hipEventRecord(main_b, c->stream);
  if (!(c->cfg.flags & MKF_F_BATCHED)) {
    launch_finalize(c->stream, P);
    ++launches;
  }
  return launches;
}

mkf_status mkf_find(mkf_ctx *c) {
  if (!c) return MKF_E_ARG;
  if (c->stage < kSeeds) return fail(c, MKF_E_ORDER, "seed first");
  FindParams P = params(c);
  int launches = 0;
  const bool graph = (c->cfg.flags & MKF_F_GRAPH) != 0;
  if (graph && !c->graph_exec) {
    if (!c->stream)
      return fail(c, MKF_E_ARG, "graph replay needs a non-default stream at mkf_create");
    HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    c->graph_launches = enqueue_find(c, P, nullptr, nullptr);
    hipError_t e = hipStreamEndCapture(c->stream, &c->graph);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      drop_graph(c);
      return fail(c, MKF_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
    }
  }
  HIP_TRY(c, hipEventRecord(c->ev_a, c->stream));
  if (graph) {
    HIP_TRY(c, hipGraphLaunch(c->graph_exec, c->stream));
    launches = c->graph_launches;
  } else {
    launches = enqueue_find(c, P, c->ev_m0, c->ev_m1);
  }
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipEventRecord(c->ev_b, c->stream));
  // (after the timed region: the checked find's record invariants)
  if (c->cfg.flags & MKF_F_CHECKED) {
    launch_check_results(c->stream, P);
    HIP_TRY(c, hipGetLastError());
  }
  // the step count and counters: two copies into pinned memory behind the
  // find on its stream, then one wait, which also completes the events
  unsigned long long *cnt = c->h_cnt + 1;
  HIP_TRY(c, hipMemcpyAsync(c->h_cnt, c->d_steps.ptr, sizeof(unsigned long long),
                            hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(cnt, c->d_cnt.ptr,
                            sizeof(unsigned long long) * kCounters * kCounterSlots,
                            hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  float ms = 0.f, mms = -1.f;
  HIP_TRY(c, hipEventElapsedTime(&ms, c->ev_a, c->ev_b));
  if (!graph) HIP_TRY(c, hipEventElapsedTime(&mms, c->ev_m0, c->ev_m1));
  const unsigned long long steps = c->h_cnt[0];
  int64_t tot[kCounters] = {};
  for (int k = 0; k < kCounters; ++k)
    for (int j = 0; j < kCounterSlots; ++j) tot[k] += (int64_t)cnt[k * kCounterSlots + j];
  c->stats.sur_kept = tot[kCntSurKept];
  c->stats.sur_rejected = tot[kCntSurRejected];
  c->stats.n_near_cut = tot[kCntNearCut];
  c->stats.n_rk_steps = tot[kCntRk];
  c->stats.n_newton = tot[kCntNewton];
  c->stats.n_check_failed = tot[kCntCheckFailed];
  c->stats.find_ms = ms;
  c->stats.main_ms = mms;
  c->stats.n_steps = (int64_t)steps;
  c->stats.n_launches = launches;
  c->stage = kFound;
  if (c->stats.n_check_failed > 0)
    return fail(c, MKF_E_NUMERIC, "checked find: %lld result records violate the find's invariants",
                (long long)c->stats.n_check_failed);
  return MKF_OK;
}

mkf_status mkf_get_tracks(mkf_ctx *c, mkf_track *out, int64_t capacity, int64_t *n_total) {
  if (!c) return MKF_E_ARG;
  if (c->stage < kFound) return fail(c, MKF_E_ORDER, "find first");
  if (n_total) *n_total = c->n_seeds;
  if (capacity < 0 || (capacity > 0 && !out)) return fail(c, MKF_E_ARG, "bad output buffer");
  const size_t N = (size_t)c->n_seeds;
  if (N > 0) {
    // results are kept by processing position, one record per seed
    std::vector<float> res((size_t)kOutWords * N);
    std::vector<int8_t> plan((size_t)kMaxPlan * N);
    HIP_TRY(c, hipMemcpyAsync(res.data(), c->d_out.ptr, sizeof(float) * kOutWords * N,
                              hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(plan.data(), c->d_plan.ptr, (size_t)kMaxPlan * N,
                              hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (size_t pos = 0; pos < N; ++pos) {
      const int seed = c->h_order[pos];
      if (seed >= capacity) continue;
      mkf_track &T = out[seed];
      const bool ok = c->h_ok[seed] != 0;
      const int plen = ok ? c->h_plen[seed] : 0;
      T.seed_id = seed;
      T.status = ok ? 1 : 0;
      auto row = [&](int r) { return res[pos * kOutWords + r]; };
      auto irow = [&](int r) {
        int32_t v;
        std::memcpy(&v, &res[pos * kOutWords + r], 4);
        return v;
      };
      const int32_t meta = irow(kOutMeta);
      T.n_hits = meta & 0xFF;
      T.n_miss = (meta >> 8) & 0xFF;
      T.plan_len = plen;
      T.chi2 = row(kOutChi2);
      for (int i = 0; i < 6; ++i) T.par[i] = row(kOutPar + i);
      for (int i = 0; i < 21; ++i) T.cov[i] = row(kOutCov + i);
      for (int k = 0; k < kMaxPlan; ++k) {
        T.plan[k] = k < plen ? plan[(size_t)seed * kMaxPlan + k] : (int8_t)-1;
        T.hit[k] = k < plen ? irow(kOutHit + k) : MKF_HIT_NONE;
      }
    }
  }
  if (capacity < c->n_seeds)
    return fail(c, MKF_E_CAPACITY, "capacity %lld < %lld tracks", (long long)capacity,
                (long long)c->n_seeds);
  return MKF_OK;
}

mkf_status mkf_propagate(mkf_ctx *c, int64_t n, const float *par, const float *cov,
                         const int32_t *layer, float *out_par, float *out_cov, float *out_l,
                         int32_t *out_status) {
  if (!c) return MKF_E_ARG;
  if (c->stage < kGeometry) return fail(c, MKF_E_ORDER, "load_geometry first");
  if (n < 0) return fail(c, MKF_E_ARG, "n < 0");
  if (n > 0 && (!par || !cov || !layer || !out_par || !out_cov || !out_l || !out_status))
    return fail(c, MKF_E_ARG, "NULL array");
  FindParams P = params(c);
  launch_propagate(c->stream, P, n, par, cov, layer, out_par, out_cov, out_l, out_status);
  HIP_TRY(c, hipGetLastError());
  return MKF_OK;
}

mkf_status mkf_fit(mkf_ctx *c, int64_t n_tracks, int32_t n_steps, const int8_t *kind,
                   const float *pos, const float *x, const float *y, const float *z,
                   const float *var_u, const float *var_v, const int32_t *len,
                   const float *init_par, const float *init_cov, float *out_par, float *out_cov,
                   float *out_chi2, int32_t *out_status) {
  if (!c) return MKF_E_ARG;
  if (n_tracks < 0 || n_steps < 0) return fail(c, MKF_E_ARG, "negative size");
  if (n_tracks > 0 && (!len || !init_par || !init_cov || !out_par || !out_cov || !out_chi2 ||
                       !out_status))
    return fail(c, MKF_E_ARG, "NULL array");
  if (n_tracks > 0 && n_steps > 0 && (!kind || !pos || !x || !y || !z || !var_u || !var_v))
    return fail(c, MKF_E_ARG, "NULL hit array");
  HIP_TRY(c, hipEventRecord(c->ev_a, c->stream));
  DevCfg fcfg = dev_cfg(c->cfg);
  fcfg.mat = c->mat;
  fcfg.field = c->field;
  launch_fit(c->stream, fcfg, n_tracks, n_steps, kind, pos, x, y, z, var_u, var_v, len,
             init_par, init_cov, out_par, out_cov, out_chi2, out_status);
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipEventRecord(c->ev_b, c->stream));
  return MKF_OK;
}

mkf_status mkf_backward_fit(mkf_ctx *c, float *out_par, float *out_cov, float *out_chi2,
                            int32_t *out_status) {
  if (!c) return MKF_E_ARG;
  if (c->stage < kFound) return fail(c, MKF_E_ORDER, "find first");
  if (c->n_seeds > 0 && (!out_par || !out_cov || !out_chi2 || !out_status))
    return fail(c, MKF_E_ARG, "NULL output array");
  HIP_TRY(c, c->d_bf_tmp.ensure(sizeof(float) * 32 * (size_t)std::max<int64_t>(c->n_seeds, 1)));
  FindParams P = params(c);
  launch_backfit(c->stream, P, c->d_seed_hits.as<int>(), c->d_bf_tmp.as<float>(), out_par,
                 out_cov, out_chi2, out_status);
  HIP_TRY(c, hipGetLastError());
  return MKF_OK;
}

mkf_status mkf_smooth(mkf_ctx *c, float *out_par, float *out_cov, int32_t *out_n) {
  if (!c) return MKF_E_ARG;
  if (c->stage < kFound) return fail(c, MKF_E_ORDER, "find first");
  if (c->n_seeds > 0 && (!out_par || !out_cov || !out_n))
    return fail(c, MKF_E_ARG, "NULL output array");
  const size_t N = (size_t)std::max<int64_t>(c->n_seeds, 1);
  HIP_TRY(c, c->d_sm_wk.ensure(sizeof(float) * 91 * (size_t)(c->max_plan_len + 1) * N));
  HIP_TRY(c, c->d_sm_n.ensure(sizeof(int) * N));
  FindParams P = params(c);
  launch_smooth(c->stream, P, c->d_seed_hits.as<int>(), c->d_sm_wk.as<float>(),
                c->d_sm_n.as<int>(), out_par, out_cov, out_n);
  HIP_TRY(c, hipGetLastError());
  return MKF_OK;
}

mkf_status mkf_make_seeds(mkf_ctx *c, const mkf_seeding *sc, int64_t capacity,
                          int32_t *out_event, int32_t *out_hits, int64_t *n_total) {
  if (!c) return MKF_E_ARG;
  if (c->stage < kHits) return fail(c, MKF_E_ORDER, "load_hits first");
  if (!sc || !n_total || capacity < 0) return fail(c, MKF_E_ARG, "NULL argument");
  if (capacity > 0 && (!out_event || !out_hits)) return fail(c, MKF_E_ARG, "NULL output array");
  for (int k = 0; k < 3; ++k) {
    const int L = sc->layers[k];
    if (L < 0 || L >= c->n_layers || c->layers[L].kind != MKF_BARREL)
      return fail(c, MKF_E_ARG, "seeding layer %d is not a barrel layer", L);
    if (k > 0 && !(c->layers[L].pos > c->layers[sc->layers[k - 1]].pos))
      return fail(c, MKF_E_ARG, "seeding layers must have increasing radii");
  }
  if (!(sc->pt_min > 0.f) || !(sc->d0_max > 0.f) || !(sc->z0_max > 0.f) || !(sc->dz_max > 0.f))
    return fail(c, MKF_E_ARG, "seeding cuts must be positive");
  if (c->cfg.bz == 0.f) return fail(c, MKF_E_ARG, "triplet seeding needs a field");
  if (c->n_events > 65535) return fail(c, MKF_E_CAPACITY, "triplet seeding takes <= 65535 events");
  *n_total = 0;
  const int64_t n = c->n_hits;
  if (n == 0) return MKF_OK;
  DevSeeding ds{};
  for (int k = 0; k < 3; ++k) ds.layer[k] = sc->layers[k];
  ds.pt_min = sc->pt_min;
  ds.d0_max = sc->d0_max;
  ds.z0_max = sc->z0_max;
  ds.dz_max = sc->dz_max;
  HIP_TRY(c, c->d_tr_cnt.ensure(sizeof(int) * (size_t)n));
  HIP_TRY(c, c->d_tr_off.ensure(sizeof(int) * (size_t)(n + 1)));
  HIP_TRY(c, c->d_tr_tmp.ensure(sizeof(int) * (size_t)(4 * (n / 2048 + 4) + 64)));
  FindParams P = params(c);
  int64_t max_ev = 0;
  for (int e = 0; e < c->n_events; ++e) max_ev = std::max(max_ev, c->ev_off[e + 1] - c->ev_off[e]);
  launch_fill_i32(c->stream, c->d_tr_cnt.as<int>(), n, 0);
  launch_triplets(c->stream, P, ds, max_ev, false, c->d_tr_cnt.as<int>(), nullptr, nullptr,
                  nullptr);
  HIP_TRY(c, hipGetLastError());
  launch_scan(c->stream, c->d_tr_cnt.as<int>(), c->d_tr_off.as<int>(), n, c->d_tr_tmp.as<int>(),
              nullptr);
  HIP_TRY(c, hipGetLastError());
  int total = 0;
  HIP_TRY(c, hipMemcpyAsync(&total, c->d_tr_off.as<int>() + n, sizeof(int), hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (total < 0) return fail(c, MKF_E_CAPACITY, "more than 2^31 triplets");
  *n_total = total;
  if (total > capacity)
    return fail(c, MKF_E_CAPACITY, "%d triplets, capacity %lld", total, (long long)capacity);
  launch_triplets(c->stream, P, ds, max_ev, true, c->d_tr_cnt.as<int>(), c->d_tr_off.as<int>(),
                  out_event, out_hits);
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return MKF_OK;
}

mkf_status mkf_find_duplicates(mkf_ctx *c, float frac, int32_t *out_dup, int64_t *n_dup) {
  if (!c) return MKF_E_ARG;
  if (c->stage < kFound) return fail(c, MKF_E_ORDER, "find first");
  if (!n_dup || (c->n_seeds > 0 && !out_dup)) return fail(c, MKF_E_ARG, "NULL argument");
  if (!(frac > 0.f && frac <= 1.f)) return fail(c, MKF_E_ARG, "frac must lie in (0, 1]");
  *n_dup = 0;
  if (c->n_seeds == 0) return MKF_OK;
  const size_t N = (size_t)c->n_seeds, H = (size_t)std::max<int64_t>(c->n_hits, 1);
  HIP_TRY(c, c->d_dup_h.ensure(sizeof(int) * kDupStride * N));
  HIP_TRY(c, c->d_dup_n.ensure(sizeof(int) * N));
  HIP_TRY(c, c->d_dup_cnt.ensure(sizeof(int) * H));
  HIP_TRY(c, c->d_dup_off.ensure(sizeof(int) * (H + 1)));
  HIP_TRY(c, c->d_dup_fill.ensure(sizeof(int) * H));
  HIP_TRY(c, c->d_dup_list.ensure(sizeof(int) * (kDupStride - 1) * N));
  HIP_TRY(c, c->d_dup_tmp.ensure(sizeof(int) * (4 * (H / 2048 + 4) + 64)));
  HIP_TRY(c, c->d_dup_total.ensure(sizeof(int)));
  FindParams P = params(c);
  launch_fill_i32(c->stream, c->d_dup_cnt.as<int>(), (int64_t)H, 0);
  launch_fill_i32(c->stream, c->d_dup_fill.as<int>(), (int64_t)H, 0);
  launch_fill_i32(c->stream, c->d_dup_total.as<int>(), 1, 0);
  launch_dup_prep(c->stream, P, c->d_seed_hits.as<int>(), c->d_dup_h.as<int>(),
                  c->d_dup_n.as<int>(), c->d_dup_cnt.as<int>());
  launch_scan(c->stream, c->d_dup_cnt.as<int>(), c->d_dup_off.as<int>(), (int64_t)H,
              c->d_dup_tmp.as<int>(), nullptr);
  launch_dup_fill(c->stream, P, c->d_dup_h.as<int>(), c->d_dup_n.as<int>(),
                  c->d_dup_off.as<int>(), c->d_dup_fill.as<int>(), c->d_dup_list.as<int>());
  launch_dup_decide(c->stream, P, c->d_seed_hits.as<int>(), c->d_dup_h.as<int>(),
                    c->d_dup_n.as<int>(), c->d_dup_off.as<int>(), c->d_dup_list.as<int>(), frac,
                    out_dup, c->d_dup_total.as<int>());
  HIP_TRY(c, hipGetLastError());
  int total = 0;
  HIP_TRY(c, hipMemcpyAsync(&total, c->d_dup_total.ptr, sizeof(int), hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  *n_dup = total;
  return MKF_OK;
}

mkf_status mkf_clean_seeds(mkf_ctx *c, const mkf_cleaning *cc, int32_t *out_keep,
                           int64_t *n_keep) {
  if (!c) return MKF_E_ARG;
  if (c->stage < kSeeds) return fail(c, MKF_E_ORDER, "seed first");
  if (!cc || !n_keep || (c->n_seeds > 0 && !out_keep)) return fail(c, MKF_E_ARG, "NULL argument");
  if (!(cc->tol_ipt >= 0.f) || !(cc->tol_eta >= 0.f) || !(cc->tol_phi >= 0.f))
    return fail(c, MKF_E_ARG, "tolerances must not be negative");
  *n_keep = 0;
  if (c->n_seeds == 0) return MKF_OK;
  const size_t N = (size_t)c->n_seeds, H = (size_t)std::max<int64_t>(c->n_hits, 1);
  // the duplicate-removal scratch serves here too (3 hits per seed)
  HIP_TRY(c, c->d_dup_h.ensure(sizeof(int) * 3 * N));
  HIP_TRY(c, c->d_dup_cnt.ensure(sizeof(int) * H));
  HIP_TRY(c, c->d_dup_off.ensure(sizeof(int) * (H + 1)));
  HIP_TRY(c, c->d_dup_fill.ensure(sizeof(int) * H));
  HIP_TRY(c, c->d_dup_list.ensure(sizeof(int) * 3 * N));
  HIP_TRY(c, c->d_dup_tmp.ensure(sizeof(int) * (4 * (H / 2048 + 4) + 64)));
  HIP_TRY(c, c->d_dup_total.ensure(sizeof(int)));
  FindParams P = params(c);
  DevCleaning dc{cc->tol_ipt, cc->tol_eta, cc->tol_phi};
  launch_fill_i32(c->stream, c->d_dup_cnt.as<int>(), (int64_t)H, 0);
  launch_fill_i32(c->stream, c->d_dup_fill.as<int>(), (int64_t)H, 0);
  launch_fill_i32(c->stream, c->d_dup_total.as<int>(), 1, 0);
  launch_clean_prep(c->stream, P, c->d_seed_hits.as<int>(), c->d_dup_h.as<int>(),
                    c->d_dup_cnt.as<int>());
  launch_scan(c->stream, c->d_dup_cnt.as<int>(), c->d_dup_off.as<int>(), (int64_t)H,
              c->d_dup_tmp.as<int>(), nullptr);
  launch_clean_fill(c->stream, P, c->d_dup_h.as<int>(), c->d_dup_off.as<int>(),
                    c->d_dup_fill.as<int>(), c->d_dup_list.as<int>());
  launch_clean_decide(c->stream, P, c->d_seed_hits.as<int>(), c->d_seed_chi2.as<float>(),
                      c->d_dup_h.as<int>(), c->d_dup_off.as<int>(), c->d_dup_list.as<int>(), dc,
                      out_keep, c->d_dup_total.as<int>());
  HIP_TRY(c, hipGetLastError());
  int total = 0;
  HIP_TRY(c, hipMemcpyAsync(&total, c->d_dup_total.ptr, sizeof(int), hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  *n_keep = total;
  return MKF_OK;
}

mkf_status mkf_get_stats(mkf_ctx *c, mkf_stats *out) {
  if (!c || !out) return MKF_E_ARG;
  *out = c->stats;
  return MKF_OK;
}

}  // extern "C"

namespace {

bool tuning_ok(const mkf_ctx *c, const mkf_tuning &t) {
  return t.waves_per_simd >= 1 && t.waves_per_simd <= 4 && t.blocks_per_cu >= 1 &&
         t.blocks_per_cu <= 32 &&
         (t.lane_group == 0 || t.lane_group == 8 || (t.lane_group == 6 && c->cfg.n_cand <= 6)) &&
         t.phi_bin_shift >= -2 && t.phi_bin_shift <= 2 && t.q_bin_shift >= -2 &&
         t.q_bin_shift <= 2;
}

// Apply a tuning; a change of the binning rebuilds the layer records and
// the index of loaded hits.
mkf_status apply_tuning(mkf_ctx *c, const mkf_tuning &t) {
  const bool rebin =
      t.phi_bin_shift != c->tuning.phi_bin_shift || t.q_bin_shift != c->tuning.q_bin_shift;
  c->tuning = t;
  drop_graph(c);
  if (!rebin || c->n_layers == 0) return MKF_OK;
  mkf_status st = upload_layers(c);
  if (st == MKF_OK && c->stage >= kHits) st = build_index(c);
  return st;
}

}  // namespace

extern "C" {

mkf_status mkf_set_tuning(mkf_ctx *c, const mkf_tuning *t) {
  if (!c) return MKF_E_ARG;
  if (!t || !tuning_ok(c, *t)) return fail(c, MKF_E_ARG, "tuning out of range");
  return apply_tuning(c, *t);
}

mkf_status mkf_get_tuning(mkf_ctx *c, mkf_tuning *t) {
  if (!c || !t) return MKF_E_ARG;
  *t = c->tuning;
  return MKF_OK;
}

mkf_status mkf_autotune(mkf_ctx *c, int32_t repeats, const char *cache_path, mkf_tuning *best) {
  if (!c) return MKF_E_ARG;
  if (c->stage < kSeeds) return fail(c, MKF_E_ORDER, "seed first");
  if (!(c->cfg.flags & MKF_F_BATCHED)) return fail(c, MKF_E_ARG, "autotune needs MKF_F_BATCHED");
  if (repeats < 1) return fail(c, MKF_E_ARG, "repeats must be >= 1");
  // workload key: architecture, compute units, kernel form, candidate
  // budget, sizes
  int lg = 0;
  while (((int64_t)1 << (lg + 1)) <= c->n_seeds) ++lg;
  const bool ext = c->mat.tab || c->field.on, sur = (c->cfg.flags & MKF_F_SURROGATE) != 0;
  const char *form = ext ? (sur ? "extended-surrogate" : "extended")
                         : (sur ? "surrogate" : "plain");
  char key[256];
  snprintf(key, sizeof key, "%s cu%d %s cand%d seeds2^%d events%d layers%d",
           c->arch.empty() ? "unknown" : c->arch.c_str(), c->n_cu, form, c->cfg.n_cand, lg,
           c->n_events, c->n_layers);
  if (cache_path) {
    if (FILE *f = fopen(cache_path, "r")) {
      char line[512];
      mkf_tuning hit{0, 0, 0, 0, 0};
      bool found = false;
      while (fgets(line, sizeof line, f)) {
        const size_t kl = strlen(key);
        mkf_tuning t{};
        if (strncmp(line, key, kl) == 0 && line[kl] == '\t' &&
            sscanf(line + kl + 1, "%d %d %d %d %d", &t.waves_per_simd, &t.blocks_per_cu,
                   &t.lane_group, &t.phi_bin_shift, &t.q_bin_shift) == 5 &&
            tuning_ok(c, t)) {
          hit = t;
          found = true;
        }
      }
      fclose(f);
      if (found) {
        mkf_status st = apply_tuning(c, hit);
        if (st == MKF_OK && best) *best = hit;
        return st;
      }
    }
  }
  const uint32_t flags = c->cfg.flags;
  c->cfg.flags &= ~MKF_F_GRAPH;  // time eager launches
  const mkf_tuning keep = c->tuning;
  mkf_tuning win = c->tuning;
  float win_ms = 1e30f;
  mkf_status st = MKF_OK;
  auto time_shape = [&](const mkf_tuning &t) -> mkf_status {
    mkf_status s2 = apply_tuning(c, t);
    if (s2 != MKF_OK) return s2;
    float ms = 1e30f;
    for (int r = 0; r < repeats; ++r) {
      s2 = mkf_find(c);
      if (s2 != MKF_OK) return s2;
      ms = std::min(ms, c->stats.main_ms);
    }
    if (ms < win_ms) {
      win_ms = ms;
      win = c->tuning;
    }
    return MKF_OK;
  };
  // launch shape at the current binning
  const int groups[2] = {6, 8};
  for (int gi = c->cfg.n_cand <= 6 ? 0 : 1; gi < 2 && st == MKF_OK; ++gi)
    for (int w = 1; w <= 4 && st == MKF_OK; ++w)
      for (int mult = 1; mult <= 2 && st == MKF_OK; ++mult)
        st = time_shape(mkf_tuning{w, w * mult, groups[gi], keep.phi_bin_shift, keep.q_bin_shift});
  // binning at that shape: phi and q bin counts x 2^s, s in -1..2 each
  const mkf_tuning shape = win;
  for (int sp = -1; sp <= 2 && st == MKF_OK; ++sp)
    for (int sq = -1; sq <= 2 && st == MKF_OK; ++sq) {
      if (sp == shape.phi_bin_shift && sq == shape.q_bin_shift) continue;
      mkf_tuning t = shape;
      t.phi_bin_shift = sp;
      t.q_bin_shift = sq;
      st = time_shape(t);
    }
  c->cfg.flags = flags;
  if (st != MKF_OK) {
    std::string e = c->err;
    (void)apply_tuning(c, keep);
    c->err = e;
    return st;
  }
  st = apply_tuning(c, win);
  if (st != MKF_OK) return st;
  if (best) *best = win;
  if (cache_path) {
    if (FILE *f = fopen(cache_path, "a")) {
      fprintf(f, "%s\t%d %d %d %d %d %.4f\n", key, win.waves_per_simd, win.blocks_per_cu,
              win.lane_group, win.phi_bin_shift, win.q_bin_shift, win_ms);
      fclose(f);
    }
  }
  return MKF_OK;
}

}  // extern "C"

// ---- learned propagation surrogate

namespace {

// ascending distinct barrel radii of the loaded geometry
std::vector<float> barrel_radii(const mkf_ctx *c) {
  std::vector<float> r;
  for (int i = 0; i < c->n_layers; ++i)
    if (c->layers[i].kind == MKF_BARREL) r.push_back(c->layers[i].pos);
  std::sort(r.begin(), r.end());
  r.erase(std::unique(r.begin(), r.end()), r.end());
  return r;
}

mkf_status gen_samples(mkf_ctx *c, int64_t n, uint64_t seed, float *x, float *t, float *valid) {
  const std::vector<float> radii = barrel_radii(c);
  if (radii.size() < 2) return fail(c, MKF_E_GEOMETRY, "the sampler needs >= 2 barrel layers");
  HIP_TRY(c, c->d_radii.ensure(sizeof(float) * radii.size()));
  HIP_TRY(c, hipMemcpyAsync(c->d_radii.ptr, radii.data(), sizeof(float) * radii.size(),
                            hipMemcpyHostToDevice, c->stream));
  launch_mlp_datagen(c->stream, params(c), n, seed, c->d_radii.as<float>(), (int)radii.size(),
                     x, t, valid);
  HIP_TRY(c, hipGetLastError());
  return MKF_OK;
}

constexpr int64_t kMaxBatch = 1 << 20;

}  // namespace

extern "C" {

mkf_status mkf_surrogate_samples(mkf_ctx *c, int64_t n, uint64_t seed, float *x, float *t,
                                 float *valid) {
  if (!c) return MKF_E_ARG;
  if (c->stage < kGeometry) return fail(c, MKF_E_ORDER, "load_geometry first");
  if (n < 0 || (n > 0 && (!x || !t || !valid))) return fail(c, MKF_E_ARG, "bad sample buffers");
  if (n == 0) return MKF_OK;
  mkf_status st = gen_samples(c, n, seed, x, t, valid);
  if (st != MKF_OK) return st;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return MKF_OK;
}

mkf_status mkf_surrogate_train(mkf_ctx *c, const mkf_train_cfg *cfg, mkf_train_report *rep) {
  if (!c) return MKF_E_ARG;
  if (c->stage < kGeometry) return fail(c, MKF_E_ORDER, "load_geometry first");
  if (!cfg) return fail(c, MKF_E_ARG, "null training settings");
  if (cfg->batch < 64 || cfg->batch % 64 != 0 || cfg->batch > kMaxBatch)
    return fail(c, MKF_E_ARG, "batch must be a multiple of 64 in 64..%lld",
                (long long)kMaxBatch);
  if (cfg->n_samples < cfg->batch) return fail(c, MKF_E_ARG, "n_samples must be >= batch");
  if (cfg->epochs < 1) return fail(c, MKF_E_ARG, "epochs must be >= 1");
  if (!(cfg->lr > 0.f) || !finite_f(cfg->lr)) return fail(c, MKF_E_ARG, "lr must be > 0");
  for (int j = 0; j < kNO; ++j)
    if (!(cfg->loss_w[j] >= 0.f) || !finite_f(cfg->loss_w[j]))
      return fail(c, MKF_E_ARG, "loss weights must be finite and >= 0");
  const int64_t n = cfg->n_samples;
  const int64_t per_epoch = n / cfg->batch;
  const int64_t steps64 = per_epoch * cfg->epochs;
  if (steps64 > (1 << 24)) return fail(c, MKF_E_ARG, "too many training steps");
  const int steps = (int)steps64;
  if (cfg->first_step < 0 || cfg->first_step >= steps)
    return fail(c, MKF_E_ARG, "first_step %d outside the schedule's %d steps", cfg->first_step,
                steps);
  if (cfg->n_steps < 0 || cfg->n_steps > steps - cfg->first_step)
    return fail(c, MKF_E_ARG, "n_steps %d beyond the schedule's end", cfg->n_steps);
  if (cfg->first_step > 0 && c->mlp_step != cfg->first_step)
    return fail(c, MKF_E_ORDER, "the optimizer state is at step %d, not %d", c->mlp_step,
                cfg->first_step);
  const int s0 = cfg->first_step;
  const int s1 = cfg->n_steps ? s0 + cfg->n_steps : steps;
  const int run = s1 - s0;
  const int waves = cfg->batch / 64;
  HIP_TRY(c, c->d_tx.ensure(sizeof(float) * 8 * n));
  HIP_TRY(c, c->d_tt.ensure(sizeof(float) * 7 * n));
  HIP_TRY(c, c->d_tvalid.ensure(sizeof(float) * n));
  HIP_TRY(c, c->d_partial.ensure(sizeof(float) * (size_t)waves * (kNParam + 1)));
  HIP_TRY(c, c->d_partial2.ensure(sizeof(float) * (size_t)(waves / kReduceGroup + 1) *
                                  (kNParam + 1)));
  HIP_TRY(c, c->d_loss.ensure(sizeof(float) * run));
  HIP_TRY(c, hipEventRecord(c->ev_a, c->stream));
  mkf_status st = gen_samples(c, n, cfg->seed, c->d_tx.as<float>(), c->d_tt.as<float>(),
                              c->d_tvalid.as<float>());
  if (st != MKF_OK) return st;
  HIP_TRY(c, hipEventRecord(c->ev_b, c->stream));
  if (s0 == 0) {  // a run from its start has fresh moments
    HIP_TRY(c, hipMemsetAsync(c->d_mlp_m.ptr, 0, sizeof(float) * kNParam, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->d_mlp_v.ptr, 0, sizeof(float) * kNParam, c->stream));
  }
  HIP_TRY(c, hipEventRecord(c->ev_m0, c->stream));
  const MlpBuffers B = mlp_buffers(c);
  const float lr_min = cfg->lr * 0.01f;
  for (int s = s0; s < s1; ++s) {
    const double u = steps > 1 ? (double)s / (steps - 1) : 0.0;
    const float lr = lr_min + 0.5f * (cfg->lr - lr_min) * (float)(1.0 + std::cos(M_PI * u));
    const int64_t begin = (s % per_epoch) * cfg->batch;
    launch_mlp_grad(c->stream, B.weights(), c->d_tx.as<float>(), c->d_tt.as<float>(),
                    c->d_tvalid.as<float>(), n, begin, cfg->batch, cfg->loss_w,
                    c->d_partial.as<float>());
    launch_mlp_reduce(c->stream, B, c->d_partial.as<float>(), waves, s + 1, lr, 1, nullptr,
                      c->d_loss.as<float>() + (s - s0), c->d_partial2.as<float>());
  }
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipEventRecord(c->ev_m1, c->stream));
  std::vector<float> loss(run), valid(n);
  HIP_TRY(c, hipMemcpyAsync(loss.data(), c->d_loss.ptr, sizeof(float) * run,
                            hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(valid.data(), c->d_tvalid.ptr, sizeof(float) * n,
                            hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->mlp_step = s1;
  if (rep) {
    float gen_ms = 0.f, train_ms = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&gen_ms, c->ev_a, c->ev_b));
    HIP_TRY(c, hipEventElapsedTime(&train_ms, c->ev_m0, c->ev_m1));
    const int k = std::max(1, run / 100);
    double first = 0.0, last = 0.0;
    for (int i = 0; i < k; ++i) {
      first += loss[i];
      last += loss[run - k + i];
    }
    int64_t nv = 0;
    for (float v : valid) nv += v != 0.f;
    rep->steps = run;
    rep->loss_first = (float)(first / k);
    rep->loss_last = (float)(last / k);
    rep->datagen_ms = gen_ms;
    rep->train_ms = train_ms;
    rep->n_valid = nv;
  }
  return MKF_OK;
}

mkf_status mkf_surrogate_get(mkf_ctx *c, float *params) {
  if (!c) return MKF_E_ARG;
  if (!params) return fail(c, MKF_E_ARG, "null parameter buffer");
  HIP_TRY(c, hipMemcpyAsync(params, c->d_mlp_param.ptr, sizeof(float) * kNParam,
                            hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return MKF_OK;
}

mkf_status mkf_surrogate_set(mkf_ctx *c, const float *params) {
  if (!c) return MKF_E_ARG;
  if (!params) return fail(c, MKF_E_ARG, "null parameter buffer");
  for (int i = 0; i < kNParam; ++i)
    if (!finite_f(params[i])) return fail(c, MKF_E_ARG, "parameter %d is not finite", i);
  HIP_TRY(c, hipMemcpyAsync(c->d_mlp_param.ptr, params, sizeof(float) * kNParam,
                            hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->d_mlp_m.ptr, 0, sizeof(float) * kNParam, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->d_mlp_v.ptr, 0, sizeof(float) * kNParam, c->stream));
  launch_mlp_images(c->stream, mlp_buffers(c));
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->mlp_step = 0;
  return MKF_OK;
}

mkf_status mkf_surrogate_get_state(mkf_ctx *c, float *params, float *m, float *v,
                                   int32_t *step) {
  if (!c) return MKF_E_ARG;
  if (!params || !m || !v || !step) return fail(c, MKF_E_ARG, "null state buffer");
  HIP_TRY(c, hipMemcpyAsync(params, c->d_mlp_param.ptr, sizeof(float) * kNParam,
                            hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(m, c->d_mlp_m.ptr, sizeof(float) * kNParam, hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipMemcpyAsync(v, c->d_mlp_v.ptr, sizeof(float) * kNParam, hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  *step = c->mlp_step;
  return MKF_OK;
}

mkf_status mkf_surrogate_set_state(mkf_ctx *c, const float *params, const float *m,
                                   const float *v, int32_t step) {
  if (!c) return MKF_E_ARG;
  if (!params || !m || !v) return fail(c, MKF_E_ARG, "null state buffer");
  if (step < 0) return fail(c, MKF_E_ARG, "step must be >= 0");
  for (int i = 0; i < kNParam; ++i) {
    if (!finite_f(params[i]) || !finite_f(m[i]) || !finite_f(v[i]))
      return fail(c, MKF_E_ARG, "state entry %d is not finite", i);
    if (v[i] < 0.f) return fail(c, MKF_E_ARG, "second moment %d is negative", i);
  }
  HIP_TRY(c, hipMemcpyAsync(c->d_mlp_param.ptr, params, sizeof(float) * kNParam,
                            hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->d_mlp_m.ptr, m, sizeof(float) * kNParam, hipMemcpyHostToDevice,
                            c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->d_mlp_v.ptr, v, sizeof(float) * kNParam, hipMemcpyHostToDevice,
                            c->stream));
  launch_mlp_images(c->stream, mlp_buffers(c));
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->mlp_step = step;
  return MKF_OK;
}

// Blob layout: the 4 bytes "MKFS", then uint32 version, uint32 parameter
// count, int32 Adam step, then the parameters, the first and the second
// moments (FP32, little-endian as in memory).
namespace {
constexpr uint32_t kBlobVersion = 1;
constexpr size_t kBlobHeader = 16;
constexpr size_t kBlobBytes = kBlobHeader + 3 * sizeof(float) * kNParam;
}  // namespace

mkf_status mkf_surrogate_save(mkf_ctx *c, void *buf, size_t cap, size_t *n) {
  if (!c) return MKF_E_ARG;
  if (!n) return fail(c, MKF_E_ARG, "n is NULL");
  *n = kBlobBytes;
  if (!buf || cap < kBlobBytes)
    return fail(c, MKF_E_CAPACITY, "the blob takes %zu bytes", kBlobBytes);
  std::vector<float> st(3 * (size_t)kNParam);
  int32_t step = 0;
  const mkf_status r = mkf_surrogate_get_state(c, st.data(), st.data() + kNParam,
                                               st.data() + 2 * kNParam, &step);
  if (r != MKF_OK) return r;
  unsigned char *b = static_cast<unsigned char *>(buf);
  const uint32_t ver = kBlobVersion, np = kNParam;
  memcpy(b, "MKFS", 4);
  memcpy(b + 4, &ver, 4);
  memcpy(b + 8, &np, 4);
  memcpy(b + 12, &step, 4);
  memcpy(b + kBlobHeader, st.data(), 3 * sizeof(float) * kNParam);
  return MKF_OK;
}

mkf_status mkf_surrogate_load(mkf_ctx *c, const void *buf, size_t n) {
  if (!c) return MKF_E_ARG;
  if (!buf) return fail(c, MKF_E_ARG, "buf is NULL");
  if (n != kBlobBytes) return fail(c, MKF_E_ARG, "a blob has %zu bytes, not %zu", kBlobBytes, n);
  const unsigned char *b = static_cast<const unsigned char *>(buf);
  uint32_t ver = 0, np = 0;
  int32_t step = 0;
  memcpy(&ver, b + 4, 4);
  memcpy(&np, b + 8, 4);
  memcpy(&step, b + 12, 4);
  if (memcmp(b, "MKFS", 4) != 0 || ver != kBlobVersion || np != (uint32_t)kNParam)
    return fail(c, MKF_E_ARG, "not a surrogate blob of this version and size");
  std::vector<float> st(3 * (size_t)kNParam);
  memcpy(st.data(), b + kBlobHeader, 3 * sizeof(float) * kNParam);
  return mkf_surrogate_set_state(c, st.data(), st.data() + kNParam, st.data() + 2 * kNParam,
                                 step);
}

mkf_status mkf_surrogate_grad(mkf_ctx *c, int32_t n, const float *x, const float *t,
                              const float *loss_w, float *grad, float *loss) {
  if (!c) return MKF_E_ARG;
  if (n < 64 || n % 64 != 0 || n > kMaxBatch)
    return fail(c, MKF_E_ARG, "n must be a multiple of 64 in 64..%lld", (long long)kMaxBatch);
  if (!x || !t || !loss_w || !grad || !loss) return fail(c, MKF_E_ARG, "null argument");
  for (int j = 0; j < kNO; ++j)
    if (!finite_f(loss_w[j])) return fail(c, MKF_E_ARG, "loss weights must be finite");
  const int waves = n / 64;
  HIP_TRY(c, c->d_partial.ensure(sizeof(float) * (size_t)waves * (kNParam + 1)));
  HIP_TRY(c, c->d_partial2.ensure(sizeof(float) * (size_t)(waves / kReduceGroup + 1) *
                                  (kNParam + 1)));
  HIP_TRY(c, c->d_grad.ensure(sizeof(float) * (kNParam + 1)));
  HIP_TRY(c, c->d_tvalid.ensure(sizeof(float) * n));
  launch_fill_i32(c->stream, c->d_tvalid.as<int>(), n, 0x3F800000);  // 1.0f
  launch_mlp_grad(c->stream, mlp_buffers(c).weights(), x, t, c->d_tvalid.as<float>(), n, 0, n,
                  loss_w, c->d_partial.as<float>());
  launch_mlp_reduce(c->stream, mlp_buffers(c), c->d_partial.as<float>(), waves, 1, 0.f, 0,
                    c->d_grad.as<float>(), c->d_grad.as<float>() + kNParam,
                    c->d_partial2.as<float>());
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipMemcpyAsync(grad, c->d_grad.ptr, sizeof(float) * kNParam, hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipMemcpyAsync(loss, c->d_grad.as<float>() + kNParam, sizeof(float),
                            hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return MKF_OK;
}

mkf_status mkf_surrogate_grad_noalloc(mkf_ctx *c, int32_t n, const float *x, const float *t,
                                      const float *loss_w, float *grad, float *loss) {
  if (!c) return MKF_E_ARG;
  if (n < 64 || n % 64 != 0)
    return fail(c, MKF_E_ARG, "n must be a positive multiple of 64");
  if (n > kNoAllocMaxSamples)
    return fail(c, MKF_E_CAPACITY, "n = %d exceeds the %d samples the fixed scratch holds", n,
                kNoAllocMaxSamples);
  if (!x || !t || !loss_w || !grad || !loss) return fail(c, MKF_E_ARG, "null argument");
  for (int j = 0; j < kNO; ++j)
    if (!finite_f(loss_w[j])) return fail(c, MKF_E_ARG, "loss weights must be finite");
  float *base = scratch_on(c->device);
  if (!base) return fail(c, MKF_E_HIP, "no scratch on device %d", c->device);
  float *partial = base, *partial2 = base + kNoAllocPartial;
  float *weight = partial2 + kNoAllocPartial2;
  const int waves = n / 64;
  launch_fill_i32(c->stream, reinterpret_cast<int *>(weight), n, 0x3F800000);  // 1.0f
  launch_mlp_grad(c->stream, mlp_buffers(c).weights(), x, t, weight, n, 0, n, loss_w, partial);
  launch_mlp_reduce(c->stream, mlp_buffers(c), partial, waves, 1, 0.f, 0, grad, loss, partial2);
  HIP_TRY(c, hipGetLastError());
  return MKF_OK;
}

mkf_status mkf_surrogate_infer(mkf_ctx *c, int64_t n, const float *x, float *y) {
  if (!c) return MKF_E_ARG;
  if (n < 0 || (n > 0 && (!x || !y))) return fail(c, MKF_E_ARG, "bad buffers");
  launch_mlp_infer(c->stream, mlp_buffers(c).weights(), n, x, y);
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return MKF_OK;
}

}  // extern "C"
