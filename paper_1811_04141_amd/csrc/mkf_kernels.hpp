// mkf_kernels.hpp -- kernel parameter blocks and launch wrappers shared by
// the kernels (mkf_kernels.hip) and the host runtime (mkf_capi.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mkf_device.hpp"
#include "mkf_mlp.hpp"
#include "../../include/mkf.h"

namespace mkf {

// Hit as stored in the binned index: one 32-byte record, two 16-byte loads.
// A hit with its covariance in the layer's local (u, v) frame (vu, vv,
// vuv: the caller's variances turned by the layer's stereo angle).
struct alignas(16) HitRec {
  float x, y, z, vu;
  float vv;
  int orig;  // event-local index in the caller's order
  float vuv;
  int pad1;
};

// Steering of one tracking region: seeds with eta_lo <= eta < eta_hi
// follow `layers` (less their seed layers) in this order.
constexpr int kMaxRegions = MKF_MAX_REGIONS;
struct DevRegion {
  double eta_lo, eta_hi;
  int n;
  int8_t layers[kMaxPlan];
};

// Candidate buffers between layer steps (layer-synchronous form), SoA by
// field over n_seeds * slots (slots = the lane group, 6 or 8) so that a
// wavefront reads consecutive floats per field.
constexpr int kCandFields = 29;  // 6 par + 21 cov + chi2 + meta (bit cast)
constexpr int kSeedWords = 28;   // a seed's state in processing order (112 bytes)
// one result record per seed (processing order), kOutWords words: par[6],
// cov[21], chi2, meta (int32 n_hits | n_miss << 8), pad, then hit[kMaxPlan]
// (int32); 256 bytes, so a tile's records are contiguous
constexpr int kOutPar = 0, kOutCov = 6, kOutChi2 = 27, kOutMeta = 28, kOutHit = 32;
constexpr int kOutWords = kOutHit + kMaxPlan;
// workgroups are dealt to the 8 XCDs of an MI355X round-robin by index
constexpr int kQueues = 8;

struct FindParams {
  // geometry and settings
  const DevLayer *layers;
  int n_layers;
  DevCfg cfg;
  // hits
  int n_events;
  const int64_t *ev_off;   // n_events + 1
  const float *hx, *hy, *hz, *hvu, *hvv;  // caller order, all events
  const int *hlayer;
  const HitRec *sorted;    // binned
  const HitRec *byorig;    // the same records in the caller's order
  const int *bin_start;    // n_events * bins_per_event + 1
  int bins_per_event;
  // seeds, by seed id (written by the seed kernel)
  int64_t n_seeds;
  const int *seed_event;
  const float *seed_state;  // [27][n_seeds]
  const int *seed_ok;
  const int *plan_len;
  const int8_t *plan;       // [n_seeds][kMaxPlan]
  const int *order;         // processing position -> seed id
  // the same, gathered once into processing order (read by the find)
  const float *pstate;      // [n_seeds][kSeedWords]: 6 par, 21 cov, event's first hit (int bits)
  const int *pinfo;         // [n_seeds] plan_len | ok << 8
  const int *pevent;        // [n_seeds]
  const int8_t *pplan;      // [n_seeds][kMaxPlan]
  // results, by processing position: one kOutWords record per seed
  float *out;
  // find state
  int slots;                // candidate slots per seed of the layer-synchronous form (6 or 8)
  float *cand;              // [kCandFields][n_seeds * slots]
  unsigned long long *fin_key;  // [n_seeds]
  float *fin_rec;           // [28][n_seeds] state + chi2 of the best retired candidate
  int *fin_meta;            // [n_seeds] n_hits | n_miss << 8
  int *bp;                  // [kMaxPlan][n_seeds][slots] back-pointers
  // persistent form: kQueues tile queues, queue q owning positions
  // [q_off[q], q_off[q+1]) (whole events); the blocks of XCD x start on
  // queue x and move on to the others when it is empty
  int *tile_counter;        // [kQueues]
  const int64_t *q_off;     // [kQueues + 1]
  int max_plan;             // longest layer plan (sizes the persistent form's LDS records)
  unsigned long long *n_steps;
  // learned surrogate (persistent form)
  MlpWeights mlp;
  // find counters [kCounters][kCounterSlots]: surrogate hints kept, hints
  // rejected, near-cut chi2 decisions, Runge-Kutta steps and Newton
  // iterations of field crossings, failed result checks; each counter is
  // spread over
  // kCounterSlots words (by block index) so that the waves' atomic adds do
  // not queue on one address; the host sums the slots
  unsigned long long *counters;
};
constexpr int kCounters = 6;
constexpr int kCounterSlots = 64;
enum {
  kCntSurKept = 0, kCntSurRejected = 1, kCntNearCut = 2, kCntRk = 3, kCntNewton = 4,
  kCntCheckFailed = 5  // result records that fail the checked find's invariants
};

// 32-bit words of one wavefront's LDS records in the persistent form:
// back-pointers [max_plan][seeds][G] and retired candidates [seeds][kFinWords]
// records allocated past the end of the sorted hits: a window scan reads
// four records from one base address without clamping them to the bin
constexpr int kHitPad = 3;
constexpr int kFinWords = 29;  // 6 + 21 state, chi2, counts
constexpr __host__ __device__ int persistent_rec_words(int max_plan, int g, int seeds) {
  return (max_plan > 0 ? max_plan : 1) * seeds * g + seeds * kFinWords;
}

// combinatorial triplet seeding: three barrel layers and the cuts
struct DevSeeding {
  int layer[3];
  float pt_min, d0_max, z0_max, dz_max;
};
// counts[i]: triplets whose first hit is the hit at binned position i
// (counting pass; the other positions are left alone); with offsets, writes
// them (event, three event-local hit indices).  max_event_hits bounds the
// hits of one event.
void launch_triplets(hipStream_t s, const FindParams &P, const DevSeeding &sc,
                     int64_t max_event_hits, bool write, int *counts, const int *offsets,
                     int *out_event, int *out_hits);
// duplicate-track removal: per track its sorted hits (hbuf [n_seeds][kDupStride],
// hn), the tracks on every hit (CSR: cnt, off, fill, list), the decision
constexpr int kDupStride = 36;
void launch_dup_prep(hipStream_t s, const FindParams &P, const int *seed_hits, int *hbuf, int *hn,
                     int *cnt);
void launch_dup_fill(hipStream_t s, const FindParams &P, const int *hbuf, const int *hn,
                     const int *off, int *fill, int *list);
void launch_dup_decide(hipStream_t s, const FindParams &P, const int *seed_hits, const int *hbuf,
                       const int *hn, const int *off, const int *list, float frac, int *out_dup,
                       int *n_dup);
// seed cleaning: tolerances, and the seeds' sorted global hits (hbuf [n_seeds][3])
struct DevCleaning {
  float tol_ipt, tol_eta, tol_phi;
};
void launch_clean_prep(hipStream_t s, const FindParams &P, const int *seed_hits, int *hbuf,
                       int *cnt);
void launch_clean_fill(hipStream_t s, const FindParams &P, const int *hbuf, const int *off,
                       int *fill, int *list);
void launch_clean_decide(hipStream_t s, const FindParams &P, const int *seed_hits,
                         const float *seed_chi2, const int *hbuf, const int *off,
                         const int *list, const DevCleaning &cc, int *out_keep, int *n_keep);
void launch_hit_bins(hipStream_t s, const FindParams &P, int64_t n_hits, const int *layer,
                     int *hit_bin, int *counts);
void launch_scan(hipStream_t s, const int *in, int *out, int64_t n, int *tmp_a, int *tmp_b);
void launch_scatter(hipStream_t s, const FindParams &P, int64_t n_hits, const int *hit_bin,
                    int *fill, HitRec *sorted, HitRec *byorig);
void launch_seed(hipStream_t s, const FindParams &P, const int *seed_hits, float *seed_state,
                 int *seed_ok, int *plan_len, int8_t *plan, double *plan_l, float *seed_chi2,
                 const DevRegion *regions, int n_regions);
void launch_permute_seeds(hipStream_t s, const FindParams &P, float *pstate, int *pinfo,
                          int *pevent, int8_t *pplan);
void launch_find_init(hipStream_t s, const FindParams &P);
void launch_find_step(hipStream_t s, const FindParams &P, int step, int64_t n_active_seeds);
// group: lanes per seed (6 or 8; 8 whenever the candidate budget exceeds 6)
void launch_find_persistent(hipStream_t s, const FindParams &P, int grid_blocks, int waves,
                            bool surrogate, int group);
void launch_finalize(hipStream_t s, const FindParams &P);
// MKF_F_CHECKED: every result record against the find's invariants; the
// failures are added to counter kCntCheckFailed
void launch_check_results(hipStream_t s, const FindParams &P);
void launch_propagate(hipStream_t s, const FindParams &P, int64_t n, const float *par,
                      const float *cov, const int *layer, float *out_par, float *out_cov,
                      float *out_l, int *out_status);
// backward fit: tmp holds 32 words per seed between its FP64 head and FP32 tail
void launch_backfit(hipStream_t s, const FindParams &P, const int *seed_hits, float *tmp,
                    float *out_par, float *out_cov, float *out_chi2, int *out_status);
// smoothing: wk holds 91 words per surface and seed (max_plan + 1 surfaces),
// n_surf one int per seed
void launch_smooth(hipStream_t s, const FindParams &P, const int *seed_hits, float *wk,
                   int *n_surf, float *out_par, float *out_cov, int *out_n);
void launch_fit(hipStream_t s, const DevCfg &cfg, int64_t n, int n_steps, const int8_t *kind,
                const float *pos, const float *x, const float *y, const float *z,
                const float *vu, const float *vv, const int *len, const float *init_par,
                const float *init_cov, float *out_par, float *out_cov, float *out_chi2,
                int *out_status);
// learned propagation surrogate (mkf_mlp.hip)
struct MlpBuffers {
  float *param, *m, *v;                 // FP32 master weights, Adam moments
  __bf16 *W1p, *W2p, *W3p, *W2T, *W3T;  // BF16 operand images (padding zero)
  float *b1, *b2, *b3;                  // biases (b3 padded to 32)
  MlpWeights weights() const { return MlpWeights{W1p, W2p, W3p, W2T, W3T, b1, b2, b3}; }
};
void launch_mlp_datagen(hipStream_t s, const FindParams &P, int64_t n, uint64_t seed,
                        const float *radii, int n_radii, float *x, float *t, float *valid);
void launch_mlp_grad(hipStream_t s, const MlpWeights &w, const float *x, const float *t,
                     const float *valid, int64_t n, int64_t begin, int batch, const float *loss_w,
                     float *partial);
// Sums n_waves partial rows (through scratch, ceil(n_waves / kReduceGroup)
// rows, when n_waves > kReduceGroup), then writes the gradient or takes an
// Adam step.
constexpr int kReduceGroup = 64;
void launch_mlp_reduce(hipStream_t s, const MlpBuffers &B, const float *partial, int n_waves,
                       int step, float lr, int adam, float *grad_out, float *loss_out,
                       float *scratch);
void launch_mlp_images(hipStream_t s, const MlpBuffers &B);
void launch_mlp_infer(hipStream_t s, const MlpWeights &w, int64_t n, const float *x, float *y);

void launch_validate_hits(hipStream_t s, int64_t n, const float *x, const float *y,
                          const float *z, const float *vu, const float *vv, const int *layer,
                          int n_layers, int *bad);
void launch_fill_u64(hipStream_t s, unsigned long long *p, int64_t n, unsigned long long v);
void launch_fill_i32(hipStream_t s, int *p, int64_t n, int v);

}  // namespace mkf
