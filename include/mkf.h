/*
 * mkf.h -- C ABI of the MI355X (gfx950) Kalman-filter track finding and
 * fitting library.
 *
 * The method is the one of "Parallelized and Vectorized Tracking Using
 * Kalman Filters with CMS Detector Geometry and Events" (arXiv:1811.04141):
 * for every track candidate and every layer of its layer plan, propagate
 * the helix state and its covariance to the layer (barrel cylinder by
 * radius, endcap disk by z), look up nearby hits in a binned layer index,
 * score every candidate-hit pair by chi2, keep the best extensions per seed,
 * and only then apply the Kalman update (the "clone engine", Introduction).
 *
 * Conventions
 *  - Units: cm, GeV/c, tesla, radians.  State p = (x, y, z, q/pT, phi,
 *    theta); covariance: 21 floats, upper triangle of the 6x6 matrix,
 *    row-major: (0,0) (0,1) .. (0,5) (1,1) .. (1,5) (2,2) .. (5,5).
 *  - Every call returns an mkf_status; no call aborts or throws.  On error
 *    mkf_last_error() describes it.
 *  - Memory: arguments marked "host" are read or written by the CPU before
 *    the call returns; arguments marked "device" are HIP device pointers
 *    read or written on the context's stream (the call returns after the
 *    work is queued unless stated otherwise).  Inputs are copied into the
 *    context: the caller may free or reuse them when the call returns.
 *  - All device work of a context is ordered on the stream given at
 *    creation.  One context per host thread; contexts do not share state.
 *  - Call order: create -> load_geometry -> load_hits -> seed -> find ->
 *    get_tracks.  Out-of-order calls return MKF_E_ORDER.
 */
#ifndef MKF_H
#define MKF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MKF_OK = 0,
  MKF_E_ARG = -1,      /* a NULL, negative, non-finite or out-of-range input */
  MKF_E_ORDER = -2,    /* call made before the data it needs was loaded */
  MKF_E_CAPACITY = -3, /* output too small or a size limit exceeded */
  MKF_E_HIP = -4,      /* a HIP runtime call failed */
  MKF_E_GEOMETRY = -5, /* invalid layer description */
  MKF_E_NUMERIC = -6
} mkf_status;

enum { MKF_BARREL = 0, MKF_DISK = 1 };
enum { MKF_MEM_HOST = 0, MKF_MEM_DEVICE = 1 };

#define MKF_MAX_LAYERS 32
#define MKF_MAX_PLAN 32
#define MKF_MAX_CAND 8

/* Find forms (mkf_config.flags). */
#define MKF_F_BATCHED 1u  /* one persistent launch over all seeds and layers */
#define MKF_F_GRAPH 2u    /* replay the find as a captured HIP graph */
#define MKF_F_SURROGATE 4u /* with MKF_F_BATCHED: barrel propagations start from the
                              learned surrogate's path length (see mkf_surrogate_*) */
#define MKF_F_CHECKED 8u  /* after each find (outside its timed region), every result
                             record is checked on the device: hits of the seed's event
                             on the plan's layers, misses, skips, then none once the
                             candidate stopped; hit and miss counts that match the
                             list; finite parameters and chi2, positive variances
                             (the position's, pinned along the last surface's normal,
                             down to -1e-5 of their sum).
                             Failures are counted in mkf_stats.n_check_failed and make
                             mkf_find return MKF_E_NUMERIC (the records stay readable). */

/* History codes in mkf_track.hit. */
#define MKF_HIT_MISS (-1) /* layer crossed, no hit taken */
#define MKF_HIT_SKIP (-2) /* layer not crossed by the candidate */
#define MKF_HIT_NONE (-3) /* candidate had already stopped */

/* One layer of the detector description (the paper's per-layer record of
 * dimensions, type and hit-search parameters, Section 2.1). */
typedef struct {
  int32_t kind;      /* MKF_BARREL (cylinder r = pos) or MKF_DISK (plane z = pos) */
  float pos;         /* radius (barrel) or signed z (disk), cm */
  float ext_lo;      /* barrel: lowest z; disk: inner radius, cm */
  float ext_hi;      /* barrel: highest z; disk: outer radius, cm */
  float var_u_max;   /* bound on the layer's hit variances along u, v (cm^2); */
  float var_v_max;   /*   search windows are sized with them               */
  int32_t n_phi_bins; /* hit index bins in phi (1..4096) */
  int32_t n_q_bins;   /* hit index bins in z (barrel) or r (disk) (1..1024) */
  float stereo;       /* stereo layer: the strips' measuring direction is
                         turned by this angle (|stereo| < pi/2) from u towards
                         v; a hit's var_u lies along it, var_v across it, and
                         var_u_max, var_v_max bound the turned covariance's
                         u-u and v-v terms.  0: var_u, var_v along u, v */
  float hole_lo;      /* no sensors for hole_lo < q < hole_hi (q: z on a  */
  float hole_hi;      /*   barrel, r on a disk); a crossing there is outside
                           the layer (a skip).  hole_lo >= hole_hi: none */
} mkf_layer;

/* Method settings.  The paper states none of these values; the defaults
 * used by the workloads are in the design notes. */
typedef struct {
  float bz;          /* uniform field along +z, T (constant field, Section 2.1) */
  float kappa;       /* curvature constant: rho = pT / (kappa |q| B) */
  float chi2_cut;    /* a hit extends a candidate if chi2 < chi2_cut (2 dof) */
  float ms_sigma;    /* multiple-scattering angle per crossed layer, rad */
  float edge_margin; /* widening of layer extents for plan and crossing tests */
  float l_min;       /* smallest admissible transverse path, cm */
  int32_t n_cand;    /* candidates kept per seed, 1..MKF_MAX_CAND */
  int32_t max_holes; /* misses allowed per candidate */
  float init_var[6]; /* diagonal prior of the seed fit */
  uint32_t flags;    /* MKF_F_* */
} mkf_config;

/* One found track: the best candidate of a seed. */
typedef struct {
  int32_t seed_id;  /* index of the seed in the mkf_seed call */
  int32_t status;   /* 1 found, 0 seed fit failed */
  int32_t n_hits;   /* including the 3 seed hits */
  int32_t n_miss;
  int32_t plan_len;
  float chi2;       /* sum over the hits added by the find */
  float par[6];
  float cov[21];
  int8_t plan[MKF_MAX_PLAN]; /* layer ids of the layer plan */
  int32_t hit[MKF_MAX_PLAN]; /* event-local hit index per plan layer, or MKF_HIT_* */
} mkf_track;

typedef struct {
  int64_t n_seeds;
  int64_t n_seeds_ok;      /* seeds whose triplet fit succeeded */
  int64_t n_steps;         /* candidate-layer steps of the last find */
  int32_t max_plan_len;
  int32_t n_launches;      /* kernel launches of the last find */
  float find_ms;           /* device time of the last find (HIP events) */
  float index_ms;          /* device time of the last hit-index build */
  float seed_ms;           /* device time of the last seeding */
  float main_ms;           /* device time of the last find's layer-step kernels
                              (all step launches, or the one persistent launch) */
  int32_t main_launches;   /* number of those launches */
  int64_t sur_kept;        /* surrogate path lengths kept after their Newton step */
  int64_t sur_rejected;    /* ... rejected (the closed-form crossing was used) */
  /* Decisions of the last find that rounding may take either way: window
   * hits whose chi2 lies within 1e-3 chi2_cut + 0.01 of the cut (the
   * band in which the FP32 result may differ from an exact evaluation). */
  int64_t n_near_cut;
  /* Work of the field crossings of the last find (parameterised field
   * only, else 0): Runge-Kutta steps (the Newton iterations' included) and
   * Newton iterations. */
  int64_t n_rk_steps;
  int64_t n_newton;
  int64_t n_check_failed;  /* MKF_F_CHECKED: records failing the checks (else 0) */
} mkf_stats;

/* Cuts of the combinatorial triplet seeding (mkf_make_seeds). */
typedef struct {
  int32_t layers[3]; /* three barrel layers, increasing radius */
  float pt_min;      /* GeV/c */
  float d0_max;      /* cm: the circle's transverse distance to the beam line */
  float z0_max;      /* cm: |z| at the point of closest approach to the beam line */
  float dz_max;      /* cm: middle hit off the s-z line through the outer two */
} mkf_seeding;

/* Steering of one tracking region (Section 2.1: each region has a list of
 * the layers the find traverses, five eta regions sufficing for CMS).  A
 * seed whose pseudorapidity eta = -ln tan(theta / 2), of the seed fit,
 * lies in [eta_lo, eta_hi) follows the first such region's list in the
 * given order, less its own three layers; a listed layer its candidates do
 * not reach inside the extent is a skip.  A seed in no region gets an
 * empty plan. */
#define MKF_MAX_REGIONS 8
typedef struct {
  float eta_lo, eta_hi;
  int32_t n_layers;              /* 0..MKF_MAX_PLAN */
  int32_t layers[MKF_MAX_PLAN];  /* layer ids, distinct, in visiting order */
} mkf_region;

/* Material map (Section 2.1: multiple scattering and energy loss from
 * two-dimensional arrays of radiation and interaction lengths indexed in
 * r-z).  Bin (iz, ir) covers r in [ir, ir + 1) r_max / n_r and z in
 * -z_max + [iz, iz + 1) 2 z_max / n_z (a crossing outside takes the nearest
 * edge bin) and gives the thickness of the layer crossed there at normal
 * incidence: x_x0 in radiation lengths, xi in g/cm^2.  At each crossing the
 * path factor 1/|cos| of the incidence (at most k_max) scales both; the
 * Highland angle of the path's radiation lengths at the momentum before the
 * loss replaces ms_sigma, and the mean ionisation loss in silicon (Bethe,
 * no density correction) at the path's mass thickness lowers |p| by
 * dE/beta (at most half of |p|; the backward fit regains it). */
typedef struct {
  int32_t n_r, n_z;  /* bins, 1..4096 each, at most 2^22 in all */
  float r_max;       /* cm, > 0 */
  float z_max;       /* cm, > 0 */
  float mass;        /* particle mass hypothesis, GeV, > 0 */
  float k_max;       /* cap on the path factor, >= 1 */
} mkf_material_info;

/* Parameterised field (Section 2.1: a constant or a parameterised field,
 * selectable per propagation): Bz(r, z) = b0 (1 + c_r2 r^2 + c_z2 z^2 +
 * c_z4 z^4) tesla (r, z in cm); the radial component is neglected, so pT and
 * theta are constants of the motion and the azimuth turns at the local
 * curvature.  Crossings come from fourth-order Runge-Kutta steps of at most
 * h_max cm of transverse path (a disk's path is exact; a barrel's last step
 * is cut by Newton iterations), within half a turn and 1000 cm; the
 * transport Jacobian is the helix's with the path's mean curvature. */
typedef struct {
  float b0;          /* T, != 0 */
  float c_r2;        /* cm^-2 */
  float c_z2;        /* cm^-2 */
  float c_z4;        /* cm^-4 */
  float h_max;       /* cm, 0.01..100 */
} mkf_field;

/* Tolerances of the seed cleaning (mkf_clean_seeds). */
typedef struct {
  float tol_ipt; /* q/pT, relative to the larger of the two */
  float tol_eta;
  float tol_phi; /* rad */
} mkf_cleaning;

typedef struct mkf_ctx mkf_ctx;

/* Create a context holding the method's settings (the find's parameters,
 * which the paper keeps in its steering and configuration, Section 2.1) and
 * every device buffer of the work it runs.  cfg is copied.  stream: a
 * hipStream_t (NULL = the default stream), e.g.
 * torch.cuda.current_stream().cuda_stream.  MKF_E_ARG for bad settings,
 * MKF_E_HIP if the device set-up fails. */
mkf_status mkf_create(const mkf_config *cfg, void *stream, mkf_ctx **out);

/* Release all device memory of ctx.  NULL is accepted. */
void mkf_destroy(mkf_ctx *ctx);

/* Text of the last error on ctx (never NULL; valid until the next call on
 * ctx).  For ctx == NULL: the last error of mkf_create. */
const char *mkf_last_error(const mkf_ctx *ctx);

/* Detector description (Section 2.1): n_layers records, host memory.
 * Replaces any previous geometry and invalidates loaded hits. */
mkf_status mkf_load_geometry(mkf_ctx *ctx, const mkf_layer *layers, int32_t n_layers);

/* Material map: info and the host tables x_x0 [n_z][n_r] (0..1) and
 * xi [n_z][n_r] (0..100 g/cm^2), copied.  info == NULL returns to the
 * constant angle ms_sigma.  Used by every later call that fits: mkf_seed,
 * mkf_find, mkf_fit, mkf_backward_fit, mkf_smooth (seed states already made
 * keep the material they were fitted with).  The surrogate form
 * (MKF_F_SURROGATE) runs with a map too: the network's path only starts the
 * barrel crossing, the material update follows it as without the network.
 * MKF_E_ARG for bad values. */
mkf_status mkf_load_material(mkf_ctx *ctx, const mkf_material_info *info, const float *x_x0,
                             const float *xi);

/* Parameterised field: f copied; NULL returns to the uniform cfg.bz.  Used
 * by every later call that propagates: mkf_seed (the seed momentum takes the
 * field at the middle hit; plans), mkf_find, mkf_fit, mkf_backward_fit,
 * mkf_smooth, mkf_propagate, and the surrogate's sampler (mkf_surrogate_train
 * and mkf_surrogate_samples then produce the field's stepped crossings).  Not
 * by mkf_make_seeds (its cuts take the uniform cfg.bz).  In the field the
 * surrogate form (MKF_F_SURROGATE) starts each barrel crossing from the
 * network's path: equal Runge-Kutta steps to it and one Newton step taken as
 * one more Runge-Kutta step, kept under the same checks as in the uniform
 * field, else the full stepped search.  MKF_E_ARG for bad values. */
mkf_status mkf_load_field(mkf_ctx *ctx, const mkf_field *f);

/* Region steering (Section 2.1): n_regions (0..MKF_MAX_REGIONS) records,
 * host memory, copied.  Layer ids refer to the loaded geometry, so load it
 * first.  Takes effect at the next mkf_seed; n_regions = 0 returns to
 * plans read from each seed's helix (every layer it crosses, by path
 * length).  Loading a geometry clears it.  MKF_E_ARG for a bad record,
 * MKF_E_ORDER without geometry. */
mkf_status mkf_load_steering(mkf_ctx *ctx, const mkf_region *regions, int32_t n_regions);

/* Hits of n_events events (hits and seeds are supplied from outside,
 * Section 2.2).  Event e owns hits [ev_off[e], ev_off[e+1]) of the arrays;
 * ev_off (host, n_events + 1 entries, ev_off[0] = 0).  x, y, z: position,
 * var_u, var_v: variances in the layer's local frame (barrel: r-phi and z;
 * disk: r-phi and r), layer: layer id.  mem says whether the six arrays are
 * host or device memory.  Builds the binned hit index (untimed
 * pre-processing).  Invalidates seeds. */
mkf_status mkf_load_hits(mkf_ctx *ctx, int32_t n_events, const int64_t *ev_off,
                         const float *x, const float *y, const float *z,
                         const float *var_u, const float *var_v,
                         const int32_t *layer, int32_t mem);

/* Seeds: n_seeds triplets; seed_event[i] is the event of seed i and
 * seed_hits[3 i .. 3 i + 2] its event-local hit indices, innermost first.
 * Both arrays host or device per mem.  Fits each triplet and builds its
 * layer plan (untimed pre-processing). */
mkf_status mkf_seed(mkf_ctx *ctx, int64_t n_seeds, const int32_t *seed_event,
                    const int32_t *seed_hits, int32_t mem);

/* Seed states after the triplet fit (host outputs, each may be NULL):
 * par [n_seeds][6], cov [n_seeds][21], ok [n_seeds], plan_len [n_seeds],
 * plan [n_seeds][MKF_MAX_PLAN] (layer ids), chi2 [n_seeds] (sum of the
 * three hit updates' chi2).  Blocks until done. */
mkf_status mkf_get_seed_states(mkf_ctx *ctx, float *par, float *cov, int32_t *ok,
                               int32_t *plan_len, int8_t *plan, float *chi2);

/* Clone-engine track finding over all seeds (the timed hot path). */
mkf_status mkf_find(mkf_ctx *ctx);

/* Copy the found tracks (one per seed, in seed order) to host memory: the
 * step that hands the result back to the caller, as the paper's framework
 * integration copies the found tracks back into the host framework's format
 * (Section 2.2).  Writes the records of seeds 0 .. min(capacity, n_seeds) - 1
 * and nothing beyond; *n_total = n_seeds; returns MKF_E_CAPACITY if
 * capacity < n_seeds, MKF_E_ARG for capacity < 0, MKF_E_ORDER before a find.
 * Blocks until done. */
mkf_status mkf_get_tracks(mkf_ctx *ctx, mkf_track *out, int64_t capacity, int64_t *n_total);

/* Propagate n states to layers of the loaded geometry (unit access to the
 * propagation of the hot path, no scattering, extent widened by
 * edge_margin).  Device pointers: par [n][6], cov [n][21], layer [n];
 * outputs out_par [n][6], out_cov [n][21], out_l [n] (transverse path),
 * out_status [n] (0 ok, 1 no crossing, 2 outside the widened extent, 3 bad
 * layer id). */
mkf_status mkf_propagate(mkf_ctx *ctx, int64_t n, const float *par, const float *cov,
                         const int32_t *layer, float *out_par, float *out_cov,
                         float *out_l, int32_t *out_status);

/* Kalman fit without search (the paper's vectorized fitting,
 * Introduction): n_tracks tracks, each through up to n_steps hits on its
 * own surfaces.  Device pointers, step-major so that consecutive tracks
 * are adjacent: kind/pos/x/y/z/var_u/var_v [n_steps][n_tracks]; len
 * [n_tracks] (hits used, <= n_steps); init_par [n_tracks][6], init_cov
 * [n_tracks][21]; outputs out_par, out_cov, out_chi2 [n_tracks],
 * out_status [n_tracks] (0 ok, k > 0: propagation to hit k-1 failed).
 * Material effects are those of the find: the loaded material map
 * (mkf_load_material), else the constant angle cfg.ms_sigma; propagation
 * takes the loaded parameterised field (mkf_load_field), else cfg.bz.  No
 * extent test. */
mkf_status mkf_fit(mkf_ctx *ctx, int64_t n_tracks, int32_t n_steps, const int8_t *kind,
                   const float *pos, const float *x, const float *y, const float *z,
                   const float *var_u, const float *var_v, const int32_t *len,
                   const float *init_par, const float *init_cov, float *out_par,
                   float *out_cov, float *out_chi2, int32_t *out_status);

/* Backward fit of the tracks of the last mkf_find (the layer plan's
 * steering carries layers used only when fitting backwards, Section 2.1;
 * the filter is the Kalman filter of the Introduction run in the reverse
 * order).  For every seed: the track's crossed plan layers (hit or
 * MKF_HIT_MISS) from the last to the first, then its three seed layers
 * from the third to the first.  The filter starts on the first of these
 * surfaces from the track's final state with the seed prior cfg.init_var
 * less its extent along the surface normal, and on every surface
 * propagates (from the second on, backwards along the helix, no extent
 * test), adds cfg.ms_sigma scattering and updates with the surface's hit
 * if it has one.  Device outputs in seed order: out_par [n_seeds][6] and
 * out_cov [n_seeds][21] (state on the first seed layer), out_chi2
 * [n_seeds] (sum over all the track's hits), out_status [n_seeds] (1 ok;
 * 0 the seed fit failed; -k: the k-th surface was not reached or its hit
 * lies in the other half of the layer; outputs zero unless 1).  The first
 * three hits are filtered in FP64 (they shrink the wide prior), the rest
 * in FP32.  Asynchronous on the context's stream; the caller owns the
 * outputs.  MKF_E_ORDER before a find. */
mkf_status mkf_backward_fit(mkf_ctx *ctx, float *out_par, float *out_cov, float *out_chi2,
                            int32_t *out_status);

/* Rauch-Tung-Striebel smoothing of the tracks of the last mkf_find (the
 * backward pass the layer plan's steering provides for, Section 2.1,
 * applied to the Kalman filter of the Introduction).  Surfaces of a track:
 * the seed's third layer (where the find starts), then every plan layer the
 * track crossed (hit or MKF_HIT_MISS), in plan order.  The forward pass is
 * the find's filter along the track in FP32 (propagate, add cfg.ms_sigma
 * scattering, update with the hit if there is one); the backward pass
 * forms xs(k) = x(k) + A (xs(k+1) - xp(k+1)), Cs(k) = C(k) + A (Cs(k+1) -
 * Cp(k+1)) A^T, A = C(k) F^T Cp(k+1)^-1, in FP32 with the inverse taken in
 * the five free coordinates of surface k+1 (a Cholesky solve).  Device outputs in seed order:
 * out_par [n_seeds][MKF_MAX_PLAN + 1][6], out_cov [n_seeds][MKF_MAX_PLAN +
 * 1][21] (the first out_n entries of a seed are written), out_n [n_seeds]
 * (surfaces; 0 the seed fit failed; -1 a propagation or hit update failed;
 * -2 a predicted covariance was not positive definite on its surface).
 * Device scratch: 364 bytes per surface and seed, held by the context.
 * Asynchronous on the context's stream.  MKF_E_ORDER before a find. */
mkf_status mkf_smooth(mkf_ctx *ctx, float *out_par, float *out_cov, int32_t *out_n);

/* Combinatorial triplet seeds from the loaded hits (the paper takes seeds
 * from outside, Section 2.2; this is the step it leaves to the host
 * framework).  A seed is a triplet of hits a, b, c on sc->layers whose
 * helix is a plausible track from the beam line: with the circle through
 * the three transverse points (radius rho, centre c0), kappa |B| rho >=
 * pt_min; | |c0| - rho | <= d0_max; a, b, c follow each other in the
 * turning sense within half a turn; |z_b - (z_a + (z_c - z_a) s_ab/s_ac)|
 * <= dz_max (s: arc lengths); and the s-z line through a and c has |z| <=
 * z0_max at the point of closest approach to the beam line, which precedes
 * a within half a turn.  The cuts are evaluated in FP64.  Device outputs:
 * out_event [capacity], out_hits [capacity][3] (event-local hit indices,
 * innermost first), ordered by event, then by the hit index's bin order of
 * a, b and c; *n_total receives the number of triplets.
 * If it exceeds capacity nothing is written and MKF_E_CAPACITY returned.
 * The outputs can go to mkf_seed with MKF_MEM_DEVICE.  Blocks until done. */
mkf_status mkf_make_seeds(mkf_ctx *ctx, const mkf_seeding *sc, int64_t capacity,
                          int32_t *out_event, int32_t *out_hits, int64_t *n_total);

/* Duplicate removal for the tracks of the last mkf_find (not yet done in
 * the paper: Introduction; Section 3 traces its duplicates to several seeds
 * per particle).  The hits of a track are its three seed hits and its found
 * hits.  Track u ranks before track t if it has more hits; with as many, a
 * smaller chi2; with the same chi2, a lexicographically smaller seed
 * triplet (event-local hit indices).  t is a duplicate if a track ranking
 * before it shares at least frac (0 < frac <= 1) of the hits of the shorter
 * of the two; a track ranking before t need not be kept itself.  Device
 * output out_dup [n_seeds] (seed order): 1 for a duplicate, 0 otherwise
 * (also for a seed whose fit failed); *n_dup receives their number.
 * Device scratch of ~150 B per seed and 12 B per hit, held by the context.
 * Blocks until done. */
mkf_status mkf_find_duplicates(mkf_ctx *ctx, float frac, int32_t *out_dup, int64_t *n_dup);

/* Seed cleaning of the last mkf_seed's seeds (Section 2.2: several seeds
 * built from hits of the same outgoing particle are reduced to one, using
 * the identity of their hits and their fitted pT, eta and phi).  Seeds of
 * one event sharing a hit are instances of one particle if their fitted
 * states (on the third seed layer) agree: |q/pT_s - q/pT_t| <= tol_ipt
 * max(|q/pT_s|, |q/pT_t|), |eta_s - eta_t| <= tol_eta, |phi_s - phi_t| <=
 * tol_phi.  Seed u ranks before t if its fit chi2 is smaller; with the same
 * chi2, if its hit triplet is lexicographically smaller.  t is kept if its
 * fit succeeded and no seed ranking before it is an instance of the same
 * particle.  Device output out_keep [n_seeds] (seed order, 1 = keep);
 * *n_keep receives their number.  The kept seeds can go back to mkf_seed.
 * Blocks until done. */
mkf_status mkf_clean_seeds(mkf_ctx *ctx, const mkf_cleaning *cc, int32_t *out_keep,
                           int64_t *n_keep);

/* Counters and timings of the last calls. */
mkf_status mkf_get_stats(mkf_ctx *ctx, mkf_stats *out);

/* Launch shape of the persistent find (MKF_F_BATCHED) and binning of the
 * hit index.  Results do not depend on it (tested bit for bit). */
typedef struct {
  int32_t waves_per_simd; /* register budget of the persistent kernel, 1..4
                             (more waves hide more latency, but spill) */
  int32_t blocks_per_cu;  /* persistent grid = blocks_per_cu x compute units, 1..32 */
  int32_t lane_group;     /* lanes per seed: 6 (a wavefront tile of 10 seeds; candidate
                             budgets up to 6) or 8 (8 seeds); 0: 6 when the budget allows */
  int32_t phi_bin_shift;  /* hit-index bins per layer: the layer records' counts times */
  int32_t q_bin_shift;    /*   2^shift (-2..2; clamped to 1..4096 in phi, 1..1024 in q) */
} mkf_tuning;

/* Set the tuning.  A change of the bin shifts rebuilds the hit index of
 * loaded hits (seeds stay valid).  MKF_E_ARG for values out of range. */
mkf_status mkf_set_tuning(mkf_ctx *ctx, const mkf_tuning *t);
mkf_status mkf_get_tuning(mkf_ctx *ctx, mkf_tuning *t);

/* Autotuner of the persistent find on the loaded seeds: first the launch
 * shape (lane group 6 or 8, waves per SIMD 1..4, 1 or 2 x waves blocks per
 * CU), then at that shape the hit-index binning (phi and q bin shifts
 * -1..2, the index rebuilt for each), each timed as the best of `repeats`
 * runs (repeats >= 1); the fastest is kept (written to *best if not NULL).
 * cache_path (may be NULL) names a text file of earlier results keyed by
 * GPU architecture, compute units, kernel form and workload size: a
 * matching line is used without searching, a search appends its result.
 * Blocks until done. */
mkf_status mkf_autotune(mkf_ctx *ctx, int32_t repeats, const char *cache_path,
                        mkf_tuning *best);

/* ---- learned propagation surrogate --------------------------------------
 * A multilayer perceptron 8 -> 64 -> 64 -> 7 (SiLU) with BF16 weights on the
 * matrix cores and FP32 accumulation, predicting the transverse path length
 * to the next barrel layer as a relative correction to the straight-line
 * path, plus a 6-value state correction.  Inputs, per sample, for a state
 * heading to the cylinder R (invariant under rotations about z):
 * (r0/R, cos a, sin a, omega R, R/70, cot(theta)/5, z/100, 0.3 q/pT), with r0
 * the start radius, a the angle from the radial direction to the transverse
 * direction, and omega the signed curvature (-kappa bz q/pT).  Outputs:
 * 10 (l/l_line - 1) / (omega R); then, scaled by 10/l_line, the end point's
 * offsets from the straight line along and across the initial direction and
 * in z; then 10 (cos, sin) of the turning angle minus (10, 0); then 0.  Only
 * the first output is used by the find; the rest are trained and reported.
 * In the find (MKF_F_SURROGATE) the network predicts, per layer step, the
 * path of each seed's leading candidate; every candidate applies that
 * relative correction to its own straight-line path and takes one exact
 * Newton step from there (in the parameterised field: Runge-Kutta steps to
 * the predicted path and the correction as one more step).  The result is
 * kept only if that step moves it by at most 1e-4 relative, the Newton error
 * bound left after it is at most 1e-7 relative and it is the first crossing;
 * otherwise the closed-form crossing (in the field, the full stepped search)
 * is used, so the tracks do not depend on the weights beyond FP32 rounding.
 * Parameters (5,191 FP32,
 * in this order): W1[64][8], b1[64], W2[64][64], b2[64], W3[7][64], b3[7]. */

typedef struct {
  int64_t n_samples; /* training propagations generated on the GPU */
  int32_t epochs;
  int32_t batch;     /* samples per Adam step, a multiple of 64 */
  float lr;          /* Adam step size (cosine-decayed to lr/100) */
  uint64_t seed;     /* seed of the counter-based sampler */
  float loss_w[7];   /* per-output weights of the squared error */
  int32_t first_step; /* first step of the schedule this call takes (see below) */
  int32_t n_steps;    /* steps this call takes; 0: to the end of the schedule */
} mkf_train_cfg;

typedef struct {
  int32_t steps;
  float loss_first;  /* mean loss over the first 1% of steps */
  float loss_last;   /* mean loss over the last 1% of steps */
  float datagen_ms;
  float train_ms;
  int64_t n_valid;   /* generated samples that reached their target layer */
} mkf_train_report;

/* Generate n_samples propagations over the barrel layers of the loaded
 * geometry with the plain propagator (tracks from the beam line, pT
 * 0.3-10 GeV/c log-uniform, |eta| < 2.4, from each barrel layer to the
 * next), then train with the library's forward/backward kernels and Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8).  The schedule has S = (n_samples /
 * batch) x epochs steps: step s (0-based) takes the samples [(s mod
 * (n_samples / batch)) batch, + batch) and the step size lr_min + (lr -
 * lr_min) (1 + cos(pi s / (S - 1))) / 2 with lr_min = lr / 100 (lr for
 * S = 1).  This call takes steps first_step .. first_step + n_steps - 1
 * (to S - 1 if n_steps = 0): with first_step = 0 from fresh moments, with
 * first_step > 0 continuing the context's optimizer state, which must then
 * be at step first_step (after an earlier call, or restored by
 * mkf_surrogate_set_state; MKF_E_ORDER otherwise).  The samples are
 * regenerated from seed, so a schedule taken in pieces gives the weights of
 * one uninterrupted call bit for bit.  Blocks until done.  Errors:
 * MKF_E_ORDER without geometry, MKF_E_GEOMETRY with fewer than 2 barrel
 * layers, MKF_E_ARG for bad settings. */
mkf_status mkf_surrogate_train(mkf_ctx *ctx, const mkf_train_cfg *cfg, mkf_train_report *rep);

/* Read or replace the parameter vector (host, 5,191 floats).  Replacing it
 * resets the optimizer state (zero moments, step 0). */
mkf_status mkf_surrogate_get(mkf_ctx *ctx, float *params);
mkf_status mkf_surrogate_set(mkf_ctx *ctx, const float *params);

/* Checkpoint of the training, all that resuming it needs: the parameters,
 * Adam's first and
 * second moments (host, 5,191 floats each) and the number of Adam steps
 * taken.  get writes them; set restores them (finite values, second
 * moments >= 0, step >= 0; MKF_E_ARG otherwise), after which
 * mkf_surrogate_train with first_step = step continues the run. */
mkf_status mkf_surrogate_get_state(mkf_ctx *ctx, float *params, float *m, float *v,
                                   int32_t *step);
mkf_status mkf_surrogate_set_state(mkf_ctx *ctx, const float *params, const float *m,
                                   const float *v, int32_t step);

/* The same checkpoint as one byte blob, for files: "MKFS", uint32 version
 * (1), uint32 parameter count (5,191), int32 Adam step, then the
 * parameters, first and second moments (FP32), 62,308 bytes in all.  save
 * sets *n to the size and writes the blob if cap is large enough
 * (MKF_E_CAPACITY otherwise, with *n set, so buf = NULL asks for the size);
 * load takes a blob of exactly that size and header (MKF_E_ARG otherwise)
 * and restores it as mkf_surrogate_set_state does. */
mkf_status mkf_surrogate_save(mkf_ctx *ctx, void *buf, size_t cap, size_t *n);
mkf_status mkf_surrogate_load(mkf_ctx *ctx, const void *buf, size_t n);

/* Loss and its gradient for the current weights on n samples (n a positive
 * multiple of 64; x [n][8], t [n][7] device; loss_w host [7]); grad host
 * [5,191], loss host.  Blocks until done. */
mkf_status mkf_surrogate_grad(mkf_ctx *ctx, int32_t n, const float *x, const float *t,
                              const float *loss_w, float *grad, float *loss);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight training loops, harnesses that forbid hipMalloc): the loss
 * and gradient of mkf_surrogate_grad, with device outputs grad [5,191] and
 * loss [1], queued on the context's stream without waiting (x, t device;
 * loss_w host [7], read before the call returns).  n is a positive multiple
 * of 64 up to MKF_NOALLOC_MAX_SAMPLES (MKF_E_CAPACITY above).  It allocates
 * nothing: its scratch is one fixed 5.5 MB array per GPU, held until the
 * process ends and shared by every context on that GPU, so calls that
 * overlap on one GPU (other streams or host threads) race and must be
 * ordered by the caller. */
#define MKF_NOALLOC_MAX_SAMPLES 16384
mkf_status mkf_surrogate_grad_noalloc(mkf_ctx *ctx, int32_t n, const float *x, const float *t,
                                      const float *loss_w, float *grad, float *loss);

/* Outputs y [n][7] (device) for inputs x [n][8] (device).  Calls of up to
 * 16,384 samples run on the find's 16-sample tiles, larger ones on 64-sample
 * tiles; the two may differ in the last bits (accumulation order). */
mkf_status mkf_surrogate_infer(mkf_ctx *ctx, int64_t n, const float *x, float *y);

/* The training sampler: n inputs x [n][8], targets t [n][7] and validity
 * flags valid [n] (device outputs).  Needs a geometry with >= 2 barrel
 * layers. */
mkf_status mkf_surrogate_samples(mkf_ctx *ctx, int64_t n, uint64_t seed, float *x, float *t,
                                 float *valid);

#ifdef __cplusplus
}
#endif
#endif
