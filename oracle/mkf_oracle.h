/*
 * mkf_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU reference of the Kalman-filter track finding and
 * fitting hot path of "Parallelized and Vectorized Tracking Using Kalman
 * Filters with CMS Detector Geometry and Events" (arXiv:1811.04141).
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg use
 * it.  It shares no code, header or constant with the GPU library.
 *
 * The paper prints no equations.  Each function names the passage it
 * follows and the textbook definition used where the paper is silent.
 *
 * Units: cm, GeV/c, tesla, radians.
 * State p = (x, y, z, q/pT, phi, theta): a point on the track, the signed
 * inverse transverse momentum, the momentum azimuth and the polar angle.
 * Covariances are full 6x6 row-major double arrays here (the oracle does
 * not pack triangles).
 */
#ifndef MKF_ORACLE_H
#define MKF_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Curvature constant c * 1e-9: transverse radius rho = pT / (k |q| B). */
#define ORC_KAPPA 0.299792458e-2

#define ORC_MAX_PLAN 32
#define ORC_ETA_TOL 1e-6

/* Outcome of a propagation. */
#define ORC_OK 0
#define ORC_NO_CROSSING 1   /* no root in the first half turn beyond l_min */
#define ORC_OUT_OF_EXTENT 2 /* crossing outside the widened layer extent */

/* History codes in a track's per-plan-layer hit list. */
#define ORC_HIT_MISS (-1)
#define ORC_HIT_SKIP (-2)
#define ORC_HIT_NONE (-3) /* the candidate retired before this layer */

typedef struct {
  int32_t kind;  /* 0 barrel cylinder, 1 endcap disk */
  double pos;    /* radius R (barrel) or signed z position Z (disk) */
  double ext_lo; /* barrel: lowest z; disk: inner radius */
  double ext_hi; /* barrel: highest z; disk: outer radius */
  double stereo; /* strip frame turned by this angle from (u, v); 0: none */
  double hole_lo, hole_hi; /* no sensors for hole_lo < q < hole_hi (q as ext) */
} orc_layer;

/* A tracking region's steering (Section 2.1): seeds whose pseudorapidity
 * (of the seed fit's theta) lies in [eta_lo, eta_hi) follow its layer list,
 * in the order given. */
typedef struct {
  double eta_lo, eta_hi;
  int32_t n_layers;
  int32_t layers[ORC_MAX_PLAN];
} orc_region;

/* Material map (Section 2.1: radiation and interaction lengths in 2-D r-z
 * arrays, indexed at each crossing).  Bin (iz, ir) covers
 * r in [ir, ir + 1) * r_max / n_r and z in -z_max + [iz, iz + 1) * 2 z_max / n_z
 * (crossings outside take the nearest edge bin) and holds the layer's
 * thickness there at normal incidence, in radiation lengths (x_x0) and as
 * mass thickness in g/cm^2 (xi, for the mean ionisation loss). */
typedef struct {
  int32_t n_r, n_z;
  double r_max, z_max;
  double mass;        /* particle mass hypothesis, GeV */
  double k_max;       /* cap on the path factor 1 / |cos(incidence)| */
  const double *x_x0; /* [n_z][n_r] */
  const double *xi;   /* [n_z][n_r] */
} orc_material;

/* Parameterised field (Section 2.1: a constant or a parameterised field):
 * Bz(r, z) = b0 (1 + c_r2 r^2 + c_z2 z^2 + c_z4 z^4), tesla, cm; the radial
 * component is neglected, so pT and theta are constants of the motion and
 * the azimuth turns at the local curvature omega = -kappa Bz (q/pT).  The
 * transport integrates (x, y, z, phi) over the transverse path with
 * fourth-order Runge-Kutta steps of at most h_max. */
typedef struct {
  double b0, c_r2, c_z2, c_z4;
  double h_max;
} orc_field;

typedef struct {
  double bz;          /* field along +z, tesla */
  double kappa;       /* curvature constant (normally ORC_KAPPA) */
  double chi2_cut;    /* accept a hit if chi2 < chi2_cut (2 dof) */
  double ms_sigma;    /* multiple-scattering angle per crossed layer, rad */
  double edge_margin; /* extent widening for plan and crossing tests, cm */
  double l_min;       /* smallest admissible transverse path, cm */
  int32_t n_cand;     /* candidates kept per seed */
  int32_t max_holes;  /* misses allowed per candidate */
  double init_var[6]; /* diagonal seed prior variances */
  /* region steering; n_regions = 0: every seed's plan from its own helix */
  const orc_region *regions;
  int32_t n_regions;
  /* material map; NULL: the constant scattering angle ms_sigma per layer */
  const orc_material *material;
  /* parameterised field; NULL: the uniform field bz */
  const orc_field *field;
} orc_cfg;

/* ---- single-state primitives (exposed for the tests) ---------------- */

/* Exact helix transport by transverse path length l. */
void orc_transport(const double p[6], double l, double bz, double kappa,
                   double out[6]);

/* Path length to a surface: smallest l > l_min inside the first half
 * turn.  Returns ORC_OK or ORC_NO_CROSSING. */
int orc_path_to_barrel(const double p[6], double R, double bz, double kappa,
                       double l_min, double *l);
int orc_path_to_disk(const double p[6], double Z, double bz, double kappa,
                     double l_min, double *l);

/* Full propagation to a layer: state, surface-constrained Jacobian F
 * (6x6, may be NULL), transported covariance F C F^T (may be NULL when C is
 * NULL).  check_extent = 0 skips the extent test (used by the fit).
 * Multiple scattering is NOT added here. */
int orc_propagate(const double p[6], const double C[36], const orc_layer *L,
                  double bz, double kappa, double l_min, double edge_margin,
                  int check_extent, double p_out[6], double C_out[36],
                  double F_out[36], double *l_out);

/* The same in the parameterised field fld (NULL: the uniform bz).  The
 * crossing is found by Runge-Kutta steps: on a disk, equal steps to the
 * exact path (Z - z) tan(theta); on a barrel, steps of h_max until r^2 - R^2
 * changes sign, then Newton iterations on the last step's length until the
 * correction falls below 1e-12 cm.  The turning must stay below half a turn
 * and the path below 1000 cm, whatever the step size.  The Jacobian is that
 * of the helix with the path's mean curvature (the turning over the path
 * length), made surface-constrained at the end point. */
int orc_propagate_f(const double p[6], const double C[36], const orc_layer *Lr,
                    double bz, double kappa, double l_min, double edge_margin,
                    int check_extent, double p_out[6], double C_out[36],
                    double F_out[36], double *l_out, const orc_field *fld);

/* Bz of the parameterised field at (x, y, z). */
double orc_field_bz(const orc_field *fld, double x, double y, double z);

/* Multiple-scattering noise for state p with angle sigma, added to C. */
void orc_add_ms(const double p[6], double sigma, double C[36]);

/* Mean ionisation loss in silicon (Bethe, no density or shell correction),
 * GeV cm^2 / g, for a particle of the given mass at beta*gamma = bg. */
double orc_bethe_si(double bg, double mass);

/* Effects of the material of one crossed layer of the given kind on the
 * state p, C at the crossing.  Without a material map: scattering with
 * cfg->ms_sigma.  With one: the Highland scattering angle of the path's
 * radiation lengths at the momentum before the loss, then the mean
 * ionisation loss of the path's mass thickness, |p| -> |p| - dir * dp
 * (dir = +1 moving forward, -1 for the backward fit, which regains it),
 * dp = dE / beta, at most half of |p|.  M (may be NULL) receives the
 * Jacobian of the state change (identity but the q/pT row, with dp held
 * fixed); C becomes M (C + Q) M^T. */
void orc_material_effects(const orc_cfg *cfg, int kind, double p[6], double C[36], int dir,
                          double M[36]);

/* Local measurement of a hit at the predicted state: residual r[2],
 * projection H (2x6) and hit variances.  Returns 0 if the hit lies in the
 * wrong hemisphere (barrel only), 1 otherwise. */
int orc_measure(const double p[6], int kind, const double hit[3],
                double r[2], double H[12]);

/* chi2 = r^T (H C H^T + V)^-1 r, V the hit covariance: var_u along the
 * layer's strip direction, turned by stereo from u, var_v across it.
 * Returns 0 if incompatible (hemisphere). */
int orc_chi2(const double p[6], const double C[36], int kind,
             const double hit[3], double var_u, double var_v, double stereo, double *chi2);

/* General linear Kalman update with an m-dimensional measurement
 * (m <= 2): K = C H^T S^-1, p += K r, C -= K S K^T (symmetrised).
 * joseph != 0 uses (I-KH) C (I-KH)^T + K V K^T instead.  chi2 out. */
void orc_kf_update(double p[6], double C[36], int m, const double *H,
                   const double *r, const double *V, int joseph,
                   double *chi2);

/* Hit update at a layer: measure + orc_kf_update + wrap phi (V as in
 * orc_chi2). */
int orc_update_hit(double p[6], double C[36], int kind, const double hit[3],
                   double var_u, double var_v, double stereo, double *chi2);

/* ---- seeding, plan, find, fit --------------------------------------- */

typedef struct {
  int32_t ok;          /* 1 if seeding succeeded */
  double par[6];       /* seed state on the third seed layer */
  double cov[36];
  int32_t plan_len;
  int32_t plan[ORC_MAX_PLAN];
  double plan_l[ORC_MAX_PLAN];
  int32_t plan_fragile; /* a crossing lies within tol of a widened edge */
  double chi2;          /* sum of the three hit updates' chi2 */
} orc_seed_out;

/* h: 3 hits x (x,y,z); hv: 3 hits x (var_u, var_v); hl: their layers.
 * pos_tol: distance to a widened edge below which the plan is flagged.
 * With region steering the plan is the seed's region's layer list less the
 * seed layers, flagged if eta lies within ORC_ETA_TOL of a region bound. */
int orc_seed(const orc_cfg *cfg, const orc_layer *layers, int32_t n_layers,
             const double h[9], const double hv[6], const int32_t hl[3],
             double pos_tol, orc_seed_out *out);

typedef struct {
  int32_t seed_ok;
  int32_t n_hits, n_miss, plan_len;
  int32_t plan[ORC_MAX_PLAN];
  int32_t hit[ORC_MAX_PLAN];
  double par[6];
  double cov[36];
  double chi2;
  /* parity bookkeeping: first plan step (0-based) at which a decision was
   * within tolerance of a cut or a tie, plan_len if the final choice was,
   * -1 if no decision was fragile. */
  int32_t fragile_step;
  int64_t n_steps; /* candidate-layer steps taken for this seed */
  int32_t plan_fragile; /* the plan itself holds a fragile decision */
} orc_track;

typedef struct {
  double chi2_rel, chi2_abs; /* chi2 tolerance: rel * chi2 + abs */
  double pos_tol;            /* cm, for extent-edge decisions */
} orc_tol;

/* Clone-engine track finding for n_seeds seeds of one event.  Hits are
 * the event's hits (FP32 inputs, original order).  seed_hits holds 3
 * event-local hit indices per seed. */
int orc_find_event(const orc_cfg *cfg, const orc_tol *tol,
                   const orc_layer *layers, int32_t n_layers, int32_t n_hits,
                   const float *x, const float *y, const float *z,
                   const float *var_u, const float *var_v,
                   const int32_t *layer, int32_t n_seeds,
                   const int32_t *seed_hits, orc_track *out);

/* Parity bookkeeping for a seed whose result differs from another
 * implementation's.  The histories (ORC_MAX_PLAN entries each) of the
 * candidates alive when the find reaches plan step `step` (those kept at
 * step - 1, in rank order), then of those retired before it; at step >=
 * plan_len the final candidates and every retired one.  Up to cap are
 * written to hist; returns their number (-1 on bad input).  Before the
 * first fragile step every decision is clear, so another implementation's
 * candidates there must be exactly these. */
int32_t orc_find_prefixes(const orc_cfg *cfg, const orc_tol *tol, const orc_layer *layers,
                          int32_t n_layers, int32_t n_hits, const float *x, const float *y,
                          const float *z, const float *var_u, const float *var_v,
                          const int32_t *layer, const int32_t seed_hits[3], int32_t step,
                          int32_t cap, int32_t *hist);

typedef struct {
  int32_t bad_step;   /* first step whose decision is invalid, -1 if none */
  int32_t n_hits, n_miss;
  double chi2;        /* sum of the hits' chi2 tests, as the find sums them */
  double max_chi2;    /* largest hit chi2 */
  int32_t n_near_cut; /* decisions within the chi2 tolerance of the cut */
  int32_t n_edge;     /* crossings within pos_tol of an extent or material edge */
  double par[6], cov[36];
} orc_path;

/* Follow a given history (hit index, ORC_HIT_MISS, ORC_HIT_SKIP or
 * ORC_HIT_NONE per plan step) of a seed with the find's filter and check
 * each decision: a hit lies on the step's layer with chi2 below cut + tol;
 * a miss needs a crossing and a hole left; a skip, no crossing inside the
 * widened extent; retiring (NONE from then on), a crossing, no hole left and
 * no hit clearly below the cut.  Crossing decisions within pos_tol of an
 * edge are accepted either way.  Returns 0 if every decision is valid, 1 if
 * not (out->bad_step), -1 if the seed fit fails or the plan differs. */
int orc_follow_path(const orc_cfg *cfg, const orc_tol *tol, const orc_layer *layers,
                    int32_t n_layers, int32_t n_hits, const float *x, const float *y,
                    const float *z, const float *var_u, const float *var_v,
                    const int32_t *layer, const int32_t seed_hits[3], int32_t plan_len,
                    const int32_t *plan, const int32_t *hist, orc_path *out);

/* Kalman fit of one track through n hits on given surfaces (no search,
 * no extent test).  kinds/pos describe each hit's surface. */
int orc_fit_track(const orc_cfg *cfg, const double p0[6], const double C0[36],
                  int32_t n, const int32_t *kinds, const double *pos,
                  const double *hits /* n x 3 */, const double *var_u,
                  const double *var_v, double p_out[6], double C_out[36],
                  double *chi2_sum);

/* Reverse the direction of motion on the same helix (q/pT, phi + pi,
 * pi - theta); C (may be NULL) becomes D C D, D = diag(1,1,1,-1,1,-1). */
void orc_flip(double p[6], double C[36]);

/* Backward fit of one found track of an event: the Kalman filter over its
 * hits in reverse order (crossed plan layers last to first, then the seed
 * layers third to first), from its final state with the seed prior.
 * Returns 1 (state on the first seed layer), 0 (seed fit failed) or -k
 * (surface k of the reversed sequence not reached or its update failed). */
int orc_backward_fit(const orc_cfg *cfg, const orc_layer *layers, int32_t n_layers,
                     const float *x, const float *y, const float *z, const float *var_u,
                     const float *var_v, const int32_t *layer, const int32_t seed_hits[3],
                     const orc_track *trk, double p_out[6], double C_out[36], double *chi2_sum,
                     int32_t *n_updates);

/* Rauch-Tung-Striebel smoothing of one found track: on the seed's third
 * layer (seed_layer, starting from the seed fit's seed_par, seed_cov) and
 * on every plan layer the track crossed, the state given all its hits.
 * Writes surf_layer [n], par_out [n][6], cov_out [n][36] with n <=
 * ORC_MAX_PLAN + 1 and returns n; 0 if the seed fit failed, -1 if a
 * propagation or update failed, -2 if a predicted covariance is singular
 * on its surface. */
int orc_smooth_track(const orc_cfg *cfg, const orc_layer *layers, int32_t n_layers,
                     const float *x, const float *y, const float *z, const float *var_u,
                     const float *var_v, int32_t seed_layer, const double seed_par[6],
                     const double seed_cov[36], const orc_track *trk, int32_t *surf_layer,
                     double *par_out, double *cov_out);

/* ---- triplet seeding (the paper takes seeds from outside) ---------- */

typedef struct {
  int32_t layer[3]; /* three barrel layers, innermost first */
  double pt_min;    /* GeV/c */
  double d0_max;    /* cm: transverse distance of the circle from the beam line */
  double z0_max;    /* cm: |z| at the point of closest approach to the beam line */
  double dz_max;    /* cm: middle hit off the s-z line of the outer two */
} orc_seeding;

/* Cut variables of one triplet (pt, d0, dz, z0, psi_ab, psi_ac, psi_0a; v
 * may be NULL) and the smallest relative margin to a cut; 1 if it passes. */
int orc_triplet_params(const orc_cfg *cfg, const orc_seeding *sc, const double a[3],
                       const double b[3], const double c[3], double v[7], double *margin);

/* Brute-force triplet seeds of one event; see the definition above. */
int64_t orc_triplet_seeds(const orc_cfg *cfg, const orc_seeding *sc, int32_t n_hits,
                          const float *x, const float *y, const float *z, const int32_t *layer,
                          int32_t a_only, double frag_tol, int64_t cap, int32_t *out,
                          int32_t *fragile, int64_t *n_fragile_out);

/* ---- duplicate-track removal ---------------------------------------- */

/* t is a duplicate if a track ranking before it (more hits; then smaller
 * chi2; then smaller seed triplet) shares at least frac of the hits of the
 * shorter of the two.  Returns the number of duplicates. */
int32_t orc_duplicates(int32_t n, int32_t stride, const int32_t *n_hits, const int32_t *hits,
                       const double *chi2, const int32_t *seed, double frac, double chi2_tol_rel,
                       double chi2_tol_abs, int32_t *dup, int32_t *fragile);

/* ---- seed cleaning (Section 2.2) ------------------------------------ */

/* Keeps a seed unless a seed ranking before it (smaller fit chi2, then
 * smaller triplet) shares a hit with it and agrees in q/pT, eta and phi
 * within the tolerances.  Returns the number kept. */
int32_t orc_clean_seeds(int32_t n, const int32_t *trip, const int32_t *ok, const double *par,
                        const double *chi2, double tol_ipt, double tol_eta, double tol_phi,
                        double frag_rel, int32_t *keep, int32_t *fragile);

#ifdef __cplusplus
}
#endif
#endif
