/*
 * TEST INFRASTRUCTURE: a driver that runs every entry point of the CPU
 * oracle on a small deterministic event, built with AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_oracle_sanitize.py.  It checks
 * memory safety and undefined behaviour only (the numerics are pinned by
 * the other oracle tests); it exits non-zero if an entry point reports an
 * error it should not.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/mkf_oracle.h"

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

int orc_mlp_nparam(void);
void orc_mlp_forward(const double *p, int B, const double *x, int round_bf16, double *y);
double orc_mlp_grad(const double *p, int B, const double *x, const double *t, const double *w,
                    int round_bf16, double *g);
void orc_adam(double *p, double *m, double *v, const double *g, int n, int t, double lr,
              double b1, double b2, double eps);
double orc_lr_cosine(double lr, int n_steps, int s);

/* 64-bit linear congruential stream (Knuth's MMIX constants) */
static unsigned long long rng_state = 0x5EED5A17ull;
static double uni(void) {
  rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

#define N_LAYERS 14
#define MAX_HITS 4096

static int fail(const char *what) {
  fprintf(stderr, "oracle driver: %s\n", what);
  return 1;
}

int main(void) {
  orc_layer L[N_LAYERS];
  const double radii[10] = {4, 7, 11, 16, 25, 34, 43, 52, 61, 70};
  for (int i = 0; i < 10; ++i) {
    orc_layer b = {0, radii[i], -100.0, 100.0, i == 4 ? 0.1 : 0.0, i == 5 ? -1.0 : 0.0,
                   i == 5 ? 1.0 : 0.0};
    L[i] = b;
  }
  for (int i = 0; i < 4; ++i) {
    orc_layer d = {1, (i < 2 ? 1.0 : -1.0) * (120.0 + 40.0 * (i % 2)), 20.0, 110.0, 0.0, 50.0,
                   55.0};
    L[10 + i] = d;
  }
  double xx0[4 * 6], xi[4 * 6];
  for (int i = 0; i < 24; ++i) {
    xx0[i] = 0.01 + 0.005 * (i % 3);
    xi[i] = 0.1 + 0.02 * (i % 5);
  }
  orc_material mat = {6, 4, 120.0, 300.0, 0.13957, 10.0, xx0, xi};
  orc_field fld = {3.8, -1e-6, -2e-6, 1e-11, 0.5};
  orc_region reg[2] = {{-0.9, 0.9, 7, {3, 4, 5, 6, 7, 8, 9}},
                       {0.9, 3.0, 6, {3, 4, 5, 10, 11, 9}}};
  orc_cfg cfg;
  memset(&cfg, 0, sizeof(cfg));
  cfg.bz = 3.8;
  cfg.kappa = ORC_KAPPA;
  cfg.chi2_cut = 30.0;
  cfg.ms_sigma = 0.001;
  cfg.edge_margin = 2.0;
  cfg.l_min = 1e-4;
  cfg.n_cand = 6;
  cfg.max_holes = 3;
  for (int i = 0; i < 6; ++i) cfg.init_var[i] = i < 3 ? 1.0 : (i == 3 ? 1.0 : 0.01);

  /* hits: exact crossings of 40 helices from the beam line, plus noise */
  static float x[MAX_HITS], y[MAX_HITS], z[MAX_HITS], vu[MAX_HITS], vv[MAX_HITS];
  static int32_t lay[MAX_HITS], seeds[40 * 3];
  int n = 0, ns = 0;
  for (int t = 0; t < 40; ++t) {
    double phi = (uni() * 2.0 - 1.0) * M_PI, eta = (uni() * 2.0 - 1.0) * 1.2;
    double pt = 0.5 + 5.0 * uni();
    double p[6] = {0.0, 0.0, (uni() - 0.5) * 5.0, (uni() < 0.5 ? -1.0 : 1.0) / pt, phi,
                   2.0 * atan(exp(-eta))};
    int first = n, k = 0;
    for (int i = 0; i < N_LAYERS && n < MAX_HITS - 8; ++i) {
      double q[6], l;
      if (orc_propagate(p, NULL, &L[i], cfg.bz, cfg.kappa, cfg.l_min, 0.0, 1, q, NULL, NULL, &l) !=
          ORC_OK)
        continue;
      x[n] = (float)(q[0] + 0.003 * (uni() - 0.5));
      y[n] = (float)(q[1] + 0.003 * (uni() - 0.5));
      z[n] = (float)q[2];
      vu[n] = 9e-6f;
      vv[n] = 1e-4f;
      lay[n] = i;
      ++n;
      ++k;
      if (L[i].kind == 0) memcpy(p, q, sizeof(q));
    }
    if (k >= 3 && lay[first] == 0 && lay[first + 1] == 1 && lay[first + 2] == 2) {
      seeds[3 * ns] = first;
      seeds[3 * ns + 1] = first + 1;
      seeds[3 * ns + 2] = first + 2;
      ++ns;
    }
  }
  for (int i = 0; i < 300 && n < MAX_HITS; ++i, ++n) {
    int li = (int)(uni() * 10);
    double a = uni() * 2.0 * M_PI;
    x[n] = (float)(radii[li] * cos(a));
    y[n] = (float)(radii[li] * sin(a));
    z[n] = (float)((uni() - 0.5) * 200.0);
    vu[n] = 9e-6f;
    vv[n] = 1e-4f;
    lay[n] = li;
  }
  if (ns < 10) return fail("too few seeds");

  orc_tol tol = {1e-3, 1e-2, 1e-3};
  orc_track *tr = (orc_track *)calloc((size_t)ns, sizeof(orc_track));
  /* plain, material, field and steering variants of the find */
  for (int v = 0; v < 4; ++v) {
    orc_cfg c = cfg;
    if (v == 1) c.material = &mat;
    if (v == 2) c.field = &fld;
    if (v == 3) {
      c.regions = reg;
      c.n_regions = 2;
    }
    if (orc_find_event(&c, &tol, L, N_LAYERS, n, x, y, z, vu, vv, lay, ns, seeds, tr) != 0)
      return fail("find");
    for (int s = 0; s < ns; ++s) {
      if (!tr[s].seed_ok) continue;
      int32_t hist[64 * ORC_MAX_PLAN];
      int32_t np = orc_find_prefixes(&c, &tol, L, N_LAYERS, n, x, y, z, vu, vv, lay,
                                     &seeds[3 * s], tr[s].plan_len, 64, hist);
      if (np < 1) return fail("prefixes");
      orc_path path;
      if (orc_follow_path(&c, &tol, L, N_LAYERS, n, x, y, z, vu, vv, lay, &seeds[3 * s],
                          tr[s].plan_len, tr[s].plan, tr[s].hit, &path) != 0)
        return fail("follow_path of the oracle's own track");
      double pb[6], Cb[36], chi2;
      int32_t nu;
      orc_backward_fit(&c, L, N_LAYERS, x, y, z, vu, vv, lay, &seeds[3 * s], &tr[s], pb, Cb,
                       &chi2, &nu);
      double h[9], hv[6];
      int32_t hl[3];
      for (int k = 0; k < 3; ++k) {
        int32_t i = seeds[3 * s + k];
        h[3 * k] = x[i];
        h[3 * k + 1] = y[i];
        h[3 * k + 2] = z[i];
        hv[2 * k] = vu[i];
        hv[2 * k + 1] = vv[i];
        hl[k] = lay[i];
      }
      orc_seed_out so;
      if (orc_seed(&c, L, N_LAYERS, h, hv, hl, 1e-3, &so)) {
        int32_t sl[ORC_MAX_PLAN + 1];
        static double sp[(ORC_MAX_PLAN + 1) * 6], sc[(ORC_MAX_PLAN + 1) * 36];
        orc_smooth_track(&c, L, N_LAYERS, x, y, z, vu, vv, hl[2], so.par, so.cov, &tr[s], sl, sp,
                         sc);
      }
    }
  }
  /* the fit through a known sequence of surfaces */
  {
    int32_t kinds[8];
    double pos[8], hh[24], fu[8], fv[8], po[6], Co[36], c2;
    double p0[6] = {0.0, 0.0, 0.0, 0.5, 0.3, 1.2}, C0[36];
    memset(C0, 0, sizeof(C0));
    for (int i = 0; i < 6; ++i) C0[7 * i] = 0.01;
    for (int i = 0; i < 8; ++i) {
      kinds[i] = 0;
      pos[i] = radii[i + 2];
      double q[6];
      if (orc_propagate(p0, NULL, &L[i + 2], cfg.bz, cfg.kappa, cfg.l_min, 0.0, 0, q, NULL, NULL,
                        NULL) != ORC_OK)
        return fail("fit inputs");
      memcpy(&hh[3 * i], q, 3 * sizeof(double));
      fu[i] = 9e-6;
      fv[i] = 1e-4;
    }
    if (orc_fit_track(&cfg, p0, C0, 8, kinds, pos, hh, fu, fv, po, Co, &c2) != 0)
      return fail("fit");
  }
  /* triplet seeding, duplicate removal and seed cleaning */
  {
    orc_seeding sc = {{0, 1, 2}, 0.3, 1.0, 15.0, 0.5};
    static int32_t trip[3 * 8192], frag[8192];
    int64_t nf = 0;
    int64_t nt = orc_triplet_seeds(&cfg, &sc, n, x, y, z, lay, -1, 1e-9, 8192, trip, frag, &nf);
    if (nt < 0 || nt > 8192) return fail("triplets");
    int32_t m = (int32_t)(nt < 400 ? nt : 400);
    orc_track *tt = (orc_track *)calloc((size_t)(m > 0 ? m : 1), sizeof(orc_track));
    if (m > 0 &&
        orc_find_event(&cfg, &tol, L, N_LAYERS, n, x, y, z, vu, vv, lay, m, trip, tt) != 0)
      return fail("find from triplets");
    int32_t stride = 3 + ORC_MAX_PLAN;
    int32_t *nh = (int32_t *)calloc((size_t)m + 1, sizeof(int32_t));
    int32_t *hits = (int32_t *)calloc((size_t)(m + 1) * stride, sizeof(int32_t));
    double *chi = (double *)calloc((size_t)m + 1, sizeof(double));
    double *par = (double *)calloc((size_t)(m + 1) * 6, sizeof(double));
    int32_t *ok = (int32_t *)calloc((size_t)m + 1, sizeof(int32_t));
    int32_t *dup = (int32_t *)calloc((size_t)m + 1, sizeof(int32_t));
    int32_t *fr = (int32_t *)calloc((size_t)m + 1, sizeof(int32_t));
    for (int i = 0; i < m; ++i) {
      int k = 0;
      for (int j = 0; j < 3; ++j) hits[i * stride + k++] = trip[3 * i + j];
      for (int j = 0; j < tt[i].plan_len; ++j)
        if (tt[i].hit[j] >= 0) hits[i * stride + k++] = tt[i].hit[j];
      nh[i] = k;
      chi[i] = tt[i].chi2;
      ok[i] = tt[i].seed_ok;
      memcpy(&par[6 * i], tt[i].par, sizeof(tt[i].par));
    }
    orc_duplicates(m, stride, nh, hits, chi, trip, 0.5, 1e-3, 1e-2, dup, fr);
    orc_clean_seeds(m, trip, ok, par, chi, 0.1, 0.05, 0.05, 1e-4, dup, fr);
    free(tt);
    free(nh);
    free(hits);
    free(chi);
    free(par);
    free(ok);
    free(dup);
    free(fr);
  }
  /* the network: forward, gradient, Adam step and schedule */
  {
    int np = orc_mlp_nparam();
    double *p = (double *)malloc(sizeof(double) * np), *g = (double *)malloc(sizeof(double) * np);
    double *m = (double *)calloc((size_t)np, sizeof(double));
    double *v = (double *)calloc((size_t)np, sizeof(double));
    double xin[16 * 8], t[16 * 7], w[7] = {1, 1, 1, 1, 1, 1, 1}, yo[16 * 7];
    for (int i = 0; i < np; ++i) p[i] = 0.1 * (uni() - 0.5);
    for (int i = 0; i < 16 * 8; ++i) xin[i] = uni();
    for (int i = 0; i < 16 * 7; ++i) t[i] = uni();
    orc_mlp_forward(p, 16, xin, 1, yo);
    orc_mlp_grad(p, 16, xin, t, w, 0, g);
    orc_adam(p, m, v, g, np, 1, orc_lr_cosine(1e-3, 10, 3), 0.9, 0.999, 1e-8);
    free(p);
    free(g);
    free(m);
    free(v);
  }
  free(tr);
  printf("oracle driver ok: %d hits, %d seeds\n", n, ns);
  return 0;
}
