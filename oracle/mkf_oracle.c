/*
 * mkf_oracle.c -- TEST INFRASTRUCTURE ONLY: a plain FP64 CPU reference of
 * Kalman-filter track finding and fitting (arXiv:1811.04141).  Used only by
 * the tests, the smoke check and the benchmark's CPU-baseline leg; the GPU
 * library never links it.
 *
 * The paper gives the method in words only (no equations, no listings):
 *   - the Kalman filter it builds on (Introduction, ref. Fruhwirth);
 *   - propagation and KF equations for both barrel cylinders and endcap
 *     disks (Introduction, the paragraph on realistic geometries);
 *   - a layer description and a per-region layer plan followed by track
 *     finding (Section 2.1);
 *   - multiple scattering from material and a constant field (Section 2.1);
 *   - the "clone engine": score all hit extensions of all candidates by
 *     chi2 first, keep the best ones, and only then run the Kalman updates
 *     (Introduction);
 *   - seeds and hits supplied from outside (Section 2.2).
 * Every formula below is therefore the textbook definition it names.  The
 * readings chosen where the paper is silent are listed in the design notes
 * and repeated next to the code that takes them.
 */
#include "mkf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ---------------------------------------------------------------- util */

static double wrap_phi(double a) {
  /* map to (-pi, pi] */
  a = fmod(a, 2.0 * M_PI);
  if (a <= -M_PI) a += 2.0 * M_PI;
  if (a > M_PI) a -= 2.0 * M_PI;
  return a;
}

static double sinc(double h) { return h == 0.0 ? 1.0 : sin(h) / h; }

/* d sinc / dh; the closed form cancels for small h, so a Taylor series is
 * used there (terms through h^7). */
static double dsinc(double h) {
  if (fabs(h) < 1e-2) {
    double h2 = h * h;
    return h * (-1.0 / 3.0 + h2 * (1.0 / 30.0 + h2 * (-1.0 / 840.0 + h2 / 45360.0)));
  }
  return (h * cos(h) - sin(h)) / (h * h);
}

static void matmul6(const double *A, const double *B, double *C) {
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      double s = 0.0;
      for (int k = 0; k < 6; ++k) s += A[i * 6 + k] * B[k * 6 + j];
      C[i * 6 + j] = s;
    }
}

static void transpose6(const double *A, double *At) {
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) At[j * 6 + i] = A[i * 6 + j];
}

static void symmetrize6(double *C) {
  for (int i = 0; i < 6; ++i)
    for (int j = i + 1; j < 6; ++j) {
      double s = 0.5 * (C[i * 6 + j] + C[j * 6 + i]);
      C[i * 6 + j] = s;
      C[j * 6 + i] = s;
    }
}

/* ------------------------------------------------------ helix transport */

/* Motion of a charge in a uniform field B along +z (Lorentz force
 * F = q v x B): the transverse projection is a circle with signed
 * curvature omega = -kappa * B * (q/pT) (a positive charge turns clockwise
 * seen from +z), and z advances by l * cot(theta).  With h = omega*l/2 the
 * chord is l*sinc(h) long and points along phi + h. */
void orc_transport(const double p[6], double l, double bz, double kappa,
                   double out[6]) {
  double w = -kappa * bz * p[3];
  double h = 0.5 * w * l;
  double L = l * sinc(h);
  double psi = p[4] + h;
  out[0] = p[0] + L * cos(psi);
  out[1] = p[1] + L * sin(psi);
  out[2] = p[2] + l * cos(p[5]) / sin(p[5]);
  out[3] = p[3];
  out[4] = wrap_phi(p[4] + w * l);
  out[5] = p[5];
}

/* ------------------------------------------------- crossing a cylinder */

/* Exact crossing of the helix with the cylinder r = R.
 *
 * With a = x cos(phi) + y sin(phi), c = y cos(phi) - x sin(phi) and
 * g0 = x^2 + y^2 - R^2, the squared radius after a transverse path l is
 *   r(l)^2 - R^2 = g0 + L^2 + 2 L (a cos h + c sin h),  L = 2 sin(h)/omega.
 * Multiplying by 1/cos^2(h) and substituting tau = (2/omega) tan(h) gives
 * the quadratic
 *   (1 + c omega + g0 omega^2 / 4) tau^2 + 2 a tau + g0 = 0,
 * whose real roots are exactly the crossings with |omega l| < pi (the
 * first half turn each way), and l = (2/omega) atan(omega tau / 2).
 * Both maps are monotonic, so the smallest admissible root in tau is the
 * smallest in l.  For omega -> 0 the quadratic becomes the straight
 * line / circle equation, so the form is well conditioned at high pT. */
static double tau_to_l(double tau, double w) {
  double zz = 0.5 * w * tau;
  double f = fabs(zz) < 1e-8 ? 1.0 - zz * zz / 3.0 : atan(zz) / zz;
  return tau * f;
}

int orc_path_to_barrel(const double p[6], double R, double bz, double kappa,
                       double l_min, double *l_out) {
  double w = -kappa * bz * p[3];
  double cphi = cos(p[4]), sphi = sin(p[4]);
  double a = p[0] * cphi + p[1] * sphi;
  double c = p[1] * cphi - p[0] * sphi;
  double g0 = p[0] * p[0] + p[1] * p[1] - R * R;
  double alpha = 1.0 + c * w + 0.25 * g0 * w * w;
  double roots[2];
  int nr = 0;
  if (alpha == 0.0) {
    if (a != 0.0) roots[nr++] = -g0 / (2.0 * a);
  } else {
    double disc = a * a - alpha * g0;
    if (disc < 0.0) return ORC_NO_CROSSING;
    double sq = sqrt(disc);
    double qq = -(a + copysign(sq, a));
    if (qq != 0.0) {
      roots[nr++] = qq / alpha;
      roots[nr++] = g0 / qq;
    } else {
      roots[nr++] = 0.0;
    }
  }
  double best = INFINITY;
  for (int i = 0; i < nr; ++i) {
    double l = tau_to_l(roots[i], w);
    if (l > l_min && l < best) best = l;
  }
  if (!(best < INFINITY)) return ORC_NO_CROSSING;
  *l_out = best;
  return ORC_OK;
}

/* Disk z = Z: z advances linearly, so l = (Z - z) tan(theta); it must be
 * beyond l_min and within the first half turn. */
int orc_path_to_disk(const double p[6], double Z, double bz, double kappa,
                     double l_min, double *l_out) {
  double ct = cos(p[5]);
  if (ct == 0.0) return ORC_NO_CROSSING;
  double l = (Z - p[2]) * sin(p[5]) / ct;
  double w = -kappa * bz * p[3];
  if (!(l > l_min) || fabs(w) * l >= M_PI) return ORC_NO_CROSSING;
  *l_out = l;
  return ORC_OK;
}

/* ------------------------------------------------- full propagation */

/* Propagation to a layer with the surface-constrained Jacobian.
 *
 * D = d p'/d p0 at fixed l follows from the transport above.  The path
 * itself depends on p0 through the surface condition g(p') = 0 (barrel:
 * g = x'^2 + y'^2 - R^2, disk: g = z' - Z), so with n = dg/dp' and
 * t = dp'/dl = (cos phi', sin phi', cot theta, 0, omega, 0):
 *   dl/dp0 = -(n^T D)/(n^T t),  F = D + t (dl/dp0)^T = (I - t n^T/(n^T t)) D.
 * C' = F C F^T then has n as a null direction (rank 5): the state is
 * constrained to the surface. */
double orc_field_bz(const orc_field *f, double x, double y, double z) {
  double r2 = x * x + y * y, z2 = z * z;
  return f->b0 * (1.0 + f->c_r2 * r2 + f->c_z2 * z2 + f->c_z4 * z2 * z2);
}

/* d(x, y, z, phi)/dl in the axial field */
static void field_deriv(const orc_field *f, double kappa, double ipt, double cot,
                        const double y[4], double d[4]) {
  d[0] = cos(y[3]);
  d[1] = sin(y[3]);
  d[2] = cot;
  d[3] = -kappa * orc_field_bz(f, y[0], y[1], y[2]) * ipt;
}

/* one classical Runge-Kutta step of transverse length h */
static void rk4(const orc_field *f, double kappa, double ipt, double cot, const double y[4],
                double h, double out[4]) {
  double k1[4], k2[4], k3[4], k4[4], t[4];
  field_deriv(f, kappa, ipt, cot, y, k1);
  for (int i = 0; i < 4; ++i) t[i] = y[i] + 0.5 * h * k1[i];
  field_deriv(f, kappa, ipt, cot, t, k2);
  for (int i = 0; i < 4; ++i) t[i] = y[i] + 0.5 * h * k2[i];
  field_deriv(f, kappa, ipt, cot, t, k3);
  for (int i = 0; i < 4; ++i) t[i] = y[i] + h * k3[i];
  field_deriv(f, kappa, ipt, cot, t, k4);
  for (int i = 0; i < 4; ++i) out[i] = y[i] + h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
}

#define ORC_FIELD_MAX_PATH 1000.0 /* cm of transverse path searched */
#define ORC_NEWTON_TOL 1e-12      /* cm: Newton stops once its correction is below this */
#define ORC_NEWTON_MAX 50

/* Crossing of a layer in the parameterised field: path l and the end
 * point y = (x, y, z, phi unwrapped).  The search is bounded by the path
 * (ORC_FIELD_MAX_PATH) and the half turn only, whatever the step size.  On
 * a barrel the last step's length s solves r(s)^2 = R^2 for the Runge-Kutta
 * step from the bracket's start, by Newton's method run to convergence. */
static int field_crossing(const double p[6], const orc_layer *Lr, double kappa, double l_min,
                          const orc_field *f, double *l_out, double yend[4]) {
  double cot = cos(p[5]) / sin(p[5]);
  double y[4] = {p[0], p[1], p[2], p[4]};
  if (Lr->kind == 1) {
    if (cos(p[5]) == 0.0) return ORC_NO_CROSSING;
    double lt = (Lr->pos - p[2]) * sin(p[5]) / cos(p[5]);
    if (!(lt > l_min) || lt > ORC_FIELD_MAX_PATH) return ORC_NO_CROSSING;
    int n = (int)ceil(lt / f->h_max);
    double h = lt / n;
    for (int k = 0; k < n; ++k) {
      rk4(f, kappa, p[3], cot, y, h, y);
      if (fabs(y[3] - p[4]) >= M_PI) return ORC_NO_CROSSING;
    }
    y[2] = Lr->pos;
    *l_out = lt;
    memcpy(yend, y, sizeof(y));
    return ORC_OK;
  }
  double R2 = Lr->pos * Lr->pos;
  double g = y[0] * y[0] + y[1] * y[1] - R2, l = 0.0;
  for (long k = 0;; ++k) {
    double yn[4];
    rk4(f, kappa, p[3], cot, y, f->h_max, yn);
    double gn = yn[0] * yn[0] + yn[1] * yn[1] - R2;
    if ((g < 0.0) != (gn < 0.0) || gn == 0.0) {
      /* Newton on the step length s from the bracket's start, from the
       * secant's guess */
      double s = g == gn ? f->h_max : f->h_max * g / (g - gn), ys[4];
      for (int it = 0; it < ORC_NEWTON_MAX; ++it) {
        rk4(f, kappa, p[3], cot, y, s, ys);
        double gs = ys[0] * ys[0] + ys[1] * ys[1] - R2;
        double gp = 2.0 * (ys[0] * cos(ys[3]) + ys[1] * sin(ys[3]));
        if (gp == 0.0) break;
        double ds = gs / gp;
        s -= ds;
        if (fabs(ds) <= ORC_NEWTON_TOL) break;
      }
      rk4(f, kappa, p[3], cot, y, s, ys);
      if (l + s > l_min && fabs(ys[3] - p[4]) < M_PI) {
        *l_out = l + s;
        memcpy(yend, ys, sizeof(ys));
        return ORC_OK;
      }
    }
    if (fabs(yn[3] - p[4]) >= M_PI) return ORC_NO_CROSSING;
    memcpy(y, yn, sizeof(yn));
    g = gn;
    l = (double)(k + 1) * f->h_max;
    if (l > ORC_FIELD_MAX_PATH) return ORC_NO_CROSSING;
  }
}

int orc_propagate(const double p[6], const double C[36], const orc_layer *Lr,
                  double bz, double kappa, double l_min, double edge_margin,
                  int check_extent, double p_out[6], double C_out[36],
                  double F_out[36], double *l_out) {
  return orc_propagate_f(p, C, Lr, bz, kappa, l_min, edge_margin, check_extent, p_out, C_out,
                         F_out, l_out, NULL);
}

int orc_propagate_f(const double p[6], const double C[36], const orc_layer *Lr,
                    double bz, double kappa, double l_min, double edge_margin,
                    int check_extent, double p_out[6], double C_out[36],
                    double F_out[36], double *l_out, const orc_field *fld) {
  double l;
  double pp[6];
  double dw = -kappa * bz; /* d omega / d(q/pT) */
  if (fld) {
    double y[4];
    int st = field_crossing(p, Lr, kappa, l_min, fld, &l, y);
    if (st != ORC_OK) return st;
    pp[0] = y[0];
    pp[1] = y[1];
    pp[2] = y[2];
    pp[3] = p[3];
    pp[4] = wrap_phi(y[3]);
    pp[5] = p[5];
    /* the helix of the path's mean curvature: omega = turning / l */
    if (p[3] != 0.0) dw = (y[3] - p[4]) / (l * p[3]);
  } else {
    int st = Lr->kind == 0
                 ? orc_path_to_barrel(p, Lr->pos, bz, kappa, l_min, &l)
                 : orc_path_to_disk(p, Lr->pos, bz, kappa, l_min, &l);
    if (st != ORC_OK) return st;
    orc_transport(p, l, bz, kappa, pp);
  }
  if (check_extent) {
    double q = Lr->kind == 0 ? pp[2] : hypot(pp[0], pp[1]);
    if (q < Lr->ext_lo - edge_margin || q > Lr->ext_hi + edge_margin)
      return ORC_OUT_OF_EXTENT;
    /* a hole (hole_lo < q < hole_hi, shrunk by the same margin) has no
     * sensors: a crossing there is outside the layer */
    if (q > Lr->hole_lo + edge_margin && q < Lr->hole_hi - edge_margin) return ORC_OUT_OF_EXTENT;
  }
  if (l_out) *l_out = l;
  memcpy(p_out, pp, sizeof(pp));
  if (!F_out && !C_out) return ORC_OK;

  double w = dw * p[3];
  double h = 0.5 * w * l;
  double L = l * sinc(h);
  double psi = p[4] + h;
  double dLdw = l * dsinc(h) * 0.5 * l;
  double st5 = sin(p[5]);
  double D[36];
  memset(D, 0, sizeof(D));
  for (int i = 0; i < 6; ++i) D[i * 6 + i] = 1.0;
  D[0 * 6 + 3] = (dLdw * cos(psi) - L * sin(psi) * 0.5 * l) * dw;
  D[0 * 6 + 4] = -L * sin(psi);
  D[1 * 6 + 3] = (dLdw * sin(psi) + L * cos(psi) * 0.5 * l) * dw;
  D[1 * 6 + 4] = L * cos(psi);
  D[2 * 6 + 5] = -l / (st5 * st5);
  D[4 * 6 + 3] = l * dw;

  double t[6] = {cos(pp[4]), sin(pp[4]), cos(pp[5]) / sin(pp[5]), 0.0, w, 0.0};
  double n[6] = {0, 0, 0, 0, 0, 0};
  if (Lr->kind == 0) {
    n[0] = 2.0 * pp[0];
    n[1] = 2.0 * pp[1];
  } else {
    n[2] = 1.0;
  }
  double nt = 0.0;
  for (int i = 0; i < 6; ++i) nt += n[i] * t[i];
  double nD[6];
  for (int j = 0; j < 6; ++j) {
    double s = 0.0;
    for (int i = 0; i < 6; ++i) s += n[i] * D[i * 6 + j];
    nD[j] = s;
  }
  double F[36];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) F[i * 6 + j] = D[i * 6 + j] - t[i] * nD[j] / nt;
  if (F_out) memcpy(F_out, F, sizeof(F));
  if (C && C_out) {
    double FC[36], Ft[36];
    matmul6(F, C, FC);
    transpose6(F, Ft);
    matmul6(FC, Ft, C_out);
    symmetrize6(C_out);
  }
  return ORC_OK;
}

/* ------------------------------------------------ multiple scattering */

/* Two independent deflections of the momentum direction, each with
 * standard deviation sigma, perpendicular to the momentum, |p| unchanged:
 * theta moves by d_theta, phi by d_alpha / sin(theta), and since
 * pT = |p| sin(theta), q/pT moves by -(q/pT) cot(theta) d_theta. */
void orc_add_ms(const double p[6], double sigma, double C[36]) {
  if (sigma == 0.0) return;
  double s2 = sigma * sigma;
  double st = sin(p[5]), cot = cos(p[5]) / st;
  double a = p[3] * cot;
  C[3 * 6 + 3] += a * a * s2;
  C[3 * 6 + 5] += -a * s2;
  C[5 * 6 + 3] += -a * s2;
  C[4 * 6 + 4] += s2 / (st * st);
  C[5 * 6 + 5] += s2;
}

/* Bethe's mean mass stopping power (PDG form: K Z/A / beta^2 *
 * (ln(2 m_e c^2 b^2 g^2 T_max / I^2) / 2 - beta^2)) for silicon, without
 * the density-effect and shell corrections. */
double orc_bethe_si(double bg, double mass) {
  const double K = 0.307075e-3;   /* GeV cm^2 / mol */
  const double ZA = 0.49848;      /* mol / g */
  const double I = 173e-9;        /* GeV */
  const double me = 0.51099895e-3; /* GeV */
  double bg2 = bg * bg, b2 = bg2 / (1.0 + bg2), g = sqrt(1.0 + bg2), r = me / mass;
  double tmax = 2.0 * me * bg2 / (1.0 + 2.0 * g * r + r * r);
  return K * ZA / b2 * (0.5 * log(2.0 * me * bg2 * tmax / (I * I)) - b2);
}

void orc_material_effects(const orc_cfg *cfg, int kind, double p[6], double C[36], int dir,
                          double M[36]) {
  if (M) {
    memset(M, 0, 36 * sizeof(double));
    for (int i = 0; i < 6; ++i) M[i * 6 + i] = 1.0;
  }
  const orc_material *m = cfg->material;
  if (!m) {
    orc_add_ms(p, cfg->ms_sigma, C);
    return;
  }
  double r = hypot(p[0], p[1]);
  int ir = (int)floor(r / m->r_max * m->n_r);
  int iz = (int)floor((p[2] + m->z_max) / (2.0 * m->z_max) * m->n_z);
  ir = ir < 0 ? 0 : (ir >= m->n_r ? m->n_r - 1 : ir);
  iz = iz < 0 ? 0 : (iz >= m->n_z ? m->n_z - 1 : iz);
  double t0 = m->x_x0[iz * m->n_r + ir], xi0 = m->xi[iz * m->n_r + ir];
  double st = sin(p[5]), ct = cos(p[5]);
  /* cosine of the angle between the direction and the surface normal */
  double cosa = kind == 0 ? st * (cos(p[4]) * p[0] + sin(p[4]) * p[1]) / r : ct;
  double k = fabs(cosa) * m->k_max > 1.0 ? 1.0 / fabs(cosa) : m->k_max;
  double pm = 1.0 / (fabs(p[3]) * st);
  double beta = pm / sqrt(pm * pm + m->mass * m->mass);
  double t = t0 * k;
  if (t > 0.0) {
    double f = 1.0 + 0.038 * log(t);
    if (f < 0.0) f = 0.0;
    orc_add_ms(p, 0.0136 / (beta * pm) * sqrt(t) * f, C);
  }
  double x = xi0 * k;
  if (x > 0.0) {
    double dp = x * orc_bethe_si(pm / m->mass, m->mass) / beta;
    if (dp > 0.5 * pm) dp = 0.5 * pm;
    double ratio = 1.0 / (1.0 - dir * dp / pm); /* |p| / |p'| */
    double J[36];
    memset(J, 0, sizeof(J));
    for (int i = 0; i < 6; ++i) J[i * 6 + i] = 1.0;
    J[3 * 6 + 3] = ratio * ratio;
    J[3 * 6 + 5] = dir * dp * p[3] * fabs(p[3]) * ct * ratio * ratio;
    p[3] *= ratio;
    double JC[36], Jt[36];
    matmul6(J, C, JC);
    transpose6(J, Jt);
    matmul6(JC, Jt, C);
    symmetrize6(C);
    if (M) memcpy(M, J, sizeof(J));
  }
}

/* ------------------------------------------------------- measurement */

/* Local 2-D frame at the predicted point: t = (-y', x')/r' along the
 * layer's azimuth, rh = (x', y')/r' radial.  Barrel: u = t.(xh - x'),
 * v = zh - z'.  Disk: u = t.(xh - x'), v = rh.(xh - x').  A barrel hit in
 * the opposite half of the cylinder (x'.xh <= 0) would alias to a small u,
 * so it is not compatible (reading). */
int orc_measure(const double p[6], int kind, const double hit[3], double r[2],
                double H[12]) {
  double rr = hypot(p[0], p[1]);
  double tx = -p[1] / rr, ty = p[0] / rr;
  double rx = p[0] / rr, ry = p[1] / rr;
  double dx = hit[0] - p[0], dy = hit[1] - p[1], dz = hit[2] - p[2];
  memset(H, 0, 12 * sizeof(double));
  H[0] = tx;
  H[1] = ty;
  r[0] = tx * dx + ty * dy;
  if (kind == 0) {
    if (p[0] * hit[0] + p[1] * hit[1] <= 0.0) return 0;
    r[1] = dz;
    H[6 + 2] = 1.0;
  } else {
    r[1] = rx * dx + ry * dy;
    H[6 + 0] = rx;
    H[6 + 1] = ry;
  }
  return 1;
}

static void residual_cov(const double C[36], int m, const double *H,
                         const double *V, double *S, double *PHt) {
  /* PHt = C H^T (6 x m), S = H C H^T + V (m x m) */
  for (int i = 0; i < 6; ++i)
    for (int a = 0; a < m; ++a) {
      double s = 0.0;
      for (int k = 0; k < 6; ++k) s += C[i * 6 + k] * H[a * 6 + k];
      PHt[i * m + a] = s;
    }
  for (int a = 0; a < m; ++a)
    for (int b = 0; b < m; ++b) {
      double s = V[a * m + b];
      for (int k = 0; k < 6; ++k) s += H[a * 6 + k] * PHt[k * m + b];
      S[a * m + b] = s;
    }
}

static void inv_small(int m, const double *S, double *Si) {
  if (m == 1) {
    Si[0] = 1.0 / S[0];
  } else {
    double det = S[0] * S[3] - S[1] * S[2];
    Si[0] = S[3] / det;
    Si[1] = -S[1] / det;
    Si[2] = -S[2] / det;
    Si[3] = S[0] / det;
  }
}

/* A hit measures along the layer's strip frame, turned by the stereo angle
 * a from the local (u, v) frame: w = cos(a) u + sin(a) v is measured with
 * variance var_u, the orthogonal direction with var_v (the Section 2.1
 * layer description's stereo layers; a = 0 for the others).  In (u, v):
 * V = R^T diag(var_u, var_v) R, R = [[c, s], [-s, c]]. */
static void hit_cov(double stereo, double var_u, double var_v, double V[4]) {
  double c = cos(stereo), s = sin(stereo);
  V[0] = c * c * var_u + s * s * var_v;
  V[1] = V[2] = c * s * (var_u - var_v);
  V[3] = s * s * var_u + c * c * var_v;
}

int orc_chi2(const double p[6], const double C[36], int kind,
             const double hit[3], double var_u, double var_v, double stereo, double *chi2) {
  double r[2], H[12], S[4], Si[4], PHt[12];
  if (!orc_measure(p, kind, hit, r, H)) return 0;
  double V[4];
  hit_cov(stereo, var_u, var_v, V);
  residual_cov(C, 2, H, V, S, PHt);
  inv_small(2, S, Si);
  *chi2 = r[0] * (Si[0] * r[0] + Si[1] * r[1]) + r[1] * (Si[2] * r[0] + Si[3] * r[1]);
  return 1;
}

/* ---------------------------------------------------- Kalman update */

/* Textbook gain-form Kalman update (Fruhwirth 1987, the filter the paper
 * builds on): S = H C H^T + V, K = C H^T S^-1, p += K r,
 * C -= K S K^T (= K (C H^T)^T), symmetrised; chi2 = r^T S^-1 r.
 * The Joseph form (I - KH) C (I - KH)^T + K V K^T is equal in exact
 * arithmetic and is kept as a cross-check. */
void orc_kf_update(double p[6], double C[36], int m, const double *H,
                   const double *r, const double *V, int joseph,
                   double *chi2) {
  double S[4], Si[4], PHt[12], K[12];
  residual_cov(C, m, H, V, S, PHt);
  inv_small(m, S, Si);
  for (int i = 0; i < 6; ++i)
    for (int a = 0; a < m; ++a) {
      double s = 0.0;
      for (int b = 0; b < m; ++b) s += PHt[i * m + b] * Si[b * m + a];
      K[i * m + a] = s;
    }
  double c2 = 0.0;
  for (int a = 0; a < m; ++a)
    for (int b = 0; b < m; ++b) c2 += r[a] * Si[a * m + b] * r[b];
  if (chi2) *chi2 = c2;
  for (int i = 0; i < 6; ++i)
    for (int a = 0; a < m; ++a) p[i] += K[i * m + a] * r[a];
  if (!joseph) {
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) {
        double s = 0.0;
        for (int a = 0; a < m; ++a) s += K[i * m + a] * PHt[j * m + a];
        C[i * 6 + j] -= s;
      }
  } else {
    double A[36], AC[36], At[36], Cn[36];
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) {
        double s = (i == j) ? 1.0 : 0.0;
        for (int a = 0; a < m; ++a) s -= K[i * m + a] * H[a * 6 + j];
        A[i * 6 + j] = s;
      }
    matmul6(A, C, AC);
    transpose6(A, At);
    matmul6(AC, At, Cn);
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) {
        double s = 0.0;
        for (int a = 0; a < m; ++a)
          for (int b = 0; b < m; ++b) s += K[i * m + a] * V[a * m + b] * K[j * m + b];
        Cn[i * 6 + j] += s;
      }
    memcpy(C, Cn, sizeof(Cn));
  }
  symmetrize6(C);
}

int orc_update_hit(double p[6], double C[36], int kind, const double hit[3],
                   double var_u, double var_v, double stereo, double *chi2) {
  double r[2], H[12];
  if (!orc_measure(p, kind, hit, r, H)) return 0;
  double V[4];
  hit_cov(stereo, var_u, var_v, V);
  orc_kf_update(p, C, 2, H, r, V, 0, chi2);
  p[4] = wrap_phi(p[4]);
  return 1;
}

/* ------------------------------------------------------------- priors */

/* The wide diagonal prior diag(init_var) for a state that lies on a layer:
 * less its extent along the layer's normal n at p (a state on a surface has
 * no freedom there), C = P diag(init_var) P^T with P = 1 - n n^T on the
 * position. */
static void surface_prior(const orc_cfg *cfg, const double p[6], int kind, double C[36]) {
  memset(C, 0, 36 * sizeof(double));
  for (int i = 0; i < 6; ++i) C[i * 6 + i] = cfg->init_var[i];
  double nv[3] = {0.0, 0.0, 1.0};
  if (kind == 0) {
    double r = hypot(p[0], p[1]);
    nv[0] = p[0] / r;
    nv[1] = p[1] / r;
    nv[2] = 0.0;
  }
  double P[36], T[36], Pt[36];
  memset(P, 0, sizeof(P));
  for (int i = 0; i < 6; ++i) P[i * 6 + i] = 1.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) P[i * 6 + j] -= nv[i] * nv[j];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) Pt[i * 6 + j] = P[j * 6 + i];
  matmul6(P, C, T);
  matmul6(T, Pt, C);
}

/* ------------------------------------------------------------ seeding */

static double edge_distance(const orc_layer *Lr, const double pp[6], double m) {
  double q = Lr->kind == 0 ? pp[2] : hypot(pp[0], pp[1]);
  double d = fmin(fabs(q - (Lr->ext_lo - m)), fabs(q - (Lr->ext_hi + m)));
  if (Lr->hole_hi - Lr->hole_lo > 2.0 * m)
    d = fmin(d, fmin(fabs(q - (Lr->hole_lo + m)), fabs(q - (Lr->hole_hi - m))));
  return d;
}

/* Seed from three hits (seeds are supplied from outside, Section 2.2):
 * the circle through the three transverse points gives the centre and the
 * radius rho; the turning sense gives the charge; pT = kappa |B| rho (B: a
 * parameterised field at the middle hit); phi
 * is the tangent at the first hit in the direction of motion; cot(theta)
 * is the z rise over the transverse arc from the first to the third hit.
 * The state starts at the first hit with a wide diagonal prior, less its
 * extent along the first seed layer's normal (the state lies on that layer),
 * and is filtered through the three hits (propagate, scatter, update),
 * ending on the third seed layer; chi2 sums the three updates' chi2.
 * The layer plan is the paper's per-region list of layers to traverse
 * (Section 2.1).  With region steering it is the list of the region holding
 * the seed's pseudorapidity, less the seed layers; without, it is read per
 * seed: every non-seed layer the seed helix crosses inside its widened
 * extent in the remaining half turn, ordered by path length. */
int orc_seed(const orc_cfg *cfg, const orc_layer *layers, int32_t n_layers,
             const double h[9], const double hv[6], const int32_t hl[3],
             double pos_tol, orc_seed_out *out) {
  memset(out, 0, sizeof(*out));
  double x1 = h[0], y1 = h[1], z1 = h[2];
  double x2 = h[3], y2 = h[4];
  double x3 = h[6], y3 = h[7], z3 = h[8];
  double ax = x2 - x1, ay = y2 - y1, bx = x3 - x1, by = y3 - y1;
  double d = 2.0 * (ax * by - ay * bx);
  if (d == 0.0 || cfg->bz == 0.0) return 0;
  double a2 = ax * ax + ay * ay, b2 = bx * bx + by * by;
  double ux = (by * a2 - ay * b2) / d;
  double uy = (ax * b2 - bx * a2) / d;
  double cx = x1 + ux, cy = y1 + uy;
  double rho = hypot(ux, uy);
  double turn = (x2 - x1) * (y3 - y2) - (y2 - y1) * (x3 - x2);
  int ccw = turn > 0.0; /* omega > 0 */
  /* a parameterised field is taken at the middle hit */
  double bz = cfg->field ? orc_field_bz(cfg->field, x2, y2, h[5]) : cfg->bz;
  if (bz == 0.0) return 0;
  double pt = cfg->kappa * fabs(bz) * rho;
  /* omega = -kappa B ipt > 0  <=>  B * ipt < 0 */
  double ipt = (ccw ? -1.0 : 1.0) * (bz > 0 ? 1.0 : -1.0) / pt;
  double r1x = x1 - cx, r1y = y1 - cy;
  double dirx = ccw ? -r1y : r1y, diry = ccw ? r1x : -r1x;
  double phi1 = atan2(diry, dirx);
  double r3x = x3 - cx, r3y = y3 - cy;
  double dpsi = atan2(r1x * r3y - r1y * r3x, r1x * r3x + r1y * r3y);
  double s13 = rho * fabs(dpsi);
  double theta = atan2(s13, z3 - z1);

  double p[6] = {x1, y1, z1, ipt, phi1, theta};
  double C[36];
  surface_prior(cfg, p, layers[hl[0]].kind, C);
  double chi2 = 0.0;

  for (int k = 0; k < 3; ++k) {
    const orc_layer *Lr = &layers[hl[k]];
    if (k > 0) {
      double pp[6], Cp[36];
      if (orc_propagate_f(p, C, Lr, cfg->bz, cfg->kappa, cfg->l_min, 0.0, 0, pp,
                          Cp, NULL, NULL, cfg->field) != ORC_OK)
        return 0;
      memcpy(p, pp, sizeof(pp));
      memcpy(C, Cp, sizeof(Cp));
    }
    orc_material_effects(cfg, Lr->kind, p, C, 1, NULL);
    double c2;
    if (!orc_update_hit(p, C, Lr->kind, &h[3 * k], hv[2 * k], hv[2 * k + 1], Lr->stereo, &c2))
      return 0;
    chi2 += c2;
  }
  memcpy(out->par, p, sizeof(p));
  memcpy(out->cov, C, sizeof(C));
  out->chi2 = chi2;

  int n = 0;
  if (cfg->n_regions > 0) {
    /* region steering: the region's list, less the seed layers; a layer the
     * track does not reach inside its extent becomes a skip in the find */
    double eta = -log(tan(0.5 * p[5]));
    const orc_region *R = NULL;
    for (int r = 0; r < cfg->n_regions; ++r) {
      const orc_region *g = &cfg->regions[r];
      if (fabs(eta - g->eta_lo) <= ORC_ETA_TOL || fabs(eta - g->eta_hi) <= ORC_ETA_TOL)
        out->plan_fragile = 1;
      if (R == NULL && eta >= g->eta_lo && eta < g->eta_hi) R = g;
    }
    for (int k = 0; R != NULL && k < R->n_layers && n < ORC_MAX_PLAN; ++k) {
      int i = R->layers[k];
      if (i == hl[0] || i == hl[1] || i == hl[2]) continue;
      out->plan[n++] = i;
    }
    out->plan_len = n;
    out->ok = 1;
    return 1;
  }
  for (int i = 0; i < n_layers; ++i) {
    if (i == hl[0] || i == hl[1] || i == hl[2]) continue;
    double pp[6], l;
    int st = orc_propagate_f(p, NULL, &layers[i], cfg->bz, cfg->kappa, cfg->l_min,
                             cfg->edge_margin, 1, pp, NULL, NULL, &l, cfg->field);
    if (st == ORC_NO_CROSSING) continue;
    if (st == ORC_OUT_OF_EXTENT) {
      /* near the widened edge the FP32 decision may flip */
      double p2[6];
      if (orc_propagate_f(p, NULL, &layers[i], cfg->bz, cfg->kappa, cfg->l_min, 0.0, 0, p2, NULL,
                          NULL, NULL, cfg->field) == ORC_OK &&
          edge_distance(&layers[i], p2, cfg->edge_margin) <= pos_tol)
        out->plan_fragile = 1;
      continue;
    }
    if (edge_distance(&layers[i], pp, cfg->edge_margin) <= pos_tol) out->plan_fragile = 1;
    if (n >= ORC_MAX_PLAN) break;
    /* insertion by path length, ties by layer index */
    int j = n;
    while (j > 0 && out->plan_l[j - 1] > l) {
      out->plan_l[j] = out->plan_l[j - 1];
      out->plan[j] = out->plan[j - 1];
      --j;
    }
    out->plan_l[j] = l;
    out->plan[j] = i;
    ++n;
  }
  out->plan_len = n;
  out->ok = 1;
  return 1;
}

/* ------------------------------------------------------- clone engine */

typedef struct {
  double p[6], C[36];
  int32_t n_hits, n_miss;
  double chi2;
  int32_t hist[ORC_MAX_PLAN];
} cand_t;

enum { EXT_HIT = 0, EXT_MISS = 1, EXT_SKIP = 2 };

typedef struct {
  int32_t n_hits;   /* after the extension */
  double chi2_sum;  /* after the extension */
  int32_t parent;   /* parent rank */
  int32_t order;    /* hit index; misses and skips after every hit */
  int32_t type;
  int32_t hit;
  double chi2;
} ext_t;

/* Ranking key (reading of "best extensions based on chi2", Introduction):
 * more hits first, then smaller accumulated chi2, then parent rank, then
 * hit index with miss/skip last.  Total and deterministic. */
static int ext_cmp(const void *A, const void *B) {
  const ext_t *a = (const ext_t *)A, *b = (const ext_t *)B;
  if (a->n_hits != b->n_hits) return a->n_hits > b->n_hits ? -1 : 1;
  if (a->chi2_sum != b->chi2_sum) return a->chi2_sum < b->chi2_sum ? -1 : 1;
  if (a->parent != b->parent) return a->parent < b->parent ? -1 : 1;
  if (a->order != b->order) return a->order < b->order ? -1 : 1;
  return 0;
}

static double tol_of(const orc_tol *t, double v) { return t->chi2_rel * fabs(v) + t->chi2_abs; }

static void mark(int32_t *fragile, int32_t step) {
  if (*fragile < 0 || step < *fragile) *fragile = step;
}

/* Distance of the crossing p to the nearest edge of its material bin across
 * which the thickness changes (INFINITY without a map or such an edge): there
 * the bin, and so the material, is a decision that rounding may flip. */
static double material_edge_distance(const orc_cfg *cfg, const double p[6]) {
  const orc_material *m = cfg->material;
  if (!m) return INFINITY;
  double r = hypot(p[0], p[1]);
  double fr = r / m->r_max * m->n_r, fz = (p[2] + m->z_max) / (2.0 * m->z_max) * m->n_z;
  int ir = (int)floor(fr), iz = (int)floor(fz);
  ir = ir < 0 ? 0 : (ir >= m->n_r ? m->n_r - 1 : ir);
  iz = iz < 0 ? 0 : (iz >= m->n_z ? m->n_z - 1 : iz);
  double best = INFINITY;
  /* the edges at ir, ir + 1 (radial) and iz, iz + 1 (in z) */
  for (int side = 0; side < 2; ++side) {
    int jr = ir + (side ? 1 : -1), jz = iz + (side ? 1 : -1);
    if (jr >= 0 && jr < m->n_r) {
      int a = iz * m->n_r + ir, b = iz * m->n_r + jr;
      if (m->x_x0[a] != m->x_x0[b] || m->xi[a] != m->xi[b])
        best = fmin(best, fabs(fr - (ir + side)) * m->r_max / m->n_r);
    }
    if (jz >= 0 && jz < m->n_z) {
      int a = iz * m->n_r + ir, b = jz * m->n_r + ir;
      if (m->x_x0[a] != m->x_x0[b] || m->xi[a] != m->xi[b])
        best = fmin(best, fabs(fz - (iz + side)) * 2.0 * m->z_max / m->n_z);
    }
  }
  return best;
}

/* Candidate histories at one step of a seed's find (orc_find_prefixes). */
typedef struct {
  int32_t step, cap, n;
  int32_t *hist; /* [cap][ORC_MAX_PLAN] */
} snap_t;

static void snap_add(snap_t *sn, const cand_t *c) {
  if (sn->n < sn->cap) memcpy(&sn->hist[(size_t)sn->n * ORC_MAX_PLAN], c->hist, sizeof(c->hist));
  sn->n++;
}

static void find_one(const orc_cfg *cfg, const orc_tol *tol, const orc_layer *layers,
                     int32_t n_layers, const int32_t *lay_off, const int32_t *lay_idx,
                     const float *x, const float *y, const float *z, const float *vu,
                     const float *vv, const int32_t *layer, const int32_t *sh,
                     orc_track *out, snap_t *snap) {
  memset(out, 0, sizeof(*out));
  out->fragile_step = -1;
  double h[9], hv[6];
  int32_t hl[3];
  for (int k = 0; k < 3; ++k) {
    int32_t i = sh[k];
    h[3 * k] = x[i];
    h[3 * k + 1] = y[i];
    h[3 * k + 2] = z[i];
    hv[2 * k] = vu[i];
    hv[2 * k + 1] = vv[i];
    hl[k] = layer[i];
  }
  orc_seed_out so;
  if (!orc_seed(cfg, layers, n_layers, h, hv, hl, tol->pos_tol, &so)) return;
  out->seed_ok = 1;
  out->plan_len = so.plan_len;
  memcpy(out->plan, so.plan, sizeof(so.plan));
  if (so.plan_fragile) {
    out->fragile_step = 0;
    out->plan_fragile = 1;
  }

  int nc = cfg->n_cand;
  cand_t *cands = (cand_t *)calloc((size_t)nc, sizeof(cand_t));
  cand_t *next = (cand_t *)calloc((size_t)nc, sizeof(cand_t));
  cand_t *fin = (cand_t *)calloc((size_t)(ORC_MAX_PLAN + 1) * nc, sizeof(cand_t));
  double *pp = (double *)malloc(sizeof(double) * 6 * nc);
  double *Cp = (double *)malloc(sizeof(double) * 36 * nc);
  int n_fin = 0;
  int n = 1;
  memcpy(cands[0].p, so.par, sizeof(so.par));
  memcpy(cands[0].C, so.cov, sizeof(so.cov));
  cands[0].n_hits = 3;
  cands[0].n_miss = 0;
  cands[0].chi2 = 0.0;
  for (int k = 0; k < ORC_MAX_PLAN; ++k) cands[0].hist[k] = ORC_HIT_NONE;

  for (int s = 0; s < so.plan_len; ++s) {
    if (snap && snap->step == s) {
      for (int c = 0; c < n; ++c) snap_add(snap, &cands[c]);
      for (int c = 0; c < n_fin; ++c) snap_add(snap, &fin[c]);
    }
    const orc_layer *Lr = &layers[so.plan[s]];
    int32_t L = so.plan[s];
    int32_t nh = lay_off[L + 1] - lay_off[L];
    ext_t *ext = (ext_t *)malloc(sizeof(ext_t) * (size_t)n * (size_t)(nh + 1));
    int ne = 0;
    out->n_steps += n;
    for (int c = 0; c < n; ++c) {
      int ne0 = ne;
      double *pc = &pp[6 * c], *Cc = &Cp[36 * c];
      double l;
      int st = orc_propagate_f(cands[c].p, cands[c].C, Lr, cfg->bz, cfg->kappa, cfg->l_min,
                               cfg->edge_margin, 1, pc, Cc, NULL, &l, cfg->field);
      if (st == ORC_OK && edge_distance(Lr, pc, cfg->edge_margin) <= tol->pos_tol) mark(&out->fragile_step, s);
      if (st == ORC_OUT_OF_EXTENT) {
        double p2[6];
        if (orc_propagate_f(cands[c].p, NULL, Lr, cfg->bz, cfg->kappa, cfg->l_min, 0.0, 0, p2,
                            NULL, NULL, NULL, cfg->field) == ORC_OK &&
            edge_distance(Lr, p2, cfg->edge_margin) <= tol->pos_tol)
          mark(&out->fragile_step, s);
      }
      if (st != ORC_OK) {
        ext_t e = {cands[c].n_hits, cands[c].chi2, c, 0x7fffffff, EXT_SKIP, ORC_HIT_SKIP, 0.0};
        ext[ne++] = e;
        continue;
      }
      if (material_edge_distance(cfg, pc) <= tol->pos_tol) mark(&out->fragile_step, s);
      orc_material_effects(cfg, Lr->kind, pc, Cc, 1, NULL);
      for (int k = lay_off[L]; k < lay_off[L + 1]; ++k) {
        int32_t hi = lay_idx[k];
        double hh[3] = {x[hi], y[hi], z[hi]};
        double c2;
        if (!orc_chi2(pc, Cc, Lr->kind, hh, vu[hi], vv[hi], Lr->stereo, &c2)) continue;
        if (fabs(c2 - cfg->chi2_cut) <= tol_of(tol, cfg->chi2_cut)) mark(&out->fragile_step, s);
        if (c2 < cfg->chi2_cut) {
          ext_t e = {cands[c].n_hits + 1, cands[c].chi2 + c2, c, hi, EXT_HIT, hi, c2};
          ext[ne++] = e;
        }
      }
      if (cands[c].n_miss < cfg->max_holes) {
        ext_t e = {cands[c].n_hits, cands[c].chi2, c, 0x7fffffff, EXT_MISS, ORC_HIT_MISS, 0.0};
        ext[ne++] = e;
      }
      if (ne == ne0) fin[n_fin++] = cands[c]; /* no extension: retired */
    }
    qsort(ext, (size_t)ne, sizeof(ext_t), ext_cmp);
    int keep = ne < nc ? ne : nc;
    if (ne > nc && ext[nc - 1].n_hits == ext[nc].n_hits &&
        fabs(ext[nc - 1].chi2_sum - ext[nc].chi2_sum) <=
            tol_of(tol, fmax(ext[nc - 1].chi2_sum, ext[nc].chi2_sum)))
      mark(&out->fragile_step, s);
    for (int r = 0; r < keep; ++r) {
      const ext_t *e = &ext[r];
      cand_t *dst = &next[r];
      const cand_t *par = &cands[e->parent];
      *dst = *par;
      if (e->type == EXT_SKIP) {
        dst->hist[s] = ORC_HIT_SKIP;
      } else {
        memcpy(dst->p, &pp[6 * e->parent], 6 * sizeof(double));
        memcpy(dst->C, &Cp[36 * e->parent], 36 * sizeof(double));
        if (e->type == EXT_MISS) {
          dst->n_miss += 1;
          dst->hist[s] = ORC_HIT_MISS;
        } else {
          double hh[3] = {x[e->hit], y[e->hit], z[e->hit]};
          double c2;
          orc_update_hit(dst->p, dst->C, Lr->kind, hh, vu[e->hit], vv[e->hit], Lr->stereo, &c2);
          dst->n_hits += 1;
          dst->chi2 = e->chi2_sum;
          dst->hist[s] = e->hit;
        }
      }
    }
    free(ext);
    cand_t *tmp = cands;
    cands = next;
    next = tmp;
    n = keep;
  }

  if (snap && snap->step >= so.plan_len) {
    for (int c = 0; c < n; ++c) snap_add(snap, &cands[c]);
    for (int c = 0; c < n_fin; ++c) snap_add(snap, &fin[c]);
  }
  /* best over final candidates (by rank) then retired ones (in order) */
  const cand_t *bc = NULL, *sc = NULL;
  for (int i = 0; i < n + n_fin; ++i) {
    const cand_t *c = i < n ? &cands[i] : &fin[i - n];
    if (!bc || c->n_hits > bc->n_hits || (c->n_hits == bc->n_hits && c->chi2 < bc->chi2)) {
      sc = bc;
      bc = c;
    } else if (!sc || c->n_hits > sc->n_hits || (c->n_hits == sc->n_hits && c->chi2 < sc->chi2)) {
      sc = c;
    }
  }
  if (bc) {
    if (sc && sc->n_hits == bc->n_hits && fabs(sc->chi2 - bc->chi2) <= tol_of(tol, fmax(sc->chi2, bc->chi2)))
      mark(&out->fragile_step, so.plan_len);
    out->n_hits = bc->n_hits;
    out->n_miss = bc->n_miss;
    out->chi2 = bc->chi2;
    memcpy(out->par, bc->p, sizeof(bc->p));
    memcpy(out->cov, bc->C, sizeof(bc->C));
    memcpy(out->hit, bc->hist, sizeof(bc->hist));
  }
  free(cands);
  free(next);
  free(fin);
  free(pp);
  free(Cp);
}

/* Hits of each layer in original order (the brute-force scans visit every
 * hit of a layer): *off [n_layers + 1], *idx [n_hits].  -1 for a bad layer. */
static int layer_lists(int32_t n_layers, int32_t n_hits, const int32_t *layer, int32_t **off_out,
                       int32_t **idx_out) {
  int32_t *off = (int32_t *)calloc((size_t)n_layers + 1, sizeof(int32_t));
  int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_hits > 0 ? n_hits : 1));
  for (int32_t i = 0; i < n_hits; ++i) {
    if (layer[i] < 0 || layer[i] >= n_layers) {
      free(off);
      free(idx);
      return -1;
    }
    off[layer[i] + 1]++;
  }
  for (int32_t L = 0; L < n_layers; ++L) off[L + 1] += off[L];
  int32_t *fill = (int32_t *)calloc((size_t)n_layers, sizeof(int32_t));
  for (int32_t i = 0; i < n_hits; ++i) idx[off[layer[i]] + fill[layer[i]]++] = i;
  free(fill);
  *off_out = off;
  *idx_out = idx;
  return 0;
}

int orc_find_event(const orc_cfg *cfg, const orc_tol *tol, const orc_layer *layers,
                   int32_t n_layers, int32_t n_hits, const float *x, const float *y,
                   const float *z, const float *var_u, const float *var_v,
                   const int32_t *layer, int32_t n_seeds, const int32_t *seed_hits,
                   orc_track *out) {
  if (cfg->n_cand < 1) return -1;
  int32_t *off, *idx;
  if (layer_lists(n_layers, n_hits, layer, &off, &idx)) return -1;
  for (int32_t s = 0; s < n_seeds; ++s)
    find_one(cfg, tol, layers, n_layers, off, idx, x, y, z, var_u, var_v, layer,
             &seed_hits[3 * s], &out[s], NULL);
  free(off);
  free(idx);
  return 0;
}

int32_t orc_find_prefixes(const orc_cfg *cfg, const orc_tol *tol, const orc_layer *layers,
                          int32_t n_layers, int32_t n_hits, const float *x, const float *y,
                          const float *z, const float *var_u, const float *var_v,
                          const int32_t *layer, const int32_t seed_hits[3], int32_t step,
                          int32_t cap, int32_t *hist) {
  if (cfg->n_cand < 1 || step < 0 || cap < 0) return -1;
  int32_t *off, *idx;
  if (layer_lists(n_layers, n_hits, layer, &off, &idx)) return -1;
  snap_t sn = {step, cap, 0, hist};
  orc_track t;
  find_one(cfg, tol, layers, n_layers, off, idx, x, y, z, var_u, var_v, layer, seed_hits, &t,
           &sn);
  free(off);
  free(idx);
  return sn.n;
}

/* Whether some hit of layer L is clearly compatible with the predicted
 * state (chi2 below cut - tol); *near_cut is set if one lies within tol of
 * the cut. */
static int any_compatible(const orc_cfg *cfg, const orc_tol *tol, const orc_layer *Lr,
                          const int32_t *lay_off, const int32_t *lay_idx, int32_t L,
                          const double pc[6], const double Cc[36], const float *x,
                          const float *y, const float *z, const float *vu, const float *vv,
                          int *near_cut) {
  int any = 0;
  for (int k = lay_off[L]; k < lay_off[L + 1]; ++k) {
    int32_t hi = lay_idx[k];
    double hh[3] = {x[hi], y[hi], z[hi]}, c2;
    if (!orc_chi2(pc, Cc, Lr->kind, hh, vu[hi], vv[hi], Lr->stereo, &c2)) continue;
    if (fabs(c2 - cfg->chi2_cut) <= tol_of(tol, cfg->chi2_cut)) *near_cut = 1;
    else if (c2 < cfg->chi2_cut) any = 1;
  }
  return any;
}

int orc_follow_path(const orc_cfg *cfg, const orc_tol *tol, const orc_layer *layers,
                    int32_t n_layers, int32_t n_hits, const float *x, const float *y,
                    const float *z, const float *var_u, const float *var_v,
                    const int32_t *layer, const int32_t seed_hits[3], int32_t plan_len,
                    const int32_t *plan, const int32_t *hist, orc_path *out) {
  memset(out, 0, sizeof(*out));
  out->bad_step = -1;
  double h[9], hv[6];
  int32_t hl[3];
  for (int k = 0; k < 3; ++k) {
    int32_t i = seed_hits[k];
    if (i < 0 || i >= n_hits) return -1;
    h[3 * k] = x[i];
    h[3 * k + 1] = y[i];
    h[3 * k + 2] = z[i];
    hv[2 * k] = var_u[i];
    hv[2 * k + 1] = var_v[i];
    hl[k] = layer[i];
  }
  orc_seed_out so;
  if (!orc_seed(cfg, layers, n_layers, h, hv, hl, tol->pos_tol, &so)) return -1;
  if (so.plan_len != plan_len) return -1;
  for (int s = 0; s < plan_len; ++s)
    if (so.plan[s] != plan[s]) return -1;
  int32_t *off, *idx;
  if (layer_lists(n_layers, n_hits, layer, &off, &idx)) return -1;
  double p[6], C[36];
  memcpy(p, so.par, sizeof(p));
  memcpy(C, so.cov, sizeof(C));
  int32_t nh = 3, nm = 0, retired = 0;
  double chi = 0.0;
#define FOLLOW_BAD(s_)       \
  do {                       \
    out->bad_step = (s_);    \
    goto done;               \
  } while (0)
  for (int s = 0; s < plan_len; ++s) {
    const orc_layer *Lr = &layers[plan[s]];
    int32_t L = plan[s], e = hist[s];
    if (retired) {
      if (e != ORC_HIT_NONE) FOLLOW_BAD(s);
      continue;
    }
    double pc[6], Cc[36];
    int st = orc_propagate_f(p, C, Lr, cfg->bz, cfg->kappa, cfg->l_min, cfg->edge_margin, 1, pc,
                             Cc, NULL, NULL, cfg->field);
    double p2[6];
    int near_edge =
        (st == ORC_OK && edge_distance(Lr, pc, cfg->edge_margin) <= tol->pos_tol) ||
        (st == ORC_OUT_OF_EXTENT &&
         orc_propagate_f(p, NULL, Lr, cfg->bz, cfg->kappa, cfg->l_min, 0.0, 0, p2, NULL, NULL,
                         NULL, cfg->field) == ORC_OK &&
         edge_distance(Lr, p2, cfg->edge_margin) <= tol->pos_tol);
    out->n_edge += near_edge;
    if (e == ORC_HIT_SKIP) {
      if (st == ORC_OK && !near_edge) FOLLOW_BAD(s);
      continue; /* the state stays where it was */
    }
    if (st != ORC_OK) {
      if (!near_edge) FOLLOW_BAD(s);
      /* a crossing within tolerance of an edge that the other side took
       * as inside: continue from the unwidened crossing */
      if (orc_propagate_f(p, C, Lr, cfg->bz, cfg->kappa, cfg->l_min, 0.0, 0, pc, Cc, NULL, NULL,
                          cfg->field) != ORC_OK)
        FOLLOW_BAD(s);
    }
    if (material_edge_distance(cfg, pc) <= tol->pos_tol) out->n_edge++;
    orc_material_effects(cfg, Lr->kind, pc, Cc, 1, NULL);
    int near_cut = 0;
    if (e == ORC_HIT_NONE) {
      /* retired here: nothing was compatible and no miss was left */
      if (nm < cfg->max_holes) FOLLOW_BAD(s);
      if (any_compatible(cfg, tol, Lr, off, idx, L, pc, Cc, x, y, z, var_u, var_v, &near_cut))
        FOLLOW_BAD(s);
      out->n_near_cut += near_cut;
      retired = 1;
      continue;
    }
    if (e == ORC_HIT_MISS) {
      if (nm >= cfg->max_holes) FOLLOW_BAD(s);
      nm += 1;
      memcpy(p, pc, sizeof(p));
      memcpy(C, Cc, sizeof(C));
      continue;
    }
    if (e < 0 || e >= n_hits || layer[e] != L) FOLLOW_BAD(s);
    double hh[3] = {x[e], y[e], z[e]}, c2;
    if (!orc_chi2(pc, Cc, Lr->kind, hh, var_u[e], var_v[e], Lr->stereo, &c2)) FOLLOW_BAD(s);
    if (c2 >= cfg->chi2_cut + tol_of(tol, cfg->chi2_cut)) FOLLOW_BAD(s);
    if (c2 >= cfg->chi2_cut) out->n_near_cut++;
    out->max_chi2 = fmax(out->max_chi2, c2);
    double c2u; /* the update's own chi2 (the find sums the test's, c2) */
    orc_update_hit(pc, Cc, Lr->kind, hh, var_u[e], var_v[e], Lr->stereo, &c2u);
    memcpy(p, pc, sizeof(p));
    memcpy(C, Cc, sizeof(C));
    nh += 1;
    chi += c2;
  }
#undef FOLLOW_BAD
done:
  out->n_hits = nh;
  out->n_miss = nm;
  out->chi2 = chi;
  memcpy(out->par, p, sizeof(p));
  memcpy(out->cov, C, sizeof(C));
  free(off);
  free(idx);
  return out->bad_step < 0 ? 0 : 1;
}

/* ------------------------------------------------------------- fitting */

/* Kalman fit through a known hit sequence (the paper's vectorized fitting,
 * Introduction): for every hit, propagate to its surface, add the
 * scattering noise, update. */
int orc_fit_track(const orc_cfg *cfg, const double p0[6], const double C0[36], int32_t n,
                  const int32_t *kinds, const double *pos, const double *hits,
                  const double *var_u, const double *var_v, double p_out[6],
                  double C_out[36], double *chi2_sum) {
  double p[6], C[36];
  memcpy(p, p0, sizeof(p));
  memcpy(C, C0, sizeof(C));
  double sum = 0.0;
  for (int32_t k = 0; k < n; ++k) {
    orc_layer Lr = {kinds[k], pos[k], 0.0, 0.0};
    double pp[6], Cp[36];
    if (orc_propagate_f(p, C, &Lr, cfg->bz, cfg->kappa, cfg->l_min, 0.0, 0, pp, Cp, NULL, NULL,
                        cfg->field) != ORC_OK)
      return -(k + 1);
    orc_material_effects(cfg, kinds[k], pp, Cp, 1, NULL);
    double c2;
    if (!orc_update_hit(pp, Cp, kinds[k], &hits[3 * k], var_u[k], var_v[k], 0.0, &c2))
      return -(k + 1);
    sum += c2;
    memcpy(p, pp, sizeof(p));
    memcpy(C, Cp, sizeof(C));
  }
  memcpy(p_out, p, sizeof(p));
  memcpy(C_out, C, sizeof(C));
  *chi2_sum = sum;
  return 0;
}

/* ------------------------------------------------------- backward fit */

/* The same helix run the other way: the track of the opposite charge
 * moving in the opposite direction, q/pT -> -q/pT, phi -> phi + pi,
 * theta -> pi - theta.  The map is linear in the parameters it changes, so
 * the covariance becomes D C D with D = diag(1, 1, 1, -1, 1, -1). */
void orc_flip(double p[6], double C[36]) {
  p[3] = -p[3];
  p[4] = wrap_phi(p[4] + M_PI);
  p[5] = M_PI - p[5];
  if (!C) return;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      int si = (i == 3 || i == 5), sj = (j == 3 || j == 5);
      if (si != sj) C[i * 6 + j] = -C[i * 6 + j];
    }
}

/* Backward fit of a found track (the layer plan's flags for layers used
 * only when fitting backwards, Section 2.1; the Kalman filter of the
 * Introduction run in the reverse order).  Reading: the surfaces are the
 * crossed plan layers (hit or miss) from the last to the first, then the
 * three seed layers from the third to the first; the filter starts at the
 * first of them from the track's final state with the seed fit's prior on
 * that surface, and runs the seed fit's loop over them: propagate (from
 * the second surface on, on the reversed helix, without extent test), add
 * the layer's scattering, update with the surface's hit if it has one.
 * Returns 1 with the state on the first seed layer, 0 for a track whose
 * seed fit failed, -k when propagation to (or the update on) the k-th
 * surface failed. */
int orc_backward_fit(const orc_cfg *cfg, const orc_layer *layers, int32_t n_layers,
                     const float *x, const float *y, const float *z, const float *var_u,
                     const float *var_v, const int32_t *layer, const int32_t seed_hits[3],
                     const orc_track *trk, double p_out[6], double C_out[36], double *chi2_sum,
                     int32_t *n_updates) {
  memset(p_out, 0, 6 * sizeof(double));
  memset(C_out, 0, 36 * sizeof(double));
  *chi2_sum = 0.0;
  *n_updates = 0;
  if (!trk->seed_ok) return 0;
  int32_t lay[ORC_MAX_PLAN + 3], hit[ORC_MAX_PLAN + 3];
  int n = 0;
  for (int s = trk->plan_len - 1; s >= 0; --s) {
    if (trk->hit[s] < ORC_HIT_MISS) continue; /* not crossed, or after the end */
    lay[n] = trk->plan[s];
    hit[n] = trk->hit[s];
    ++n;
  }
  for (int j = 2; j >= 0; --j) {
    lay[n] = layer[seed_hits[j]];
    hit[n] = seed_hits[j];
    ++n;
  }
  double p[6], C[36], sum = 0.0;
  memcpy(p, trk->par, sizeof(p));
  if (lay[0] < 0 || lay[0] >= n_layers) return -1;
  surface_prior(cfg, p, layers[lay[0]].kind, C);
  int nu = 0;
  for (int k = 0; k < n; ++k) {
    if (lay[k] < 0 || lay[k] >= n_layers) return -(k + 1);
    const orc_layer *Lr = &layers[lay[k]];
    if (k > 0) {
      double pp[6], Cp[36];
      orc_flip(p, C);
      if (orc_propagate_f(p, C, Lr, cfg->bz, cfg->kappa, cfg->l_min, 0.0, 0, pp, Cp, NULL, NULL,
                          cfg->field) != ORC_OK)
        return -(k + 1);
      orc_flip(pp, Cp);
      memcpy(p, pp, sizeof(pp));
      memcpy(C, Cp, sizeof(Cp));
    }
    orc_material_effects(cfg, Lr->kind, p, C, -1, NULL);
    if (hit[k] >= 0) {
      const double h[3] = {x[hit[k]], y[hit[k]], z[hit[k]]};
      double c2;
      if (!orc_update_hit(p, C, Lr->kind, h, var_u[hit[k]], var_v[hit[k]], Lr->stereo, &c2))
        return -(k + 1);
      sum += c2;
      ++nu;
    }
  }
  memcpy(p_out, p, sizeof(p));
  memcpy(C_out, C, sizeof(C));
  *chi2_sum = sum;
  *n_updates = nu;
  return 1;
}

/* ---------------------------------------------------------- smoothing */

/* Inverse of a general n x n matrix by Gauss-Jordan elimination with
 * partial pivoting; 0 if singular. */
static int inv_gauss(int n, const double *A, double *Ai) {
  double M[6][12];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      M[i][j] = A[i * n + j];
      M[i][n + j] = i == j ? 1.0 : 0.0;
    }
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (fabs(M[r][c]) > fabs(M[piv][c])) piv = r;
    if (M[piv][c] == 0.0) return 0;
    if (piv != c)
      for (int j = 0; j < 2 * n; ++j) {
        double t = M[c][j];
        M[c][j] = M[piv][j];
        M[piv][j] = t;
      }
    double d = M[c][c];
    for (int j = 0; j < 2 * n; ++j) M[c][j] /= d;
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = M[r][c];
      for (int j = 0; j < 2 * n; ++j) M[r][j] -= f * M[c][j];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Ai[i * n + j] = M[i][n + j];
  return 1;
}

/* Rauch-Tung-Striebel smoothing of a found track (the second half of the
 * backward pass the layer plan's steering provides for, Section 2.1; the
 * filter is the Kalman filter of the Introduction).  Surfaces: the seed's
 * third layer, where the find starts from the seed fit's state, then the
 * plan layers the track crossed (hit or miss), in plan order.  Forward:
 * the find's filter along the track (propagate, add the layer's
 * scattering, update with the hit if there is one), keeping on every
 * surface the filtered state x(k), C(k), the predicted state xp(k), Cp(k)
 * after scattering and the transport Jacobian F(k) from the previous
 * surface.  Backward, from the last surface where the smoothed state is
 * the filtered one:
 *   A = C(k) F(k+1)^T Cp(k+1)^-1,
 *   xs(k) = x(k) + A (xs(k+1) - xp(k+1)),
 *   Cs(k) = C(k) + A (Cs(k+1) - Cp(k+1)) A^T.
 * Cp(k+1) has no extent along the normal n of its surface and every vector
 * it is applied to lies in the surface, so its inverse is taken as that of
 * Cp + s n n^T (s: the largest position variance), which is the same there.
 * Outputs (up to ORC_MAX_PLAN + 1 surfaces): the layer id of each surface,
 * the smoothed states [k][6] and covariances [k][36].  Returns the number
 * of surfaces, 0 for a track whose seed fit failed, -1 on a failed
 * propagation or update, -2 on a singular predicted covariance. */
int orc_smooth_track(const orc_cfg *cfg, const orc_layer *layers, int32_t n_layers,
                     const float *x, const float *y, const float *z, const float *var_u,
                     const float *var_v, int32_t seed_layer, const double seed_par[6],
                     const double seed_cov[36], const orc_track *trk, int32_t *surf_layer,
                     double *par_out, double *cov_out) {
  if (!trk->seed_ok) return 0;
  enum { NS = ORC_MAX_PLAN + 1 };
  double xf[NS][6], Cf[NS][36], xp[NS][6], Cpr[NS][36], F[NS][36];
  int n = 1;
  memcpy(xf[0], seed_par, sizeof(xf[0]));
  memcpy(Cf[0], seed_cov, sizeof(Cf[0]));
  surf_layer[0] = seed_layer;
  for (int s = 0; s < trk->plan_len; ++s) {
    int code = trk->hit[s];
    if (code < ORC_HIT_MISS) continue;
    int L = trk->plan[s];
    if (L < 0 || L >= n_layers) return -1;
    const orc_layer *Lr = &layers[L];
    double pp[6], Cp[36];
    if (orc_propagate_f(xf[n - 1], Cf[n - 1], Lr, cfg->bz, cfg->kappa, cfg->l_min, 0.0, 0, pp,
                        Cp, F[n], NULL, cfg->field) != ORC_OK)
      return -1;
    double Mm[36], MF[36];
    orc_material_effects(cfg, Lr->kind, pp, Cp, 1, Mm);
    matmul6(Mm, F[n], MF);
    memcpy(F[n], MF, sizeof(MF));
    memcpy(xp[n], pp, sizeof(pp));
    memcpy(Cpr[n], Cp, sizeof(Cp));
    if (code >= 0) {
      const double h[3] = {x[code], y[code], z[code]};
      double c2;
      if (!orc_update_hit(pp, Cp, Lr->kind, h, var_u[code], var_v[code], Lr->stereo, &c2))
        return -1;
    }
    memcpy(xf[n], pp, sizeof(pp));
    memcpy(Cf[n], Cp, sizeof(Cp));
    surf_layer[n] = L;
    ++n;
  }
  memcpy(&par_out[6 * (n - 1)], xf[n - 1], sizeof(xf[0]));
  memcpy(&cov_out[36 * (n - 1)], Cf[n - 1], sizeof(Cf[0]));
  for (int k = n - 2; k >= 0; --k) {
    const double *xs1 = &par_out[6 * (k + 1)], *Cs1 = &cov_out[36 * (k + 1)];
    /* the predicted covariance on surface k+1, made invertible along n */
    double nv[3] = {0.0, 0.0, 1.0};
    if (layers[surf_layer[k + 1]].kind == 0) {
      double r = hypot(xp[k + 1][0], xp[k + 1][1]);
      nv[0] = xp[k + 1][0] / r;
      nv[1] = xp[k + 1][1] / r;
      nv[2] = 0.0;
    }
    double S[36], Si[36];
    memcpy(S, Cpr[k + 1], sizeof(S));
    double sc = fmax(S[0], fmax(S[7], S[14]));
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) S[i * 6 + j] += sc * nv[i] * nv[j];
    if (!inv_gauss(6, S, Si)) return -2;
    /* A = C(k) F^T S^-1 */
    double Ft[36], CFt[36], A[36];
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) Ft[i * 6 + j] = F[k + 1][j * 6 + i];
    matmul6(Cf[k], Ft, CFt);
    matmul6(CFt, Si, A);
    double d[6];
    for (int i = 0; i < 6; ++i) d[i] = xs1[i] - xp[k + 1][i];
    d[4] = wrap_phi(d[4]);
    double *xs = &par_out[6 * k], *Cs = &cov_out[36 * k];
    for (int i = 0; i < 6; ++i) {
      double a = xf[k][i];
      for (int j = 0; j < 6; ++j) a += A[i * 6 + j] * d[j];
      xs[i] = a;
    }
    xs[4] = wrap_phi(xs[4]);
    double D[36], AD[36], At[36], ADAt[36];
    for (int i = 0; i < 36; ++i) D[i] = Cs1[i] - Cpr[k + 1][i];
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) At[i * 6 + j] = A[j * 6 + i];
    matmul6(A, D, AD);
    matmul6(AD, At, ADAt);
    for (int i = 0; i < 36; ++i) Cs[i] = Cf[k][i] + ADAt[i];
  }
  return n;
}

/* --------------------------------------------------- triplet seeding */

/* Seeds are supplied from outside in the paper (Section 2.2); building them
 * from the hits is the step the paper leaves to the host framework.
 * Reading: a seed is a triplet of hits on three barrel layers (innermost
 * first) whose helix is a plausible track from the beam line.  The circle
 * through the three transverse points gives the centre c and the radius rho;
 * the triplet passes if
 *   pT = kappa |B| rho >= pt_min,
 *   d0 = | |c| - rho | <= d0_max        (transverse distance to the beam line),
 *   the hits follow each other along the circle in the turning sense within
 *   half a turn (0 < psi_ab < psi_ac < pi),
 *   |z_b - (z_a + (z_c - z_a) s_ab / s_ac)| <= dz_max   (s: arc lengths),
 *   the point of closest approach to the beam line precedes a within half a
 *   turn, and there |z0| <= z0_max, z0 = z_a - (z_c - z_a) s_0a / s_ac.
 * Writes the cut variables (pt, d0, dz, z0, psi_ab, psi_ac, psi_0a) to v
 * (may be NULL) and, in *margin, the smallest distance of a variable to its
 * cut relative to the cut's scale (angles relative to pi); when pT or d0
 * misses its cut by more than half of it only those two are computed (the
 * others are NaN in v).  Returns 1 if the triplet passes. */
int orc_triplet_params(const orc_cfg *cfg, const orc_seeding *sc, const double a[3],
                       const double b[3], const double c[3], double v[7], double *margin) {
  *margin = 0.0;
  double abx = b[0] - a[0], aby = b[1] - a[1], acx = c[0] - a[0], acy = c[1] - a[1];
  double cr = abx * acy - aby * acx;
  if (cr == 0.0) return 0; /* collinear: no circle */
  double ab2 = abx * abx + aby * aby, ac2 = acx * acx + acy * acy;
  /* centre relative to a: solves 2 u.ab = |ab|^2, 2 u.ac = |ac|^2 */
  double ux = (acy * ab2 - aby * ac2) / (2.0 * cr);
  double uy = (abx * ac2 - acx * ab2) / (2.0 * cr);
  double cx = a[0] + ux, cy = a[1] + uy;
  double rho = hypot(ux, uy);
  double pt = cfg->kappa * fabs(cfg->bz) * rho;
  double D = hypot(cx, cy);
  if (D == 0.0) return 0;
  double d0 = fabs(D - rho);
  {
    /* far from the pT or d0 cut: fails whatever the rest (saves the
     * arctangents of most combinations in the brute force) */
    double m_pt = (pt - sc->pt_min) / sc->pt_min, m_d0 = (sc->d0_max - d0) / sc->d0_max;
    if (m_pt < -0.5 || m_d0 < -0.5) {
      *margin = fmin(m_pt, m_d0);
      if (v)
        for (int i = 0; i < 7; ++i) v[i] = i == 0 ? pt : (i == 1 ? d0 : NAN);
      return 0;
    }
  }
  double sgn = cr > 0.0 ? 1.0 : -1.0; /* turning sense of a -> b -> c */
  double pa = atan2(a[1] - cy, a[0] - cx), pb = atan2(b[1] - cy, b[0] - cx);
  double pc = atan2(c[1] - cy, c[0] - cx), p0 = atan2(-cy, -cx);
  double psi_ab = fmod(sgn * (pb - pa) + 4.0 * M_PI, 2.0 * M_PI);
  double psi_ac = fmod(sgn * (pc - pa) + 4.0 * M_PI, 2.0 * M_PI);
  double psi_0a = fmod(sgn * (pa - p0) + 4.0 * M_PI, 2.0 * M_PI);
  double s_ab = rho * psi_ab, s_ac = rho * psi_ac, s_0a = rho * psi_0a;
  double slope = s_ac > 0.0 ? (c[2] - a[2]) / s_ac : 0.0;
  double dz = b[2] - (a[2] + slope * s_ab);
  double z0 = a[2] - slope * s_0a;
  if (v) {
    v[0] = pt;
    v[1] = d0;
    v[2] = dz;
    v[3] = z0;
    v[4] = psi_ab;
    v[5] = psi_ac;
    v[6] = psi_0a;
  }
  double m[7] = {(pt - sc->pt_min) / sc->pt_min, (sc->d0_max - d0) / sc->d0_max,
                 (sc->dz_max - fabs(dz)) / sc->dz_max, (sc->z0_max - fabs(z0)) / sc->z0_max,
                 psi_ab / M_PI, (psi_ac - psi_ab) / M_PI, (M_PI - psi_ac) / M_PI};
  double mn = m[0];
  for (int i = 1; i < 7; ++i) mn = fmin(mn, m[i]);
  mn = fmin(mn, (M_PI - psi_0a) / M_PI);
  *margin = mn;
  return mn > 0.0;
}

/* All triplets of one event that pass (brute force over every hit of the
 * three seeding layers, a in the caller's order, then b, then c; only those
 * starting at hit a_only if a_only >= 0).  Writes up
 * to cap triplets (event-local hit indices, innermost first) and, for each,
 * fragile = 1 if a cut variable lies within frag_tol (relative) of its cut;
 * triplets that fail by less than frag_tol are counted in *n_fragile_out.
 * Returns the number that pass. */
int64_t orc_triplet_seeds(const orc_cfg *cfg, const orc_seeding *sc, int32_t n_hits,
                          const float *x, const float *y, const float *z, const int32_t *layer,
                          int32_t a_only, double frag_tol, int64_t cap, int32_t *out,
                          int32_t *fragile, int64_t *n_fragile_out) {
  int64_t n = 0, nf = 0;
  for (int32_t i = 0; i < n_hits; ++i) {
    if (layer[i] != sc->layer[0] || (a_only >= 0 && i != a_only)) continue;
    const double a[3] = {x[i], y[i], z[i]};
    for (int32_t j = 0; j < n_hits; ++j) {
      if (layer[j] != sc->layer[1]) continue;
      const double b[3] = {x[j], y[j], z[j]};
      for (int32_t k = 0; k < n_hits; ++k) {
        if (layer[k] != sc->layer[2]) continue;
        const double c[3] = {x[k], y[k], z[k]};
        double margin;
        int ok = orc_triplet_params(cfg, sc, a, b, c, NULL, &margin);
        if (!ok) {
          if (margin > -frag_tol && margin != 0.0) ++nf;
          continue;
        }
        if (n < cap) {
          out[3 * n] = i;
          out[3 * n + 1] = j;
          out[3 * n + 2] = k;
          fragile[n] = margin < frag_tol;
        }
        ++n;
      }
    }
  }
  *n_fragile_out = nf;
  return n;
}

/* -------------------------------------------------- duplicate removal */

/* Removal of duplicate tracks, which the paper lists as not yet done
 * (Introduction; Section 3: duplicates from several seeds per particle).
 * Reading: the hits of a track are its three seed hits and its found hits.
 * Track u ranks before track t if it has more hits; with as many, a smaller
 * chi2; with the same chi2, a lexicographically smaller seed triplet.  t is a
 * duplicate if some track ranking before it shares at least frac of the
 * hits of the shorter of the two.  hits: n x stride event-local indices
 * (n_hits[t] used), seed: n x 3.  dup[t] = 1 for duplicates.  fragile[t] =
 * 1 if the decision involves two tracks with as many hits and chi2 within
 * chi2_tol_rel * chi2 + chi2_tol_abs, whose order rounding could swap.
 * Returns the number of duplicates. */
int32_t orc_duplicates(int32_t n, int32_t stride, const int32_t *n_hits, const int32_t *hits,
                       const double *chi2, const int32_t *seed, double frac, double chi2_tol_rel,
                       double chi2_tol_abs, int32_t *dup, int32_t *fragile) {
  int32_t nd = 0;
  for (int32_t t = 0; t < n; ++t) {
    dup[t] = 0;
    fragile[t] = 0;
    for (int32_t u = 0; u < n; ++u) {
      if (u == t) continue;
      int shared = 0;
      for (int i = 0; i < n_hits[t]; ++i)
        for (int j = 0; j < n_hits[u]; ++j) shared += hits[t * stride + i] == hits[u * stride + j];
      int mn = n_hits[t] < n_hits[u] ? n_hits[t] : n_hits[u];
      if (shared == 0 || (double)shared < frac * (double)mn) continue;
      int before;
      if (n_hits[u] != n_hits[t]) {
        before = n_hits[u] > n_hits[t];
      } else {
        if (fabs(chi2[u] - chi2[t]) <= chi2_tol_rel * fabs(chi2[t]) + chi2_tol_abs) fragile[t] = 1;
        if (chi2[u] != chi2[t]) {
          before = chi2[u] < chi2[t];
        } else {
          int k = 0;
          while (k < 3 && seed[3 * u + k] == seed[3 * t + k]) ++k;
          before = k < 3 && seed[3 * u + k] < seed[3 * t + k];
        }
      }
      if (before) dup[t] = 1;
    }
    nd += dup[t];
  }
  return nd;
}

/* ------------------------------------------------------ seed cleaning */

/* Seed cleaning (Section 2.2: several seeds built from hits of the same
 * outgoing particle are reduced to one, using the identity of their hits
 * and their fitted pT, eta and phi).  Reading: seeds s and t of one event
 * are instances of one particle if they share at least one hit and their
 * fitted states (on the third seed layer) agree: |q/pT_s - q/pT_t| <=
 * tol_ipt max(|q/pT_s|, |q/pT_t|), |eta_s - eta_t| <= tol_eta and |phi_s -
 * phi_t| <= tol_phi (wrapped).  Seed u ranks before t if its fit chi2 is
 * smaller; with the same chi2, if its hit triplet is lexicographically
 * smaller.  t is kept if its fit succeeded and no seed ranking before it is
 * an instance of the same particle.  trip: n x 3 event-local hit indices of
 * one event; par: n x 6 fitted states; ok: fit succeeded.  fragile[t] = 1 if
 * the decision involves a closeness test within frag_rel of its tolerance
 * or two chi2 within frag_rel of each other.  Returns the number kept. */
int32_t orc_clean_seeds(int32_t n, const int32_t *trip, const int32_t *ok, const double *par,
                        const double *chi2, double tol_ipt, double tol_eta, double tol_phi,
                        double frag_rel, int32_t *keep, int32_t *fragile) {
  int32_t nk = 0;
  for (int32_t t = 0; t < n; ++t) {
    keep[t] = ok[t] ? 1 : 0;
    fragile[t] = 0;
    if (!ok[t]) continue;
    const double eta_t = -log(tan(0.5 * par[6 * t + 5]));
    for (int32_t u = 0; u < n; ++u) {
      if (u == t || !ok[u]) continue;
      int share = 0;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) share |= trip[3 * t + i] == trip[3 * u + j];
      if (!share) continue;
      const double eta_u = -log(tan(0.5 * par[6 * u + 5]));
      const double a = par[6 * t + 3], b = par[6 * u + 3];
      const double m_ipt = tol_ipt * fmax(fabs(a), fabs(b)) - fabs(a - b);
      const double m_eta = tol_eta - fabs(eta_t - eta_u);
      const double m_phi = tol_phi - fabs(wrap_phi(par[6 * t + 4] - par[6 * u + 4]));
      if (fabs(m_ipt) <= frag_rel * tol_ipt * fmax(fabs(a), fabs(b)) ||
          fabs(m_eta) <= frag_rel * tol_eta || fabs(m_phi) <= frag_rel * tol_phi)
        fragile[t] = 1;
      if (m_ipt < 0.0 || m_eta < 0.0 || m_phi < 0.0) continue;
      int before;
      if (fabs(chi2[u] - chi2[t]) <= frag_rel * fmax(fabs(chi2[u]), fabs(chi2[t])))
        fragile[t] = 1;
      if (chi2[u] != chi2[t]) {
        before = chi2[u] < chi2[t];
      } else {
        int k = 0;
        while (k < 3 && trip[3 * u + k] == trip[3 * t + k]) ++k;
        before = k < 3 && trip[3 * u + k] < trip[3 * t + k];
      }
      if (before) keep[t] = 0;
    }
    nk += keep[t];
  }
  return nk;
}
