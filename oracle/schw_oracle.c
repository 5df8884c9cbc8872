/*
 * FP64 CPU oracle for the Schwarzschild model-build hot path.
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.
 *
 * Built with -ffp-contract=off so that every expression below is evaluated
 * exactly in the order it is written.
 *
 * Passages followed (SchwarMAX paper, arXiv 2607.00117):
 *   potentials ........ Sec. 2.1; NFW Eq. 8-9; Miyamoto-Nagai Eq. 10-11.
 *                        Plummer, Kepler, isochrone and the Ferrers n=2 bar
 *                        are textbook pairs (Binney & Tremaine 2008, Sec. 2.2,
 *                        2.5); the Ferrers potential is the homoeoid-theorem
 *                        integral for rho = rho_c (1 - m^2)^2.
 *   needle bars ........ Eq. 12 and App. A: the T3 and V4 parent pairs with
 *                        each R^-n replaced by its convolution with the
 *                        needle density f along the bar's x axis.
 *   integration ........ Sec. 2.2.2: fixed number of steps, corotating bar
 *                        frame, velocities kept inertial, Jacobi-energy cut.
 *   symmetrisation ..... Sec. 2.2.2, Table 1 (four mirror copies).
 *   projection ......... Sec. 2.2.3, Eq. 1 (z-x-z Euler rotation), line of
 *                        sight along z'.
 *   binning ............ Sec. 2.2.4 (time-weighted samples into 3D cells and
 *                        sky apertures x LOS-velocity bins).
 */
#include "schw_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* NFW halo (Eq. 8-9): M_DM from M200 and c; R_s = R200 / c, where      */
/* R200 encloses 200 rho_crit, rho_crit = 3 H0^2 / (8 pi G).            */
/* ------------------------------------------------------------------ */
void orc_nfw_derived(double M200, double c, double H0, double out[3]) {
  if (H0 <= 0.0) H0 = 70.0;
  double H = H0 / 1000.0; /* km/s/kpc */
  double rho_crit = 3.0 * H * H / (8.0 * M_PI * ORC_G);
  double R200 = cbrt(3.0 * M200 / (4.0 * M_PI * 200.0 * rho_crit));
  double Rs = R200 / c;
  double Mdm = M200 / (log(1.0 + c) - c / (1.0 + c));
  out[0] = Rs;
  out[1] = Mdm;
  out[2] = R200;
}

/* ------------------------------------------------------------------ */
/* Ferrers n = 2 ellipsoid: rho = rho_c (1 - m^2)^2 inside m < 1.        */
/*   Phi(x)   = -(pi G a b c rho_c / 3) Int_lam^inf (1 - m^2(u))^3 du / Delta(u)
 *   dPhi/dx_i = 2 pi G a b c rho_c x_i Int_lam^inf (1 - m^2(u))^2 du / ((a_i^2+u) Delta(u))
 * m^2(u) = sum_j x_j^2 / (a_j^2 + u), Delta = sqrt(prod_j (a_j^2 + u)),
 * lam = 0 inside, else the root of m^2(lam) = 1.                          */
/* ------------------------------------------------------------------ */
static double m2_of(const double A2[3], const double x[3], double u) {
  return x[0] * x[0] / (A2[0] + u) + x[1] * x[1] / (A2[1] + u) + x[2] * x[2] / (A2[2] + u);
}

double orc_ferrers_lambda(double a, double b, double c, const double x[3]) {
  double A2[3] = {a * a, b * b, c * c};
  if (m2_of(A2, x, 0.0) <= 1.0) return 0.0;
  /* m^2 decreases in u and m^2(r^2) < 1, so [0, r^2] brackets the root */
  double lo = 0.0, hi = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
  for (int it = 0; it < 400; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (m2_of(A2, x, mid) > 1.0) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

/* Gauss-Kronrod 7/15 abscissae and weights (QUADPACK qk15). */
static const double XGK[8] = {
    0.991455371120812639206854697526329, 0.949107912342758524526189684047851,
    0.864864423359769072789712788640926, 0.741531185599394439863864773280788,
    0.586087235467691130294144845693013, 0.405845151377397166906606412076961,
    0.207784955007898467600689403773245, 0.000000000000000000000000000000000};
static const double WGK[8] = {
    0.022935322010529224963732008058970, 0.063092092629978553290700663189204,
    0.104790010322250183839876322541518, 0.140653259715525918745189590510238,
    0.169004726639267902826583426598550, 0.190350578064785409913256402421014,
    0.204432940075298892414161999234649, 0.209482141084727828012999174891714};
static const double WG[4] = {
    0.129484966168869693270611432679082, 0.279705391489276667901467771423780,
    0.381830050505118944950369775488975, 0.417959183673469387755102040816327};

typedef struct {
  double A2[3];
  double x[3];
  double lam, K;
} fer_ctx;

/* integrand vector at t in (0,1]: u = lam + K (1/t^2 - 1), du = 2 K t^-3 dt
 * f[0] = (1-m^2)^3 / Delta, f[1+i] = (1-m^2)^2 / ((a_i^2+u) Delta)          */
static void fer_integrand(const fer_ctx* C, double t, double f[4]) {
  double q = 1.0 / (t * t) - 1.0;
  double u = C->lam + C->K * q;
  double d0 = C->A2[0] + u, d1 = C->A2[1] + u, d2 = C->A2[2] + u;
  double Delta = sqrt(d0 * d1 * d2);
  double m2 = C->x[0] * C->x[0] / d0 + C->x[1] * C->x[1] / d1 + C->x[2] * C->x[2] / d2;
  double w = 1.0 - m2;
  if (w < 0.0) w = 0.0; /* only at round-off distance from t = 1 */
  double jac = 2.0 * C->K / (t * t * t);
  f[0] = w * w * w / Delta * jac;
  f[1] = w * w / (d0 * Delta) * jac;
  f[2] = w * w / (d1 * Delta) * jac;
  f[3] = w * w / (d2 * Delta) * jac;
}

static void gk15(const fer_ctx* C, double lo, double hi, double res[4], double err[4]) {
  double half = 0.5 * (hi - lo), mid = 0.5 * (hi + lo);
  double k[4] = {0, 0, 0, 0}, g[4] = {0, 0, 0, 0}, f1[4], f2[4];
  fer_integrand(C, mid, f1);
  for (int j = 0; j < 4; ++j) { k[j] = WGK[7] * f1[j]; g[j] = WG[3] * f1[j]; }
  for (int i = 0; i < 7; ++i) {
    fer_integrand(C, mid - half * XGK[i], f1);
    fer_integrand(C, mid + half * XGK[i], f2);
    for (int j = 0; j < 4; ++j) {
      k[j] += WGK[i] * (f1[j] + f2[j]);
      if (i & 1) g[j] += WG[i / 2] * (f1[j] + f2[j]);
    }
  }
  for (int j = 0; j < 4; ++j) {
    res[j] = k[j] * half;
    err[j] = fabs((k[j] - g[j]) * half);
  }
}

static void adapt(const fer_ctx* C, double lo, double hi, double tol, int depth, double out[4]) {
  double r[4], e[4];
  gk15(C, lo, hi, r, e);
  int ok = 1;
  for (int j = 0; j < 4; ++j)
    if (e[j] > tol * fabs(r[j]) && e[j] > 1e-300) ok = 0;
  if (ok || depth >= 40) {
    for (int j = 0; j < 4; ++j) out[j] += r[j];
    return;
  }
  double mid = 0.5 * (lo + hi);
  adapt(C, lo, mid, tol, depth + 1, out);
  adapt(C, mid, hi, tol, depth + 1, out);
}

/* Timing mode: a fixed n-point Gauss-Legendre rule over t in (0, 1] in place
 * of the adaptive rule (n = 0, the default).  The nodes are the roots of P_n
 * found by Newton's method from the usual cosine first guesses, the weights
 * 2 / ((1 - x^2) P_n'(x)^2).  The integrand is smooth in t for a fixed point,
 * so 64 nodes reproduce the adaptive integrals to ~1e-13. */
#define FER_GL_MAX 128
static int g_fer_gl_n = 0;
static double g_fer_gl_x[FER_GL_MAX], g_fer_gl_w[FER_GL_MAX];

int orc_set_ferrers_rule(int n) {
  if (n < 0 || n > FER_GL_MAX) return -1;
  for (int i = 0; i < n; ++i) {
    double z = cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    g_fer_gl_x[i] = z;
    g_fer_gl_w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
  g_fer_gl_n = n;
  return 0;
}

static void fixed_gl(const fer_ctx* C, double out[4]) {
  double f[4];
  for (int i = 0; i < g_fer_gl_n; ++i) {
    fer_integrand(C, 0.5 + 0.5 * g_fer_gl_x[i], f);
    for (int j = 0; j < 4; ++j) out[j] += 0.5 * g_fer_gl_w[i] * f[j];
  }
}

/* I[0] = potential integral, I[1..3] = force integrals */
static void ferrers_integrals(double a, double b, double c, const double x[3], double I[4]) {
  fer_ctx C;
  C.A2[0] = a * a; C.A2[1] = b * b; C.A2[2] = c * c;
  C.x[0] = x[0]; C.x[1] = x[1]; C.x[2] = x[2];
  C.lam = orc_ferrers_lambda(a, b, c, x);
  double amin2 = C.A2[0];
  if (C.A2[1] < amin2) amin2 = C.A2[1];
  if (C.A2[2] < amin2) amin2 = C.A2[2];
  C.K = amin2 + C.lam;
  I[0] = I[1] = I[2] = I[3] = 0.0;
  if (g_fer_gl_n > 0)
    fixed_gl(&C, I);
  else
    adapt(&C, 0.0, 1.0, 1e-13, 0, I);
}

static double ferrers_rho_c(const double* p) { return 105.0 * p[0] / (32.0 * M_PI * p[1] * p[2] * p[3]); }

/* ------------------------------------------------------------------ */
/* Dehnen-Aly needle bars (Eq. 12, App. A).  For the point (x, y, z),  */
/* Z = a + zeta, zeta = sqrt(z^2 + b^2), and k = 0..6:                  */
/*   J_k = int_{-L}^{L} f(s) D(s)^-(2k+1)/2 ds,                          */
/*   X_k = int_{-L}^{L} f(s) (x - s) D(s)^-(2k+1)/2 ds,                  */
/*   D(s) = (x - s)^2 + y^2 + Z^2,                                       */
/*   f(s) = (1 + eta (1 - 2|s|/L)) / (2L) on |s| < L,                    */
/* so J_k is Eq. 12's I_n for n = 2k + 1 (with x' = x - s).  Each half  */
/* of the needle is integrated adaptively (f is linear there).          */
/* ------------------------------------------------------------------ */
#define DA_K 7

typedef struct {
  double x, y2Z2, L, eta;
  double sgn; /* +1: s in [0, L]; -1: s in [-L, 0] (s = sgn * u, u in [0, L]) */
} da_ctx;

static void da_integrand(const da_ctx* C, double u, double f[2 * DA_K]) {
  double s = C->sgn * u;
  double fs = (1.0 + C->eta * (1.0 - 2.0 * u / C->L)) / (2.0 * C->L);
  double dx = C->x - s;
  double D = dx * dx + C->y2Z2;
  double p = fs / sqrt(D);
  for (int k = 0; k < DA_K; ++k) {
    f[k] = p;
    f[DA_K + k] = p * dx;
    p = p / D;
  }
}

static void da_gk15(const da_ctx* C, double lo, double hi, double res[2 * DA_K], double err[2 * DA_K]) {
  double half = 0.5 * (hi - lo), mid = 0.5 * (hi + lo);
  double k[2 * DA_K], g[2 * DA_K], f1[2 * DA_K], f2[2 * DA_K];
  da_integrand(C, mid, f1);
  for (int j = 0; j < 2 * DA_K; ++j) { k[j] = WGK[7] * f1[j]; g[j] = WG[3] * f1[j]; }
  for (int i = 0; i < 7; ++i) {
    da_integrand(C, mid - half * XGK[i], f1);
    da_integrand(C, mid + half * XGK[i], f2);
    for (int j = 0; j < 2 * DA_K; ++j) {
      k[j] += WGK[i] * (f1[j] + f2[j]);
      if (i & 1) g[j] += WG[i / 2] * (f1[j] + f2[j]);
    }
  }
  for (int j = 0; j < 2 * DA_K; ++j) {
    res[j] = k[j] * half;
    err[j] = fabs((k[j] - g[j]) * half);
  }
}

/* absolute tolerance per entry: tol times the entry's size over the whole half */
static void da_adapt(const da_ctx* C, double lo, double hi, const double scale[2 * DA_K], double tol, int depth,
                     double out[2 * DA_K]) {
  double r[2 * DA_K], e[2 * DA_K];
  da_gk15(C, lo, hi, r, e);
  int ok = 1;
  for (int j = 0; j < 2 * DA_K; ++j)
    if (e[j] > tol * scale[j] && e[j] > 1e-300) ok = 0;
  if (ok || depth >= 40) {
    for (int j = 0; j < 2 * DA_K; ++j) out[j] += r[j];
    return;
  }
  double mid = 0.5 * (lo + hi);
  da_adapt(C, lo, mid, scale, tol, depth + 1, out);
  da_adapt(C, mid, hi, scale, tol, depth + 1, out);
}

/* J[k], X[k] of the needle bar with parameters p (M, a, b, L, eta) at x */
static void da_integrals(const double* p, const double x[3], double J[DA_K], double X[DA_K], double* Z,
                         double* zeta) {
  double a = p[1], b = p[2];
  *zeta = sqrt(x[2] * x[2] + b * b);
  *Z = a + *zeta;
  double out[2 * DA_K];
  for (int j = 0; j < 2 * DA_K; ++j) out[j] = 0.0;
  for (int h = 0; h < 2; ++h) {
    da_ctx C;
    C.x = x[0];
    C.y2Z2 = x[1] * x[1] + (*Z) * (*Z);
    C.L = p[3];
    C.eta = p[4];
    C.sgn = h == 0 ? 1.0 : -1.0;
    double r[2 * DA_K], e[2 * DA_K], scale[2 * DA_K];
    da_gk15(&C, 0.0, C.L, r, e);
    for (int j = 0; j < 2 * DA_K; ++j) scale[j] = fabs(r[j]) + 1e-300;
    da_adapt(&C, 0.0, C.L, scale, 1e-14, 0, out);
  }
  for (int k = 0; k < DA_K; ++k) {
    J[k] = out[k];
    X[k] = out[DA_K + k];
  }
}

/* The parent potential -GM sum_n c_n R^-n written as coefficients c_n(Z, zeta)
 * of n = 1, 3, 5, ... (index k = (n - 1) / 2) and their derivatives dc_n/dzeta
 * (Z = a + zeta); returns the number of terms. */
static int da_coeffs(int kind, double a, double b, double Z, double zeta, double c[5], double dc[5]) {
  double b2 = b * b;
  if (kind == ORC_DA_T3) {
    /* App. A: Phi_T3 = -GM [1/R + a (Z - a/3)/R^3 + a^2 Z^2/R^5] */
    c[0] = 1.0; dc[0] = 0.0;
    c[1] = a * (Z - a / 3.0); dc[1] = a;
    c[2] = a * a * Z * Z; dc[2] = 2.0 * a * a * Z;
    return 3;
  }
  /* App. A: Phi_V4 = -GM [1/R + (a (Z - 2a/5) + b^2/2)/R^3
   *   + 3a (a Z (2Z - a)/5 + (b^2/2)(Z - a/5))/R^5 + a^2 Z^2 (a Z + 3 b^2)/R^7
   *   + 7 a^3 b^2 Z^4 / (2 zeta R^9)] */
  c[0] = 1.0; dc[0] = 0.0;
  c[1] = a * (Z - 2.0 * a / 5.0) + b2 / 2.0; dc[1] = a;
  c[2] = 3.0 * a * (a * Z * (2.0 * Z - a) / 5.0 + (b2 / 2.0) * (Z - a / 5.0));
  dc[2] = 3.0 * a * (a * (4.0 * Z - a) / 5.0 + b2 / 2.0);
  c[3] = a * a * Z * Z * (a * Z + 3.0 * b2);
  dc[3] = 3.0 * a * a * a * Z * Z + 6.0 * a * a * b2 * Z;
  c[4] = 7.0 * a * a * a * b2 * Z * Z * Z * Z / (2.0 * zeta);
  dc[4] = (7.0 * a * a * a * b2 / 2.0) * (4.0 * Z * Z * Z / zeta - Z * Z * Z * Z / (zeta * zeta));
  return 5;
}

static double da_phi(int kind, const double* p, const double x[3]) {
  double J[DA_K], X[DA_K], Z, zeta, c[5], dc[5];
  da_integrals(p, x, J, X, &Z, &zeta);
  int nt = da_coeffs(kind, p[1], p[2], Z, zeta, c, dc);
  double s = 0.0;
  for (int k = 0; k < nt; ++k) s = s + c[k] * J[k];
  return -ORC_G * p[0] * s;
}

/* g = -grad Phi: with dI_n/dx = -n X_(n+2), dI_n/dy = -n y J_(n+2),
 * dI_n/dZ = -n Z J_(n+2) and dZ/dz = z / zeta */
static void da_accel_add(int kind, const double* p, const double x[3], double g[3]) {
  double J[DA_K], X[DA_K], Z, zeta, c[5], dc[5];
  da_integrals(p, x, J, X, &Z, &zeta);
  int nt = da_coeffs(kind, p[1], p[2], Z, zeta, c, dc);
  double GM = ORC_G * p[0];
  double sx = 0.0, sy = 0.0, sz = 0.0;
  for (int k = 0; k < nt; ++k) {
    double n = 2.0 * k + 1.0;
    sx = sx + n * c[k] * X[k + 1];
    sy = sy + n * c[k] * J[k + 1];
    sz = sz + (dc[k] * J[k] - n * c[k] * Z * J[k + 1]);
  }
  g[0] = g[0] - GM * sx;
  g[1] = g[1] - GM * x[1] * sy;
  g[2] = g[2] + GM * sz * x[2] / zeta;
}

/* App. A densities with the same replacement (n = 5, 7, 9 for T3; 7..13 for V4) */
static double da_density(int kind, const double* p, const double x[3]) {
  double J[DA_K], X[DA_K], Z, zeta;
  da_integrals(p, x, J, X, &Z, &zeta);
  double M = p[0], a = p[1], b = p[2], e = zeta;
  if (kind == ORC_DA_T3)
    return (M * b * b / (4.0 * M_PI)) *
           (3.0 * J[2] + 5.0 * a * Z * Z * (3.0 * e * e - 2.0 * a * e + a * a) / (e * e * e) * J[3] +
            35.0 * a * a * Z * Z * Z * Z / (e * e) * J[4]);
  return (3.0 * M * b * b * b * b / (8.0 * M_PI)) *
         (5.0 * J[3] +
          7.0 * a * Z * Z * (5.0 * e * e * e * e - 4.0 * a * e * e * e + 3.0 * a * a * e * e - 2.0 * a * a * a * e +
                             a * a * a * a) / (e * e * e * e * e) * J[4] +
          63.0 * a * a * Z * Z * Z * Z * (2.0 * e * e - 2.0 * a * e + a * a) / (e * e * e * e) * J[5] +
          231.0 * a * a * a * Z * Z * Z * Z * Z * Z / (e * e * e) * J[6]);
}

/* ------------------------------------------------------------------ */
/* Components.                                                          */
/* ------------------------------------------------------------------ */
static double comp_phi(const orc_comp* C, const double x[3]) {
  const double* p = C->p;
  double GM = ORC_G * p[0];
  switch (C->kind) {
    case ORC_KEPLER: {
      double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
      return -GM / r;
    }
    case ORC_ISOCHRONE: {
      double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
      return -GM / (p[1] + sqrt(p[1] * p[1] + r2));
    }
    case ORC_PLUMMER: {
      double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
      return -GM / sqrt(r2 + p[1] * p[1]);
    }
    case ORC_MN: {
      double R2 = x[0] * x[0] + x[1] * x[1];
      double zeta = sqrt(x[2] * x[2] + p[2] * p[2]);
      double s = p[1] + zeta;
      return -GM / sqrt(R2 + s * s);
    }
    case ORC_NFW_Q: {
      double d[3];
      orc_nfw_derived(p[0], p[1], p[3], d);
      double q = p[2];
      double m = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2] / (q * q));
      double GMd = ORC_G * d[1];
      if (m == 0.0) return -GMd / d[0];
      return -GMd * log1p(m / d[0]) / m;
    }
    case ORC_FERRERS2: {
      double I[4];
      ferrers_integrals(p[1], p[2], p[3], x, I);
      return -(M_PI * ORC_G * p[1] * p[2] * p[3] * ferrers_rho_c(p) / 3.0) * I[0];
    }
    case ORC_DA_T3:
    case ORC_DA_V4:
      return da_phi(C->kind, p, x);
  }
  return NAN;
}

/* acceleration g = -grad Phi, added into g[] */
static void comp_accel_add(const orc_comp* C, const double x[3], double g[3]) {
  const double* p = C->p;
  double GM = ORC_G * p[0];
  switch (C->kind) {
    case ORC_KEPLER: {
      double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
      double r = sqrt(r2);
      double f = GM / (r2 * r);
      g[0] = g[0] - f * x[0];
      g[1] = g[1] - f * x[1];
      g[2] = g[2] - f * x[2];
      return;
    }
    case ORC_ISOCHRONE: {
      double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
      double s = sqrt(p[1] * p[1] + r2);
      double den = p[1] + s;
      double f = GM / (den * den * s); /* dPhi/dr / r */
      g[0] = g[0] - f * x[0];
      g[1] = g[1] - f * x[1];
      g[2] = g[2] - f * x[2];
      return;
    }
    case ORC_PLUMMER: {
      double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
      double d2 = r2 + p[1] * p[1];
      double d = sqrt(d2);
      double f = GM / (d2 * d);
      g[0] = g[0] - f * x[0];
      g[1] = g[1] - f * x[1];
      g[2] = g[2] - f * x[2];
      return;
    }
    case ORC_MN: {
      double R2 = x[0] * x[0] + x[1] * x[1];
      double zeta = sqrt(x[2] * x[2] + p[2] * p[2]);
      double s = p[1] + zeta;
      double D2 = R2 + s * s;
      double D = sqrt(D2);
      double f = GM / (D2 * D);
      g[0] = g[0] - f * x[0];
      g[1] = g[1] - f * x[1];
      g[2] = g[2] - f * x[2] * s / zeta;
      return;
    }
    case ORC_NFW_Q: {
      double d[3];
      orc_nfw_derived(p[0], p[1], p[3], d);
      double q = p[2], Rs = d[0], GMd = ORC_G * d[1];
      double m = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2] / (q * q));
      if (m == 0.0) return;
      /* dPhi/dm = G M_DM [ ln(1+m/Rs)/m^2 - 1/(m (Rs+m)) ] */
      double dphidm = GMd * (log1p(m / Rs) / (m * m) - 1.0 / (m * (Rs + m)));
      double f = dphidm / m;
      g[0] = g[0] - f * x[0];
      g[1] = g[1] - f * x[1];
      g[2] = g[2] - f * x[2] / (q * q);
      return;
    }
    case ORC_FERRERS2: {
      double I[4];
      ferrers_integrals(p[1], p[2], p[3], x, I);
      double k = 2.0 * M_PI * ORC_G * p[1] * p[2] * p[3] * ferrers_rho_c(p);
      g[0] = g[0] - k * x[0] * I[1];
      g[1] = g[1] - k * x[1] * I[2];
      g[2] = g[2] - k * x[2] * I[3];
      return;
    }
    case ORC_DA_T3:
    case ORC_DA_V4:
      da_accel_add(C->kind, p, x, g);
      return;
  }
}

static double comp_density(const orc_comp* C, const double x[3]) {
  const double* p = C->p;
  double M = p[0];
  switch (C->kind) {
    case ORC_KEPLER:
      return 0.0;
    case ORC_ISOCHRONE: {
      double b = p[1];
      double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
      double a = sqrt(b * b + r2);
      return M * (3.0 * (b + a) * a * a - r2 * (b + 3.0 * a)) / (4.0 * M_PI * pow(b + a, 3) * a * a * a);
    }
    case ORC_PLUMMER: {
      double b = p[1];
      double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
      return 3.0 * M / (4.0 * M_PI * b * b * b) * pow(1.0 + r2 / (b * b), -2.5);
    }
    case ORC_MN: { /* Eq. 11 */
      double a = p[1], b = p[2];
      double R2 = x[0] * x[0] + x[1] * x[1];
      double zeta = sqrt(x[2] * x[2] + b * b);
      double calR2 = R2 + (a + zeta) * (a + zeta);
      double calR = sqrt(calR2);
      return (b * b * M / (4.0 * M_PI)) * (a * calR2 + 3.0 * zeta * (zeta + a) * (zeta + a)) /
             (pow(calR, 5) * zeta * zeta * zeta);
    }
    case ORC_NFW_Q: { /* Eq. 8, spherical case only */
      if (p[2] != 1.0) return NAN;
      double d[3];
      orc_nfw_derived(p[0], p[1], p[3], d);
      double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]) / d[0];
      return d[1] / (4.0 * M_PI * d[0] * d[0] * d[0]) / (r * (1.0 + r) * (1.0 + r));
    }
    case ORC_FERRERS2: {
      double m2 = x[0] * x[0] / (p[1] * p[1]) + x[1] * x[1] / (p[2] * p[2]) + x[2] * x[2] / (p[3] * p[3]);
      if (m2 >= 1.0) return 0.0;
      return ferrers_rho_c(p) * (1.0 - m2) * (1.0 - m2);
    }
    case ORC_DA_T3:
    case ORC_DA_V4:
      return da_density(C->kind, p, x);
  }
  return NAN;
}

double orc_phi(const orc_pot* P, const double x[3]) {
  double s = 0.0;
  for (int i = 0; i < P->ncomp; ++i) s = s + comp_phi(&P->comp[i], x);
  return s;
}

void orc_accel(const orc_pot* P, const double x[3], double g[3]) {
  g[0] = g[1] = g[2] = 0.0;
  for (int i = 0; i < P->ncomp; ++i) comp_accel_add(&P->comp[i], x, g);
}

double orc_density(const orc_pot* P, const double x[3]) {
  double s = 0.0;
  for (int i = 0; i < P->ncomp; ++i) s = s + comp_density(&P->comp[i], x);
  return s;
}

/* Jacobi energy E_J = |p|^2/2 + Phi(x) - Omega (x p_y - y p_x), with p the
 * inertial velocity expressed on the rotating axes. */
double orc_jacobi(const orc_pot* P, const double s[6]) {
  double kin = 0.5 * (s[3] * s[3] + s[4] * s[4] + s[5] * s[5]);
  double Lz = s[0] * s[4] - s[1] * s[3];
  return kin + orc_phi(P, s) - P->omega * Lz;
}

/* Eq. 1: R = R_z(gamma) R_x(beta) R_z(alpha), active right-handed rotations */
static void matmul3(const double A[9], const double B[9], double C[9]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s = s + A[3 * i + k] * B[3 * k + j];
      C[3 * i + j] = s;
    }
}

void orc_euler_matrix(double alpha, double beta, double gamma, double R[9]) {
  double ca = cos(alpha), sa = sin(alpha), cb = cos(beta), sb = sin(beta), cg = cos(gamma), sg = sin(gamma);
  double Rza[9] = {ca, -sa, 0, sa, ca, 0, 0, 0, 1};
  double Rxb[9] = {1, 0, 0, 0, cb, -sb, 0, sb, cb};
  double Rzg[9] = {cg, -sg, 0, sg, cg, 0, 0, 0, 1};
  double T[9];
  matmul3(Rxb, Rza, T);
  matmul3(Rzg, T, R);
}

/* Kick-drift-kick step of H = |p|^2/2 + Phi(x) - Omega L_z.
 * The drift is the exact flow of |p|^2/2 - Omega L_z: a straight-line move
 * by dt p followed by a rotation of both x and p by -Omega dt about z. */
void orc_step(const orc_pot* P, double s[6], double dt) {
  double g[3];
  double h = 0.5 * dt;
  orc_accel(P, s, g);
  s[3] = s[3] + h * g[0];
  s[4] = s[4] + h * g[1];
  s[5] = s[5] + h * g[2];
  s[0] = s[0] + dt * s[3];
  s[1] = s[1] + dt * s[4];
  s[2] = s[2] + dt * s[5];
  double c = cos(P->omega * dt), sn = sin(P->omega * dt);
  double x = c * s[0] + sn * s[1];
  double y = c * s[1] - sn * s[0];
  double px = c * s[3] + sn * s[4];
  double py = c * s[4] - sn * s[3];
  s[0] = x; s[1] = y; s[3] = px; s[4] = py;
  orc_accel(P, s, g);
  s[3] = s[3] + h * g[0];
  s[4] = s[4] + h * g[1];
  s[5] = s[5] + h * g[2];
}

void orc_orbit(const orc_pot* P, const double ic[6], double dt, int nsteps, double* traj) {
  double s[6];
  memcpy(s, ic, sizeof s);
  memcpy(traj, s, sizeof s);
  for (int k = 1; k <= nsteps; ++k) {
    orc_step(P, s, dt);
    memcpy(traj + 6 * (long)k, s, sizeof s);
  }
}

int orc_ncon(const orc_obs* O) { return O->nx * O->ny * O->nz + O->n_ap * O->nv + (O->surface ? O->n_ap : 0); }

/* ------------------------------------------------------------------ */
/* Binning (Sec. 2.2.4).  A coordinate v falls in bin floor(t) with      */
/* t = (v - lo) * (n / (hi - lo)), the scale taken in double precision;  */
/* the sample is inside iff 0 <= t < n.                                  */
/* ------------------------------------------------------------------ */
static int bin_d(double v, double lo, double inv, int n) {
  double t = (v - lo) * inv;
  if (!(t >= 0.0 && t < (double)n)) return -1;
  return (int)t;
}
static int bin_f(float v, float lo, float inv, int n) {
  float t = (v - lo) * inv;
  if (!(t >= 0.0f && t < (float)n)) return -1;
  return (int)t;
}

static const double MIRROR[4][3] = {{1, 1, 1}, {1, 1, -1}, {-1, -1, 1}, {-1, -1, -1}};

/* Cylindrical mass grid (Sec. 2.2.4: bins uniform in R, phi, z), decided
 * exactly in the working precision: R bin k iff e_k^2 <= x^2 + y^2 < e_(k+1)^2,
 * e_k = lo + k w; sector k iff the point is on or counterclockwise of the
 * edge at phi_k = -pi + 2 pi k / n and clockwise of the edge at phi_(k+1)
 * (cross products with the edge directions, cos and sin taken in double);
 * a point that no sector's test takes (the axis, and the edge at phi = pi)
 * goes to the last sector.  Scanned from k = 0: the first k whose test holds. */
static int cyl_r_d(double R2, double lo, double w, int n) {
  for (int k = 0; k < n; ++k) {
    double e0 = lo + (double)k * w, e1 = lo + (double)(k + 1) * w;
    if (R2 >= e0 * e0 && R2 < e1 * e1) return k;
  }
  return -1;
}
static int cyl_r_f(float R2, float lo, float w, int n) {
  for (int k = 0; k < n; ++k) {
    float e0 = lo + (float)k * w, e1 = lo + (float)(k + 1) * w;
    if (R2 >= e0 * e0 && R2 < e1 * e1) return k;
  }
  return -1;
}
static int ccw_d(double x, double y, int k, int n) {
  double ph = -M_PI + 2.0 * M_PI * k / n;
  return cos(ph) * y - sin(ph) * x >= 0.0;
}
static int ccw_f(float x, float y, int k, int n) {
  double ph = -M_PI + 2.0 * M_PI * k / n;
  float c = (float)cos(ph), s = (float)sin(ph);
  return c * y - s * x >= 0.0f;
}
static int cyl_sector_d(double x, double y, int n) {
  for (int k = 0; k < n; ++k)
    if (ccw_d(x, y, k, n) && !ccw_d(x, y, k + 1, n)) return k;
  return n - 1;
}
static int cyl_sector_f(float x, float y, int n) {
  for (int k = 0; k < n; ++k)
    if (ccw_f(x, y, k, n) && !ccw_f(x, y, k + 1, n)) return k;
  return n - 1;
}

static void cells_d(const orc_obs* O, const double s6[6], int copy, int* mcell, int* kcell, int* acell) {
  double x = MIRROR[copy][0] * s6[0], y = MIRROR[copy][1] * s6[1], z = MIRROR[copy][2] * s6[2];
  double px = MIRROR[copy][0] * s6[3], py = MIRROR[copy][1] * s6[4], pz = MIRROR[copy][2] * s6[5];
  int ix = bin_d(x, O->lo[0], O->nx / (O->hi[0] - O->lo[0]), O->nx);
  int iy = bin_d(y, O->lo[1], O->ny / (O->hi[1] - O->lo[1]), O->ny);
  int iz = bin_d(z, O->lo[2], O->nz / (O->hi[2] - O->lo[2]), O->nz);
  if (O->grid == 1) {
    ix = cyl_r_d(x * x + y * y, O->lo[0], (O->hi[0] - O->lo[0]) / O->nx, O->nx);
    iy = cyl_sector_d(x, y, O->ny);
  }
  *mcell = (ix < 0 || iy < 0 || iz < 0) ? -1 : (ix * O->ny + iy) * O->nz + iz;
  const double* R = O->R;
  double X = R[0] * x + R[1] * y + R[2] * z;
  double Y = R[3] * x + R[4] * y + R[5] * z;
  double V = R[6] * px + R[7] * py + R[8] * pz;
  int jx = bin_d(X, O->plo[0], O->npx / (O->phi[0] - O->plo[0]), O->npx);
  int jy = bin_d(Y, O->plo[1], O->npy / (O->phi[1] - O->plo[1]), O->npy);
  int kv = bin_d(V, O->vlo, O->nv / (O->vhi - O->vlo), O->nv);
  int ap = -1;
  if (jx >= 0 && jy >= 0) {
    int pix = jx * O->npy + jy;
    ap = O->pix2ap ? O->pix2ap[pix] : pix;
  }
  *kcell = (ap < 0 || kv < 0) ? -1 : ap * O->nv + kv;
  *acell = ap;
}

static void cells_f(const orc_obs* O, const float s6[6], int copy, int* mcell, int* kcell, int* acell) {
  float sx = (float)MIRROR[copy][0], sy = (float)MIRROR[copy][1], sz = (float)MIRROR[copy][2];
  float x = sx * s6[0], y = sy * s6[1], z = sz * s6[2];
  float px = sx * s6[3], py = sy * s6[4], pz = sz * s6[5];
  int ix = bin_f(x, (float)O->lo[0], (float)(O->nx / (O->hi[0] - O->lo[0])), O->nx);
  int iy = bin_f(y, (float)O->lo[1], (float)(O->ny / (O->hi[1] - O->lo[1])), O->ny);
  int iz = bin_f(z, (float)O->lo[2], (float)(O->nz / (O->hi[2] - O->lo[2])), O->nz);
  if (O->grid == 1) {
    ix = cyl_r_f(x * x + y * y, (float)O->lo[0], (float)((O->hi[0] - O->lo[0]) / O->nx), O->nx);
    iy = cyl_sector_f(x, y, O->ny);
  }
  *mcell = (ix < 0 || iy < 0 || iz < 0) ? -1 : (ix * O->ny + iy) * O->nz + iz;
  float R[9];
  for (int i = 0; i < 9; ++i) R[i] = (float)O->R[i];
  float X = R[0] * x + R[1] * y + R[2] * z;
  float Y = R[3] * x + R[4] * y + R[5] * z;
  float V = R[6] * px + R[7] * py + R[8] * pz;
  int jx = bin_f(X, (float)O->plo[0], (float)(O->npx / (O->phi[0] - O->plo[0])), O->npx);
  int jy = bin_f(Y, (float)O->plo[1], (float)(O->npy / (O->phi[1] - O->plo[1])), O->npy);
  int kv = bin_f(V, (float)O->vlo, (float)(O->nv / (O->vhi - O->vlo)), O->nv);
  int ap = -1;
  if (jx >= 0 && jy >= 0) {
    int pix = jx * O->npy + jy;
    ap = O->pix2ap ? O->pix2ap[pix] : pix;
  }
  *kcell = (ap < 0 || kv < 0) ? -1 : ap * O->nv + kv;
  *acell = ap;
}

/* kinematic cell as bin_points reports it: with the surface block on, an
 * event in aperture a whose velocity is outside the range reports n_ap*nv + a */
static int kin_code(const orc_obs* O, int k, int a) {
  if (k >= 0) return k;
  return (O->surface && a >= 0) ? O->n_ap * O->nv + a : -1;
}

void orc_bin_points_f64(const orc_obs* O, long n, const double* pts, int32_t* mass, int32_t* kin) {
  for (long i = 0; i < n; ++i) {
    double s6[6];
    for (int j = 0; j < 6; ++j) s6[j] = pts[j * n + i];
    for (int c = 0; c < 4; ++c) {
      int m, k, a;
      cells_d(O, s6, c, &m, &k, &a);
      mass[4 * i + c] = m;
      kin[4 * i + c] = kin_code(O, k, a);
    }
  }
}

void orc_bin_points_f32(const orc_obs* O, long n, const float* pts, int32_t* mass, int32_t* kin) {
  for (long i = 0; i < n; ++i) {
    float s6[6];
    for (int j = 0; j < 6; ++j) s6[j] = pts[j * n + i];
    for (int c = 0; c < 4; ++c) {
      int m, k, a;
      cells_f(O, s6, c, &m, &k, &a);
      mass[4 * i + c] = m;
      kin[4 * i + c] = kin_code(O, k, a);
    }
  }
}

static void integrate_and_bin_impl(const orc_pot* P, const orc_obs* O, long n, const double* ics,
                                   const double* dt, int nsteps, int32_t* counts, int64_t* overflow,
                                   double* drift, uint8_t* flags, int nthreads, int round_state) {
  int ncon = orc_ncon(O);
  int nmass = O->nx * O->ny * O->nz, nkin = O->n_ap * O->nv;
  int ncopy = O->symmetrize ? 4 : 1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (long i = 0; i < n; ++i) {
    double s[6];
    for (int j = 0; j < 6; ++j) s[j] = ics[j * n + i];
    int32_t* row = counts + i * (long)ncon;
    memset(row, 0, sizeof(int32_t) * (size_t)ncon);
    int64_t ovm = 0, ovk = 0;
    double E0 = orc_jacobi(P, s), dmax = 0.0;
    int nonfinite = 0;
    for (int k = 1; k <= nsteps; ++k) {
      orc_step(P, s, dt[i]);
      if (round_state)
        for (int j = 0; j < 6; ++j) s[j] = (double)(float)s[j];
      for (int j = 0; j < 6; ++j)
        if (!isfinite(s[j])) nonfinite = 1;
      for (int c = 0; c < ncopy; ++c) {
        int m, kc, a;
        cells_d(O, s, c, &m, &kc, &a);
        if (m >= 0) row[m] += 1; else ovm += 1;
        if (kc >= 0) row[nmass + kc] += 1; else ovk += 1;
        if (O->surface && a >= 0) row[nmass + nkin + a] += 1;
      }
      if (O->drift_every > 0 && k % O->drift_every == 0) {
        double e = fabs(orc_jacobi(P, s) / E0 - 1.0);
        if (!(e <= dmax)) dmax = e; /* NaN propagates */
      }
    }
    overflow[2 * i] = ovm;
    overflow[2 * i + 1] = ovk;
    drift[i] = dmax;
    uint8_t f = 0;
    if (!(dmax <= 0.1)) f |= 1;
    if (nonfinite) f |= 2;
    flags[i] = f;
  }
}

void orc_integrate_and_bin(const orc_pot* P, const orc_obs* O, long n, const double* ics,
                           const double* dt, int nsteps, int32_t* counts, int64_t* overflow,
                           double* drift, uint8_t* flags, int nthreads) {
  integrate_and_bin_impl(P, O, n, ics, dt, nsteps, counts, overflow, drift, flags, nthreads, 0);
}

void orc_integrate_and_bin_f32state(const orc_pot* P, const orc_obs* O, long n, const double* ics,
                                    const double* dt, int nsteps, int32_t* counts, int64_t* overflow,
                                    double* drift, uint8_t* flags, int nthreads) {
  integrate_and_bin_impl(P, O, n, ics, dt, nsteps, counts, overflow, drift, flags, nthreads, 1);
}

/* ------------------------------------------------------------------ */
/* Target cell masses m*_n (Sec. 2.2.4): the mass of the potential's    */
/* density (all of its components) in each cell of the mass grid,       */
/*   Cartesian:   int dx int dy int dz rho(x, y, z),                    */
/*   cylindrical: int R dR int dphi int dz rho(R cos phi, R sin phi, z),*/
/* cell edges lo + k (hi - lo) / n (R, z) and -pi + 2 pi k / ny (phi).  */
/* Each of the three nested integrals is adaptive Gauss-Kronrod (7/15   */
/* points), bisecting until |K15 - G7| <= rel_tol |K15| on the piece.   */
/* The densities are non-negative, so a relative test is meaningful.    */
/* ------------------------------------------------------------------ */
typedef double (*cm_fn)(void* ctx, double t);

static double cm_gk15(cm_fn f, void* ctx, double lo, double hi, double* err) {
  double half = 0.5 * (hi - lo), mid = 0.5 * (hi + lo);
  double fc = f(ctx, mid);
  double k = WGK[7] * fc, g = WG[3] * fc;
  for (int i = 0; i < 7; ++i) {
    double s = f(ctx, mid - half * XGK[i]) + f(ctx, mid + half * XGK[i]);
    k += WGK[i] * s;
    if (i & 1) g += WG[i / 2] * s;
  }
  *err = fabs((k - g) * half);
  return k * half;
}

/* accepts a piece when |K15 - G7| <= max(rel_tol |K15|, abs_tol); the halves
 * of a bisected piece share its absolute tolerance */
static double cm_adapt(cm_fn f, void* ctx, double lo, double hi, double rel_tol, double abs_tol, int depth) {
  double err, r = cm_gk15(f, ctx, lo, hi, &err);
  if (!isfinite(r) || err <= fmax(rel_tol * fabs(r), abs_tol) || depth >= 30) return r;
  double mid = 0.5 * (lo + hi);
  return cm_adapt(f, ctx, lo, mid, rel_tol, 0.5 * abs_tol, depth + 1) +
         cm_adapt(f, ctx, mid, hi, rel_tol, 0.5 * abs_tol, depth + 1);
}

typedef struct {
  const orc_pot* P;
  int cyl;
  double u, v;        /* outer coordinates: (x, y) or (R, phi) */
  double lo[3], hi[3]; /* the cell */
  double tol, atol[3]; /* relative tolerance; absolute one of each level's integral */
} cm_ctx;

static double cm_f3(void* c, double z) {
  cm_ctx* C = (cm_ctx*)c;
  double x[3];
  if (C->cyl) {
    x[0] = C->u * cos(C->v);
    x[1] = C->u * sin(C->v);
  } else {
    x[0] = C->u;
    x[1] = C->v;
  }
  x[2] = z;
  return orc_density(C->P, x);
}

static double cm_f2(void* c, double v) {
  cm_ctx* C = (cm_ctx*)c;
  C->v = v;
  return cm_adapt(cm_f3, c, C->lo[2], C->hi[2], C->tol, C->atol[2], 0);
}

static double cm_f1(void* c, double u) {
  cm_ctx* C = (cm_ctx*)c;
  C->u = u;
  double s = cm_adapt(cm_f2, c, C->lo[1], C->hi[1], C->tol, C->atol[1], 0);
  return C->cyl ? u * s : s;
}

double orc_cell_mass(const orc_pot* P, const orc_obs* O, int cell, double rel_tol, double abs_tol) {
  int ix = cell / (O->ny * O->nz), iy = (cell / O->nz) % O->ny, iz = cell % O->nz;
  cm_ctx C;
  C.P = P;
  C.cyl = O->grid == 1;
  C.tol = rel_tol;
  int idx[3] = {ix, iy, iz}, n[3] = {O->nx, O->ny, O->nz};
  for (int d = 0; d < 3; ++d) {
    double w = (O->hi[d] - O->lo[d]) / n[d];
    C.lo[d] = O->lo[d] + idx[d] * w;
    C.hi[d] = O->lo[d] + (idx[d] + 1) * w;
  }
  if (C.cyl) {
    C.lo[1] = -M_PI + 2.0 * M_PI * iy / O->ny;
    C.hi[1] = -M_PI + 2.0 * M_PI * (iy + 1) / O->ny;
  }
  /* an error e in an inner integral adds at most e times the outer extent
   * (times R, cylindrical) to the cell's mass */
  double l0 = C.hi[0] - C.lo[0], l1 = C.hi[1] - C.lo[1], rmax = C.cyl ? C.hi[0] : 1.0;
  C.atol[0] = abs_tol;
  C.atol[1] = abs_tol / (l0 * rmax);
  C.atol[2] = abs_tol / (l0 * rmax * l1);
  return cm_adapt(cm_f1, &C, C.lo[0], C.hi[0], rel_tol, abs_tol, 0);
}

/* ------------------------------------------------------------------ */
/* Initial velocities from the anisotropic Jeans equations in the       */
/* axisymmetrised potential (Sec. 2.2.1).  Tracer density: the fiducial */
/* nu(R, z) ~ exp(-R/hR - |z|/hz) the positions are drawn from; the      */
/* velocity ellipsoid is aligned with (R, phi, z), sigma_R^2 = b         */
/* sigma_z^2.  With F the azimuth-averaged force:                        */
/*   sigma_z^2(R, z) = (1/nu) int_|z|^inf nu(R, z') (-F_z(R, z')) dz'    */
/*                   = hz int_0^inf e^-s (-F_z(R, |z| + hz s)) ds,      */
/*   <v_phi^2> = b sigma_z^2 + (R/nu) d(b nu sigma_z^2)/dR - R F_R(R, z) */
/*             = b [sigma_z^2 (1 - R/hR) + R d sigma_z^2/dR] - R F_R,    */
/*   sigma_phi = sigma_R (isotropic in the plane), and the mean          */
/*   azimuthal velocity sqrt(max(<v_phi^2> - sigma_phi^2, 0)) (the        */
/*   rotation curve less the asymmetric drift).                          */
/* Every integral is adaptive Gauss-Kronrod; d/dR is a Richardson-        */
/* extrapolated central difference.                                      */
/* ------------------------------------------------------------------ */
typedef struct {
  const orc_pot* P;
  double R, z, tol;
  int comp; /* 0: F_R, 1: F_z */
  double hz, zabs;
} jn_ctx;

static double jn_fphi(void* c, double ph) {
  jn_ctx* C = (jn_ctx*)c;
  double x[3] = {C->R * cos(ph), C->R * sin(ph), C->z}, g[3];
  orc_accel(C->P, x, g);
  return C->comp == 0 ? g[0] * cos(ph) + g[1] * sin(ph) : g[2];
}

/* azimuth average of F_R (comp 0) or F_z (comp 1) at (R, z) */
static double jn_favg(const orc_pot* P, double R, double z, int comp, double tol) {
  jn_ctx C = {P, R, z, tol, comp, 0.0, 0.0};
  return cm_adapt(jn_fphi, &C, 0.0, 2.0 * M_PI, tol, 1e-300, 0) / (2.0 * M_PI);
}

static double jn_fs(void* c, double s) {
  jn_ctx* C = (jn_ctx*)c;
  return exp(-s) * -jn_favg(C->P, C->R, C->zabs + C->hz * s, 1, C->tol);
}

static double jn_sigz2(const orc_pot* P, double R, double z, double hz, double tol) {
  jn_ctx C = {P, R, 0.0, tol, 1, hz, fabs(z)};
  /* e^-s below 1e-30 of its start beyond s = 70 */
  double a = 0.0, s = 0.0;
  for (double b = 0.5; b <= 70.0; b *= 2.0) { /* panels [0,.5], [.5,1], [1,2], ... */
    a += cm_adapt(jn_fs, &C, s, b, tol, 1e-300, 0);
    s = b;
  }
  return hz * a;
}

void orc_jeans(const orc_pot* P, double hR, double hz, double b, long n, const double* pos, const double* eps,
               double* mom, double* ics) {
  const double tol = 1e-11;
  for (long i = 0; i < n; ++i) {
    double x = pos[i], y = pos[n + i], z = pos[2 * n + i];
    double R = sqrt(x * x + y * y), ph = atan2(y, x);
    double s0 = jn_sigz2(P, R, z, hz, tol);
    double h = 2e-3 * fmax(R, hz);
    double d1 = (jn_sigz2(P, R + h, z, hz, tol) - jn_sigz2(P, R - h, z, hz, tol)) / (2.0 * h);
    double d2 = (jn_sigz2(P, R + 0.5 * h, z, hz, tol) - jn_sigz2(P, R - 0.5 * h, z, hz, tol)) / h;
    double dsig = (4.0 * d2 - d1) / 3.0;
    double vcz2 = -R * jn_favg(P, R, z, 0, tol); /* circular speed^2 at the star's (R, z) */
    double vphi2 = b * (s0 * (1.0 - R / hR) + R * dsig) + vcz2;
    double sz = sqrt(fmax(s0, 0.0)), sR = sqrt(b) * sz, sp = sR;
    double vc = sqrt(fmax(vphi2 - b * s0, 0.0));
    mom[i] = sR;
    mom[n + i] = sp;
    mom[2 * n + i] = sz;
    mom[3 * n + i] = vc;
    mom[4 * n + i] = sqrt(fmax(vcz2, 0.0));
    double vR = sR * eps[i], vp = vc + sp * eps[n + i], vz = sz * eps[2 * n + i];
    ics[i] = x;
    ics[n + i] = y;
    ics[2 * n + i] = z;
    ics[3 * n + i] = vR * cos(ph) - vp * sin(ph);
    ics[4 * n + i] = vR * sin(ph) + vp * cos(ph);
    ics[5 * n + i] = vz;
  }
}

/* ------------------------------------------------------------------ */
/* Adaptive Bogacki-Shampine 3(2) integration (Sec. 2.2.2) with a fixed */
/* number of accepted steps, and the time-weighted binning of Sec.      */
/* 2.2.4: the state after accepted step k is a sample of weight         */
/* dt_k / t_total, t_total the sum of the accepted steps.               */
/* Equations of motion in the bar frame, (x, p) with p the inertial     */
/* velocity on the rotating axes:                                       */
/*   dx/dt = p + Omega (y, -x, 0),  dp/dt = -grad Phi + Omega (p_y, -p_x, 0). */
/* Error per step: max_i |y3_i - y2_i| / (atol + rtol max(|y_i|, |y3_i|)); */
/* accepted when <= 1; next step h min(5, max(0.2, 0.9 err^(-1/3))).     */
/* ------------------------------------------------------------------ */
static void bs_rhs(const orc_pot* P, const double* y, double* f) {
  double g[3];
  orc_accel(P, y, g);
  double W = P->omega;
  f[0] = y[3] + W * y[1];
  f[1] = y[4] - W * y[0];
  f[2] = y[5];
  f[3] = g[0] + W * y[4];
  f[4] = g[1] - W * y[3];
  f[5] = g[2];
}

/* one accepted step from y (k1 = f(y) on entry, f(y_new) on return); h is the
 * step tried first and, on return, the next one; returns the step taken, or 0
 * after 100 rejections in a row */
static double bs_step(const orc_pot* P, double* y, double* k1, double* h, double rtol, double atol) {
  for (int tries = 0; tries < 100; ++tries) {
    double hh = *h, t[6], k2[6], k3[6], y3[6], k4[6];
    for (int i = 0; i < 6; ++i) t[i] = y[i] + 0.5 * hh * k1[i];
    bs_rhs(P, t, k2);
    for (int i = 0; i < 6; ++i) t[i] = y[i] + 0.75 * hh * k2[i];
    bs_rhs(P, t, k3);
    for (int i = 0; i < 6; ++i) y3[i] = y[i] + hh * (2.0 / 9.0 * k1[i] + 1.0 / 3.0 * k2[i] + 4.0 / 9.0 * k3[i]);
    bs_rhs(P, y3, k4);
    double err = 0.0;
    for (int i = 0; i < 6; ++i) {
      double y2 = y[i] + hh * (7.0 / 24.0 * k1[i] + 0.25 * k2[i] + 1.0 / 3.0 * k3[i] + 0.125 * k4[i]);
      double sc = atol + rtol * fmax(fabs(y[i]), fabs(y3[i]));
      err = fmax(err, fabs(y3[i] - y2) / sc);
    }
    double fac = err > 0.0 ? 0.9 * pow(err, -1.0 / 3.0) : 5.0;
    fac = fmin(5.0, fmax(0.2, fac));
    if (err <= 1.0) {
      for (int i = 0; i < 6; ++i) { y[i] = y3[i]; k1[i] = k4[i]; }
      *h = hh * fac;
      return hh;
    }
    *h = hh * fac;
  }
  return 0.0;
}

void orc_orbit_bs23(const orc_pot* P, const double ic[6], double h0, int nsteps, double rtol, double atol,
                    double* traj, double* dts) {
  double y[6], k1[6], h = h0;
  for (int i = 0; i < 6; ++i) { y[i] = ic[i]; traj[i] = ic[i]; }
  bs_rhs(P, y, k1);
  for (int k = 1; k <= nsteps; ++k) {
    dts[k - 1] = bs_step(P, y, k1, &h, rtol, atol);
    for (int i = 0; i < 6; ++i) traj[6 * k + i] = y[i];
  }
}

void orc_integrate_bs23_and_bin(const orc_pot* P, const orc_obs* O, long n, const double* ics, const double* h0,
                                int nsteps, double rtol, double atol, double* A, double* overflow, double* drift,
                                uint8_t* flags, int nthreads) {
  int ncon = orc_ncon(O), nmass = O->nx * O->ny * O->nz, nkin = O->n_ap * O->nv;
  int ncopy = O->symmetrize ? 4 : 1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (long i = 0; i < n; ++i) {
    double y[6], k1[6], h = h0[i];
    for (int j = 0; j < 6; ++j) y[j] = ics[j * n + i];
    double* row = A + i * (long)ncon;
    for (int c = 0; c < ncon; ++c) row[c] = 0.0;
    double ovm = 0.0, ovk = 0.0, ttot = 0.0, E0 = orc_jacobi(P, y), dmax = 0.0;
    int bad = 0;
    bs_rhs(P, y, k1);
    for (int k = 1; k <= nsteps; ++k) {
      double dt = bs_step(P, y, k1, &h, rtol, atol);
      if (dt == 0.0) bad = 1;
      for (int j = 0; j < 6; ++j)
        if (!isfinite(y[j])) bad = 1;
      ttot += dt;
      for (int c = 0; c < ncopy; ++c) {
        int m, kc, a;
        cells_d(O, y, c, &m, &kc, &a);
        if (m >= 0) row[m] += dt; else ovm += dt;
        if (kc >= 0) row[nmass + kc] += dt; else ovk += dt;
        if (O->surface && a >= 0) row[nmass + nkin + a] += dt;
      }
      if (O->drift_every > 0 && k % O->drift_every == 0) {
        double e = fabs(orc_jacobi(P, y) / E0 - 1.0);
        if (!(e <= dmax)) dmax = e;
      }
    }
    double den = (double)ncopy * ttot;
    for (int c = 0; c < ncon; ++c) row[c] /= den;
    if (O->surface)
      for (int c = nmass + nkin; c < ncon; ++c) row[c] /= O->upsilon;
    overflow[2 * i] = ovm / den;
    overflow[2 * i + 1] = ovk / den;
    drift[i] = dmax;
    uint8_t f = 0;
    if (!(dmax <= 0.1)) f |= 1;
    if (bad) f |= 2;
    flags[i] = f;
  }
}
