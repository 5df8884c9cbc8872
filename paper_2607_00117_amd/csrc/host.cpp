// Host-side entry points: build_potential, error reporting, observable checks.
#include <cmath>
#include <cstdarg>
#include <cstring>

#include "common.h"

namespace sw {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

int hip_fail(hipError_t e, const char* what) {
  set_error("HIP error %d (%s) in %s", (int)e, hipGetErrorString(e), what);
  return SW_EHIP;
}

// Gauss-Legendre nodes and weights on [-1, 1] by Newton iteration on P_n
// (three-term recurrence for P_n and its derivative).
static void gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
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
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// Nodes of the bar quadrature: t = (x + 1) / 2 on (0, 1), q = 1/t^2 - 1,
// W = (w / 2) * 2 / t^3.
template <typename T>
static void bar_rule(int n, T* q, T* W) {
  double x[64], w[64];
  gauss_legendre(n, x, w);
  for (int i = 0; i < n; ++i) {
    double t = 0.5 * (x[i] + 1.0);
    q[i] = (T)(1.0 / (t * t) - 1.0);
    W[i] = (T)(w[i] / (t * t * t));
  }
}

static void matmul3(const double A[9], const double B[9], double C[9]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s = s + A[3 * i + k] * B[3 * k + j];
      C[3 * i + j] = s;
    }
}

bool obs_to_k(const sw_obs_spec* o, ObsK* k) {
  if (!o) return false;
  if (o->nx <= 0 || o->ny <= 0 || o->nz <= 0 || o->npx <= 0 || o->npy <= 0 || o->nv <= 0) return false;
  for (int i = 0; i < 3; ++i)
    if (!(std::isfinite(o->lo[i]) && std::isfinite(o->hi[i]) && o->hi[i] > o->lo[i])) return false;
  for (int i = 0; i < 2; ++i)
    if (!(std::isfinite(o->plo[i]) && std::isfinite(o->phi[i]) && o->phi[i] > o->plo[i])) return false;
  if (!(std::isfinite(o->vlo) && std::isfinite(o->vhi) && o->vhi > o->vlo)) return false;
  if (o->drift_every < 0) return false;
  if (o->grid != SW_GRID_CARTESIAN && o->grid != SW_GRID_CYLINDRICAL) return false;
  if (o->grid == SW_GRID_CYLINDRICAL && (o->lo[0] < 0.0 || o->ny > kMaxSectors)) return false;
  int64_t n_ap = o->pix2ap ? o->n_ap : (int64_t)o->npx * o->npy;
  if (n_ap <= 0) return false;
  int64_t n_mass = (int64_t)o->nx * o->ny * o->nz, n_kin = n_ap * o->nv;
  if (n_mass >= 65535 || n_kin >= 65535) return false;
  if (o->surface != 0 && o->surface != 1) return false;
  if (o->surface && (!(std::isfinite(o->upsilon) && o->upsilon > 0.0) || n_kin + n_ap >= 65535)) return false;
  k->surface = o->surface;
  k->nx = o->nx; k->ny = o->ny; k->nz = o->nz;
  k->npx = o->npx; k->npy = o->npy; k->nv = o->nv;
  k->n_ap = (int32_t)n_ap;
  k->ncopy = o->symmetrize ? 4 : 1;
  k->n_mass = (int32_t)n_mass;
  k->n_kin = (int32_t)n_kin;
  const int32_t n3[3] = {o->nx, o->ny, o->nz};
  for (int i = 0; i < 3; ++i) {
    k->lo[i] = o->lo[i];
    k->inv[i] = n3[i] / (o->hi[i] - o->lo[i]);
  }
  const int32_t n2[2] = {o->npx, o->npy};
  for (int i = 0; i < 2; ++i) {
    k->plo[i] = o->plo[i];
    k->pinv[i] = n2[i] / (o->phi[i] - o->plo[i]);
  }
  k->vlo = o->vlo;
  k->vinv = o->nv / (o->vhi - o->vlo);
  for (int i = 0; i < 3; ++i) { k->lof[i] = (float)k->lo[i]; k->invf[i] = (float)k->inv[i]; }
  for (int i = 0; i < 2; ++i) { k->plof[i] = (float)k->plo[i]; k->pinvf[i] = (float)k->pinv[i]; }
  k->vlof = (float)k->vlo;
  k->vinvf = (float)k->vinv;
  k->pix2ap = o->pix2ap;
  k->drift_every = o->drift_every;
  k->cyl = o->grid == SW_GRID_CYLINDRICAL ? 1 : 0;
  k->rw = (o->hi[0] - o->lo[0]) / o->nx;
  k->rwf = (float)k->rw;
  for (int j = 0; j <= kMaxSectors; ++j) {
    const double ph = -M_PI + 2.0 * M_PI * j / (k->cyl ? o->ny : 1);
    k->sc[j] = j <= o->ny ? std::cos(ph) : 0.0;
    k->ss[j] = j <= o->ny ? std::sin(ph) : 0.0;
    k->scf[j] = (float)k->sc[j];
    k->ssf[j] = (float)k->ss[j];
  }
  return true;
}

}  // namespace sw

using namespace sw;

extern "C" const char* sw_last_error(void) { return g_err; }

static bool pos_finite(double v) { return std::isfinite(v) && v > 0.0; }

extern "C" int build_potential(const sw_potential_desc* in, sw_potential* out) {
  SW_CHECK(in && out, "build_potential: null argument");
  SW_CHECK(in->n_comp >= 1 && in->n_comp <= SW_MAX_COMP, "build_potential: n_comp=%d out of range", in->n_comp);
  SW_CHECK(std::isfinite(in->omega_b), "build_potential: non-finite pattern speed");
  for (int i = 0; i < 3; ++i) SW_CHECK(std::isfinite(in->euler[i]), "build_potential: non-finite Euler angle");
  PotK P;
  std::memset(&P, 0, sizeof P);
  P.n_comp = in->n_comp;
  for (int i = 0; i < in->n_comp; ++i) {
    const sw_component& c = in->comp[i];
    CompK& k = P.comp[i];
    k.kind = c.kind;
    const double* p = c.p;
    SW_CHECK(pos_finite(p[0]), "build_potential: component %d mass must be finite and > 0", i);
    double GM = kG * p[0];
    switch (c.kind) {
      case SW_KEPLER:
        k.c[0] = GM;
        break;
      case SW_ISOCHRONE:
        SW_CHECK(pos_finite(p[1]), "build_potential: isochrone b must be > 0");
        k.c[0] = GM; k.c[1] = p[1]; k.c[2] = p[1] * p[1];
        break;
      case SW_PLUMMER:
        SW_CHECK(pos_finite(p[1]), "build_potential: Plummer b must be > 0");
        k.c[0] = GM; k.c[1] = p[1] * p[1];
        break;
      case SW_MN:
        SW_CHECK(std::isfinite(p[1]) && p[1] >= 0.0 && pos_finite(p[2]),
                 "build_potential: Miyamoto-Nagai needs a >= 0, b > 0");
        k.c[0] = GM; k.c[1] = p[1]; k.c[2] = p[2] * p[2];
        break;
      case SW_NFW_Q: {
        SW_CHECK(pos_finite(p[1]) && pos_finite(p[2]), "build_potential: NFW needs c > 0, q > 0");
        SW_CHECK(std::isfinite(p[3]), "build_potential: NFW H0 must be finite");
        double H0 = p[3] > 0.0 ? p[3] : 70.0;
        double H = H0 / 1000.0;
        double rho_crit = 3.0 * H * H / (8.0 * M_PI * kG);
        double R200 = std::cbrt(3.0 * p[0] / (4.0 * M_PI * 200.0 * rho_crit));
        double Rs = R200 / p[1];
        double Mdm = p[0] / (std::log(1.0 + p[1]) - p[1] / (1.0 + p[1]));
        double q2 = p[2] * p[2];
        k.c[0] = kG * Mdm; k.c[1] = Rs; k.c[2] = 1.0 / q2; k.c[3] = q2;
        k.c[4] = kG * Mdm / (Rs * Rs); k.c[5] = 1.0 / Rs;
        break;
      }
      case SW_FERRERS2: {
        SW_CHECK(pos_finite(p[1]) && pos_finite(p[2]) && pos_finite(p[3]),
                 "build_potential: Ferrers axes must be > 0");
        double a = p[1], b = p[2], cc = p[3];
        double rho_c = 105.0 * p[0] / (32.0 * M_PI * a * b * cc);
        k.c[0] = a * a; k.c[1] = b * b; k.c[2] = cc * cc;
        k.c[3] = std::fmin(k.c[0], std::fmin(k.c[1], k.c[2]));
        k.c[4] = 2.0 * M_PI * kG * a * b * cc * rho_c;
        k.c[5] = M_PI * kG * a * b * cc * rho_c / 3.0;
        k.c[6] = std::fmax(k.c[0], std::fmax(k.c[1], k.c[2]));
        break;
      }
      case SW_DA_T3:
      case SW_DA_V4:
        SW_CHECK(std::isfinite(p[1]) && p[1] >= 0.0 && pos_finite(p[2]) && pos_finite(p[3]),
                 "build_potential: needle bar needs a >= 0, b > 0, L > 0");
        SW_CHECK(std::isfinite(p[4]) && p[4] >= -1.0 && p[4] <= 1.0, "build_potential: needle bar eta in [-1, 1]");
        k.c[0] = GM; k.c[1] = p[1]; k.c[2] = p[2] * p[2]; k.c[3] = p[3]; k.c[4] = p[4];
        k.c[5] = 1.0 / (2.0 * p[3]);
        break;
      default:
        SW_CHECK(false, "build_potential: unknown component kind %d", c.kind);
    }
  }
  for (int i = 0; i < in->n_comp; ++i)
    for (int j = 0; j < 12; ++j) P.comp[i].f[j] = (float)P.comp[i].c[j];
  P.omega = in->omega_b;
  // Eq. 1: R = R_z(gamma) R_x(beta) R_z(alpha), active right-handed rotations.
  double ca = std::cos(in->euler[0]), sa = std::sin(in->euler[0]);
  double cb = std::cos(in->euler[1]), sb = std::sin(in->euler[1]);
  double cg = std::cos(in->euler[2]), sg = std::sin(in->euler[2]);
  const double Rza[9] = {ca, -sa, 0, sa, ca, 0, 0, 0, 1};
  const double Rxb[9] = {1, 0, 0, 0, cb, -sb, 0, sb, cb};
  const double Rzg[9] = {cg, -sg, 0, sg, cg, 0, 0, 0, 1};
  double T[9];
  matmul3(Rxb, Rza, T);
  matmul3(Rzg, T, P.R);
  for (int i = 0; i < 9; ++i) P.Rf[i] = (float)P.R[i];
  bar_rule<float>(kGL32, P.gq32, P.gw32);
  bar_rule<double>(kGL64, P.gq64, P.gw64);
  std::memset(out, 0, sizeof *out);
  std::memcpy(out, &P, sizeof P);
  return SW_OK;
}
