// Target cell masses m*_n (Sec. 2.2.4): the mass of the model's stellar
// density in each cell of the self-consistency grid, the constraint the orbit
// weights must reproduce.
//
// One workgroup per cell.  The cell is cut into n_sub^3 boxes in its own
// coordinates ((x, y, z), or (R, phi, z) with the Jacobian R) and each box
// takes an 8 x 8 x 8 Gauss-Legendre rule.  The lanes own (u, v) columns of the
// rule and sum the density along z in order; the workgroup adds the lanes'
// sums by a fixed tree, so a cell's value does not depend on timing.
//
// Densities of the selected components, in Msun / kpc^3 (closed forms):
//   Plummer   3M/(4 pi) b^2 (b^2 + r^2)^(-5/2)
//   isochrone M [3 (b + s) s^2 - r^2 (b + 3 s)] / (4 pi (b + s)^3 s^3), s^2 = b^2 + r^2
//   MN        (Eq. 11) b^2 M/(4 pi) [a R^2 + (a + 3 zeta)(a + zeta)^2] / ((R^2 + (a + zeta)^2)^(5/2) zeta^3)
//   Ferrers   rho_c (1 - m^2)^2 inside m < 1
//   T3, V4    App. A's parent densities with R^-n replaced by the needle integral I_n (Eq. 12)
// A point mass (Kepler) has no density and the NFW halo is not stellar (its
// flattened potential has no closed-form density); both are rejected.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "common.h"
#include "potential.h"

namespace sw {
namespace {

constexpr int kCmQ = 8;        // Gauss-Legendre nodes per box and dimension
constexpr int kCmMaxSub = 16;  // boxes per cell and dimension
constexpr int kCmThreads = 256;

struct CellK {
  int32_t nx, ny, nz, cyl, n_sub;
  uint32_t mask;
  double lo[3], w[3];          // first edge and cell width per coordinate (cylindrical: R, phi, z)
  double gt[kCmQ], gw[kCmQ];   // Gauss-Legendre rule on [-1, 1]
};

// App. A densities of the needle bars, I_n = J[(n - 1) / 2]
template <int KIND>
__device__ double needle_density(const PotK& P, const CompK& C, double x, double y, double z) {
  constexpr int NK = KIND == SW_DA_T3 ? 5 : 7;
  const double M = C.c[0] / kG, a = C.c[1], b2 = C.c[2], L = C.c[3], eta = C.c[4];
  const double zeta = sqrt(z * z + b2), Z = a + zeta;
  const double c = sqrt(y * y + Z * Z);
  double J[NK], X[NK];
  needle_sums<double, NK, kGL64>(P.gq64, P.gw64, x, c, L, eta, J, X);
  const double Z2 = Z * Z, Z4 = Z2 * Z2, e = zeta, e2 = e * e;
  if constexpr (KIND == SW_DA_T3) {
    return (M * b2 / (4.0 * M_PI)) * (3.0 * J[2] + 5.0 * a * Z2 * (3.0 * e2 - 2.0 * a * e + a * a) / (e2 * e) * J[3] +
                                      35.0 * a * a * Z4 / e2 * J[4]);
  } else {
    const double a2 = a * a, a3 = a2 * a;
    return (3.0 * M * b2 * b2 / (8.0 * M_PI)) *
           (5.0 * J[3] +
            7.0 * a * Z2 * (5.0 * e2 * e2 - 4.0 * a * e2 * e + 3.0 * a2 * e2 - 2.0 * a3 * e + a2 * a2) / (e2 * e2 * e) *
                J[4] +
            63.0 * a2 * Z4 * (2.0 * e2 - 2.0 * a * e + a2) / (e2 * e2) * J[5] + 231.0 * a3 * Z4 * Z2 / (e2 * e) * J[6]);
  }
}

template <bool NB>
__device__ double stellar_density(const PotK& P, uint32_t mask, double x, double y, double z) {
  double rho = 0.0;
  const double r2 = x * x + y * y + z * z;
  for (int i = 0; i < P.n_comp; ++i) {
    if (!((mask >> i) & 1u)) continue;
    const CompK& C = P.comp[i];
    const double M = C.c[0] / kG;
    switch (C.kind) {
      case SW_PLUMMER: {
        const double b2 = C.c[1], q = b2 + r2, iq = 1.0 / q;
        rho += (3.0 * M / (4.0 * M_PI)) * b2 * iq * iq / sqrt(q);
        break;
      }
      case SW_ISOCHRONE: {
        const double b = C.c[1], s = sqrt(C.c[2] + r2), bs = b + s;
        rho += M * (3.0 * bs * s * s - r2 * (b + 3.0 * s)) / (4.0 * M_PI * bs * bs * bs * s * s * s);
        break;
      }
      case SW_MN: {
        const double a = C.c[1], b2 = C.c[2];
        const double R2 = x * x + y * y, zeta = sqrt(z * z + b2), az = a + zeta;
        const double D = R2 + az * az;
        rho += (b2 * M / (4.0 * M_PI)) * (a * R2 + (a + 3.0 * zeta) * az * az) / (D * D * sqrt(D) * zeta * zeta * zeta);
        break;
      }
      case SW_FERRERS2: {
        const double m2 = x * x / C.c[0] + y * y / C.c[1] + z * z / C.c[2];
        if (m2 < 1.0) {
          const double rho_c = C.c[4] / (2.0 * M_PI * kG * sqrt(C.c[0] * C.c[1] * C.c[2]));
          rho += rho_c * (1.0 - m2) * (1.0 - m2);
        }
        break;
      }
      case SW_DA_T3:
        if constexpr (NB) rho += needle_density<SW_DA_T3>(P, C, x, y, z);
        break;
      case SW_DA_V4:
        if constexpr (NB) rho += needle_density<SW_DA_V4>(P, C, x, y, z);
        break;
      default:
        break;
    }
  }
  return rho;
}

template <bool NB>
__global__ __launch_bounds__(kCmThreads) void k_cell_mass(PotK P, CellK K, double* __restrict__ out) {
  __shared__ double red[kCmThreads];
  const int cell = blockIdx.x;
  const int iz = cell % K.nz, iy = (cell / K.nz) % K.ny, ix = cell / (K.nz * K.ny);
  const int nu = kCmQ * K.n_sub;
  const double h0 = K.w[0] / K.n_sub, h1 = K.w[1] / K.n_sub, h2 = K.w[2] / K.n_sub;
  const double u0 = K.lo[0] + ix * K.w[0], v0 = K.lo[1] + iy * K.w[1], z0 = K.lo[2] + iz * K.w[2];
  double acc = 0.0;
  for (int col = threadIdx.x; col < nu * nu; col += kCmThreads) {
    const int iu = col / nu, iv = col % nu;
    const double u = u0 + h0 * ((iu / kCmQ) + 0.5 + 0.5 * K.gt[iu % kCmQ]);
    const double v = v0 + h1 * ((iv / kCmQ) + 0.5 + 0.5 * K.gt[iv % kCmQ]);
    double wuv = 0.25 * h0 * h1 * K.gw[iu % kCmQ] * K.gw[iv % kCmQ];
    double x = u, y = v;
    if (K.cyl) {
      double s, c;
      sincos(v, &s, &c);
      x = u * c;
      y = u * s;
      wuv *= u;
    }
    double colsum = 0.0;
    for (int k = 0; k < nu; ++k) {
      const double z = z0 + h2 * ((k / kCmQ) + 0.5 + 0.5 * K.gt[k % kCmQ]);
      colsum += (0.5 * h2 * K.gw[k % kCmQ]) * stellar_density<NB>(P, K.mask, x, y, z);
    }
    acc += wuv * colsum;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kCmThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[cell] = red[0];
}

// n-point Gauss-Legendre rule on [-1, 1]: Newton's iteration on P_n from the
// Chebyshev-like first guess cos(pi (i + 3/4) / (n + 1/2))
void gauss_legendre(int n, double* t, double* w) {
  for (int i = 0; i < n; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    t[i] = -x;
    w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
}

}  // namespace
}  // namespace sw

using namespace sw;

extern "C" int cell_masses(const sw_potential* pot, const sw_obs_spec* obs, uint32_t comp_mask, int32_t n_sub,
                           double* out, void* stream) {
  SW_CHECK(pot && obs && out, "cell_masses: null argument");
  SW_CHECK(n_sub >= 1 && n_sub <= kCmMaxSub, "cell_masses: n_sub must be in [1, %d]", kCmMaxSub);
  PotK P;
  std::memcpy(&P, pot, sizeof P);
  SW_CHECK(P.n_comp >= 1 && P.n_comp <= SW_MAX_COMP, "cell_masses: potential not built");
  SW_CHECK(comp_mask != 0 && (comp_mask >> P.n_comp) == 0, "cell_masses: component mask selects no or missing components");
  bool nb = false;
  for (int i = 0; i < P.n_comp; ++i) {
    if (!((comp_mask >> i) & 1u)) continue;
    const int k = P.comp[i].kind;
    SW_CHECK(k == SW_PLUMMER || k == SW_ISOCHRONE || k == SW_MN || k == SW_FERRERS2 || k == SW_DA_T3 || k == SW_DA_V4,
             "cell_masses: component %d (kind %d) has no stellar density", i, k);
    nb = nb || k == SW_DA_T3 || k == SW_DA_V4;
  }
  SW_CHECK(obs->nx >= 1 && obs->ny >= 1 && obs->nz >= 1, "cell_masses: grid dimensions must be >= 1");
  SW_CHECK(obs->grid == SW_GRID_CARTESIAN || obs->grid == SW_GRID_CYLINDRICAL, "cell_masses: unknown grid type");
  const int64_t n_cells = (int64_t)obs->nx * obs->ny * obs->nz;
  SW_CHECK(n_cells <= 0x7fffffff, "cell_masses: too many cells");
  CellK K;
  std::memset(&K, 0, sizeof K);
  K.nx = obs->nx;
  K.ny = obs->ny;
  K.nz = obs->nz;
  K.cyl = obs->grid == SW_GRID_CYLINDRICAL;
  K.n_sub = n_sub;
  K.mask = comp_mask;
  const int32_t n[3] = {obs->nx, obs->ny, obs->nz};
  for (int d = 0; d < 3; ++d) {
    SW_CHECK((std::isfinite(obs->lo[d]) && std::isfinite(obs->hi[d]) && obs->hi[d] > obs->lo[d]) ||
                 (K.cyl && d == 1),
             "cell_masses: need finite lo < hi on axis %d", d);
    K.lo[d] = obs->lo[d];
    K.w[d] = (obs->hi[d] - obs->lo[d]) / n[d];
  }
  if (K.cyl) {
    SW_CHECK(obs->lo[0] >= 0.0, "cell_masses: cylindrical grid needs lo[0] >= 0");
    K.lo[1] = -M_PI;
    K.w[1] = 2.0 * M_PI / obs->ny;
  }
  gauss_legendre(kCmQ, K.gt, K.gw);
  hipStream_t st = (hipStream_t)stream;
  if (nb)
    hipLaunchKernelGGL(k_cell_mass<true>, dim3((unsigned)n_cells), dim3(kCmThreads), 0, st, P, K, out);
  else
    hipLaunchKernelGGL(k_cell_mass<false>, dim3((unsigned)n_cells), dim3(kCmThreads), 0, st, P, K, out);
  SW_HIP(hipGetLastError());
  return SW_OK;
}
