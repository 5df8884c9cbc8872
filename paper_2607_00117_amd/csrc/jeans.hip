// Initial conditions of the orbit library (Sec. 2.2.1): velocities from the
// anisotropic Jeans equations, dithered realisations, and the bundle means of
// the orbit matrix.
//
// jeans_ics: at each starting position, the velocity dispersions and the
// mean rotation of a tracer with the fiducial density
// nu(R, z) ~ exp(-R/h_R - |z|/h_z) in the azimuth-averaged potential, then one
// Gaussian draw per velocity component.
//
// With the velocity ellipsoid aligned with (R, phi, z), sigma_R^2 = b sigma_z^2,
// sigma_phi = sigma_R and F the azimuth-averaged force:
//   sigma_z^2(R, z) = h_z int_0^inf e^-s (-F_z(R, |z| + h_z s)) ds   (vertical equation)
//   <v_phi^2> = b [sigma_z^2 (1 - R/h_R) + R d sigma_z^2/dR] - R F_R(R, z)   (radial equation)
//   mean v_phi = sqrt(max(<v_phi^2> - sigma_phi^2, 0)).
// The ln-nu gradients of the exponential tracer are constants, so only the
// force enters the integrals.  d/dR is the Richardson combination of central
// differences with steps h and h/2, h = 2e-3 max(R, h_z).
//
// One workgroup per position.  The s-integral uses 13 panels with edges 0 and
// 2^-6 .. 2^6 (fine near s = 0, where a thin disc's force turns over), each with
// an 8-point Gauss-Legendre rule; the azimuth average is the 128-point
// trapezoid rule (periodic integrand).  The lanes own (s, phi) node pairs and
// evaluate the force at the five radii; the workgroup adds the partial sums by
// a fixed tree.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "common.h"
#include "potential.h"

namespace sw {
namespace {

constexpr int kJnThreads = 256;
constexpr int kJnQ = 8;
constexpr int kJnPanels = 13;
constexpr int kJnS = kJnQ * kJnPanels;
constexpr int kJnPhi = 128;
constexpr int kJnSums = 6;  // sigma_z^2 integrals at R - h, R - h/2, R, R + h/2, R + h; F_R at (R, z)

struct JeansK {
  double hR, hz, b;
  double gt[kJnQ], gw[kJnQ];  // Gauss-Legendre rule on [-1, 1]
};

__device__ __forceinline__ double panel_edge(int k) { return k == 0 ? 0.0 : ldexp(1.0, k - 7); }

template <bool NB>
__global__ __launch_bounds__(kJnThreads) void k_jeans(PotK P, JeansK K, const double* __restrict__ pos,
                                                       const double* __restrict__ eps, int64_t n,
                                                       double* __restrict__ mom, double* __restrict__ ics) {
  __shared__ double red[kJnSums][kJnThreads];
  const int64_t i = blockIdx.x;
  const int tid = threadIdx.x;
  const double x = pos[i], y = pos[n + i], z = pos[2 * n + i];
  const double R = sqrt(x * x + y * y), az = fabs(z);
  const double h = 2e-3 * fmax(R, K.hz);
  const double radii[5] = {R - h, R - 0.5 * h, R, R + 0.5 * h, R + h};
  double acc[kJnSums];
#pragma unroll
  for (int r = 0; r < kJnSums; ++r) acc[r] = 0.0;
  for (int p = tid; p < kJnS * kJnPhi; p += kJnThreads) {
    const int j = p / kJnPhi, k = p % kJnPhi;
    const int pj = j / kJnQ, q = j % kJnQ;
    const double e0 = panel_edge(pj), e1 = panel_edge(pj + 1);
    const double half = 0.5 * (e1 - e0), s = 0.5 * (e0 + e1) + half * K.gt[q];
    const double ws = half * K.gw[q] * exp(-s);
    double sp, cp;
    sincospi((double)k * (2.0 / kJnPhi), &sp, &cp);
    const double zz = az + K.hz * s;
#pragma unroll
    for (int r = 0; r < 5; ++r) {
      const double xv[3] = {radii[r] * cp, radii[r] * sp, zz};
      double g[3];
      accel_f64<NB>(P, xv, g);
      acc[r] += ws * -g[2];
    }
  }
  for (int k = tid; k < kJnPhi; k += kJnThreads) {
    double sp, cp;
    sincospi((double)k * (2.0 / kJnPhi), &sp, &cp);
    const double xv[3] = {R * cp, R * sp, z};
    double g[3];
    accel_f64<NB>(P, xv, g);
    acc[5] += g[0] * cp + g[1] * sp;
  }
#pragma unroll
  for (int r = 0; r < kJnSums; ++r) red[r][tid] = acc[r];
  __syncthreads();
  for (int st = kJnThreads / 2; st > 0; st >>= 1) {
    if (tid < st) {
#pragma unroll
      for (int r = 0; r < kJnSums; ++r) red[r][tid] += red[r][tid + st];
    }
    __syncthreads();
  }
  if (tid == 0) {
    double sig[5];
#pragma unroll
    for (int r = 0; r < 5; ++r) sig[r] = K.hz * red[r][0] / kJnPhi;
    const double FR = red[5][0] / kJnPhi;
    const double d1 = (sig[4] - sig[0]) / (2.0 * h), d2 = (sig[3] - sig[1]) / h;
    const double dsig = (4.0 * d2 - d1) / 3.0;
    const double s0 = sig[2], b = K.b;
    const double vphi2 = b * (s0 * (1.0 - R / K.hR) + R * dsig) - R * FR;
    const double sz = sqrt(fmax(s0, 0.0)), sR = sqrt(b) * sz;
    const double mean = sqrt(fmax(vphi2 - b * s0, 0.0));
    mom[i] = sR;
    mom[n + i] = sR;
    mom[2 * n + i] = sz;
    mom[3 * n + i] = mean;
    mom[4 * n + i] = sqrt(fmax(-R * FR, 0.0));
    const double ph = atan2(y, x), c = cos(ph), sn = sin(ph);
    const double vR = sR * eps[i], vp = mean + sR * eps[n + i], vz = sz * eps[2 * n + i];
    ics[i] = x;
    ics[n + i] = y;
    ics[2 * n + i] = z;
    ics[3 * n + i] = vR * c - vp * sn;
    ics[4 * n + i] = vR * sn + vp * c;
    ics[5 * n + i] = vz;
  }
}

// realisation k of initial condition i -> column i nd + k: each coordinate
// moved by its deviate times dx (positions) or fv v_c (velocities); products
// and sums rounded separately
__global__ void k_dither(const double* __restrict__ ics, const double* __restrict__ vc, const double* __restrict__ u,
                         int64_t n, int32_t nd, double dx, double fv, double* __restrict__ out) {
#pragma clang fp contract(off)
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, m = n * nd;
  if (j >= m) return;
  const int64_t i = j / nd, k = j % nd;
  for (int c = 0; c < 6; ++c) {
    const double scale = c < 3 ? dx : fv * vc[i];
    out[c * m + j] = ics[c * n + i] + u[(k * 6 + c) * n + i] * scale;
  }
}

// bundle row b = mean of rows b nd .. b nd + nd - 1, summed in row order in FP64
template <typename T>
__global__ void k_bundle(const T* __restrict__ A, int64_t nb, int64_t C, int32_t nd, T* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nb * C) return;
  const int64_t b = idx / C, c = idx % C;
  const T* a = A + (b * nd) * C + c;
  double s = (double)a[0];
  for (int k = 1; k < nd; ++k) s = s + (double)a[(int64_t)k * C];
  out[idx] = (T)(s / nd);
}

// n-point Gauss-Legendre rule on [-1, 1] by Newton's iteration on P_n
void gl_rule(int n, double* t, double* w) {
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

extern "C" int jeans_ics(const sw_potential* pot, const double* pos, const double* eps, int64_t n, double h_R,
                         double h_z, double b, double* moments, double* ics, void* stream) {
  SW_CHECK(pot, "jeans_ics: null potential");
  SW_CHECK(n >= 0 && n <= 0x7fffffff, "jeans_ics: n must be in [0, 2^31)");
  SW_CHECK(std::isfinite(h_R) && h_R > 0.0 && std::isfinite(h_z) && h_z > 0.0,
           "jeans_ics: tracer scale lengths must be finite and > 0");
  SW_CHECK(std::isfinite(b) && b > 0.0, "jeans_ics: b = sigma_R^2 / sigma_z^2 must be finite and > 0");
  if (n == 0) return SW_OK;
  SW_CHECK(pos && eps && moments && ics, "jeans_ics: null device buffer");
  PotK P;
  std::memcpy(&P, pot, sizeof P);
  SW_CHECK(P.n_comp >= 1 && P.n_comp <= SW_MAX_COMP, "jeans_ics: potential not built");
  bool nb = false;
  for (int c = 0; c < P.n_comp; ++c) nb = nb || P.comp[c].kind == SW_DA_T3 || P.comp[c].kind == SW_DA_V4;
  JeansK K;
  std::memset(&K, 0, sizeof K);
  K.hR = h_R;
  K.hz = h_z;
  K.b = b;
  gl_rule(kJnQ, K.gt, K.gw);
  hipStream_t st = (hipStream_t)stream;
  if (nb)
    hipLaunchKernelGGL(k_jeans<true>, dim3((unsigned)n), dim3(kJnThreads), 0, st, P, K, pos, eps, n, moments, ics);
  else
    hipLaunchKernelGGL(k_jeans<false>, dim3((unsigned)n), dim3(kJnThreads), 0, st, P, K, pos, eps, n, moments, ics);
  SW_HIP(hipGetLastError());
  return SW_OK;
}

extern "C" int dither_ics(const double* ics, const double* vc, const double* u, int64_t n, int32_t n_dither, double dx,
                          double fv, double* out, void* stream) {
  SW_CHECK(n >= 0 && n_dither >= 1 && n_dither <= 64, "dither_ics: need n >= 0 and 1 <= n_dither <= 64");
  SW_CHECK(std::isfinite(dx) && dx >= 0.0 && std::isfinite(fv) && fv >= 0.0, "dither_ics: box sizes must be >= 0");
  if (n == 0) return SW_OK;
  SW_CHECK(ics && vc && u && out, "dither_ics: null device buffer");
  const int64_t m = n * n_dither;
  SW_CHECK((m + 255) / 256 <= 0x7fffffff, "dither_ics: too many realisations for one launch");
  hipLaunchKernelGGL(k_dither, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, (hipStream_t)stream, ics, vc, u, n,
                     n_dither, dx, fv, out);
  SW_HIP(hipGetLastError());
  return SW_OK;
}

extern "C" int bundle_rows(const void* A, int32_t dtype, int64_t n_bundle, int64_t n_con, int32_t n_dither, void* out,
                           void* stream) {
  SW_CHECK(dtype == SW_F32 || dtype == SW_F64, "bundle_rows: dtype must be SW_F32 or SW_F64");
  SW_CHECK(n_bundle >= 0 && n_con >= 0 && n_dither >= 1, "bundle_rows: need n_bundle, n_con >= 0, n_dither >= 1");
  const int64_t m = n_bundle * n_con;
  if (m == 0) return SW_OK;
  SW_CHECK(A && out && A != out, "bundle_rows: null or aliased device buffer");
  SW_CHECK((m + 255) / 256 <= 0x7fffffff, "bundle_rows: too many entries for one launch");
  const dim3 grid((unsigned)((m + 255) / 256));
  hipStream_t st = (hipStream_t)stream;
  if (dtype == SW_F32)
    hipLaunchKernelGGL(k_bundle<float>, grid, dim3(256), 0, st, (const float*)A, n_bundle, n_con, n_dither,
                       (float*)out);
  else
    hipLaunchKernelGGL(k_bundle<double>, grid, dim3(256), 0, st, (const double*)A, n_bundle, n_con, n_dither,
                       (double*)out);
  SW_HIP(hipGetLastError());
  return SW_OK;
}
