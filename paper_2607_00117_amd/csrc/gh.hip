// Gauss-Hermite moments of the orbits' line-of-sight velocity histograms
// (Sec. 2.2.4, Eq. 2).
//
// Eq. 2 expands an LOSVD about a reference Gaussian (centre v0, width s) in the
// modified Hermite polynomials H_m (orthonormal: int alpha^2 H_m H_n dw =
// delta_mn / (2 sqrt(pi)), alpha(w) = exp(-w^2/2)/sqrt(2 pi)).  The linear
// moment g_m = 2 sqrt(pi) int f alpha(w) H_m(w) dv equals gamma h_m (g_0 =
// gamma), so the moments of a weighted orbit sum are the weighted sums of the
// orbits' moments.  A histogram bin is read as mass spread uniformly over the
// bin, so each orbit's moment is a fixed linear map of its velocity bins in
// each aperture: out[i][a][m] = sum_k G_a[m][k] A[i][kin0 + a nv + k].
// G is built on the host in closed form: alpha H_m is a polynomial times the
// normal density, whose integrals over [w_k, w_k+1] follow from
//   I_0 = Phi(b) - Phi(a),  I_1 = phi(a) - phi(b),
//   I_j = [w^{j-1} phi(w)]_b^a + (j - 1) I_{j-2}.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "common.h"

namespace sw {

constexpr int kMaxGH = 8;

// coefficients of H_m(w) = sum_j c[m][j] w^j by the recurrence
// H_{m+1} = (sqrt(2) w H_m - sqrt(m) H_{m-1}) / sqrt(m + 1)
static void hermite_coefficients(int n_gh, double c[kMaxGH + 1][kMaxGH + 1]) {
  for (int m = 0; m <= kMaxGH; ++m)
    for (int j = 0; j <= kMaxGH; ++j) c[m][j] = 0.0;
  c[0][0] = 1.0;
  if (n_gh >= 1) c[1][1] = std::sqrt(2.0);
  for (int m = 1; m < n_gh; ++m)
    for (int j = 0; j <= m + 1; ++j) {
      const double up = j > 0 ? std::sqrt(2.0) * c[m][j - 1] : 0.0;
      c[m + 1][j] = (up - std::sqrt((double)m) * c[m - 1][j]) / std::sqrt((double)(m + 1));
    }
}

// G[m][k] for one aperture: 2 sqrt(pi) (s / dv) int_{w_k}^{w_k+1} phi(w) H_m(w) dw
static void bin_kernel(double vlo, double vhi, int nv, double v0, double s, int n_gh,
                       const double c[kMaxGH + 1][kMaxGH + 1], double* G) {
  const double dv = (vhi - vlo) / nv;
  const double inv_sqrt2pi = 1.0 / std::sqrt(2.0 * M_PI);
  for (int k = 0; k < nv; ++k) {
    const double a = (vlo + k * dv - v0) / s, b = (vlo + (k + 1) * dv - v0) / s;
    const double pa = inv_sqrt2pi * std::exp(-0.5 * a * a), pb = inv_sqrt2pi * std::exp(-0.5 * b * b);
    double I[kMaxGH + 1];
    I[0] = 0.5 * (std::erfc(-b / std::sqrt(2.0)) - std::erfc(-a / std::sqrt(2.0)));
    if (n_gh >= 1) I[1] = pa - pb;
    double wa = 1.0, wb = 1.0;  // a^{j-1}, b^{j-1}
    for (int j = 2; j <= n_gh; ++j) {
      wa *= a;
      wb *= b;
      I[j] = wa * pa - wb * pb + (j - 1) * I[j - 2];
    }
    for (int m = 0; m <= n_gh; ++m) {
      double acc = 0.0;
      for (int j = 0; j <= m; ++j) acc += c[m][j] * I[j];
      G[(size_t)m * nv + k] = 2.0 * std::sqrt(M_PI) * (s / dv) * acc;
    }
  }
}

// one thread per (orbit, aperture); G_a = G + a (n_gh + 1) nv
template <typename TA>
__global__ __launch_bounds__(256) void k_gh_moments(const TA* __restrict__ A, int64_t n_orb, int64_t n_con,
                                                    int64_t kin0, int32_t n_ap, int32_t nv, int32_t n_gh,
                                                    const double* __restrict__ G, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_orb * n_ap) return;
  const int64_t i = t / n_ap;
  const int a = (int)(t - i * n_ap);
  const TA* row = A + i * n_con + kin0 + (int64_t)a * nv;
  const double* Ga = G + (size_t)a * (n_gh + 1) * nv;
  double acc[kMaxGH + 1];
#pragma unroll
  for (int m = 0; m <= kMaxGH; ++m) acc[m] = 0.0;
  for (int k = 0; k < nv; ++k) {
    const double v = (double)row[k];
    if (v == 0.0) continue;
#pragma unroll
    for (int m = 0; m <= kMaxGH; ++m)
      if (m <= n_gh) acc[m] += Ga[(size_t)m * nv + k] * v;
  }
  double* o = out + t * (n_gh + 1);
#pragma unroll
  for (int m = 0; m <= kMaxGH; ++m)
    if (m <= n_gh) o[m] = acc[m];
}

// Rows of the fit matrix (Eq. 3): the mass block and the surface-density
// columns copied, out[i][0, n_mass) = A[i][0, n_mass), out[i][n_mass + a] =
// A[i][surf0 + a] (surf0 >= 0).  One thread per output entry.
template <typename TA>
__global__ __launch_bounds__(256) void k_fit_copy(const TA* __restrict__ A, int64_t n_orb, int64_t n_con,
                                                  int64_t n_mass, int64_t surf0, int32_t n_sigma, int64_t n_out,
                                                  TA* __restrict__ out) {
  const int64_t w = n_mass + n_sigma;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_orb * w) return;
  const int64_t i = t / w, c = t - i * w;
  out[i * n_out + c] = c < n_mass ? A[i * n_con + c] : A[i * n_con + surf0 + (c - n_mass)];
}

// The Gauss-Hermite block of the fit matrix: out[i][h0 + (m - 1) n_ap + a] =
// g_m(i, a) / gamma[a], m = 1..n_gh, one thread per (orbit, aperture).
template <typename TA>
__global__ __launch_bounds__(256) void k_fit_gh(const TA* __restrict__ A, int64_t n_orb, int64_t n_con, int64_t kin0,
                                                int32_t n_ap, int32_t nv, int32_t n_gh, const double* __restrict__ G,
                                                const double* __restrict__ inv_gamma, int64_t h0, int64_t n_out,
                                                TA* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_orb * n_ap) return;
  const int64_t i = t / n_ap;
  const int a = (int)(t - i * n_ap);
  const TA* row = A + i * n_con + kin0 + (int64_t)a * nv;
  const double* Ga = G + (size_t)a * (n_gh + 1) * nv;
  double acc[kMaxGH + 1];
#pragma unroll
  for (int m = 0; m <= kMaxGH; ++m) acc[m] = 0.0;
  for (int k = 0; k < nv; ++k) {
    const double v = (double)row[k];
    if (v == 0.0) continue;
#pragma unroll
    for (int m = 1; m <= kMaxGH; ++m)
      if (m <= n_gh) acc[m] += Ga[(size_t)m * nv + k] * v;
  }
  TA* o = out + i * n_out + h0 + a;
  const double ig = inv_gamma[a];
#pragma unroll
  for (int m = 1; m <= kMaxGH; ++m)
    if (m <= n_gh) o[(int64_t)(m - 1) * n_ap] = (TA)(acc[m] * ig);
}

}  // namespace sw

using namespace sw;

extern "C" size_t gh_workspace_bytes(int32_t n_ap, int32_t nv, int32_t n_gh) {
  if (n_ap < 1 || nv < 1 || n_gh < 0 || n_gh > kMaxGH) return 0;
  return (size_t)n_ap * (n_gh + 1) * nv * sizeof(double);
}

extern "C" int gh_moments(const void* A, int32_t dtype, int64_t n_orb, int64_t n_con, int64_t kin0, int32_t n_ap,
                          int32_t nv, double vlo, double vhi, const double* v0, const double* s, int32_t n_gh,
                          double* out, void* workspace, size_t ws_bytes, void* stream) {
  SW_CHECK(dtype == SW_F32 || dtype == SW_F64, "gh_moments: dtype must be SW_F32 or SW_F64");
  SW_CHECK(n_orb >= 0 && n_ap >= 1 && nv >= 1, "gh_moments: need n_orb >= 0, n_ap >= 1, nv >= 1");
  SW_CHECK(n_gh >= 0 && n_gh <= kMaxGH, "gh_moments: n_gh in [0, %d]", kMaxGH);
  SW_CHECK(kin0 >= 0 && kin0 + (int64_t)n_ap * nv <= n_con, "gh_moments: kinematic block beyond n_con");
  SW_CHECK(std::isfinite(vlo) && std::isfinite(vhi) && vhi > vlo, "gh_moments: need vhi > vlo");
  SW_CHECK(v0 && s, "gh_moments: null v0 / s");
  for (int a = 0; a < n_ap; ++a)
    SW_CHECK(std::isfinite(v0[a]) && std::isfinite(s[a]) && s[a] > 0.0, "gh_moments: aperture %d needs s > 0", a);
  const size_t need = gh_workspace_bytes(n_ap, nv, n_gh);
  if (ws_bytes < need || !workspace) {
    set_error("gh_moments: workspace of %zu bytes, %zu needed", ws_bytes, need);
    return SW_ENOMEM;
  }
  if (n_orb == 0) return SW_OK;
  SW_CHECK(A && out, "gh_moments: null device buffer");
  double c[kMaxGH + 1][kMaxGH + 1];
  hermite_coefficients(n_gh, c);
  std::vector<double> G(need / sizeof(double));
  for (int a = 0; a < n_ap; ++a) bin_kernel(vlo, vhi, nv, v0[a], s[a], n_gh, c, G.data() + (size_t)a * (n_gh + 1) * nv);
  hipStream_t st = (hipStream_t)stream;
  SW_HIP(hipMemcpyAsync(workspace, G.data(), need, hipMemcpyHostToDevice, st));
  const int64_t n = n_orb * n_ap;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (dtype == SW_F32)
    hipLaunchKernelGGL(k_gh_moments<float>, dim3(blocks), dim3(256), 0, st, (const float*)A, n_orb, n_con, kin0, n_ap,
                       nv, n_gh, (const double*)workspace, out);
  else
    hipLaunchKernelGGL(k_gh_moments<double>, dim3(blocks), dim3(256), 0, st, (const double*)A, n_orb, n_con, kin0,
                       n_ap, nv, n_gh, (const double*)workspace, out);
  SW_HIP(hipGetLastError());
  // the host copy of G must outlive the transfer
  SW_HIP(hipStreamSynchronize(st));
  return SW_OK;
}

extern "C" size_t gh_fit_workspace_bytes(int32_t n_ap, int32_t nv, int32_t n_gh) {
  const size_t g = gh_workspace_bytes(n_ap, nv, n_gh);
  return g ? g + (size_t)n_ap * sizeof(double) : 0;
}

extern "C" int gh_fit_matrix(const void* A, int32_t dtype, int64_t n_orb, int64_t n_con, int64_t n_mass, int64_t kin0,
                             int64_t surf0, int32_t n_ap, int32_t nv, double vlo, double vhi, const double* v0,
                             const double* s, const double* gamma, int32_t n_gh, void* out, void* workspace,
                             size_t ws_bytes, void* stream) {
  SW_CHECK(dtype == SW_F32 || dtype == SW_F64, "gh_fit_matrix: dtype must be SW_F32 or SW_F64");
  SW_CHECK(n_orb >= 0 && n_ap >= 1 && nv >= 1, "gh_fit_matrix: need n_orb >= 0, n_ap >= 1, nv >= 1");
  SW_CHECK(n_gh >= 1 && n_gh <= kMaxGH, "gh_fit_matrix: n_gh in [1, %d]", kMaxGH);
  SW_CHECK(n_mass >= 0 && n_mass <= n_con, "gh_fit_matrix: mass block beyond n_con");
  SW_CHECK(kin0 >= 0 && kin0 + (int64_t)n_ap * nv <= n_con, "gh_fit_matrix: kinematic block beyond n_con");
  SW_CHECK(surf0 < 0 || surf0 + n_ap <= n_con, "gh_fit_matrix: surface block beyond n_con");
  SW_CHECK(std::isfinite(vlo) && std::isfinite(vhi) && vhi > vlo, "gh_fit_matrix: need vhi > vlo");
  SW_CHECK(v0 && s && gamma, "gh_fit_matrix: null v0 / s / gamma");
  for (int a = 0; a < n_ap; ++a) {
    SW_CHECK(std::isfinite(v0[a]) && std::isfinite(s[a]) && s[a] > 0.0, "gh_fit_matrix: aperture %d needs s > 0", a);
    SW_CHECK(std::isfinite(gamma[a]) && gamma[a] > 0.0, "gh_fit_matrix: aperture %d needs gamma > 0", a);
  }
  const size_t gbytes = gh_workspace_bytes(n_ap, nv, n_gh), need = gh_fit_workspace_bytes(n_ap, nv, n_gh);
  if (ws_bytes < need || !workspace) {
    set_error("gh_fit_matrix: workspace of %zu bytes, %zu needed", ws_bytes, need);
    return SW_ENOMEM;
  }
  if (n_orb == 0) return SW_OK;
  SW_CHECK(A && out, "gh_fit_matrix: null device buffer");
  double c[kMaxGH + 1][kMaxGH + 1];
  hermite_coefficients(n_gh, c);
  std::vector<double> G(gbytes / sizeof(double) + n_ap);
  for (int a = 0; a < n_ap; ++a) bin_kernel(vlo, vhi, nv, v0[a], s[a], n_gh, c, G.data() + (size_t)a * (n_gh + 1) * nv);
  for (int a = 0; a < n_ap; ++a) G[gbytes / sizeof(double) + a] = 1.0 / gamma[a];
  hipStream_t st = (hipStream_t)stream;
  SW_HIP(hipMemcpyAsync(workspace, G.data(), need, hipMemcpyHostToDevice, st));
  const double* Gd = (const double*)workspace;
  const double* ig = Gd + gbytes / sizeof(double);
  const int32_t n_sig = surf0 >= 0 ? n_ap : 0;
  const int64_t h0 = n_mass + n_sig, n_out = h0 + (int64_t)n_gh * n_ap;
  const int64_t nc = n_orb * (n_mass + n_sig), ng = n_orb * n_ap;
  if (dtype == SW_F32) {
    if (nc > 0)
      hipLaunchKernelGGL(k_fit_copy<float>, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, (const float*)A, n_orb,
                         n_con, n_mass, surf0, n_sig, n_out, (float*)out);
    hipLaunchKernelGGL(k_fit_gh<float>, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, st, (const float*)A, n_orb,
                       n_con, kin0, n_ap, nv, n_gh, Gd, ig, h0, n_out, (float*)out);
  } else {
    if (nc > 0)
      hipLaunchKernelGGL(k_fit_copy<double>, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, (const double*)A,
                         n_orb, n_con, n_mass, surf0, n_sig, n_out, (double*)out);
    hipLaunchKernelGGL(k_fit_gh<double>, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, st, (const double*)A, n_orb,
                       n_con, kin0, n_ap, nv, n_gh, Gd, ig, h0, n_out, (double*)out);
  }
  SW_HIP(hipGetLastError());
  SW_HIP(hipStreamSynchronize(st));  // the host copy of the maps must outlive the transfer
  return SW_OK;
}
