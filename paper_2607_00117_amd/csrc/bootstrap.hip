// Bootstrap realisations of the observed maps and the bootstrap-marginalised
// chi^2 (Sec. 2.3-2.4, Eq. 6).
//
// Each realisation perturbs the observed surface-density and kinematic
// constraints by their measurement errors (normal deviates times sigma); the
// intrinsic density constraint is fixed by the trial potential and is left as
// it is.  The realisations share the orbit matrix, so their weight problems are
// solved together by solve_weights_multi.  Eq. 6 then combines the chi^2 of
// the realisations' weights; its printed form (a log-sum-exp of chi2_min - chi2_b
// plus a constant) does not grow with the fit's chi^2, so it is read as the
// log-mean-exp marginalisation
//   chi2_model = chi2_min - 2 ln[(1/B) sum_b exp(-(chi2_b - chi2_min) / 2)],
// which lies in [chi2_min, chi2_min + 2 ln B] and equals chi2 when every
// chi2_b does.
#include <hip/hip_runtime.h>

#include <cmath>

#include "common.h"

namespace sw {

// out[b][n] = d[n] + sigma[n] eps[b][n] for n in [cb, ce), else d[n]; the
// product and the sum are rounded separately (contraction to a fused
// multiply-add is switched off), so each value is the FP64 evaluation of that
// expression as written
__global__ void k_bootstrap_data(const double* __restrict__ d, const double* __restrict__ sigma,
                                 const double* __restrict__ eps, int64_t C, int64_t cb, int64_t ce,
                                 double* __restrict__ out) {
#pragma clang fp contract(off)
  const int64_t b = blockIdx.y;
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= C) return;
  const double e = sigma[n] * eps[b * C + n];
  out[b * C + n] = (n >= cb && n < ce) ? d[n] + e : d[n];
}

}  // namespace sw

using namespace sw;

extern "C" int bootstrap_data(const double* d, const double* sigma, const double* eps, int64_t n_con, int32_t n_rhs,
                              int64_t col_begin, int64_t col_end, double* out, void* stream) {
  SW_CHECK(n_con > 0 && n_rhs >= 1, "bootstrap_data: need n_con > 0 and n_rhs >= 1");
  SW_CHECK(n_rhs <= 65535, "bootstrap_data: at most 65535 realisations per call");
  SW_CHECK(col_begin >= 0 && col_begin <= col_end && col_end <= n_con, "bootstrap_data: bad column range");
  SW_CHECK(d && sigma && eps && out, "bootstrap_data: null argument");
  const dim3 grid((unsigned)((n_con + 255) / 256), (unsigned)n_rhs);
  hipLaunchKernelGGL(k_bootstrap_data, grid, dim3(256), 0, (hipStream_t)stream, d, sigma, eps, n_con, col_begin,
                     col_end, out);
  SW_HIP(hipGetLastError());
  return SW_OK;
}

extern "C" int chi2_model(const double* chi2_b, int32_t n, double* out) {
  SW_CHECK(chi2_b && out && n >= 1, "chi2_model: need n >= 1 values and an output");
  double lo = chi2_b[0];
  for (int32_t b = 0; b < n; ++b) {
    SW_CHECK(std::isfinite(chi2_b[b]) && chi2_b[b] >= 0.0, "chi2_model: chi2 values must be finite and >= 0");
    lo = std::fmin(lo, chi2_b[b]);
  }
  // every term is in (0, 1] and the minimum contributes exactly 1
  double s = 0.0;
  for (int32_t b = 0; b < n; ++b) s += std::exp(-0.5 * (chi2_b[b] - lo));
  *out = lo - 2.0 * std::log(s / (double)n);
  return SW_OK;
}
