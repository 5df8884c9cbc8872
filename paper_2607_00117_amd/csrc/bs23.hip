// Adaptive orbit integration (Sec. 2.2.2: Bogacki-Shampine 3(2) with a fixed
// number of accepted steps) and time-weighted binning (Sec. 2.2.4: the sample
// after accepted step k weighs dt_k / t_total), in FP64.
//
// Two kernels:
//  1. k_bs23: one orbit per lane, in double or in single precision (the
//     single-precision force is the leapfrog integrator's: the bar's 16-node
//     rule, hardware reciprocals); the total time is summed and the Jacobi
//     drift evaluated in double either way.  Equations of motion in the bar frame for
//     (x, p), p the inertial velocity on the rotating axes:
//       dx/dt = p + Omega (y, -x, 0),  dp/dt = -grad Phi + Omega (p_y, -p_x, 0).
//     Per attempt: stages k2 = f(y + h/2 k1), k3 = f(y + 3h/4 k2), the third-order
//     solution y3 = y + h (2/9 k1 + 1/3 k2 + 4/9 k3), k4 = f(y3) (reused as the
//     next k1), the embedded second-order y2 = y + h (7/24 k1 + 1/4 k2 + 1/3 k3
//     + 1/8 k4); err = max_i |y3_i - y2_i| / (atol + rtol max(|y_i|, |y3_i|)),
//     accepted when err <= 1, next step h min(5, max(0.2, 0.9 err^(-1/3))); 100
//     rejections in a row end the orbit with the non-finite flag.  Every
//     accepted step appends its mirror copies' packed cells (as the leapfrog
//     path does) and its step to the orbit's streams.
//  2. k_hist_w: one workgroup per orbit and column window: each event's weight
//     dt_k / t_total is rounded to a 64-bit fixed-point integer in units of
//     2^-52 and added into an LDS histogram of integers, written as
//     sum / (copies 2^52) (divided by Upsilon for the surface block).  Integer
//     adds are exact, so the result does not depend on the order in which the
//     lanes add (repeated runs are identical to the bit); the rounding moves
//     each weight by at most 2^-53, under 1e-12 of an entry over 5,000 steps.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "common.h"
#include "potential.h"

namespace sw {
namespace {

constexpr int kBsWindow = 8000;  // histogram columns per pass (64 KB of doubles)

template <bool NB>
__device__ __forceinline__ void bs_rhs(const PotK& P, const double* y, double* f) {
#pragma clang fp contract(off)
  double g[3];
  accel_f64<NB>(P, y, g);
  const double W = P.omega;
  f[0] = y[3] + W * y[1];
  f[1] = y[4] - W * y[0];
  f[2] = y[5];
  f[3] = g[0] + W * y[4];
  f[4] = g[1] - W * y[3];
  f[5] = g[2];
}

// single precision: the bar's 16-node rule with hardware reciprocals, lam warm
// started from the previous evaluation (as the leapfrog integrator does)
template <bool NB>
__device__ __forceinline__ void bs_rhs(const PotK& P, const float* y, float* f, float& lamw) {
  float g[3], gb[3];
  accel_f32<1, NB>(P, y[0], y[1], y[2], g[0], g[1], g[2], gb, lamw, 0);
  const float W = (float)P.omega;
  f[0] = y[3] + W * y[1];
  f[1] = y[4] - W * y[0];
  f[2] = y[5];
  f[3] = (g[0] + gb[0]) + W * y[4];
  f[4] = (g[1] + gb[1]) - W * y[3];
  f[5] = g[2] + gb[2];
}

template <bool NB>
__device__ __forceinline__ void bs_rhs(const PotK& P, const double* y, double* f, float&) {
  bs_rhs<NB>(P, y, f);
}

template <bool NB>
__device__ __forceinline__ double bs_jacobi(const PotK& P, const double* y, float) {
  return jacobi_f64<NB>(P, y);
}

template <bool NB>
__device__ __forceinline__ double bs_jacobi(const PotK& P, const float* y, float lamw) {
  double yd[6];
  for (int i = 0; i < 6; ++i) yd[i] = (double)y[i];
  return jacobi_f64_drift<NB>(P, yd, lamw);
}

__device__ __forceinline__ double bs_pow(double e) { return pow(e, -1.0 / 3.0); }
__device__ __forceinline__ float bs_pow(float e) { return powf(e, -1.0f / 3.0f); }

// T: the arithmetic of the state, the stages and the step control (the total
// time is summed in double, the Jacobi drift evaluated in double)
template <typename T, bool NB, bool CYL>
__global__ __launch_bounds__(64) void k_bs23(PotK P, ObsK O, const double* __restrict__ ics,
                                              const double* __restrict__ h0, int64_t n, int32_t S, double rtol,
                                              double atol, uint64_t* __restrict__ ev_m, uint64_t* __restrict__ ev_k,
                                              double* __restrict__ wts, double* __restrict__ ttot,
                                              double* __restrict__ drift, uint8_t* __restrict__ flags) {
#pragma clang fp contract(off)
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n) return;
  T y[6], k1[6];
  for (int i = 0; i < 6; ++i) y[i] = (T)ics[(int64_t)i * n + o];
  const T rt = (T)rtol, at = (T)atol;
  T h = (T)h0[o];
  double tt = 0.0, dmax = 0.0;
  float lamw = -1.0f;
  bool bad = false;
  bs_rhs<NB>(P, y, k1, lamw);
  const double E0 = bs_jacobi<NB>(P, y, lamw);
  for (int s = 0; s < S; ++s) {
    T dt = (T)0;
    for (int tries = 0; tries < 100; ++tries) {
      const T hh = h;
      T t[6], k2[6], k3[6], y3[6], k4[6];
      for (int i = 0; i < 6; ++i) t[i] = y[i] + (T)0.5 * hh * k1[i];
      bs_rhs<NB>(P, t, k2, lamw);
      for (int i = 0; i < 6; ++i) t[i] = y[i] + (T)0.75 * hh * k2[i];
      bs_rhs<NB>(P, t, k3, lamw);
      for (int i = 0; i < 6; ++i)
        y3[i] = y[i] + hh * ((T)(2.0 / 9.0) * k1[i] + (T)(1.0 / 3.0) * k2[i] + (T)(4.0 / 9.0) * k3[i]);
      bs_rhs<NB>(P, y3, k4, lamw);
      T err = (T)0;
      for (int i = 0; i < 6; ++i) {
        const T y2 = y[i] + hh * ((T)(7.0 / 24.0) * k1[i] + (T)0.25 * k2[i] + (T)(1.0 / 3.0) * k3[i] +
                                  (T)0.125 * k4[i]);
        const T sc = at + rt * fmax(fabs(y[i]), fabs(y3[i]));
        err = fmax(err, fabs(y3[i] - y2) / sc);
      }
      T fac = err > (T)0 ? (T)0.9 * bs_pow(err) : (T)5;
      fac = fmin((T)5, fmax((T)0.2, fac));
      h = hh * fac;
      if (err <= (T)1) {
        for (int i = 0; i < 6; ++i) {
          y[i] = y3[i];
          k1[i] = k4[i];
        }
        dt = hh;
        break;
      }
    }
    if (dt == (T)0) bad = true;
    for (int i = 0; i < 6; ++i)
      if (!isfinite(y[i])) bad = true;
    tt += (double)dt;
    int mc[4], kc[4];
    cells4<T, CYL>(P, O, y, mc, kc);
    uint64_t vm = 0, vk = 0;
    for (int c = 0; c < 4; ++c) {
      vm |= (uint64_t)(uint16_t)(mc[c] < 0 ? 0xFFFF : mc[c]) << (16 * c);
      vk |= (uint64_t)(uint16_t)(kc[c] < 0 ? 0xFFFF : kc[c]) << (16 * c);
    }
    const int64_t e = o * S + s;
    ev_m[e] = vm;
    ev_k[e] = vk;
    wts[e] = (double)dt;
    if (O.drift_every > 0 && (s + 1) % O.drift_every == 0) {
      const double d = fabs(bs_jacobi<NB>(P, y, lamw) / E0 - 1.0);
      if (!(d <= dmax)) dmax = d;
    }
  }
  ttot[o] = tt;
  drift[o] = dmax;
  flags[o] = (uint8_t)((!(dmax <= 0.1) ? SW_FLAG_DRIFT : 0) | (bad ? SW_FLAG_NONFINITE : 0));
}

// columns [win0, win0 + wn) of one block; fold_nv > 0: surface pass (codes fold
// to their aperture); slot >= 0 and win0 == 0: the block's overflow is written
__global__ __launch_bounds__(256) void k_hist_w(const uint64_t* __restrict__ ev, const double* __restrict__ wts,
                                                const double* __restrict__ ttot, int32_t S, int32_t ncopy,
                                                int32_t ncell, int32_t win0, int32_t wn, int64_t n_con,
                                                int32_t col_off, double* __restrict__ A,
                                                double* __restrict__ overflow, int32_t slot, int32_t fold_nv,
                                                int32_t fold_nkin, double div) {
  extern __shared__ unsigned long long hq[];
  __shared__ unsigned long long ovq;
  const int64_t o = blockIdx.x;
  const int tid = threadIdx.x;
  for (int c = tid; c < wn; c += 256) hq[c] = 0ull;
  if (tid == 0) ovq = 0ull;
  __syncthreads();
  const double inv_t = 1.0 / ttot[o];
  for (int s = tid; s < S; s += 256) {
    const uint64_t v = ev[o * S + s];
    const unsigned long long q = (unsigned long long)llrint(wts[o * S + s] * inv_t * 0x1p52);
    for (int c = 0; c < ncopy; ++c) {
      uint32_t idx = (uint32_t)(v >> (16 * c)) & 0xFFFFu;
      if (fold_nv > 0 && idx != 0xFFFFu)
        idx = idx < (uint32_t)fold_nkin ? idx / (uint32_t)fold_nv : idx - (uint32_t)fold_nkin;
      if (idx >= (uint32_t)ncell) {
        if (win0 == 0) atomicAdd(&ovq, q);
      } else if (idx >= (uint32_t)win0 && idx < (uint32_t)(win0 + wn)) {
        atomicAdd(&hq[idx - win0], q);
      }
    }
  }
  __syncthreads();
  const double scale = 0x1p-52 / (double)ncopy;
  double* row = A + o * n_con + col_off + win0;
  for (int c = tid; c < wn; c += 256) row[c] = (double)hq[c] * scale / div;
  if (tid == 0 && slot >= 0 && win0 == 0) overflow[o * 2 + slot] = (double)ovq * scale;
}

size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

int hist_w(const uint64_t* ev, const double* wts, const double* ttot, int64_t n, int32_t S, int32_t ncopy,
           int32_t ncell, int64_t n_con, int32_t col_off, double* A, double* overflow, int32_t slot, hipStream_t st,
           int32_t fold_nv = 0, int32_t fold_nkin = 0, double div = 1.0) {
  for (int32_t w0 = 0; w0 < ncell; w0 += kBsWindow) {
    const int32_t wn = ncell - w0 < kBsWindow ? ncell - w0 : kBsWindow;
    hipLaunchKernelGGL(k_hist_w, dim3((unsigned)n), dim3(256), (size_t)wn * sizeof(double), st, ev, wts, ttot, S,
                       ncopy, ncell, w0, wn, n_con, col_off, A, overflow, slot, fold_nv, fold_nkin, div);
    SW_HIP(hipGetLastError());
  }
  return SW_OK;
}

}  // namespace
}  // namespace sw

using namespace sw;

extern "C" size_t integrate_bs23_workspace_bytes(int64_t n_orb, int32_t n_steps) {
  if (n_orb < 0 || n_steps < 1) return 0;
  const size_t per = (size_t)n_orb * (size_t)n_steps * 8;
  return 3 * al256(per) + al256((size_t)n_orb * 8);
}

extern "C" int integrate_bs23_and_bin(const sw_potential* pot, const double* ics, const double* h0, int64_t n_orb,
                                      int32_t n_steps, double rtol, double atol, int32_t precision,
                                      const sw_obs_spec* obs, double* A, double* overflow, double* drift,
                                      uint8_t* flags, void* workspace, size_t ws_bytes, void* stream) {
  SW_CHECK(pot && obs, "integrate_bs23_and_bin: null argument");
  SW_CHECK(precision == SW_F32 || precision == SW_F64, "integrate_bs23_and_bin: precision must be SW_F32 or SW_F64");
  SW_CHECK(n_orb >= 0 && n_orb <= 0x7fffffffLL && n_steps >= 1,
           "integrate_bs23_and_bin: need n_orb >= 0 and n_steps >= 1");
  SW_CHECK(std::isfinite(rtol) && rtol > 0.0 && std::isfinite(atol) && atol > 0.0,
           "integrate_bs23_and_bin: tolerances must be finite and > 0");
  ObsK O;
  SW_CHECK(obs_to_k(obs, &O), "integrate_bs23_and_bin: invalid observable specification");
  if (n_orb == 0) return SW_OK;
  SW_CHECK(ics && h0 && A && overflow && drift && flags && workspace, "integrate_bs23_and_bin: null device buffer");
  SW_CHECK(ws_bytes >= integrate_bs23_workspace_bytes(n_orb, n_steps), "integrate_bs23_and_bin: workspace too small");
  PotK P;
  std::memcpy(&P, pot, sizeof P);
  bool nb = false;
  for (int c = 0; c < P.n_comp; ++c) nb = nb || P.comp[c].kind == SW_DA_T3 || P.comp[c].kind == SW_DA_V4;
  const size_t per = al256((size_t)n_orb * (size_t)n_steps * 8);
  char* ws = (char*)workspace;
  uint64_t* ev_m = (uint64_t*)ws;
  uint64_t* ev_k = (uint64_t*)(ws + per);
  double* wts = (double*)(ws + 2 * per);
  double* ttot = (double*)(ws + 3 * per);
  hipStream_t st = (hipStream_t)stream;
  const dim3 grid((unsigned)((n_orb + 63) / 64)), block(64);
#define SW_BS23_LAUNCH(T, NB, CYL)                                                                                \
  hipLaunchKernelGGL((k_bs23<T, NB, CYL>), grid, block, 0, st, P, O, ics, h0, n_orb, n_steps, rtol, atol, ev_m, ev_k, \
                     wts, ttot, drift, flags)
  if (precision == SW_F32) {
    if (O.cyl) {
      if (nb) SW_BS23_LAUNCH(float, true, true);
      else SW_BS23_LAUNCH(float, false, true);
    } else {
      if (nb) SW_BS23_LAUNCH(float, true, false);
      else SW_BS23_LAUNCH(float, false, false);
    }
  } else {
    if (O.cyl) {
      if (nb) SW_BS23_LAUNCH(double, true, true);
      else SW_BS23_LAUNCH(double, false, true);
    } else {
      if (nb) SW_BS23_LAUNCH(double, true, false);
      else SW_BS23_LAUNCH(double, false, false);
    }
  }
#undef SW_BS23_LAUNCH
  SW_HIP(hipGetLastError());
  const int64_t n_con = (int64_t)O.n_mass + O.n_kin + (O.surface ? O.n_ap : 0);
  int rc = hist_w(ev_m, wts, ttot, n_orb, n_steps, O.ncopy, O.n_mass, n_con, 0, A, overflow, 0, st);
  if (rc == SW_OK) rc = hist_w(ev_k, wts, ttot, n_orb, n_steps, O.ncopy, O.n_kin, n_con, O.n_mass, A, overflow, 1, st);
  if (rc == SW_OK && O.surface)
    rc = hist_w(ev_k, wts, ttot, n_orb, n_steps, O.ncopy, O.n_ap, n_con, O.n_mass + O.n_kin, A, overflow, -1, st,
                O.nv, O.n_kin, obs->upsilon);
  return rc;
}
