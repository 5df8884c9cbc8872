// Orbit integration kernel (Sec. 2.2.2-2.2.4), templated on the working
// precision.  One orbit per lane.  Each lane integrates its orbit with a
// kick-drift-kick leapfrog in the corotating bar frame, keeps the force of the
// last kick for the next step's first kick, bins the four mirror copies of
// every synchronised state and stages the packed cell indices of
// kStage steps in LDS.  The wave then writes each orbit's staged steps as one
// contiguous 128-byte segment of that orbit's event stream, so the stream is
// written with full-line stores although each lane owns a different orbit.
//
// Event word (uint64, one per orbit per step per block): four 16-bit cell
// indices, copy c in bits [16c, 16c+16), 0xFFFF = outside the block.
#pragma once
#include "potential.h"

namespace sw {

constexpr int kStage = 16;
constexpr int kWave = 64;

// lamw: the single-precision path's warm-start state of the bar's lam (unused in double)
template <typename T>
struct Prec;
template <>
struct Prec<float> {
  // LPO lanes per orbit: each lane's share, then the sum over the lane group
  // (the same sum in every lane of the group, so their states stay identical)
  template <int LPO = 1, bool NB = false>
  __device__ static void accel(const PotK& P, const float* s, float* g, float& lamw, int part = 0) {
    float gb[3];
    accel_f32<LPO, NB>(P, s[0], s[1], s[2], g[0], g[1], g[2], gb, lamw, part);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if constexpr (LPO == 2) gb[k] += __shfl_xor(gb[k], 1, 64);
      g[k] += gb[k];
    }
  }
  template <bool NB = false>
  __device__ static double jacobi(const PotK& P, const double* sd, float lamw) {
    return jacobi_f64_drift<NB>(P, sd, lamw);
  }
};
template <>
struct Prec<double> {
  template <int LPO = 1, bool NB = false>
  __device__ static void accel(const PotK& P, const double* s, double* g, float&, int = 0) {
    static_assert(LPO == 1, "the double-precision path runs one lane per orbit");
    accel_f64<NB>(P, s, g);
  }
  template <bool NB = false>
  __device__ static double jacobi(const PotK& P, const double* sd, float) { return jacobi_f64<NB>(P, sd); }
};

__device__ __forceinline__ uint64_t pack4(const int* c) {
  uint64_t v = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) v |= (uint64_t)(uint16_t)(c[i] < 0 ? 0xFFFF : c[i]) << (16 * i);
  return v;
}

// Potential index of orbit o: the last k with offsets[k] <= o.
__device__ __forceinline__ int pot_index(const int64_t* offsets, int n_pot, int64_t o) {
  int lo = 0, hi = n_pot - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (offsets[mid] <= o) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// At most 168 registers, so that three waves share a SIMD (the default
// allocation lands one register above that, at two waves); no spills.
//
// LPO lanes per orbit (1, or 2 in single precision): a wave carries 64 / LPO
// orbits; the lanes of a pair hold the same state, each evaluates its share of
// the force and the pair adds the shares, so both advance identically; the
// first lane of the pair writes the orbit's events and results.
template <typename T, bool BATCHED, bool BIN, int LPO = 1, bool NB = false, bool CYL = false>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(3)))
void k_integrate(const PotK p0, const sw_potential* __restrict__ pots, const int64_t* __restrict__ offsets,
                 int32_t n_pot, ObsK O, const T* __restrict__ ics, const T* __restrict__ dts, int64_t n_orb,
                 int64_t orb0, int64_t n_chunk, int32_t n_steps, uint64_t* __restrict__ ev_m,
                 uint64_t* __restrict__ ev_k, double* __restrict__ drift, uint8_t* __restrict__ flags,
                 T* __restrict__ final_state) {
  constexpr int OPW = kWave / LPO;  // orbits per wave
  __shared__ uint64_t stm[kStage][OPW + 1];
  __shared__ uint64_t stk[kStage][OPW + 1];
  const int lane = threadIdx.x;
  const int part = lane % LPO, lo = lane / LPO;  // share and orbit of this lane
  const int64_t n_tiles = (n_chunk + OPW - 1) / OPW;
  // persistent launch: each wave walks the orbit tiles t = blockIdx.x, + gridDim.x, ...
  for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
  const int64_t jbase = tile * OPW;  // chunk-local index of the tile's first orbit
  const int64_t j = jbase + lo;
  const bool valid = j < n_chunk;
  const int64_t o = orb0 + (valid ? j : n_chunk - 1);
  const int kpot = BATCHED ? pot_index(offsets, n_pot, o) : 0;
  const PotK& P = BATCHED ? *reinterpret_cast<const PotK*>(pots + kpot) : p0;

  T s[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) s[i] = ics[(int64_t)i * n_orb + o];
  const T dt = dts[o];
  const T h = T(0.5) * dt;
  const double th = P.omega * (double)dt;
  // FP64 rotates with (cos, sin) exactly as the oracle does.  FP32 rotates with
  // (cos - 1, sin): cos rounded to binary32 would scale the radius by up to one
  // ulp of 1 per step, a systematic drift over 10^4 steps, whereas cos - 1 =
  // -2 sin^2(th/2) keeps its full relative precision.
  const T c = (T)cos(th), sn = (T)sin(th);
  const T cm1 = (T)(-2.0 * sin(0.5 * th) * sin(0.5 * th));

  float lamw = -1.0f;
  T g[3];
  Prec<T>::template accel<LPO, NB>(P, s, g, lamw, part);
  double sd[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) sd[i] = (double)s[i];
  const double E0 = Prec<T>::template jacobi<NB>(P, sd, lamw);
  double dmax = 0.0;
  const int de = O.drift_every;

  int slot = 0;
  for (int k = 1; k <= n_steps; ++k) {
    s[3] = s[3] + h * g[0];
    s[4] = s[4] + h * g[1];
    s[5] = s[5] + h * g[2];
    s[0] = s[0] + dt * s[3];
    s[1] = s[1] + dt * s[4];
    s[2] = s[2] + dt * s[5];
    if constexpr (sizeof(T) == 8) {
      T x = c * s[0] + sn * s[1];
      T y = c * s[1] - sn * s[0];
      T px = c * s[3] + sn * s[4];
      T py = c * s[4] - sn * s[3];
      s[0] = x; s[1] = y; s[3] = px; s[4] = py;
    } else {
      T x = s[0] + (cm1 * s[0] + sn * s[1]);
      T y = s[1] + (cm1 * s[1] - sn * s[0]);
      T px = s[3] + (cm1 * s[3] + sn * s[4]);
      T py = s[4] + (cm1 * s[4] - sn * s[3]);
      s[0] = x; s[1] = y; s[3] = px; s[4] = py;
    }
    Prec<T>::template accel<LPO, NB>(P, s, g, lamw, part);
    s[3] = s[3] + h * g[0];
    s[4] = s[4] + h * g[1];
    s[5] = s[5] + h * g[2];

    if (de > 0 && k % de == 0) {
#pragma unroll
      for (int i = 0; i < 6; ++i) sd[i] = (double)s[i];
      double e = fabs(Prec<T>::template jacobi<NB>(P, sd, lamw) / E0 - 1.0);
      if (!(e <= dmax)) dmax = e;
    }
    if constexpr (BIN) {
      int mc[4], kc[4];
      cells4<T, CYL>(P, O, s, mc, kc);
      if (part == 0) {
        stm[slot][lo] = pack4(mc);
        stk[slot][lo] = pack4(kc);
      }
      ++slot;
      if (slot == kStage || k == n_steps) {
        __syncthreads();
        const int64_t step0 = k - slot;
        const int total = slot * OPW;
        for (int idx = lane; idx < total; idx += kWave) {
          const int jj = idx / slot, ss = idx - jj * slot;
          const int64_t jo = jbase + jj;
          if (jo < n_chunk) {
            const int64_t at = jo * n_steps + step0 + ss;
            ev_m[at] = stm[ss][jj];
            ev_k[at] = stk[ss][jj];
          }
        }
        __syncthreads();
        slot = 0;
      }
    }
  }
  if (valid && part == 0) {
    bool nonfinite = false;
#pragma unroll
    for (int i = 0; i < 6; ++i) nonfinite |= !isfinite(s[i]);
    if (drift) drift[o] = dmax;
    if (flags) flags[o] = (uint8_t)((!(dmax <= 0.1) ? SW_FLAG_DRIFT : 0) | (nonfinite ? SW_FLAG_NONFINITE : 0));
    if constexpr (!BIN) {
#pragma unroll
      for (int i = 0; i < 6; ++i) final_state[(int64_t)i * n_orb + o] = s[i];
    }
  }
  }  // tile loop
}

// the integration kernels take the potential and the observables by value
static_assert(sizeof(PotK) + sizeof(ObsK) + 256 <= 4096, "kernel arguments exceed 4 KiB");

struct IntegrateLaunch {
  PotK p0;                     // the potential when n_pot == 1
  const sw_potential* pots_dev;  // device copies when n_pot > 1
  const int64_t* offsets_dev;
  int32_t n_pot;
  ObsK obs;
  const void* ics;
  const void* dt;
  int64_t n_orb, orb0, n_chunk;
  int32_t n_steps;
  uint64_t* ev_m;
  uint64_t* ev_k;
  double* drift;
  uint8_t* flags;
  void* final_state;
  bool bin;
  bool needle;  // some potential holds a needle bar: the kernels built with its code
};

// Process-wide launch knobs (set through sw_set_tuning):
//  g_waves_per_cu  0: one wave per 64-orbit tile; k > 0: persistent grid of k waves per CU
//  g_hist_lds_kb   LDS budget of one histogram workgroup (orbits per workgroup follow)
extern int g_waves_per_cu;
extern int g_hist_lds_kb;
extern int g_lanes_per_orbit;  // 1 or 2 lanes per orbit (single precision with binning)
extern int g_num_cus;

template <typename T>
hipError_t launch_integrate_t(const IntegrateLaunch& L, hipStream_t st) {
  // potentials with needle bars, and cylindrical grids, run one lane per orbit
  const int lpo = (sizeof(T) == 4 && L.bin && g_lanes_per_orbit == 2 && !L.needle && !L.obs.cyl) ? 2 : 1;
  int64_t tiles = (L.n_chunk + kWave / lpo - 1) / (kWave / lpo);
  if (g_waves_per_cu > 0) {
    const int64_t cap = (int64_t)g_waves_per_cu * g_num_cus;
    if (tiles > cap) tiles = cap;
  }
  dim3 grid((unsigned)tiles), block(kWave);
  const T* ics = (const T*)L.ics;
  const T* dt = (const T*)L.dt;
  T* fs = (T*)L.final_state;
  if (L.bin && L.obs.cyl) {
    // cylindrical mass grid: one lane per orbit, needle bars compiled in when present
    if (L.n_pot > 1) {
      if (L.needle)
        hipLaunchKernelGGL((k_integrate<T, true, true, 1, true, true>), grid, block, 0, st, L.p0, L.pots_dev,
                           L.offsets_dev, L.n_pot, L.obs, ics, dt, L.n_orb, L.orb0, L.n_chunk, L.n_steps, L.ev_m,
                           L.ev_k, L.drift, L.flags, fs);
      else
        hipLaunchKernelGGL((k_integrate<T, true, true, 1, false, true>), grid, block, 0, st, L.p0, L.pots_dev,
                           L.offsets_dev, L.n_pot, L.obs, ics, dt, L.n_orb, L.orb0, L.n_chunk, L.n_steps, L.ev_m,
                           L.ev_k, L.drift, L.flags, fs);
    } else {
      if (L.needle)
        hipLaunchKernelGGL((k_integrate<T, false, true, 1, true, true>), grid, block, 0, st, L.p0, L.pots_dev,
                           L.offsets_dev, L.n_pot, L.obs, ics, dt, L.n_orb, L.orb0, L.n_chunk, L.n_steps, L.ev_m,
                           L.ev_k, L.drift, L.flags, fs);
      else
        hipLaunchKernelGGL((k_integrate<T, false, true, 1, false, true>), grid, block, 0, st, L.p0, L.pots_dev,
                           L.offsets_dev, L.n_pot, L.obs, ics, dt, L.n_orb, L.orb0, L.n_chunk, L.n_steps, L.ev_m,
                           L.ev_k, L.drift, L.flags, fs);
    }
    return hipGetLastError();
  }
  if (L.needle) {
    if (!L.bin)
      hipLaunchKernelGGL((k_integrate<T, false, false, 1, true>), grid, block, 0, st, L.p0, L.pots_dev, L.offsets_dev,
                         L.n_pot, L.obs, ics, dt, L.n_orb, L.orb0, L.n_chunk, L.n_steps, L.ev_m, L.ev_k, L.drift,
                         L.flags, fs);
    else if (L.n_pot > 1)
      hipLaunchKernelGGL((k_integrate<T, true, true, 1, true>), grid, block, 0, st, L.p0, L.pots_dev, L.offsets_dev,
                         L.n_pot, L.obs, ics, dt, L.n_orb, L.orb0, L.n_chunk, L.n_steps, L.ev_m, L.ev_k, L.drift,
                         L.flags, fs);
    else
      hipLaunchKernelGGL((k_integrate<T, false, true, 1, true>), grid, block, 0, st, L.p0, L.pots_dev, L.offsets_dev,
                         L.n_pot, L.obs, ics, dt, L.n_orb, L.orb0, L.n_chunk, L.n_steps, L.ev_m, L.ev_k, L.drift,
                         L.flags, fs);
    return hipGetLastError();
  }
  if (L.bin) {
    if constexpr (sizeof(T) == 4) {
      if (lpo == 2) {
        if (L.n_pot > 1)
          hipLaunchKernelGGL((k_integrate<T, true, true, 2>), grid, block, 0, st, L.p0, L.pots_dev, L.offsets_dev,
                             L.n_pot, L.obs, ics, dt, L.n_orb, L.orb0, L.n_chunk, L.n_steps, L.ev_m, L.ev_k, L.drift,
                             L.flags, fs);
        else
          hipLaunchKernelGGL((k_integrate<T, false, true, 2>), grid, block, 0, st, L.p0, L.pots_dev, L.offsets_dev,
                             L.n_pot, L.obs, ics, dt, L.n_orb, L.orb0, L.n_chunk, L.n_steps, L.ev_m, L.ev_k, L.drift,
                             L.flags, fs);
        return hipGetLastError();
      }
    }
    if (L.n_pot > 1)
      hipLaunchKernelGGL((k_integrate<T, true, true>), grid, block, 0, st, L.p0, L.pots_dev, L.offsets_dev, L.n_pot, L.obs,
                         ics, dt, L.n_orb, L.orb0, L.n_chunk, L.n_steps, L.ev_m, L.ev_k, L.drift, L.flags, fs);
    else
      hipLaunchKernelGGL((k_integrate<T, false, true>), grid, block, 0, st, L.p0, L.pots_dev, L.offsets_dev, L.n_pot, L.obs,
                         ics, dt, L.n_orb, L.orb0, L.n_chunk, L.n_steps, L.ev_m, L.ev_k, L.drift, L.flags, fs);
  } else {
    hipLaunchKernelGGL((k_integrate<T, false, false>), grid, block, 0, st, L.p0, L.pots_dev, L.offsets_dev, L.n_pot, L.obs,
                       ics, dt, L.n_orb, L.orb0, L.n_chunk, L.n_steps, L.ev_m, L.ev_k, L.drift, L.flags, fs);
  }
  return hipGetLastError();
}

hipError_t launch_integrate_f32(const IntegrateLaunch& L, hipStream_t st);
hipError_t launch_integrate_f64(const IntegrateLaunch& L, hipStream_t st);

}  // namespace sw
