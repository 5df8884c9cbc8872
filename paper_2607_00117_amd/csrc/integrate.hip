// integrate_and_bin, bin_points, integrate_orbits and the histogram kernel.
//
// integrate_and_bin runs in two kernels per orbit chunk:
//  1. k_integrate: one orbit per lane, packed cell indices of every step and
//     mirror copy appended to each orbit's event stream (workspace);
//  2. k_hist: one workgroup per group of orbits per block; the orbit's row is
//     an LDS-privatised histogram of 16-bit counters (two per 32-bit word,
//     ds_add of 1 or 1<<16), filled from the event stream and written to the
//     orbit matrix as time fractions with consecutive, coalesced stores.
// No global atomics are used: every orbit's row is owned by one workgroup.
#include <cstring>
#include <string>

#include "integrate_impl.h"

namespace sw {

constexpr int kHistThreads = 256;

int g_waves_per_cu = 0;
int g_hist_lds_kb = 64;
int g_lanes_per_orbit = 1;
int g_num_cus = 256;

template <typename T>
__global__ __launch_bounds__(kHistThreads) void k_hist(const uint64_t* __restrict__ ev, int64_t n_chunk,
                                                       int32_t n_steps, int32_t ncopy, int32_t ncell, int32_t opw,
                                                       int32_t wide, int64_t row0, int64_t n_con, int32_t col_off,
                                                       T* __restrict__ A, double* __restrict__ overflow,
                                                       int32_t slot, int32_t fold_nv, int32_t fold_nkin,
                                                       double div) {
  extern __shared__ uint32_t hist[];
  __shared__ uint32_t ovc[32];
  const int tid = threadIdx.x;
  const int nw = wide ? ncell : (ncell + 1) >> 1;
  for (int i = tid; i < opw * nw; i += kHistThreads) hist[i] = 0u;
  if (tid < 32) ovc[tid] = 0u;
  __syncthreads();
  for (int g = 0; g < opw; ++g) {
    const int64_t j = (int64_t)blockIdx.x * opw + g;
    if (j >= n_chunk) break;
    const uint64_t* e = ev + j * (int64_t)n_steps;
    uint32_t* hg = hist + g * nw;
    uint32_t ov = 0;
    for (int s = tid; s < n_steps; s += kHistThreads) {
      const uint64_t v = e[s];
      for (int c = 0; c < ncopy; ++c) {
        uint32_t idx = (uint32_t)(v >> (16 * c)) & 0xFFFFu;
        // surface pass: kinematic codes ap*nv + v_bin and n_kin + ap fold to ap
        if (fold_nv > 0 && idx != 0xFFFFu)
          idx = idx < (uint32_t)fold_nkin ? idx / (uint32_t)fold_nv : idx - (uint32_t)fold_nkin;
        if (idx >= (uint32_t)ncell) {  // 0xFFFF, or a surface-only code in the kinematic pass
          ++ov;
        } else if (wide) {
          atomicAdd(&hg[idx], 1u);
        } else {
          atomicAdd(&hg[idx >> 1], 1u << ((idx & 1u) * 16u));
        }
      }
    }
    // wavefront reduction of the overflow count, one LDS atomic per wave
    for (int off = 32; off > 0; off >>= 1) ov += __shfl_xor(ov, off, 64);
    if ((tid & 63) == 0 && ov) atomicAdd(&ovc[g], ov);
  }
  __syncthreads();
  const double denom = (double)ncopy * (double)n_steps;
  for (int g = 0; g < opw; ++g) {
    const int64_t j = (int64_t)blockIdx.x * opw + g;
    if (j >= n_chunk) break;
    const uint32_t* hg = hist + g * nw;
    T* row = A + (row0 + j) * n_con + col_off;
    for (int c = tid; c < ncell; c += kHistThreads) {
      const uint32_t cnt = wide ? hg[c] : (hg[c >> 1] >> ((c & 1) * 16)) & 0xFFFFu;
      row[c] = (T)((double)cnt / denom / div);
    }
    if (tid == 0 && slot >= 0) overflow[(row0 + j) * 2 + slot] = (double)ovc[g] / denom;
  }
}

template <typename T, bool CYL>
__global__ void k_bin_points(const PotK P, ObsK O, const T* __restrict__ pts, int64_t n, int32_t* __restrict__ mass,
                             int32_t* __restrict__ kin) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T s[6];
  for (int k = 0; k < 6; ++k) s[k] = pts[(int64_t)k * n + i];
  int mc[4], kc[4];
  cells4<T, CYL>(P, O, s, mc, kc);
  for (int c = 0; c < 4; ++c) {
    mass[4 * i + c] = mc[c];
    kin[4 * i + c] = kc[c];
  }
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

static size_t header_bytes(int32_t n_pot) {
  return align256((size_t)n_pot * sizeof(sw_potential)) + align256((size_t)(n_pot + 1) * sizeof(int64_t));
}

}  // namespace sw

using namespace sw;

extern "C" int sw_set_tuning(const char* key, int32_t value) {
  SW_CHECK(key, "sw_set_tuning: null key");
  const std::string k(key);
  if (k == "integrate_waves_per_cu") {
    SW_CHECK(value >= 0 && value <= 64, "sw_set_tuning: integrate_waves_per_cu in [0, 64]");
    g_waves_per_cu = value;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) ==
                                                  hipSuccess && cus > 0)
      g_num_cus = cus;
    return SW_OK;
  }
  if (k == "hist_lds_kb") {
    SW_CHECK(value >= 4 && value <= 160, "sw_set_tuning: hist_lds_kb in [4, 160]");
    g_hist_lds_kb = value;
    return SW_OK;
  }
  if (k == "integrate_lanes_per_orbit") {
    SW_CHECK(value == 1 || value == 2, "sw_set_tuning: integrate_lanes_per_orbit is 1 or 2");
    g_lanes_per_orbit = value;
    return SW_OK;
  }
  if (k == "sparse_rows_per_wg" || k == "sparse_cols_per_wg") {
    SW_CHECK(value >= 0 && value <= 512 && value % 16 == 0, "sw_set_tuning: %s: 0 (automatic) or a multiple of 16 "
             "up to 512", key);
    (k == "sparse_rows_per_wg" ? g_sparse_rows : g_sparse_cols) = value;
    return SW_OK;
  }
  if (k == "sparse_lanes_per_row") {
    SW_CHECK(value == 0 || value == 16 || value == 64, "sw_set_tuning: sparse_lanes_per_row: 0 (automatic), 16 or 64");
    g_sparse_lanes = value;
    return SW_OK;
  }
  if (k == "multi_dense") {
    SW_CHECK(value >= 0 && value <= 2, "sw_set_tuning: multi_dense: 0 (by cost), 1 (dense MFMA), 2 (compressed)");
    g_multi_dense = value;
    return SW_OK;
  }
  if (k == "gram_counts") {
    SW_CHECK(value == 0 || value == 1, "sw_set_tuning: gram_counts is 0 or 1");
    g_gram_counts = value;
    return SW_OK;
  }
  if (k == "trmv_rows") {
    SW_CHECK(value == 2 || value == 16, "sw_set_tuning: trmv_rows is 2 or 16");
    g_trmv_rows = value;
    return SW_OK;
  }
  if (k == "refine_rebound_checks") {
    SW_CHECK(value >= 1, "sw_set_tuning: refine_rebound_checks >= 1");
    g_refine_rebound_checks = value;
    return SW_OK;
  }
  if (k == "refine_rebound") {
    SW_CHECK(value >= 0, "sw_set_tuning: refine_rebound: a factor >= 0");
    g_refine_rebound = value;
    return SW_OK;
  }
  if (k == "refine_passes") {
    SW_CHECK(value == 2 || value == 4, "sw_set_tuning: refine_passes: 2 (h carried) or 4 (residual from A)");
    g_refine_two = value == 2 ? 1 : 0;
    return SW_OK;
  }
  if (k == "gram_skip") {
    SW_CHECK(value == 0 || value == 1, "sw_set_tuning: gram_skip: 1 (skip zero panels) or 0 (stream every stage)");
    g_gram_dense = value ? 0 : 1;
    return SW_OK;
  }
  if (k == "factor_gemm") {
    SW_CHECK(value == 0 || value == 1, "sw_set_tuning: factor_gemm: 0 (fp32 MFMA) or 1 (bf16x3 MFMA)");
    g_factor_x3 = value;
    return SW_OK;
  }
  if (k == "rhs_per_group") {
    SW_CHECK(value == 0 || value == 1 || value == 2 || value == 4 || value == 8,
             "sw_set_tuning: rhs_per_group: 0 (automatic), 1, 2, 4 or 8");
    g_rhs_group = value;
    return SW_OK;
  }
  SW_CHECK(false, "sw_set_tuning: unknown key %s", key);
}

extern "C" int32_t sw_get_tuning(const char* key) {
  if (!key) return -1;
  const std::string k(key);
  if (k == "integrate_waves_per_cu") return g_waves_per_cu;
  if (k == "hist_lds_kb") return g_hist_lds_kb;
  if (k == "integrate_lanes_per_orbit") return g_lanes_per_orbit;
  if (k == "sparse_rows_per_wg") return g_sparse_rows;
  if (k == "sparse_cols_per_wg") return g_sparse_cols;
  if (k == "sparse_lanes_per_row") return g_sparse_lanes;
  if (k == "rhs_per_group") return g_rhs_group;
  if (k == "factor_gemm") return g_factor_x3;
  if (k == "gram_skip") return g_gram_dense ? 0 : 1;
  if (k == "refine_passes") return g_refine_two ? 2 : 4;
  if (k == "multi_dense") return g_multi_dense;
  if (k == "refine_rebound") return g_refine_rebound;
  if (k == "refine_rebound_checks") return g_refine_rebound_checks;
  if (k == "trmv_rows") return g_trmv_rows;
  if (k == "gram_counts") return g_gram_counts;
  return -1;
}

extern "C" size_t integrate_workspace_bytes(const sw_obs_spec* obs, int32_t n_pot, int64_t n_orb, int32_t n_steps,
                                            int32_t dtype) {
  (void)obs;
  (void)dtype;
  if (n_pot < 1 || n_orb < 0 || n_steps < 1) return 0;
  return header_bytes(n_pot) + 2 * align256((size_t)n_orb * (size_t)n_steps * sizeof(uint64_t));
}

template <typename T>
static int launch_hist(const uint64_t* ev, int64_t n_chunk, int32_t n_steps, int32_t ncopy, int32_t ncell,
                       int64_t row0, int64_t n_con, int32_t col_off, void* A, double* overflow, int32_t slot,
                       hipStream_t st, int32_t fold_nv = 0, int32_t fold_nkin = 0, double div = 1.0) {
  const int wide = (int64_t)ncopy * n_steps > 65535 ? 1 : 0;
  const int nw = wide ? ncell : (ncell + 1) / 2;
  int opw = (g_hist_lds_kb * 1024) / (4 * nw);
  if (opw < 1) opw = 1;
  if (opw > 32) opw = 32;
  const size_t lds = (size_t)opw * nw * 4;
  if (lds > 160 * 1024) {
    set_error("integrate_and_bin: block of %d cells does not fit the LDS histogram", ncell);
    return SW_EINVAL;
  }
  dim3 grid((unsigned)((n_chunk + opw - 1) / opw)), block(kHistThreads);
  hipLaunchKernelGGL(k_hist<T>, grid, block, lds, st, ev, n_chunk, n_steps, ncopy, ncell, opw, wide, row0, n_con,
                     col_off, (T*)A, overflow, slot, fold_nv, fold_nkin, div);
  SW_HIP(hipGetLastError());
  return SW_OK;
}

// whether a potential holds a needle bar (its kernels carry the bar's code)
static bool has_needle(const sw_potential* p) {
  PotK P;
  std::memcpy(&P, p, sizeof P);
  for (int i = 0; i < P.n_comp && i < SW_MAX_COMP; ++i)
    if (P.comp[i].kind == SW_DA_T3 || P.comp[i].kind == SW_DA_V4) return true;
  return false;
}

extern "C" int integrate_and_bin(const sw_potential* pots, int32_t n_pot, const int64_t* orbit_offsets,
                                 const void* ics, const void* dt, int64_t n_orb, int32_t n_steps, int32_t dtype,
                                 const sw_obs_spec* obs, void* A, double* overflow, double* drift, uint8_t* flags,
                                 void* workspace, size_t ws_bytes, void* stream) {
  SW_CHECK(pots && orbit_offsets && obs, "integrate_and_bin: null argument");
  SW_CHECK(n_pot >= 1, "integrate_and_bin: n_pot must be >= 1");
  SW_CHECK(n_orb >= 0 && n_steps >= 1, "integrate_and_bin: need n_orb >= 0 and n_steps >= 1");
  SW_CHECK(dtype == SW_F32 || dtype == SW_F64, "integrate_and_bin: dtype must be SW_F32 or SW_F64");
  SW_CHECK(orbit_offsets[0] == 0 && orbit_offsets[n_pot] == n_orb,
           "integrate_and_bin: orbit_offsets must start at 0 and end at n_orb");
  for (int k = 0; k < n_pot; ++k)
    SW_CHECK(orbit_offsets[k + 1] >= orbit_offsets[k], "integrate_and_bin: orbit_offsets must be non-decreasing");
  ObsK O;
  SW_CHECK(obs_to_k(obs, &O), "integrate_and_bin: invalid observable specification");
  const double upsilon = obs->upsilon;
  if (n_orb == 0) return SW_OK;
  SW_CHECK(ics && dt && A && overflow && drift && flags, "integrate_and_bin: null device buffer");
  const size_t hdr = header_bytes(n_pot);
  SW_CHECK(workspace != nullptr, "integrate_and_bin: null workspace");
  // event streams of `c` orbits: two buffers of c * n_steps words each
  auto need = [&](int64_t c) { return hdr + 2 * align256((size_t)c * (size_t)n_steps * sizeof(uint64_t)); };
  int64_t chunk = n_orb;
  if (ws_bytes < need(chunk)) {
    const size_t per = 2 * (size_t)n_steps * sizeof(uint64_t);
    chunk = ws_bytes > hdr + 512 ? (int64_t)((ws_bytes - hdr - 512) / per) : 0;
    chunk = (chunk / kWave) * kWave;
    if (chunk < kWave) {
      set_error("integrate_and_bin: workspace of %zu bytes is too small (at least %zu needed)", ws_bytes,
                need(n_orb < kWave ? n_orb : kWave));
      return SW_ENOMEM;
    }
  }
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  IntegrateLaunch L;
  std::memset(&L, 0, sizeof L);
  std::memcpy(&L.p0, &pots[0], sizeof(PotK));
  L.n_pot = n_pot;
  for (int b = 0; b < n_pot; ++b) L.needle = L.needle || has_needle(&pots[b]);
  if (n_pot > 1) {
    L.pots_dev = (const sw_potential*)ws;
    L.offsets_dev = (const int64_t*)(ws + align256((size_t)n_pot * sizeof(sw_potential)));
    SW_HIP(hipMemcpyAsync((void*)L.pots_dev, pots, (size_t)n_pot * sizeof(sw_potential), hipMemcpyHostToDevice, st));
    SW_HIP(hipMemcpyAsync((void*)L.offsets_dev, orbit_offsets, (size_t)(n_pot + 1) * sizeof(int64_t),
                          hipMemcpyHostToDevice, st));
  }
  L.obs = O;
  L.ics = ics;
  L.dt = dt;
  L.n_orb = n_orb;
  L.n_steps = n_steps;
  L.ev_m = (uint64_t*)(ws + hdr);
  L.ev_k = (uint64_t*)(ws + hdr + align256((size_t)chunk * n_steps * sizeof(uint64_t)));
  L.drift = drift;
  L.flags = flags;
  L.bin = true;
  const int64_t n_con = (int64_t)O.n_mass + O.n_kin + (O.surface ? O.n_ap : 0);
  for (int64_t orb0 = 0; orb0 < n_orb; orb0 += chunk) {
    L.orb0 = orb0;
    L.n_chunk = (n_orb - orb0 < chunk) ? n_orb - orb0 : chunk;
    SW_HIP(dtype == SW_F32 ? launch_integrate_f32(L, st) : launch_integrate_f64(L, st));
    int rc;
    if (dtype == SW_F32) {
      rc = launch_hist<float>(L.ev_m, L.n_chunk, n_steps, O.ncopy, O.n_mass, orb0, n_con, 0, A, overflow, 0, st);
      if (rc == SW_OK)
        rc = launch_hist<float>(L.ev_k, L.n_chunk, n_steps, O.ncopy, O.n_kin, orb0, n_con, O.n_mass, A, overflow, 1, st);
      if (rc == SW_OK && O.surface)
        rc = launch_hist<float>(L.ev_k, L.n_chunk, n_steps, O.ncopy, O.n_ap, orb0, n_con, O.n_mass + O.n_kin, A,
                                overflow, -1, st, O.nv, O.n_kin, upsilon);
    } else {
      rc = launch_hist<double>(L.ev_m, L.n_chunk, n_steps, O.ncopy, O.n_mass, orb0, n_con, 0, A, overflow, 0, st);
      if (rc == SW_OK)
        rc = launch_hist<double>(L.ev_k, L.n_chunk, n_steps, O.ncopy, O.n_kin, orb0, n_con, O.n_mass, A, overflow, 1, st);
      if (rc == SW_OK && O.surface)
        rc = launch_hist<double>(L.ev_k, L.n_chunk, n_steps, O.ncopy, O.n_ap, orb0, n_con, O.n_mass + O.n_kin, A,
                                 overflow, -1, st, O.nv, O.n_kin, upsilon);
    }
    if (rc != SW_OK) return rc;
  }
  return SW_OK;
}

template <typename T>
static void launch_bin_points(bool cyl, dim3 grid, dim3 block, hipStream_t st, const PotK& P, const ObsK& O,
                              const T* pts, int64_t n, int32_t* mass, int32_t* kin) {
  if (cyl)
    hipLaunchKernelGGL((k_bin_points<T, true>), grid, block, 0, st, P, O, pts, n, mass, kin);
  else
    hipLaunchKernelGGL((k_bin_points<T, false>), grid, block, 0, st, P, O, pts, n, mass, kin);
}

extern "C" int bin_points(const sw_potential* pot, const sw_obs_spec* obs, const void* pts, int64_t n, int32_t dtype,
                          int32_t* mass, int32_t* kin, void* stream) {
  SW_CHECK(pot && obs, "bin_points: null argument");
  SW_CHECK(dtype == SW_F32 || dtype == SW_F64, "bin_points: dtype must be SW_F32 or SW_F64");
  SW_CHECK(n >= 0, "bin_points: n must be >= 0");
  ObsK O;
  SW_CHECK(obs_to_k(obs, &O), "bin_points: invalid observable specification");
  if (n == 0) return SW_OK;
  SW_CHECK(pts && mass && kin, "bin_points: null device buffer");
  PotK P;
  std::memcpy(&P, pot, sizeof P);
  dim3 grid((unsigned)((n + 255) / 256)), block(256);
  hipStream_t st = (hipStream_t)stream;
  if (dtype == SW_F32)
    launch_bin_points<float>(O.cyl != 0, grid, block, st, P, O, (const float*)pts, n, mass, kin);
  else
    launch_bin_points<double>(O.cyl != 0, grid, block, st, P, O, (const double*)pts, n, mass, kin);
  SW_HIP(hipGetLastError());
  return SW_OK;
}

extern "C" int integrate_orbits(const sw_potential* pot, const void* ics, const void* dt, int64_t n, int32_t n_steps,
                                int32_t dtype, void* out, void* stream) {
  SW_CHECK(pot, "integrate_orbits: null potential");
  SW_CHECK(dtype == SW_F32 || dtype == SW_F64, "integrate_orbits: dtype must be SW_F32 or SW_F64");
  SW_CHECK(n >= 0 && n_steps >= 0, "integrate_orbits: need n >= 0 and n_steps >= 0");
  if (n == 0) return SW_OK;
  SW_CHECK(ics && dt && out, "integrate_orbits: null device buffer");
  IntegrateLaunch L;
  std::memset(&L, 0, sizeof L);
  std::memcpy(&L.p0, pot, sizeof(PotK));
  L.n_pot = 1;
  L.needle = has_needle(pot);
  L.obs.drift_every = 0;
  L.ics = ics;
  L.dt = dt;
  L.n_orb = n;
  L.orb0 = 0;
  L.n_chunk = n;
  L.n_steps = n_steps;
  L.final_state = out;
  L.bin = false;
  hipStream_t st = (hipStream_t)stream;
  SW_HIP(dtype == SW_F32 ? launch_integrate_f32(L, st) : launch_integrate_f64(L, st));
  return SW_OK;
}
