// Internal definitions shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/schw.h"

namespace sw {

constexpr double kG = 4.300917270e-6;  // kpc (km/s)^2 / Msun
constexpr int kGL32 = 16;              // bar quadrature nodes, single precision path
constexpr int kGL64 = 32;              // bar quadrature nodes, double precision path

// Derived constants of one component.  Slot meaning per kind:
//  KEPLER    c0 = GM
//  ISOCHRONE c0 = GM, c1 = b, c2 = b^2
//  PLUMMER   c0 = GM, c1 = b^2
//  MN        c0 = GM, c1 = a, c2 = b^2
//  NFW_Q     c0 = G M_DM, c1 = R_s, c2 = 1/q^2, c3 = q^2, c4 = G M_DM / R_s^2, c5 = 1 / R_s
//  FERRERS2  c0..2 = a^2, b^2, c^2, c3 = smallest of them,
//            c4 = 2 pi G a b c rho_c (force), c5 = pi G a b c rho_c / 3 (potential),
//            c6 = largest squared axis
struct CompK {
  int32_t kind;
  int32_t pad;
  double c[12];
  float f[12];  // the same constants rounded to single precision
};

struct PotK {
  int32_t n_comp;
  int32_t pad[3];
  CompK comp[SW_MAX_COMP];
  double omega;
  double R[9];  // row-major Eq. 1 projection
  float Rf[9];
  // Gauss-Legendre rule on t in (0,1) after u = lam + K (1/t^2 - 1):
  // q_n = 1/t_n^2 - 1 and W_n = w_n * 2 / t_n^3
  float gq32[kGL32], gw32[kGL32];
  double gq64[kGL64], gw64[kGL64];
};
static_assert(sizeof(PotK) <= sizeof(sw_potential), "PotK does not fit sw_potential");

constexpr int kMaxSectors = 32;  // azimuthal sectors of the cylindrical mass grid
struct ObsK {
  int32_t nx, ny, nz, npx, npy, nv, n_ap, ncopy, n_mass, n_kin;
  double lo[3], inv[3], plo[2], pinv[2], vlo, vinv;
  float lof[3], invf[3], plof[2], pinvf[2], vlof, vinvf;
  const int32_t* pix2ap;
  int32_t drift_every;
  // cylindrical mass grid: R-edge spacing, sector edge directions (cos, sin) of
  // -pi + 2 pi k / ny, k = 0..ny, in both precisions
  int32_t cyl;
  int32_t surface;  // surface-density block on: out-of-range velocities keep their aperture
  double rw;
  float rwf;
  double sc[kMaxSectors + 1], ss[kMaxSectors + 1];
  float scf[kMaxSectors + 1], ssf[kMaxSectors + 1];
};

void set_error(const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
bool obs_to_k(const sw_obs_spec* o, ObsK* k);

// Workgroup shape of the compressed passes of the weight solve, set through
// sw_set_tuning (0 = automatic):
//  g_sparse_rows   orbits per row-dot workgroup
//  g_sparse_cols   constraints per column-sum workgroup
//  g_sparse_lanes  lanes per row in the row dots (16 or 64)
//  g_rhs_group     right-hand sides of one shared matrix per workgroup (1, 2, 4, 8)
//  g_factor_x3     1: the factorisation's large products on bf16x3 MFMA, 0: fp32 MFMA
extern int g_factor_x3;
//  g_gram_dense    1: the Gram streams every 32-orbit stage (no zero-panel skipping)
//  g_refine_two    1: two passes over A per FP64 iteration (U^T U x carried), 0: four
extern int g_gram_dense;
extern int g_refine_two;
//  g_trmv_rows     rows per wave of the inverse factor's triangle passes: 16 (row-blocked) or 2
extern int g_trmv_rows;
//  g_gram_counts   1: a matrix of counts (solve opts.quantum) enters the Gram as its counts
extern int g_gram_counts;
//  g_refine_rebound  two-pass FP64 stage: falls back to four passes when a KKT residual exceeds this times its minimum
extern int g_refine_rebound;
//  g_refine_rebound_checks  ... at this many consecutive convergence checks
extern int g_refine_rebound_checks;
//  g_multi_dense   shared-matrix solves: 0 picks dense MFMA or compressed passes by cost, 1 dense, 2 compressed
extern int g_multi_dense;
extern int g_sparse_rows;
extern int g_sparse_cols;
extern int g_sparse_lanes;
extern int g_rhs_group;

}  // namespace sw

#define SW_HIP(call)                                              \
  do {                                                            \
    hipError_t e_ = (call);                                       \
    if (e_ != hipSuccess) return ::sw::hip_fail(e_, #call);       \
  } while (0)

#define SW_CHECK(cond, ...)             \
  do {                                  \
    if (!(cond)) {                      \
      ::sw::set_error(__VA_ARGS__);     \
      return SW_EINVAL;                 \
    }                                   \
  } while (0)
