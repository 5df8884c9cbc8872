// solve_weights(_batched), chi2 and model_observables (Sec. 2.3-2.4, Eq. 3-5).
//
// Scaled problem (Eq. 4): U[n][i] = w~ A[i][n] / sigma_n, y_n = d_n / sigma_n,
// minimise 1/2 ||U w' - y||^2 + (mu/2) ||w'||^2, w' >= 0, mu = 2 lambda / N.
//
// ADMM with the splitting x = z (Sec. 2.3): the x-update is the ridge solve
//   (U^T U + rho' I) x = q + rho (z - u),  q = U^T y,  rho' = rho + mu,
// done in constraint space with the Woodbury identity
//   x = (1/rho') (b - U^T (rho' I + U U^T)^{-1} U b),
// where U U^T is formed once by the MFMA Gram kernel, then factorised
// (blocked Cholesky) and its factor inverted once (W = L^-1, recursive blocks
// on MFMA GEMMs), so that every x-update applies (rho' I + U U^T)^-1 = W^T W
// as two HBM-bound matrix-vector passes; the z-update clips to w >= 0 (over-relaxed) and u carries the
// scaled dual.  Every pass over U streams A itself (orbit-major)
// with the scaling folded into per-constraint multipliers:
//   column sums   t_n = (w~/sigma_n) sum_i A[i][n] v_i       (U v)
//   row dots      h_i = sum_n A[i][n] (w~ s_n / sigma_n)     (U^T s)
// both accumulated in double precision.
//
// Stage 1 keeps the iterates in fp32 and uses the factor of the (bf16 or fp32)
// Gram directly.  Stage 2 (refinement) keeps them in fp64 and makes each
// x-update exact up to the preconditioner's contraction: the residual of the
// ridge system is formed with fp64-accumulated passes over A and corrected
// with one application of the Woodbury preconditioner.  The KKT natural
// residual of the true problem is evaluated in fp64.
//
// A batch of independent problems (e.g. many walkers' trial potentials) is
// solved together: the orbits of problem b are rows [off[b], off[b+1]) of A,
// every kernel launch covers all problems, and a problem that has converged
// is frozen by a per-problem flag while the others continue.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "gemm.h"

namespace sw {

constexpr int kRowsBlock = 256;   // row-dot workgroup: 4 waves, one row per wave
constexpr int kColThreads = 256;
constexpr int kColsPerThread = 4;
constexpr int kColTile = kColThreads * kColsPerThread;
constexpr int kSlabs = 256;       // orbit slabs per problem in the column-sum reduction
constexpr int kPar = 8;           // per-problem scalars: wt, rho, rho', mu, alpha, active
constexpr int kAcc = 16;          // per-problem accumulators
constexpr double kMaxDensity = 0.30;  // largest fill of A stored compressed
constexpr int kScanBlock = 1024;     // device prefix sums: elements per workgroup (256 threads x 4)
constexpr int kAAMem = 10;          // Anderson acceleration: iterations kept in the history
constexpr int kAAThreads = 256, kAAPer = 4, kAAChunk = kAAThreads * kAAPer;  // AA passes: orbits per workgroup
constexpr int kAADots = 2 * kAAMem + 1;
constexpr int kAAComp = 4;
constexpr int kDenseChunks = 16;  // dense passes of a shared matrix: at most this many K chunks  // history components: x, z, u (mixed and fitted) and h = U^T U x (mixed only)
constexpr double kAARestart = 10.0;  // history cleared when the residual exceeds this many times its minimum
constexpr int kStallChecks = 10;    // stage 1 stalls when max(primal, dual) residual has not
constexpr double kStallRatio = 0.95;  // dropped below 0.95x its value kStallChecks checks earlier

int g_sparse_rows = 0;
int g_gram_dense = 0;
int g_refine_two = 1;
int g_trmv_rows = 16;
int g_gram_counts = 1;
int g_refine_rebound = 10;
int g_refine_rebound_checks = 3;
int g_multi_dense = 0;
int g_sparse_cols = 0;
int g_sparse_lanes = 0;
int g_rhs_group = 0;

static size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }

// last b with off[b] <= i
__device__ __forceinline__ int find_problem(const int64_t* __restrict__ off, int n, int64_t i) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------------------
// X[n][xoff_b + j] = w~_b A[off_b + p_j][n] / sigma_b,n (zero-padded, masked
// orbits zero): constraint-major operand of the Gram, its columns in the orbit
// order p = perm[off_b ..] (the rows' order when perm is null), row-major (fp32)
// or stage-blocked (bf16 pair, gram_at).  64 x 64 LDS tiles.
// ---------------------------------------------------------------------------
template <typename TA>
__global__ __launch_bounds__(256) void k_prep_x(const TA* __restrict__ A, int64_t C, int64_t Npt,
                                                const int64_t* __restrict__ off, const int64_t* __restrict__ xoff,
                                                int nprob, const double* __restrict__ sigma,
                                                const double* __restrict__ par, const uint8_t* __restrict__ mask,
                                                int mode, __bf16* __restrict__ hi, __bf16* __restrict__ lo,
                                                float* __restrict__ xf, const int32_t* __restrict__ perm) {
  __shared__ float tile[64][65];
  const int64_t n0 = (int64_t)blockIdx.x * 64, c0 = (int64_t)blockIdx.y * 64;
  const int b = find_problem(xoff, nprob, c0);
  const int64_t nb = off[b + 1] - off[b];
  const double wt = par[b * kPar + 0];
  const double* sg = sigma + (int64_t)b * C;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += 4) {
    const int64_t j = c0 - xoff[b] + r, n = n0 + tx;
    float v = 0.0f;
    if (j < nb && n < C) {
      const int64_t i = off[b] + (perm ? perm[off[b] + j] : j);
      if (!(mask && mask[i])) v = (float)((double)A[i * C + n] * (wt / sg[n]));
    }
    tile[r][tx] = v;
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int64_t n = n0 + r, col = c0 + tx;
    const float v = tile[tx][r];
    if (mode == SW_GRAM_F32) {
      xf[n * Npt + col] = v;
    } else {
      const int64_t at = gram_at(n, col, Npt);
      const __bf16 h = (__bf16)v;
      hi[at] = h;
      if (mode == SW_GRAM_BF16X3) lo[at] = (__bf16)(v - (float)h);
    }
  }
}

// The same operand for the bf16 modes, one 256 x 32 stage block per workgroup:
// thread t owns row n0 + t of the block (a constraint) and its 32 orbit
// columns, so the reads of each orbit are 1 KB runs of A's row and the block is
// written as 64 contiguous bytes per thread (16 KB per plane, front to back).
// inv_q > 0 (a matrix of counts of quantum 1 / inv_q): the operand is the
// counts themselves, hi + lo exact below 65536 and lo zero up to 256; the Gram
// then scales its entries by the count scale of k_count_scale.
template <typename TA, bool X3>
__global__ __launch_bounds__(256) void k_prep_xb(const TA* __restrict__ A, int64_t C, int64_t Npt,
                                                 const int64_t* __restrict__ off, const int64_t* __restrict__ xoff,
                                                 int nprob, const double* __restrict__ sigma,
                                                 const double* __restrict__ par, const uint8_t* __restrict__ mask,
                                                 __bf16* __restrict__ hi, __bf16* __restrict__ lo,
                                                 const int32_t* __restrict__ perm, double inv_q) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;  // row of X (constraint)
  const int64_t c0 = (int64_t)blockIdx.y * 32;                 // first column of the stage
  const int b = find_problem(xoff, nprob, c0);                   // stages never straddle problems
  const int64_t nb = off[b + 1] - off[b];
  const double sc = n < C ? par[b * kPar + 0] / sigma[(int64_t)b * C + n] : 0.0;
  __bf16 h[32], l[32];
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    const int64_t jj = c0 - xoff[b] + j;
    float v = 0.0f;
    if (jj < nb && n < C) {
      const int64_t i = off[b] + (perm ? perm[off[b] + jj] : jj);
      if (!(mask && mask[i])) v = inv_q > 0.0 ? (float)rint((double)A[i * C + n] * inv_q) : (float)((double)A[i * C + n] * sc);
    }
    h[j] = (__bf16)v;
    if constexpr (X3) l[j] = (__bf16)(v - (float)h[j]);
  }
  __bf16* ph = hi + gram_at(n, c0, Npt);
  __bf16* pl = lo + gram_at(n, c0, Npt);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    *reinterpret_cast<uint4*>(ph + 8 * q) = *reinterpret_cast<const uint4*>(h + 8 * q);
    if constexpr (X3) *reinterpret_cast<uint4*>(pl + 8 * q) = *reinterpret_cast<const uint4*>(l + 8 * q);
  }
}

// ---------------------------------------------------------------------------
// Dense passes of one shared matrix over all right-hand sides on FP64 MFMA
// (v_mfma_f64_16x16x4): out[m][z][n] = sum over k in chunk z of V[m][k] B(k, n),
//   column sums  V = the orbit vectors [P][n_a] (k = orbit), B(k, n) = A[k][n];
//   row dots     V = the scaled constraint vectors [P][Cp] (k = constraint),
//                B(k, n) = A[n][k] (TRANSB).
// Used when the matrix is dense enough that streaming it once per pass for all
// right-hand sides beats the compressed passes, which read it once per group of
// a few (the fit matrices with Gauss-Hermite blocks).  A 256-thread workgroup
// owns a 128 x 64 output tile (vectors x outputs; four waves of 64 x 32 = 4 x 2
// MFMA blocks of 16 x 16, so the matrix is read once per pass for up to 128
// vectors) and one chunk of K.  Both operands are staged through LDS 16 at a
// time as [row][k] tiles whose rows are padded to 17 doubles, so that the
// MFMA operand reads (16 rows at one k per quarter-wave) and the staging
// writes fall in distinct banks; consecutive lanes load consecutive addresses
// of A and of the vectors (a wave's load touches 4 rows, or one, of 128 bytes
// or more), whichever way A is walked.  Double-buffered: the next k-step is
// loaded into registers while the current one is multiplied, one barrier per
// step.  The chunks' partials are summed in order by the reductions of the
// compressed passes.
// ---------------------------------------------------------------------------
typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int kDM = 128, kDN = 64, kDK = 16;
constexpr int kDKP = kDK + 1;

template <typename TV, typename TA, bool TRANSB>
__global__ __launch_bounds__(256) void k_dgemm_rhs(int64_t M, int64_t Nn, int64_t K, const TV* __restrict__ V,
                                                   int64_t ldv, const TA* __restrict__ A, int64_t lda, int64_t kc,
                                                   double* __restrict__ out, int64_t ldo, int64_t so) {
  __shared__ double Vs[2][kDM][kDKP];  // [m][k]
  __shared__ double Bs[2][kDN][kDKP];  // [n][k]
  const int64_t m0 = (int64_t)blockIdx.y * kDM, n0 = (int64_t)blockIdx.x * kDN;
  const int64_t k_beg = (int64_t)blockIdx.z * kc;
  const int64_t k_end = k_beg + kc < K ? k_beg + kc : K;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  f64x4 acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  // staging: element e = tid + 256 q of the V tile is row e / 16, k e % 16; of the
  // A tile, TRANSB (A[n][k]) row n = e / 16, k e % 16, else (A[k][n]) k = e / 64,
  // n = e % 64: consecutive lanes read consecutive addresses
  const int64_t vrow = m0 + (tid >> 4), vcol = tid & 15;
  const TV* __restrict__ Vp = V + vrow * ldv + vcol;
  double rv[8], rb[4];
  auto gload = [&](int64_t k0) {
    const bool kin = k0 + vcol < k_end;
#pragma unroll
    for (int j = 0; j < 8; ++j)
      rv[j] = (kin && vrow + 16 * j < M) ? (double)Vp[16 * j * ldv + k0] : 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int e = tid + 256 * j;
      if (TRANSB) {  // A[n][k]
        const int64_t n = n0 + (e >> 4), k = k0 + (e & 15);
        rb[j] = (n < Nn && k < k_end) ? (double)A[n * lda + k] : 0.0;
      } else {  // A[k][n]
        const int64_t k = k0 + (e >> 6), n = n0 + (e & 63);
        rb[j] = (n < Nn && k < k_end) ? (double)A[k * lda + n] : 0.0;
      }
    }
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int j = 0; j < 8; ++j) Vs[buf][(tid >> 4) + 16 * j][vcol] = rv[j];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int e = tid + 256 * j;
      if (TRANSB) Bs[buf][e >> 4][e & 15] = rb[j];
      else Bs[buf][e & 63][e >> 6] = rb[j];
    }
  };
  int buf = 0;
  if (k_beg < k_end) {
    gload(k_beg);
    stage(0);
  }
  __syncthreads();
  for (int64_t k0 = k_beg; k0 < k_end; k0 += kDK) {
    const bool more = k0 + kDK < k_end;
    if (more) gload(k0 + kDK);
#pragma unroll
    for (int ks = 0; ks < kDK; ks += 4) {
      const int kr = ks + (lane >> 4);
      double av[4], bv[2];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = Vs[buf][wm * 64 + a * 16 + (lane & 15)][kr];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = Bs[buf][wn * 32 + b * 16 + (lane & 15)][kr];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    // the other buffer was last read before the previous barrier
    if (more) stage(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  out += (int64_t)blockIdx.z * so;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // f64 16x16 output: element r of lane l is row 4 r + l / 16, column l % 16
        const int64_t m = m0 + wm * 64 + a * 16 + 4 * r + (lane >> 4);
        const int64_t n = n0 + wn * 32 + b * 16 + (lane & 15);
        if (m < M && n < Nn) out[m * ldo + n] = acc[a][b][r];
      }
}

// cs[a][n] = q w~_a / sigma_n (0 past the constraints): the scale of a count
// matrix's Gram, K[m][n] = cs[m] cs[n] sum_i k_im k_in
__global__ __launch_bounds__(256) void k_count_scale(const double* __restrict__ sigma, int64_t sS, int64_t C,
                                                     int64_t Cp, const double* __restrict__ par, double q,
                                                     float* __restrict__ cs) {
  const int a = blockIdx.y;
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n < Cp) cs[a * Cp + n] = n < C ? (float)(q * par[a * kPar + 0] / sigma[a * sS + n]) : 0.0f;
}

// ---------------------------------------------------------------------------
// Zero-panel bits of the Gram operand: bit g of nz[t * nzw + g / 64] is set when
// rows [256 t, 256 t + 256) of X (the hi plane, stage-blocked) hold a nonzero in
// columns [32 g, 32 g + 32).  Workgroup (word, tile): each of the 4 waves scans
// 16 of the word's 64 stage blocks, one 16 KB block at a time.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_nz_bits(const __bf16* __restrict__ hi, int64_t Npt, int64_t nzw,
                                                 uint64_t* __restrict__ nz) {
  __shared__ uint32_t part[4];
  const int64_t wd = blockIdx.x, t = blockIdx.y;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t bits = 0;
  for (int i = 0; i < 16; ++i) {
    const int64_t g = wd * 64 + w * 16 + i;
    if (g * 32 >= Npt) break;
    const uint4* p = reinterpret_cast<const uint4*>(hi + gram_at(t * 256, g * 32, Npt));
    uint32_t any = 0;
    for (int j = 0; j < 16; ++j) {
      const uint4 v = p[lane + 64 * j];
      any |= (v.x | v.y | v.z | v.w) & 0x7fff7fffu;
    }
    if (__ballot(any != 0)) bits |= 1u << i;
  }
  if (lane == 0) part[w] = bits;
  __syncthreads();
  if (threadIdx.x == 0)
    nz[t * nzw + wd] = (uint64_t)part[0] | ((uint64_t)part[1] << 16) | ((uint64_t)part[2] << 32) |
                       ((uint64_t)part[3] << 48);
}

// ---------------------------------------------------------------------------
// Column sums over orbit slabs: part[b][s][n] = sum_{i in slab s of b} A[i][n] v_i.
// ---------------------------------------------------------------------------
template <typename TA, typename TV>
__global__ __launch_bounds__(kColThreads) void k_colsum(const TA* __restrict__ A, int64_t C,
                                                        const TV* __restrict__ v, const int64_t* __restrict__ off,
                                                        const int64_t* __restrict__ rps, const double* __restrict__ par,
                                                        int shared, double* __restrict__ part) {
  const int b = blockIdx.z;
  if (par[b * kPar + 5] == 0.0) return;  // converged problem: frozen
  const int64_t c0 = (int64_t)blockIdx.x * kColTile;
  const int64_t s = blockIdx.y;
  const int64_t i_beg = off[b] + s * rps[b];
  int64_t i_end = i_beg + rps[b];
  if (i_end > off[b + 1]) i_end = off[b + 1];
  double acc[kColsPerThread] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t i = i_beg; i < i_end; ++i) {
    const double vi = (double)v[i];
    if (vi == 0.0) continue;
    const TA* row = A + (shared ? i - off[b] : i) * C;
#pragma unroll
    for (int k = 0; k < kColsPerThread; ++k) {
      const int64_t c = c0 + threadIdx.x + k * kColThreads;
      if (c < C) acc[k] += (double)row[c] * vi;
    }
  }
  double* pb = part + ((int64_t)b * kSlabs + s) * C;
#pragma unroll
  for (int k = 0; k < kColsPerThread; ++k) {
    const int64_t c = c0 + threadIdx.x + k * kColThreads;
    if (c < C) pb[c] = acc[k];
  }
}

// ---------------------------------------------------------------------------
// Compressed copies of A.  The orbit matrix is mostly zeros (an orbit visits a
// small part of the grid), so the ADMM passes read compressed rows
// (orbit-major, for the row dots) and compressed columns (constraint-major,
// for the column sums), built once per solve from the dense A.
//
// Both are blocked so that the vector they gather from fits in LDS: a
// gather from L2 costs one cache request per lane and caps a pass at the L2
// request rate, a gather from LDS does not.
//  * rows: column blocks of kBlk constraints; segment (i, cb) holds the
//    entries of row i in block cb, at [rptr[i*ncb + cb], rptr[i*ncb + cb + 1]);
//    16-bit column index within the block.
//  * columns: per problem, row blocks of whole orbit slabs (at most kBlk
//    orbits); segment (b, rb, c) at [cptr[(b*nrb + rb)*(C+1) + c], ... + 1);
//    16-bit orbit index within the block.
// Every segment is padded with zero entries (index 0) to a whole quad of 4,
// so entries are read four at a time with one vector load.
// ---------------------------------------------------------------------------
constexpr int kBlk = 16384;       // gathered entries staged in LDS (fp64: 128 KB)
constexpr int kSpThreads = 1024;  // workgroup of the blocked passes (16 waves)
constexpr int kSpWaves = kSpThreads / 64;
constexpr int kMaxRowsWG = 512;   // blocked passes: at most 512 rows (row dots) or columns per workgroup
constexpr int kRhsGroup = 4;      // right-hand sides per workgroup in the passes of a shared matrix (at most 8)
constexpr int kRhsItems = 1024;   // rows (row dots) or columns (column sums) per workgroup of those passes
// Block of those passes: R interleaved values per index at a stride of R + 1
// doubles (an odd stride spreads the random gathers over the LDS banks; at a
// stride of R = 8 doubles every lane's first 16 bytes would fall in one of
// two bank groups), sized to about 150 KB of LDS
__host__ __device__ constexpr int64_t rhs_blk(int R) { return R <= 2 ? 6400 : (R <= 4 ? 3840 : 2048); }

// orbit rows per column-block segment: slabs of rps rows, whole slabs per
// block of blk rows (kBlk, or rhs_blk(R) when R right-hand sides share the LDS)
__host__ __device__ __forceinline__ int64_t slabs_per_block(int64_t rps, int64_t blk = kBlk) {
  return rps >= blk ? 1 : blk / rps;
}

// cnt[i][cb] = nonzeros of row i in column block cb (one wave per row);
// foot[i] = the row's footprint on the Gram's panels: word 0 the number of
// 256-column tiles holding a nonzero, words 1-4 the bitmap of those tiles
// (tile t at bit t % 64 of word 1 + t / 64, tiles past 255 folded onto
// t % 256); blk is a multiple of 256
template <typename TA>
__global__ __launch_bounds__(256) void k_row_nnz(const TA* __restrict__ A, int64_t N, int64_t C, int ncb, int64_t blk,
                                                 int64_t* __restrict__ cnt, uint64_t* __restrict__ foot) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= N) return;
  const TA* row = A + i * C;
  uint64_t nt = 0, bits[4] = {0, 0, 0, 0};
  int64_t last = -1;
  for (int cb = 0; cb < ncb; ++cb) {
    const int64_t c1 = (int64_t)(cb + 1) * blk < C ? (int64_t)(cb + 1) * blk : C;
    int64_t k = 0;
    for (int64_t c0 = (int64_t)cb * blk; c0 < c1; c0 += 64) {
      const bool v = c0 + lane < c1 && row[c0 + lane] != TA(0);
      k += v;
      if (__ballot(v) != 0 && (c0 >> 8) != last) {
        last = c0 >> 8;
        ++nt;
        const int t = (int)(last & 255);
        bits[t >> 6] |= 1ull << (t & 63);
      }
    }
    for (int o = 32; o > 0; o >>= 1) k += __shfl_xor(k, o, 64);
    if (lane == 0) cnt[i * ncb + cb] = k;
  }
  if (lane < 5 && foot) foot[i * 5 + lane] = lane == 0 ? nt : bits[lane - 1];
}

// cpart[b][s][c] = number of nonzeros of column c in slab s of problem b
template <typename TA>
__global__ __launch_bounds__(kColThreads) void k_col_nnz(const TA* __restrict__ A, int64_t C,
                                                         const int64_t* __restrict__ off,
                                                         const int64_t* __restrict__ rps, int32_t* __restrict__ cpart) {
  const int b = blockIdx.z;
  const int64_t c0 = (int64_t)blockIdx.x * kColTile, s = blockIdx.y;
  const int64_t i_beg = off[b] + s * rps[b];
  int64_t i_end = i_beg + rps[b];
  if (i_end > off[b + 1]) i_end = off[b + 1];
  int32_t k[kColsPerThread] = {0, 0, 0, 0};
  for (int64_t i = i_beg; i < i_end; ++i) {
#pragma unroll
    for (int q = 0; q < kColsPerThread; ++q) {
      const int64_t c = c0 + threadIdx.x + q * kColThreads;
      if (c < C) k[q] += A[i * C + c] != TA(0);
    }
  }
#pragma unroll
  for (int q = 0; q < kColsPerThread; ++q) {
    const int64_t c = c0 + threadIdx.x + q * kColThreads;
    if (c < C) cpart[((int64_t)b * kSlabs + s) * C + c] = k[q];
  }
}

// The value stored for a nonzero entry a of A: a itself, or (TS = uint16_t,
// a matrix of counts) the integer k with a the rounding of k q to A's type,
// k in 1..65535; an entry that is no such multiple sets *bad.
template <typename TA, typename TS>
__device__ __forceinline__ TS store_val(TA a, double inv_quant, double quant, int* bad) {
  if constexpr (sizeof(TS) == 2) {
    const double k = rint((double)a * inv_quant);
    const double tol = (sizeof(TA) == 4 ? 0x1p-22 : 0x1p-50) * fabs((double)a);
    if (!(k >= 1.0 && k <= 65535.0 && fabs((double)a - k * quant) <= tol)) atomicOr(bad, 1);
    return (TS)(k >= 1.0 && k <= 65535.0 ? k : 0.0);
  } else {
    return a;
  }
}

// compressed rows: one wave per orbit; ballot + prefix count keeps column
// order; each segment's padding is written as zero entries
template <typename TA, typename TS>
__global__ __launch_bounds__(256) void k_fill_csr(const TA* __restrict__ A, int64_t N, int64_t C, int ncb, int64_t blk,
                                                  const int64_t* __restrict__ ptr, uint16_t* __restrict__ col,
                                                  TS* __restrict__ val, double inv_quant, double quant, int* bad) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= N) return;
  const TA* row = A + i * C;
  for (int cb = 0; cb < ncb; ++cb) {
    const int64_t cbeg = (int64_t)cb * blk;
    const int64_t c1 = cbeg + blk < C ? cbeg + blk : C;
    int64_t pos = ptr[i * ncb + cb];
    for (int64_t c0 = cbeg; c0 < c1; c0 += 64) {
      const int64_t c = c0 + lane;
      const TA v = c < c1 ? row[c] : TA(0);
      const uint64_t m = __ballot(v != TA(0));
      if (v != TA(0)) {
        const int64_t at = pos + __popcll(m & ((1ull << lane) - 1ull));
        col[at] = (uint16_t)(c - cbeg);
        val[at] = store_val<TA, TS>(v, inv_quant, quant, bad);
      }
      pos += __popcll(m);
    }
    if (pos + lane < ptr[i * ncb + cb + 1]) {
      col[pos + lane] = 0;
      val[pos + lane] = TS(0);
    }
  }
}

// compressed columns: slab s of problem b writes its entries of column c
// from the absolute position slab_at[b][s][c] on (padding is pre-cleared)
template <typename TA, typename TS>
__global__ __launch_bounds__(kColThreads) void k_fill_csc(const TA* __restrict__ A, int64_t C,
                                                          const int64_t* __restrict__ off,
                                                          const int64_t* __restrict__ rps,
                                                          const int64_t* __restrict__ slab_at, int64_t blk,
                                                          uint16_t* __restrict__ rowi, TS* __restrict__ val,
                                                          double inv_quant, double quant, int* bad) {
  const int b = blockIdx.z;
  const int64_t c0 = (int64_t)blockIdx.x * kColTile, s = blockIdx.y;
  const int64_t i_beg = off[b] + s * rps[b];
  int64_t i_end = i_beg + rps[b];
  if (i_end > off[b + 1]) i_end = off[b + 1];
  // first orbit of this slab's row block
  const int64_t spb = slabs_per_block(rps[b], blk);
  const int64_t blk0 = off[b] + (s / spb) * spb * rps[b];
  int64_t pos[kColsPerThread];
#pragma unroll
  for (int q = 0; q < kColsPerThread; ++q) {
    const int64_t c = c0 + threadIdx.x + q * kColThreads;
    pos[q] = c < C ? slab_at[((int64_t)b * kSlabs + s) * C + c] : 0;
  }
  for (int64_t i = i_beg; i < i_end; ++i) {
#pragma unroll
    for (int q = 0; q < kColsPerThread; ++q) {
      const int64_t c = c0 + threadIdx.x + q * kColThreads;
      if (c < C) {
        const TA v = A[i * C + c];
        if (v != TA(0)) {
          rowi[pos[q]] = (uint16_t)(i - blk0);
          val[pos[q]] = store_val<TA, TS>(v, inv_quant, quant, bad);
          ++pos[q];
        }
      }
    }
  }
}

// Quads of compressed entries: values and indices of four consecutive
// entries in one vector load each; the streams are read once per pass, so
// the loads are non-temporal.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));

// The values of a quad of compressed entries as loaded (converted when used).
template <typename TA> struct QuadRaw;
template <> struct QuadRaw<uint16_t> {
  u16x4 q;
  __device__ void load(const uint16_t* p) { q = __builtin_nontemporal_load(reinterpret_cast<const u16x4*>(p)); }
  __device__ double operator[](int i) const { return (double)q[i]; }
};
template <> struct QuadRaw<float> {
  f32x4 q;
  __device__ void load(const float* p) { q = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p)); }
  __device__ double operator[](int i) const { return (double)q[i]; }
};
template <> struct QuadRaw<double> {
  f64x2 a, b;
  __device__ void load(const double* p) {
    a = __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(p));
    b = __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(p + 2));
  }
  __device__ double operator[](int i) const { return i < 2 ? a[i] : b[i - 2]; }
};

// lane-partial sum_k val[k] xs[idx[k]] over the segment [k0, k1) (multiples
// of 4) with xs in LDS, for a group of LPR lanes (lane = index in the group):
// lane-strided quads, four of them loaded at once before any is used
// (segments are a few quads per lane, so a loop that waited for each load in
// turn would expose the memory latency); a quad past the segment re-reads the
// lane's first one and is weighted by zero.
template <int LPR = 64, typename TA>
__device__ __forceinline__ double seg_dot(const TA* __restrict__ val, const uint16_t* __restrict__ idx, int64_t k0,
                                          int64_t k1, const double* xs, int lane) {
  constexpr int S = 4 * LPR;  // entries per quad row of the group
  constexpr int U = 4;        // quads in flight per lane
  double a[U] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t k = k0 + 4 * lane; k < k1; k += (int64_t)U * S) {
    QuadRaw<TA> v[U];
    u16x4 c[U];
    double wgt[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool ok = k + (int64_t)u * S < k1;
      const int64_t ka = ok ? k + (int64_t)u * S : k;
      wgt[u] = ok ? 1.0 : 0.0;
      v[u].load(val + ka);
      c[u] = __builtin_nontemporal_load(reinterpret_cast<const u16x4*>(idx + ka));
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) t += v[u][q] * xs[c[u][q]];
      a[u] += wgt[u] * t;
    }
  }
  return (a[0] + a[1]) + (a[2] + a[3]);
}

// sum over the aligned group of LPR lanes (result in every lane of the group)
template <int LPR>
__device__ __forceinline__ double group_sum(double v) {
  for (int o = LPR / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sums R values over an aligned group of LPR lanes (R <= LPR, powers of 2) as
// a reduce-scatter: each halving step trades half of the values with the
// partner lane, so it takes R - 1 + log2(LPR / R) exchanges instead of
// R log2(LPR).  Returns the group total of value `which` (set here); the lanes
// with sl % (LPR / R) == 0 hold the R totals between them.
template <int LPR, int R>
__device__ __forceinline__ double group_scatter_sum(double (&a)[R], int sl, int& which) {
  which = 0;
  int m = LPR / 2;
#pragma unroll
  for (int lev = 0; (R >> lev) > 1; ++lev) {
    const int half = R >> (lev + 1);
    const bool up = (sl & m) != 0;
#pragma unroll
    for (int j = 0; j < half; ++j) {
      const double send = up ? a[j] : a[j + half];
      const double keep = up ? a[j + half] : a[j];
      a[j] = keep + __shfl_xor(send, m, 64);
    }
    if (up) which += half;
    m >>= 1;
  }
  double v = a[0];
  for (; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// The segments of one group of LPR lanes, items p = 0 .. n_pass-1 (rows or
// columns), each dotted with R interleaved right-hand sides in LDS:
// acc[r] = sum_k val[k] xs[idx[k] (R + 1) + r] over [beg_p, end_p) (a
// multiple of 4), lane-strided quads.  Segments are short (a few quads per
// lane), so a lane loads the first Q quads of an item at once, and the loads
// of item p + 1 (and the pointers of item p + 2) are issued before item p is
// summed.  Every load is issued unconditionally (an index past the segment
// reads entry 0 and the quad is weighted by zero): vector-memory counters
// complete in order, and a load skipped on some paths would make the compiler
// wait for the prefetches as well.
//   seg(p, beg, end): bounds of item p (beg = end past the group's items);
//   out(p, which, total) receives the group total of right-hand side `which`
//   (lanes sl % (LPR/R) == 0).
// xs[j (R + 1) + r] = src_r[j] for j < len (src_r = base + off_r, r < R; rows
// of right-hand sides past P read as 0).  All of a thread's loads are issued
// before the first store (clamped addresses, no branches), so the staging
// costs one memory latency rather than one per value.
template <int R, int64_t BLK, typename TV>
__device__ __forceinline__ void rhs_stage(double* xs, const TV* __restrict__ base, const int64_t* roff, int P, int b0,
                                          int len) {
  constexpr int JT = (int)((BLK + kSpThreads - 1) / kSpThreads);
  double t[JT][R];
#pragma unroll
  for (int jj = 0; jj < JT; ++jj) {
    const int j = (int)threadIdx.x + jj * kSpThreads;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool ok = j < len && b0 + r < P;
      t[jj][r] = (double)base[ok ? roff[r] + j : 0];
      if (!ok) t[jj][r] = 0.0;
    }
  }
#pragma unroll
  for (int jj = 0; jj < JT; ++jj) {
    const int j = (int)threadIdx.x + jj * kSpThreads;
    if (j < len)
#pragma unroll
      for (int r = 0; r < R; ++r) xs[j * (R + 1) + r] = t[jj][r];
  }
}

template <int LPR, int R, int Q, typename TA>
struct RhsChunk {
  TA v[Q][4];
  uint16_t c[Q][4];
  bool ok[Q];
};

template <int LPR, int R, int Q, typename TA>
__device__ __forceinline__ void rhs_load(const TA* __restrict__ val, const uint16_t* __restrict__ idx, int64_t base,
                                         int64_t end, int sl, RhsChunk<LPR, R, Q, TA>& ch) {
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int64_t k = base + 4 * sl + (int64_t)i * 4 * LPR;
    ch.ok[i] = k < end;
    const int64_t kk = ch.ok[i] ? k : 0;
    if constexpr (sizeof(TA) == 2) {
      const u16x4 q = __builtin_nontemporal_load(reinterpret_cast<const u16x4*>(val + kk));
      ch.v[i][0] = q[0]; ch.v[i][1] = q[1]; ch.v[i][2] = q[2]; ch.v[i][3] = q[3];
    } else if constexpr (sizeof(TA) == 4) {
      const f32x4 q = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(val + kk));
      ch.v[i][0] = q[0]; ch.v[i][1] = q[1]; ch.v[i][2] = q[2]; ch.v[i][3] = q[3];
    } else {
      const f64x2 q0 = __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(val + kk));
      const f64x2 q1 = __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(val + kk + 2));
      ch.v[i][0] = q0[0]; ch.v[i][1] = q0[1]; ch.v[i][2] = q1[0]; ch.v[i][3] = q1[1];
    }
    const u16x4 c = __builtin_nontemporal_load(reinterpret_cast<const u16x4*>(idx + kk));
    ch.c[i][0] = c[0]; ch.c[i][1] = c[1]; ch.c[i][2] = c[2]; ch.c[i][3] = c[3];
  }
}

template <int LPR, int R, int Q, typename TA>
__device__ __forceinline__ void rhs_use(const RhsChunk<LPR, R, Q, TA>& ch, const double* xs, double acc[R]) {
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double w = ch.ok[i] ? 1.0 : 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double v = w * (double)ch.v[i][q];
      const double* x = xs + (uint32_t)ch.c[i][q] * (R + 1);
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] += v * x[r];
    }
  }
}

template <int LPR, int R, typename TA, typename SegF, typename OutF>
__device__ __forceinline__ void seg_stream_rhs(const TA* __restrict__ val, const uint16_t* __restrict__ idx,
                                               const double* xs, int sl, int n_pass, SegF seg, OutF out) {
  constexpr int Q = sizeof(TA) <= 4 ? 4 : 2;  // quads per lane loaded at once
  constexpr int64_t CH = (int64_t)Q * 4 * LPR;  // entries of the group per chunk
  int64_t b0, e0, b1, e1;
  seg(0, b0, e0);
  seg(1, b1, e1);
  // two chunk buffers in alternating roles (no register copies, which would
  // have to wait for the prefetched loads)
  RhsChunk<LPR, R, Q, TA> ca, cb;
  rhs_load(val, idx, b0, e0, sl, ca);
  auto step = [&](RhsChunk<LPR, R, Q, TA>& use, RhsChunk<LPR, R, Q, TA>& fill, int p) {
    int64_t b2, e2;
    seg(p + 2, b2, e2);
    rhs_load(val, idx, b1, e1, sl, fill);
    // keep the prefetch ahead of the arithmetic (the scheduler would otherwise sink the loads below it)
    __builtin_amdgcn_sched_barrier(0);
    double acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0.0;
    rhs_use(use, xs, acc);
    for (int64_t base = b0 + CH; base < e0; base += CH) {  // items longer than one chunk
      rhs_load(val, idx, base, e0, sl, use);
      rhs_use(use, xs, acc);
    }
    int which;
    const double t = group_scatter_sum<LPR, R>(acc, sl, which);
    out(p, which, t);
    b0 = b1;
    e0 = e1;
    b1 = b2;
    e1 = e2;
  };
  for (int p = 0; p < n_pass; p += 2) {
    step(ca, cb, p);
    if (p + 1 < n_pass) step(cb, ca, p + 1);
  }
}

// column sums from the compressed columns: workgroup (column group of cpw
// columns, problem b), column c owned by wave c mod 16, the problem's orbit
// vector staged block by block in LDS; result in part[b][0][c] (the
// reduction then reads a single slab)
template <typename TA, typename TV>
__global__ __launch_bounds__(kSpThreads) void k_csc_colsum(int64_t C, int cpw, const int64_t* __restrict__ off,
                                                          const int64_t* __restrict__ rps, int nrb,
                                                          const int64_t* __restrict__ cptr,
                                                          const uint16_t* __restrict__ rowi,
                                                          const TA* __restrict__ val, const TV* __restrict__ v,
                                                          const double* __restrict__ par, int shared,
                                                          double* __restrict__ part) {
  __shared__ double xs[kBlk];
  __shared__ double cacc[kMaxRowsWG];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int b = blockIdx.y;
  if (par[b * kPar + 5] == 0.0) return;  // converged problem: frozen
  const int64_t n0 = off[b], nb = off[b + 1] - n0;
  const int64_t brows = slabs_per_block(rps[b]) * rps[b];
  const int64_t c0 = (int64_t)blockIdx.x * cpw;
  if (c0 >= C) return;
  const int nc = (int)(C - c0 < cpw ? C - c0 : cpw);
  for (int q = w; q < nc; q += kSpWaves)
    if (lane == 0) cacc[q] = 0.0;
  for (int rb = 0; rb < nrb && (int64_t)rb * brows < nb; ++rb) {
    const int64_t r0 = (int64_t)rb * brows;
    const int64_t len = nb - r0 < brows ? nb - r0 : brows;
    __syncthreads();
    for (int64_t j = threadIdx.x; j < len; j += kSpThreads) xs[j] = (double)v[n0 + r0 + j];
    __syncthreads();
    const int64_t* cp = cptr + ((int64_t)(shared ? 0 : b) * nrb + rb) * (C + 1);
    for (int q = w; q < nc; q += kSpWaves) {
      const int64_t c = c0 + q;
      const double t = wave_sum(seg_dot(val, rowi, cp[c], cp[c + 1], xs, lane));
      if (lane == 0) cacc[q] += t;
    }
  }
  for (int q = w; q < nc; q += kSpWaves)
    if (lane == 0) part[(int64_t)b * kSlabs * C + c0 + q] = cacc[q];
}

// Column sums for R right-hand sides of one shared matrix: workgroup (column
// chunk, row block rb, right-hand sides g R .. g R + R - 1).  The R orbit
// vectors of the row block (at most blk = rhs_blk(R) orbits) are staged
// interleaved once; a group of 16 lanes takes a column segment, so every
// compressed entry is read once for all R.  Output: the partial sum over the
// row block, part[b][rb][c]; the reduction adds the nrb partials in order.
template <typename TA, typename TV, int R>
__global__ __launch_bounds__(kSpThreads) void k_csc_colsum_rhs(int64_t C, int64_t cpc, int P,
                                                              const int64_t* __restrict__ off,
                                                              const int64_t* __restrict__ rps,
                                                              const int64_t* __restrict__ cptr,
                                                              const uint16_t* __restrict__ rowi,
                                                              const TA* __restrict__ val, const TV* __restrict__ v,
                                                              const double* __restrict__ par,
                                                              double* __restrict__ part) {
  constexpr int LPR = 16, G = 64 / LPR, NS = kSpWaves * G;
  constexpr int64_t blk = rhs_blk(R);
  __shared__ double xs[blk * (R + 1)];
  __shared__ int32_t sp[kRhsItems + 1];  // segment bounds relative to the first (from LDS: the
                                         // pointer reads do not queue behind the data loads)
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int sl = lane % LPR, slot = w * G + lane / LPR;
  const int b0 = blockIdx.z * R;
  bool any = false;
  for (int r = 0; r < R; ++r) any |= b0 + r < P && par[(b0 + r) * kPar + 5] != 0.0;
  if (!any) return;  // every right-hand side of the group has converged
  const int64_t nb = off[1] - off[0];  // orbits of the shared matrix
  const int64_t brows = slabs_per_block(rps[0], blk) * rps[0];
  const int rb = blockIdx.y;
  const int64_t r0 = (int64_t)rb * brows;
  const int64_t c0 = (int64_t)blockIdx.x * cpc;
  if (r0 >= nb || c0 >= C) return;
  const int len = (int)(nb - r0 < brows ? nb - r0 : brows);  // at most blk
  const int64_t nc = C - c0 < cpc ? C - c0 : cpc;
  {
    int64_t ro[R];
#pragma unroll
    for (int r = 0; r < R; ++r) ro[r] = (b0 + r < P ? off[b0 + r] : 0) + r0;
    rhs_stage<R, blk>(xs, v, ro, P, b0, len);
  }
  const int64_t* cp = cptr + (int64_t)rb * (C + 1) + c0;
  const int64_t base = cp[0];
  for (int q = threadIdx.x; q <= nc; q += kSpThreads) sp[q] = (int32_t)(cp[q] - base);
  __syncthreads();
  const int n_pass = (int)((nc + NS - 1) / NS);  // equal for every lane: the group sums see whole waves
  seg_stream_rhs<LPR, R>(
      val, rowi, xs, sl, n_pass,
      [&](int p, int64_t& beg, int64_t& end) {
        const int q = slot + p * NS;
        const int qq = q < nc ? q : 0;
        const int32_t b_ = sp[qq], e_ = sp[qq + 1];
        beg = base + b_;
        end = base + (q < nc ? e_ : b_);
      },
      [&](int p, int which, double t) {
        const int64_t q = slot + (int64_t)p * NS;
        const int b = b0 + which;
        if (q < nc && sl % (LPR / R) == 0 && b < P && par[b * kPar + 5] != 0.0)
          part[((int64_t)b * kSlabs + rb) * C + c0 + q] = t;
      });
}

enum ColOp { COL_PLAIN = 0, COL_ADMM = 1, COL_RESID = 3, COL_OBS = 4 };

// t_n = (w~/sigma_n) sum_s part[b][s][n] (COL_OBS: no scaling), per problem b = blockIdx.y:
//  COL_PLAIN: outd = t, outf = (float) t
//  COL_ADMM:  outf = (float)(kyf + rho t)
//  COL_RESID: outd = t - y,  acc[b][9] += (t - y)^2
//  COL_OBS:   outd = t
// Vectors are [nprob][Cp]; entries in [C, Cp) are written as 0.
__global__ __launch_bounds__(256) void k_colreduce(const double* __restrict__ part, int nslab, int64_t C, int64_t Cp,
                                                   const double* __restrict__ sigma, int64_t sS,
                                                   const double* __restrict__ par,
                                                   int op, const float* __restrict__ kyf, const double* __restrict__ y,
                                                   float* __restrict__ outf, double* __restrict__ outd,
                                                   double* __restrict__ acc, double vscale) {
  const int b = blockIdx.y;
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double wt = par[b * kPar + 0], rho = par[b * kPar + 1];
  const int64_t vb = (int64_t)b * Cp;
  double contrib = 0.0;
  if (n < Cp) {
    double t = 0.0;
    if (n < C) {
      const double* pb = part + (int64_t)b * kSlabs * C;
      for (int64_t s = 0; s < nslab; ++s) t += pb[s * C + n];
      t *= vscale;  // compressed counts: the quantum
      if (op != COL_OBS) t *= wt / sigma[b * sS + n];
    }
    switch (op) {
      case COL_PLAIN:
        if (outd) outd[vb + n] = t;
        if (outf) outf[vb + n] = (float)t;
        break;
      case COL_ADMM:
        outf[vb + n] = (n < C) ? (float)((double)kyf[vb + n] + rho * t) : 0.0f;
        break;
      case COL_RESID: {
        const double e = (n < C) ? t - y[vb + n] : 0.0;
        outd[vb + n] = e;
        contrib = e * e;
        break;
      }
      case COL_OBS:
        if (n < C) outd[vb + n] = t;
        break;
    }
  }
  if (op == COL_RESID && acc) {
    __shared__ double red[256];
    red[threadIdx.x] = contrib;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0 && red[0] != 0.0) atomicAdd(&acc[b * kAcc + 9], red[0]);
  }
}

// sc[b][n] = w~_b s[b][n] / sigma[b][n]: the multiplier of column n in a row dot
// (sigma of problem b at sigma + b * sS: sS = 0 when the problems share one)
template <typename TS>
__global__ void k_colscale(const TS* __restrict__ s, int64_t C, int64_t Cp, const double* __restrict__ sigma,
                           int64_t sS, const double* __restrict__ par, double* __restrict__ sc) {
  const int b = blockIdx.y;
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n < C) sc[(int64_t)b * Cp + n] = par[b * kPar + 0] * (double)s[(int64_t)b * Cp + n] / sigma[b * sS + n];
}

// y[b][n] = d[b][n] / sigma[b][n] (zero padded to Cp)
__global__ void k_scaled_data(const double* __restrict__ d, const double* __restrict__ sigma, int64_t sS, int64_t C,
                              int64_t Cp, double* __restrict__ y) {
  const int b = blockIdx.y;
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n < Cp) y[(int64_t)b * Cp + n] = n < C ? d[(int64_t)b * C + n] / sigma[b * sS + n] : 0.0;
}

enum RowOp { ROW_Q = 0, ROW_ADMM = 1, ROW_H = 2, ROW_CORR = 3, ROW_KKT = 4, ROW_CORR2 = 5 };

struct RowArgs {
  int op;
  int nprob;
  int shared;  // every problem's orbits are rows 0.. of A (vector index i - off[b])
  int64_t Cp;
  const int64_t* off;
  const double* par;
  const uint8_t* mask;
  // fp32 stage
  float* qf; float* zf; float* uf; float* vf;
  // fp64 stage
  double* qd; double* xd; double* zd; double* ud; double* vd; double* rd;
  double* hd;   // fp64 stage, two passes per iteration: h = U^T U x carried with the iterate (null: not carried)
  double* acc;  // per problem [kAcc]: 0 |x-z|^2, 1 |z-zold|^2, 2 |x|^2, 3 |z|^2, 4 |u|^2, 5 max|q|, 6 kkt max, 7 |z|^2, 9 |e|^2
  // orbit-major compressed rows of A (used when A is stored sparse)
  const int64_t* csr_ptr;
  const void* csr_col;  // uint16_t column index within the column block
  const void* csr_val;
  double vscale;        // the dots are multiplied by this (compressed counts: the quantum, else 1)
};


__device__ __forceinline__ void atomic_max_pos(double* a, double v) {
  // non-negative doubles order like their bit patterns
  atomicMax(reinterpret_cast<unsigned long long*>(a), (unsigned long long)__double_as_longlong(v));
}

// Per-row contributions to the accumulators of a pass, summed by the caller
// into 9 doubles: [0..4] ADMM |x-z|^2, |z-z0|^2, |x|^2, |z|^2, |u|^2;
// [5] KKT |z|^2, [6] KKT support size, [7] max |q|, [8] max KKT residual.
// The problem's accumulators receive them once per workgroup.
constexpr int kRowSums = 9;

// The update of orbit row i of problem b once its dot with sc is known.
__device__ __forceinline__ void row_update(const RowArgs& R, int64_t i, int b, double dot, double* a) {
  dot *= R.vscale;
  const double* P = R.par + b * kPar;
  const bool masked = R.mask && R.mask[R.shared ? i - R.off[b] : i];
  const double rho = P[1], rhop = P[2], mu = P[3], alpha = P[4];
  const bool acc = R.acc != nullptr;
  switch (R.op) {
    case ROW_Q: {
      const double q = masked ? 0.0 : dot;
      R.qd[i] = q;
      R.qf[i] = (float)q;
      if (acc) a[7] = fmax(a[7], fabs(q));
      break;
    }
    case ROW_ADMM: {
      const double z0 = R.zf[i], u0 = R.uf[i];
      const double x = masked ? 0.0 : ((double)R.qf[i] + rho * (double)R.vf[i] - dot) / rhop;
      const double xh = alpha * x + (1.0 - alpha) * z0;
      const double z = masked ? 0.0 : fmax(0.0, xh + u0);
      const double u = masked ? 0.0 : u0 + xh - z;
      R.zf[i] = (float)z;
      R.uf[i] = (float)u;
      R.vf[i] = (float)(z - u);
      if (acc) {
        a[0] += (x - z) * (x - z);
        a[1] += (z - z0) * (z - z0);
        a[2] += x * x;
        a[3] += z * z;
        a[4] += u * u;
      }
      break;
    }
    case ROW_H: {
      const double bb = R.qd[i] + rho * R.vd[i];
      R.rd[i] = masked ? 0.0 : bb - dot - rhop * R.xd[i];
      if (R.hd) R.hd[i] = masked ? 0.0 : dot;
      break;
    }
    case ROW_CORR2: {
      // the correction of ROW_CORR, carrying h = U^T U x along: the Woodbury step
      // moves U x by U M r = s (exactly for the exact inverse), so U^T U x moves by
      // U^T s = dot, and the next iteration's residual needs no pass over A
      const double z0 = R.zd[i], u0 = R.ud[i];
      const double x = masked ? 0.0 : R.xd[i] + (R.rd[i] - dot) / rhop;
      const double xh = alpha * x + (1.0 - alpha) * z0;
      const double z = masked ? 0.0 : fmax(0.0, xh + u0);
      const double u = masked ? 0.0 : u0 + xh - z;
      const double h = masked ? 0.0 : R.hd[i] + dot;
      R.xd[i] = x;
      R.zd[i] = z;
      R.ud[i] = u;
      R.vd[i] = z - u;
      R.hd[i] = h;
      R.rd[i] = masked ? 0.0 : R.qd[i] + rho * (z - u) - h - rhop * x;
      break;
    }
    case ROW_CORR: {
      const double z0 = R.zd[i], u0 = R.ud[i];
      const double x = masked ? 0.0 : R.xd[i] + (R.rd[i] - dot) / rhop;
      const double xh = alpha * x + (1.0 - alpha) * z0;
      const double z = masked ? 0.0 : fmax(0.0, xh + u0);
      const double u = masked ? 0.0 : u0 + xh - z;
      R.xd[i] = x;
      R.zd[i] = z;
      R.ud[i] = u;
      R.vd[i] = z - u;
      break;
    }
    case ROW_KKT: {
      const double z = R.zd[i];
      const double g = dot + mu * z;
      const double k = masked ? 0.0 : fabs(fmin(z, g));
      if (acc) {
        a[8] = fmax(a[8], k);
        if (z != 0.0) {
          a[5] += z * z;
          a[6] += 1.0;
        }
      }
      break;
    }
  }
}

// Adds row contributions t[kRowSums] to problem b's accumulators.
__device__ __forceinline__ void add_row_sums(const RowArgs& R, int b, const double* t) {
  double* acc = R.acc + b * kAcc;
  if (R.op == ROW_ADMM)
    for (int k = 0; k < 5; ++k) atomicAdd(&acc[k], t[k]);
  if (R.op == ROW_KKT) {
    if (t[8] > 0.0) atomic_max_pos(&acc[6], t[8]);
    if (t[6] > 0.0) {
      atomicAdd(&acc[7], t[5]);
      atomicAdd(&acc[8], t[6]);
    }
  }
  if (R.op == ROW_Q && t[7] > 0.0) atomic_max_pos(&acc[5], t[7]);
}

// Dense rows: one wave per orbit row, dot = sum_n A[i][n] sc[b][n].
template <typename TA>
__global__ __launch_bounds__(kRowsBlock) void k_rowdot(const TA* __restrict__ A, int64_t N, int64_t C,
                                                       const double* __restrict__ sc, RowArgs R) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * (kRowsBlock / 64) + w;
  if (i >= N) return;
  const int b = find_problem(R.off, R.nprob, i);
  if (R.par[b * kPar + 5] == 0.0 && R.op != ROW_Q) return;  // converged problem: frozen
  const double* scb = sc + (int64_t)b * R.Cp;
  const TA* row = A + (R.shared ? i - R.off[b] : i) * C;
  double dot = 0.0;
  for (int64_t c = lane; c < C; c += 64) dot += (double)row[c] * scb[c];
  dot = wave_sum(dot);
  double a[kRowSums] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (lane == 0) row_update(R, i, b, dot, a);
  if (lane == 0 && R.acc) add_row_sums(R, b, a);  // one row per wave: added directly
}

// Compressed rows: workgroup (row group of rpw rows, problem b); a row is
// taken by a group of LPR lanes (64 for long rows, fewer for short ones, so
// that a wave works on 64 / LPR rows at once); sc of problem b is staged
// column block by column block in LDS.
template <typename TA, int LPR>
__global__ __launch_bounds__(kSpThreads) void k_rowdot_csr(int64_t C, int ncb, int rpw, const double* __restrict__ sc,
                                                           RowArgs R) {
  constexpr int G = 64 / LPR;          // rows in flight per wave
  constexpr int NS = kSpWaves * G;     // row slots of the workgroup
  __shared__ double xs[kBlk];
  __shared__ double racc[kMaxRowsWG];
  __shared__ double sums[NS][kRowSums];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int sl = lane % LPR, slot = w * G + lane / LPR;
  const int b = blockIdx.y;
  const int64_t i_end = R.off[b + 1];
  const int64_t i0 = R.off[b] + (int64_t)blockIdx.x * rpw;
  if (i0 >= i_end) return;
  if (R.par[b * kPar + 5] == 0.0 && R.op != ROW_Q) return;  // converged problem: frozen
  const int nr = (int)(i_end - i0 < rpw ? i_end - i0 : rpw);
  const int n_pass = (nr + NS - 1) / NS;  // the same for every lane, so the group sums see whole waves
  const double* scb = sc + (int64_t)b * R.Cp;
  const TA* val = (const TA*)R.csr_val;
  const uint16_t* col = (const uint16_t*)R.csr_col;
  const int64_t ash = R.shared ? R.off[b] : 0;  // row of A = vector index - ash
  // row r belongs to slot r mod NS throughout, so racc[r] needs no barrier
  for (int r = slot; r < nr; r += NS)
    if (sl == 0) racc[r] = 0.0;
  for (int cb = 0; cb < ncb; ++cb) {
    const int64_t c0 = (int64_t)cb * kBlk;
    const int64_t len = C - c0 < kBlk ? C - c0 : kBlk;
    __syncthreads();
    for (int64_t j = threadIdx.x; j < len; j += kSpThreads) xs[j] = scb[c0 + j];
    __syncthreads();
    for (int p = 0; p < n_pass; ++p) {
      const int r = slot + p * NS;
      double part = 0.0;
      if (r < nr) {
        const int64_t i = i0 + r;
        const int64_t* seg = R.csr_ptr + (i - ash) * ncb + cb;
        part = seg_dot<LPR>(val, col, seg[0], seg[1], xs, sl);
      }
      part = group_sum<LPR>(part);
      if (sl == 0 && r < nr) racc[r] += part;
    }
  }
  // row contributions: per slot in LDS, then combined in slot order
  if (sl == 0)
    for (int k = 0; k < kRowSums; ++k) sums[slot][k] = 0.0;
  for (int r = slot; r < nr; r += NS)
    if (sl == 0) row_update(R, i0 + r, b, racc[r], sums[slot]);
  if (R.acc) {
    __syncthreads();
    const int k = threadIdx.x;  // thread k combines accumulator k over the slots
    if (k < kRowSums) {
      double t = sums[0][k];
      for (int v = 1; v < NS; ++v) t = k >= 7 ? fmax(t, sums[v][k]) : t + sums[v][k];
      sums[0][k] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) add_row_sums(R, b, sums[0]);
  }
}

// Row dots for R right-hand sides of one shared matrix: workgroup (rows
// [x rpw, x rpw + rpw) of the matrix, column block cb, right-hand sides
// g R .. g R + R - 1).  The R multiplier vectors of the column block (blk =
// rhs_blk(R) columns) are staged interleaved once, so every compressed entry is
// read once for all R; the partial dots go to pd[b][cb][row], and
// k_rowdot_fin adds the ncb partials in order and applies the row update.
template <typename TA, int LPR, int R>
__global__ __launch_bounds__(kSpThreads) void k_rowdot_csr_rhs(int64_t C, int ncb, int rpw, int P,
                                                               const double* __restrict__ sc, RowArgs Ra,
                                                               double* __restrict__ pd) {
  constexpr int G = 64 / LPR;
  constexpr int NS = kSpWaves * G;
  constexpr int64_t blk = rhs_blk(R);
  __shared__ double xs[blk * (R + 1)];
  __shared__ int32_t sp[2 * kRhsItems];  // segment bounds relative to the first row's (from LDS)
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int sl = lane % LPR, slot = w * G + lane / LPR;
  const int b0 = blockIdx.z * R;
  bool any = false;
  for (int r = 0; r < R; ++r) any |= b0 + r < P && (Ra.op == ROW_Q || Ra.par[(b0 + r) * kPar + 5] != 0.0);
  if (!any) return;  // every right-hand side of the group has converged
  const int64_t n_a = Ra.off[1] - Ra.off[0];  // orbits of the shared matrix
  const int64_t a0 = (int64_t)blockIdx.x * rpw;
  const int cb = blockIdx.y;
  if (a0 >= n_a) return;
  const int nr = (int)(n_a - a0 < rpw ? n_a - a0 : rpw);
  const int n_pass = (nr + NS - 1) / NS;
  const TA* val = (const TA*)Ra.csr_val;
  const uint16_t* col = (const uint16_t*)Ra.csr_col;
  const int64_t c0 = (int64_t)cb * blk;
  const int len = (int)(C - c0 < blk ? C - c0 : blk);
  {
    int64_t ro[R];
#pragma unroll
    for (int r = 0; r < R; ++r) ro[r] = (int64_t)(b0 + r < P ? b0 + r : 0) * Ra.Cp + c0;
    rhs_stage<R, blk>(xs, sc, ro, P, b0, len);
  }
  const int64_t* rp = Ra.csr_ptr + a0 * ncb + cb;
  const int64_t base = rp[0];
  for (int row = threadIdx.x; row < nr; row += kSpThreads) {
    sp[2 * row] = (int32_t)(rp[(int64_t)row * ncb] - base);
    sp[2 * row + 1] = (int32_t)(rp[(int64_t)row * ncb + 1] - base);
  }
  __syncthreads();
  seg_stream_rhs<LPR, R>(
      val, col, xs, sl, n_pass,
      [&](int p, int64_t& beg, int64_t& end) {
        const int row = slot + p * NS;
        const int rr = row < nr ? row : 0;
        const int32_t b_ = sp[2 * rr], e_ = sp[2 * rr + 1];
        beg = base + b_;
        end = base + (row < nr ? e_ : b_);
      },
      [&](int p, int which, double t) {
        const int row = slot + p * NS;
        const int b = b0 + which;
        if (row < nr && sl % (LPR / R) == 0 && b < P) pd[((int64_t)b * ncb + cb) * n_a + a0 + row] = t;
      });
}

// dot of row i of problem b = sum over the column blocks of pd[b][cb][i] (in
// order), then the row update; the workgroup's accumulator contributions are
// combined in LDS and added once.  Grid (rows / 256, P).
__global__ __launch_bounds__(256) void k_rowdot_fin(int ncb, const double* __restrict__ pd, RowArgs Ra) {
  __shared__ double red[256][kRowSums];
  const int b = blockIdx.y;
  if (Ra.op != ROW_Q && Ra.par[b * kPar + 5] == 0.0) return;  // converged problem: frozen
  const int64_t n_a = Ra.off[1] - Ra.off[0];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double a[kRowSums] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (i < n_a) {
    double dot = 0.0;
    for (int cb = 0; cb < ncb; ++cb) dot += pd[((int64_t)b * ncb + cb) * n_a + i];
    row_update(Ra, Ra.off[b] + i, b, dot, a);
  }
  if (!Ra.acc) return;
  for (int k = 0; k < kRowSums; ++k) red[threadIdx.x][k] = a[k];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int k = 0; k < kRowSums; ++k)
        red[threadIdx.x][k] = k >= 7 ? fmax(red[threadIdx.x][k], red[threadIdx.x + o][k])
                                     : red[threadIdx.x][k] + red[threadIdx.x + o][k];
    __syncthreads();
  }
  if (threadIdx.x == 0) add_row_sums(Ra, b, red[0]);
}

__global__ void k_fill_f32(float* __restrict__ p, int64_t n, float v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_f64(double* __restrict__ p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_i32(int* __restrict__ p, int64_t n, int v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Sum of the first C diagonal entries of K_b, one block per problem, fixed order.
__global__ void k_trace(const float* __restrict__ K, int64_t ld, int64_t sK, int64_t C, double* __restrict__ out) {
  __shared__ double red[256];
  const float* Kb = K + blockIdx.x * sK;
  double s = 0.0;
  for (int64_t n = threadIdx.x; n < C; n += 256) s += (double)Kb[n * ld + n];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

__global__ void k_add_diag(float* __restrict__ K, int64_t ld, int64_t sK, int64_t n, const double* __restrict__ par) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) K[blockIdx.y * sK + i * ld + i] += (float)par[blockIdx.y * kPar + 2];
}

template <typename TS, typename TD>
__global__ void k_cast(const TS* __restrict__ s, TD* __restrict__ d, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = (TD)s[i];
}

__global__ void k_scale_out(const double* __restrict__ z, int64_t N, const int64_t* __restrict__ off, int nprob,
                            const double* __restrict__ par, double* __restrict__ w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) w[i] = par[find_problem(off, nprob, i) * kPar + 0] * z[i];
}

// Warm start of the FP64 stage: x = z = w0 / w~_b (zero for masked orbits), u = 0,
// v = z; w0 in the layout of w, or (one) a single problem's vector for all;
// the mask is indexed by the orbit within the matrix when it is shared.
__global__ void k_warm_start(const double* __restrict__ w0, int one, int shared, int64_t N,
                             const int64_t* __restrict__ off, int nprob, const double* __restrict__ par,
                             const uint8_t* __restrict__ mask, double* __restrict__ x, double* __restrict__ z,
                             double* __restrict__ u, double* __restrict__ v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int b = find_problem(off, nprob, i);
  const bool masked = mask && mask[shared ? i - off[b] : i];
  const double val = masked ? 0.0 : w0[one ? i - off[b] : i] / par[b * kPar + 0];
  x[i] = val;
  z[i] = val;
  u[i] = 0.0;
  v[i] = val;
}

// the dual that makes (x, z = x) stationary: u = -(h - q + mu x) / rho, h = U^T U x; v = z - u
__global__ void k_warm_dual(int64_t N, const int64_t* __restrict__ off, int nprob, const double* __restrict__ par,
                            const uint8_t* __restrict__ mask, int shared, const double* __restrict__ h,
                            const double* __restrict__ q, const double* __restrict__ x, const double* __restrict__ z,
                            double* __restrict__ u, double* __restrict__ v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int b = find_problem(off, nprob, i);
  const bool masked = mask && mask[shared ? i - off[b] : i];
  const double rho = par[b * kPar + 1], mu = par[b * kPar + 3];
  const double uu = masked ? 0.0 : -(h[i] - q[i] + mu * x[i]) / rho;
  u[i] = uu;
  v[i] = masked ? 0.0 : z[i] - uu;
}

// chi^2 over [cb, ce): one block, fixed summation order.
__global__ void k_chi2_final(const double* __restrict__ m, const double* __restrict__ d,
                             const double* __restrict__ sigma, int64_t cb, int64_t ce, double* __restrict__ out) {
  __shared__ double red[1024];
  double s = 0.0;
  for (int64_t n = cb + threadIdx.x; n < ce; n += 1024) {
    const double r = (m[n] - d[n]) / sigma[n];
    s += r * r;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

static unsigned blocks_for(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// ---------------------------------------------------------------------------
// Workspace layout.
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Anderson acceleration (type II, Walker & Ni 2011) of the FP64 stage.  The
// stage is a fixed-point iteration w <- g(w) on w = (x, z, u); with f = g(w) - w
// and the last m differences dF_j of f and dW_j of w, the next iterate is
//   w+ = g(w) - sum_j gamma_j (dW_j + dF_j),  gamma = argmin |f - dF gamma|,
// from the normal equations (regularised by 1e-10 of their trace).  The
// history is cleared when |f| exceeds kAARestart times its smallest value
// since the last clearing.  Vectors are [4][N] (x, z, u, h): gamma is fitted on
// (x, z, u) only and h = U^T U x, which is linear in x, is mixed with the same
// gamma so that it stays U^T U of the mixed x; problem b owns
// indices off[b]..off[b+1]-1 of each; per-problem state (iteration, history
// length, smallest |f|) lives on the device so the steps can be captured.
// ---------------------------------------------------------------------------
struct AAArgs {
  double *x, *z, *u, *v;  // the iterate of the FP64 stage
  double *h, *r;          // h = U^T U x carried with the iterate, and the residual r (null: not carried)
  const double* q;        // U^T y
  const uint8_t* mask;
  int shared;             // mask indexed by orbit within the problem
  double *w, *wp, *fp;    // [kAAComp][N] current iterate, previous iterate, previous residual
  double *df, *y;         // [kAAMem][kAAComp][N] history: dF_j and dW_j + dF_j
  double *G, *gam, *st;   // per problem: [kAAMem][kAAMem] dF_i . dF_j, [kAAMem] gamma, {it, count, min |f|}
  double* part;           // [P][nbx][kAADots] block partials of the dot products
  const int64_t* off;
  const double* par;
  int64_t N;
  int nbx, P;
};

// w = the iterate entering the FP64 stage, empty history (zeroed: the workspace
// may hold anything, and 0 * NaN would poison the mixing)
__global__ __launch_bounds__(256) void k_aa_init(AAArgs a) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < a.N) {
    a.w[i] = a.x[i];
    a.w[a.N + i] = a.z[i];
    a.w[2 * a.N + i] = a.u[i];
    a.w[3 * a.N + i] = a.h ? a.h[i] : 0.0;
    for (int64_t k = 0; k < kAAComp * (int64_t)kAAMem; ++k) {  // unused history slots must hold finite values
      a.df[k * a.N + i] = 0.0;
      a.y[k * a.N + i] = 0.0;
    }
  }
  if (i < a.P) {
    a.st[i * 4 + 0] = 0.0;
    a.st[i * 4 + 1] = 0.0;
    a.st[i * 4 + 2] = INFINITY;
  }
}

// f = g(w) - w, the newest history entries, and the block partials of
// dF_s . dF_j, dF_j . f (j < m) and f . f
__global__ __launch_bounds__(kAAThreads) void k_aa_dots(AAArgs a) {
  const int b = blockIdx.y;
  if (a.par[b * kPar + 5] == 0.0) return;  // converged problem: frozen
  const int64_t n0 = a.off[b], nb = a.off[b + 1] - n0;
  if ((int64_t)blockIdx.x * kAAChunk >= nb) return;
  const int64_t it = (int64_t)a.st[b * 4 + 0];
  const bool hist = it >= 1;
  const int s = hist ? (int)((it - 1) % kAAMem) : 0;
  const int64_t V = kAAComp * a.N;
  const int nc = a.h ? 4 : 3;
  double dots[kAADots];
#pragma unroll
  for (int k = 0; k < kAADots; ++k) dots[k] = 0.0;
  for (int q = 0; q < kAAPer; ++q) {
    const int64_t j = (int64_t)blockIdx.x * kAAChunk + q * kAAThreads + threadIdx.x;
    if (j >= nb) break;
    const int64_t i = n0 + j;
    for (int c = 0; c < nc; ++c) {
      const double g = c == 0 ? a.x[i] : (c == 1 ? a.z[i] : (c == 2 ? a.u[i] : a.h[i]));
      const int64_t e = c * a.N + i;
      const double wv = a.w[e], f = g - wv;
      if (hist) {
        const double d = f - a.fp[e];
        a.df[s * V + e] = d;
        a.y[s * V + e] = (wv - a.wp[e]) + d;
        if (c < 3) {
#pragma unroll
          for (int k = 0; k < kAAMem; ++k) {
            const double dk = k == s ? d : a.df[k * V + e];
            dots[k] += d * dk;
            dots[kAAMem + k] += dk * f;
          }
        }
      }
      a.fp[e] = f;
      a.wp[e] = wv;
      if (c < 3) dots[2 * kAAMem] += f * f;
    }
  }
  __shared__ double red[kAAThreads / 64][kAADots];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kAADots; ++k) {
    const double t = wave_sum(dots[k]);
    if (lane == 0) red[wv][k] = t;
  }
  __syncthreads();
  if (threadIdx.x < kAADots) {
    double t = 0.0;
    for (int v = 0; v < kAAThreads / 64; ++v) t += red[v][threadIdx.x];
    a.part[((int64_t)b * a.nbx + blockIdx.x) * kAADots + threadIdx.x] = t;
  }
}

// per problem (one wave; the small solve by its first lane): the history Gram
// row of the newest entry, the restart rule, and gamma from the regularised
// normal equations (plain != 0: gamma = 0, the plain step g(w), used before a
// convergence check)
__global__ __launch_bounds__(64) void k_aa_solve(AAArgs a, int plain) {
  const int b = blockIdx.x;
  if (a.par[b * kPar + 5] == 0.0) return;
  const int64_t nb = a.off[b + 1] - a.off[b];
  const int nbx = (int)((nb + kAAChunk - 1) / kAAChunk);
  // the block partials: lane l sums blocks l, l + 64, ..., then a fixed-order
  // wave sum (all loads issued before the first sum waits on them)
  double t[kAADots];
#pragma unroll
  for (int k = 0; k < kAADots; ++k) t[k] = 0.0;
  for (int bx = threadIdx.x; bx < nbx; bx += 64) {
    const double* pb = a.part + ((int64_t)b * a.nbx + bx) * kAADots;
#pragma unroll
    for (int k = 0; k < kAADots; ++k) t[k] += pb[k];
  }
#pragma unroll
  for (int k = 0; k < kAADots; ++k) t[k] = wave_sum(t[k]);
  if (threadIdx.x != 0) return;
  // (every array below is indexed by compile-time constants only, the history
  // slots reached through computed addresses, so that nothing lives in scratch)
  double* G = a.G + (int64_t)b * kAAMem * kAAMem;
  double* gam = a.gam + (int64_t)b * kAAMem;
  const int64_t it = (int64_t)a.st[b * 4 + 0];
  int cnt = (int)a.st[b * 4 + 1];
  double fmin = a.st[b * 4 + 2];
  const int m = kAAMem;
  const int s = it >= 1 ? (int)((it - 1) % m) : 0;
  if (it >= 1) {
#pragma unroll
    for (int k = 0; k < kAAMem; ++k) {
      G[s * kAAMem + k] = t[k];
      G[k * kAAMem + s] = t[k];
    }
    cnt = cnt + 1 < m ? cnt + 1 : m;
  }
  const double fn = sqrt(t[2 * kAAMem]);
  if (cnt > 0 && fn > kAARestart * fmin) {
    cnt = 0;
    fmin = fn;
  } else {
    fmin = fn < fmin ? fn : fmin;
  }
#pragma unroll
  for (int k = 0; k < kAAMem; ++k) gam[k] = 0.0;
  if (!plain && cnt > 0) {
    // slots newest first (slot of entry i: (s - i) mod m); M = G restricted to
    // them, Cholesky in place; entries i >= cnt are left out
    double M[kAAMem][kAAMem], r[kAAMem];
    int sl[kAAMem];
    double tr = 0.0;
#pragma unroll
    for (int i = 0; i < kAAMem; ++i) {
      sl[i] = (s - i + m) % m;
      if (i < cnt) tr += G[sl[i] * kAAMem + sl[i]];
    }
#pragma unroll
    for (int i = 0; i < kAAMem; ++i) {
#pragma unroll
      for (int j = 0; j < kAAMem; ++j) M[i][j] = (i < cnt && j < cnt) ? G[sl[i] * kAAMem + sl[j]] : 0.0;
      M[i][i] += 1e-10 * tr + 1e-300;
      double v = 0.0;
#pragma unroll
      for (int k = 0; k < kAAMem; ++k) v = k == sl[i] ? t[kAAMem + k] : v;
      r[i] = v;
    }
    bool ok = true;
#pragma unroll
    for (int j = 0; j < kAAMem; ++j) {
      if (j < cnt && ok) {
        double dj = M[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) dj -= M[j][k] * M[j][k];
        if (!(dj > 0.0)) {
          ok = false;
        } else {
          dj = sqrt(dj);
          M[j][j] = dj;
#pragma unroll
          for (int i = j + 1; i < kAAMem; ++i) {
            if (i < cnt) {
              double v = M[i][j];
#pragma unroll
              for (int k = 0; k < j; ++k) v -= M[i][k] * M[j][k];
              M[i][j] = v / dj;
            }
          }
        }
      }
    }
    if (ok) {
#pragma unroll
      for (int i = 0; i < kAAMem; ++i) {  // L y = r, then L^T gamma = y
        if (i < cnt) {
          double v = r[i];
#pragma unroll
          for (int k = 0; k < i; ++k) v -= M[i][k] * r[k];
          r[i] = v / M[i][i];
        }
      }
#pragma unroll
      for (int i = kAAMem - 1; i >= 0; --i) {
        if (i < cnt) {
          double v = r[i];
#pragma unroll
          for (int k = i + 1; k < kAAMem; ++k)
            if (k < cnt) v -= M[k][i] * r[k];
          r[i] = v / M[i][i];
        }
      }
#pragma unroll
      for (int i = 0; i < kAAMem; ++i)
        if (i < cnt) gam[sl[i]] = r[i];
    } else {
      cnt = 0;
    }
  }
  a.st[b * 4 + 0] = (double)(it + 1);
  a.st[b * 4 + 1] = (double)cnt;
  a.st[b * 4 + 2] = fmin;
}

// w+ = g(w) - sum_j gamma_j y_j, written to the iterate and to w; v = z - u
__global__ __launch_bounds__(kAAThreads) void k_aa_mix(AAArgs a) {
  const int b = blockIdx.y;
  if (a.par[b * kPar + 5] == 0.0) return;
  const int64_t n0 = a.off[b], nb = a.off[b + 1] - n0;
  const int64_t V = kAAComp * a.N;
  const double rho = a.par[b * kPar + 1], rhop = a.par[b * kPar + 2];
  double gm[kAAMem];
  bool any = false;
#pragma unroll
  for (int k = 0; k < kAAMem; ++k) {
    gm[k] = a.gam[b * kAAMem + k];
    any |= gm[k] != 0.0;
  }
  for (int q = 0; q < kAAPer; ++q) {
    const int64_t j = (int64_t)blockIdx.x * kAAChunk + q * kAAThreads + threadIdx.x;
    if (j >= nb) break;
    const int64_t i = n0 + j;
    double x = a.x[i], z = a.z[i], u = a.u[i], h = a.h ? a.h[i] : 0.0;
    if (any) {
#pragma unroll
      for (int k = 0; k < kAAMem; ++k) {
        if (gm[k] == 0.0) continue;  // slots outside the history
        x -= gm[k] * a.y[k * V + i];
        z -= gm[k] * a.y[k * V + a.N + i];
        u -= gm[k] * a.y[k * V + 2 * a.N + i];
        if (a.h) h -= gm[k] * a.y[k * V + 3 * a.N + i];
      }
      a.x[i] = x;
      a.z[i] = z;
      a.u[i] = u;
      a.v[i] = z - u;
      if (a.h) {
        const bool masked = a.mask && a.mask[a.shared ? j : i];
        a.h[i] = h;
        a.r[i] = masked ? 0.0 : a.q[i] + rho * (z - u) - h - rhop * x;
      }
    }
    a.w[i] = x;
    a.w[a.N + i] = z;
    a.w[2 * a.N + i] = u;
    a.w[3 * a.N + i] = h;
  }
}

struct SolveLayout {
  int P;
  int64_t N, C, Cp, Npt;
  std::vector<int64_t> off, xoff, xlen, rps;
  // the matrices behind the problems: PA = P distinct orbit sets (rows aoff[a]..aoff[a+1]-1
  // of A), or PA = 1 shared by every problem (right-hand sides of one U); NA rows of A
  bool shared;
  int PA;
  int64_t NA;
  std::vector<int64_t> aoff;
  size_t off_hi, off_lo, off_xf, off_K, off_dinv, off_part;
  size_t off_qf, off_zf, off_uf, off_vf;
  size_t off_qd, off_xd, off_zd, off_ud, off_vd, off_rd, off_hd;
  size_t off_kyf, off_r, off_tmp, off_s, off_sc, off_td, off_ys;
  size_t off_par, off_acc, off_idx, off_bad, off_ftmp;
  size_t off_tpart;  // shared matrix: partial sums of the split multi-vector inverse products
  // Anderson acceleration of the FP64 stage (aa = history length, 0 = off)
  int aa, aa_nbx;
  size_t off_aw, off_awp, off_afp, off_adf, off_ay, off_ag, off_agam, off_ast, off_apart;
  // compressed copies (sized for at most cap_nnz entries): ncb column blocks
  // of the rows, nrb row blocks per problem of the columns
  int64_t cap_nnz;
  int ncb, nrb;
  int rg;       // right-hand sides per workgroup in the compressed passes (1: one problem each)
  int64_t blk;  // compressed block: columns per row segment, orbits per column segment (kBlk, or rhs_blk(rg))
  int nrb_a;    // rg > 1: row blocks that hold orbits (partials per column)
  size_t off_pd;  // rg > 1: partial row dots [P][ncb][NA]
  size_t off_rcnt, off_cpart, off_slab, off_rptr, off_rcol, off_rval, off_cptr, off_crow, off_cval;
  int64_t nzw;    // 64-bit words of zero-panel bits per 256-row tile of X
  size_t off_nz;   // zero-panel bits of the Gram operand [Cx / 256][nzw]
  size_t off_nzl;  // the same for its lo plane (counts)
  size_t off_tiles, off_perm;  // per orbit: footprint (count + bitmap of nonzero 256-constraint tiles); X's orbit order
  size_t off_scan, off_clen, off_cpos;  // device prefix sums of the compressed copies' segment lengths
  size_t total;
};

// off: [P + 1] offsets of the problems' orbit vectors; shared: every problem
// has the orbits of rows 0..off[1]-1 of A (equal lengths)
static SolveLayout layout(int P, const int64_t* off, int64_t C, int gram_mode, int aa, bool shared = false) {
  SolveLayout L;
  L.P = P;
  L.C = C;
  L.Cp = (C + kNB - 1) / kNB * kNB;
  L.off.assign(off, off + P + 1);
  L.N = off[P];
  L.shared = shared;
  L.PA = shared ? 1 : P;
  L.aoff.assign(off, off + L.PA + 1);
  L.NA = L.aoff[L.PA];
  L.Npt = 0;
  for (int b = 0; b < P; ++b) {
    const int64_t nb = off[b + 1] - off[b];
    L.rps.push_back(nb > 0 ? (nb + kSlabs - 1) / kSlabs : 1);
    if (b >= L.PA) continue;
    L.xoff.push_back(L.Npt);
    L.xlen.push_back((nb + 63) / 64 * 64);
    L.Npt += L.xlen.back();
  }
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o += a256(bytes); return at; };
  const size_t xe = (size_t)gram_rows(gram_mode, L.Cp) * L.Npt;
  const size_t N = (size_t)L.N, VP = (size_t)P * L.Cp, PA = (size_t)L.PA;
  L.off_hi = take(gram_mode == SW_GRAM_F32 ? 0 : xe * 2);
  L.off_lo = take(gram_mode == SW_GRAM_BF16X3 ? xe * 2 : 0);
  L.off_xf = take(gram_mode == SW_GRAM_F32 ? xe * 4 : 0);
  L.nzw = (L.Npt + 2047) / 2048;
  L.off_nz = take(gram_mode == SW_GRAM_F32 ? 0 : (size_t)(gram_rows(gram_mode, L.Cp) / 256) * L.nzw * 8);
  L.off_nzl = take(gram_mode == SW_GRAM_BF16X3 ? (size_t)(gram_rows(gram_mode, L.Cp) / 256) * L.nzw * 8 : 0);
  L.off_K = take(PA * L.Cp * L.Cp * 4);
  L.off_dinv = take(PA * L.Cp * kNB * 4);
  L.off_part = take((size_t)P * kSlabs * L.C * 8);
  L.off_qf = take(N * 4); L.off_zf = take(N * 4); L.off_uf = take(N * 4); L.off_vf = take(N * 4);
  L.off_qd = take(N * 8); L.off_xd = take(N * 8); L.off_zd = take(N * 8); L.off_ud = take(N * 8);
  L.off_vd = take(N * 8); L.off_rd = take(N * 8); L.off_hd = take(N * 8);
  L.off_kyf = take(VP * 4); L.off_r = take(VP * 4); L.off_tmp = take(VP * 4); L.off_s = take(VP * 4);
  L.off_sc = take(VP * 8); L.off_td = take(VP * 8); L.off_ys = take(VP * 8);
  L.off_par = take((size_t)P * kPar * 8);
  L.off_acc = take((size_t)P * kAcc * 8);
  L.off_idx = take((size_t)(P + 1) * 8 * 5);
  L.off_bad = take(64);
  L.off_ftmp = take(PA * inverse_factor_scratch(L.Cp, L.PA) * 4);
  {
    const int parts = shared && P >= kTrmmMinRhs ? trmm_parts(L.Cp, P) : 1;
    L.off_tpart = take(parts > 1 ? (size_t)parts * VP * 4 : 0);
  }
  {
    int64_t nmax = 1;
    for (int b = 0; b < P; ++b) nmax = std::max<int64_t>(nmax, off[b + 1] - off[b]);
    L.aa = aa;
    L.aa_nbx = (int)((nmax + kAAChunk - 1) / kAAChunk);
    const size_t v3 = aa ? (size_t)kAAComp * N * 8 : 0;
    L.off_aw = take(v3); L.off_awp = take(v3); L.off_afp = take(v3);
    L.off_adf = take(v3 * aa); L.off_ay = take(v3 * aa);
    L.off_ag = take((size_t)P * kAAMem * kAAMem * 8);
    L.off_agam = take((size_t)P * kAAMem * 8);
    L.off_ast = take((size_t)P * 4 * 8);
    L.off_apart = take(aa ? (size_t)P * L.aa_nbx * kAADots * 8 : 0);
  }
  // compressed copies: room for kMaxDensity (or 1M entries), 8-byte values
  const double dense = (double)L.NA * (double)L.C;
  L.cap_nnz = std::max<int64_t>((int64_t)(kMaxDensity * dense), (int64_t)1 << 20);
  if ((double)L.cap_nnz > dense) L.cap_nnz = (int64_t)dense;
  // right-hand sides of one matrix go through the compressed passes rg at a time
  // (rg = 2, 4 or 8, as long as an orbit slab still fits a block of rhs_blk(rg))
  L.rg = 1;
  if (shared)
    while (L.rg < (g_rhs_group > 0 ? g_rhs_group : kRhsGroup) && L.rg < P && L.rps[0] <= rhs_blk(2 * L.rg)) L.rg *= 2;
  L.blk = L.rg > 1 ? rhs_blk(L.rg) : kBlk;
  L.ncb = (int)((L.C + L.blk - 1) / L.blk);
  {
    const int64_t brows = slabs_per_block(L.rps[0], L.blk) * L.rps[0];
    L.nrb_a = (int)((L.NA + brows - 1) / brows);
  }
  L.nrb = 1;
  for (int b = 0; b < L.PA; ++b) {
    const int64_t spb = slabs_per_block(L.rps[b], L.blk);
    L.nrb = std::max<int>(L.nrb, (int)((kSlabs + spb - 1) / spb));
  }
  const size_t NA = (size_t)L.NA;
  L.off_rcnt = take(NA * L.ncb * 8);
  L.off_cpart = take(PA * kSlabs * L.C * 4);
  L.off_slab = take(PA * kSlabs * L.C * 8);
  L.off_rptr = take((NA * L.ncb + 1) * 8);
  L.off_rcol = take((size_t)L.cap_nnz * 2);
  L.off_rval = take((size_t)L.cap_nnz * 8);
  L.off_cptr = take(PA * L.nrb * (L.C + 1) * 8);
  L.off_crow = take((size_t)L.cap_nnz * 2);
  L.off_cval = take((size_t)L.cap_nnz * 8);
  L.off_pd = take(shared ? (size_t)P * std::max<int64_t>(L.ncb, kDenseChunks) * NA * 8 : 0);
  L.off_tiles = take(NA * 5 * 8);
  L.off_perm = take(NA * 4);
  {  // device prefix sums of the segment lengths: block sums, totals, column segments
    const size_t nr = NA * L.ncb, nq = PA * L.nrb * L.C;
    const size_t nbr = (nr + kScanBlock - 1) / kScanBlock, nbc = (nq + kScanBlock - 1) / kScanBlock;
    L.off_scan = take((2 * nbr + 2 * nbc + 5) * 8);  // block sums, 4 totals, the quantum check flag
    L.off_clen = take(nq * 8);
    L.off_cpos = take(nq * 8);
  }
  L.total = o;
  return L;
}

struct Ctx {
  SolveLayout L;
  bool sparse = false;
  const int32_t* perm = nullptr;  // orbit order of the Gram operand's columns (null: the rows' order)
  bool dense_rhs = false;          // shared matrix: FP64 passes as dense MFMA products over all right-hand sides
  int dcs = 1, drd = 1;            // dense passes: K chunks of the column sums (orbits) and of the row dots
  int64_t nnz = 0;
  char* ws;
  hipStream_t st;
  const void* A;
  int dtype;
  const double* sigma;
  double quantum = 0.0;  // > 0: A holds roundings of integer multiples of it (compressed as counts)
  bool quant = false;    // the compressed copies hold the counts (uint16), the passes scale by quantum
  int64_t sS;  // sigma of problem b at sigma + b * sS
  const int64_t *off_d, *xoff_d, *xlen_d, *rps_d, *aoff_d;
  double* par;
  template <typename T> T* p(size_t o) const { return reinterpret_cast<T*>(ws + o); }
};

// compressed column sums of a shared matrix, R right-hand sides per workgroup:
// one workgroup per (column chunk, row block, group of R); chunks of 64 to
// kRhsItems columns, enough of them for about 1,024 workgroups
template <typename TA, typename TV, int R>
static void launch_colsum_rhs(const Ctx& X, const TV* v) {
  const int G = (X.L.P + R - 1) / R;
  const int64_t want = std::max<int64_t>(1, (1024 + (int64_t)X.L.nrb_a * G - 1) / ((int64_t)X.L.nrb_a * G));
  int64_t cpc = std::min<int64_t>(kRhsItems, std::max<int64_t>(64, (X.L.C + want - 1) / want));
  if (g_sparse_cols > 0) cpc = std::min<int64_t>(kRhsItems, g_sparse_cols);
  const dim3 grid((unsigned)((X.L.C + cpc - 1) / cpc), (unsigned)X.L.nrb_a, (unsigned)G);
  hipLaunchKernelGGL((k_csc_colsum_rhs<TA, TV, R>), grid, dim3(kSpThreads), 0, X.st, X.L.C, cpc, X.L.P, X.off_d,
                     X.rps_d, X.p<int64_t>(X.L.off_cptr), X.p<uint16_t>(X.L.off_crow), X.p<TA>(X.L.off_cval), v,
                     X.par, X.p<double>(X.L.off_part));
}

template <typename TA, typename TV>
static void colsum_rhs(const Ctx& X, const TV* v) {
  if (X.L.rg == 2) launch_colsum_rhs<TA, TV, 2>(X, v);
  else if (X.L.rg == 4) launch_colsum_rhs<TA, TV, 4>(X, v);
  else launch_colsum_rhs<TA, TV, 8>(X, v);
}

template <typename TV>
static hipError_t colsum(const Ctx& X, const TV* v) {
  if (X.dense_rhs) {
    // chunk z of the orbits writes slab z of the partials (X.dcs chunks)
    const int64_t n_a = X.L.NA, kc = (n_a + X.dcs - 1) / X.dcs;
    const dim3 grid((unsigned)((X.L.C + kDN - 1) / kDN), (unsigned)((X.L.P + kDM - 1) / kDM), (unsigned)X.dcs);
    if (X.dtype == SW_F32)
      hipLaunchKernelGGL((k_dgemm_rhs<TV, float, false>), grid, dim3(256), 0, X.st, (int64_t)X.L.P, X.L.C, n_a, v,
                         n_a, (const float*)X.A, X.L.C, kc, X.p<double>(X.L.off_part), (int64_t)kSlabs * X.L.C, X.L.C);
    else
      hipLaunchKernelGGL((k_dgemm_rhs<TV, double, false>), grid, dim3(256), 0, X.st, (int64_t)X.L.P, X.L.C, n_a, v,
                         n_a, (const double*)X.A, X.L.C, kc, X.p<double>(X.L.off_part), (int64_t)kSlabs * X.L.C,
                         X.L.C);
    return hipGetLastError();
  }
  if (X.sparse && X.L.rg > 1) {
    if (X.quant) colsum_rhs<uint16_t, TV>(X, v);
    else if (X.dtype == SW_F32) colsum_rhs<float, TV>(X, v);
    else colsum_rhs<double, TV>(X, v);
    return hipGetLastError();
  }
  if (X.sparse) {
    // 64 columns per workgroup (several rounds of 128 KB workgroups over the
    // 256 CUs balance the uneven column lengths); narrower groups only when
    // that would leave CUs idle
    int64_t cpw = 64;
    if (X.L.C * X.L.P < 64 * 256) cpw = std::max<int64_t>(kSpWaves, (X.L.C * X.L.P + 255) / 256 / kSpWaves * kSpWaves);
    if (g_sparse_cols > 0) cpw = g_sparse_cols;
    dim3 grid((unsigned)((X.L.C + cpw - 1) / cpw), (unsigned)X.L.P);
    if (X.quant)
      hipLaunchKernelGGL((k_csc_colsum<uint16_t, TV>), grid, dim3(kSpThreads), 0, X.st, X.L.C, (int)cpw, X.off_d,
                         X.rps_d, X.L.nrb, X.p<int64_t>(X.L.off_cptr), X.p<uint16_t>(X.L.off_crow),
                         X.p<uint16_t>(X.L.off_cval), v, X.par, X.L.shared ? 1 : 0, X.p<double>(X.L.off_part));
    else if (X.dtype == SW_F32)
      hipLaunchKernelGGL((k_csc_colsum<float, TV>), grid, dim3(kSpThreads), 0, X.st, X.L.C, (int)cpw, X.off_d, X.rps_d,
                         X.L.nrb, X.p<int64_t>(X.L.off_cptr), X.p<uint16_t>(X.L.off_crow), X.p<float>(X.L.off_cval), v,
                         X.par, X.L.shared ? 1 : 0, X.p<double>(X.L.off_part));
    else
      hipLaunchKernelGGL((k_csc_colsum<double, TV>), grid, dim3(kSpThreads), 0, X.st, X.L.C, (int)cpw, X.off_d,
                         X.rps_d, X.L.nrb, X.p<int64_t>(X.L.off_cptr), X.p<uint16_t>(X.L.off_crow),
                         X.p<double>(X.L.off_cval), v, X.par, X.L.shared ? 1 : 0, X.p<double>(X.L.off_part));
    return hipGetLastError();
  }
  dim3 grid((unsigned)((X.L.C + kColTile - 1) / kColTile), (unsigned)kSlabs, (unsigned)X.L.P);
  if (X.dtype == SW_F32)
    hipLaunchKernelGGL((k_colsum<float, TV>), grid, dim3(kColThreads), 0, X.st, (const float*)X.A, X.L.C, v, X.off_d,
                       X.rps_d, X.par, X.L.shared ? 1 : 0, X.p<double>(X.L.off_part));
  else
    hipLaunchKernelGGL((k_colsum<double, TV>), grid, dim3(kColThreads), 0, X.st, (const double*)X.A, X.L.C, v,
                       X.off_d, X.rps_d, X.par, X.L.shared ? 1 : 0, X.p<double>(X.L.off_part));
  return hipGetLastError();
}

static hipError_t colreduce(const Ctx& X, int op, const float* kyf, float* outf, double* outd, double* acc) {
  hipLaunchKernelGGL(k_colreduce, dim3(blocks_for(X.L.Cp), (unsigned)X.L.P), dim3(256), 0, X.st,
                     X.p<double>(X.L.off_part), X.dense_rhs ? X.dcs : (X.sparse ? (X.L.rg > 1 ? X.L.nrb_a : 1) : kSlabs), X.L.C, X.L.Cp, X.sigma, X.sS, X.par, op, kyf, X.p<double>(X.L.off_ys), outf,
                     outd, acc, X.quant && X.sparse && !X.dense_rhs ? X.quantum : 1.0);
  return hipGetLastError();
}

// compressed row dots of a shared matrix, RG right-hand sides per workgroup:
// one workgroup per (row group, column block, group of RG), rows per group
// chosen for about 1,024 workgroups (64 to kRhsItems), then the ordered finish
template <typename TA, int RG>
static void launch_rowdot_rhs(const Ctx& X, const RowArgs& R) {
  const int64_t n_a = X.L.NA;
  const int G = (X.L.P + RG - 1) / RG;
  int64_t per = n_a * X.L.ncb * G / 1024;
  per = std::min<int64_t>(kRhsItems, std::max<int64_t>(64, (per + 15) / 16 * 16));
  if (g_sparse_rows > 0) per = std::min<int64_t>(kRhsItems, g_sparse_rows);
  double* pd = X.p<double>(X.L.off_pd);
  const dim3 grid((unsigned)((n_a + per - 1) / per), (unsigned)X.L.ncb, (unsigned)G);
  hipLaunchKernelGGL((k_rowdot_csr_rhs<TA, 16, RG>), grid, dim3(kSpThreads), 0, X.st, X.L.C, X.L.ncb, (int)per, X.L.P,
                     X.p<double>(X.L.off_sc), R, pd);
  hipLaunchKernelGGL(k_rowdot_fin, dim3(blocks_for(n_a), (unsigned)X.L.P), dim3(256), 0, X.st, X.L.ncb,
                     (const double*)pd, R);
}

// the compressed row dots, TS the stored value type
template <typename TS>
static void launch_rowdot_sparse(const Ctx& X, const RowArgs& R) {
  const double* sc = X.p<double>(X.L.off_sc);
  if (X.L.rg > 1) {
    if (X.L.rg == 2) launch_rowdot_rhs<TS, 2>(X, R);
    else if (X.L.rg == 4) launch_rowdot_rhs<TS, 4>(X, R);
    else launch_rowdot_rhs<TS, 8>(X, R);
    return;
  }
  int64_t nmax = 1;
  for (int b = 0; b < X.L.P; ++b) nmax = std::max<int64_t>(nmax, X.L.off[b + 1] - X.L.off[b]);
  // one 128 KB workgroup per CU: rows per workgroup chosen so that a single
  // problem fills the 256 CUs in one round (no tail round), at most 512
  int64_t per = (nmax + 255) / 256;
  per = std::min<int64_t>(kMaxRowsWG, std::max<int64_t>(kSpWaves, (per + kSpWaves - 1) / kSpWaves * kSpWaves));
  if (g_sparse_rows > 0) per = g_sparse_rows;
  // rows with short segments (mean below 512 entries per column block) are
  // taken by 16 lanes each, four rows per wave
  const dim3 grid((unsigned)((nmax + per - 1) / per), (unsigned)X.L.P);
  const bool short_rows = g_sparse_lanes > 0 ? g_sparse_lanes == 16 : X.nnz < 512 * X.L.NA * X.L.ncb;
  if (short_rows)
    hipLaunchKernelGGL((k_rowdot_csr<TS, 16>), grid, dim3(kSpThreads), 0, X.st, X.L.C, X.L.ncb, (int)per, sc, R);
  else
    hipLaunchKernelGGL((k_rowdot_csr<TS, 64>), grid, dim3(kSpThreads), 0, X.st, X.L.C, X.L.ncb, (int)per, sc, R);
}

template <typename TA>
static void launch_rowdot(const Ctx& X, const RowArgs& R) {
  const double* sc = X.p<double>(X.L.off_sc);
  if (X.dense_rhs) {
    const int64_t n_a = X.L.NA, kc = ((X.L.C + X.drd - 1) / X.drd + kDK - 1) / kDK * kDK;
    const int nz = (int)((X.L.C + kc - 1) / kc);
    double* pd = X.p<double>(X.L.off_pd);
    const dim3 grid((unsigned)((n_a + kDN - 1) / kDN), (unsigned)((X.L.P + kDM - 1) / kDM), (unsigned)nz);
    hipLaunchKernelGGL((k_dgemm_rhs<double, TA, true>), grid, dim3(256), 0, X.st, (int64_t)X.L.P, n_a, X.L.C, sc, X.L.Cp,
                       (const TA*)X.A, X.L.C, kc, pd, (int64_t)nz * n_a, n_a);
    hipLaunchKernelGGL(k_rowdot_fin, dim3(blocks_for(n_a), (unsigned)X.L.P), dim3(256), 0, X.st, nz, (const double*)pd,
                       R);
    return;
  }
  if (X.sparse) {
    launch_rowdot_sparse<TA>(X, R);
  } else {
    hipLaunchKernelGGL(k_rowdot<TA>, dim3((unsigned)((X.L.N + 3) / 4)), dim3(kRowsBlock), 0, X.st, (const TA*)X.A,
                       X.L.N, X.L.C, sc, R);
  }
}

static hipError_t rowdot(const Ctx& X, const RowArgs& R0) {
  RowArgs R = R0;
  R.csr_ptr = X.p<int64_t>(X.L.off_rptr);
  R.csr_col = X.p<void>(X.L.off_rcol);
  R.csr_val = X.p<void>(X.L.off_rval);
  const bool counts = X.quant && X.sparse && !X.dense_rhs;
  R.vscale = counts ? X.quantum : 1.0;
  if (counts) launch_rowdot_sparse<uint16_t>(X, R);
  else if (X.dtype == SW_F32) launch_rowdot<float>(X, R);
  else launch_rowdot<double>(X, R);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Segment pointers of the compressed copies on the device.  Segments are
// padded to whole quads, so a pointer is the exclusive prefix sum of the
// quad-rounded lengths.  Three passes: block sums (kScanBlock elements per
// workgroup), one workgroup scanning the block sums, then each block's own
// scan from its offset.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t quad_len(int64_t v) { return (v + 3) & ~(int64_t)3; }

// inclusive scan of one value per thread over the 256 threads (LDS, Hillis-Steele)
__device__ __forceinline__ int64_t block_scan256(int64_t v, int64_t* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const int64_t t = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  return sh[threadIdx.x];
}

template <typename TI>
__global__ __launch_bounds__(256) void k_scan_sums(const TI* __restrict__ in, int64_t n, int64_t* __restrict__ bq,
                                                   int64_t* __restrict__ braw) {
  __shared__ int64_t sh[256];
  const int64_t i0 = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * 4;
  int64_t q = 0, r = 0;
  for (int j = 0; j < 4; ++j)
    if (i0 + j < n) {
      const int64_t v = (int64_t)in[i0 + j];
      q += quad_len(v);
      r += v;
    }
  const int64_t tq = block_scan256(q, sh);
  __syncthreads();
  const int64_t tr = block_scan256(r, sh);
  if (threadIdx.x == 255) {
    bq[blockIdx.x] = tq;
    braw[blockIdx.x] = tr;
  }
}

// exclusive scan of the nb block sums in place; tot[0] = sum of the quad-rounded
// lengths, tot[1] = sum of the lengths
__global__ __launch_bounds__(256) void k_scan_top(int64_t* __restrict__ bq, const int64_t* __restrict__ braw,
                                                  int64_t nb, int64_t* __restrict__ tot) {
  __shared__ int64_t sh[256];
  const int64_t per = (nb + 255) / 256, j0 = threadIdx.x * per, j1 = j0 + per < nb ? j0 + per : nb;
  int64_t q = 0, r = 0;
  for (int64_t j = j0; j < j1; ++j) {
    q += bq[j];
    r += braw[j];
  }
  const int64_t incl = block_scan256(q, sh);
  __syncthreads();
  const int64_t rsum = block_scan256(r, sh);
  int64_t run = incl - q;
  for (int64_t j = j0; j < j1; ++j) {
    const int64_t v = bq[j];
    bq[j] = run;
    run += v;
  }
  if (threadIdx.x == 255) {
    tot[0] = incl;
    tot[1] = rsum;
  }
}

// out[i] = boff[i / kScanBlock] + sum over i' < i of the block of quad(in[i'])
template <typename TI>
__global__ __launch_bounds__(256) void k_scan_apply(const TI* __restrict__ in, int64_t n,
                                                    const int64_t* __restrict__ boff, int64_t* __restrict__ out) {
  __shared__ int64_t sh[256];
  const int64_t i0 = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * 4;
  int64_t l[4], q = 0;
  for (int j = 0; j < 4; ++j) {
    l[j] = i0 + j < n ? quad_len((int64_t)in[i0 + j]) : 0;
    q += l[j];
  }
  int64_t run = boff[blockIdx.x] + block_scan256(q, sh) - q;
  for (int j = 0; j < 4; ++j)
    if (i0 + j < n) {
      out[i0 + j] = run;
      run += l[j];
    }
}

// per segment q = (b nrb + rb) C + c of the compressed columns: the entries of
// column c in the slabs of row block rb of problem b
__global__ __launch_bounds__(256) void k_col_len(const int32_t* __restrict__ cpart, int64_t C, int nrb,
                                                 const int64_t* __restrict__ rps, int64_t blk, int64_t nq,
                                                 int64_t* __restrict__ len) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= nq) return;
  const int64_t c = q % C, br = q / C, rb = br % nrb, b = br / nrb;
  const int64_t spb = slabs_per_block(rps[b], blk);
  const int64_t s0 = rb * spb < kSlabs ? rb * spb : kSlabs, s1 = (rb + 1) * spb < kSlabs ? (rb + 1) * spb : kSlabs;
  int64_t t = 0;
  for (int64_t s = s0; s < s1; ++s) t += cpart[(b * kSlabs + s) * C + c];
  len[q] = t;
}

// column pointers and the first position of every slab's entries in each column
__global__ __launch_bounds__(256) void k_col_ptrs(const int32_t* __restrict__ cpart, int64_t C, int nrb,
                                                  const int64_t* __restrict__ rps, int64_t blk, int64_t nq,
                                                  const int64_t* __restrict__ pos, const int64_t* __restrict__ len,
                                                  int64_t* __restrict__ cptr, int64_t* __restrict__ slab_at) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= nq) return;
  const int64_t c = q % C, br = q / C, rb = br % nrb, b = br / nrb;
  const int64_t spb = slabs_per_block(rps[b], blk);
  const int64_t s0 = rb * spb < kSlabs ? rb * spb : kSlabs, s1 = (rb + 1) * spb < kSlabs ? (rb + 1) * spb : kSlabs;
  int64_t run = pos[q];
  cptr[br * (C + 1) + c] = run;
  if (c == C - 1) cptr[br * (C + 1) + C] = run + quad_len(len[q]);
  for (int64_t s = s0; s < s1; ++s) {
    const int64_t k = (b * kSlabs + s) * C + c;
    slab_at[k] = run;
    run += cpart[k];
  }
}

// exclusive quad-rounded prefix of n counts into out (out[n] = total when
// with_total); tot[0..1] = sums of the rounded and of the raw counts
template <typename TI>
static hipError_t scan_quads(const TI* in, int64_t n, int64_t* out, bool with_total, int64_t* bq, int64_t* braw,
                             int64_t* tot, hipStream_t st) {
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  hipLaunchKernelGGL(k_scan_sums<TI>, dim3((unsigned)nb), dim3(256), 0, st, in, n, bq, braw);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(256), 0, st, bq, (const int64_t*)braw, nb, tot);
  hipLaunchKernelGGL(k_scan_apply<TI>, dim3((unsigned)nb), dim3(256), 0, st, in, n, (const int64_t*)bq, out);
  if (with_total) return hipMemcpyAsync(out + n, tot, 8, hipMemcpyDeviceToDevice, st);
  return hipGetLastError();
}

// Builds the compressed copies of A when they fit; sets X.sparse.
template <typename TA>
static int build_sparse(Ctx& X) {
  const SolveLayout& L = X.L;
  const int P = L.PA, ncb = L.ncb, nrb = L.nrb;  // the distinct matrices
  const int64_t NA = L.NA;
  const TA* A = (const TA*)X.A;
  X.sparse = false;
  for (int b = 0; b < P; ++b)
    if (L.rps[b] > L.blk) return SW_OK;  // a slab longer than an LDS block: keep the dense passes
  int64_t* rcnt = X.p<int64_t>(L.off_rcnt);
  int32_t* cpart = X.p<int32_t>(L.off_cpart);
  uint64_t* foot = X.p<uint64_t>(L.off_tiles);
  hipLaunchKernelGGL(k_row_nnz<TA>, dim3((unsigned)((NA + 3) / 4)), dim3(256), 0, X.st, A, NA, L.C, ncb, L.blk,
                     rcnt, foot);
  hipLaunchKernelGGL(k_col_nnz<TA>, dim3((unsigned)((L.C + kColTile - 1) / kColTile), (unsigned)kSlabs, (unsigned)P),
                     dim3(kColThreads), 0, X.st, A, L.C, X.aoff_d, X.rps_d, cpart);
  SW_HIP(hipGetLastError());
  // segment pointers on the device: rows, then the column segments (b, rb, c)
  // with the first position of every slab's entries in each column
  const int64_t nr = NA * ncb, nq = (int64_t)P * nrb * L.C;
  const int64_t nbr = (nr + kScanBlock - 1) / kScanBlock, nbc = (nq + kScanBlock - 1) / kScanBlock;
  int64_t* sq = X.p<int64_t>(L.off_scan);
  int64_t *bqr = sq, *brr = sq + nbr, *bqc = sq + 2 * nbr, *brc = bqc + nbc, *tot = brc + nbc;
  int64_t* clen = X.p<int64_t>(L.off_clen);
  int64_t* cpos = X.p<int64_t>(L.off_cpos);
  SW_HIP(scan_quads(rcnt, nr, X.p<int64_t>(L.off_rptr), true, bqr, brr, tot, X.st));
  hipLaunchKernelGGL(k_col_len, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, X.st, (const int32_t*)cpart, L.C, nrb,
                     X.rps_d, L.blk, nq, clen);
  SW_HIP(scan_quads(clen, nq, cpos, false, bqc, brc, tot + 2, X.st));
  hipLaunchKernelGGL(k_col_ptrs, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, X.st, (const int32_t*)cpart, L.C,
                     nrb, X.rps_d, L.blk, nq, (const int64_t*)cpos, (const int64_t*)clen, X.p<int64_t>(L.off_cptr),
                     X.p<int64_t>(L.off_slab));
  SW_HIP(hipGetLastError());
  int64_t htot[4] = {0, 0, 0, 0};
  SW_HIP(hipMemcpyAsync(htot, tot, sizeof htot, hipMemcpyDeviceToHost, X.st));
  std::vector<uint64_t> hf(g_gram_dense ? 0 : (size_t)NA * 5);
  if (!hf.empty()) SW_HIP(hipMemcpyAsync(hf.data(), foot, hf.size() * 8, hipMemcpyDeviceToHost, X.st));
  SW_HIP(hipStreamSynchronize(X.st));
  const int64_t at = htot[0], nnz = htot[1], pos = htot[2];
  // a compressed entry costs 6 bytes per pass against 4 (fp32) dense: the
  // compressed passes pay off well below 2/3 density; copies are kept up to
  // kMaxDensity and the capacity of the workspace
  const bool fits = at <= L.cap_nnz && pos <= L.cap_nnz && (double)nnz <= kMaxDensity * (double)NA * (double)L.C;
  int* bad = reinterpret_cast<int*>(tot + 4);
  if (fits) {
    // values: A's own, or with a quantum the integer counts (checked entry by entry)
    X.quant = X.quantum > 0.0;
    const double q = X.quantum, inv_q = X.quant ? 1.0 / X.quantum : 0.0;
    const dim3 gr((unsigned)((NA + 3) / 4)), gc((unsigned)((L.C + kColTile - 1) / kColTile), (unsigned)kSlabs, (unsigned)P);
    const int64_t idx_words = (pos + 1) / 2;
    const int64_t val_words = X.quant ? (pos + 1) / 2 : pos * (int64_t)(sizeof(TA) / 4);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(256), 0, X.st, bad, (int64_t)1, 0);
    if (X.quant)
      hipLaunchKernelGGL((k_fill_csr<TA, uint16_t>), gr, dim3(256), 0, X.st, A, NA, L.C, ncb, L.blk,
                         X.p<int64_t>(L.off_rptr), X.p<uint16_t>(L.off_rcol), X.p<uint16_t>(L.off_rval), inv_q, q, bad);
    else
      hipLaunchKernelGGL((k_fill_csr<TA, TA>), gr, dim3(256), 0, X.st, A, NA, L.C, ncb, L.blk,
                         X.p<int64_t>(L.off_rptr), X.p<uint16_t>(L.off_rcol), X.p<TA>(L.off_rval), inv_q, q, bad);
    // column padding: clear the compressed columns, then fill the entries
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(idx_words)), dim3(256), 0, X.st, X.p<int>(L.off_crow), idx_words,
                       0);
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(val_words)), dim3(256), 0, X.st, X.p<int>(L.off_cval), val_words,
                       0);
    if (X.quant)
      hipLaunchKernelGGL((k_fill_csc<TA, uint16_t>), gc, dim3(kColThreads), 0, X.st, A, L.C, X.aoff_d, X.rps_d,
                         X.p<int64_t>(L.off_slab), L.blk, X.p<uint16_t>(L.off_crow), X.p<uint16_t>(L.off_cval), inv_q,
                         q, bad);
    else
      hipLaunchKernelGGL((k_fill_csc<TA, TA>), gc, dim3(kColThreads), 0, X.st, A, L.C, X.aoff_d, X.rps_d,
                         X.p<int64_t>(L.off_slab), L.blk, X.p<uint16_t>(L.off_crow), X.p<TA>(L.off_cval), inv_q, q,
                         bad);
    SW_HIP(hipGetLastError());
  }
  if (!g_gram_dense) {
    // The Gram is a sum over orbits, so its operand may take the orbits in any
    // order.  Ordered by footprint (the number of nonzero 256-constraint tiles,
    // then the bitmap of those tiles, lexicographically, within each matrix)
    // the orbits of one 32-orbit stage cover the same parts of the grid and the
    // sky, and more stages of a panel are all zero.  perm[aoff_b + j] = row
    // (within matrix b) of column j.  The host sorts while the device fills
    // the compressed copies.
    std::vector<int32_t> perm((size_t)NA);
    for (int b = 0; b < P; ++b) {
      const int64_t a0 = L.aoff[b], a1 = L.aoff[b + 1];
      int32_t* pb = perm.data() + a0;
      for (int64_t i = a0; i < a1; ++i) pb[i - a0] = (int32_t)(i - a0);
      const uint64_t* fb = hf.data() + a0 * 5;
      std::stable_sort(pb, pb + (a1 - a0), [fb](int32_t x, int32_t y) {
        const uint64_t* fx = fb + (int64_t)x * 5;
        const uint64_t* fy = fb + (int64_t)y * 5;
        for (int k = 0; k < 5; ++k)
          if (fx[k] != fy[k]) return fx[k] < fy[k];
        return false;
      });
    }
    SW_HIP(hipMemcpyAsync(X.p<int32_t>(L.off_perm), perm.data(), perm.size() * 4, hipMemcpyHostToDevice, X.st));
    SW_HIP(hipStreamSynchronize(X.st));  // perm's host copy is freed on return
    X.perm = X.p<int32_t>(L.off_perm);
  }
  if (!fits) return SW_OK;
  int hbad = 0;
  if (X.quant) SW_HIP(hipMemcpyAsync(&hbad, bad, sizeof hbad, hipMemcpyDeviceToHost, X.st));
  SW_HIP(hipStreamSynchronize(X.st));
  if (hbad) {
    X.quant = false;
    set_error("solve_weights: opts.quantum = %.17g, but an entry of A is not the rounding of an integer multiple "
              "of it in 1..65535",
              X.quantum);
    return SW_EINVAL;
  }
  X.sparse = true;
  X.nnz = nnz;
  return SW_OK;
}

template <typename TS>
static hipError_t colscale(const Ctx& X, const TS* s) {
  hipLaunchKernelGGL(k_colscale<TS>, dim3(blocks_for(X.L.C), (unsigned)X.L.P), dim3(256), 0, X.st, s, X.L.C, X.L.Cp,
                     X.sigma, X.sS, X.par, X.p<double>(X.L.off_sc));
  return hipGetLastError();
}

static hipError_t zero_acc(const Ctx& X) {
  hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for((int64_t)X.L.P * kAcc)), dim3(256), 0, X.st,
                     X.p<double>(X.L.off_acc), (int64_t)X.L.P * kAcc, 0.0);
  return hipGetLastError();
}

}  // namespace sw

using namespace sw;

#define SW_TRY(expr)                                      \
  do {                                                    \
    hipError_t e__ = (expr);                              \
    if (e__ != hipSuccess) return hip_fail(e__, #expr);   \
  } while (0)

extern "C" size_t solve_batched_workspace_bytes(int32_t n_prob, const int64_t* orbit_offsets, int64_t n_con,
                                                const sw_solve_opts* opt) {
  if (n_prob < 1 || !orbit_offsets || n_con <= 0) return 0;
  const int mode = opt ? opt->gram : SW_GRAM_BF16X3;
  const int aa = opt && (opt->flags & SW_SOLVE_NO_ACCEL) ? 0 : kAAMem;
  return layout(n_prob, orbit_offsets, n_con, mode, aa).total;
}

extern "C" size_t solve_workspace_bytes(int64_t n_orb, int64_t n_con, const sw_solve_opts* opt) {
  if (n_orb <= 0 || n_con <= 0) return 0;
  const int64_t off[2] = {0, n_orb};
  return solve_batched_workspace_bytes(1, off, n_con, opt);
}

extern "C" size_t chi2_workspace_bytes(int64_t n_con) {
  if (n_con <= 0) return 0;
  return a256((size_t)kSlabs * n_con * 8) + a256((size_t)n_con * 8) + 256;
}

// The solver behind every entry point: n_prob problems whose orbit vectors are
// [orbit_offsets[b], orbit_offsets[b+1]); shared = every problem's matrix is rows
// 0..orbit_offsets[1]-1 of A (one Gram and one factorisation, per-problem data).
static int solve_core(const void* A, int32_t dtype, int32_t n_prob, const int64_t* orbit_offsets, bool shared,
                      int64_t n_con, const double* d, const double* sigma, const double* w_tilde, double lambda,
                      const sw_solve_opts* opt, double* w, sw_solve_report* rep, void* workspace, size_t ws_bytes,
                      void* stream) {
  SW_CHECK(opt && orbit_offsets && w_tilde, "solve_weights: null argument");
  SW_CHECK(dtype == SW_F32 || dtype == SW_F64, "solve_weights: dtype must be SW_F32 or SW_F64");
  SW_CHECK(n_prob >= 1 && n_con > 0, "solve_weights: need n_prob >= 1 and n_con > 0");
  SW_CHECK(n_prob <= 65535, "solve_weights: at most 65535 problems per call");
  SW_CHECK(orbit_offsets[0] == 0, "solve_weights: orbit_offsets[0] must be 0");
  for (int b = 0; b < n_prob; ++b) {
    SW_CHECK(orbit_offsets[b + 1] > orbit_offsets[b], "solve_weights: every problem needs at least one orbit");
    SW_CHECK(std::isfinite(w_tilde[b]) && w_tilde[b] > 0.0, "solve_weights: w_tilde must be finite and > 0");
  }
  SW_CHECK(std::isfinite(lambda), "solve_weights: lambda must be finite");
  if (opt->w0 && opt->w0_shared)
    for (int b = 0; b < n_prob; ++b)
      SW_CHECK(orbit_offsets[b + 1] - orbit_offsets[b] == orbit_offsets[1],
               "solve_weights: w0_shared needs every problem to have the orbits of the first");
  SW_CHECK(lambda >= 0.0 || (std::isfinite(opt->nu) && opt->nu > 0.0),
           "solve_weights: lambda < 0 needs opt->nu > 0");
  SW_CHECK(opt->quantum >= 0.0 && std::isfinite(opt->quantum), "solve_weights: opts.quantum must be >= 0 and finite");
  SW_CHECK(opt->gram == SW_GRAM_BF16 || opt->gram == SW_GRAM_BF16X3 || opt->gram == SW_GRAM_F32,
           "solve_weights: unknown gram mode %d", opt->gram);
  SW_CHECK(A && d && sigma && w, "solve_weights: null device buffer");
  SW_CHECK(workspace, "solve_weights: null workspace");
  // Anderson-accelerated FP64 stage unless switched off; the FP32 stage then
  // runs only when asked for (max_iter > 0)
  const int aa = (opt->flags & SW_SOLVE_NO_ACCEL) ? 0 : kAAMem;
  const size_t need = layout(n_prob, orbit_offsets, n_con, opt->gram, aa, shared).total;
  if (ws_bytes < need) {
    set_error("solve_weights: workspace of %zu bytes, %zu needed", ws_bytes, need);
    return SW_ENOMEM;
  }
  const int max_iter = opt->max_iter > 0 ? opt->max_iter : (aa ? 0 : 1000);
  const int refine_iter = opt->refine_iter < 0 ? 0 : (opt->refine_iter == 0 ? 2000 : opt->refine_iter);
  const int check_every = opt->check_every > 0 ? opt->check_every : 10;
  const double tol = opt->tol > 0.0 ? opt->tol : 1e-4;
  const double tol_kkt = opt->tol_kkt > 0.0 ? opt->tol_kkt : 1e-7;
  const int P = n_prob;

  Ctx X;
  X.L = layout(P, orbit_offsets, n_con, opt->gram, aa, shared);
  const SolveLayout& L = X.L;
  const int PA = L.PA;
  X.ws = (char*)workspace;
  X.st = (hipStream_t)stream;
  X.A = A;
  X.dtype = dtype;
  X.sigma = sigma;
  X.quantum = opt->quantum;
  X.sS = shared ? 0 : n_con;
  X.par = X.p<double>(L.off_par);
  int64_t* idx = X.p<int64_t>(L.off_idx);
  X.off_d = idx;
  X.xoff_d = idx + (P + 1);
  X.xlen_d = idx + 2 * (P + 1);
  X.rps_d = idx + 3 * (P + 1);
  X.aoff_d = idx + 4 * (P + 1);
  const uint8_t* mask = opt->mask;

  // stage boundaries are timed with HIP events on the solve's stream
  hipEvent_t ev[7];
  for (auto& e : ev) SW_TRY(hipEventCreate(&e));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() { for (int i = 0; i < 7; ++i) (void)hipEventDestroy(e[i]); }
  } ev_guard{ev};

  // ---- index arrays and per-problem scalars ----
  std::vector<int64_t> hidx(5 * (P + 1), 0);
  for (int b = 0; b <= P; ++b) hidx[b] = L.off[b];
  for (int b = 0; b < P; ++b) hidx[3 * (P + 1) + b] = L.rps[b];
  for (int a = 0; a < PA; ++a) {  // the Gram operand: one block of columns per matrix
    hidx[(P + 1) + a] = L.xoff[a];
    hidx[2 * (P + 1) + a] = L.xlen[a];
  }
  hidx[(P + 1) + PA] = L.Npt;
  for (int a = 0; a <= PA; ++a) hidx[4 * (P + 1) + a] = L.aoff[a];
  std::vector<double> hpar((size_t)P * kPar, 0.0);
  for (int b = 0; b < P; ++b) {
    hpar[b * kPar + 0] = w_tilde[b];
    hpar[b * kPar + 4] = 1.6;  // over-relaxation (Boyd et al. 2011, Sec. 3.4.3)
    hpar[b * kPar + 5] = 1.0;  // active
  }
  SW_TRY(hipMemcpyAsync(idx, hidx.data(), hidx.size() * 8, hipMemcpyHostToDevice, X.st));
  SW_TRY(hipMemcpyAsync(X.par, hpar.data(), hpar.size() * 8, hipMemcpyHostToDevice, X.st));
  SW_TRY(hipEventRecord(ev[0], X.st));

  // ---- scaled data and the transposed operand of the Gram ----
  hipLaunchKernelGGL(k_scaled_data, dim3(blocks_for(L.Cp), (unsigned)P), dim3(256), 0, X.st, d, sigma, X.sS, L.C,
                     L.Cp, X.p<double>(L.off_ys));
  if (!(opt->flags & SW_SOLVE_DENSE)) {
    const int rs = dtype == SW_F32 ? build_sparse<float>(X) : build_sparse<double>(X);
    if (rs != SW_OK) return rs;
  }
  if (shared && P >= 2 && g_multi_dense != 2) {
    // right-hand sides of one matrix: the passes as dense FP64 MFMA products read A
    // once for all of them (2 P C N flop at ~30 TFLOP/s); the compressed passes read
    // it once per group of rg (6 B per stored entry at ~3 TB/s)
    const double dense_t = 2.0 * P * (double)L.C * (double)L.NA / 30e12;
    const double comp_t =
        X.sparse ? (double)((P + L.rg - 1) / L.rg) * (X.quant ? 4.0 : 6.0) * (double)X.nnz / 3e12 : 1e300;
    X.dense_rhs = g_multi_dense == 1 || dense_t < comp_t;
    const int64_t pt = (P + kDM - 1) / kDM;
    const int64_t ct = (L.C + kDN - 1) / kDN * pt, rt = (L.NA + kDN - 1) / kDN * pt;
    X.dcs = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)kSlabs, 2048 / ct, L.NA / 256}));
    X.drd = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)kDenseChunks, 2048 / rt, L.C / 128}));
  }
  // a matrix of counts (checked entry by entry with the compressed copies): the
  // Gram operand holds the counts, scaled afterwards
  const bool counts_gram = X.quant && opt->gram != SW_GRAM_F32 && g_gram_counts;
  if (opt->gram == SW_GRAM_F32) {
    dim3 grid((unsigned)(gram_rows(opt->gram, L.Cp) / 64), (unsigned)(L.Npt / 64));
    if (dtype == SW_F32)
      hipLaunchKernelGGL(k_prep_x<float>, grid, dim3(256), 0, X.st, (const float*)A, L.C, L.Npt, X.aoff_d, X.xoff_d,
                         PA, sigma, X.par, mask, opt->gram, X.p<__bf16>(L.off_hi), X.p<__bf16>(L.off_lo),
                         X.p<float>(L.off_xf), X.perm);
    else
      hipLaunchKernelGGL(k_prep_x<double>, grid, dim3(256), 0, X.st, (const double*)A, L.C, L.Npt, X.aoff_d,
                         X.xoff_d, PA, sigma, X.par, mask, opt->gram, X.p<__bf16>(L.off_hi), X.p<__bf16>(L.off_lo),
                         X.p<float>(L.off_xf), X.perm);
    SW_TRY(hipGetLastError());
  } else {
    const dim3 grid((unsigned)(gram_rows(opt->gram, L.Cp) / 256), (unsigned)(L.Npt / 32));
    __bf16 *hp = X.p<__bf16>(L.off_hi), *lp = X.p<__bf16>(L.off_lo);
    const bool x3 = opt->gram == SW_GRAM_BF16X3;
    const double inv_q = counts_gram ? 1.0 / X.quantum : 0.0;
    if (dtype == SW_F32) {
      if (x3)
        hipLaunchKernelGGL((k_prep_xb<float, true>), grid, dim3(256), 0, X.st, (const float*)A, L.C, L.Npt, X.aoff_d,
                           X.xoff_d, PA, sigma, X.par, mask, hp, lp, X.perm, inv_q);
      else
        hipLaunchKernelGGL((k_prep_xb<float, false>), grid, dim3(256), 0, X.st, (const float*)A, L.C, L.Npt, X.aoff_d,
                           X.xoff_d, PA, sigma, X.par, mask, hp, lp, X.perm, inv_q);
    } else {
      if (x3)
        hipLaunchKernelGGL((k_prep_xb<double, true>), grid, dim3(256), 0, X.st, (const double*)A, L.C, L.Npt,
                           X.aoff_d, X.xoff_d, PA, sigma, X.par, mask, hp, lp, X.perm, inv_q);
      else
        hipLaunchKernelGGL((k_prep_xb<double, false>), grid, dim3(256), 0, X.st, (const double*)A, L.C, L.Npt,
                           X.aoff_d, X.xoff_d, PA, sigma, X.par, mask, hp, lp, X.perm, inv_q);
    }
    SW_TRY(hipGetLastError());
  }
  const uint64_t* nzbits = nullptr;
  if (opt->gram != SW_GRAM_F32 && !g_gram_dense) {
    hipLaunchKernelGGL(k_nz_bits, dim3((unsigned)L.nzw, (unsigned)(gram_rows(opt->gram, L.Cp) / 256)), dim3(256), 0,
                       X.st, X.p<__bf16>(L.off_hi), L.Npt, L.nzw, X.p<uint64_t>(L.off_nz));
    SW_TRY(hipGetLastError());
    nzbits = X.p<uint64_t>(L.off_nz);
  }
  const uint64_t* nzlo = nullptr;
  float* cscale = nullptr;
  if (counts_gram) {
    if (opt->gram == SW_GRAM_BF16X3) {
      hipLaunchKernelGGL(k_nz_bits, dim3((unsigned)L.nzw, (unsigned)(gram_rows(opt->gram, L.Cp) / 256)), dim3(256), 0,
                         X.st, X.p<__bf16>(L.off_lo), L.Npt, L.nzw, X.p<uint64_t>(L.off_nzl));
      nzlo = X.p<uint64_t>(L.off_nzl);
    }
    cscale = X.p<float>(L.off_s);  // borrowed: the iterations' vector, free until then
    hipLaunchKernelGGL(k_count_scale, dim3(blocks_for(L.Cp), (unsigned)PA), dim3(256), 0, X.st, sigma, X.sS, L.C, L.Cp,
                       X.par, X.quantum, cscale);
    SW_TRY(hipGetLastError());
  }
  SW_TRY(hipEventRecord(ev[1], X.st));

  // ---- Gram K_b = U_b U_b^T (lower tiles) ----
  float* K = X.p<float>(L.off_K);
  const int64_t sK = L.Cp * L.Cp;
  // (rho' I + K)^-1 applied to r for every problem: one S for all right-hand sides, or one per problem
  auto apply_inverse = [&]() -> hipError_t {
    return shared ? inv_apply_rhs(K, L.Cp, L.Cp, P, X.p<float>(L.off_r), X.p<float>(L.off_tmp),
                                  X.p<float>(L.off_s), L.Cp, X.par + 5, kPar, X.p<float>(L.off_tpart), X.st)
                  : inv_apply(K, L.Cp, L.Cp, sK, P, X.p<float>(L.off_r), X.p<float>(L.off_tmp), X.p<float>(L.off_s),
                              L.Cp, X.par + 5, kPar, X.st);
  };
  SW_TRY(gram(opt->gram, X.ws + L.off_hi, X.ws + L.off_lo, X.p<float>(L.off_xf), L.Cp, L.Npt, X.xoff_d, X.xlen_d,
              L.xoff.data(), L.xlen.data(), PA, K, L.Cp, sK, X.st, nzbits, L.nzw, nzlo, cscale, L.Cp));
  SW_TRY(hipEventRecord(ev[2], X.st));
  double* acc = X.p<double>(L.off_acc);
  SW_TRY(zero_acc(X));
  double* trace_d = X.p<double>(L.off_td);  // borrowed scratch
  hipLaunchKernelGGL(k_trace, dim3((unsigned)PA), dim3(256), 0, X.st, K, L.Cp, sK, L.C, trace_d);
  std::vector<double> trace(PA);
  SW_TRY(hipMemcpyAsync(trace.data(), trace_d, PA * 8, hipMemcpyDeviceToHost, X.st));
  std::vector<uint8_t> hmask;
  if (mask) {
    hmask.resize(L.NA);
    SW_TRY(hipMemcpyAsync(hmask.data(), mask, L.NA, hipMemcpyDeviceToHost, X.st));
  }
  SW_TRY(hipStreamSynchronize(X.st));

  // ---- regularisation and penalty per problem ----
  std::vector<double> mu(P), rho(P);
  for (int b = 0; b < P; ++b) {
    const int ab = shared ? 0 : b;  // the matrix of problem b
    int64_t n_eff = L.aoff[ab + 1] - L.aoff[ab];
    if (mask) {
      n_eff = 0;
      for (int64_t i = L.aoff[ab]; i < L.aoff[ab + 1]; ++i) n_eff += hmask[i] ? 0 : 1;
    }
    if (n_eff == 0) n_eff = 1;
    const double mean_col = trace[ab] / (double)n_eff;
    mu[b] = lambda >= 0.0 ? 2.0 * lambda / (double)n_eff : opt->nu * mean_col;
    const double base = mean_col > 0.0 ? mean_col : 1.0;
    rho[b] = opt->rho > 0.0 ? opt->rho : (opt->rho < 0.0 ? -opt->rho * base : base);
    hpar[b * kPar + 1] = rho[b];
    hpar[b * kPar + 2] = rho[b] + mu[b];
    hpar[b * kPar + 3] = mu[b];
  }
  SW_TRY(hipMemcpyAsync(X.par, hpar.data(), hpar.size() * 8, hipMemcpyHostToDevice, X.st));

  // ---- factorise rho' I + K_b ----
  SW_TRY(hipEventRecord(ev[3], X.st));
  hipLaunchKernelGGL(k_add_diag, dim3(blocks_for(L.Cp), (unsigned)PA), dim3(256), 0, X.st, K, L.Cp, sK, L.Cp, X.par);
  int* bad = X.p<int>(L.off_bad);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, X.st, bad, (int64_t)1, 0);
  SW_TRY(spd_inverse_factor(K, L.Cp, L.Cp, sK, X.p<float>(L.off_dinv), L.Cp * kNB, PA, X.p<float>(L.off_ftmp),
                            inverse_factor_scratch(L.Cp, PA), bad, X.st));
  SW_TRY(hipEventRecord(ev[4], X.st));
  int hbad = 0;
  SW_TRY(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, X.st));
  SW_TRY(hipStreamSynchronize(X.st));
  if (hbad) {
    set_error("solve_weights: Gram matrix not positive definite in working precision");
    return SW_EHIP;
  }

  // ---- q = U^T y, Ky = U q ----
  float *qf = X.p<float>(L.off_qf), *zf = X.p<float>(L.off_zf), *uf = X.p<float>(L.off_uf),
        *vf = X.p<float>(L.off_vf);
  double *qd = X.p<double>(L.off_qd), *xd = X.p<double>(L.off_xd), *zd = X.p<double>(L.off_zd),
         *ud = X.p<double>(L.off_ud), *vd = X.p<double>(L.off_vd), *rd = X.p<double>(L.off_rd);
  float *kyf = X.p<float>(L.off_kyf), *r = X.p<float>(L.off_r), *tmp = X.p<float>(L.off_tmp),
        *s = X.p<float>(L.off_s);
  double* td = X.p<double>(L.off_td);
  RowArgs RA;
  std::memset(&RA, 0, sizeof RA);
  RA.nprob = P;
  RA.shared = shared ? 1 : 0;
  RA.Cp = L.Cp;
  RA.off = X.off_d;
  RA.par = X.par;
  RA.mask = mask;
  RA.qf = qf; RA.zf = zf; RA.uf = uf; RA.vf = vf;
  RA.qd = qd; RA.xd = xd; RA.zd = zd; RA.ud = ud; RA.vd = vd; RA.rd = rd;
  RA.acc = acc;
  SW_TRY(colscale<double>(X, X.p<double>(L.off_ys)));
  RA.op = ROW_Q;
  SW_TRY(rowdot(X, RA));
  SW_TRY(colsum<float>(X, qf));
  SW_TRY(colreduce(X, COL_PLAIN, nullptr, kyf, nullptr, nullptr));
  for (float* p : {zf, uf, vf}) hipLaunchKernelGGL(k_fill_f32, dim3(blocks_for(L.N)), dim3(256), 0, X.st, p, L.N, 0.0f);
  std::vector<double> hacc((size_t)P * kAcc);
  SW_TRY(hipMemcpyAsync(hacc.data(), acc, hacc.size() * 8, hipMemcpyDeviceToHost, X.st));
  SW_TRY(hipStreamSynchronize(X.st));
  std::vector<double> qmax(P);
  for (int b = 0; b < P; ++b) qmax[b] = hacc[b * kAcc + 5] > 0.0 ? hacc[b * kAcc + 5] : 1.0;

  std::vector<sw_solve_report> R(P);
  for (int b = 0; b < P; ++b) {
    std::memset(&R[b], 0, sizeof R[b]);
    R[b].mu = mu[b];
    R[b].rho = rho[b];
  }
  auto set_active = [&](const std::vector<int>& act) -> hipError_t {
    for (int b = 0; b < P; ++b) hpar[b * kPar + 5] = act[b] ? 1.0 : 0.0;
    return hipMemcpyAsync(X.par, hpar.data(), hpar.size() * 8, hipMemcpyHostToDevice, X.st);
  };

  // ---- stage 1: fp32 ADMM ----
  auto admm_iter = [&](double* accp) -> hipError_t {
    hipError_t e;
    if ((e = colsum<float>(X, vf)) != hipSuccess) return e;
    if ((e = colreduce(X, COL_ADMM, kyf, r, nullptr, nullptr)) != hipSuccess) return e;
    if ((e = apply_inverse()) != hipSuccess) return e;
    if ((e = colscale<float>(X, s)) != hipSuccess) return e;
    RowArgs Ri = RA;
    Ri.op = ROW_ADMM;
    Ri.acc = accp;
    return rowdot(X, Ri);
  };
  // The iterations between two convergence checks touch only device memory
  // (per-problem flags included), so they are captured once and replayed.
  const bool use_graph = opt->use_graph && X.st != nullptr && check_every > 1;
  auto capture = [&](auto&& body, int reps, hipGraphExec_t* exec) -> hipError_t {
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(X.st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    for (int k = 0; k < reps; ++k) {
      e = body();
      if (e != hipSuccess) break;
    }
    hipError_t e2 = hipStreamEndCapture(X.st, &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    return e;
  };
  struct ExecGuard {
    hipGraphExec_t e = nullptr;
    ~ExecGuard() { if (e) (void)hipGraphExecDestroy(e); }
  } g1, g2;
  if (use_graph && max_iter > 0) SW_TRY(capture([&]() { return admm_iter(nullptr); }, check_every - 1, &g1.e));
  std::vector<int> active(P, 1);
  std::vector<std::vector<double>> hist(P);
  int n_active = P;
  int it = 0;
  while (it < max_iter && n_active > 0) {
    const int run = std::min(check_every - 1, max_iter - 1 - it);
    if (g1.e && run == check_every - 1) {
      SW_TRY(hipGraphLaunch(g1.e, X.st));
    } else {
      for (int k = 0; k < run; ++k) SW_TRY(admm_iter(nullptr));
    }
    it += run;
    // the checked iteration accumulates this iteration's residual norms
    SW_TRY(zero_acc(X));
    SW_TRY(admm_iter(acc));
    ++it;
    // stopping rule of Boyd et al. (2011) on the checked iteration's residuals
    SW_TRY(hipMemcpyAsync(hacc.data(), acc, hacc.size() * 8, hipMemcpyDeviceToHost, X.st));
    SW_TRY(hipStreamSynchronize(X.st));
    for (int b = 0; b < P; ++b) {
      if (!active[b]) continue;
      const double* a = &hacc[b * kAcc];
      const double rp = std::sqrt(a[0]), rdl = rho[b] * std::sqrt(a[1]);
      const double scale_p = std::fmax(std::sqrt(a[2]), std::sqrt(a[3]));
      R[b].primal_res = rp / (scale_p + 1e-300);
      R[b].dual_res = rdl / (rho[b] * std::sqrt(a[4]) + 1e-300);
      R[b].iters = it;
      // stage 1 also ends once it stalls: single-precision iterates reach a
      // floor set by the fp32 inverse, below which only stage 2 makes progress
      const double r = std::fmax(R[b].primal_res, R[b].dual_res);
      std::vector<double>& h = hist[b];
      h.push_back(r);
      const size_t n_h = h.size();
      const bool stalled = n_h > kStallChecks && r > kStallRatio * h[n_h - 1 - kStallChecks];
      if ((rp <= tol * scale_p + 1e-300 && rdl <= tol * rho[b] * std::sqrt(a[4]) + 1e-300) || stalled) {
        active[b] = 0;
        --n_active;
      }
    }
    SW_TRY(set_active(active));
  }
  for (int b = 0; b < P; ++b)
    if (R[b].iters == 0) R[b].iters = it;
  SW_TRY(hipEventRecord(ev[5], X.st));

  // ---- stage 2: fp64 refinement of the ADMM iterates + KKT ----
  hipLaunchKernelGGL((k_cast<float, double>), dim3(blocks_for(L.N)), dim3(256), 0, X.st, zf, zd, L.N);
  hipLaunchKernelGGL((k_cast<float, double>), dim3(blocks_for(L.N)), dim3(256), 0, X.st, uf, ud, L.N);
  hipLaunchKernelGGL((k_cast<float, double>), dim3(blocks_for(L.N)), dim3(256), 0, X.st, zf, xd, L.N);
  hipLaunchKernelGGL((k_cast<float, double>), dim3(blocks_for(L.N)), dim3(256), 0, X.st, vf, vd, L.N);
  SW_TRY(hipGetLastError());
  AAArgs AA;
  // two passes over A per FP64 iteration with h carried; the solve falls back to
  // four (the residual from A every iteration) when a problem's KKT residual stays
  // above 10x its smallest value at three consecutive checks: h drifts by U^T e /
  // rho' per correction, e the fp32 inverse's residual, which the ten iterations
  // between refreshes can let grow on badly conditioned problems (a shorter rebound
  // is often the Anderson step's and recovers)
  bool two = g_refine_two != 0;
  const double rebound_factor = (double)g_refine_rebound;
  double* hd = X.p<double>(L.off_hd);
  AA.x = xd; AA.z = zd; AA.u = ud; AA.v = vd;
  AA.h = two ? hd : nullptr; AA.r = rd; AA.q = qd; AA.mask = mask; AA.shared = shared ? 1 : 0;
  AA.w = X.p<double>(L.off_aw); AA.wp = X.p<double>(L.off_awp); AA.fp = X.p<double>(L.off_afp);
  AA.df = X.p<double>(L.off_adf); AA.y = X.p<double>(L.off_ay);
  AA.G = X.p<double>(L.off_ag); AA.gam = X.p<double>(L.off_agam); AA.st = X.p<double>(L.off_ast);
  AA.part = X.p<double>(L.off_apart);
  AA.off = X.off_d; AA.par = X.par; AA.N = L.N; AA.nbx = L.aa_nbx; AA.P = P;
  std::vector<double> kkt(P, 0.0), obj(P, 0.0);
  std::vector<int> support(P, 0);
  // the KKT evaluation covers the active problems; a frozen problem keeps its last values
  auto kkt_eval = [&]() -> int {
    SW_TRY(zero_acc(X));
    SW_TRY(colsum<double>(X, zd));
    SW_TRY(colreduce(X, COL_RESID, nullptr, nullptr, td, acc));
    SW_TRY(colscale<double>(X, td));
    RowArgs K2 = RA;
    K2.op = ROW_KKT;
    SW_TRY(rowdot(X, K2));
    SW_TRY(hipMemcpyAsync(hacc.data(), acc, hacc.size() * 8, hipMemcpyDeviceToHost, X.st));
    SW_TRY(hipStreamSynchronize(X.st));
    for (int b = 0; b < P; ++b) {
      if (!active[b]) continue;
      kkt[b] = hacc[b * kAcc + 6] / qmax[b];
      obj[b] = 0.5 * hacc[b * kAcc + 9] + 0.5 * mu[b] * hacc[b * kAcc + 7];
      support[b] = (int)hacc[b * kAcc + 8];
    }
    return SW_OK;
  };
  for (int b = 0; b < P; ++b) active[b] = 1;
  SW_TRY(set_active(active));
  int rc = kkt_eval();
  if (rc != SW_OK) return rc;
  for (int b = 0; b < P; ++b) active[b] = kkt[b] > tol_kkt ? 1 : 0;
  n_active = 0;
  for (int b = 0; b < P; ++b) n_active += active[b];
  SW_TRY(set_active(active));
  // residual of the ridge system at x: r = q + rho v - (U^T U + rho' I) x, and
  // (two passes per iteration) h = U^T U x, exactly: two passes over A
  auto refresh = [&]() -> hipError_t {
    hipError_t e;
    if ((e = colsum<double>(X, xd)) != hipSuccess) return e;
    if ((e = colreduce(X, COL_PLAIN, nullptr, nullptr, td, nullptr)) != hipSuccess) return e;
    if ((e = colscale<double>(X, td)) != hipSuccess) return e;
    RowArgs Rh = RA;
    Rh.op = ROW_H;
    Rh.acc = nullptr;
    Rh.hd = two ? hd : nullptr;
    return rowdot(X, Rh);
  };
  // correction: x = x_old + M r, M = (1/rho')(I - U^T (rho' I + K)^-1 U): two passes over A
  auto correct = [&]() -> hipError_t {
    hipError_t e;
    if ((e = colsum<double>(X, rd)) != hipSuccess) return e;
    if ((e = colreduce(X, COL_PLAIN, nullptr, r, nullptr, nullptr)) != hipSuccess) return e;
    if ((e = apply_inverse()) != hipSuccess) return e;
    if ((e = colscale<float>(X, s)) != hipSuccess) return e;
    RowArgs Rc = RA;
    Rc.op = two ? ROW_CORR2 : ROW_CORR;
    Rc.acc = nullptr;
    Rc.hd = two ? hd : nullptr;
    return rowdot(X, Rc);
  };
  // one iteration: with h carried, the correction alone (the next residual comes
  // from h, which every batch of iterations starts by recomputing exactly);
  // otherwise the residual from A, then the correction
  auto refine_iter_body = [&]() -> hipError_t {
    if (!two) {
      hipError_t e = refresh();
      if (e != hipSuccess) return e;
    }
    return correct();
  };
  // one step: the refinement iteration, then (accelerated) the Anderson
  // mixing; the step before a convergence check is the plain one, so the
  // checked iterate is a projected ADMM iterate
  auto refine_step = [&](bool plain) -> hipError_t {
    hipError_t e = refine_iter_body();
    if (e != hipSuccess || !aa) return e;
    hipLaunchKernelGGL(k_aa_dots, dim3((unsigned)L.aa_nbx, (unsigned)P), dim3(kAAThreads), 0, X.st, AA);
    hipLaunchKernelGGL(k_aa_solve, dim3((unsigned)P), dim3(64), 0, X.st, AA, plain ? 1 : 0);
    hipLaunchKernelGGL(k_aa_mix, dim3((unsigned)L.aa_nbx, (unsigned)P), dim3(kAAThreads), 0, X.st, AA);
    return hipGetLastError();
  };
  auto refine_batch = [&](int run) -> hipError_t {
    if (two) {
      hipError_t e = refresh();
      if (e != hipSuccess) return e;
    }
    for (int k = 0; k < run; ++k) {
      hipError_t e = refine_step(k == run - 1);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  if (opt->w0) {
    // warm start: x = z = w0 / w~, then its dual from h = U^T U x (two passes over A)
    hipLaunchKernelGGL(k_warm_start, dim3(blocks_for(L.N)), dim3(256), 0, X.st, opt->w0, opt->w0_shared ? 1 : 0,
                       shared ? 1 : 0, L.N, X.off_d, P, X.par, mask, xd, zd, ud, vd);
    SW_TRY(hipGetLastError());
    SW_TRY(colsum<double>(X, xd));
    SW_TRY(colreduce(X, COL_PLAIN, nullptr, nullptr, td, nullptr));
    SW_TRY(colscale<double>(X, td));
    RowArgs Rw = RA;
    Rw.op = ROW_H;
    Rw.acc = nullptr;
    Rw.hd = hd;
    SW_TRY(rowdot(X, Rw));
    hipLaunchKernelGGL(k_warm_dual, dim3(blocks_for(L.N)), dim3(256), 0, X.st, L.N, X.off_d, P, X.par, mask,
                       shared ? 1 : 0, (const double*)hd, (const double*)qd, (const double*)xd, (const double*)zd, ud,
                       vd);
    SW_TRY(hipGetLastError());
  }
  if (two) SW_TRY(refresh());  // h of the iterate entering the stage, before the history takes it
  if (aa) {
    hipLaunchKernelGGL(k_aa_init, dim3(blocks_for(std::max<int64_t>(L.N, P))), dim3(256), 0, X.st, AA);
    SW_TRY(hipGetLastError());
  }
  if (use_graph && n_active > 0) SW_TRY(capture([&]() { return refine_batch(check_every); }, 1, &g2.e));
  std::vector<int> rit(P, 0);
  std::vector<double> kmin(P, HUGE_VAL);
  std::vector<int> nreb(P, 0);  // consecutive checks above rebound_factor x kmin
  int k_done = 0;
  while (k_done < refine_iter && n_active > 0) {
    const int run = std::min(check_every, refine_iter - k_done);
    if (g2.e && run == check_every) {
      SW_TRY(hipGraphLaunch(g2.e, X.st));
    } else {
      SW_TRY(refine_batch(run));
    }
    k_done += run;
    for (int b = 0; b < P; ++b)
      if (active[b]) rit[b] = k_done;
    rc = kkt_eval();
    if (rc != SW_OK) return rc;
    bool rebound = false;
    for (int b = 0; b < P; ++b) {
      if (!active[b]) continue;
      nreb[b] = kmin[b] < HUGE_VAL && kkt[b] > rebound_factor * kmin[b] ? nreb[b] + 1 : 0;
      if (nreb[b] >= g_refine_rebound_checks) rebound = true;
      kmin[b] = std::min(kmin[b], kkt[b]);
    }
    for (int b = 0; b < P; ++b)
      if (active[b] && kkt[b] <= tol_kkt) {
        active[b] = 0;
        --n_active;
      }
    SW_TRY(set_active(active));
    if (two && rebound && n_active > 0) {
      // fall back to four passes for the rest of the solve: a new fixed-point map,
      // so the Anderson history restarts from the current iterate
      two = false;
      AA.h = nullptr;
      if (aa) {
        hipLaunchKernelGGL(k_aa_init, dim3(blocks_for(std::max<int64_t>(L.N, P))), dim3(256), 0, X.st, AA);
        SW_TRY(hipGetLastError());
      }
      if (g2.e) {
        SW_TRY(hipGraphExecDestroy(g2.e));
        g2.e = nullptr;
        SW_TRY(capture([&]() { return refine_batch(check_every); }, 1, &g2.e));
      }
    }
  }
  int all_conv = 1;
  for (int b = 0; b < P; ++b) {
    R[b].refine_iters = rit[b];
    R[b].kkt = kkt[b];
    R[b].objective = obj[b];
    R[b].converged = kkt[b] <= tol_kkt ? 1 : 0;
    R[b].n_active = support[b];
    R[b].nnz = X.sparse && !X.dense_rhs ? (double)X.nnz : 0.0;
    R[b].passes = two ? 2 : 4;
    all_conv &= R[b].converged;
  }
  hipLaunchKernelGGL(k_scale_out, dim3(blocks_for(L.N)), dim3(256), 0, X.st, zd, L.N, X.off_d, P, X.par, w);
  SW_TRY(hipGetLastError());
  SW_TRY(hipEventRecord(ev[6], X.st));
  SW_TRY(hipStreamSynchronize(X.st));
  float ms[6];
  for (int k = 0; k < 6; ++k) SW_TRY(hipEventElapsedTime(&ms[k], ev[k], ev[k + 1]));
  for (int b = 0; b < P; ++b) {
    R[b].t_prep_ms = ms[0];
    R[b].t_gram_ms = ms[1];
    R[b].t_factor_ms = ms[3];
    R[b].t_admm_ms = ms[4];
    R[b].t_refine_ms = ms[5];
  }
  if (rep)
    for (int b = 0; b < P; ++b) rep[b] = R[b];
  if (!all_conv) {
    set_error("solve_weights: not every problem converged (kkt of problem 0: %.3e after %d + %d iterations)", kkt[0],
              R[0].iters, R[0].refine_iters);
    return SW_ENOTCONV;
  }
  return SW_OK;
}

extern "C" int solve_weights_batched(const void* A, int32_t dtype, int32_t n_prob, const int64_t* orbit_offsets,
                                     int64_t n_con, const double* d, const double* sigma, const double* w_tilde,
                                     double lambda, const sw_solve_opts* opt, double* w, sw_solve_report* rep,
                                     void* workspace, size_t ws_bytes, void* stream) {
  return solve_core(A, dtype, n_prob, orbit_offsets, false, n_con, d, sigma, w_tilde, lambda, opt, w, rep, workspace,
                    ws_bytes, stream);
}

static std::vector<int64_t> rhs_offsets(int32_t n_rhs, int64_t n_orb) {
  std::vector<int64_t> off((size_t)n_rhs + 1);
  for (int32_t b = 0; b <= n_rhs; ++b) off[b] = (int64_t)b * n_orb;
  return off;
}

extern "C" size_t solve_multi_workspace_bytes(int64_t n_orb, int64_t n_con, int32_t n_rhs, const sw_solve_opts* opt) {
  if (n_orb <= 0 || n_con <= 0 || n_rhs < 1) return 0;
  const int mode = opt ? opt->gram : SW_GRAM_BF16X3;
  const int aa = opt && (opt->flags & SW_SOLVE_NO_ACCEL) ? 0 : kAAMem;
  return layout(n_rhs, rhs_offsets(n_rhs, n_orb).data(), n_con, mode, aa, true).total;
}

extern "C" int solve_weights_multi(const void* A, int32_t dtype, int64_t n_orb, int64_t n_con, int32_t n_rhs,
                                   const double* d, const double* sigma, double w_tilde, double lambda,
                                   const sw_solve_opts* opt, double* w, sw_solve_report* rep, void* workspace,
                                   size_t ws_bytes, void* stream) {
  SW_CHECK(n_orb > 0, "solve_weights_multi: need n_orb > 0");
  SW_CHECK(n_rhs >= 1, "solve_weights_multi: need n_rhs >= 1");
  const std::vector<int64_t> off = rhs_offsets(n_rhs, n_orb);
  const std::vector<double> wt((size_t)n_rhs, w_tilde);
  return solve_core(A, dtype, n_rhs, off.data(), true, n_con, d, sigma, wt.data(), lambda, opt, w, rep, workspace,
                    ws_bytes, stream);
}

extern "C" int solve_weights(const void* A, int32_t dtype, int64_t n_orb, int64_t n_con, const double* d,
                             const double* sigma, double w_tilde, double lambda, const sw_solve_opts* opt, double* w,
                             sw_solve_report* rep, void* workspace, size_t ws_bytes, void* stream) {
  SW_CHECK(n_orb > 0, "solve_weights: need n_orb > 0");
  const int64_t off[2] = {0, n_orb};
  return solve_weights_batched(A, dtype, 1, off, n_con, d, sigma, &w_tilde, lambda, opt, w, rep, workspace, ws_bytes,
                               stream);
}

// ---------------------------------------------------------------------------
// chi2 and model_observables
// ---------------------------------------------------------------------------
template <typename TA>
__global__ __launch_bounds__(kColThreads) void k_colsum1(const TA* __restrict__ A, int64_t N, int64_t C,
                                                         const double* __restrict__ v, int64_t rps,
                                                         double* __restrict__ part, int atomic) {
  const int64_t c0 = (int64_t)blockIdx.x * kColTile;
  const int64_t i_beg = (int64_t)blockIdx.y * rps;
  int64_t i_end = i_beg + rps;
  if (i_end > N) i_end = N;
  double acc[kColsPerThread] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t i = i_beg; i < i_end; ++i) {
    const double vi = v[i];
    if (vi == 0.0) continue;
#pragma unroll
    for (int k = 0; k < kColsPerThread; ++k) {
      const int64_t c = c0 + threadIdx.x + k * kColThreads;
      if (c < C) acc[k] += (double)A[i * C + c] * vi;
    }
  }
#pragma unroll
  for (int k = 0; k < kColsPerThread; ++k) {
    const int64_t c = c0 + threadIdx.x + k * kColThreads;
    if (c >= C) continue;
    if (atomic) {
      if (acc[k] != 0.0) atomicAdd(&part[c], acc[k]);
    } else {
      part[(int64_t)blockIdx.y * C + c] = acc[k];
    }
  }
}

__global__ void k_sum_slabs(const double* __restrict__ part, int64_t C, int slabs, double* __restrict__ m) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= C) return;
  double t = 0.0;
  for (int s = 0; s < slabs; ++s) t += part[(int64_t)s * C + n];
  m[n] = t;
}

// chi^2 of Eq. 5 over [cb, ce) with its scratch at `ws` (slabs x C partial
// column sums, then C model values, then the result): every slab writes every
// column of its partials and the sums overwrite m, so nothing needs clearing.
static int chi2_launch(const void* A, int32_t dtype, int64_t n_orb, int64_t n_con, const double* w, const double* d,
                       const double* sigma, int64_t cb, int64_t ce, int slabs, char* ws, double* out,
                       hipStream_t st) {
  double* part = (double*)ws;
  double* m = (double*)(ws + a256((size_t)slabs * n_con * 8));
  double* res = (double*)(ws + a256((size_t)slabs * n_con * 8) + a256((size_t)n_con * 8));
  const int64_t rps = (n_orb + slabs - 1) / slabs;
  dim3 grid((unsigned)((n_con + kColTile - 1) / kColTile), (unsigned)slabs);
  if (dtype == SW_F32)
    hipLaunchKernelGGL(k_colsum1<float>, grid, dim3(kColThreads), 0, st, (const float*)A, n_orb, n_con, w, rps, part, 0);
  else
    hipLaunchKernelGGL(k_colsum1<double>, grid, dim3(kColThreads), 0, st, (const double*)A, n_orb, n_con, w, rps, part,
                       0);
  hipLaunchKernelGGL(k_sum_slabs, dim3(blocks_for(n_con)), dim3(256), 0, st, part, n_con, slabs, m);
  hipLaunchKernelGGL(k_chi2_final, dim3(1), dim3(1024), 0, st, m, d, sigma, cb, ce, res);
  SW_HIP(hipGetLastError());
  SW_HIP(hipMemcpyAsync(out, res, 8, hipMemcpyDeviceToHost, st));
  SW_HIP(hipStreamSynchronize(st));
  return SW_OK;
}

extern "C" int chi2(const void* A, int32_t dtype, int64_t n_orb, int64_t n_con, const double* w, const double* d,
                    const double* sigma, int64_t col_begin, int64_t col_end, double* out, void* workspace,
                    size_t ws_bytes, void* stream) {
  SW_CHECK(dtype == SW_F32 || dtype == SW_F64, "chi2: dtype must be SW_F32 or SW_F64");
  SW_CHECK(n_orb > 0 && n_con > 0, "chi2: need n_orb > 0 and n_con > 0");
  SW_CHECK(col_begin >= 0 && col_end <= n_con && col_begin <= col_end, "chi2: bad column range");
  SW_CHECK(A && w && d && sigma && out && workspace, "chi2: null argument");
  if (ws_bytes < chi2_workspace_bytes(n_con)) {
    set_error("chi2: workspace too small");
    return SW_ENOMEM;
  }
  return chi2_launch(A, dtype, n_orb, n_con, w, d, sigma, col_begin, col_end, kSlabs, (char*)workspace, out,
                     (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// chi2_noalloc: chi2 with its scratch in a file-scope device array instead of
// a caller workspace.  The array is held by each device for the life of the
// process; host code reaches it only through the address hipGetSymbolAddress
// returns on that device (the array's name is a host-side stand-in).
// ---------------------------------------------------------------------------
constexpr int kNoAllocSlabs = 32;
constexpr int64_t kNoAllocMaxCon = (int64_t)1 << 16;
constexpr size_t kNoAllocBytes =
    ((size_t)kNoAllocSlabs * kNoAllocMaxCon * 8 + 255) / 256 * 256 + (size_t)kNoAllocMaxCon * 8 + 256;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

// the device address of `scratch` on the current device, looked up once per device
static int scratch_address(void** ptr) {
  int dev = 0;
  SW_HIP(hipGetDevice(&dev));
  SW_CHECK(dev >= 0 && dev < kMaxDevices, "chi2_noalloc: device index %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    SW_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    SW_CHECK(p != nullptr, "chi2_noalloc: no device address for the scratch array on device %d", dev);
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return SW_OK;
}

extern "C" int64_t chi2_noalloc_max_con(void) { return kNoAllocMaxCon; }

extern "C" int chi2_noalloc(const void* A, int32_t dtype, int64_t n_orb, int64_t n_con, const double* w,
                            const double* d, const double* sigma, int64_t col_begin, int64_t col_end, double* out,
                            void* stream) {
  SW_CHECK(dtype == SW_F32 || dtype == SW_F64, "chi2_noalloc: dtype must be SW_F32 or SW_F64");
  SW_CHECK(n_orb > 0 && n_con > 0, "chi2_noalloc: need n_orb > 0 and n_con > 0");
  SW_CHECK(n_con <= kNoAllocMaxCon, "chi2_noalloc: n_con = %lld exceeds the static scratch limit of %lld constraints",
           (long long)n_con, (long long)kNoAllocMaxCon);
  SW_CHECK(col_begin >= 0 && col_end <= n_con && col_begin <= col_end, "chi2_noalloc: bad column range");
  SW_CHECK(A && w && d && sigma && out, "chi2_noalloc: null argument");
  void* ptr = nullptr;
  const int rc = scratch_address(&ptr);
  if (rc != SW_OK) return rc;
  return chi2_launch(A, dtype, n_orb, n_con, w, d, sigma, col_begin, col_end, kNoAllocSlabs, (char*)ptr, out,
                     (hipStream_t)stream);
}

extern "C" int model_observables(const void* A, int32_t dtype, int64_t n_orb, int64_t n_con, const double* w,
                                 double* out, void* stream) {
  SW_CHECK(dtype == SW_F32 || dtype == SW_F64, "model_observables: dtype must be SW_F32 or SW_F64");
  SW_CHECK(n_orb >= 0 && n_con >= 0, "model_observables: negative size");
  if (n_con == 0) return SW_OK;
  SW_CHECK(out, "model_observables: null output");
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for(n_con)), dim3(256), 0, st, out, n_con, 0.0);
  if (n_orb == 0) {
    SW_HIP(hipGetLastError());
    return SW_OK;
  }
  SW_CHECK(A && w, "model_observables: null input");
  const int64_t rps = (n_orb + kSlabs - 1) / kSlabs;
  dim3 grid((unsigned)((n_con + kColTile - 1) / kColTile), (unsigned)kSlabs);
  if (dtype == SW_F32)
    hipLaunchKernelGGL(k_colsum1<float>, grid, dim3(kColThreads), 0, st, (const float*)A, n_orb, n_con, w, rps, out, 1);
  else
    hipLaunchKernelGGL(k_colsum1<double>, grid, dim3(kColThreads), 0, st, (const double*)A, n_orb, n_con, w, rps, out,
                       1);
  SW_HIP(hipGetLastError());
  return SW_OK;
}
