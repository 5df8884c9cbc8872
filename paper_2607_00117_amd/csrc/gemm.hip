// MFMA kernels of the weight solve: the constraint-space Gram matrix, the
// fp32 GEMM used by the blocked Cholesky factorisation and the inversion of
// its factor, the diagonal-block factor + inverse, and the matrix-vector
// products that apply the inverse.
//
// Tiling: a 256-thread workgroup (4 waves in a 2 x 2 grid) owns a 128 x 128
// output tile; each wave owns 64 x 64 = 2 x 2 blocks of the 32 x 32 MFMA
// output.  Operands are staged through LDS with row padding chosen so that
// the per-lane MFMA operand reads hit distinct banks.  Symmetric outputs
// launch only the tiles on or below the diagonal, and consecutive workgroup
// ids are spread so that each XCD (ids congruent mod 8) works on a
// contiguous run of tiles, which share operand panels in that XCD's L2.
#include <algorithm>

#include "gemm.h"

namespace sw {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kT = 128;      // output tile
constexpr int kThreads = 256;
constexpr int kXcd = 8;

// workgroup id -> tile id so that XCD x (ids = x mod 8) gets a contiguous range
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
  const int64_t per = (nb + kXcd - 1) / kXcd;
  const int64_t x = b % kXcd, r = b / kXcd;
  const int64_t t = x * per + r;
  return t;  // may exceed nb - 1 for the last XCD; caller checks
}

// Super-tiled schedule of a lower-triangular tile grid (nt x nt tiles).  The
// grid is cut into kSuper x kSuper super-tiles; super-tile s (lower triangle,
// row-major) is processed by XCD s mod 8 as kSuper^2 consecutive workgroups of
// that XCD, so the workgroups resident on one XCD at a time share kSuper row
// panels and kSuper column panels in its L2 instead of streaming a new panel
// each.  Workgroup ids are dealt to XCDs round-robin (id mod 8).
constexpr int kSuper = 8;

__device__ __forceinline__ int64_t super_count(int64_t nt) {
  const int64_t S = (nt + kSuper - 1) / kSuper;
  return S * (S + 1) / 2;
}

// tile id -> (row tile, col tile) over the lower triangle, row-major
__device__ __forceinline__ void tri_tile(int64_t t, int64_t& tm, int64_t& tn) {
  int64_t m = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((m + 1) * (m + 2) / 2 <= t) ++m;
  while (m * (m + 1) / 2 > t) --m;
  tm = m;
  tn = t - m * (m + 1) / 2;
}

// workgroup id -> tile of the super-tiled schedule; false when the workgroup
// has no tile (above the diagonal of a diagonal super-tile, or past the edge)
__device__ __forceinline__ bool super_tile(int64_t b, int64_t nt, int64_t& tm, int64_t& tn) {
  const int64_t x = b % kXcd, r = b / kXcd;
  const int64_t s = (r / (kSuper * kSuper)) * kXcd + x, q = r % (kSuper * kSuper);
  if (s >= super_count(nt)) return false;
  int64_t I, J;
  tri_tile(s, I, J);
  tm = I * kSuper + q / kSuper;
  tn = J * kSuper + q % kSuper;
  return tm < nt && tn <= tm;
}

// number of workgroups for the super-tiled schedule
static int64_t super_grid(int64_t nt) {
  const int64_t S = (nt + kSuper - 1) / kSuper;
  const int64_t ns = S * (S + 1) / 2;
  return ((ns + kXcd - 1) / kXcd) * kXcd * kSuper * kSuper;
}

// ---------------------------------------------------------------------------
// Gram: K[m][n] = sum_k X[m][k] X[n][k], bf16 operands, fp32 accumulate.
//
// A 512-thread workgroup owns a 256 x 256 tile of K; its 8 waves form a
// 2 x 4 grid of 128 x 64 blocks (4 x 2 MFMA 32x32 outputs each), so a wave
// issues 24 (X3: hi.hi + hi.lo + lo.hi) MFMAs per 12 operand reads from LDS.
// Operands stream through two LDS buffers in k-stages of 32 (rows padded to
// 80 bytes so the 16-byte reads of a half-wave hit distinct banks): while a
// stage is consumed from one buffer the next is fetched into registers and
// then written to the other, one barrier per stage.  On diagonal tiles the
// row and column panels coincide and are staged once.
// X is stored stage-blocked (gram_at): the 256 x 32 block of a row panel and a
// stage is 16 KB of contiguous memory, so a stage's fetch is two fully
// coalesced 8 KB sweeps of the workgroup instead of 256 row pieces of 64 bytes
// spread over the whole panel.
// Stage skipping: when `nz` is given, bit g of nz[t * nzw + g / 64] says
// whether rows [256 t, 256 t + 256) of X have a nonzero in columns
// [32 g, 32 g + 32) (global stage g); a stage whose row panel or column panel
// is zero adds nothing and is skipped.
// Low-plane skipping (X3): when `nzl` is given (same layout, for the lo plane),
// a stage whose row panel has a zero lo plane needs no lo(A) hi(B) product and
// one whose column panel has none no hi(A) lo(B) product; their lo planes are
// then neither fetched nor staged.  For a matrix of counts the operand is the
// counts themselves, whose lo plane is zero up to 256, and `cs` (per row of X)
// scales the result: K[m][n] = cs[m] cs[n] sum_k X[m][k] X[n][k].
// X has Mx rows (a multiple of 256, zero past the constraints); entries of K
// are stored for rows and columns below M only.
// ---------------------------------------------------------------------------
constexpr int kGT = 256;
constexpr int kGThreads = 512;
constexpr int kGBK = 32;
constexpr int kGPad = kGBK + 8;

template <bool X3>
__global__ __launch_bounds__(kGThreads) void k_gram_bf16(const __bf16* __restrict__ hi, const __bf16* __restrict__ lo,
                                                         const int64_t* __restrict__ xoff,
                                                         const int64_t* __restrict__ xlen, int64_t ld,
                                                         float* __restrict__ Kall, int64_t ldk, int64_t sK, int64_t M,
                                                         int64_t nt, const uint64_t* __restrict__ nz, int64_t nzw,
                                                         const uint64_t* __restrict__ nzl,
                                                         const float* __restrict__ csall, int64_t scs) {
  constexpr int NM = X3 ? 4 : 2;  // staged panels: A hi, B hi (, A lo, B lo)
  __shared__ __attribute__((aligned(16))) __bf16 sm[2][NM][kGT][kGPad];
  const int64_t bp = blockIdx.y;
  int64_t tm, tn;
  if (!super_tile(blockIdx.x, nt, tm, tn)) return;
  const int64_t g0 = xoff[bp] / kGBK, g1 = (xoff[bp] + xlen[bp]) / kGBK;  // global stages of problem bp
  float* __restrict__ K = Kall + bp * sK;
  const bool diag = tm == tn;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 2, wn = w & 3;  // wave block: rows wm*128.., cols wn*64..
  floatx16 acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.0f;

  // the next stage >= g whose row and column panels both hold a nonzero (g1: none)
  const uint64_t* nzA = nz ? nz + tm * nzw : nullptr;
  const uint64_t* nzB = nz ? nz + tn * nzw : nullptr;
  const uint64_t* nlA = nzl ? nzl + tm * nzw : nullptr;
  const uint64_t* nlB = nzl ? nzl + tn * nzw : nullptr;
  // whether stage g's lo plane of the row (column) panel holds a nonzero
  auto lo_a = [&](int64_t g) -> bool { return !nlA || ((nlA[g >> 6] >> (g & 63)) & 1ull); };
  auto lo_b = [&](int64_t g) -> bool { return !nlB || ((nlB[g >> 6] >> (g & 63)) & 1ull); };
  auto next = [&](int64_t g) -> int64_t {
    if (!nzA) return g;
    while (g < g1) {
      const int64_t wd = g >> 6;
      const uint64_t m = (nzA[wd] & nzB[wd]) & (~0ull << (g & 63));
      if (m) {
        const int64_t c = (wd << 6) + __builtin_ctzll(m);
        return c < g1 ? c : g1;
      }
      g = (wd + 1) << 6;
    }
    return g1;
  };

  // a panel stage is 256 rows x 32 k = 1024 chunks of 16 B, 2 per thread:
  // chunk q = tid + 512 j is row q / 4, k offset 8 (q % 4)
  // (in the stage block, chunk q sits at element 8 q: the workgroup reads the
  // block's two halves front to back)
  const int r0 = tid >> 2, r1 = r0 + kGThreads / 4, cc = (tid & 3) * 8;
  const __bf16* pAh = hi + tm * kGT * ld + tid * 8;
  const __bf16* pBh = hi + tn * kGT * ld + tid * 8;
  const __bf16* pAl = lo + tm * kGT * ld + tid * 8;
  const __bf16* pBl = lo + tn * kGT * ld + tid * 8;
  constexpr int64_t kHalf = kGThreads * 8;  // elements in half a stage block
  uint4 gAh0, gAh1, gBh0, gBh1, gAl0, gAl1, gBl0, gBl1;
  // la / lb: the stage's lo planes of the row / column panel are used
  auto gload = [&](int64_t g, bool la, bool lb) {
    const int64_t k0 = g * (kGT * kGBK);
    gAh0 = *reinterpret_cast<const uint4*>(pAh + k0);
    gAh1 = *reinterpret_cast<const uint4*>(pAh + k0 + kHalf);
    if (!diag) {
      gBh0 = *reinterpret_cast<const uint4*>(pBh + k0);
      gBh1 = *reinterpret_cast<const uint4*>(pBh + k0 + kHalf);
    }
    if constexpr (X3) {
      if (la) {
        gAl0 = *reinterpret_cast<const uint4*>(pAl + k0);
        gAl1 = *reinterpret_cast<const uint4*>(pAl + k0 + kHalf);
      }
      if (!diag && lb) {
        gBl0 = *reinterpret_cast<const uint4*>(pBl + k0);
        gBl1 = *reinterpret_cast<const uint4*>(pBl + k0 + kHalf);
      }
    }
  };
  auto stage = [&](int buf, bool la, bool lb) {
    *reinterpret_cast<uint4*>(&sm[buf][0][r0][cc]) = gAh0;
    *reinterpret_cast<uint4*>(&sm[buf][0][r1][cc]) = gAh1;
    if (!diag) {
      *reinterpret_cast<uint4*>(&sm[buf][1][r0][cc]) = gBh0;
      *reinterpret_cast<uint4*>(&sm[buf][1][r1][cc]) = gBh1;
    }
    if constexpr (X3) {
      if (la) {
        *reinterpret_cast<uint4*>(&sm[buf][2][r0][cc]) = gAl0;
        *reinterpret_cast<uint4*>(&sm[buf][2][r1][cc]) = gAl1;
      }
      if (!diag && lb) {
        *reinterpret_cast<uint4*>(&sm[buf][3][r0][cc]) = gBl0;
        *reinterpret_cast<uint4*>(&sm[buf][3][r1][cc]) = gBl1;
      }
    }
  };
  const int bA = 0, bB = diag ? 0 : 1;  // LDS panels read as A and as B
  int64_t g = next(g0);
  int buf = 0;
  bool la = false, lb = false;  // lo planes of the current stage
  if (g < g1) {
    la = lo_a(g);
    lb = diag ? la : lo_b(g);
    gload(g, la, lb);
    stage(0, la, lb);
  }
  __syncthreads();
  while (g < g1) {
    const int64_t gn = next(g + 1);
    bool lan = false, lbn = false;
    if (gn < g1) {
      lan = lo_a(gn);
      lbn = diag ? lan : lo_b(gn);
      gload(gn, lan, lbn);
    }
#pragma unroll
    for (int ks = 0; ks < kGBK / 16; ++ks) {
      const int kc = ks * 16 + 8 * (lane >> 5);
      bf16x8 bn[2], bnl[2], am[4], aml[4];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        bn[b] = *reinterpret_cast<const bf16x8*>(&sm[buf][bB][wn * 64 + b * 32 + (lane & 31)][kc]);
        if constexpr (X3)
          if (lb) bnl[b] = *reinterpret_cast<const bf16x8*>(&sm[buf][bB + 2][wn * 64 + b * 32 + (lane & 31)][kc]);
      }
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        am[a] = *reinterpret_cast<const bf16x8*>(&sm[buf][bA][wm * 128 + a * 32 + (lane & 31)][kc]);
        if constexpr (X3)
          if (la) aml[a] = *reinterpret_cast<const bf16x8*>(&sm[buf][bA + 2][wm * 128 + a * 32 + (lane & 31)][kc]);
      }
      // each sweep issues 8 MFMAs on 8 different accumulators, so no MFMA waits
      // for the one before it
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am[a], bn[b], acc[a][b], 0, 0, 0);
      if constexpr (X3) {
        if (lb) {
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
              acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am[a], bnl[b], acc[a][b], 0, 0, 0);
        }
        if (la) {
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
              acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aml[a], bn[b], acc[a][b], 0, 0, 0);
        }
      }
    }
    // the other buffer was last read before the previous barrier
    if (gn < g1) stage(buf ^ 1, lan, lbn);
    __syncthreads();
    buf ^= 1;
    g = gn;
    la = lan;
    lb = lbn;
  }
  const bool edge = (tm + 1) * kGT > M;  // only the last tile row/column can cross M
  const float* cs = csall ? csall + bp * scs : nullptr;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int64_t col = tn * kGT + wn * 64 + b * 32 + (lane & 31);
      const float sn = cs && col < M ? cs[col] : 1.0f;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int64_t row = tm * kGT + wm * 128 + a * 32 + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
        if (!edge || (row < M && col < M)) K[row * ldk + col] = cs ? acc[a][b][i] * (cs[row] * sn) : acc[a][b][i];
      }
    }
}

// Tile of a 128-tiled GEMM workgroup (false: none).  With a lower-triangular
// A (a_lower) and a full output, row tile tm has (tm + 1) * 128 inner terms;
// row tiles are then dealt to the XCDs round-robin from the longest down (XCD
// x gets the k-th longest for k = x mod 8), each XCD taking all column tiles
// of its row tiles: every XCD gets an equal share of long and short tiles, and
// an A row panel is read by one XCD only.  Otherwise XCD x takes a contiguous
// run of tiles (row-major, or the lower triangle when `lower`).
__device__ __forceinline__ bool gemm_tile(int64_t ntn, int lower, int a_lower, int64_t n_tiles, int64_t& tm,
                                          int64_t& tn) {
  if (a_lower && !lower) {
    const int64_t ntm = n_tiles / ntn;
    const int64_t x = blockIdx.x % kXcd, r = blockIdx.x / kXcd, i = r / ntn;
    const int64_t k = i * kXcd + x;
    if (k >= ntm) return false;
    tm = ntm - 1 - k;
    tn = r - i * ntn;
    return true;
  }
  const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
  if (t >= n_tiles) return false;
  if (lower) tri_tile(t, tm, tn);
  else { tm = t / ntn; tn = t - tm * ntn; }
  return true;
}

// ---------------------------------------------------------------------------
// fp32 GEMM, C = beta C + alpha A B^T, MFMA 32x32x2 f32.
// ---------------------------------------------------------------------------
constexpr int kBKf = 32;
constexpr int kPadF = kBKf + 1;
typedef float f32x4v __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kThreads) void k_gemm_nt_f32(int64_t ntn, int64_t K, float alpha,
                                                          const float* __restrict__ A, int64_t lda, int64_t sA,
                                                          const float* __restrict__ B, int64_t ldb, int64_t sB,
                                                          float beta, float* __restrict__ C, int64_t ldc, int64_t sC,
                                                          int lower, int a_lower, int64_t n_tiles, int64_t kc,
                                                          int64_t sPart) {
  A += blockIdx.y * sA;
  B += blockIdx.y * sB;
  C += blockIdx.y * sC;
  __shared__ float As[kT][kPadF];
  __shared__ float Bs[kT][kPadF];
  int64_t tm, tn;
  if (!gemm_tile(ntn, lower, a_lower, n_tiles, tm, tn)) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  floatx16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.0f;
  const float* Ab = A + tm * kT * lda;
  const float* Bb = B + tn * kT * ldb;
  float4 ra[4], rb[4];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int idx = tid + kThreads * i;
      const int r = idx >> 3, c = (idx & 7) * 4;
      ra[i] = *reinterpret_cast<const float4*>(Ab + (int64_t)r * lda + k0 + c);
      rb[i] = *reinterpret_cast<const float4*>(Bb + (int64_t)r * ldb + k0 + c);
    }
  };
  // a_lower: A is lower triangular in 128-tiles, so row tile tm needs k < (tm + 1) * 128 only
  int64_t Kend = (a_lower && (tm + 1) * kT < K) ? (tm + 1) * kT : K;
  int64_t kbeg = 0;
  if (kc > 0) {  // split K: chunk z covers [z kc, (z+1) kc) and writes its own partial product
    kbeg = (int64_t)blockIdx.z * kc;
    if (kbeg >= Kend) return;
    Kend = kbeg + kc < Kend ? kbeg + kc : Kend;
    C += (int64_t)blockIdx.z * sPart;
  }
  gload(kbeg);
  for (int64_t k0 = kbeg; k0 < Kend; k0 += kBKf) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int idx = tid + kThreads * i;
      const int r = idx >> 3, c = (idx & 7) * 4;
      As[r][c] = ra[i].x; As[r][c + 1] = ra[i].y; As[r][c + 2] = ra[i].z; As[r][c + 3] = ra[i].w;
      Bs[r][c] = rb[i].x; Bs[r][c + 1] = rb[i].y; Bs[r][c + 2] = rb[i].z; Bs[r][c + 3] = rb[i].w;
    }
    __syncthreads();
    if (k0 + kBKf < Kend) gload(k0 + kBKf);
#pragma unroll
    for (int kk = 0; kk < kBKf; kk += 2) {
      const int kc = kk + (lane >> 5);
      float am[2], bn[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        am[a] = As[wm * 64 + a * 32 + (lane & 31)][kc];
        bn[a] = Bs[wn * 64 + a * 32 + (lane & 31)][kc];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(am[a], bn[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int64_t row = tm * kT + wm * 64 + a * 32 + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
        const int64_t col = tn * kT + wn * 64 + b * 32 + (lane & 31);
        float* cp = C + row * ldc + col;
        const float v = alpha * acc[a][b][i];
        *cp = (beta == 0.0f) ? v : beta * (*cp) + v;
      }
}

// ---------------------------------------------------------------------------
// The same product with each fp32 operand split on the fly into a bf16 pair,
// x = hi + lo (hi = x rounded to bf16, lo = the remainder rounded to bf16), and
// C = beta C + alpha (A_hi B_hi^T + A_hi B_lo^T + A_lo B_hi^T) on bf16 MFMA
// (32x32x16) with fp32 accumulation: the dropped terms are ~2^-16 of each
// product.  Same tiles, schedule and split-K as k_gemm_nt_f32; operands are
// staged as hi/lo planes in two LDS buffers (rows padded to 80 bytes).
// ---------------------------------------------------------------------------
constexpr int kX3Pad = kBKf + 8;

__global__ __launch_bounds__(kThreads) void k_gemm_nt_x3(int64_t ntn, int64_t K, float alpha,
                                                         const float* __restrict__ A, int64_t lda, int64_t sA,
                                                         const float* __restrict__ B, int64_t ldb, int64_t sB,
                                                         float beta, float* __restrict__ C, int64_t ldc, int64_t sC,
                                                         int lower, int a_lower, int64_t n_tiles, int64_t kc,
                                                         int64_t sPart) {
  A += blockIdx.y * sA;
  B += blockIdx.y * sB;
  C += blockIdx.y * sC;
  __shared__ __attribute__((aligned(16))) __bf16 sm[2][4][kT][kX3Pad];  // [buffer] A hi, B hi, A lo, B lo
  int64_t tm, tn;
  if (!gemm_tile(ntn, lower, a_lower, n_tiles, tm, tn)) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  floatx16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.0f;
  const float* Ab = A + tm * kT * lda;
  const float* Bb = B + tn * kT * ldb;
  // a stage is 128 rows x 32 k of each operand: thread t loads rows t/8 + 32 i,
  // k offset 4 (t % 8), as four float4 per operand
  float4 ra[4], rb[4];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int idx = tid + kThreads * i;
      const int r = idx >> 3, c = (idx & 7) * 4;
      ra[i] = *reinterpret_cast<const float4*>(Ab + (int64_t)r * lda + k0 + c);
      rb[i] = *reinterpret_cast<const float4*>(Bb + (int64_t)r * ldb + k0 + c);
    }
  };
  auto split4 = [](const float4 v, __bf16* hi, __bf16* lo) {
    const float x[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const __bf16 h = (__bf16)x[j];
      hi[j] = h;
      lo[j] = (__bf16)(x[j] - (float)h);
    }
  };
  int64_t Kend = (a_lower && (tm + 1) * kT < K) ? (tm + 1) * kT : K;
  int64_t kbeg = 0;
  if (kc > 0) {
    kbeg = (int64_t)blockIdx.z * kc;
    if (kbeg >= Kend) return;
    Kend = kbeg + kc < Kend ? kbeg + kc : Kend;
    C += (int64_t)blockIdx.z * sPart;
  }
  auto stage = [&](int buf) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int idx = tid + kThreads * i;
      const int r = idx >> 3, c = (idx & 7) * 4;
      __bf16 h[4], l[4];
      split4(ra[i], h, l);
      *reinterpret_cast<uint2*>(&sm[buf][0][r][c]) = *reinterpret_cast<const uint2*>(h);
      *reinterpret_cast<uint2*>(&sm[buf][2][r][c]) = *reinterpret_cast<const uint2*>(l);
      split4(rb[i], h, l);
      *reinterpret_cast<uint2*>(&sm[buf][1][r][c]) = *reinterpret_cast<const uint2*>(h);
      *reinterpret_cast<uint2*>(&sm[buf][3][r][c]) = *reinterpret_cast<const uint2*>(l);
    }
  };
  // two stage buffers: while one is multiplied the next stage is fetched into
  // registers and then written to the other, one barrier per stage
  int buf = 0;
  gload(kbeg);
  stage(0);
  __syncthreads();
  for (int64_t k0 = kbeg; k0 < Kend; k0 += kBKf) {
    const bool more = k0 + kBKf < Kend;
    if (more) gload(k0 + kBKf);
#pragma unroll
    for (int ks = 0; ks < kBKf / 16; ++ks) {
      const int kcol = ks * 16 + 8 * (lane >> 5);
      bf16x8 bh[2], bl[2];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        bh[b] = *reinterpret_cast<const bf16x8*>(&sm[buf][1][wn * 64 + b * 32 + (lane & 31)][kcol]);
        bl[b] = *reinterpret_cast<const bf16x8*>(&sm[buf][3][wn * 64 + b * 32 + (lane & 31)][kcol]);
      }
      bf16x8 ah[2], al[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        ah[a] = *reinterpret_cast<const bf16x8*>(&sm[buf][0][wm * 64 + a * 32 + (lane & 31)][kcol]);
        al[a] = *reinterpret_cast<const bf16x8*>(&sm[buf][2][wm * 64 + a * 32 + (lane & 31)][kcol]);
      }
      // sweeps over the 4 accumulators: no MFMA waits for the one before it
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
    }
    // the other buffer was last read before the previous barrier
    if (more) stage(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int64_t row = tm * kT + wm * 64 + a * 32 + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
        const int64_t col = tn * kT + wn * 64 + b * 32 + (lane & 31);
        float* cp = C + row * ldc + col;
        const float v = alpha * acc[a][b][i];
        *cp = (beta == 0.0f) ? v : beta * (*cp) + v;
      }
}

// Sum of the split-K partials of an M x N product (partials compact, ld N)
// whose row tile tm has min((tm + 1) 128, K) inner terms (a lower-triangular
// left operand): out (ld ldo) = sum over the chunks that tile has, in chunk
// order.
__global__ __launch_bounds__(kThreads) void k_sum_parts(const float* __restrict__ parts, int64_t sPart, int64_t sP,
                                                        int64_t M, int64_t N, int64_t K, int64_t kc,
                                                        float* __restrict__ out, int64_t ldo, int64_t sOut) {
  parts += blockIdx.y * sP;
  out += blockIdx.y * sOut;
  const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;  // float4 index
  const int64_t n4 = N / 4;
  if (q >= M * n4) return;
  const int64_t r = q / n4, c4 = q - r * n4;
  const int64_t tm = r / kT;
  const int64_t kend = (tm + 1) * kT < K ? (tm + 1) * kT : K;
  const int64_t nc = (kend + kc - 1) / kc;
  const f32x4v* p = reinterpret_cast<const f32x4v*>(parts) + q;
  f32x4v acc = p[0];
  for (int64_t c = 1; c < nc; ++c) acc += p[c * (sPart / 4)];
  reinterpret_cast<f32x4v*>(out + r * ldo)[c4] = acc;
}

// out[r][c] = 0 for a rows x cols block (cols multiple of 4), ld ldo
__global__ __launch_bounds__(kThreads) void k_zero_block(float* __restrict__ out, int64_t ldo, int64_t sOut,
                                                         int64_t rows, int64_t cols) {
  out += blockIdx.y * sOut;
  const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t c4 = cols / 4;
  if (q >= rows * c4) return;
  const int64_t r = q / c4;
  reinterpret_cast<f32x4v*>(out + r * ldo)[q - r * c4] = f32x4v{0.0f, 0.0f, 0.0f, 0.0f};
}

// ---------------------------------------------------------------------------
// Diagonal block of the factorisation: unblocked right-looking Cholesky of a
// 128 x 128 block fused with the inverse of its factor by right-looking
// forward substitution on the identity; the factor overwrites the block and
// its inverse goes to dinv.  The block lives in registers: thread (ty, tx) of
// a 32 x 32 grid owns the elements (ty + 32p, tx + 32q), p, q < 4, a cyclic
// layout that keeps every thread busy down to the last columns.  Step k
// finishes column k of the factor and row k of the inverse, broadcasts them
// through LDS with the entries that must not change set to zero, and applies
// both rank-1 updates as 32 unconditional fused multiply-adds per thread,
// which leave finished rows and columns exactly as they are.  A non-positive
// pivot sets *bad and is replaced by a tiny positive value so the factor stays
// finite.
// ---------------------------------------------------------------------------
constexpr int kPotrfThreads = 1024;

__global__ __launch_bounds__(kPotrfThreads) void k_potrf_diag(float* __restrict__ Kd, int64_t ld, int64_t sK,
                                                              float* __restrict__ dinv, int64_t sD,
                                                              int* __restrict__ bad) {
  Kd += blockIdx.x * sK;
  dinv += blockIdx.x * sD;
  __shared__ float col[kNB];  // column k of the factor below the diagonal, 0 elsewhere
  __shared__ float row[kNB];  // row k of the inverse
  __shared__ float dg[kNB];   // pending pivot of each step
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  float a[4][4], x[4][4];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = ty + 32 * p, j = tx + 32 * q;
      a[p][q] = (j <= i) ? Kd[(int64_t)i * ld + j] : 0.0f;
      x[p][q] = (i == j) ? 1.0f : 0.0f;
    }
  if (threadIdx.x == 0) dg[0] = a[0][0];
  __syncthreads();
  for (int k = 0; k < kNB; ++k) {
    const int pk = k >> 5, rk = k & 31;
    float piv = dg[k];
    if (!(piv > 0.0f)) {
      if (threadIdx.x == 0) atomicExch(bad, 1);
      piv = 1e-30f;
    }
    piv = sqrtf(piv);
    const float ip = 1.0f / piv;
    if (tx == rk) {  // owners of column k
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (q != pk) continue;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const int i = ty + 32 * p;
          const float v = (i > k) ? a[p][q] * ip : 0.0f;
          if (i > k) a[p][q] = v;
          if (i == k) a[p][q] = piv;
          col[i] = v;
        }
      }
    }
    if (ty == rk) {  // owners of row k of the inverse: final once scaled by 1/L_kk
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        if (p != pk) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          x[p][q] *= ip;
          row[tx + 32 * q] = x[p][q];
        }
      }
    }
    __syncthreads();
    float ci[4], cj[4], rj[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) ci[p] = col[ty + 32 * p];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      cj[q] = col[tx + 32 * q];
      rj[q] = row[tx + 32 * q];
    }
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[p][q] -= ci[p] * cj[q];
        x[p][q] -= ci[p] * rj[q];
      }
    if (k + 1 < kNB) {
      const int k1 = k + 1, r1 = k1 & 31, p1 = k1 >> 5;
      if (tx == r1 && ty == r1) {
#pragma unroll
        for (int p = 0; p < 4; ++p)
          if (p == p1) dg[k1] = a[p][p];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = ty + 32 * p, j = tx + 32 * q;
      Kd[(int64_t)i * ld + j] = (j <= i) ? a[p][q] : 0.0f;
      dinv[i * kNB + j] = (j <= i) ? x[p][q] : 0.0f;
    }
}

// ---------------------------------------------------------------------------
// Explicit inverse of the Cholesky factor, W = L^-1, and its application.
// The factor buffer ends up holding S = W + W^T - diag(W): W in the lower
// triangle, W^T in the upper one (they agree on the diagonal), so that
//   (L L^T)^-1 r = W^T (W r)
// is two row-major matrix-vector products over the two halves of S, each a
// single HBM-bound pass with no dependency chain between row blocks.
// ---------------------------------------------------------------------------
constexpr int kTT = 64;  // transpose tile

// dst[c][r] = src[r][c] for a rows x cols block (both multiples of 64)
__global__ __launch_bounds__(kThreads) void k_transpose(const float* __restrict__ src, int64_t lds, int64_t sS,
                                                        float* __restrict__ dst, int64_t ldd, int64_t sDst,
                                                        int64_t tiles_c) {
  __shared__ float t[kTT][kTT + 1];
  src += blockIdx.y * sS;
  dst += blockIdx.y * sDst;
  const int64_t tr = blockIdx.x / tiles_c, tc = blockIdx.x - tr * tiles_c;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int i = ty; i < kTT; i += 4) t[i][tx] = src[(tr * kTT + i) * lds + tc * kTT + tx];
  __syncthreads();
  for (int i = ty; i < kTT; i += 4) dst[(tc * kTT + i) * ldd + tr * kTT + tx] = t[tx][i];
}

// diagonal block j of the factor buffer <- inv(L_jj) (lower, zeros above)
__global__ __launch_bounds__(kThreads) void k_set_diag_inv(float* __restrict__ K, int64_t ld, int64_t sK,
                                                           const float* __restrict__ dinv, int64_t sD) {
  K += blockIdx.y * sK;
  dinv += blockIdx.y * sD;
  const int64_t j = blockIdx.x;
  const float* D = dinv + j * kNB * kNB;
  for (int idx = threadIdx.x; idx < kNB * kNB; idx += kThreads) {
    const int r = idx / kNB, c = idx - r * kNB;
    K[(j * kNB + r) * ld + j * kNB + c] = D[idx];
  }
}

// S[c][r] = S[r][c] for r > c: the strictly lower triangle mirrored upward,
// one 64 x 64 tile on or below the diagonal per workgroup
__global__ __launch_bounds__(kThreads) void k_mirror_lower(float* __restrict__ S, int64_t ld, int64_t sK) {
  __shared__ float t[kTT][kTT + 1];
  S += blockIdx.y * sK;
  int64_t tr, tc;
  tri_tile(blockIdx.x, tr, tc);
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int i = ty; i < kTT; i += 4) t[i][tx] = S[(tr * kTT + i) * ld + tc * kTT + tx];
  __syncthreads();
  for (int i = ty; i < kTT; i += 4) {
    // destination row tc*64+i, column tr*64+tx holds source (tr*64+tx, tc*64+i)
    if (tr != tc || tx > i) S[(tc * kTT + i) * ld + tr * kTT + tx] = t[tx][i];
  }
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// y = T x over one half of S (LOWER: j <= i, else j >= i).  One wave owns the
// row pair (i, n-1-i), so every wave streams n+1 entries; loads of S bypass
// the caches (each entry is read once) while x stays resident in L2.
template <bool LOWER>
__device__ __forceinline__ float trmv_row(const float* __restrict__ Sr, const float* __restrict__ x, int64_t i,
                                          int64_t n, int lane) {
  int64_t j0 = LOWER ? 0 : i, j1 = LOWER ? i + 1 : n;
  float acc = 0.0f;
  // unaligned head (UPPER) / tail (LOWER), at most 3 entries
  const int64_t a0 = (j0 + 3) & ~(int64_t)3, a1 = j1 & ~(int64_t)3;
  if (lane < a0 - j0) acc += Sr[j0 + lane] * x[j0 + lane];
  if (lane < j1 - a1 && a1 >= a0) acc += Sr[a1 + lane] * x[a1 + lane];
  float acc2 = 0.0f;
  int64_t j = a0 + 4 * lane;
  for (; j + 256 < a1; j += 512) {
    const f32x4 s0 = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(Sr + j));
    const f32x4 s1 = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(Sr + j + 256));
    const f32x4 x0 = *reinterpret_cast<const f32x4*>(x + j);
    const f32x4 x1 = *reinterpret_cast<const f32x4*>(x + j + 256);
    acc += s0[0] * x0[0] + s0[1] * x0[1] + s0[2] * x0[2] + s0[3] * x0[3];
    acc2 += s1[0] * x1[0] + s1[1] * x1[1] + s1[2] * x1[2] + s1[3] * x1[3];
  }
  if (j < a1) {
    const f32x4 s0 = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(Sr + j));
    const f32x4 x0 = *reinterpret_cast<const f32x4*>(x + j);
    acc += s0[0] * x0[0] + s0[1] * x0[1] + s0[2] * x0[2] + s0[3] * x0[3];
  }
  acc += acc2;
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  return acc;
}

template <bool LOWER>
__global__ __launch_bounds__(kThreads) void k_trmv(const float* __restrict__ S, int64_t n, int64_t ld, int64_t sK,
                                                   const float* __restrict__ x, float* __restrict__ y, int64_t sv,
                                                   const double* __restrict__ act, int act_stride) {
  const int64_t b = blockIdx.y;
  if (act && act[b * act_stride] == 0.0) return;
  S += b * sK;
  x += b * sv;
  y += b * sv;
  const int lane = threadIdx.x & 63;
  const int64_t wv = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (wv >= n / 2) return;
  const int64_t i0 = wv, i1 = n - 1 - wv;
  const float v0 = trmv_row<LOWER>(S + i0 * ld, x, i0, n, lane);
  const float v1 = trmv_row<LOWER>(S + i1 * ld, x, i1, n, lane);
  if (lane == 0) {
    y[i0] = v0;
    y[i1] = v1;
  }
}

// y = T x, T the lower (j <= i) or upper (j >= i) half of the row-major S
// (leading dimension ld), n a multiple of 16.  Wave g owns rows 8g .. 8g+7
// and their mirror rows n-8-8g .. n-1-8g (8 (n + 1) entries of the half for
// every wave) and streams their columns 256 at a time, four per lane: one load
// of x serves up to 16 rows.  A chunk that straddles the diagonal of a group
// of rows is masked entry by entry; a chunk outside a group's half is skipped.
template <bool LOWER>
__global__ __launch_bounds__(kThreads) void k_trmv16(const float* __restrict__ S, int64_t n, int64_t ld, int64_t sK,
                                                     const float* __restrict__ x, float* __restrict__ y, int64_t sv,
                                                     const double* __restrict__ act, int act_stride) {
  const int64_t b = blockIdx.y;
  if (act && act[b * act_stride] == 0.0) return;
  S += b * sK;
  x += b * sv;
  y += b * sv;
  const int lane = threadIdx.x & 63;
  const int64_t g = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (g >= n / 16) return;
  const int64_t R[2] = {8 * g, n - 8 - 8 * g};  // first rows of the two groups
  // the columns that a row of either group holds
  const int64_t lo = LOWER ? 0 : R[0] & ~(int64_t)255, hi = LOWER ? R[1] + 8 : n;
  float acc[2][8];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int r = 0; r < 8; ++r) acc[h][r] = 0.0f;
  for (int64_t jb = lo; jb < hi; jb += 256) {
    const int64_t j = jb + 4 * lane;
    const bool in = j < n;
    bool use[2], full[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      use[h] = LOWER ? jb <= R[h] + 7 : jb + 255 >= R[h];
      full[h] = LOWER ? jb + 255 <= R[h] : jb >= R[h] + 7;
    }
    f32x4 sr[2][8];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int r = 0; r < 8; ++r)
        sr[h][r] = use[h] && in ? __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(S + (R[h] + r) * ld + j))
                                : f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const f32x4 xv = in ? *reinterpret_cast<const f32x4*>(x + j) : f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (!use[h]) continue;
      if (full[h]) {
#pragma unroll
        for (int r = 0; r < 8; ++r)
          acc[h][r] += sr[h][r][0] * xv[0] + sr[h][r][1] * xv[1] + sr[h][r][2] * xv[2] + sr[h][r][3] * xv[3];
      } else {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const int64_t row = R[h] + r;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const bool ok = LOWER ? j + q <= row : j + q >= row;
            acc[h][r] += ok ? sr[h][r][q] * xv[q] : 0.0f;
          }
        }
      }
    }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      float v = acc[h][r];
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
      if (lane == 0) y[R[h] + r] = v;
    }
}

// ---------------------------------------------------------------------------
// Many right-hand sides against one S: Y[b][i] = sum_j T[i][j] X[b][j] for
// b < P, T = the lower (j <= i) or upper (j >= i) half of S, as an fp32 MFMA
// product.  A workgroup owns a pair of 128-row tiles of T, tm and ntm-1-tm, so
// every workgroup streams the same number of entries (the two halves of the
// triangle it covers add up to ntm + 1 tiles of 128 columns), an RHS tile of
// 128 (blockIdx.y) and part z of nzc (blockIdx.z) of each tile's column range
// (split in whole 32-column steps), so that small matrices still give enough
// workgroups; part z of the sums goes to Y + z * sz (nzc == 1: the result).
// Entries of the diagonal tiles outside the half are zeroed as they are staged.
// 4 waves as 2 x 2 blocks of 64 x 64 (MFMA 32x32x2 f32).
// ---------------------------------------------------------------------------
template <bool LOWER>
__global__ __launch_bounds__(kThreads) void k_trmm_rhs(const float* __restrict__ S, int64_t n, int64_t ld,
                                                       const float* __restrict__ X, float* __restrict__ Y,
                                                       int64_t sv, int P, int nzc, int64_t sz) {
  __shared__ float Ts[kT][kPadF];
  __shared__ float Xs[kT][kPadF];
  const int64_t ntm = n / kT;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int64_t b0 = (int64_t)blockIdx.y * kT;
  for (int half = 0; half < 2; ++half) {
    const int64_t tm = half == 0 ? (int64_t)blockIdx.x : ntm - 1 - (int64_t)blockIdx.x;
    if (half == 1 && tm == (int64_t)blockIdx.x) break;  // odd tile count: the middle tile has no partner
    floatx16 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[a][c][i] = 0.0f;
    const int64_t k_lo = LOWER ? 0 : tm * kT, k_hi = LOWER ? (tm + 1) * kT : n;
    const int64_t steps = (k_hi - k_lo) / kBKf, per = (steps + nzc - 1) / nzc;
    const int64_t kbeg = std::min(k_hi, k_lo + (int64_t)blockIdx.z * per * kBKf);
    const int64_t kend = std::min(k_hi, kbeg + per * kBKf);
    const float* Tb = S + tm * kT * ld;
    float4 ra[4], rb[4];
    auto gload = [&](int64_t k0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int idx = tid + kThreads * i;
        const int r = idx >> 3, c = (idx & 7) * 4;
        ra[i] = *reinterpret_cast<const float4*>(Tb + (int64_t)r * ld + k0 + c);
        rb[i] = b0 + r < P ? *reinterpret_cast<const float4*>(X + (b0 + r) * sv + k0 + c)
                           : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      }
    };
    if (kbeg < kend) gload(kbeg);
    for (int64_t k0 = kbeg; k0 < kend; k0 += kBKf) {
      const bool diag = k0 >= tm * kT && k0 < (tm + 1) * kT;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int idx = tid + kThreads * i;
        const int r = idx >> 3, c = (idx & 7) * 4;
        float t[4] = {ra[i].x, ra[i].y, ra[i].z, ra[i].w};
        if (diag) {
          const int64_t row = tm * kT + r;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int64_t col = k0 + c + q;
            if (LOWER ? col > row : col < row) t[q] = 0.0f;
          }
        }
        Ts[r][c] = t[0]; Ts[r][c + 1] = t[1]; Ts[r][c + 2] = t[2]; Ts[r][c + 3] = t[3];
        Xs[r][c] = rb[i].x; Xs[r][c + 1] = rb[i].y; Xs[r][c + 2] = rb[i].z; Xs[r][c + 3] = rb[i].w;
      }
      __syncthreads();
      if (k0 + kBKf < kend) gload(k0 + kBKf);
#pragma unroll
      for (int kk = 0; kk < kBKf; kk += 2) {
        const int kc = kk + (lane >> 5);
        float am[2], bn[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          am[a] = Ts[wm * 64 + a * 32 + (lane & 31)][kc];
          bn[a] = Xs[wn * 64 + a * 32 + (lane & 31)][kc];
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int c = 0; c < 2; ++c)
            acc[a][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(am[a], bn[c], acc[a][c], 0, 0, 0);
      }
      __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int64_t row = tm * kT + wm * 64 + a * 32 + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
          const int64_t b = b0 + wn * 64 + c * 32 + (lane & 31);
          if (b < P) Y[blockIdx.z * sz + b * sv + row] = acc[a][c][i];
        }
  }
}

// Y[b][i] = sum over z < nzc of part[z][b][i], in order (vectors at stride sv).
__global__ __launch_bounds__(256) void k_trmm_sum(const float* __restrict__ part, int nzc, int64_t sz, int64_t n,
                                                  int64_t sv, float* __restrict__ Y) {
  const int64_t b = blockIdx.y, i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  float t = 0.0f;
  for (int z = 0; z < nzc; ++z) t += part[z * sz + b * sv + i];
  Y[b * sv + i] = t;
}

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
hipError_t gram(int mode, const void* hi, const void* lo, const float* xf, int64_t M, int64_t ld, const int64_t* xoff_d,
                const int64_t* xlen_d, const int64_t* xoff_h, const int64_t* xlen_h, int nb, float* K, int64_t ldk,
                int64_t sK, hipStream_t st, const uint64_t* nz, int64_t nzw, const uint64_t* nzl, const float* cs,
                int64_t scs) {
  if (mode == SW_GRAM_F32) {
    for (int b = 0; b < nb; ++b) {
      hipError_t e = gemm_nt_f32(M, M, xlen_h[b], 1.0f, xf + xoff_h[b], ld, 0, xf + xoff_h[b], ld, 0, 0.0f, K + b * sK,
                                 ldk, 0, true, 1, st);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  const int64_t nt = (M + kGT - 1) / kGT;
  const int64_t grid = super_grid(nt);
  if (mode == SW_GRAM_BF16X3) {
    hipLaunchKernelGGL(k_gram_bf16<true>, dim3((unsigned)grid, (unsigned)nb), dim3(kGThreads), 0, st,
                       (const __bf16*)hi, (const __bf16*)lo, xoff_d, xlen_d, ld, K, ldk, sK, M, nt, nz, nzw, nzl, cs,
                       scs);
  } else {
    hipLaunchKernelGGL(k_gram_bf16<false>, dim3((unsigned)grid, (unsigned)nb), dim3(kGThreads), 0, st,
                       (const __bf16*)hi, (const __bf16*)hi, xoff_d, xlen_d, ld, K, ldk, sK, M, nt, nz, nzw,
                       (const uint64_t*)nullptr, cs, scs);
  }
  return hipGetLastError();
}

int g_factor_x3 = 1;

hipError_t gemm_nt_f32(int64_t M, int64_t N, int64_t K, float alpha, const float* A, int64_t lda, int64_t sA,
                       const float* B, int64_t ldb, int64_t sB, float beta, float* C, int64_t ldc, int64_t sC,
                       bool lower, int nb, hipStream_t st, bool a_lower, bool x3) {
  const int64_t ntm = M / kT, ntn = N / kT;
  const int64_t n_tiles = lower ? ntm * (ntm + 1) / 2 : ntm * ntn;
  if (n_tiles == 0) return hipSuccess;
  const int64_t grid = (a_lower && !lower) ? kXcd * ((ntm + kXcd - 1) / kXcd) * ntn
                                           : ((n_tiles + kXcd - 1) / kXcd) * kXcd;
  hipLaunchKernelGGL(x3 ? k_gemm_nt_x3 : k_gemm_nt_f32, dim3((unsigned)grid, (unsigned)nb), dim3(kThreads), 0, st, ntn,
                     K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, lower ? 1 : 0, a_lower ? 1 : 0, n_tiles,
                     (int64_t)0, (int64_t)0);
  return hipGetLastError();
}

// Chunk length of the split-K product in the factor inversion: with row
// tiles of a lower-triangular M x M operand and ntn column tiles, about
// (M/128)^2 ntn 128 / (2 kc) chunks per problem; kc is chosen so that all nb
// problems together give a few thousand workgroups, and is at least 512.
// kc >= M means no split.
static int64_t split_kc(int64_t M, int64_t ntn, int nb) {
  const int64_t nt = M / kT;
  int64_t kc = (nt * nt * ntn * (int64_t)nb) / 32;
  kc = ((kc + 511) / 512) * 512;
  return kc < 512 ? 512 : kc;
}

static int64_t split_parts_floats(int64_t M, int64_t N, int nb) {
  const int64_t kc = split_kc(M, N / kT, nb);
  return kc >= M ? 0 : ((M + kc - 1) / kc) * M * N;
}

// X = W P^T for the factor inversion: W (M x M, lower triangular in 128-tiles),
// P (N x M), X (M x N, ld ldx), split over K into chunks reduced by k_sum_parts.
static hipError_t gemm_lower_split(int64_t M, int64_t N, const float* W, int64_t ldw, int64_t sW, const float* Pt,
                                   int64_t ldp, int64_t sPt, float* X, int64_t ldx, int64_t sX, float* parts,
                                   int64_t sParts, int nb, hipStream_t st) {
  const int64_t ntn = N / kT;
  const int64_t kc = split_kc(M, ntn, nb);
  const bool x3 = g_factor_x3 != 0;
  if (kc >= M) return gemm_nt_f32(M, N, M, 1.0f, W, ldw, sW, Pt, ldp, sPt, 0.0f, X, ldx, sX, false, nb, st, true, x3);
  const int64_t ntm = M / kT, n_tiles = ntm * ntn, nchunk = (M + kc - 1) / kc;
  const int64_t grid = kXcd * ((ntm + kXcd - 1) / kXcd) * ntn;
  hipLaunchKernelGGL(x3 ? k_gemm_nt_x3 : k_gemm_nt_f32, dim3((unsigned)grid, (unsigned)nb, (unsigned)nchunk),
                     dim3(kThreads), 0, st, ntn, M, 1.0f, W, ldw, sW, Pt, ldp, sPt, 0.0f, parts, N, sParts, 0, 1, n_tiles,
                     kc, M * N);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t nq = M * (N / 4);
  hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((nq + kThreads - 1) / kThreads), (unsigned)nb), dim3(kThreads), 0,
                     st, parts, M * N, sParts, M, N, M, kc, X, ldx, sX);
  return hipGetLastError();
}

// Blocked right-looking Cholesky with the trailing update deferred over a
// group of kCholGroup block columns: inside a group each block column is
// first brought up to date by the group's earlier panels (left-looking, a
// narrow product), then factorised; the rest of the matrix is updated once
// per group with a rank-(kCholGroup * 128) product, which reads and writes the
// trailing matrix kCholGroup times less often than one update per block.
static int kCholGroup = 8;

static hipError_t cholesky(float* K, int64_t n, int64_t ld, int64_t sK, float* dinv, int64_t sD, int nb_prob,
                           hipStream_t st, int* bad) {
  const int64_t nb = n / kNB;
  hipError_t e;
  for (int64_t j0 = 0; j0 < nb; j0 += kCholGroup) {
    const int64_t j1 = std::min(nb, j0 + (int64_t)kCholGroup);
    for (int64_t j = j0; j < j1; ++j) {
      float* Kjj = K + j * kNB * ld + j * kNB;
      if (j > j0) {
        // block column j (rows from its diagonal down) -= its rows of the group's panels times theirs
        const float* Pg = K + j * kNB * ld + j0 * kNB;
        e = gemm_nt_f32(n - j * kNB, kNB, (j - j0) * kNB, -1.0f, Pg, ld, sK, Pg, ld, sK, 1.0f, Kjj, ld, sK, false,
                        nb_prob, st, false, g_factor_x3 != 0);
        if (e != hipSuccess) return e;
      }
      hipLaunchKernelGGL(k_potrf_diag, dim3((unsigned)nb_prob), dim3(kPotrfThreads), 0, st, Kjj, ld, sK,
                         dinv + j * kNB * kNB, sD, bad);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      const int64_t rest = n - (j + 1) * kNB;
      if (rest == 0) break;
      float* Pj = K + (j + 1) * kNB * ld + j * kNB;  // panel below the diagonal block
      // L_panel = K_panel inv(L_jj)^T  (each workgroup owns its row block: in place)
      e = gemm_nt_f32(rest, kNB, kNB, 1.0f, Pj, ld, sK, dinv + j * kNB * kNB, kNB, sD, 0.0f, Pj, ld, sK, false,
                      nb_prob, st);
      if (e != hipSuccess) return e;
    }
    const int64_t rest = n - j1 * kNB;
    if (rest == 0) break;
    // trailing update K_22 -= L_g L_g^T over the group's panels (lower tiles)
    const float* Pg = K + j1 * kNB * ld + j0 * kNB;
    e = gemm_nt_f32(rest, rest, (j1 - j0) * kNB, -1.0f, Pg, ld, sK, Pg, ld, sK, 1.0f, K + j1 * kNB * ld + j1 * kNB, ld,
                    sK, true, nb_prob, st, false, g_factor_x3 != 0);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Factor inversion, column blocks from the right in groups J = [j0, j1) of
// kInvGroup blocks.  For j in J,
//   W_{>j,j} = -(W_{>j,T} L_{T,j} + W_{>j,(j,j1)} L_{(j,j1),j}) W_jj,
// T = the blocks right of the group (already final; W_{J,T} = 0).  The first
// product is formed for the whole group at once (a kInvGroup * 128 wide
// product that reads W_{T,T} once per group instead of once per block), the
// second block by block inside the group; the terms are the same as in one
// product per block, only summed in two parts.
static int kInvGroup = 8;

static int64_t inv_group(int64_t n) { return std::max<int64_t>(1, std::min<int64_t>(kInvGroup, n / kNB)); }

struct InvScratch {  // per-problem scratch of the factor inversion (floats)
  int64_t xg, pt, lt, dt, parts, total;
  InvScratch(int64_t n, int nb) {
    const int64_t G = inv_group(n), w = G * kNB;
    int64_t pmax = 0;  // the largest split-K partial set over the groups, as invert_factor forms them
    for (int64_t j1 = n / kNB; j1 > 0; j1 -= G) {
      const int64_t gw = (j1 - std::max<int64_t>(0, j1 - G)) * kNB, tn = n - j1 * kNB;
      if (tn > 0) pmax = std::max(pmax, split_parts_floats(tn, gw, nb));
    }
    xg = 0;
    pt = xg + n * w;
    lt = pt + w * n;
    dt = lt + kNB * w;
    parts = dt + kNB * kNB;
    total = parts + pmax;
  }
};

static hipError_t invert_factor(float* K, int64_t n, int64_t ld, int64_t sK, const float* dinv, int64_t sD, int nb_prob,
                                float* tmp, int64_t sT, hipStream_t st) {
  const int64_t nb = n / kNB, G = inv_group(n), w = G * kNB;
  const InvScratch L(n, nb_prob);
  float *XG = tmp + L.xg, *Pt = tmp + L.pt, *Lt = tmp + L.lt, *Dt = tmp + L.dt, *parts = tmp + L.parts;
  hipError_t e;
  hipLaunchKernelGGL(k_set_diag_inv, dim3((unsigned)nb, (unsigned)nb_prob), dim3(kThreads), 0, st, K, ld, sK, dinv, sD);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int64_t j1 = nb; j1 > 0; j1 -= G) {
    const int64_t j0 = std::max<int64_t>(0, j1 - G), gw = (j1 - j0) * kNB;
    const int64_t t0 = j1 * kNB, tn = n - t0;
    // rows of the group in XG start at zero (W_{J,T} = 0)
    const int64_t nz = gw * (gw / 4);
    hipLaunchKernelGGL(k_zero_block, dim3((unsigned)((nz + kThreads - 1) / kThreads), (unsigned)nb_prob),
                       dim3(kThreads), 0, st, XG + j0 * kNB * w, w, sT, gw, gw);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (tn > 0) {
      // XG[T rows, J cols] = W_{T,T} L_{T,J}
      hipLaunchKernelGGL(k_transpose, dim3((unsigned)(tn / kTT * (gw / kTT)), (unsigned)nb_prob), dim3(kThreads), 0,
                         st, K + t0 * ld + j0 * kNB, ld, sK, Pt, n, sT, (int64_t)(gw / kTT));
      if ((e = hipGetLastError()) != hipSuccess) return e;
      e = gemm_lower_split(tn, gw, K + t0 * ld + t0, ld, sK, Pt, n, sT, XG + t0 * w, w, sT, parts, sT, nb_prob, st);
      if (e != hipSuccess) return e;
    }
    for (int64_t j = j1 - 1; j >= j0; --j) {
      const int64_t r1 = (j + 1) * kNB, rest = n - r1;
      if (rest == 0) continue;
      float* C = XG + r1 * w + (j - j0) * kNB;  // rows > j of column block j of the group
      const int64_t kin = (j1 - j - 1) * kNB;
      if (kin > 0) {
        // C += W_{>j,(j,j1)} L_{(j,j1),j}
        hipLaunchKernelGGL(k_transpose, dim3((unsigned)(kin / kTT * (kNB / kTT)), (unsigned)nb_prob), dim3(kThreads),
                           0, st, K + r1 * ld + j * kNB, ld, sK, Lt, kin, sT, (int64_t)(kNB / kTT));
        if ((e = hipGetLastError()) != hipSuccess) return e;
        e = gemm_nt_f32(rest, kNB, kin, 1.0f, K + r1 * ld + r1, ld, sK, Lt, kin, sT, 1.0f, C, w, sT, false, nb_prob, st,
                        true, g_factor_x3 != 0);
        if (e != hipSuccess) return e;
      }
      hipLaunchKernelGGL(k_transpose, dim3((unsigned)((kNB / kTT) * (kNB / kTT)), (unsigned)nb_prob), dim3(kThreads),
                         0, st, dinv + j * kNB * kNB, (int64_t)kNB, sD, Dt, (int64_t)kNB, sT, (int64_t)(kNB / kTT));
      if ((e = hipGetLastError()) != hipSuccess) return e;
      // W_{>j,j} = -C W_jj
      e = gemm_nt_f32(rest, kNB, kNB, -1.0f, C, w, sT, Dt, kNB, sT, 0.0f, K + r1 * ld + j * kNB, ld, sK, false, nb_prob,
                      st);
      if (e != hipSuccess) return e;
    }
  }
  const int64_t t = n / kTT;
  hipLaunchKernelGGL(k_mirror_lower, dim3((unsigned)(t * (t + 1) / 2), (unsigned)nb_prob), dim3(kThreads), 0, st, K, ld,
                     sK);
  return hipGetLastError();
}

int64_t inverse_factor_scratch(int64_t n, int nb) { return InvScratch(n, nb).total; }

hipError_t spd_inverse_factor(float* S, int64_t n, int64_t ld, int64_t sK, float* dinv, int64_t sD, int nb,
                              float* tmp, int64_t sT, int* bad, hipStream_t st) {
  hipError_t e = cholesky(S, n, ld, sK, dinv, sD, nb, st, bad);
  if (e != hipSuccess) return e;
  return invert_factor(S, n, ld, sK, dinv, sD, nb, tmp, sT, st);
}

int trmm_parts(int64_t n, int P) {
  const int64_t wg = (n / kT + 1) / 2 * ((P + kT - 1) / kT);
  return (int)std::max<int64_t>(1, std::min<int64_t>(kTrmmMaxParts, (kTrmmWorkgroups + wg - 1) / wg));
}

hipError_t inv_apply_rhs(const float* S, int64_t n, int64_t ld, int P, const float* r, float* tmp, float* s,
                         int64_t sv, const double* act, int act_stride, float* part, hipStream_t st) {
  if (P < kTrmmMinRhs) return inv_apply(S, n, ld, 0, P, r, tmp, s, sv, act, act_stride, st);
  const int nzc = trmm_parts(n, P);
  const dim3 grid((unsigned)((n / kT + 1) / 2), (unsigned)((P + kT - 1) / kT), (unsigned)nzc);
  const int64_t sz = (int64_t)P * sv;
  if (nzc == 1) {
    hipLaunchKernelGGL(k_trmm_rhs<true>, grid, dim3(kThreads), 0, st, S, n, ld, r, tmp, sv, P, 1, sz);
    hipLaunchKernelGGL(k_trmm_rhs<false>, grid, dim3(kThreads), 0, st, S, n, ld, tmp, s, sv, P, 1, sz);
    return hipGetLastError();
  }
  const dim3 sgrid((unsigned)((n + 255) / 256), (unsigned)P);
  hipLaunchKernelGGL(k_trmm_rhs<true>, grid, dim3(kThreads), 0, st, S, n, ld, r, part, sv, P, nzc, sz);
  hipLaunchKernelGGL(k_trmm_sum, sgrid, dim3(256), 0, st, (const float*)part, nzc, sz, n, sv, tmp);
  hipLaunchKernelGGL(k_trmm_rhs<false>, grid, dim3(kThreads), 0, st, S, n, ld, tmp, part, sv, P, nzc, sz);
  hipLaunchKernelGGL(k_trmm_sum, sgrid, dim3(256), 0, st, (const float*)part, nzc, sz, n, sv, s);
  return hipGetLastError();
}

hipError_t inv_apply(const float* S, int64_t n, int64_t ld, int64_t sK, int nb_prob, const float* r, float* tmp,
                     float* s, int64_t sv, const double* act, int act_stride, hipStream_t st) {
  if (n % 16 == 0 && g_trmv_rows == 16) {
    const unsigned g = (unsigned)((n / 16 + kThreads / 64 - 1) / (kThreads / 64));
    hipLaunchKernelGGL(k_trmv16<true>, dim3(g, (unsigned)nb_prob), dim3(kThreads), 0, st, S, n, ld, sK, r, tmp, sv,
                       act, act_stride);
    hipLaunchKernelGGL(k_trmv16<false>, dim3(g, (unsigned)nb_prob), dim3(kThreads), 0, st, S, n, ld, sK, tmp, s, sv,
                       act, act_stride);
    return hipGetLastError();
  }
  const unsigned g = (unsigned)((n / 2 + kThreads / 64 - 1) / (kThreads / 64));
  hipLaunchKernelGGL(k_trmv<true>, dim3(g, (unsigned)nb_prob), dim3(kThreads), 0, st, S, n, ld, sK, r, tmp, sv, act,
                     act_stride);
  hipLaunchKernelGGL(k_trmv<false>, dim3(g, (unsigned)nb_prob), dim3(kThreads), 0, st, S, n, ld, sK, tmp, s, sv, act,
                     act_stride);
  return hipGetLastError();
}

}  // namespace sw
