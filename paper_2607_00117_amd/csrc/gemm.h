// Dense linear-algebra kernels of the weight solve (internal interface).
// Every routine works on a batch of `nb` independent problems laid out with
// fixed strides (s*), launched together (grid.y or grid.x = problem).
#pragma once
#include "common.h"

namespace sw {

constexpr int kNB = 128;  // Cholesky / triangular-solve block size, also the GEMM tile

// Gram of the scaled orbit matrix held constraint-major: X[m][k] (k = orbit).
// Problem b uses columns [xoff[b], xoff[b] + xlen[b]) (xlen multiple of 64):
// K_b[m][n] = sum_k X[m][xoff_b + k] X[n][xoff_b + k] for tiles on or below the diagonal.
//  mode SW_GRAM_BF16:   X = hi (bf16)
//  mode SW_GRAM_BF16X3: X = hi + lo (bf16 pair), K ~ hi hi^T + hi lo^T + lo hi^T
//  mode SW_GRAM_F32:    X = xf (fp32)
// M = rows of K (multiple of 128); X has gram_rows(mode, M) rows (bf16 modes:
// a multiple of 256, rows past M zero) and ld columns (a multiple of 32);
// xoff/xlen given on the device (bf16 modes) and on the host (fp32 mode);
// K_b = K + b * sK.  fp32 mode: X row-major, entry (m, k) at m * ld + k.
// bf16 modes: X stage-blocked, entry (m, k) at gram_at(m, k, ld): the rows of a
// 256-row panel and the 32 columns of a stage form one contiguous 256 x 32
// row-major block, blocks in stage order within a panel, panels in row order.
inline int64_t gram_rows(int mode, int64_t M) { return mode == SW_GRAM_F32 ? M : (M + 255) / 256 * 256; }
__host__ __device__ inline int64_t gram_at(int64_t m, int64_t k, int64_t ld) {
  return (m >> 8) * 256 * ld + (k >> 5) * 8192 + (m & 255) * 32 + (k & 31);
}
// nz (bf16 modes, may be null): bit g of nz[t * nzw + g / 64] is set when rows
// [256 t, 256 t + 256) of X hold a nonzero in columns [32 g, 32 g + 32); the
// 32-column stages whose row or column panel is zero are skipped.
hipError_t gram(int mode, const void* hi, const void* lo, const float* xf, int64_t M, int64_t ld, const int64_t* xoff_d,
                const int64_t* xlen_d, const int64_t* xoff_h, const int64_t* xlen_h, int nb, float* K, int64_t ldk,
                int64_t sK, hipStream_t st, const uint64_t* nz = nullptr, int64_t nzw = 0,
                const uint64_t* nzl = nullptr, const float* cs = nullptr, int64_t scs = 0);

// C = beta C + alpha A B^T per problem (fp32 MFMA, fp32 accumulate).
// M, N, K multiples of 128 (K multiple of 32).  lower: only tiles with tile_m >= tile_n.
// a_lower: A is lower triangular in 128-tiles (row tile m reads k < 128 (m + 1) only).
// x3: the same product with the operands split into bf16 pairs (hi + lo) on
// bf16 MFMA, three products per pair (~2^-16 of each product dropped).
hipError_t gemm_nt_f32(int64_t M, int64_t N, int64_t K, float alpha, const float* A, int64_t lda, int64_t sA,
                       const float* B, int64_t ldb, int64_t sB, float beta, float* C, int64_t ldc, int64_t sC,
                       bool lower, int nb, hipStream_t st, bool a_lower = false, bool x3 = false);

// Cholesky factor L_b of each n x n (n multiple of 128) SPD matrix held in
// the lower triangle of S_b (row-major, ld): blocked right-looking, 128 x 128
// diagonal blocks factorised and inverted in LDS (inverses to dinv_b[n/128]
// [128][128] at stride sD), panels solved with those inverses and trailing
// updates by fp32 MFMA; then its inverse W = L_b^-1 column block by column
// block from the right, W_{>j,j} = -W_{>j,>j} L_{>j,j} inv(L_jj), which only
// ever multiplies by the inverse of one 128 x 128 block.  S_b ends as
// W + W^T - diag(W) over the whole buffer.  tmp: inverse_factor_scratch(n, nb)
// floats per problem at stride sT.  bad: device int set to 1 when a pivot is
// not positive (the factor stays finite).
int64_t inverse_factor_scratch(int64_t n, int nb);
hipError_t spd_inverse_factor(float* S, int64_t n, int64_t ld, int64_t sK, float* dinv, int64_t sD, int nb,
                              float* tmp, int64_t sT, int* bad, hipStream_t st);

// s_b = (L_b L_b^T)^-1 r_b = W^T (W r_b) from S_b (fp32, vectors of length n at
// stride sv; tmp: scratch of the same shape).  Problems with act[b * act_stride]
// == 0 are skipped (act may be null).
hipError_t inv_apply(const float* S, int64_t n, int64_t ld, int64_t sK, int nb, const float* r, float* tmp, float* s,
                     int64_t sv, const double* act, int act_stride, hipStream_t st);

// The same for P right-hand sides of one S (r, tmp, s: [P] vectors at stride
// sv): from kTrmmMinRhs of them on, two MFMA passes that read each half of S
// once for all of them (every right-hand side is computed, act is not read);
// below that, one matrix-vector pass per right-hand side.  The MFMA passes split
// each tile's column range into trmm_parts(n, P) parts when the tiles alone give
// fewer than kTrmmWorkgroups workgroups; part: trmm_parts(n, P) * P * sv floats
// for their partial sums (unused when that is 1).
constexpr int kTrmmMinRhs = 8;
constexpr int kTrmmWorkgroups = 512;
constexpr int kTrmmMaxParts = 32;
int trmm_parts(int64_t n, int P);
hipError_t inv_apply_rhs(const float* S, int64_t n, int64_t ld, int P, const float* r, float* tmp, float* s,
                         int64_t sv, const double* act, int act_stride, float* part, hipStream_t st);

}  // namespace sw
