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
// M = rows of K (multiple of 128); X has gram_rows(M) rows (bf16 modes: a
// multiple of 256, rows past M zero), ld = row stride of X; xoff/xlen given on
// the device (bf16 modes) and on the host (fp32 mode); K_b = K + b * sK.
inline int64_t gram_rows(int mode, int64_t M) { return mode == SW_GRAM_F32 ? M : (M + 255) / 256 * 256; }
hipError_t gram(int mode, const void* hi, const void* lo, const float* xf, int64_t M, int64_t ld, const int64_t* xoff_d,
                const int64_t* xlen_d, const int64_t* xoff_h, const int64_t* xlen_h, int nb, float* K, int64_t ldk,
                int64_t sK, hipStream_t st);

// C = beta C + alpha A B^T per problem (fp32 MFMA, fp32 accumulate).
// M, N, K multiples of 128 (K multiple of 32).  lower: only tiles with tile_m >= tile_n.
// a_lower: A is lower triangular in 128-tiles (row tile m reads k < 128 (m + 1) only).
hipError_t gemm_nt_f32(int64_t M, int64_t N, int64_t K, float alpha, const float* A, int64_t lda, int64_t sA,
                       const float* B, int64_t ldb, int64_t sB, float beta, float* C, int64_t ldc, int64_t sC,
                       bool lower, int nb, hipStream_t st, bool a_lower = false);

// Blocked right-looking Cholesky of each n x n (n multiple of 128) SPD matrix
// in the lower triangle of K_b (row-major, ld); the factor overwrites it and
// the inverses of its diagonal blocks go to dinv_b[n/128][128][128].
// bad: device int set to 1 when a pivot is not positive.
hipError_t cholesky(float* K, int64_t n, int64_t ld, int64_t sK, float* dinv, int64_t sD, int nb, hipStream_t st,
                    int* bad);

// Replaces the factor L_b (lower triangle of K_b, as left by cholesky) with
// S_b = W + W^T - diag(W), W = L_b^-1, filling the whole n x n buffer.
// Scratch per problem: Pt [128][n] (stride sPt), Xb [n][128] (sX), Dt [128][128] (sDt).
hipError_t invert_factor(float* K, int64_t n, int64_t ld, int64_t sK, const float* dinv, int64_t sD, int nb,
                         float* Pt, int64_t sPt, float* Xb, int64_t sX, float* Dt, int64_t sDt, hipStream_t st);

// s_b = (L_b L_b^T)^-1 r_b = W^T (W r_b) from S_b (fp32, vectors of length n at
// stride sv; tmp: scratch of the same shape).  Problems with act[b * act_stride]
// == 0 are skipped (act may be null).
hipError_t inv_apply(const float* S, int64_t n, int64_t ld, int64_t sK, int nb, const float* r, float* tmp, float* s,
                     int64_t sv, const double* act, int act_stride, hipStream_t st);

}  // namespace sw
