// MFMA kernels of the weight solve: the constraint-space Gram matrix, the
// fp32 GEMM used by the blocked Cholesky factorisation, the diagonal-block
// factor + inverse, and the blocked triangular solves.
//
// Tiling: a 256-thread workgroup (4 waves in a 2 x 2 grid) owns a 128 x 128
// output tile; each wave owns 64 x 64 = 2 x 2 blocks of the 32 x 32 MFMA
// output.  Operands are staged through LDS with row padding chosen so that
// the per-lane MFMA operand reads hit distinct banks.  Symmetric outputs
// launch only the tiles on or below the diagonal, and consecutive workgroup
// ids are spread so that each XCD (ids congruent mod 8) works on a
// contiguous run of tiles, which share operand panels in that XCD's L2.
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

// tile id -> (row tile, col tile) over the lower triangle, row-major
__device__ __forceinline__ void tri_tile(int64_t t, int64_t& tm, int64_t& tn) {
  int64_t m = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((m + 1) * (m + 2) / 2 <= t) ++m;
  while (m * (m + 1) / 2 > t) --m;
  tm = m;
  tn = t - m * (m + 1) / 2;
}

// ---------------------------------------------------------------------------
// Gram: K[m][n] = sum_k X[m][k] X[n][k], bf16 operands, fp32 accumulate.
// ---------------------------------------------------------------------------
constexpr int kBKb = 64;            // k per LDS stage (bf16)
constexpr int kPadB = kBKb + 8;     // padded row (elements): 144 B rows

template <bool X3>
__global__ __launch_bounds__(kThreads) void k_gram_bf16(const __bf16* __restrict__ hi, const __bf16* __restrict__ lo,
                                                        const int64_t* __restrict__ xoff, const int64_t* __restrict__ xlen,
                                                        int64_t ld, float* __restrict__ Kall, int64_t ldk, int64_t sK,
                                                        int64_t n_tiles) {
  const int64_t bp = blockIdx.y;
  const int64_t Kd = xlen[bp];
  hi += xoff[bp];
  lo += xoff[bp];
  float* __restrict__ K = Kall + bp * sK;
  __shared__ __attribute__((aligned(16))) __bf16 sm[X3 ? 4 : 2][kT][kPadB];
  const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
  if (t >= n_tiles) return;
  int64_t tm, tn;
  tri_tile(t, tm, tn);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  floatx16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.0f;

  const __bf16* src[4] = {hi + tm * kT * ld, hi + tn * kT * ld, lo + tm * kT * ld, lo + tn * kT * ld};
  constexpr int NM = X3 ? 4 : 2;
  uint4 reg[NM][4];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int mtx = 0; mtx < NM; ++mtx)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int idx = tid + kThreads * i;
        const int r = idx >> 3, c = (idx & 7) * 8;
        reg[mtx][i] = *reinterpret_cast<const uint4*>(src[mtx] + (int64_t)r * ld + k0 + c);
      }
  };
  gload(0);
  for (int64_t k0 = 0; k0 < Kd; k0 += kBKb) {
#pragma unroll
    for (int mtx = 0; mtx < NM; ++mtx)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int idx = tid + kThreads * i;
        const int r = idx >> 3, c = (idx & 7) * 8;
        *reinterpret_cast<uint4*>(&sm[mtx][r][c]) = reg[mtx][i];
      }
    __syncthreads();
    if (k0 + kBKb < Kd) gload(k0 + kBKb);
#pragma unroll
    for (int ks = 0; ks < kBKb / 16; ++ks) {
      const int kc = ks * 16 + 8 * (lane >> 5);
      bf16x8 am[2], bn[2], aml[2], bnl[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        am[a] = *reinterpret_cast<const bf16x8*>(&sm[0][wm * 64 + a * 32 + (lane & 31)][kc]);
        bn[a] = *reinterpret_cast<const bf16x8*>(&sm[1][wn * 64 + a * 32 + (lane & 31)][kc]);
        if constexpr (X3) {
          aml[a] = *reinterpret_cast<const bf16x8*>(&sm[2][wm * 64 + a * 32 + (lane & 31)][kc]);
          bnl[a] = *reinterpret_cast<const bf16x8*>(&sm[3][wn * 64 + a * 32 + (lane & 31)][kc]);
        }
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am[a], bn[b], acc[a][b], 0, 0, 0);
          if constexpr (X3) {
            acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am[a], bnl[b], acc[a][b], 0, 0, 0);
            acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aml[a], bn[b], acc[a][b], 0, 0, 0);
          }
        }
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
        K[row * ldk + col] = acc[a][b][i];
      }
}

// ---------------------------------------------------------------------------
// fp32 GEMM, C = beta C + alpha A B^T, MFMA 32x32x2 f32.
// ---------------------------------------------------------------------------
constexpr int kBKf = 32;
constexpr int kPadF = kBKf + 1;

__global__ __launch_bounds__(kThreads) void k_gemm_nt_f32(int64_t ntn, int64_t K, float alpha,
                                                          const float* __restrict__ A, int64_t lda, int64_t sA,
                                                          const float* __restrict__ B, int64_t ldb, int64_t sB,
                                                          float beta, float* __restrict__ C, int64_t ldc, int64_t sC,
                                                          int lower, int64_t n_tiles) {
  A += blockIdx.y * sA;
  B += blockIdx.y * sB;
  C += blockIdx.y * sC;
  __shared__ float As[kT][kPadF];
  __shared__ float Bs[kT][kPadF];
  const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
  if (t >= n_tiles) return;
  int64_t tm, tn;
  if (lower) tri_tile(t, tm, tn);
  else { tm = t / ntn; tn = t - tm * ntn; }
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
  gload(0);
  for (int64_t k0 = 0; k0 < K; k0 += kBKf) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int idx = tid + kThreads * i;
      const int r = idx >> 3, c = (idx & 7) * 4;
      As[r][c] = ra[i].x; As[r][c + 1] = ra[i].y; As[r][c + 2] = ra[i].z; As[r][c + 3] = ra[i].w;
      Bs[r][c] = rb[i].x; Bs[r][c + 1] = rb[i].y; Bs[r][c + 2] = rb[i].z; Bs[r][c + 3] = rb[i].w;
    }
    __syncthreads();
    if (k0 + kBKf < K) gload(k0 + kBKf);
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
// Diagonal block: unblocked Cholesky of the 128 x 128 block in LDS, then the
// inverse of the factor, one column per thread by forward substitution.
// A non-positive pivot sets *bad and is replaced by a tiny positive value so
// the factor stays finite.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_potrf_diag(float* __restrict__ Kd, int64_t ld, int64_t sK,
                                                         float* __restrict__ dinv, int64_t sD, int* __restrict__ bad) {
  Kd += blockIdx.x * sK;
  dinv += blockIdx.x * sD;
  __shared__ float a[kNB][kNB + 1];
  __shared__ float x[kNB][kNB + 1];
  const int tid = threadIdx.x;
  for (int idx = tid; idx < kNB * kNB; idx += kThreads) {
    const int i = idx / kNB, j = idx % kNB;
    a[i][j] = (j <= i) ? Kd[(int64_t)i * ld + j] : 0.0f;
  }
  __syncthreads();
  for (int k = 0; k < kNB; ++k) {
    if (tid == 0) {
      float p = a[k][k];
      if (!(p > 0.0f)) {
        atomicExch(bad, 1);
        p = 1e-30f;
      }
      a[k][k] = sqrtf(p);
    }
    __syncthreads();
    const float piv = a[k][k];
    for (int i = k + 1 + tid; i < kNB; i += kThreads) a[i][k] /= piv;
    __syncthreads();
    const int rem = kNB - 1 - k;
    for (int idx = tid; idx < rem * rem; idx += kThreads) {
      const int i = k + 1 + idx / rem, j = k + 1 + idx % rem;
      if (j <= i) a[i][j] -= a[i][k] * a[j][k];
    }
    __syncthreads();
  }
  if (tid < kNB) {
    const int c = tid;
    for (int i = 0; i < kNB; ++i) {
      float v;
      if (i < c) v = 0.0f;
      else if (i == c) v = 1.0f / a[c][c];
      else {
        float s = 0.0f;
        for (int k = c; k < i; ++k) s += a[i][k] * x[k][c];
        v = -s / a[i][i];
      }
      x[i][c] = v;
    }
  }
  __syncthreads();
  for (int idx = tid; idx < kNB * kNB; idx += kThreads) {
    const int i = idx / kNB, j = idx % kNB;
    Kd[(int64_t)i * ld + j] = (j <= i) ? a[i][j] : 0.0f;
    dinv[idx] = x[i][j];
  }
}

// ---------------------------------------------------------------------------
// Blocked triangular solves.  Step j of the forward solve: every workgroup
// forms z_j = inv(L_jj) r_j; workgroup 0 stores it, workgroup b >= 1 updates
// r_{j+b} -= L_{j+b,j} z_j.  The backward solve mirrors it with L^T.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_trsv_fwd(const float* __restrict__ L, int64_t ld, int64_t sK,
                                                       const float* __restrict__ dinv, int64_t sD, int64_t j,
                                                       float* __restrict__ r, float* __restrict__ z, int64_t sv) {
  __shared__ float rj[kNB], zj[kNB];
  L += blockIdx.y * sK;
  dinv += blockIdx.y * sD;
  r += blockIdx.y * sv;
  z += blockIdx.y * sv;
  const int tid = threadIdx.x;
  if (tid < kNB) rj[tid] = r[j * kNB + tid];
  __syncthreads();
  const int row = tid >> 1, half = tid & 1;
  const float* Dj = dinv + j * kNB * kNB;
  float s = 0.0f;
  for (int c = half * 64; c < half * 64 + 64; ++c) s += Dj[row * kNB + c] * rj[c];
  s += __shfl_xor(s, 1, 64);
  if (half == 0) zj[row] = s;
  __syncthreads();
  const int64_t b = blockIdx.x;
  if (b == 0) {
    if (tid < kNB) z[j * kNB + tid] = zj[tid];
    return;
  }
  const int64_t i = j + b;
  const float* Li = L + (i * kNB + row) * ld + j * kNB;
  float u = 0.0f;
  for (int c = half * 64; c < half * 64 + 64; ++c) u += Li[c] * zj[c];
  u += __shfl_xor(u, 1, 64);
  if (half == 0) r[i * kNB + row] -= u;
}

__global__ __launch_bounds__(kThreads) void k_trsv_bwd(const float* __restrict__ L, int64_t ld, int64_t sK,
                                                       const float* __restrict__ dinv, int64_t sD, int64_t j,
                                                       float* __restrict__ z, float* __restrict__ x, int64_t sv) {
  __shared__ float zj[kNB], xj[kNB];
  L += blockIdx.y * sK;
  dinv += blockIdx.y * sD;
  z += blockIdx.y * sv;
  x += blockIdx.y * sv;
  const int tid = threadIdx.x;
  if (tid < kNB) zj[tid] = z[j * kNB + tid];
  __syncthreads();
  const float* Dj = dinv + j * kNB * kNB;
  if (tid < kNB) {  // x_j = inv(L_jj)^T z_j
    float s = 0.0f;
    for (int c = tid; c < kNB; ++c) s += Dj[c * kNB + tid] * zj[c];
    xj[tid] = s;
  }
  __syncthreads();
  const int64_t b = blockIdx.x;
  if (b == 0) {
    if (tid < kNB) x[j * kNB + tid] = xj[tid];
    return;
  }
  const int64_t i = j - b;  // column block of L_{j,i}
  if (tid < kNB) {
    const int c = tid;
    float u = 0.0f;
    for (int rr = 0; rr < kNB; ++rr) u += L[(j * kNB + rr) * ld + i * kNB + c] * xj[rr];
    z[i * kNB + c] -= u;
  }
}

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
hipError_t gram(int mode, const void* hi, const void* lo, const float* xf, int64_t M, int64_t ld, const int64_t* xoff_d,
                const int64_t* xlen_d, const int64_t* xoff_h, const int64_t* xlen_h, int nb, float* K, int64_t ldk,
                int64_t sK, hipStream_t st) {
  if (mode == SW_GRAM_F32) {
    for (int b = 0; b < nb; ++b) {
      hipError_t e = gemm_nt_f32(M, M, xlen_h[b], 1.0f, xf + xoff_h[b], ld, 0, xf + xoff_h[b], ld, 0, 0.0f, K + b * sK,
                                 ldk, 0, true, 1, st);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  const int64_t nt = M / kT;
  const int64_t n_tiles = nt * (nt + 1) / 2;
  const int64_t grid = ((n_tiles + kXcd - 1) / kXcd) * kXcd;
  if (mode == SW_GRAM_BF16X3)
    hipLaunchKernelGGL(k_gram_bf16<true>, dim3((unsigned)grid, (unsigned)nb), dim3(kThreads), 0, st,
                       (const __bf16*)hi, (const __bf16*)lo, xoff_d, xlen_d, ld, K, ldk, sK, n_tiles);
  else
    hipLaunchKernelGGL(k_gram_bf16<false>, dim3((unsigned)grid, (unsigned)nb), dim3(kThreads), 0, st,
                       (const __bf16*)hi, (const __bf16*)hi, xoff_d, xlen_d, ld, K, ldk, sK, n_tiles);
  return hipGetLastError();
}

hipError_t gemm_nt_f32(int64_t M, int64_t N, int64_t K, float alpha, const float* A, int64_t lda, int64_t sA,
                       const float* B, int64_t ldb, int64_t sB, float beta, float* C, int64_t ldc, int64_t sC,
                       bool lower, int nb, hipStream_t st) {
  const int64_t ntm = M / kT, ntn = N / kT;
  const int64_t n_tiles = lower ? ntm * (ntm + 1) / 2 : ntm * ntn;
  if (n_tiles == 0) return hipSuccess;
  const int64_t grid = ((n_tiles + kXcd - 1) / kXcd) * kXcd;
  hipLaunchKernelGGL(k_gemm_nt_f32, dim3((unsigned)grid, (unsigned)nb), dim3(kThreads), 0, st, ntn, K, alpha, A, lda,
                     sA, B, ldb, sB, beta, C, ldc, sC, lower ? 1 : 0, n_tiles);
  return hipGetLastError();
}

hipError_t cholesky(float* K, int64_t n, int64_t ld, int64_t sK, float* dinv, int64_t sD, int nb_prob, hipStream_t st,
                    int* bad) {
  const int64_t nb = n / kNB;
  for (int64_t j = 0; j < nb; ++j) {
    float* Kjj = K + j * kNB * ld + j * kNB;
    hipLaunchKernelGGL(k_potrf_diag, dim3((unsigned)nb_prob), dim3(kThreads), 0, st, Kjj, ld, sK,
                       dinv + j * kNB * kNB, sD, bad);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t rest = n - (j + 1) * kNB;
    if (rest == 0) break;
    float* Pj = K + (j + 1) * kNB * ld + j * kNB;  // panel below the diagonal block
    // L_panel = K_panel inv(L_jj)^T  (each workgroup owns its row block: in place)
    e = gemm_nt_f32(rest, kNB, kNB, 1.0f, Pj, ld, sK, dinv + j * kNB * kNB, kNB, sD, 0.0f, Pj, ld, sK, false, nb_prob,
                    st);
    if (e != hipSuccess) return e;
    // trailing update K_22 -= L_panel L_panel^T (lower tiles)
    e = gemm_nt_f32(rest, rest, kNB, -1.0f, Pj, ld, sK, Pj, ld, sK, 1.0f, K + (j + 1) * kNB * ld + (j + 1) * kNB, ld,
                    sK, true, nb_prob, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t chol_solve(const float* L, int64_t n, int64_t ld, int64_t sK, const float* dinv, int64_t sD, int nb_prob,
                      float* r, float* tmp, float* s, int64_t sv, hipStream_t st) {
  const int64_t nb = n / kNB;
  for (int64_t j = 0; j < nb; ++j)
    hipLaunchKernelGGL(k_trsv_fwd, dim3((unsigned)(nb - j), (unsigned)nb_prob), dim3(kThreads), 0, st, L, ld, sK,
                       dinv, sD, j, r, tmp, sv);
  for (int64_t j = nb - 1; j >= 0; --j)
    hipLaunchKernelGGL(k_trsv_bwd, dim3((unsigned)(j + 1), (unsigned)nb_prob), dim3(kThreads), 0, st, L, ld, sK,
                       dinv, sD, j, tmp, s, sv);
  return hipGetLastError();
}

}  // namespace sw
