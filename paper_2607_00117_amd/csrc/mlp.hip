// Surrogate MLP of chi^2(theta): 12 -> 256 -> 256 -> 256 -> 1, SiLU on the
// hidden layers.  Training kernels (forward with cached activations,
// backward, Adam) work in fp32; inference runs one fused kernel with bf16
// weights and fp32 accumulation.
//
// Parameter packing (fp32): [W1 (256x12), b1 (256), W2 (256x256), b2, W3 (256x256), b3, W4 (1x256), b4 (1)],
// weights row-major [out][in].
#include <hip/hip_runtime.h>

#include "common.h"

namespace sw {

constexpr int kIn = 12, kHid = 256;
constexpr int64_t kOffW1 = 0, kOffB1 = kOffW1 + kHid * kIn, kOffW2 = kOffB1 + kHid, kOffB2 = kOffW2 + kHid * kHid,
                  kOffW3 = kOffB2 + kHid, kOffB3 = kOffW3 + kHid * kHid, kOffW4 = kOffB3 + kHid,
                  kOffB4 = kOffW4 + kHid, kNParam = kOffB4 + 1;

__device__ __forceinline__ float sigmoidf_(float z) { return 1.0f / (1.0f + __expf(-z)); }

// ---------------------------------------------------------------------------
// Generic small GEMM with strided operands: C[m][n] = sum_k A(m,k) B(k,n),
// A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn], 64 x 64 tiles, 256
// threads computing 4 x 4 outputs each, k staged through LDS in chunks of 16.
// Epilogues:
//  EPI_LINEAR:  Z = acc + bias[n]; C = Z, C2 = silu(Z)         (forward layer)
//  EPI_PLAIN:   C = acc                                        (weight gradients)
//  EPI_DSILU:   C = acc * silu'(Z[m][n])                       (backprop through SiLU)
// ---------------------------------------------------------------------------
enum Epi { EPI_LINEAR = 0, EPI_PLAIN = 1, EPI_DSILU = 2 };

__global__ __launch_bounds__(256) void k_mlp_gemm(int M, int N, int K, const float* __restrict__ A, int64_t sam,
                                                  int64_t sak, const float* __restrict__ B, int64_t sbk, int64_t sbn,
                                                  float* __restrict__ C, float* __restrict__ C2, int64_t ldc,
                                                  const float* __restrict__ bias, const float* __restrict__ Z,
                                                  int epi) {
  __shared__ float As[16][64 + 1];
  __shared__ float Bs[16][64 + 1];
  const int tm = blockIdx.y * 64, tn = blockIdx.x * 64;
  const int tid = threadIdx.x;
  const int ty = tid / 16, tx = tid % 16;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int idx = tid; idx < 16 * 64; idx += 256) {
      const int kk = idx / 64, mm = idx % 64;
      const int m = tm + mm, k = k0 + kk;
      As[kk][mm] = (m < M && k < K) ? A[(int64_t)m * sam + (int64_t)k * sak] : 0.0f;
      const int n = tn + mm;
      Bs[kk][mm] = (n < N && k < K) ? B[(int64_t)k * sbk + (int64_t)n * sbn] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int m = tm + ty * 4 + i, n = tn + tx * 4 + j;
      if (m >= M || n >= N) continue;
      const int64_t at = (int64_t)m * ldc + n;
      if (epi == EPI_LINEAR) {
        const float z = acc[i][j] + (bias ? bias[n] : 0.0f);
        C[at] = z;
        if (C2) C2[at] = z * sigmoidf_(z);
      } else if (epi == EPI_PLAIN) {
        C[at] = acc[i][j];
      } else {
        const float z = Z[at];
        const float s = sigmoidf_(z);
        C[at] = acc[i][j] * (s * (1.0f + z * (1.0f - s)));
      }
    }
}

// column sums over the batch: out[n] = sum_m X[m][n]   (bias gradients)
__global__ void k_colsum_small(const float* __restrict__ X, int M, int N, float* __restrict__ out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.0f;
  for (int m = 0; m < M; ++m) s += X[(int64_t)m * N + n];
  out[n] = s;
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       int64_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_mse_grad(const float* __restrict__ y, const float* __restrict__ t, int64_t B,
                           float* __restrict__ dy) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < B) dy[i] = 2.0f * (y[i] - t[i]) / (float)B;
}

__global__ void k_to_bf16(const float* __restrict__ p, __bf16* __restrict__ q, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) q[i] = (__bf16)p[i];
}

// Fused bf16 inference: one workgroup of 256 threads carries 16 samples through
// every layer in LDS; thread t owns hidden unit t; weights bf16, sums fp32.
constexpr int kInferRows = 16;
__global__ __launch_bounds__(256) void k_mlp_infer_bf16(const __bf16* __restrict__ q, const float* __restrict__ x,
                                                        int64_t B, float* __restrict__ y) {
  __shared__ float h[2][kInferRows][kHid];
  __shared__ float xin[kInferRows][kIn];
  const int t = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * kInferRows;
  for (int idx = t; idx < kInferRows * kIn; idx += 256) {
    const int r = idx / kIn, c = idx % kIn;
    xin[r][c] = (r0 + r < B) ? x[(r0 + r) * kIn + c] : 0.0f;
  }
  __syncthreads();
  {  // layer 1
    float w[kIn];
    for (int c = 0; c < kIn; ++c) w[c] = (float)q[kOffW1 + t * kIn + c];
    const float bb = (float)q[kOffB1 + t];
    for (int r = 0; r < kInferRows; ++r) {
      float z = bb;
      for (int c = 0; c < kIn; ++c) z += w[c] * xin[r][c];
      h[0][r][t] = z * sigmoidf_(z);
    }
  }
  __syncthreads();
  int cur = 0;
  for (int layer = 0; layer < 2; ++layer) {
    const __bf16* W = q + (layer == 0 ? kOffW2 : kOffW3) + (int64_t)t * kHid;
    const float bb = (float)q[(layer == 0 ? kOffB2 : kOffB3) + t];
    float z[kInferRows];
    for (int r = 0; r < kInferRows; ++r) z[r] = bb;
    for (int c = 0; c < kHid; c += 8) {
      float wv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) wv[u] = (float)W[c + u];
      for (int r = 0; r < kInferRows; ++r)
#pragma unroll
        for (int u = 0; u < 8; ++u) z[r] += wv[u] * h[cur][r][c + u];
    }
    for (int r = 0; r < kInferRows; ++r) h[cur ^ 1][r][t] = z[r] * sigmoidf_(z[r]);
    __syncthreads();
    cur ^= 1;
  }
  // output layer: reduce over hidden units per sample (wave reductions)
  const float w4 = (float)q[kOffW4 + t];
  for (int r = 0; r < kInferRows; ++r) {
    float v = w4 * h[cur][r][t];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __shared__ float part[kInferRows][4];
    if ((t & 63) == 0) part[r][t >> 6] = v;
    __syncthreads();
    if (t == 0 && r0 + r < B) y[r0 + r] = part[r][0] + part[r][1] + part[r][2] + part[r][3] + (float)q[kOffB4];
    __syncthreads();
  }
}

static hipError_t gemm(int M, int N, int K, const float* A, int64_t sam, int64_t sak, const float* B, int64_t sbk,
                       int64_t sbn, float* C, float* C2, int64_t ldc, const float* bias, const float* Z, int epi,
                       hipStream_t st) {
  dim3 grid((N + 63) / 64, (M + 63) / 64);
  hipLaunchKernelGGL(k_mlp_gemm, grid, dim3(256), 0, st, M, N, K, A, sam, sak, B, sbk, sbn, C, C2, ldc, bias, Z, epi);
  return hipGetLastError();
}

// workspace: Z1, A1, Z2, A2, Z3, A3 ([B][256] each), dA and dZ scratch ([B][256] x 2)
static size_t act_bytes(int64_t B) { return (size_t)B * kHid * 4; }

}  // namespace sw

using namespace sw;

extern "C" int64_t mlp_param_count(void) { return kNParam; }

extern "C" size_t mlp_workspace_bytes(int64_t batch) { return batch > 0 ? 8 * act_bytes(batch) : 0; }

extern "C" int mlp_forward(const float* params, const float* x, int64_t B, float* y, void* workspace, size_t ws_bytes,
                           void* stream) {
  SW_CHECK(params && x && y && workspace, "mlp_forward: null argument");
  SW_CHECK(B > 0 && B < (1 << 30), "mlp_forward: bad batch");
  SW_CHECK(ws_bytes >= mlp_workspace_bytes(B), "mlp_forward: workspace too small");
  hipStream_t st = (hipStream_t)stream;
  float* ws = (float*)workspace;
  const int64_t S = B * kHid;
  float *Z1 = ws, *A1 = ws + S, *Z2 = ws + 2 * S, *A2 = ws + 3 * S, *Z3 = ws + 4 * S, *A3 = ws + 5 * S;
  const int b = (int)B;
  SW_HIP(gemm(b, kHid, kIn, x, kIn, 1, params + kOffW1, 1, kIn, Z1, A1, kHid, params + kOffB1, nullptr, EPI_LINEAR, st));
  SW_HIP(gemm(b, kHid, kHid, A1, kHid, 1, params + kOffW2, 1, kHid, Z2, A2, kHid, params + kOffB2, nullptr, EPI_LINEAR,
              st));
  SW_HIP(gemm(b, kHid, kHid, A2, kHid, 1, params + kOffW3, 1, kHid, Z3, A3, kHid, params + kOffB3, nullptr, EPI_LINEAR,
              st));
  SW_HIP(gemm(b, 1, kHid, A3, kHid, 1, params + kOffW4, 1, kHid, y, nullptr, 1, params + kOffB4, nullptr, EPI_LINEAR,
              st));
  return SW_OK;
}

// Gradients of sum_b dy[b] * y[b] with respect to the parameters, using the
// activations cached by mlp_forward on the same x and params.
extern "C" int mlp_backward(const float* params, const float* x, int64_t B, const float* dy, float* grad,
                            void* workspace, size_t ws_bytes, void* stream) {
  SW_CHECK(params && x && dy && grad && workspace, "mlp_backward: null argument");
  SW_CHECK(B > 0 && B < (1 << 30), "mlp_backward: bad batch");
  SW_CHECK(ws_bytes >= mlp_workspace_bytes(B), "mlp_backward: workspace too small");
  hipStream_t st = (hipStream_t)stream;
  float* ws = (float*)workspace;
  const int64_t S = B * kHid;
  float *Z1 = ws, *A1 = ws + S, *Z2 = ws + 2 * S, *A2 = ws + 3 * S, *Z3 = ws + 4 * S, *A3 = ws + 5 * S;
  float *dZa = ws + 6 * S, *dZb = ws + 7 * S;
  const int b = (int)B;
  // output layer: dW4[0][k] = sum_b dy[b] A3[b][k]; db4 = sum dy; dZ3 = dy W4 * silu'(Z3)
  SW_HIP(gemm(1, kHid, b, dy, 0, 1, A3, kHid, 1, grad + kOffW4, nullptr, kHid, nullptr, nullptr, EPI_PLAIN, st));
  hipLaunchKernelGGL(k_colsum_small, dim3(1), dim3(64), 0, st, dy, b, 1, grad + kOffB4);
  SW_HIP(gemm(b, kHid, 1, dy, 1, 1, params + kOffW4, 0, 1, dZa, nullptr, kHid, nullptr, Z3, EPI_DSILU, st));
  // layer 3: dW3 = dZ3^T A2, db3 = colsum dZ3, dZ2 = (dZ3 W3) * silu'(Z2)
  SW_HIP(gemm(kHid, kHid, b, dZa, 1, kHid, A2, kHid, 1, grad + kOffW3, nullptr, kHid, nullptr, nullptr, EPI_PLAIN, st));
  hipLaunchKernelGGL(k_colsum_small, dim3(1), dim3(256), 0, st, dZa, b, kHid, grad + kOffB3);
  SW_HIP(gemm(b, kHid, kHid, dZa, kHid, 1, params + kOffW3, kHid, 1, dZb, nullptr, kHid, nullptr, Z2, EPI_DSILU, st));
  // layer 2
  SW_HIP(gemm(kHid, kHid, b, dZb, 1, kHid, A1, kHid, 1, grad + kOffW2, nullptr, kHid, nullptr, nullptr, EPI_PLAIN, st));
  hipLaunchKernelGGL(k_colsum_small, dim3(1), dim3(256), 0, st, dZb, b, kHid, grad + kOffB2);
  SW_HIP(gemm(b, kHid, kHid, dZb, kHid, 1, params + kOffW2, kHid, 1, dZa, nullptr, kHid, nullptr, Z1, EPI_DSILU, st));
  // layer 1
  SW_HIP(gemm(kHid, kIn, b, dZa, 1, kHid, x, kIn, 1, grad + kOffW1, nullptr, kIn, nullptr, nullptr, EPI_PLAIN, st));
  hipLaunchKernelGGL(k_colsum_small, dim3(1), dim3(256), 0, st, dZa, b, kHid, grad + kOffB1);
  SW_HIP(hipGetLastError());
  return SW_OK;
}

extern "C" int mlp_adam_step(float* params, const float* grad, float* m, float* v, int64_t n, int32_t t, float lr,
                             float beta1, float beta2, float eps, void* stream) {
  SW_CHECK(params && grad && m && v, "mlp_adam_step: null argument");
  SW_CHECK(n > 0 && t >= 1, "mlp_adam_step: need n > 0 and t >= 1");
  const float c1 = 1.0f - powf(beta1, (float)t), c2 = 1.0f - powf(beta2, (float)t);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, params, grad, m, v,
                     n, lr, beta1, beta2, eps, c1, c2);
  SW_HIP(hipGetLastError());
  return SW_OK;
}

// dL/dy of L = mean_b (y_b - t_b)^2
extern "C" int mlp_mse_grad(const float* y, const float* t, int64_t B, float* dy, void* stream) {
  SW_CHECK(y && t && dy && B > 0, "mlp_mse_grad: bad argument");
  hipLaunchKernelGGL(k_mse_grad, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, (hipStream_t)stream, y, t, B, dy);
  SW_HIP(hipGetLastError());
  return SW_OK;
}

extern "C" int mlp_pack_bf16(const float* params, void* packed, void* stream) {
  SW_CHECK(params && packed, "mlp_pack_bf16: null argument");
  hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((kNParam + 255) / 256)), dim3(256), 0, (hipStream_t)stream, params,
                     (__bf16*)packed, kNParam);
  SW_HIP(hipGetLastError());
  return SW_OK;
}

extern "C" int mlp_infer_bf16(const void* packed, const float* x, int64_t B, float* y, void* stream) {
  SW_CHECK(packed && x && y, "mlp_infer_bf16: null argument");
  SW_CHECK(B >= 0, "mlp_infer_bf16: bad batch");
  if (B == 0) return SW_OK;
  hipLaunchKernelGGL(k_mlp_infer_bf16, dim3((unsigned)((B + kInferRows - 1) / kInferRows)), dim3(256), 0,
                     (hipStream_t)stream, (const __bf16*)packed, x, B, y);
  SW_HIP(hipGetLastError());
  return SW_OK;
}
