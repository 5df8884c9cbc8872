// Device-side potentials, forces, Jacobi energy and binning.
//
// Two evaluation paths:
//  * single precision (the fast path): hardware reciprocal / reciprocal
//    square root, the Ferrers bar by a 16-node Gauss-Legendre rule after the
//    change of variable u = lam + K (1/t^2 - 1), lam from a fixed number of
//    Newton steps on m^2(lam) = 1;
//  * double precision: IEEE square root and division, the analytic
//    components written operation for operation in the order of their
//    textbook formulas, the bar by a 32-node rule.  With contraction of
//    a*b+c disabled this path is deterministic to the last bit.
#pragma once
#include "common.h"

namespace sw {

__device__ __forceinline__ float rcpf_(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float rsqf_(float x) { return __builtin_amdgcn_rsqf(x); }

// ---------------------------------------------------------------------------
// Ferrers n = 2 bar.  With e_j = (a_j^2 + u) / K:
//   int (1 - m^2)^2 du / ((a_i^2 + u) Delta) = K^-3/2 sum_n W_n (1 - m_n^2)^2 / (e_i sqrt(e_x e_y e_z))
//   int (1 - m^2)^3 du / Delta               = K^-1/2 sum_n W_n (1 - m_n^2)^3 / sqrt(e_x e_y e_z)
// with m_n^2 = sum_j (x_j^2 / K) / e_j.  The scaling by K keeps every
// product in range for any radius.
// ---------------------------------------------------------------------------
constexpr int kNewton32 = 7;      // Newton steps from the left bracket
constexpr int kNewtonWarm32 = 3;  // Newton steps from the previous step's lam

// lam_io < 0: cold start from the left bracket max(0, r^2 - a_max^2).
// lam_io >= 0: warm start from that value (the root at the orbit's previous
// position); m^2(lam) is convex and decreasing, so a start right of the root
// lands left of it after one step and then rises monotonically.  lam_io
// returns the root found.
// With LPO > 1 lanes per orbit, lane `part` of the group takes the nodes
// n = part, part + LPO, ... and returns its share of the force (the shares
// add up across the group); every lane computes lam.
template <int LPO = 1>
__device__ __forceinline__ void ferrers_accel_f32(const CompK& C, const float* gq, const float* gw, float x,
                                                  float y, float z, float& gx, float& gy, float& gz,
                                                  float& lam_io, int part = 0) {
  const float A0 = C.f[0], A1 = C.f[1], A2 = C.f[2], Amin = C.f[3], kF = C.f[4], Amax = C.f[6];
  const float x2 = x * x, y2 = y * y, z2 = z * z;
  const bool cold = lam_io < 0.0f;
  float lam = cold ? fmaxf(0.0f, x2 + y2 + z2 - Amax) : lam_io;
  const int n_it = cold ? kNewton32 : kNewtonWarm32;
  for (int it = 0; it < n_it; ++it) {
    float i0 = rcpf_(A0 + lam), i1 = rcpf_(A1 + lam), i2 = rcpf_(A2 + lam);
    float t0 = x2 * i0, t1 = y2 * i1, t2 = z2 * i2;
    float f = (t0 + t1) + (t2 - 1.0f);
    float fp = t0 * i0 + t1 * i1 + t2 * i2;
    lam = fmaxf(0.0f, lam + f * rcpf_(fp));
  }
  lam_io = lam;
  const float K = Amin + lam;
  const float iK = rcpf_(K);
  const float D0 = (A0 + lam) * iK, D1 = (A1 + lam) * iK, D2 = (A2 + lam) * iK;
  const float xs = x2 * iK, ys = y2 * iK, zs = z2 * iK;
  float F0 = 0.0f, F1 = 0.0f, F2 = 0.0f;
#pragma unroll
  for (int m = 0; m < kGL32 / LPO; ++m) {
    // the node of this lane, chosen between uniform loads (no per-lane index)
    float q = gq[m * LPO], W = gw[m * LPO];
    if constexpr (LPO == 2) {
      q = part ? gq[m * LPO + 1] : q;
      W = part ? gw[m * LPO + 1] : W;
    }
    float e0 = D0 + q, e1 = D1 + q, e2 = D2 + q;
    float e12 = e1 * e2, e02 = e0 * e2, e01 = e0 * e1;
    float s = rsqf_(e0 * e12);
    float iP = s * s;
    float i0 = e12 * iP, i1 = e02 * iP, i2 = e01 * iP;
    float w = fmaxf(1.0f - (xs * i0 + ys * i1 + zs * i2), 0.0f);
    float c = W * (w * w) * s;
    F0 += c * i0;
    F1 += c * i1;
    F2 += c * i2;
  }
  const float sc = kF * iK * rsqf_(K);
  gx -= sc * x * F0;
  gy -= sc * y * F1;
  gz -= sc * z * F2;
}

// lam by Newton from the left bracket, converged in double precision.
__device__ __forceinline__ double ferrers_lambda_f64(const CompK& C, double x2, double y2, double z2) {
  const double A0 = C.c[0], A1 = C.c[1], A2 = C.c[2], Amax = C.c[6];
  double lam = fmax(0.0, x2 + y2 + z2 - Amax);
  for (int it = 0; it < 60; ++it) {
    double i0 = 1.0 / (A0 + lam), i1 = 1.0 / (A1 + lam), i2 = 1.0 / (A2 + lam);
    double t0 = x2 * i0, t1 = y2 * i1, t2 = z2 * i2;
    double f = t0 + t1 + t2 - 1.0;
    if (!(f > 0.0)) break;
    double fp = t0 * i0 + t1 * i1 + t2 * i2;
    double nl = lam + f / fp;
    if (!(nl > lam)) break;
    lam = nl;
  }
  return lam;
}

// Potential and acceleration of the bar in double precision (32 nodes).
__device__ inline void ferrers_f64(const CompK& C, const double* gq, const double* gw, double x, double y,
                                   double z, double* phi, double* g) {
  const double x2 = x * x, y2 = y * y, z2 = z * z;
  const double lam = ferrers_lambda_f64(C, x2, y2, z2);
  const double K = C.c[3] + lam;
  const double D0 = (C.c[0] + lam) / K, D1 = (C.c[1] + lam) / K, D2 = (C.c[2] + lam) / K;
  const double xs = x2 / K, ys = y2 / K, zs = z2 / K;
  double F0 = 0.0, F1 = 0.0, F2 = 0.0, Fp = 0.0;
  for (int n = 0; n < kGL64; ++n) {
    const double q = gq[n], W = gw[n];
    double e0 = D0 + q, e1 = D1 + q, e2 = D2 + q;
    double s = 1.0 / sqrt(e0 * e1 * e2);
    double w = 1.0 - (xs / e0 + ys / e1 + zs / e2);
    if (w < 0.0) w = 0.0;
    double c = W * w * w * s;
    F0 += c / e0;
    F1 += c / e1;
    F2 += c / e2;
    Fp += c * w;
  }
  const double sK = sqrt(K);
  if (phi) *phi = -C.c[5] * Fp / sK;
  if (g) {
    const double sc = C.c[4] / (K * sK);
    g[0] = g[0] - sc * x * F0;
    g[1] = g[1] - sc * y * F1;
    g[2] = g[2] - sc * z * F2;
  }
}

// ---------------------------------------------------------------------------
// Dehnen-Aly needle bars (Eq. 12, App. A).  The T3 or V4 parent potential
// -GM sum_n c_n(Z) R^-n (R^2 = x^2 + y^2 + Z^2, Z = a + zeta, zeta =
// sqrt(z^2 + b^2)) with each R^-n replaced by its convolution along x with
// the needle density f(s) = (1 + eta (1 - 2|s|/L)) / (2L):
//   I_n = int_{-L}^{L} f(s) D^-n/2 ds,  D = (x - s)^2 + c^2,  c^2 = y^2 + Z^2.
// Each half of the needle is integrated by Gauss-Legendre after
// s = x + c sinh u: then ds = c cosh u du and D = (c cosh u)^2, so the
// n = 2k + 1 integrand is f (c cosh u)^-2k, smooth where D^-n/2 is sharply
// peaked at s = x.  The nodes t on (0, 1) and weights w come from the bar
// rule (q = 1/t^2 - 1, W = 2 w / t^3).  Sums for k = 0 .. NK-1:
//   J_k = int f D^-(2k+1)/2 ds,  X_k = int f (x - s) D^-(2k+1)/2 ds.
// Derivatives: dI_n/dx = -n X_(n+2), dI_n/dy = -n y J_(n+2), dI_n/dZ = -n Z J_(n+2).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T asinh_(T v) {
  const T av = v < T(0) ? -v : v;
  const T r = log(av + sqrt(av * av + T(1)));
  return v < T(0) ? -r : r;
}
template <>
__device__ __forceinline__ float asinh_<float>(float v) {
  const float av = fabsf(v), q = av * av + 1.0f;
  const float r = __logf(av + q * rsqf_(q));
  return v < 0.0f ? -r : r;
}

template <typename T, int NK, int NG>
__device__ __forceinline__ void needle_sums(const T* gq, const T* gw, T x, T c, T L, T eta, T* J, T* X) {
#pragma unroll
  for (int k = 0; k < NK; ++k) { J[k] = T(0); X[k] = T(0); }
  const T ic = T(1) / c, i2L = T(1) / (T(2) * L), iL2 = T(2) / L;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const T ua = asinh_<T>(((h ? -L : T(0)) - x) * ic), ub = asinh_<T>(((h ? T(0) : L) - x) * ic);
    const T du = ub - ua;
    for (int j = 0; j < NG; ++j) {
      T t, w, e, ie;
      if constexpr (sizeof(T) == 4) {
        t = rsqf_(1.0f + gq[j]);
        e = __expf(ua + du * t);
        ie = rcpf_(e);
      } else {
        t = T(1) / sqrt(T(1) + gq[j]);
        e = exp(ua + du * t);
        ie = T(1) / e;
      }
      w = T(0.5) * gw[j] * (t * t * t);
      const T sh = T(0.5) * (e - ie), ch = T(0.5) * (e + ie);
      const T s = x + c * sh;
      const T as = s < T(0) ? -s : s;
      T p = du * w * ((T(1) + eta * (T(1) - as * iL2)) * i2L);
      const T cc = c * ch;
      T iD;
      if constexpr (sizeof(T) == 4) iD = rcpf_(cc * cc);
      else iD = T(1) / (cc * cc);
      const T dx = -c * sh;
#pragma unroll
      for (int k = 0; k < NK; ++k) {
        J[k] += p;
        X[k] += p * dx;
        p *= iD;
      }
    }
  }
}

// c_n and dc_n/dzeta (Z = a + zeta) of the parent, n = 2k + 1; NT terms
// (T3: 3, V4: 5)
template <typename T, int NT>
__device__ __forceinline__ void needle_coeffs(T a, T b2, T Z, T zeta, T* c, T* dc) {
  c[0] = T(1); dc[0] = T(0);
  if constexpr (NT == 3) {
    // T3: 1/R + a (Z - a/3)/R^3 + a^2 Z^2/R^5
    c[1] = a * (Z - a / T(3)); dc[1] = a;
    c[2] = a * a * Z * Z; dc[2] = T(2) * a * a * Z;
  } else {
    // V4: 1/R + (a (Z - 2a/5) + b^2/2)/R^3 + 3a (a Z (2Z - a)/5 + (b^2/2)(Z - a/5))/R^5
    //     + a^2 Z^2 (a Z + 3 b^2)/R^7 + 7 a^3 b^2 Z^4 / (2 zeta R^9)
    const T h = T(0.5) * b2;
    c[1] = a * (Z - T(0.4) * a) + h; dc[1] = a;
    c[2] = T(3) * a * (T(0.2) * a * Z * (T(2) * Z - a) + h * (Z - T(0.2) * a));
    dc[2] = T(3) * a * (T(0.2) * a * (T(4) * Z - a) + h);
    c[3] = a * a * Z * Z * (a * Z + T(3) * b2);
    dc[3] = T(3) * a * a * a * Z * Z + T(6) * a * a * b2 * Z;
    const T k9 = T(3.5) * a * a * a * b2, Z3 = Z * Z * Z, iz = T(1) / zeta;
    c[4] = k9 * Z3 * Z * iz;
    dc[4] = k9 * (T(4) * Z3 * iz - Z3 * Z * iz * iz);
  }
}

// potential (phi != null) and acceleration added into g (g != null) of one needle bar;
// K holds GM, a, b^2, L, eta (C.c or C.f)
template <typename T, int NT, int NG>
__device__ __forceinline__ void needle_bar(const T* K, const T* gq, const T* gw, T x, T y, T z, T* phi, T* g) {
  const T GM = K[0], a = K[1], b2 = K[2], L = K[3], eta = K[4];
  T zeta, c;
  if constexpr (sizeof(T) == 4) {
    const float izz = rsqf_(z * z + b2);
    zeta = (z * z + b2) * izz;
  } else {
    zeta = sqrt(z * z + b2);
  }
  const T Z = a + zeta;
  if constexpr (sizeof(T) == 4) {
    const float q = y * y + Z * Z;
    c = q * rsqf_(q);
  } else {
    c = sqrt(y * y + Z * Z);
  }
  T J[NT + 1], X[NT + 1], cf[NT], dcf[NT];
  needle_sums<T, NT + 1, NG>(gq, gw, x, c, L, eta, J, X);
  needle_coeffs<T, NT>(a, b2, Z, zeta, cf, dcf);
  if (phi) {
    T sp = T(0);
#pragma unroll
    for (int k = 0; k < NT; ++k) sp += cf[k] * J[k];
    *phi = -GM * sp;
  }
  if (g) {
    T sx = T(0), sy = T(0), sz = T(0);
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      const T n = T(2 * k + 1);
      sx += n * cf[k] * X[k + 1];
      sy += n * cf[k] * J[k + 1];
      sz += dcf[k] * J[k] - n * cf[k] * Z * J[k + 1];
    }
    g[0] -= GM * sx;
    g[1] -= GM * y * sy;
    g[2] += GM * sz * z / zeta;
  }
}

// ---------------------------------------------------------------------------
// Single-precision acceleration (fast path).
// ---------------------------------------------------------------------------
// lamw: warm-start state of the first bar component (< 0: none yet); a
// second bar component, if any, always starts cold.
// With LPO lanes per orbit every lane evaluates the analytic components in
// full (into g) and its share of every bar's quadrature nodes (into gb): the
// force is g + the sum of gb over the lane group.  With LPO = 1, gb is the
// whole bar force and the caller adds it.  NB: the potential may hold needle
// bars (their code is compiled in only then, so that it does not weigh on the
// registers of the kernels that integrate other potentials).
template <int LPO = 1, bool NB = false>
__device__ __forceinline__ void accel_f32(const PotK& P, float x, float y, float z, float& gx, float& gy,
                                          float& gz, float* gb, float& lamw, int part = 0) {
  gx = 0.0f; gy = 0.0f; gz = 0.0f;
  gb[0] = 0.0f; gb[1] = 0.0f; gb[2] = 0.0f;
  const int nc = P.n_comp;
  bool first_bar = true;
  for (int i = 0; i < nc; ++i) {
    const CompK& C = P.comp[i];
    switch (C.kind) {
      case SW_KEPLER: {
        float ir = rsqf_(x * x + y * y + z * z);
        float f = C.f[0] * ir * ir * ir;
        gx -= f * x; gy -= f * y; gz -= f * z;
        break;
      }
      case SW_ISOCHRONE: {
        float r2 = x * x + y * y + z * z;
        float u = C.f[2] + r2;
        float iu = rsqf_(u);
        float s = u * iu;
        float den = C.f[1] + s;
        float f = C.f[0] * rcpf_(den * den) * iu;
        gx -= f * x; gy -= f * y; gz -= f * z;
        break;
      }
      case SW_PLUMMER: {
        float id = rsqf_(x * x + y * y + z * z + C.f[1]);
        float f = C.f[0] * id * id * id;
        gx -= f * x; gy -= f * y; gz -= f * z;
        break;
      }
      case SW_MN: {
        float zz = z * z + C.f[2];
        float iz = rsqf_(zz);
        float s = C.f[1] + zz * iz;
        float iD = rsqf_(x * x + y * y + s * s);
        float f = C.f[0] * iD * iD * iD;
        gx -= f * x; gy -= f * y; gz -= f * z * s * iz;
        break;
      }
      case SW_NFW_Q: {
        float m2 = x * x + y * y + z * z * C.f[2];
        float im = rsqf_(m2);
        float xr = m2 * im * C.f[5];  // m / R_s
        // T(x) = ln(1+x)/x^2 - 1/(x(1+x)); dPhi/dm = G M_DM / R_s^2 * T(m / R_s)
        float T;
        if (xr < 0.1f) {
          T = 0.5f + xr * (-2.0f / 3 + xr * (0.75f + xr * (-0.8f + xr * (5.0f / 6 + xr * (-6.0f / 7 +
              xr * (0.875f + xr * (-8.0f / 9)))))));
        } else {
          float ix = rcpf_(xr);
          T = ix * (__logf(1.0f + xr) * ix - rcpf_(1.0f + xr));
        }
        float f = (m2 > 0.0f) ? C.f[4] * T * im : 0.0f;
        gx -= f * x; gy -= f * y; gz -= f * z * C.f[2];
        break;
      }
      case SW_DA_T3:
      case SW_DA_V4:
        if constexpr (NB) {
          float gg[3] = {0.0f, 0.0f, 0.0f};
          if (C.kind == SW_DA_T3) needle_bar<float, 3, kGL32>(C.f, P.gq32, P.gw32, x, y, z, nullptr, gg);
          else needle_bar<float, 5, kGL32>(C.f, P.gq32, P.gw32, x, y, z, nullptr, gg);
          gx += gg[0]; gy += gg[1]; gz += gg[2];
        }
        break;
      case SW_FERRERS2:
        if (first_bar) {
          ferrers_accel_f32<LPO>(C, P.gq32, P.gw32, x, y, z, gb[0], gb[1], gb[2], lamw, part);
          first_bar = false;
        } else {
          float cold = -1.0f;
          ferrers_accel_f32<LPO>(C, P.gq32, P.gw32, x, y, z, gb[0], gb[1], gb[2], cold, part);
        }
        break;
      default:
        break;
    }
  }
}

// ---------------------------------------------------------------------------
// Double-precision acceleration and potential.  The analytic components use
// exactly the operation order of their defining formulas.
// ---------------------------------------------------------------------------
template <bool NB = false>
__device__ inline void accel_f64(const PotK& P, const double* xv, double* g) {
  const double x = xv[0], y = xv[1], z = xv[2];
  g[0] = 0.0; g[1] = 0.0; g[2] = 0.0;
  for (int i = 0; i < P.n_comp; ++i) {
    const CompK& C = P.comp[i];
    switch (C.kind) {
      case SW_KEPLER: {
        double r2 = x * x + y * y + z * z;
        double r = sqrt(r2);
        double f = C.c[0] / (r2 * r);
        g[0] = g[0] - f * x; g[1] = g[1] - f * y; g[2] = g[2] - f * z;
        break;
      }
      case SW_ISOCHRONE: {
        double r2 = x * x + y * y + z * z;
        double s = sqrt(C.c[2] + r2);
        double den = C.c[1] + s;
        double f = C.c[0] / (den * den * s);
        g[0] = g[0] - f * x; g[1] = g[1] - f * y; g[2] = g[2] - f * z;
        break;
      }
      case SW_PLUMMER: {
        double r2 = x * x + y * y + z * z;
        double d2 = r2 + C.c[1];
        double d = sqrt(d2);
        double f = C.c[0] / (d2 * d);
        g[0] = g[0] - f * x; g[1] = g[1] - f * y; g[2] = g[2] - f * z;
        break;
      }
      case SW_MN: {
        double R2 = x * x + y * y;
        double zeta = sqrt(z * z + C.c[2]);
        double s = C.c[1] + zeta;
        double D2 = R2 + s * s;
        double D = sqrt(D2);
        double f = C.c[0] / (D2 * D);
        g[0] = g[0] - f * x; g[1] = g[1] - f * y; g[2] = g[2] - f * z * s / zeta;
        break;
      }
      case SW_NFW_Q: {
        double m = sqrt(x * x + y * y + z * z / C.c[3]);
        if (m == 0.0) break;
        double Rs = C.c[1];
        double dphidm = C.c[0] * (log1p(m / Rs) / (m * m) - 1.0 / (m * (Rs + m)));
        double f = dphidm / m;
        g[0] = g[0] - f * x; g[1] = g[1] - f * y; g[2] = g[2] - f * z / C.c[3];
        break;
      }
      case SW_FERRERS2:
        ferrers_f64(C, P.gq64, P.gw64, x, y, z, nullptr, g);
        break;
      case SW_DA_T3:
        if constexpr (NB) needle_bar<double, 3, kGL64>(C.c, P.gq64, P.gw64, x, y, z, nullptr, g);
        break;
      case SW_DA_V4:
        if constexpr (NB) needle_bar<double, 5, kGL64>(C.c, P.gq64, P.gw64, x, y, z, nullptr, g);
        break;
      default:
        break;
    }
  }
}

// potential of a needle bar in double precision (32-node rule per half)
__device__ inline double needle_phi_f64(const PotK& P, const CompK& C, double x, double y, double z) {
  double v = 0.0;
  if (C.kind == SW_DA_T3) needle_bar<double, 3, kGL64>(C.c, P.gq64, P.gw64, x, y, z, &v, nullptr);
  else needle_bar<double, 5, kGL64>(C.c, P.gq64, P.gw64, x, y, z, &v, nullptr);
  return v;
}

// Potential of one analytic (non-bar) component.
__device__ inline double phi_analytic_f64(const CompK& C, double x, double y, double z) {
  double v = 0.0;
  switch (C.kind) {
    case SW_KEPLER:
      v = -C.c[0] / sqrt(x * x + y * y + z * z);
      break;
    case SW_ISOCHRONE: {
      double r2 = x * x + y * y + z * z;
      v = -C.c[0] / (C.c[1] + sqrt(C.c[2] + r2));
      break;
    }
    case SW_PLUMMER: {
      double r2 = x * x + y * y + z * z;
      v = -C.c[0] / sqrt(r2 + C.c[1]);
      break;
    }
    case SW_MN: {
      double R2 = x * x + y * y;
      double zeta = sqrt(z * z + C.c[2]);
      double sm = C.c[1] + zeta;
      v = -C.c[0] / sqrt(R2 + sm * sm);
      break;
    }
    case SW_NFW_Q: {
      double m = sqrt(x * x + y * y + z * z / C.c[3]);
      v = (m == 0.0) ? -C.c[0] / C.c[1] : -C.c[0] * log1p(m / C.c[1]) / m;
      break;
    }
    default:
      break;
  }
  return v;
}

template <bool NB = false>
__device__ inline double phi_f64(const PotK& P, const double* xv) {
  const double x = xv[0], y = xv[1], z = xv[2];
  double s = 0.0;
  for (int i = 0; i < P.n_comp; ++i) {
    const CompK& C = P.comp[i];
    double v = 0.0;
    if (C.kind == SW_FERRERS2) ferrers_f64(C, P.gq64, P.gw64, x, y, z, &v, nullptr);
    else if (C.kind == SW_DA_T3 || C.kind == SW_DA_V4) {
      if constexpr (NB) v = needle_phi_f64(P, C, x, y, z);
    } else v = phi_analytic_f64(C, x, y, z);
    s = s + v;
  }
  return s;
}

// E_J = |p|^2/2 + Phi(x) - Omega (x p_y - y p_x)
template <bool NB = false>
__device__ inline double jacobi_f64(const PotK& P, const double* s6) {
  double kin = 0.5 * (s6[3] * s6[3] + s6[4] * s6[4] + s6[5] * s6[5]);
  double Lz = s6[0] * s6[4] - s6[1] * s6[3];
  return kin + phi_f64<NB>(P, s6) - P.omega * Lz;
}

// ---------------------------------------------------------------------------
// Jacobi energy for the drift check of the single-precision integrator, in
// double precision.  The bar uses that integrator's own 16-node rule (nodes
// and weights widened to double: a fixed rule, so E_J(t) and E_J(0) see the
// same quadrature), lam refined by two double Newton steps from the
// integrator's lam at the same point, and the hardware reciprocal square
// root refined by two Newton-Raphson steps; the analytic components are as
// in phi_f64.  Its error against phi_f64 is far below the drift it checks.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double rsq_f64(double v) {
  double y = __builtin_amdgcn_rsq(v);
  y = y * (1.5 - 0.5 * v * y * y);
  y = y * (1.5 - 0.5 * v * y * y);
  return y;
}

__device__ inline double ferrers_phi_drift(const CompK& C, const float* gq, const float* gw, double x, double y,
                                           double z, double lam) {
  const double x2 = x * x, y2 = y * y, z2 = z * z;
  for (int it = 0; it < 2; ++it) {
    const double i0 = 1.0 / (C.c[0] + lam), i1 = 1.0 / (C.c[1] + lam), i2 = 1.0 / (C.c[2] + lam);
    const double t0 = x2 * i0, t1 = y2 * i1, t2 = z2 * i2;
    const double f = t0 + t1 + t2 - 1.0;
    const double fp = t0 * i0 + t1 * i1 + t2 * i2;
    lam = fmax(0.0, lam + f / fp);
  }
  const double K = C.c[3] + lam, iK = 1.0 / K;
  const double D0 = (C.c[0] + lam) * iK, D1 = (C.c[1] + lam) * iK, D2 = (C.c[2] + lam) * iK;
  const double xs = x2 * iK, ys = y2 * iK, zs = z2 * iK;
  double Fp = 0.0;
  for (int n = 0; n < kGL32; ++n) {
    const double q = (double)gq[n], W = (double)gw[n];
    const double e0 = D0 + q, e1 = D1 + q, e2 = D2 + q;
    const double e12 = e1 * e2;
    const double sv = rsq_f64(e0 * e12);
    const double iP = sv * sv;
    const double w = fmax(1.0 - (xs * e12 + ys * e0 * e2 + zs * e0 * e1) * iP, 0.0);
    Fp += W * (w * w * w) * sv;
  }
  return -C.c[5] * Fp * rsq_f64(K);
}

template <bool NB = false>
__device__ inline double jacobi_f64_drift(const PotK& P, const double* s6, float lamw) {
  const double x = s6[0], y = s6[1], z = s6[2];
  double phi = 0.0;
  bool first_bar = true;
  for (int i = 0; i < P.n_comp; ++i) {
    const CompK& C = P.comp[i];
    double v;
    if (C.kind == SW_FERRERS2) {
      const double lam = (first_bar && lamw >= 0.0f) ? (double)lamw : ferrers_lambda_f64(C, x * x, y * y, z * z);
      first_bar = false;
      v = ferrers_phi_drift(C, P.gq32, P.gw32, x, y, z, lam);
    } else if (C.kind == SW_DA_T3 || C.kind == SW_DA_V4) {
      v = 0.0;
      if constexpr (NB) v = needle_phi_f64(P, C, x, y, z);
    } else {
      v = phi_analytic_f64(C, x, y, z);
    }
    phi = phi + v;
  }
  const double kin = 0.5 * (s6[3] * s6[3] + s6[4] * s6[4] + s6[5] * s6[5]);
  const double Lz = s6[0] * s6[4] - s6[1] * s6[3];
  return kin + phi - P.omega * Lz;
}

// ---------------------------------------------------------------------------
// Binning.  Contraction is disabled so that the decision is the same
// whether the values come from the integrator or from a test.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ int bin1(T v, T lo, T inv, int n) {
#pragma clang fp contract(off)
  T t = (v - lo) * inv;
  return (t >= T(0) && t < T(n)) ? (int)t : -1;
}

// Cylindrical mass grid (exact decisions; see sw_obs_spec): R bin k iff
// e_k^2 <= R^2 < e_(k+1)^2, e_k = lo + k w; sector k iff the point is on or
// counterclockwise of its lower edge and clockwise of its upper edge, the
// first such k, else the last sector.  A first guess from sqrt / atan2 is
// corrected by walking to the neighbour whose test holds.  Helpers without
// contraction of a*b+c.
template <typename T>
__device__ __forceinline__ T cyl_e2(T lo, T w, int k) {
#pragma clang fp contract(off)
  const T e = lo + (T)k * w;
  return e * e;
}
template <typename T>
__device__ __forceinline__ bool cyl_ccw(const T* c, const T* s, int k, T x, T y) {
#pragma clang fp contract(off)
  return c[k] * y - s[k] * x >= T(0);
}
template <typename T>
__device__ __forceinline__ int cyl_rbin(T R2, T lo, T w, T inv, int n) {
  if (R2 < cyl_e2<T>(lo, w, 0) || !(R2 < cyl_e2<T>(lo, w, n))) return -1;
  int k = (int)((sqrt(R2) - lo) * inv);
  k = k < 0 ? 0 : (k > n - 1 ? n - 1 : k);
  while (k > 0 && R2 < cyl_e2<T>(lo, w, k)) --k;
  while (k < n - 1 && !(R2 < cyl_e2<T>(lo, w, k + 1))) ++k;
  return k;
}
template <typename T>
__device__ __forceinline__ int cyl_sector(T x, T y, const T* c, const T* s, int n) {
  // Away from underflow every cross product with an edge that is not nearly
  // parallel to the point has its exact sign, so the edges counterclockwise
  // of the point form one arc: among sectors 0..n-2 at most one passes the
  // test, and the last sector competes with an earlier one only when edge 0
  // (the same direction as edge n) also passes.  The guess is walked to the
  // passing sector; tiny points, a failed test and that one case take the
  // scan in sector order.
  constexpr T kTiny = sizeof(T) == 8 ? T(0x1p-1000) : T(0x1p-100);
  int k = (int)((atan2(y, x) + T(M_PI)) * (T(n) / T(2.0 * M_PI)));
  k = k < 0 ? 0 : (k > n - 1 ? n - 1 : k);
  while (k > 0 && !cyl_ccw<T>(c, s, k, x, y)) --k;
  while (k < n - 1 && cyl_ccw<T>(c, s, k + 1, x, y)) ++k;
  const T ax = fabs(x), ay = fabs(y);
  if ((ax > ay ? ax : ay) < kTiny || !(cyl_ccw<T>(c, s, k, x, y) && !cyl_ccw<T>(c, s, k + 1, x, y)) ||
      (k == n - 1 && cyl_ccw<T>(c, s, 0, x, y))) {
    k = n - 1;
    for (int j = 0; j < n - 1; ++j)
      if (cyl_ccw<T>(c, s, j, x, y) && !cyl_ccw<T>(c, s, j + 1, x, y)) {
        k = j;
        break;
      }
  }
  return k;
}

template <typename T>
struct ObsT;
template <>
struct ObsT<float> {
  __device__ static float lo(const ObsK& O, int i) { return O.lof[i]; }
  __device__ static float inv(const ObsK& O, int i) { return O.invf[i]; }
  __device__ static float plo(const ObsK& O, int i) { return O.plof[i]; }
  __device__ static float pinv(const ObsK& O, int i) { return O.pinvf[i]; }
  __device__ static float vlo(const ObsK& O) { return O.vlof; }
  __device__ static float vinv(const ObsK& O) { return O.vinvf; }
  __device__ static float R(const PotK& P, int i) { return P.Rf[i]; }
  __device__ static float rw(const ObsK& O) { return O.rwf; }
  __device__ static const float* sc(const ObsK& O) { return O.scf; }
  __device__ static const float* ss(const ObsK& O) { return O.ssf; }
};
template <>
struct ObsT<double> {
  __device__ static double lo(const ObsK& O, int i) { return O.lo[i]; }
  __device__ static double inv(const ObsK& O, int i) { return O.inv[i]; }
  __device__ static double plo(const ObsK& O, int i) { return O.plo[i]; }
  __device__ static double pinv(const ObsK& O, int i) { return O.pinv[i]; }
  __device__ static double vlo(const ObsK& O) { return O.vlo; }
  __device__ static double vinv(const ObsK& O) { return O.vinv; }
  __device__ static double R(const PotK& P, int i) { return P.R[i]; }
  __device__ static double rw(const ObsK& O) { return O.rw; }
  __device__ static const double* sc(const ObsK& O) { return O.sc; }
  __device__ static const double* ss(const ObsK& O) { return O.ss; }
};

template <typename T>
__device__ __forceinline__ T proj3(T r0, T r1, T r2, T a, T b, T c) {
#pragma clang fp contract(off)
  return r0 * a + r1 * b + r2 * c;
}

// Cells of the four mirror copies (Table 1) of one bar-frame state.
// Copies: 0 (x,y,z), 1 (x,y,-z), 2 (-x,-y,z), 3 (-x,-y,-z), applied to
// position and velocity alike.  Projections of copies 2 and 3 are exactly
// the negations of copies 1 and 0 (IEEE rounding is sign-symmetric).
// mcell/kcell: -1 when outside the block.
// CYL: the mass grid is cylindrical (compiled in only for such grids: the
// sector tables are indexed at run time, which would weigh on the registers of
// the Cartesian kernels)
template <typename T, bool CYL = false>
__device__ __forceinline__ void cells4(const PotK& P, const ObsK& O, const T* s6, int* mcell, int* kcell) {
  using Q = ObsT<T>;
  const T x = s6[0], y = s6[1], z = s6[2], px = s6[3], py = s6[4], pz = s6[5];
  const int ixp = bin1<T>(x, Q::lo(O, 0), Q::inv(O, 0), O.nx), ixm = bin1<T>(-x, Q::lo(O, 0), Q::inv(O, 0), O.nx);
  const int iyp = bin1<T>(y, Q::lo(O, 1), Q::inv(O, 1), O.ny), iym = bin1<T>(-y, Q::lo(O, 1), Q::inv(O, 1), O.ny);
  const int izp = bin1<T>(z, Q::lo(O, 2), Q::inv(O, 2), O.nz), izm = bin1<T>(-z, Q::lo(O, 2), Q::inv(O, 2), O.nz);
  int ixs[4] = {ixp, ixp, ixm, ixm}, iys[4] = {iyp, iyp, iym, iym};
  const int izs[4] = {izp, izm, izp, izm};
  if constexpr (CYL) {
    // (R, phi, z): R is the same for the four copies, the sector of (-x, -y) is that of the opposite point
    T R2;
    {
#pragma clang fp contract(off)
      R2 = x * x + y * y;
    }
    const int ir = cyl_rbin<T>(R2, Q::lo(O, 0), Q::rw(O), Q::inv(O, 0), O.nx);
    const int sp = cyl_sector<T>(x, y, Q::sc(O), Q::ss(O), O.ny), sm = cyl_sector<T>(-x, -y, Q::sc(O), Q::ss(O), O.ny);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      ixs[c] = ir;
      iys[c] = c < 2 ? sp : sm;
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c)
    mcell[c] = (ixs[c] < 0 || iys[c] < 0 || izs[c] < 0) ? -1 : (ixs[c] * O.ny + iys[c]) * O.nz + izs[c];
  const T X0 = proj3<T>(Q::R(P, 0), Q::R(P, 1), Q::R(P, 2), x, y, z);
  const T Y0 = proj3<T>(Q::R(P, 3), Q::R(P, 4), Q::R(P, 5), x, y, z);
  const T V0 = proj3<T>(Q::R(P, 6), Q::R(P, 7), Q::R(P, 8), px, py, pz);
  const T X1 = proj3<T>(Q::R(P, 0), Q::R(P, 1), Q::R(P, 2), x, y, -z);
  const T Y1 = proj3<T>(Q::R(P, 3), Q::R(P, 4), Q::R(P, 5), x, y, -z);
  const T V1 = proj3<T>(Q::R(P, 6), Q::R(P, 7), Q::R(P, 8), px, py, -pz);
  const T Xs[4] = {X0, X1, -X1, -X0}, Ys[4] = {Y0, Y1, -Y1, -Y0}, Vs[4] = {V0, V1, -V1, -V0};
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    int jx = bin1<T>(Xs[c], Q::plo(O, 0), Q::pinv(O, 0), O.npx);
    int jy = bin1<T>(Ys[c], Q::plo(O, 1), Q::pinv(O, 1), O.npy);
    int kv = bin1<T>(Vs[c], Q::vlo(O), Q::vinv(O), O.nv);
    int ap = -1;
    if (jx >= 0 && jy >= 0) {
      int pix = jx * O.npy + jy;
      ap = O.pix2ap ? O.pix2ap[pix] : pix;
    }
    // with the surface block on, an event in an aperture outside the velocity
    // range keeps its aperture as code n_kin + ap (counted by that block only)
    kcell[c] = ap < 0 ? -1 : (kv >= 0 ? ap * O.nv + kv : (O.surface ? O.n_kin + ap : -1));
  }
}

}  // namespace sw
