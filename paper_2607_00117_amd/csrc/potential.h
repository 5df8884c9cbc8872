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
// Single-precision acceleration (fast path).
// ---------------------------------------------------------------------------
// lamw: warm-start state of the first bar component (< 0: none yet); a
// second bar component, if any, always starts cold.
// With LPO lanes per orbit every lane evaluates the analytic components in
// full (into g) and its share of every bar's quadrature nodes (into gb): the
// force is g + the sum of gb over the lane group.  With LPO = 1, gb is the
// whole bar force and the caller adds it.
template <int LPO = 1>
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
      default:
        break;
    }
  }
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

__device__ inline double phi_f64(const PotK& P, const double* xv) {
  const double x = xv[0], y = xv[1], z = xv[2];
  double s = 0.0;
  for (int i = 0; i < P.n_comp; ++i) {
    const CompK& C = P.comp[i];
    double v = 0.0;
    if (C.kind == SW_FERRERS2) ferrers_f64(C, P.gq64, P.gw64, x, y, z, &v, nullptr);
    else v = phi_analytic_f64(C, x, y, z);
    s = s + v;
  }
  return s;
}

// E_J = |p|^2/2 + Phi(x) - Omega (x p_y - y p_x)
__device__ inline double jacobi_f64(const PotK& P, const double* s6) {
  double kin = 0.5 * (s6[3] * s6[3] + s6[4] * s6[4] + s6[5] * s6[5]);
  double Lz = s6[0] * s6[4] - s6[1] * s6[3];
  return kin + phi_f64(P, s6) - P.omega * Lz;
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
template <typename T>
__device__ __forceinline__ void cells4(const PotK& P, const ObsK& O, const T* s6, int* mcell, int* kcell) {
  using Q = ObsT<T>;
  const T x = s6[0], y = s6[1], z = s6[2], px = s6[3], py = s6[4], pz = s6[5];
  const int ixp = bin1<T>(x, Q::lo(O, 0), Q::inv(O, 0), O.nx), ixm = bin1<T>(-x, Q::lo(O, 0), Q::inv(O, 0), O.nx);
  const int iyp = bin1<T>(y, Q::lo(O, 1), Q::inv(O, 1), O.ny), iym = bin1<T>(-y, Q::lo(O, 1), Q::inv(O, 1), O.ny);
  const int izp = bin1<T>(z, Q::lo(O, 2), Q::inv(O, 2), O.nz), izm = bin1<T>(-z, Q::lo(O, 2), Q::inv(O, 2), O.nz);
  const int ixs[4] = {ixp, ixp, ixm, ixm}, iys[4] = {iyp, iyp, iym, iym}, izs[4] = {izp, izm, izp, izm};
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
    kcell[c] = (ap < 0 || kv < 0) ? -1 : ap * O.nv + kv;
  }
}

}  // namespace sw
