// Matern covariance (paper eq. 3) and its theta-derivatives on the device.
//
//   Sigma(r) = sigma2 c(nu) x^nu K_nu(x),   x = r / beta,   c(nu) = 2^(1-nu) / Gamma(nu)
//
// K_nu comes from its integral form  K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt
// (DLMF 10.32.9), evaluated as  e^-x * T(x)  with the trapezoidal rule
//   T(x) = h [ f(0)/2 + sum_{k>=1} f(k h) ],  f(t) = exp(-x (cosh t - 1)) cosh(nu t),
// which converges geometrically in 1/h for this analytic, doubly decaying
// integrand (Trefethen & Weideman, SIAM Review 56, 2014).  The step depends on
// x through 10 buckets, h_m = 0.1 * 2^(-m/2) for x <= 9 * 2^m (h <= 0.3/sqrt(x)),
// and the sum stops once x (cosh t - 1) - nu t > 45 (terms below e^-45 of the
// first one); relative error below 1e-14 for nu up to 15 and x in [1e-12, 700]
// (checked against 30-digit values).  The same exponentials give K_{nu-1} (weight cosh((nu-1) t)) and
// dK_nu/dnu (weight t sinh(nu t), the nu-derivative of the integrand), so one
// set of exp() calls serves all three derivatives:
//   dSigma/dsigma2 = Sigma / sigma2
//   dSigma/dbeta   = sigma2 c x^(nu+1) K_{nu-1}(x) / beta        (DLMF 10.29.4, 10.27.3)
//   dSigma/dnu     = Sigma (-ln 2 - psi(nu) + ln x) + sigma2 c x^nu dK_nu/dnu(x)
// Sigma(0) = sigma2 and every nu- or beta-derivative vanishes at r = 0; for
// x > 700 the covariance is below 1e-250 and is returned as 0.
//
// Per-entry evaluation does not run the quadrature: for each theta the three
// smooth, positive functions of s = ln x
//   u0 = x^nu e^x K_nu(x),  u1 = x^(nu+1) e^x K_{nu-1}(x),  u2 = x^nu e^x dK_nu/dnu(x)
// are sampled by the quadrature at the 13 Chebyshev points of each of 119
// segments of width 1/4 covering ln x in [-23, ln 700]; on each segment
// u = u(centre) exp(p(t)) with p the degree-12 Chebyshev interpolant of
// ln(u / u(centre)) (Clenshaw's recurrence).  In s the logarithms are analytic
// in the strip |Im s| < pi/2 (K_nu has no zeros or singularities for Re x > 0)
// and nearly linear, so on a segment of half-width 1/8 the interpolant is
// exact to rounding, and interpolating relative to the centre keeps the
// rounding of large logarithms out (checked against 30-digit values: below
// 5e-14 relative for nu up to 15).  x below e^-23 falls back to the quadrature.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace exg {

constexpr int QNB = 10;     // step buckets
constexpr int QNK = 400;    // nodes per bucket (reaches t = 39.9 at h = 0.1)
constexpr int QW = 5;       // per node: cosh t - 1, t, w0, w1, w2
constexpr double QCUT = 45.0;
constexpr double XMAX = 700.0;
// Chebyshev tables, stored after the quadrature nodes in the same array
constexpr int CH_N = 13;          // points per segment (degree 12)
constexpr int CH_NSEG = 119;      // segments of ln x
constexpr int CH_STRIDE = 48;     // doubles per segment: 3 functions x 16 (13 coefficients, centre value)
constexpr int CH_MID = 6;         // the middle Chebyshev point, t = 0
constexpr double CH_SLO = -23.0;  // ln x of the first segment's left end
constexpr double CH_DS = 0.25;    // segment width in ln x
constexpr int QT_CHEB_OFF = QNB * QNK * QW;
constexpr int QT_TOTAL = QT_CHEB_OFF + CH_NSEG * CH_STRIDE;

// per-theta constants written by the table kernel
enum { C_S2 = 0, C_BETA, C_NU, C_C, C_PSI, C_S2C, C_METRIC, C_NUG, C_COUNT = 8 };

constexpr double EARTH_RADIUS_KM = 6371.0;

// distance between two locations: Euclidean, or (cst[C_METRIC] = 1) the
// great-circle distance in km between (longitude, latitude) pairs in degrees
// by the haversine formula
__device__ __forceinline__ double loc_dist(double x1, double y1, double x2, double y2, const double* __restrict__ cst) {
  if (cst[C_METRIC] == 0.0) {
    const double dx = x1 - x2, dy = y1 - y2;
    return sqrt(dx * dx + dy * dy);
  }
  const double d2r = 3.14159265358979323846 / 180.0;
  const double sp = sin(0.5 * (y2 - y1) * d2r), sl = sin(0.5 * (x2 - x1) * d2r);
  const double a = sp * sp + cos(y1 * d2r) * cos(y2 * d2r) * sl * sl;
  return 2.0 * EARTH_RADIUS_KM * asin(fmin(1.0, sqrt(a)));
}

__device__ __forceinline__ int quad_bucket(double x) {
  if (x <= 9.0) return 0;
  int m = (int)ceil(log2(x * (1.0 / 9.0)));
  return m < QNB - 1 ? m : QNB - 1;
}

// T0 = e^x K_nu(x)
__device__ __forceinline__ double quad_k0(const double* __restrict__ qt, double x, double nu) {
  const double* q = qt + quad_bucket(x) * QNK * QW;
  double s = 0.0;
  for (int k = 0; k < QNK; ++k, q += QW) {
    const double c = q[0];
    if (k > 0 && x * c - nu * q[1] > QCUT) break;
    s += exp(-x * c) * q[2];
  }
  return s;
}

// (e^x K_nu, e^x K_{nu-1}, e^x dK_nu/dnu)
__device__ __forceinline__ void quad_k3(const double* __restrict__ qt, double x, double nu, double* s0, double* s1,
                                        double* s2) {
  const double* q = qt + quad_bucket(x) * QNK * QW;
  double a = 0.0, b = 0.0, c2 = 0.0;
  for (int k = 0; k < QNK; ++k, q += QW) {
    const double c = q[0];
    if (k > 0 && x * c - nu * q[1] > QCUT + 5.0) break;
    const double e = exp(-x * c);
    a += e * q[2];
    b += e * q[3];
    c2 += e * q[4];
  }
  *s0 = a;
  *s1 = b;
  *s2 = c2;
}

// sum_k c_k T_k(t) - c_0 / 2 (Clenshaw)
__device__ __forceinline__ double cheb_eval(const double* __restrict__ c, double t) {
  double b1 = 0.0, b2 = 0.0;
  const double t2 = 2.0 * t;
#pragma unroll
  for (int k = CH_N - 1; k >= 1; --k) {
    const double b0 = fma(t2, b1, c[k] - b2);
    b2 = b1;
    b1 = b0;
  }
  return fma(t, b1, 0.5 * c[0] - b2);
}

// segment and local coordinate t in [-1, 1] of ln x; false below the table
__device__ __forceinline__ bool cheb_locate(double x, int* seg, double* t) {
  const double s = log(x) - CH_SLO;
  if (!(s >= 0.0)) return false;
  int j = (int)(s * (1.0 / CH_DS));
  j = j < CH_NSEG - 1 ? j : CH_NSEG - 1;
  *seg = j;
  *t = (s - j * CH_DS) * (2.0 / CH_DS) - 1.0;
  return true;
}

__device__ __forceinline__ double matern_value(double r, const double* __restrict__ cst, const double* __restrict__ qt) {
  if (r == 0.0) return cst[C_S2];
  const double x = r / cst[C_BETA];
  if (x > XMAX) return 0.0;
  int seg;
  double t;
  if (cheb_locate(x, &seg, &t)) {
    const double* c = qt + QT_CHEB_OFF + seg * CH_STRIDE;
    return cst[C_S2C] * exp(-x) * (c[CH_N] * exp(cheb_eval(c, t)));
  }
  const double nu = cst[C_NU];
  return cst[C_S2C] * pow(x, nu) * exp(-x) * quad_k0(qt, x, nu);
}

// d[0..2] = dSigma/d(sigma2, beta, nu) at distance r
__device__ __forceinline__ void matern_grad(double r, const double* __restrict__ cst, const double* __restrict__ qt,
                                            double* d0, double* d1, double* d2) {
  if (r == 0.0) {
    *d0 = 1.0;
    *d1 = 0.0;
    *d2 = 0.0;
    return;
  }
  const double beta = cst[C_BETA];
  const double x = r / beta;
  if (x > XMAX) {
    *d0 = 0.0;
    *d1 = 0.0;
    *d2 = 0.0;
    return;
  }
  const double nu = cst[C_NU];
  int seg;
  double t;
  if (cheb_locate(x, &seg, &t)) {
    const double* c = qt + QT_CHEB_OFF + seg * CH_STRIDE;
    const double E = cst[C_S2C] * exp(-x);
    const double sig = E * (c[CH_N] * exp(cheb_eval(c, t)));
    *d0 = sig / cst[C_S2];
    *d1 = E * (c[16 + CH_N] * exp(cheb_eval(c + 16, t))) / beta;
    *d2 = sig * (-0.69314718055994530942 - cst[C_PSI] + log(x)) + E * (c[32 + CH_N] * exp(cheb_eval(c + 32, t)));
    return;
  }
  double t0, t1, t2;
  quad_k3(qt, x, nu, &t0, &t1, &t2);
  const double P = cst[C_S2C] * pow(x, nu) * exp(-x);
  const double sig = P * t0;
  *d0 = sig / cst[C_S2];
  *d1 = P * x * t1 / beta;
  *d2 = sig * (-0.69314718055994530942 - cst[C_PSI] + log(x)) + P * t2;
}

}  // namespace exg
