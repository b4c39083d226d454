// Device helpers shared by the tendency kernels: reciprocal, the centred
// fourth-order interpolation and the five-point WENO reconstructions
// (finite-volume appendix of arXiv 2502.14148: upwind-biased WENO5 with the
// WENO-Z weights of Borges et al. 2008, q = 2; Jiang & Shu 1996 candidate
// stencils and smoothness indicators).
#pragma once

#include <hip/hip_runtime.h>

namespace oc {
namespace tz {

enum { SCHEME_NONE = 0, SCHEME_WENOZ = 1, SCHEME_LINEAR = 2 };

__device__ inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double rcp(double x) {
  // hardware estimate refined by two Newton steps (about 1 ulp)
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

template <class T>
__device__ inline T interp4(T a0, T a1, T a2, T a3) {
  return ((a1 + a2) * T(7) - (a0 + a3)) * T(1.0 / 12.0);
}

// Reconstruction at the interface between q_{-1} and q_0 from the six values
// q_{-3..2}; `vel` selects the upwind side.
template <class T, int SCHEME>
__device__ inline T rec6(T m3, T m2, T m1, T p0, T p1, T p2, T vel, T eps) {
  const bool pos = vel > T(0);
  const T a = pos ? m3 : p2;
  const T b = pos ? m2 : p1;
  const T c = pos ? m1 : p0;
  const T d = pos ? p0 : m1;
  const T e = pos ? p1 : m2;
  if (SCHEME == SCHEME_LINEAR)
    return (T(2) * a - T(13) * b + T(47) * c + T(27) * d - T(3) * e) * T(1.0 / 60.0);
  const T r0 = T(2) * a - T(7) * b + T(11) * c;
  const T r1 = -b + T(5) * c + T(2) * d;
  const T r2 = T(2) * c + T(5) * d - e;
  const T t0 = a - T(2) * b + c, u0 = a - T(4) * b + T(3) * c;
  const T t1 = b - T(2) * c + d, u1 = b - d;
  const T t2 = c - T(2) * d + e, u2 = T(3) * c - T(4) * d + e;
  const T b0 = T(13.0 / 12.0) * t0 * t0 + T(0.25) * u0 * u0;
  const T b1 = T(13.0 / 12.0) * t1 * t1 + T(0.25) * u1 * u1;
  const T b2 = T(13.0 / 12.0) * t2 * t2 + T(0.25) * u2 * u2;
  const T tau = fabs(b0 - b2);
  const T q0 = tau * rcp(b0 + eps), q1 = tau * rcp(b1 + eps), q2 = tau * rcp(b2 + eps);
  const T w0 = T(0.1) * (T(1) + q0 * q0);
  const T w1 = T(0.6) * (T(1) + q1 * q1);
  const T w2 = T(0.3) * (T(1) + q2 * q2);
  return (w0 * r0 + w1 * r1 + w2 * r2) * rcp(T(6) * (w0 + w1 + w2));
}

}  // namespace tz
}  // namespace oc
