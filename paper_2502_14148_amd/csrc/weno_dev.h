// Device helpers shared by the tendency kernels: reciprocal, the centred
// interpolations of the advecting velocity and the WENO reconstructions of
// orders 5, 7 and 9
// (finite-volume appendix of arXiv 2502.14148: upwind-biased WENO5 with the
// WENO-Z weights of Borges et al. 2008, q = 2; Jiang & Shu 1996 candidate
// stencils and smoothness indicators).
#pragma once

#include <hip/hip_runtime.h>

#include "weno_coeffs.h"

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

// Centred reconstruction of order 2R - 2 at the midpoint of a[R-2] and
// a[R-1] from a[0 .. 2R-3] (order 4: interp4).
template <class T, int R>
__device__ inline T interpc(const T* a) {
  if constexpr (R == 3) {
    return interp4(a[0], a[1], a[2], a[3]);
  } else {
    using C = WenoCoef<R>;
    T s = T(0);
#pragma unroll
    for (int o = 0; o < R - 1; ++o) s += T(C::centred[o]) * (a[o] + a[2 * R - 3 - o]);
    return s;
  }
}

// Reconstruction of order 2R - 1 (R = 4, 5) at the interface between q[R-1]
// and q[R] from q[0 .. 2R-1]; `vel` selects the upwind side.  Every
// combination is taken on deviations from the upwind neighbour of the
// interface, and the indicators on differences of neighbouring values, so
// that a large mean of the data does not cost precision.
// A value the optimiser cannot trace back to the load that produced it: a
// choice between two elements of a register array stays a choice between
// two values instead of becoming a dynamically indexed array access.
template <class T>
__device__ inline T opaque(T x) {
  asm("" : "+v"(x));
  return x;
}

template <class T, int SCHEME, int R>
__device__ inline T recw(const T* q, T vel, T eps) {
  using C = WenoCoef<R>;
  constexpr int N = 2 * R - 1;
  const bool pos = vel > T(0);
  T v[N];
#pragma unroll
  for (int t = 0; t < N; ++t) {
    const T a = opaque(q[t]), b = opaque(q[2 * R - 1 - t]);
    v[t] = pos ? a : b;
  }
  const T base = v[R - 1];
  T dv[N];
#pragma unroll
  for (int t = 0; t < N; ++t) dv[t] = v[t] - base;
  if constexpr (SCHEME == SCHEME_LINEAR) {
    T s = T(0);
#pragma unroll
    for (int t = 0; t < N; ++t)
      if (t != R - 1) s += T(C::full[t]) * dv[t];
    return base + s;
  } else {
    T dl[N - 1];
#pragma unroll
    for (int t = 0; t < N - 1; ++t) dl[t] = v[t + 1] - v[t];
    T beta[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      T b = T(0);
#pragma unroll
      for (int m = 0; m < R - 1; ++m) {
        T y = dl[k + m];
#pragma unroll
        for (int t = m + 1; t < R - 1; ++t) y += T(C::Lt[k][m][t]) * dl[k + t];
        b += T(C::D[k][m]) * y * y;
      }
      beta[k] = b;
    }
    T tau = T(0);
#pragma unroll
    for (int k = 0; k < R; ++k) tau += T(C::tau[k]) * beta[k];
    tau = fabs(tau);
    T num = T(0), den = T(0);
#pragma unroll
    for (int k = 0; k < R; ++k) {
      T rk = T(0);
#pragma unroll
      for (int t = 0; t < R; ++t)
        if (k + t != R - 1) rk += T(C::cand[k][t]) * dv[k + t];
      const T qk = tau * rcp(beta[k] + eps);
      const T a = T(C::ideal[k]) * (T(1) + qk * qk);
      num += a * rk;
      den += a;
    }
    return base + num * rcp(den);
  }
}

}  // namespace tz
}  // namespace oc
