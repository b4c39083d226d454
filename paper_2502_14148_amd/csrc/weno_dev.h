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

__device__ inline float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <class T>
__device__ inline T interp4(T a0, T a1, T a2, T a3) {
  return ((a1 + a2) * T(7) - (a0 + a3)) * T(1.0 / 12.0);
}

// Reconstruction at the interface between q_{-1} and q_0 from the six values
// q_{-3..2}; `vel` selects the upwind side.
//
// WENO-Z form used here (equal to the textbook form in exact arithmetic):
// with the upwind-ordered stencil (a, b, c, d, e) and its differences
// d1 = b - a, ..., d4 = e - d,
//   * candidates as deviations from the upwind neighbour c:
//       r0 - c = (5 d2 - 2 d1)/6, r1 - c = (d2 + 2 d3)/6, r2 - c = (4 d3 - d4)/6;
//   * four times the Jiang-Shu indicators plus eps:
//       s_k = 13/3 t_k^2 + u_k^2 + 4 eps, t = (d2 - d1, d3 - d2, d4 - d3),
//       u = (3 d2 - d1, d2 + d3, d4 - 3 d3)
//     (the weights only see ratios, so the common factor 4 drops out);
//   * WENO-Z weights d_k (1 + (tau / s_k)^2), tau = |s_0 - s_2|, multiplied
//     through by s_1^2:  a_k = s_1^2 + (tau s_1 / s_k)^2, a_1 = s_1^2 + tau^2,
//     so two reciprocals (of s_0 and s_2) replace three;
//   * W = c + sum d_k a_k (r_k - c) / sum d_k a_k.
// FP32 range: tau s_1 / s_k stays below 1.8e19 for indicators up to ~1e2 in
// the field's units squared next to an exactly flat stencil.
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
  const T d1 = b - a, d2 = c - b, d3 = d - c, d4 = e - d;
  // ideal weights (1/10, 6/10, 3/10) folded into the candidate deviations
  const T e0 = T(5.0 / 60.0) * d2 - T(2.0 / 60.0) * d1;
  const T e1 = T(6.0 / 60.0) * d2 + T(12.0 / 60.0) * d3;
  const T e2 = T(12.0 / 60.0) * d3 - T(3.0 / 60.0) * d4;
  const T t0 = d2 - d1, t1 = d3 - d2, t2 = d4 - d3;
  const T u0 = T(3) * d2 - d1, u1 = d2 + d3, u2 = d4 - T(3) * d3;
  const T e4 = T(4) * eps;
  const T s0 = fmad(T(13.0 / 3.0) * t0, t0, fmad(u0, u0, e4));
  const T s1 = fmad(T(13.0 / 3.0) * t1, t1, fmad(u1, u1, e4));
  const T s2 = fmad(T(13.0 / 3.0) * t2, t2, fmad(u2, u2, e4));
  const T tau = fabs(s0 - s2);
  const T s1s = s1 * s1;
  const T g0 = tau * (s1 * rcp(s0));
  const T g2 = tau * (s1 * rcp(s2));
  const T a0 = fmad(g0, g0, s1s);
  const T a1 = fmad(tau, tau, s1s);
  const T a2 = fmad(g2, g2, s1s);
  const T num = a0 * e0 + a1 * e1 + a2 * e2;
  const T den = T(0.1) * a0 + T(0.6) * a1 + T(0.3) * a2;
  return fmad(num, rcp(den), c);
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
