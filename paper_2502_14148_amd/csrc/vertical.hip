// Vertically implicit diffusion (vertically implicit time-discretisation
// paragraph of the time-stepping appendix of arXiv 2502.14148: the tracer
// and predictor-velocity equations (1 - dt d/dz K d/dz) X^new = X~ with a
// second-order discretisation of the vertical diffusion operator, solved
// with a tridiagonal algorithm per column).
//
// Every column of a field shares one matrix (K and the z grid do not vary
// horizontally), so everything that depends on the matrix alone is computed
// once on the host in FP64.  The elimination is written as two first-order
// linear recurrences,
//   forward:  d_q = A_q d_{q-1} + I_q x~_q      (A_q = -s_q / p_q, I_q = 1/p_q)
//   backward: x_q = d_q + B_q x_{q+1}           (B_q = -sup_q / p_q)
// with s, sup the sub- and super-diagonal and p the pivots.  The n unknowns
// of a column are split into VCH chunks of C levels, one per wavefront of a
// workgroup, each wave holding its chunk of 64 columns in registers.  A chunk
// solves its recurrences from zero; the true solution adds the incoming
// value times the precomputed products P_q = A_{q0}..A_q (forward) and
// Q_q = B_q..B_{q1-1} (backward), and the incoming values are chained across
// the chunks through LDS.  Each element is read once and written once.
#include <algorithm>
#include <vector>

#include "oc_internal.h"

namespace oc {

namespace {
constexpr int VCH = 8;      // chunks (wavefronts) per column group
constexpr int VCMAX = 32;   // levels per chunk at most (n <= 256)
}  // namespace

int vertical_chunk(int n) { return (n + VCH - 1) / VCH; }

void vertical_factors(const double* dzc, const double* dzf, int nz, double K, double dt,
                      int wface, double* out) {
  const int n = wface ? nz - 1 : nz;
  const int C = vertical_chunk(n);
  double* A = out;
  double* I = out + n;
  double* P = out + 2 * n;
  double* B = out + 3 * n;
  double* Q = out + 4 * n;
  double* PE = out + 5 * n;         // per chunk: P at its last level (1 if empty)
  double* QS = PE + VCH;            // per chunk: Q at its first level (1 if empty)
  std::vector<double> sup(n);
  double cprev = 0.0;
  for (int q = 0; q < n; ++q) {
    double lo, up, diag;
    if (wface) {
      // w on face k = q + 1, between the centres k - 1 and k (w = 0 on walls)
      const int k = q + 1;
      lo = K / (dzc[k - 1] * dzf[k]);
      up = K / (dzc[k] * dzf[k]);
      diag = 1.0 + dt * (lo + up);
      if (q == 0) lo = 0.0;
      if (q == n - 1) up = 0.0;
    } else {
      // centred cell k = q; no diffusive flux through the walls
      lo = (q > 0) ? K / (dzc[q] * dzf[q]) : 0.0;
      up = (q < n - 1) ? K / (dzc[q] * dzf[q + 1]) : 0.0;
      diag = 1.0 + dt * (lo + up);
    }
    const double s = -dt * lo;
    const double piv = diag - s * cprev;
    I[q] = 1.0 / piv;
    A[q] = -s / piv;
    sup[q] = -dt * up;
    cprev = sup[q] / piv;
    B[q] = -cprev;
  }
  for (int c = 0; c < VCH; ++c) {
    const int q0 = c * C, q1 = std::min(q0 + C, n);
    double prod = 1.0;
    for (int q = q0; q < q1; ++q) {
      prod *= A[q];
      P[q] = prod;
    }
    PE[c] = (q1 > q0) ? P[q1 - 1] : 1.0;
    prod = 1.0;
    for (int q = q1 - 1; q >= q0; --q) {
      prod *= B[q];
      Q[q] = prod;
    }
    QS[c] = (q1 > q0) ? Q[q0] : 1.0;
  }
}

int vertical_factors_len(int nz) { return 5 * nz + 2 * VCH; }

namespace {

template <class T>
__global__ void __launch_bounds__(64 * VCH) vimplicit_kernel(Dims d, VImplicitArgs<T> a) {
  __shared__ T endv[VCH][64];
  __shared__ T startv[VCH][64];
  const int fld = blockIdx.y;
  T* __restrict__ f = a.f[fld];
  const int wface = a.wface[fld];
  const T* __restrict__ tab = a.fac[fld];
  const int n = wface ? d.nz - 1 : d.nz, k0 = wface ? 1 : 0;
  const int C = (n + VCH - 1) / VCH;
  const T* A = tab;
  const T* I = tab + n;
  const T* P = tab + 2 * n;
  const T* B = tab + 3 * n;
  const T* Q = tab + 4 * n;
  const T* PE = tab + 5 * n;
  const T* QS = PE + VCH;
  // the chunk is the wavefront index: uniform, so the tables are scalar loads
  const int lane = threadIdx.x & 63;
  const int c = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // Workgroups are dealt round-robin to the 8 XCDs (XCD x takes x, x + 8,
  // ...); renumber the column groups so that each XCD takes a contiguous run
  // of them: neighbouring groups share the cache lines at their ends (rows
  // are not 128-byte aligned), which then meet in one L2
  const int ng = (int)gridDim.x, bx = (int)blockIdx.x, xcd = bx % 8;
  const int grp = xcd * (ng / 8) + min(xcd, ng % 8) + bx / 8;
  const int col = grp * 64 + lane;
  const bool valid = col < d.nx * d.ny;
  const int i = valid ? col % d.nx : 0, j = valid ? col / d.nx : 0;
  const int q0 = c * C;
  const int q1 = min(q0 + C, n);
  const long sz = d.sz;
  T* __restrict__ base = f + pidx(d, i, j, k0);
  T x[VCMAX];
#pragma unroll
  for (int r = 0; r < VCMAX; ++r)
    if (valid && q0 + r < q1) x[r] = base[(long)(q0 + r) * sz];
  // forward recurrence within the chunk, from zero
  T dl = T(0);
#pragma unroll
  for (int r = 0; r < VCMAX; ++r) {
    const int q = q0 + r;
    if (q < q1) {
      dl = A[q] * dl + I[q] * x[r];
      x[r] = dl;
    }
  }
  endv[c][lane] = dl;
  __syncthreads();
  T din = T(0);
  for (int cc = 0; cc < c; ++cc) din = PE[cc] * din + endv[cc][lane];
  // backward recurrence within the chunk (after the forward correction)
  T xl = T(0);
#pragma unroll
  for (int r = VCMAX - 1; r >= 0; --r) {
    const int q = q0 + r;
    if (q < q1) {
      xl = (x[r] + P[q] * din) + B[q] * xl;
      x[r] = xl;
    }
  }
  startv[c][lane] = xl;
  __syncthreads();
  T xin = T(0);
  for (int cc = VCH - 1; cc > c; --cc) xin = QS[cc] * xin + startv[cc][lane];
  if (!valid) return;
#pragma unroll
  for (int r = 0; r < VCMAX; ++r) x[r] += Q[min(q0 + r, n - 1)] * xin;
  // plain stores, plus the periodic x / y images of the h columns next to
  // each side (per-lane offsets, masked off everywhere else; a column of an
  // axis shorter than 2H has an image at both ends)
  const long sy = d.sy;
  const int H = d.h;
  const long oxa = (i < H) ? d.nx : 0, oxb = (i >= d.nx - H) ? -(long)d.nx : 0;
  const long oya = (j < H) ? d.ny * sy : 0, oyb = (j >= d.ny - H) ? -(long)d.ny * sy : 0;
#pragma unroll
  for (int r = 0; r < VCMAX; ++r) {
    const int q = q0 + r;
    if (q < q1) {
      T* p = base + (long)q * sz;
      p[0] = x[r];
      if (oxa) p[oxa] = x[r];
      if (oxb) p[oxb] = x[r];
      if (oya) {
        p[oya] = x[r];
        if (oxa) p[oya + oxa] = x[r];
        if (oxb) p[oya + oxb] = x[r];
      }
      if (oyb) {
        p[oyb] = x[r];
        if (oxa) p[oyb + oxa] = x[r];
        if (oxb) p[oyb + oxb] = x[r];
      }
    }
  }
  // the mirror images of the levels next to the walls (first and last
  // chunks only; uniform across the wavefront)
  if (k0 + q0 <= H || k0 + q1 >= d.nz - H) {
#pragma unroll
    for (int r = 0; r < VCMAX; ++r) {
      const int q = q0 + r, k = k0 + q;
      if (q < q1 && (k <= H || k >= d.nz - H))
        store_with_images(f, d, i, j, k, x[r], wface != 0);
    }
  }
}

}  // namespace

template <class T>
hipError_t launch_vertical_implicit(const Dims& d, const VImplicitArgs<T>& a, int nfields,
                                    hipStream_t s) {
  if (!d.zb || d.nz > VCH * VCMAX || nfields < 1 || nfields > MAXF) return hipErrorInvalidValue;
  const int cols = d.nx * d.ny;
  hipLaunchKernelGGL(vimplicit_kernel<T>, dim3((cols + 63) / 64, nfields), dim3(64 * VCH), 0, s,
                     d, a);
  return hipGetLastError();
}

template hipError_t launch_vertical_implicit<float>(const Dims&, const VImplicitArgs<float>&, int,
                                                    hipStream_t);
template hipError_t launch_vertical_implicit<double>(const Dims&, const VImplicitArgs<double>&,
                                                     int, hipStream_t);

}  // namespace oc
