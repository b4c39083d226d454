// Vertically implicit diffusion (vertically implicit time-discretisation
// paragraph of the time-stepping appendix of arXiv 2502.14148: the tracer
// and predictor-velocity equations (1 - dt d/dz K d/dz) X^new = X~ with a
// second-order discretisation of the vertical diffusion operator, solved
// with a tridiagonal algorithm per column).
//
// Every column of a field shares one matrix (K and the z grid do not vary
// horizontally), so its elimination factors are computed once on the host in
// FP64: sub-diagonal s_q, inverse pivot 1/p_q and c_q = sup_q / p_q.  The
// kernel then runs, per column, the forward sweep d_q = (x_q - s_q d_{q-1})
// / p_q and the back substitution x_q = d_q - c_q x_{q+1}.  One thread owns
// one column; the forward results are kept in place in the field, and
// columns are read and written in batches of VB levels so that a batch's
// loads are all in flight before its first use.
#include "oc_internal.h"

namespace oc {

void vertical_factors(const double* dzc, const double* dzf, int nz, double K, double dt,
                      int wface, double* out) {
  const int n = wface ? nz - 1 : nz;
  double* sub = out;
  double* inv = out + n;
  double* cq = out + 2 * n;
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
    sub[q] = s;
    inv[q] = 1.0 / piv;
    cq[q] = (-dt * up) / piv;
    cprev = cq[q];
  }
}

namespace {

constexpr int VB = 8;

template <class T>
__global__ void __launch_bounds__(256) vimplicit_kernel(Dims d, T* __restrict__ f, int wface,
                                                        const T* __restrict__ fac) {
  const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (t >= d.nx * d.ny) return;
  const int i = t % d.nx, j = t / d.nx;
  const int k0 = wface ? 1 : 0, n = wface ? d.nz - 1 : d.nz;
  const T* sub = fac;
  const T* inv = fac + n;
  const T* cq = fac + 2 * n;
  T* __restrict__ col = f + pidx(d, i, j, k0);
  const long sz = d.sz;
  // forward sweep, results in place
  T prev = T(0);
  for (int q0 = 0; q0 < n; q0 += VB) {
    T x[VB];
#pragma unroll
    for (int b = 0; b < VB; ++b)
      if (q0 + b < n) x[b] = col[(long)(q0 + b) * sz];
#pragma unroll
    for (int b = 0; b < VB; ++b) {
      const int q = q0 + b;
      if (q < n) {
        prev = (x[b] - sub[q] * prev) * inv[q];
        col[(long)q * sz] = prev;
      }
    }
  }
  // back substitution from the top, with the halo images
  T xn = T(0);
  for (int q1 = n - 1; q1 >= 0; q1 -= VB) {
    T dq[VB];
#pragma unroll
    for (int b = 0; b < VB; ++b)
      if (q1 - b >= 0) dq[b] = col[(long)(q1 - b) * sz];
#pragma unroll
    for (int b = 0; b < VB; ++b) {
      const int q = q1 - b;
      if (q >= 0) {
        xn = (q == n - 1) ? dq[b] : dq[b] - cq[q] * xn;
        store_with_images(f, d, i, j, k0 + q, xn, wface != 0);
      }
    }
  }
}

}  // namespace

template <class T>
hipError_t launch_vertical_implicit(const Dims& d, T* f, int wface, const T* fac, hipStream_t s) {
  if (!d.zb) return hipErrorInvalidValue;
  const int cols = d.nx * d.ny;
  hipLaunchKernelGGL(vimplicit_kernel<T>, dim3((cols + 255) / 256), dim3(256), 0, s, d, f, wface,
                     fac);
  return hipGetLastError();
}

template hipError_t launch_vertical_implicit<float>(const Dims&, float*, int, const float*,
                                                    hipStream_t);
template hipError_t launch_vertical_implicit<double>(const Dims&, double*, int, const double*,
                                                     hipStream_t);

}  // namespace oc
