// Coarse-graining of a fine nonhydrostatic state onto a grid r times coarser
// in every direction, and the vertical subgrid fluxes that a learned closure
// is trained to predict (the regridding paragraph of the finite-volume
// appendix of arXiv 2502.14148: averages weighted by volume or face area,
// which preserve integrals and the discrete divergence).
//
//   centred fields : mean over the r^3 fine cells of a coarse cell;
//   u (v, w)       : mean over the r^2 fine faces lying on the coarse face;
//   fluxes         : <q w> - <q><w> over the r^3 box for q = u, v, w, b with
//                    u, v, w first averaged to the fine cell centres.
// Sums are accumulated in FP64.  One thread per coarse cell.
#include "oc_internal.h"

namespace oc {

namespace {

template <class T>
__global__ void __launch_bounds__(256) coarse_grain_kernel(CoarseArgs<T> a) {
  const Dims df = a.df, dc = a.dc;
  const long n = (long)dc.nx * dc.ny * dc.nz;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int I = (int)(t % dc.nx);
  const int J = (int)((t / dc.nx) % dc.ny);
  const int K = (int)(t / ((long)dc.nx * dc.ny));
  const int r = a.r;
  const int i0 = r * I, j0 = r * J, k0 = r * K;
  double su = 0, sv = 0, sw = 0, st = 0, ss = 0;
  // box sums of the centred velocities, buoyancy and their products with w
  double qu = 0, qv = 0, qw = 0, qb = 0, cu = 0, cv = 0, cw = 0, cb = 0;
  for (int kk = 0; kk < r; ++kk)
    for (int jj = 0; jj < r; ++jj) {
      const long row = pidx(df, i0, j0 + jj, k0 + kk);
      // faces on the coarse faces
      su += (double)a.u[row];
      if (jj == 0)
        for (int ii = 0; ii < r; ++ii) sv += (double)a.v[row + ii];
      if (kk == 0)
        for (int ii = 0; ii < r; ++ii) sw += (double)a.w[row + ii];
      for (int ii = 0; ii < r; ++ii) {
        const long c = row + ii;
        const double tc = (double)a.t[c], sc = (double)a.s[c];
        st += tc;
        ss += sc;
        const double uc = 0.5 * ((double)a.u[c] + (double)a.u[c + 1]);
        const double vc = 0.5 * ((double)a.v[c] + (double)a.v[c + df.sy]);
        const double wc = 0.5 * ((double)a.w[c] + (double)a.w[c + df.sz]);
        const double b = a.ga * (tc - a.tref) - a.gb * (sc - a.sref);
        cu += uc; cv += vc; cw += wc; cb += b;
        qu += uc * wc; qv += vc * wc; qw += wc * wc; qb += b * wc;
      }
    }
  const double r2 = 1.0 / ((double)r * r), r3 = r2 / r;
  const long oc_ = pidx(dc, I, J, K);
  a.U[oc_] = (T)(su * r2);
  a.V[oc_] = (T)(sv * r2);
  a.W[oc_] = (T)(sw * r2);
  a.Tc[oc_] = (T)(st * r3);
  a.Sc[oc_] = (T)(ss * r3);
  if (a.flux) {
    const double mw = cw * r3;
    const long plane = n;
    a.flux[0 * plane + t] = (float)(qu * r3 - cu * r3 * mw);
    a.flux[1 * plane + t] = (float)(qv * r3 - cv * r3 * mw);
    a.flux[2 * plane + t] = (float)(qw * r3 - mw * mw);
    a.flux[3 * plane + t] = (float)(qb * r3 - cb * r3 * mw);
  }
}

}  // namespace

template <class T>
hipError_t launch_coarse_grain(const CoarseArgs<T>& a, hipStream_t s) {
  const long n = (long)a.dc.nx * a.dc.ny * a.dc.nz;
  hipLaunchKernelGGL(coarse_grain_kernel<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

template hipError_t launch_coarse_grain<float>(const CoarseArgs<float>&, hipStream_t);
template hipError_t launch_coarse_grain<double>(const CoarseArgs<double>&, hipStream_t);

}  // namespace oc
