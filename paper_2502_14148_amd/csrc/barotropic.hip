// Split-explicit barotropic substeps of the hydrostatic model on gfx950
// (hydrostatic time-discretisation appendix of arXiv 2502.14148).
//
// One launch per substep; a substep reads (eta, U, V)^n from one buffer set
// and writes (eta, U, V)^{n+1} to the other.  Each workgroup recomputes
// eta^{n+1} on a one-cell halo (left column, bottom row) of its tile, so the
// forward (eta) and backward (U, V) halves of the substep fuse into one
// kernel without a grid-wide barrier.  The running averages are accumulated
// in place in FP64.  All 2D arrays are dense FP64, x fastest; x is
// periodic, y has walls (V = 0 on faces 0 and ny).
#include "oc_internal.h"

namespace oc {

namespace {

constexpr int BTX = 32, BTY = 8;

// transport divergence at cell (i, j)
__device__ inline double baro_div(const BaroBufs& b, int i, int j) {
  const int ip = (i + 1 == b.nx) ? 0 : i + 1;
  const long r = (long)j * b.nx;
  const double fx = b.len_u[j] * (b.U[r + ip] - b.U[r + i]);
  const double fy = b.len_v[j + 1] * b.V[r + b.nx + i] - b.len_v[j] * b.V[r + i];
  return (fx + fy) / b.area[j];
}

__global__ void __launch_bounds__(BTX * BTY) baro_substep_kernel(BaroBufs b, double dtau, double gH,
                                                                 double wn) {
  __shared__ double eta1[BTY + 1][BTX + 1];
  const int i0 = blockIdx.x * BTX, j0 = blockIdx.y * BTY;
  const int tid = threadIdx.x;
  // eta^{n+1} on the tile plus its left column and bottom row
  for (int e = tid; e < (BTX + 1) * (BTY + 1); e += BTX * BTY) {
    const int ly = e / (BTX + 1), lx = e - ly * (BTX + 1);
    int i = i0 - 1 + lx;
    if (i < 0) i += b.nx;
    const int j = j0 - 1 + ly;
    double v = 0.0;
    if (j >= 0 && j < b.ny && i < b.nx) v = b.eta[(long)j * b.nx + i] - dtau * baro_div(b, i, j);
    eta1[ly][lx] = v;
  }
  __syncthreads();
  const int tx = tid % BTX, ty = tid / BTX;
  const int i = i0 + tx, j = j0 + ty;
  if (i >= b.nx || j >= b.ny) return;
  const long c = (long)j * b.nx + i;
  const double en = eta1[ty + 1][tx + 1];
  const double un = b.U[c] - dtau * (gH * (en - eta1[ty + 1][tx]) / b.dx_u[j] - b.GU[c]);
  double vn = 0.0;  // the southern wall face j = 0 stays closed
  if (j > 0) vn = b.V[c] - dtau * (gH * (en - eta1[ty][tx + 1]) / b.dy_v[j] - b.GV[c]);
  b.eta1[c] = en;
  b.U1[c] = un;
  b.V1[c] = vn;
  b.etab[c] += wn * en;
  b.Ub[c] += wn * un;
  b.Vb[c] += wn * vn;
}

__global__ void baro_fill_kernel(double* a, double v, long n) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) a[t] = v;
}

__global__ void baro_copy_kernel(double* dst, const double* src, long n) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) dst[t] = src[t];
}

// u <- u + (Ubar - dz sum_k u) / H on every column of a 3D field stored in
// the padded layout; `nyf` rows (v: the interior faces 1..ny-1 only).
template <class T>
__global__ void baro_correct_kernel(Dims d, T* __restrict__ f, const double* __restrict__ bar,
                                    int j_lo, int j_hi, double dz, double inv_h) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = j_lo + blockIdx.y;
  if (i >= d.nx || j >= j_hi) return;
  const long c0 = pidx(d, i, j, 0);
  double sum = 0.0;
  for (int k = 0; k < d.nz; ++k) sum += (double)f[c0 + (long)k * d.sz];
  const double corr = (bar[(long)j * d.nx + i] - dz * sum) * inv_h;
  for (int k = 0; k < d.nz; ++k) {
    const long c = c0 + (long)k * d.sz;
    f[c] = (T)((double)f[c] + corr);
  }
}

}  // namespace

hipError_t launch_baro_fill(double* a, double v, long n, hipStream_t s) {
  hipLaunchKernelGGL(baro_fill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, v, n);
  return hipGetLastError();
}

hipError_t launch_baro_copy(double* dst, const double* src, long n, hipStream_t s) {
  hipLaunchKernelGGL(baro_copy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dst,
                     src, n);
  return hipGetLastError();
}

hipError_t launch_baro_substep(const BaroBufs& b, double dtau, double gH, double wn,
                               hipStream_t s) {
  dim3 grid((b.nx + BTX - 1) / BTX, (b.ny + BTY - 1) / BTY);
  hipLaunchKernelGGL(baro_substep_kernel, grid, dim3(BTX * BTY), 0, s, b, dtau, gH, wn);
  return hipGetLastError();
}

template <class T>
hipError_t launch_baro_correct(const Dims& d, T* f, const double* bar, int j_lo, int j_hi,
                               double dz, double depth, hipStream_t s) {
  if (j_hi <= j_lo) return hipSuccess;
  dim3 grid((d.nx + 63) / 64, j_hi - j_lo);
  hipLaunchKernelGGL(baro_correct_kernel<T>, grid, dim3(64), 0, s, d, f, bar, j_lo, j_hi, dz,
                     1.0 / depth);
  return hipGetLastError();
}

template hipError_t launch_baro_correct<float>(const Dims&, float*, const double*, int, int, double,
                                               double, hipStream_t);
template hipError_t launch_baro_correct<double>(const Dims&, double*, const double*, int, int,
                                                double, double, hipStream_t);

}  // namespace oc
