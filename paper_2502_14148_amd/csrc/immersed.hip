// Grid-fitted immersed boundaries: the vector kernels of the preconditioned
// conjugate-gradient pressure solve (pressure solver for irregular domains of
// the pressure-correction appendix of arXiv 2502.14148) and the masking of
// velocities on closed faces.
//
// The equation: on the fluid cells, the 7-point Laplacian with no flux
// through faces next to an immersed cell (or a wall) equals div(u~)/dt_eff;
// gauge: zero mean over the fluid cells.  The preconditioner is the FFT/DCT
// solve of the whole box (poisson.hip) applied to the residual, which is zero
// in immersed cells, with its result masked to the fluid.
//
// Vectors are dense FP64 (nz, ny, nx), x fastest; the geometry comes as one
// byte per cell (IB_* bits: the cell is fluid, and which of its six faces
// are open).  Reductions are
// deterministic: every reducing kernel runs a fixed grid of IB_NPART
// workgroups over a fixed grid-stride partition, each writing one partial
// sum, and a single-workgroup kernel adds the partials in a fixed order and
// updates the iteration's scalars on the device (no host round trip inside
// an iteration).
#include "oc_internal.h"

namespace oc {

namespace {

constexpr int IB_NT = 256;

__device__ inline double block_sum(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
#pragma unroll
  for (int s = IB_NT / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  return sh[0];
}

// Workgroups are dealt round-robin to the 8 XCDs; the stencil kernels
// renumber them so that each XCD sweeps a contiguous range of cells in every
// round of the grid-stride loop, and the neighbouring planes a cell reads
// stay in that XCD's L2.
__device__ inline long first_cell() {
  const unsigned nb = gridDim.x, b = blockIdx.x;
  const unsigned vb = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
  return (long)vb * IB_NT + threadIdx.x;
}

// (i, j, k) of a dense index (32-bit arithmetic: N < 2^31)
__device__ inline void cell_of(const Dims& d, long n, int& i, int& j, int& k) {
  const unsigned u = (unsigned)n, nx = (unsigned)d.nx, ny = (unsigned)d.ny;
  const unsigned r = u / nx;
  i = (int)(u - r * nx);
  k = (int)(r / ny);
  j = (int)(r - (unsigned)k * ny);
}

// b = div(u~) / dt_eff in fluid cells (face velocities times their open
// flags), 0 in immersed cells; r = b, x = 0; partial sums of b^2.
template <class T>
__global__ void __launch_bounds__(IB_NT) ib_rhs_kernel(Dims d, const T* __restrict__ u,
                                                       const T* __restrict__ v,
                                                       const T* __restrict__ w,
                                                       const uint8_t* __restrict__ bits,
                                                       double inv_dt, double rdx, double rdy,
                                                       double rdz, CgBufs cg) {
  __shared__ double sh[IB_NT];
  const long N = (long)d.nx * d.ny * d.nz;
  double acc = 0.0;
  for (long n = first_cell(); n < N; n += (long)gridDim.x * IB_NT) {
    const unsigned fb = bits[n];
    double b = 0.0;
    if (fb & IB_FLUID) {
      int i, j, k;
      cell_of(d, n, i, j, k);
      const long c = pidx(d, i, j, k);
      const double ul = (fb & IB_XM) ? (double)u[c] : 0.0;
      const double ur = (fb & IB_XP) ? (double)u[pidx(d, (i + 1 == d.nx) ? 0 : i + 1, j, k)] : 0.0;
      const double vl = (fb & IB_YM) ? (double)v[c] : 0.0;
      const double vr = (fb & IB_YP) ? (double)v[pidx(d, i, (j + 1 == d.ny) ? 0 : j + 1, k)] : 0.0;
      const double wb = (fb & IB_ZM) ? (double)w[c] : 0.0;
      const double wt = (fb & IB_ZP) ? (double)w[pidx(d, i, j, (k + 1 == d.nz) ? 0 : k + 1)] : 0.0;
      b = ((ur - ul) * rdx + (vr - vl) * rdy + (wt - wb) * rdz) * inv_dt;
    }
    cg.r[n] = b;
    cg.x[n] = 0.0;
    acc += b * b;
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) cg.part[blockIdx.x] = s;
}

// aq = A q (the masked 7-point operator, zero in immersed cells); partial
// sums of q . aq.  Work items are 32 x 8 column tiles of IB_KC levels; each
// workgroup takes items b, b + IB_NPART, ... (XCD-contiguous numbering) and
// marches its columns up the levels, so q of a column is fetched once and
// carried in registers as the z neighbours of the next levels; the four
// in-plane neighbours come through the caches.  Every neighbour is loaded
// and weighted by its face's open flag; z neighbours beyond a wall are read
// from the periodic image, which the flag then discards.
constexpr int IB_TX = 32, IB_TY = 8, IB_KC = 16;

__global__ void __launch_bounds__(IB_NT) ib_apply_kernel(Dims d, const uint8_t* __restrict__ bits,
                                                         double rdx2, double rdy2, double rdz2,
                                                         CgBufs cg) {
  __shared__ double sh[IB_NT];
  if (cg.scal[CG_DONE] != 0.0) return;
  const int nbx = (d.nx + IB_TX - 1) / IB_TX, nby = (d.ny + IB_TY - 1) / IB_TY;
  const int nbz = (d.nz + IB_KC - 1) / IB_KC;
  const int items = nbx * nby * nbz;
  const unsigned plane = (unsigned)d.nx * d.ny;
  const double* __restrict__ q = cg.q;
  double* __restrict__ aq = cg.aq;
  const int tx = threadIdx.x % IB_TX, ty = threadIdx.x / IB_TX;
  const unsigned nb = gridDim.x, b0 = blockIdx.x;
  const int vb = (int)((nb % 8 == 0) ? (b0 % 8) * (nb / 8) + b0 / 8 : b0);
  double acc = 0.0;
  for (int item = vb; item < items; item += (int)nb) {
    const int i = (item % nbx) * IB_TX + tx;
    const int j = ((item / nbx) % nby) * IB_TY + ty;
    const int kb = (item / (nbx * nby)) * IB_KC, ke = min(kb + IB_KC, d.nz);
    if (i >= d.nx || j >= d.ny) continue;
    // in-plane offsets of the own cell and its x, y neighbours (periodic)
    const unsigned c = (unsigned)j * d.nx + i;
    const unsigned cxm = (i == 0) ? c + d.nx - 1 : c - 1;
    const unsigned cxp = (i + 1 == d.nx) ? c - (d.nx - 1) : c + 1;
    const unsigned cym = (j == 0) ? c + plane - d.nx : c - d.nx;
    const unsigned cyp = (j + 1 == d.ny) ? c - plane + d.nx : c + d.nx;
    double qm = q[(kb == 0 ? (unsigned)(d.nz - 1) : (unsigned)(kb - 1)) * plane + c];
    double q0 = q[(unsigned)kb * plane + c];
    for (int k = kb; k < ke; ++k) {
      const unsigned pk = (unsigned)k * plane;
      const double qp = q[(k + 1 == d.nz ? 0u : pk + plane) + c];
      const unsigned fb = bits[pk + c];
      const double qxm = q[pk + cxm], qxp = q[pk + cxp];
      const double qym = q[pk + cym], qyp = q[pk + cyp];
      auto on = [fb](unsigned bit) { return (fb & bit) ? 1.0 : 0.0; };
      const double a = (on(IB_XM) * (qxm - q0) + on(IB_XP) * (qxp - q0)) * rdx2 +
                       (on(IB_YM) * (qym - q0) + on(IB_YP) * (qyp - q0)) * rdy2 +
                       (on(IB_ZM) * (qm - q0) + on(IB_ZP) * (qp - q0)) * rdz2;
      aq[pk + c] = a;
      acc += q0 * a;
      qm = q0;
      q0 = qp;
    }
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) cg.part[blockIdx.x] = s;
}

// r -= alpha aq; partial sums of r^2 (x takes alpha q in ib_dir_kernel, or
// in ib_xfinal_kernel after the last iteration).
__global__ void __launch_bounds__(IB_NT) ib_update_kernel(long N, CgBufs cg) {
  __shared__ double sh[IB_NT];
  if (cg.scal[CG_DONE] != 0.0) return;
  const double alpha = cg.scal[CG_ALPHA];
  double acc = 0.0;
  for (long n = blockIdx.x * (long)IB_NT + threadIdx.x; n < N; n += (long)gridDim.x * IB_NT) {
    const double r = cg.r[n] - alpha * cg.aq[n];
    cg.r[n] = r;
    acc += r * r;
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) cg.part[blockIdx.x] = s;
}

// x += alpha q (the step of the iteration that just ended; alpha = 0 before
// the first), then q = (z in fluid cells) + beta q
__global__ void __launch_bounds__(IB_NT) ib_dir_kernel(long N, const uint8_t* __restrict__ bits,
                                                       CgBufs cg, const double* __restrict__ z) {
  if (cg.scal[CG_DONE] != 0.0) return;
  const double beta = cg.scal[CG_BETA];
  const double alpha = cg.scal[CG_IT] > 0.0 ? cg.scal[CG_ALPHA] : 0.0;
  for (long n = blockIdx.x * (long)IB_NT + threadIdx.x; n < N; n += (long)gridDim.x * IB_NT) {
    const double q = cg.q[n];
    if (alpha != 0.0) cg.x[n] += alpha * q;
    cg.q[n] = ((bits[n] & IB_FLUID) ? z[n] : 0.0) + (beta != 0.0 ? beta * q : 0.0);
  }
}

// after the last iteration: x += alpha q (nothing if no iteration ran)
__global__ void __launch_bounds__(IB_NT) ib_xfinal_kernel(long N, CgBufs cg) {
  if (cg.scal[CG_IT] == 0.0) return;
  const double alpha = cg.scal[CG_ALPHA];
  for (long n = blockIdx.x * (long)IB_NT + threadIdx.x; n < N; n += (long)gridDim.x * IB_NT)
    cg.x[n] += alpha * cg.q[n];
}

// partial sums of x (zero in immersed cells) for the gauge
__global__ void __launch_bounds__(IB_NT) ib_sum_kernel(long N, CgBufs cg) {
  __shared__ double sh[IB_NT];
  double acc = 0.0;
  for (long n = blockIdx.x * (long)IB_NT + threadIdx.x; n < N; n += (long)gridDim.x * IB_NT)
    acc += cg.x[n];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) cg.part[blockIdx.x] = s;
}

// x -= mean over the fluid cells, in fluid cells
__global__ void __launch_bounds__(IB_NT) ib_shift_kernel(long N, const uint8_t* __restrict__ bits,
                                                         CgBufs cg) {
  const double mean = cg.scal[CG_MEAN];
  for (long n = blockIdx.x * (long)IB_NT + threadIdx.x; n < N; n += (long)gridDim.x * IB_NT)
    cg.x[n] = (bits[n] & IB_FLUID) ? cg.x[n] - mean : 0.0;
}

// Add the IB_NPART partials in a fixed order and update the scalars.
__global__ void __launch_bounds__(IB_NT) ib_finalize_kernel(CgBufs cg, int what, double tol2,
                                                            int maxiter, double nfluid,
                                                            int npart) {
  __shared__ double sh[IB_NT];
  double* sc = cg.scal;
  if (what != CG_FIN_MEAN && what != CG_FIN_BNORM && sc[CG_DONE] != 0.0) return;
  double acc = 0.0;
  for (int b = threadIdx.x; b < npart; b += IB_NT) acc += cg.part[b];
  const double s = block_sum(acc, sh);
  if (threadIdx.x != 0) return;
  switch (what) {
    case CG_FIN_BNORM:
      sc[CG_BNORM2] = s;
      sc[CG_RNORM2] = s;
      sc[CG_IT] = 0.0;
      sc[CG_DONE] = (s == 0.0) ? 1.0 : 0.0;
      break;
    case CG_FIN_RZ0:
      sc[CG_RZ] = s;
      sc[CG_BETA] = 0.0;
      break;
    case CG_FIN_ALPHA:
      sc[CG_ALPHA] = sc[CG_RZ] / s;
      break;
    case CG_FIN_RES:
      sc[CG_RNORM2] = s;
      sc[CG_IT] += 1.0;
      if (s <= tol2 * sc[CG_BNORM2] || sc[CG_IT] >= (double)maxiter) sc[CG_DONE] = 1.0;
      break;
    case CG_FIN_BETA:
      sc[CG_BETA] = s / sc[CG_RZ];
      sc[CG_RZ] = s;
      break;
    default:  // CG_FIN_MEAN
      sc[CG_MEAN] = s / nfluid;
  }
}

// Velocities on closed faces set to zero (interior faces; halos refilled by
// the caller).  Wall faces of w are zero already.
template <class T>
__global__ void __launch_bounds__(IB_NT) ib_mask_velocity_kernel(Dims d, T* __restrict__ u,
                                                                 T* __restrict__ v,
                                                                 T* __restrict__ w,
                                                                 const T* __restrict__ mask) {
  const long N = (long)d.nx * d.ny * d.nz;
  for (long n = blockIdx.x * (long)IB_NT + threadIdx.x; n < N; n += (long)gridDim.x * IB_NT) {
    int i, j, k;
    cell_of(d, n, i, j, k);
    const long c = pidx(d, i, j, k);
    const T m0 = mask[c];
    u[c] = u[c] * (m0 * mask[c - 1]);
    v[c] = v[c] * (m0 * mask[c - d.sy]);
    if (!d.zb || k > 0) w[c] = w[c] * (m0 * mask[c - d.sz]);
  }
}

int ib_grid(long N) {
  const long b = (N + IB_NT - 1) / IB_NT;
  return (int)(b < IB_NPART ? b : IB_NPART);
}

}  // namespace

// Every reducing kernel uses exactly IB_NPART workgroups (the partial array
// is read whole); the others use up to that many.
template <class T>
hipError_t launch_ib_rhs(const Dims& d, const T* u, const T* v, const T* w,
                         const uint8_t* bits, double inv_dt, double rdx, double rdy, double rdz,
                         const CgBufs& cg, hipStream_t s) {
  hipLaunchKernelGGL(ib_rhs_kernel<T>, dim3(IB_NPART), dim3(IB_NT), 0, s, d, u, v, w, bits,
                     inv_dt, rdx, rdy, rdz, cg);
  return hipGetLastError();
}

hipError_t launch_ib_apply(const Dims& d, const uint8_t* bits, double rdx2, double rdy2,
                           double rdz2, const CgBufs& cg, hipStream_t s) {
  hipLaunchKernelGGL(ib_apply_kernel, dim3(IB_NPART), dim3(IB_NT), 0, s, d, bits, rdx2, rdy2,
                     rdz2, cg);
  return hipGetLastError();
}

hipError_t launch_ib_update(const Dims& d, const CgBufs& cg, hipStream_t s) {
  hipLaunchKernelGGL(ib_update_kernel, dim3(IB_NPART), dim3(IB_NT), 0, s,
                     (long)d.nx * d.ny * d.nz, cg);
  return hipGetLastError();
}

hipError_t launch_ib_dir(const Dims& d, const uint8_t* bits, const CgBufs& cg, const double* z,
                         hipStream_t s) {
  const long N = (long)d.nx * d.ny * d.nz;
  hipLaunchKernelGGL(ib_dir_kernel, dim3(ib_grid(N)), dim3(IB_NT), 0, s, N, bits, cg, z);
  return hipGetLastError();
}

hipError_t launch_ib_gauge(const Dims& d, const uint8_t* bits, const CgBufs& cg, double nfluid,
                           hipStream_t s) {
  const long N = (long)d.nx * d.ny * d.nz;
  hipLaunchKernelGGL(ib_sum_kernel, dim3(IB_NPART), dim3(IB_NT), 0, s, N, cg);
  hipLaunchKernelGGL(ib_finalize_kernel, dim3(1), dim3(IB_NT), 0, s, cg, (int)CG_FIN_MEAN, 0.0, 0,
                     nfluid, (int)IB_NPART);
  hipLaunchKernelGGL(ib_shift_kernel, dim3(ib_grid(N)), dim3(IB_NT), 0, s, N, bits, cg);
  return hipGetLastError();
}

hipError_t launch_ib_finalize(const CgBufs& cg, int what, double tol2, int maxiter,
                              hipStream_t s, int npart) {
  hipLaunchKernelGGL(ib_finalize_kernel, dim3(1), dim3(IB_NT), 0, s, cg, what, tol2, maxiter,
                     1.0, npart);
  return hipGetLastError();
}

hipError_t launch_ib_xfinal(const Dims& d, const CgBufs& cg, hipStream_t s) {
  const long N = (long)d.nx * d.ny * d.nz;
  hipLaunchKernelGGL(ib_xfinal_kernel, dim3(ib_grid(N)), dim3(IB_NT), 0, s, N, cg);
  return hipGetLastError();
}

template <class T>
hipError_t launch_ib_mask_velocity(const Dims& d, T* u, T* v, T* w, const T* mask,
                                   hipStream_t s) {
  hipLaunchKernelGGL(ib_mask_velocity_kernel<T>, dim3(ib_grid((long)d.nx * d.ny * d.nz)),
                     dim3(IB_NT), 0, s, d, u, v, w, mask);
  return hipGetLastError();
}

#define OC_IB_INST(T)                                                                        \
  template hipError_t launch_ib_rhs<T>(const Dims&, const T*, const T*, const T*,             \
                                       const uint8_t*, double, double, double, double,        \
                                       const CgBufs&, hipStream_t);                           \
  template hipError_t launch_ib_mask_velocity<T>(const Dims&, T*, T*, T*, const T*,           \
                                                 hipStream_t);
OC_IB_INST(float)
OC_IB_INST(double)
#undef OC_IB_INST

}  // namespace oc
