// Stencil kernels of the nonhydrostatic model on gfx950: halo fill (C-grid
// staggering of the finite-volume appendix of arXiv 2502.14148, face i left
// of cell i), dense <-> padded copies and FP64 diagnostics.
#include <mutex>

#include "oc_internal.h"

namespace oc {

// ---------------------------------------------------------------------------
// Halo fill: one thread per padded element; every halo element copies an
// interior element chosen axis by axis (periodic wrap; even mirror in a
// bounded z for centred data; odd mirror about the wall face for w, whose
// top wall face (stored in the first upper halo plane) is set to 0).  Sources
// are always interior, so one pass fills corners too.
// ---------------------------------------------------------------------------
template <class T>
struct HaloArgs {
  T* f[MAXF];
  int kind[MAXF];  // 0 centred in z, 1 on z faces (w)
};

template <class T>
__global__ void __launch_bounds__(256) halo_fill_kernel(Dims d, HaloArgs<T> a, long total) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int fld = blockIdx.y;
  if (t >= total) return;
  const int pi = (int)(t % d.px);
  const int pj = (int)((t / d.px) % d.py);
  const int pk = (int)(t / ((long)d.px * d.py));
  int i = pi - d.h, j = pj - d.h, k = pk - d.h;
  const bool inx = (i >= 0 && i < d.nx), iny = (j >= 0 && j < d.ny);
  const int kind = a.kind[fld];
  bool inz;
  T sign = T(1);
  bool zero = false;
  int ks = k;
  if (!d.zb) {
    inz = (k >= 0 && k < d.nz);
    ks = (k + d.nz) % d.nz;
  } else if (kind == 0) {
    inz = (k >= 0 && k < d.nz);
    if (k < 0) ks = -1 - k;
    else if (k >= d.nz) ks = 2 * d.nz - 1 - k;
  } else {
    // w faces 0..nz; face 0 is interior (kept at 0 by the kernels), face nz
    // is the top wall stored in the halo
    inz = (k >= 0 && k < d.nz);
    if (k < 0) { ks = -k; sign = T(-1); }
    else if (k == d.nz) { zero = true; }
    else if (k > d.nz) { ks = 2 * d.nz - k; sign = T(-1); }
  }
  if (inx && iny && inz) return;
  const int is = (i + d.nx) % d.nx;
  const int js = (j + d.ny) % d.ny;
  T* f = a.f[fld];
  f[t] = zero ? T(0) : sign * f[pidx(d, is, js, ks)];
}

template <class T>
hipError_t launch_halo_fill(const Dims& d, T* const* fields, const int* kinds, int nf,
                            hipStream_t s) {
  HaloArgs<T> a;
  for (int q = 0; q < nf; ++q) { a.f[q] = fields[q]; a.kind[q] = kinds[q]; }
  long total = padded_elems(d);
  dim3 grid((unsigned)((total + 255) / 256), nf);
  hipLaunchKernelGGL(halo_fill_kernel<T>, grid, dim3(256), 0, s, d, a, total);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Dense (nzf, ny, nx) <-> padded copies with dtype conversion.
// ---------------------------------------------------------------------------
// `offset` is the storage offset of the field: stored = value - offset
// (FP32 tracers are kept as anomalies about the equation-of-state reference).
template <class T, class D>
__global__ void __launch_bounds__(256) pack_kernel(Dims d, int nzf, int nyf, T* padded, D* dense,
                                                   int to_dense, double offset) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long n = (long)nzf * nyf * d.nx;
  if (t >= n) return;
  int i = (int)(t % d.nx);
  int j = (int)((t / d.nx) % nyf);
  int k = (int)(t / ((long)d.nx * nyf));
  long p = pidx(d, i, j, k);
  if (to_dense) dense[t] = (D)((double)padded[p] + offset);
  else padded[p] = (T)((double)dense[t] - offset);
}

template <class T>
hipError_t launch_pack(const Dims& d, int nzf, int nyf, const T* padded, void* dense, int dtype,
                       int to_dense, double offset, hipStream_t s) {
  long n = (long)nzf * nyf * d.nx;
  dim3 grid((unsigned)((n + 255) / 256));
  T* pp = const_cast<T*>(padded);
  if (dtype == OC_F32)
    hipLaunchKernelGGL((pack_kernel<T, float>), grid, dim3(256), 0, s, d, nzf, nyf, pp,
                       (float*)dense, to_dense, offset);
  else
    hipLaunchKernelGGL((pack_kernel<T, double>), grid, dim3(256), 0, s, d, nzf, nyf, pp,
                       (double*)dense, to_dense, offset);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Diagnostics: per-block partials in a fixed order (deterministic), reduced
// on the host in block order.  Per block: max|div|, max|u|, max|v|, max|w|,
// thickness-weighted sums of tracers 0..3, the non-finite count, and the
// thickness-weighted sums of u, v (cell thickness) and w (face spacing).
// ---------------------------------------------------------------------------
constexpr int NPART = 12;
static_assert(NPART == DIAG_NPART, "partials per block");

template <class T>
struct DiagArgs {
  const T* f[MAXF];
  int nf;
};

// Accumulate cell (i, j, k) into the partials acc[NPART].
template <class T>
__device__ inline void diag_cell(const Dims& d, const DiagArgs<T>& a, double rdx, double rdy,
                                 const double* __restrict__ rdzc, const double* __restrict__ dzc,
                                 const double* __restrict__ dzf, int i, int j, int k,
                                 double* acc) {
  const long c = pidx(d, i, j, k);
  const int ip = (i + 1) % d.nx, jp = (j + 1) % d.ny;
  const double uu = (double)a.f[0][c], vv = (double)a.f[1][c], ww = (double)a.f[2][c];
  double wt;
  if (d.zb) wt = (k + 1 == d.nz) ? 0.0 : (double)a.f[2][c + d.sz];
  else wt = (double)a.f[2][pidx(d, i, j, (k + 1) % d.nz)];
  const double div = ((double)a.f[0][pidx(d, ip, j, k)] - uu) * rdx +
                     ((double)a.f[1][pidx(d, i, jp, k)] - vv) * rdy + (wt - ww) * rdzc[k];
  acc[0] = fmax(acc[0], fabs(div));
  acc[1] = fmax(acc[1], fabs(uu));
  acc[2] = fmax(acc[2], fabs(vv));
  acc[3] = fmax(acc[3], fabs(ww));
  bool bad = !isfinite(uu) || !isfinite(vv) || !isfinite(ww);
  for (int q = 3; q < a.nf; ++q) {
    const double x = (double)a.f[q][c];
    acc[1 + q] += x * dzc[k];  // layer thickness weight
    bad = bad || !isfinite(x);
  }
  if (bad) acc[8] += 1.0;
  // momentum: u and v cells have the thickness of cell k; w face k (the
  // bottom wall face is 0 in a bounded z) the spacing of the centres either
  // side of it
  acc[9] += uu * dzc[k];
  acc[10] += vv * dzc[k];
  acc[11] += ww * dzf[k];
}

// Block-wide reduction of acc[NPART] in a fixed order (maxima for 0..3, sums
// otherwise); thread q < NPART writes partial q to out[q].
__device__ inline void diag_block_reduce(double* acc, double* out) {
  __shared__ double red[NPART][256];
  for (int q = 0; q < NPART; ++q) red[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      for (int q = 0; q < NPART; ++q) {
        double x = red[q][threadIdx.x], y = red[q][threadIdx.x + w];
        red[q][threadIdx.x] = (q < 4) ? fmax(x, y) : x + y;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < NPART) out[threadIdx.x] = red[threadIdx.x][0];
}

template <class T>
__global__ void __launch_bounds__(256) diag_kernel(Dims d, DiagArgs<T> a, double rdx, double rdy,
                                                   const double* __restrict__ rdzc,
                                                   const double* __restrict__ dzc,
                                                   const double* __restrict__ dzf, double* part) {
  double acc[NPART];
  for (int q = 0; q < NPART; ++q) acc[q] = 0.0;
  const long n = (long)d.nx * d.ny * d.nz;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (long)gridDim.x * blockDim.x) {
    const int i = (int)(t % d.nx);
    const int j = (int)((t / d.nx) % d.ny);
    const int k = (int)(t / ((long)d.nx * d.ny));
    diag_cell(d, a, rdx, rdy, rdzc, dzc, dzf, i, j, k, acc);
  }
  diag_block_reduce(acc, part + (long)blockIdx.x * NPART);
}

template <class T>
hipError_t launch_diagnostics(const Dims& d, T* const* fields, int nf, double rdx, double rdy,
                              const double* rdzc, const double* dzc, const double* dzf,
                              double* scratch, int nblocks, hipStream_t s) {
  DiagArgs<T> a;
  for (int q = 0; q < nf; ++q) a.f[q] = fields[q];
  a.nf = nf;
  hipLaunchKernelGGL(diag_kernel<T>, dim3(nblocks), dim3(256), 0, s, d, a, rdx, rdy, rdzc, dzc,
                     dzf, scratch);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Diagnostics without allocation or host synchronisation: one workgroup per
// level writes that level's partials to `scratch` (a file-scope device array
// of DIAG_MAX_LEVELS x NPART doubles per GPU), then one workgroup reduces the
// levels in order and writes the finished values to the caller's device
// buffer.  Calls that overlap on one GPU share (and race on) the array.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[DIAG_MAX_LEVELS * NPART];

template <class T>
__global__ void __launch_bounds__(256) diag_level_kernel(Dims d, DiagArgs<T> a, double rdx,
                                                         double rdy,
                                                         const double* __restrict__ rdzc,
                                                         const double* __restrict__ dzc,
                                                         const double* __restrict__ dzf,
                                                         double* part) {
  double acc[NPART];
  for (int q = 0; q < NPART; ++q) acc[q] = 0.0;
  const int k = blockIdx.x;
  const int n = d.nx * d.ny;
  for (int t = threadIdx.x; t < n; t += blockDim.x)
    diag_cell(d, a, rdx, rdy, rdzc, dzc, dzf, t % d.nx, t / d.nx, k, acc);
  diag_block_reduce(acc, part + (long)k * NPART);
}

// Reduce the nz levels' partials in level order and finish the values as
// oc_diagnostics does on the host: out[0] max|div| * hmin, [1..3] max|u|,
// |v|, |w|, [4..7] tracer integrals (stored sums + offset x cells x dz, times
// dx dy), [8..10] momentum integrals, [11] CFL rate, [12] non-finite count.
__global__ void diag_finish_kernel(const double* __restrict__ part, int nz, DiagFinish f,
                                   double* __restrict__ out) {
  __shared__ double acc[NPART];
  const int q = threadIdx.x;
  if (q < NPART) {
    double x = 0.0;
    for (int k = 0; k < nz; ++k) {
      const double y = part[(long)k * NPART + q];
      x = (q < 4) ? fmax(x, y) : x + y;
    }
    acc[q] = x;
  }
  __syncthreads();
  if (q == 0) {
    out[0] = acc[0] * f.hmin;
    out[1] = acc[1];
    out[2] = acc[2];
    out[3] = acc[3];
    for (int t = 0; t < 4; ++t) out[4 + t] = (acc[4 + t] + f.toff[t]) * f.area;
    for (int t = 0; t < 3; ++t) out[8 + t] = acc[9 + t] * f.area;
    out[11] = fmax(acc[1] * f.rdx, fmax(acc[2] * f.rdy, acc[3] * f.rdzmin));
    out[12] = acc[8];
  }
}

// The array's device address on each GPU, looked up once per device with that
// device current (the host-side name of a __device__ array is not a device
// address).
static double* g_scratch[64];
static std::mutex g_scratch_mu;

static hipError_t scratch_address(double** p) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* q = nullptr;
    e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = (double*)q;
  }
  *p = g_scratch[dev];
  return hipSuccess;
}

template <class T>
hipError_t launch_diagnostics_noalloc(const Dims& d, T* const* fields, int nf, double rdx,
                                      double rdy, const double* rdzc, const double* dzc,
                                      const double* dzf, const DiagFinish& f, double* out,
                                      hipStream_t s) {
  if (d.nz > DIAG_MAX_LEVELS) return hipErrorInvalidValue;
  double* part = nullptr;
  hipError_t e = scratch_address(&part);
  if (e != hipSuccess) return e;
  DiagArgs<T> a;
  for (int q = 0; q < nf; ++q) a.f[q] = fields[q];
  a.nf = nf;
  hipLaunchKernelGGL(diag_level_kernel<T>, dim3(d.nz), dim3(256), 0, s, d, a, rdx, rdy, rdzc,
                     dzc, dzf, part);
  hipLaunchKernelGGL(diag_finish_kernel, dim3(1), dim3(64), 0, s, part, d.nz, f, out);
  return hipGetLastError();
}

template hipError_t launch_halo_fill<float>(const Dims&, float* const*, const int*, int, hipStream_t);
template hipError_t launch_halo_fill<double>(const Dims&, double* const*, const int*, int, hipStream_t);
template hipError_t launch_pack<float>(const Dims&, int, int, const float*, void*, int, int,
                                       double, hipStream_t);
template hipError_t launch_pack<double>(const Dims&, int, int, const double*, void*, int, int,
                                        double, hipStream_t);
template hipError_t launch_diagnostics<float>(const Dims&, float* const*, int, double, double,
                                              const double*, const double*, const double*,
                                              double*, int, hipStream_t);
template hipError_t launch_diagnostics<double>(const Dims&, double* const*, int, double, double,
                                               const double*, const double*, const double*,
                                               double*, int, hipStream_t);
template hipError_t launch_diagnostics_noalloc<float>(const Dims&, float* const*, int, double,
                                                      double, const double*, const double*,
                                                      const double*, const DiagFinish&, double*,
                                                      hipStream_t);
template hipError_t launch_diagnostics_noalloc<double>(const Dims&, double* const*, int, double,
                                                       double, const double*, const double*,
                                                       const double*, const DiagFinish&, double*,
                                                       hipStream_t);

}  // namespace oc
