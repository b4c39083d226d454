// Split-explicit barotropic substeps of the hydrostatic model on gfx950
// (hydrostatic time-discretisation appendix of arXiv 2502.14148).
//
// A launch advances up to BHS substeps (temporal blocking, below); it reads
// (eta, U, V)^n from one buffer set and writes the state after its last
// substep to the other.  Each workgroup recomputes the substeps on a halo
// around its tile, so neither the forward (eta) and backward (U, V) halves
// of a substep nor successive substeps need a grid-wide barrier.  The
// running averages are accumulated in place in FP64.  All 2D arrays are
// dense FP64, x fastest; x is periodic, y has walls (V = 0 on faces 0 and
// ny).
#include "oc_internal.h"

namespace oc {

namespace {

// Own tile of a workgroup (one cell per thread) and the substeps per launch:
// on the 1440 x 560 sector, 32 x 32 tiles took 0.82 ms per 59 substeps (plus
// correction and restart) with 6 substeps per launch, 0.83 with 5, 0.86
// with 4; 32 x 16 tiles 0.95 and 32 x 8 tiles 1.10 with 4.
constexpr int BTX = 32, BTY = 32;

// Up to BHS substeps in one launch (temporal blocking).  A workgroup owns a
// BTX x BTY tile and stages eta, U, V, GU, GV on the tile widened by BHS
// cells on every side (plus the U column and V row beyond) in LDS.  Each
// substep is valid on a region one cell narrower per side than the last
// (eta needs U, V one cell right/above; U, V need eta one cell left/below),
// so after ns <= BHS substeps the own tile is exact.  Rows outside the
// domain hold zeros and the wall faces V(0), V(ny) stay zero; x wraps
// periodically.  The running averages of the own cells take the substeps'
// terms one at a time, in substep order.
constexpr int BHS = 6;
constexpr int BEX = BTX + 2 * BHS, BEY = BTY + 2 * BHS;   // widened tile
constexpr int BPX = BEX + 1, BPY = BEY + 1;               // + U column, V row
struct BaroWeights {
  double w[BHS];
};

__global__ void __launch_bounds__(BTX * BTY) baro_multi_kernel(BaroBufs b, double dtau,
                                                               double gH, BaroWeights wts,
                                                               int ns) {
  __shared__ double E[BPY][BPX], Us[BPY][BPX], Vs[BPY][BPX], Gu[BPY][BPX], Gv[BPY][BPX];
  const int i0 = blockIdx.x * BTX - BHS, j0 = blockIdx.y * BTY - BHS;   // corner of the widened tile
  const int tid = threadIdx.x;
  for (int e = tid; e < BPX * BPY; e += BTX * BTY) {
    const int y = e / BPX, x = e - y * BPX;
    int gi = (i0 + x) % b.nx;
    if (gi < 0) gi += b.nx;
    const int gj = j0 + y;
    double ev = 0.0, uv = 0.0, vv = 0.0, gu = 0.0, gv = 0.0;
    if (gj >= 0 && gj < b.ny) {
      const long c = (long)gj * b.nx + gi;
      ev = b.eta[c];
      uv = b.U[c];
      gu = b.GU[c];
      if (gj > 0) {
        vv = b.V[c];
        gv = b.GV[c];
      }
    }
    E[y][x] = ev;
    Us[y][x] = uv;
    Vs[y][x] = vv;
    Gu[y][x] = gu;
    Gv[y][x] = gv;
  }
  // own cell of this thread and its running averages
  const int tx = tid % BTX, ty = tid / BTX;
  const int oi = i0 + BHS + tx, oj = j0 + BHS + ty;
  const bool own = oi < b.nx && oj < b.ny;
  const long oc = (long)oj * b.nx + oi;
  double ea = 0.0, ua = 0.0, va = 0.0;
  if (own) {
    ea = b.etab[oc];
    ua = b.Ub[oc];
    va = b.Vb[oc];
  }
  __syncthreads();
  for (int sstep = 0; sstep < ns; ++sstep) {
    // eta^{n+1} = eta^n - dtau div(U^n, V^n) on rows 0..BEY-1, columns 0..BEX-1
    for (int e = tid; e < BEX * BEY; e += BTX * BTY) {
      const int y = e / BEX, x = e - y * BEX;
      const int gj = j0 + y;
      if (gj >= 0 && gj < b.ny) {
        const double fx = b.len_u[gj] * (Us[y][x + 1] - Us[y][x]);
        const double fy = b.len_v[gj + 1] * Vs[y + 1][x] - b.len_v[gj] * Vs[y][x];
        E[y][x] = E[y][x] - dtau * ((fx + fy) / b.area[gj]);
      }
    }
    __syncthreads();
    // eta is not written again before the next substep's first barrier
    const double wn = wts.w[sstep];
    if (own) ea += wn * E[BHS + ty][BHS + tx];
    // U^{n+1}, V^{n+1} from eta^{n+1} (columns / rows 1.. of the widened tile)
    for (int e = tid; e < BEX * BEY; e += BTX * BTY) {
      const int y = e / BEX, x = e - y * BEX;
      const int gj = j0 + y;
      if (gj >= 0 && gj < b.ny) {
        const double en = E[y][x];
        if (x > 0) Us[y][x] = Us[y][x] - dtau * (gH * (en - E[y][x - 1]) / b.dx_u[gj] - Gu[y][x]);
        if (y > 0)
          Vs[y][x] = (gj > 0)
                         ? Vs[y][x] - dtau * (gH * (en - E[y - 1][x]) / b.dy_v[gj] - Gv[y][x])
                         : 0.0;
      }
    }
    __syncthreads();
    // U and V are not written again before the next substep's second barrier
    if (own) {
      ua += wn * Us[BHS + ty][BHS + tx];
      va += wn * Vs[BHS + ty][BHS + tx];
    }
  }
  if (!own) return;
  b.eta1[oc] = E[BHS + ty][BHS + tx];
  b.U1[oc] = Us[BHS + ty][BHS + tx];
  b.V1[oc] = Vs[BHS + ty][BHS + tx];
  b.etab[oc] = ea;
  b.Ub[oc] = ua;
  b.Vb[oc] = va;
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
  // levels fetched CKB at a time so that their loads are in flight together
  constexpr int CKB = 10;
  double sum = 0.0;
  for (int k0 = 0; k0 < d.nz; k0 += CKB) {
    T x[CKB];
#pragma unroll
    for (int q = 0; q < CKB; ++q) x[q] = f[c0 + (long)min(k0 + q, d.nz - 1) * d.sz];
#pragma unroll
    for (int q = 0; q < CKB; ++q)
      if (k0 + q < d.nz) sum += (double)x[q];
  }
  const double corr = (bar[(long)j * d.nx + i] - dz * sum) * inv_h;
  for (int k0 = 0; k0 < d.nz; k0 += CKB) {
    T x[CKB];
#pragma unroll
    for (int q = 0; q < CKB; ++q) x[q] = f[c0 + (long)min(k0 + q, d.nz - 1) * d.sz];
#pragma unroll
    for (int q = 0; q < CKB; ++q)
      if (k0 + q < d.nz) f[c0 + (long)(k0 + q) * d.sz] = (T)((double)x[q] + corr);
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

int baro_max_fused() { return BHS; }

hipError_t launch_baro_substeps(const BaroBufs& b, double dtau, double gH, const double* wn,
                                int ns, hipStream_t s) {
  if (ns < 1 || ns > BHS) return hipErrorInvalidValue;
  BaroWeights w{};
  for (int q = 0; q < ns; ++q) w.w[q] = wn[q];
  dim3 grid((b.nx + BTX - 1) / BTX, (b.ny + BTY - 1) / BTY);
  hipLaunchKernelGGL(baro_multi_kernel, grid, dim3(BTX * BTY), 0, s, b, dtau, gH, w, ns);
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
