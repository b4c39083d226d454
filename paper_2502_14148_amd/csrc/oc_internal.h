// Internal definitions shared by the HIP translation units of liboc.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "oc.h"

namespace oc {

constexpr int MAXF = 3 + OC_MAX_TRACERS;
constexpr int HMAX = 5;         // widest halo: the WENO9 stencil reaches 5 cells

// Halo width a model's advection scheme needs: the reach of its
// reconstruction (3 cells for WENO5, 4 for WENO7, 5 for WENO9).
inline int halo_width(int advection) {
  return advection == OC_ADV_WENO9Z || advection == OC_ADV_WENO9_LINEAR   ? 5
         : advection == OC_ADV_WENO7Z || advection == OC_ADV_WENO7_LINEAR ? 4
                                                                          : 3;
}

// Halo-padded layout: (nz + 2h) x (ny + 2h) x (nx + 2h), x fastest.
struct Dims {
  int nx, ny, nz;
  int px, py, pz;
  long sy, sz;     // strides of j and k in elements (x stride is 1)
  int zb;          // 1 if z is bounded by walls
  int h;           // halo width
};

// Every buffer the kernels address lives in device (global) memory.  Pointers
// that reach a kernel through a struct or a table are generic to the
// compiler, which then issues flat loads and stores: these count against the
// LDS counter too and stall LDS waits behind global traffic.  The cast makes
// them global operations.
template <class T>
__device__ inline __attribute__((address_space(1))) T* glb(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// double2 (a class type) cannot live in a qualified address space: complex
// values go through a native vector type.
typedef double oc_dbl2 __attribute__((ext_vector_type(2)));
__device__ inline double2 ld2(const double2* p, long i) {
  const oc_dbl2 v = ((const __attribute__((address_space(1))) oc_dbl2*)p)[i];
  return make_double2(v.x, v.y);
}
__device__ inline void st2(double2* p, long i, double2 x) {
  ((__attribute__((address_space(1))) oc_dbl2*)p)[i] = oc_dbl2{x.x, x.y};
}

// Four consecutive elements in one 16- (FP32) or 32-byte (FP64) load; the
// address need only be element-aligned.
template <class T>
using v4u = T __attribute__((ext_vector_type(4), aligned(sizeof(T))));
template <class T>
__device__ inline v4u<T> ld4(const T* p, long i) {
  return *(const __attribute__((address_space(1))) v4u<T>*)(p + i);
}

__host__ __device__ inline long pidx(const Dims& d, int i, int j, int k) {
  return (long)(k + d.h) * d.sz + (long)(j + d.h) * d.sy + (long)(i + d.h);
}

// Store a value at interior point (i, j, k) of a padded field and at its halo
// images: periodic wrap in x, y (and z when periodic); in a bounded z, an even
// mirror for data centred in z (wface = false) or an odd mirror about the
// wall faces for w (wface = true).  Wall faces of w are never images.  A
// point within h of both ends of a short axis has an image at each end.
// own = false: the images only (the caller stores the point itself).
template <class T>
__device__ inline void store_with_images(T* __restrict__ f, const Dims& d, int i, int j, int k,
                                         T val, bool wface, bool own = true) {
  const int H = d.h;
  // element offsets of the images along each axis (0: none; an image is
  // never at offset 0)
  const long xa = (i < H) ? d.nx : 0, xb = (i >= d.nx - H) ? -(long)d.nx : 0;
  const long ya = (j < H) ? d.ny * d.sy : 0, yb = (j >= d.ny - H) ? -(long)d.ny * d.sy : 0;
  long za = 0, zb = 0;
  T zs = T(1);
  if (!d.zb) {
    if (k < H) za = d.nz * d.sz;
    if (k >= d.nz - H) zb = -(long)d.nz * d.sz;
  } else if (!wface) {
    if (k < H) za = (long)(-1 - 2 * k) * d.sz;                // image -1 - k
    if (k >= d.nz - H) zb = (long)(2 * d.nz - 1 - 2 * k) * d.sz;  // image 2nz - 1 - k
  } else {
    zs = T(-1);
    if (k >= 1 && k <= H) za = (long)(-2 * k) * d.sz;          // image -k
    if (k >= d.nz - H + 1 && k <= d.nz - 1) zb = (long)(2 * d.nz - 2 * k) * d.sz;  // 2nz - k
  }
  auto* __restrict__ p0 = glb(f) + pidx(d, i, j, k);
  auto plane = [&](decltype(p0) q, T v, bool self) {
    if (self) q[0] = v;
    if (xa) q[xa] = v;
    if (xb) q[xb] = v;
    if (ya) {
      q[ya] = v;
      if (xa) q[ya + xa] = v;
      if (xb) q[ya + xb] = v;
    }
    if (yb) {
      q[yb] = v;
      if (xa) q[yb + xa] = v;
      if (xb) q[yb + xb] = v;
    }
  };
  plane(p0, val, own);
  if (za) plane(p0 + za, zs * val, true);
  if (zb) plane(p0 + zb, zs * val, true);
}

inline Dims make_dims(int nx, int ny, int nz, int zb, int h) {
  Dims d;
  d.nx = nx; d.ny = ny; d.nz = nz;
  d.h = h;
  d.px = nx + 2 * h; d.py = ny + 2 * h; d.pz = nz + 2 * h;
  d.sy = d.px; d.sz = (long)d.px * d.py;
  d.zb = zb;
  return d;
}

inline long padded_elems(const Dims& d) { return (long)d.px * d.py * d.pz; }

// Physics and RK3 coefficients handed to the tendency kernel.
template <class T>
struct TendParams {
  T rdx, rdy;                // inverse horizontal spacings
  // inverse vertical spacings (device tables): rdzc[k] = 1/dzc_k, the cell
  // thickness, valid for k = -1..nz (mirror images at -1 and nz);
  // rdzf[k] = 1/dzf_k, the distance between the centres about face k,
  // k = 0..nz.  Uniform grids hold 1/dz everywhere.
  const T* rdzc;
  const T* rdzf;
  T nu, kappa;               // horizontal (and explicit vertical) diffusion
  T nuz, kappaz;             // explicit vertical diffusion (0 when implicit)
  T f;
  T g_alpha, g_beta, t_ref, s_ref;
  int buoyancy;
  int ntr;                   // number of tracers
  T top_flux[OC_MAX_TRACERS];
  T toff[OC_MAX_TRACERS];    // tracer storage offsets (stored = value - toff)
  T eps;                     // WENO-Z regulariser
  T dt, gam, zet;            // RK3 substage coefficients (dt * ...)
  int stage;                 // 0, 1, 2
  int combine;               // 1: write X~ = X + dt(gam G - zet Gprev); 0: only G
  int images;                // 1: also write the halo images of the tracer outputs
};

template <class T>
struct FieldSet {
  const T* in[MAXF];
  T* out[MAXF];
  T* G[MAXF];
  const T* closure[MAXF];  // optional closure tendencies per field (learned
                           // closure: u, v, w, tracer 0; LES: every field),
                           // padded layout, added to G; null when off
  const T* mask;           // immersed boundary: 1 in fluid, 0 in immersed
                           // cells (padded, with halo images); null when off
  // Buffer addressing of the tendency kernels (set by fieldset_offsets):
  // every field above lies within 4 GiB of `base`; byte offsets from it.
  const char* base;
  uint32_t oin[MAXF], oout[MAXF], oG[MAXF], oclo[MAXF], omask;
};

// Fill the buffer-addressing members of fs: base = the lowest field pointer,
// offsets in bytes.  False if some field of `bytes` bytes (one padded field)
// does not end within 4 GiB of base.
template <class T>
inline bool fieldset_offsets(FieldSet<T>& fs, uint64_t bytes) {
  const char* lo = nullptr;
  auto see = [&](const void* p) {
    if (p && (!lo || (const char*)p < lo)) lo = (const char*)p;
  };
  for (int q = 0; q < MAXF; ++q) {
    see(fs.in[q]); see(fs.out[q]); see(fs.G[q]); see(fs.closure[q]);
  }
  see(fs.mask);
  if (!lo) return false;
  fs.base = lo;
  bool ok = true;
  auto off = [&](const void* p) -> uint32_t {
    if (!p) return 0u;
    const uint64_t o = (uint64_t)((const char*)p - lo);
    if (o + bytes > 0xFFFFFFFFull) ok = false;
    return (uint32_t)o;
  };
  for (int q = 0; q < MAXF; ++q) {
    fs.oin[q] = off(fs.in[q]);
    fs.oout[q] = off(fs.out[q]);
    fs.oG[q] = off(fs.G[q]);
    fs.oclo[q] = off(fs.closure[q]);
  }
  fs.omask = off(fs.mask);
  return ok;
}

// Spectral-solve tables and buffers (FP64).
struct SpecBufs {
  double2* spec;             // (nz, ny, nxp) half spectrum, kx fastest
  double* p;                 // (nz, ny, nx) pressure
  const double2* twx;        // exp(-2 pi i m / nx), m < nx
  const double2* twy;
  const double2* twz;
  const double2* dctz;       // exp(-i pi k / (2 nz)), k < nz (bounded z only)
  const double* lamx;        // eigenvalues of delta_x^2 / dx^2, k < nx
  const double* lamy;
  const double* lamz;
  int nxh;                   // nx / 2 + 1 stored wavenumbers
  int nxp;                   // row pitch: nxh rounded up to 8 (128-byte rows)
  const double* stop = nullptr;  // optional device flag: while *stop != 0 the
                                 // passes return at once (a converged iteration)
};

// Row pitch of the half spectrum in complex elements: column groups of 8 start
// on 128-byte boundaries, so the y and z passes fetch whole cache lines.
inline int spec_pitch(int nx) { return ((nx / 2 + 1) + 7) / 8 * 8; }

// 2D barotropic buffers and metric factors of the hydrostatic model (FP64,
// dense, x fastest; V-like arrays have ny + 1 rows).
struct BaroBufs {
  const double* eta;
  const double* U;
  const double* V;
  double* eta1;
  double* U1;
  double* V1;
  const double* GU;
  const double* GV;
  double* etab;
  double* Ub;
  double* Vb;
  const double* len_u;   // (ny)     length of an x face
  const double* dx_u;    // (ny)     centre distance across an x face
  const double* len_v;   // (ny + 1) length of a y face
  const double* dy_v;    // (ny + 1) centre distance across a y face
  const double* area;    // (ny)     cell area
  int nx, ny;
};

hipError_t launch_baro_fill(double* a, double v, long n, hipStream_t s);
hipError_t launch_baro_copy(double* dst, const double* src, long n, hipStream_t s);
// ns (1..baro_max_fused()) barotropic substeps in one launch, with the
// averaging weights wn[0..ns-1] (host array).
int baro_max_fused();
hipError_t launch_baro_substeps(const BaroBufs& b, double dtau, double gH, const double* wn,
                                int ns, hipStream_t s);
template <class T>
hipError_t launch_baro_correct(const Dims& d, T* f, const double* bar, int j_lo, int j_hi,
                               double dz, double depth, hipStream_t s);

// ---- Baroclinic step of the hydrostatic model
// Row tables of the lat-lon C-grid (FP64), index j + H for rows
// j = -H .. ny + H (the formulas continue past the walls).
struct HydroMetric {
  const double* dxc;     // R cos(phi_c(j)) dlambda: x spacing along row j
  const double* dxf;     // R cos(phi_f(j)) dlambda: x length of y face j
  const double* areac;   // area of the cells of row j
  const double* areaz;   // area of the dual cell around y face j
  const double* fc;      // 2 Omega sin(phi_c(j))
  const double* ff;      // 2 Omega sin(phi_f(j))
  double dy, dz;
};
constexpr int HYDRO_NMET = 6;

template <class T>
struct HydroBufs {
  Dims d;
  HydroMetric m;
  T eps, nu, kappa;
  T ga, gb, tref, sref;     // b = ga (T - tref) - gb (S - sref) on the stored values
  const T* u; const T* v; const T* t; const T* s;   // state at step n (halos filled)
  T* uo; T* vo; T* to; T* so;                       // predicted state (QAB2)
  T* Gu; T* Gv; T* Gt; T* Gs;                       // G^{n-1} in, G^n out
  T* w; T* zeta; T* px; T* py;                      // diagnostic fields
  const double* taux; const double* tauy;           // kinematic surface stress
  double* gub; double* gvb;                         // slow forcing of U, V
  double* gub1; double* gvb1;                       // partial sums of the upper levels
};

template <class T>
struct HydroStep {
  T dt, a1, a0;             // X~ = X + dt (a1 G^n - a0 G^{n-1})
  int first;                // 1: G^{n-1} is not read
  int kc;                   // levels per chunk (set by the launcher)
};

template <class T>
hipError_t launch_hydro_diag(const HydroBufs<T>& a, hipStream_t s);
template <class T>
hipError_t launch_hydro_tendency(const HydroBufs<T>& a, const HydroStep<T>& st, int scheme,
                                 hipStream_t s);
template <class T>
hipError_t launch_hydro_halo(const Dims& d, T* u, T* v, T* t, T* sf, hipStream_t s);

// ---- MLP closure (500 -> 256 -> 256 -> 4; device widths 512 and 32)
constexpr int MLP_NIN = 500, MLP_NH = 256, MLP_NOUT = 4, MLP_KIN = 512, MLP_NOUTP = 32;
constexpr int MLP_OFF_W1 = 0;
constexpr int MLP_OFF_B1 = MLP_OFF_W1 + MLP_NH * MLP_NIN;
constexpr int MLP_OFF_W2 = MLP_OFF_B1 + MLP_NH;
constexpr int MLP_OFF_B2 = MLP_OFF_W2 + MLP_NH * MLP_NH;
constexpr int MLP_OFF_W3 = MLP_OFF_B2 + MLP_NH;
constexpr int MLP_OFF_B3 = MLP_OFF_W3 + MLP_NOUT * MLP_NH;
constexpr int MLP_NPARAM = MLP_OFF_B3 + MLP_NOUT;

enum { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_GELU = 2, EPI_GELU_BWD = 3 };

struct GemmArgs {
  const __bf16* A;
  int lda, transA;          // transA = 0: A[m][k] at A[m*lda + k]; 1: at A[k*lda + m]
  const __bf16* B;
  int ldb, transB;          // transB = 0: B[k][n] at B[k*ldb + n]; 1: at B[n*ldb + k]
  int M, N, K;              // K a multiple of 32
  int epi;
  float* C;
  int ldc;
  const float* bias;        // EPI_BIAS, EPI_BIAS_GELU
  const float* Z;           // EPI_GELU_BWD: pre-activation, same layout as C
  __bf16* H;                // EPI_BIAS_GELU / EPI_GELU_BWD: BF16 copy of the result
  int ldh;
  int ksplit;               // > 1: K split over blockIdx.z (EPI_STORE only), partial
  float* part;              // results in part[z][M][N], summed in z order into C
};
constexpr int MLP_MAX_KSPLIT = 64;
// FP32 scratch of the split-K partials and the column-sum partials
constexpr long MLP_PART_FLOATS = (long)MLP_MAX_KSPLIT * MLP_NH * MLP_KIN;
constexpr int COLSUM_MAX_CHUNKS = 256;

struct MlpParams {
  float* master;            // FP32: W1 | b1 | W2 | b2 | W3 | b3
  __bf16* W1b;              // 256 x 512 (columns >= 500 zero)
  __bf16* W2b;              // 256 x 256
  __bf16* W2bT;             // its transpose (backward pass)
  __bf16* W3b;              // 32 x 256 (rows >= 4 zero)
};

__device__ void mlp_write_bf16(const MlpParams& p, int t, float w);
hipError_t launch_gemm_bf16(const GemmArgs& g, hipStream_t s);
hipError_t launch_loss_grad(const float* Y, int ldy, const float* T, int B, float* dY, __bf16* dYb,
                            int ldd, double* partial, int nblocks, hipStream_t s);
hipError_t launch_colsum(const float* a, int rows, int cols, int lda, float* out, float* part,
                         hipStream_t s);
hipError_t launch_features_to_bf16(const float* x, int B, __bf16* xb, hipStream_t s);
hipError_t launch_adam(const MlpParams& p, const float* grad, float* m1, float* m2, int n, float lr,
                       int step, hipStream_t s);
hipError_t launch_refresh_bf16(const MlpParams& p, int n, hipStream_t s);

// Closure statistics: input mean/std of (u, v, w, b), output mean/std of the
// four fluxes; buoyancy parameters to form b from the stored T, S.
struct ClosureStats {
  float in_mean[4], in_std[4], out_mean[4], out_std[4];
  float in_rstd[4];                      // 1 / in_std
  float g_alpha, g_beta, t_ref, s_ref;   // b = g_alpha (T - t_ref) - g_beta (S - s_ref)
  float inv_galpha;                      // temperature flux = buoyancy flux / (g alpha)
};
template <class T>
hipError_t launch_closure_features(const Dims& d, const T* u, const T* v, const T* w, const T* t,
                                   const T* s, ClosureStats st, __bf16* xb, hipStream_t stream);
template <class T>
hipError_t launch_closure_apply(const Dims& d, const float* y, ClosureStats st, double rdz,
                                T* gu, T* gv, T* gw, T* gt, hipStream_t stream);

template <class T>
hipError_t launch_closure_mlp_fused(const Dims& d, const T* u, const T* v, const T* w, const T* t,
                                    const T* s, ClosureStats st, const MlpParams& p, float* y,
                                    hipStream_t stream);
template <class T>
hipError_t launch_closure_features_f32(const Dims& d, const T* u, const T* v, const T* w,
                                       const T* t, const T* s, ClosureStats st, float* x,
                                       hipStream_t stream);

// Coarse-graining of a fine state (halos filled) onto a grid r times coarser.
template <class T>
struct CoarseArgs {
  Dims df, dc;
  int r;
  const T* u; const T* v; const T* w; const T* t; const T* s;   // fine
  T* U; T* V; T* W; T* Tc; T* Sc;                               // coarse (interior written)
  float* flux;          // (4, nzc, nyc, nxc) subgrid fluxes, or null
  double ga, gb, tref, sref;   // b = ga (T - tref) - gb (S - sref) on stored values
};
template <class T>
hipError_t launch_coarse_grain(const CoarseArgs<T>& a, hipStream_t s);

// Access to a network from the model's step (implemented in closure_api.hip).
__bf16* mlp_input(oc_mlp* net);
const float* mlp_output(oc_mlp* net);
float* mlp_output_rw(oc_mlp* net);
const MlpParams& mlp_params(const oc_mlp* net);
int mlp_max_batch(const oc_mlp* net);
int mlp_run_forward(oc_mlp* net, int batch, hipStream_t s);
int mlp_params_finite(oc_mlp* net, hipStream_t s);  // 1, 0, or a negative error

// Host-side error reporting (per thread).
void set_error(const char* fmt, ...);

// Kernel launchers (defined in the .hip translation units).
template <class T>
hipError_t launch_halo_fill(const Dims& d, T* const* fields, const int* kinds, int nf,
                            hipStream_t s);
// Fused tendency (+ RK3 combine) of one model; advection is OC_ADV_*.
template <class T>
hipError_t launch_tendency_fast(const Dims& d, const FieldSet<T>& fs, const TendParams<T>& p,
                                int advection, hipStream_t s);
// Spacings of the pressure passes: rdzc (nz) and rdzf (nz + 1) are device
// tables of 1/dzc_k and 1/dzf_k as in TendParams.
struct Spacing {
  double rdx, rdy;
  const double* rdzc;
  const double* rdzf;
};

// ---- Ensembles: one tendency launch for many models
// Member descriptor (device table): the state pointers for both buffer
// parities and the tendency parameters of the three RK3 substages.
template <class T>
struct EnsMember {
  Dims d;
  int nbx, nby, nbz, kc;     // column tiles and k chunks of this member
  FieldSet<T> fs[2];         // parity 0: in = A, out = B; parity 1: swapped
  TendParams<T> P[3];
};
// Launch configuration picked by the autotuner: tile 0 = 32 x 8, 1 = 16 x 8,
// 2 = 8 x 8 columns; persistent grid of nblocks workgroups or one per item.
struct EnsTuning {
  int tile;
  int persistent;
  int nblocks;
  int kc_div;
};
constexpr int ENS_TILE_X[3] = {32, 16, 8};
constexpr int ENS_TILE_Y[3] = {8, 8, 8};
template <class T>
hipError_t launch_tendency_ensemble(const EnsMember<T>* mem, const int2* items, int nitems,
                                   int* counter, int parity, int stage, const EnsTuning& tn,
                                   hipStream_t s);

template <class T>
int ensemble_blocks_per_cu(int tile);

// Per-member pointers of a batched Poisson launch (member = blockIdx.z).
constexpr int ENS_MAX_SLOTS = 64;
struct PoissonSlots {
  void* u[ENS_MAX_SLOTS];
  void* v[ENS_MAX_SLOTS];
  void* w[ENS_MAX_SLOTS];
  double2* spec[ENS_MAX_SLOTS];
  double* p[ENS_MAX_SLOTS];
};
template <class T>
hipError_t launch_poisson_x_forward(const Dims& d, const T* u, const T* v, const T* w,
                                   double inv_dt, Spacing sp, const SpecBufs& sb, hipStream_t s,
                                   const PoissonSlots* bs = nullptr, int nslots = 1);
// bs (device table, may be null): nslots members of identical dims and tables
// transformed in one launch, member z taking its pointers from slot z
hipError_t launch_poisson_y(const Dims& d, const SpecBufs& sb, int dir, hipStream_t s,
                            const PoissonSlots* bs = nullptr, int nslots = 1);
hipError_t launch_poisson_spectral(const Dims& d, const SpecBufs& sb, hipStream_t s,
                                   const PoissonSlots* bs = nullptr, int nslots = 1);
hipError_t launch_poisson_x_inverse(const Dims& d, const SpecBufs& sb, hipStream_t s,
                                    const PoissonSlots* bs = nullptr, int nslots = 1);
template <class T>
hipError_t launch_project(const Dims& d, T* u, T* v, T* w, double scale, const Spacing& sp,
                          const double* p, hipStream_t s, const PoissonSlots* bs = nullptr,
                          int nslots = 1, const T* mask = nullptr);
// The inverse x pass fused with the projection: u, v, w -= scale grad p with
// p taken from sb.spec on the fly; sb.p is not written (launch
// launch_poisson_x_inverse on the same spectrum for it).
template <class T>
hipError_t launch_poisson_x_inverse_project(const Dims& d, const SpecBufs& sb, T* u, T* v, T* w,
                                            double scale, const Spacing& sp, hipStream_t s,
                                            const PoissonSlots* bs = nullptr, int nslots = 1);
// The forward x transform of a dense FP64 (nz, ny, nx) field into sb.spec
// (the first pass of the FFT solve applied to a given right-hand side).
hipError_t launch_poisson_x_forward_dense(const Dims& d, const double* src, const SpecBufs& sb,
                                          hipStream_t s);
// The inverse x pass that also leaves partial sums of rdot . p (one per
// workgroup, *npart of them, at most part_cap) in part.
hipError_t launch_poisson_x_inverse_dot(const Dims& d, const SpecBufs& sb, const double* rdot,
                                        double* part, int part_cap, int* npart, hipStream_t s);

// ---- Immersed boundaries (immersed.hip): preconditioned conjugate gradients
// on dense FP64 (nz, ny, nx) vectors.  Reducing kernels run IB_NPART
// workgroups and leave one partial sum each in part; launch_ib_finalize adds
// them in a fixed order and updates the scalars in scal (indices CG_*).
constexpr int IB_NPART = 4096;
constexpr int IB_PART_CAP = 16384;   // room for the partials of the fused inverse pass
enum { CG_RZ = 0, CG_ALPHA, CG_BETA, CG_BNORM2, CG_RNORM2, CG_IT, CG_DONE, CG_MEAN, CG_NSCAL };
enum { CG_FIN_BNORM = 0, CG_FIN_RZ0, CG_FIN_ALPHA, CG_FIN_RES, CG_FIN_BETA, CG_FIN_MEAN };
struct CgBufs {
  double* x;     // iterate (the pressure)
  double* r;     // residual
  double* q;     // search direction
  double* aq;    // A q
  double* part;  // IB_NPART partial sums
  double* scal;  // CG_NSCAL scalars
};
// Per-cell geometry byte (dense, x fastest): the cell is fluid, and which of
// its faces are open (both neighbours fluid; walls closed).
enum { IB_XM = 1, IB_XP = 2, IB_YM = 4, IB_YP = 8, IB_ZM = 16, IB_ZP = 32, IB_FLUID = 64 };
template <class T>
hipError_t launch_ib_rhs(const Dims& d, const T* u, const T* v, const T* w,
                         const uint8_t* bits, double inv_dt, double rdx, double rdy, double rdz,
                         const CgBufs& cg, hipStream_t s);
hipError_t launch_ib_apply(const Dims& d, const uint8_t* bits, double rdx2, double rdy2,
                           double rdz2, const CgBufs& cg, hipStream_t s);
hipError_t launch_ib_update(const Dims& d, const CgBufs& cg, hipStream_t s);
hipError_t launch_ib_dir(const Dims& d, const uint8_t* bits, const CgBufs& cg, const double* z,
                         hipStream_t s);
hipError_t launch_ib_gauge(const Dims& d, const uint8_t* bits, const CgBufs& cg, double nfluid,
                           hipStream_t s);
hipError_t launch_ib_finalize(const CgBufs& cg, int what, double tol2, int maxiter,
                              hipStream_t s, int npart = IB_NPART);
hipError_t launch_ib_xfinal(const Dims& d, const CgBufs& cg, hipStream_t s);
template <class T>
hipError_t launch_ib_mask_velocity(const Dims& d, T* u, T* v, T* w, const T* mask,
                                   hipStream_t s);
// Stretched z: the tridiagonal solve along z of every (kx, ky) mode in place
// of the z transform pass; lo, up (nz) are the off-diagonals of the vertical
// operator, dzc (nz) the cell thicknesses and dzf (nz + 1) the centre
// distances about the faces (the horizontally uniform mode is integrated).
hipError_t launch_poisson_tridiag(const Dims& d, const SpecBufs& sb, const double* lo,
                                  const double* up, const double* dzc, const double* dzf,
                                  hipStream_t s);
// Implicit vertical diffusion of several fields in place (one launch, field
// = blockIdx.y): fac[q] holds the recurrence tables of vertical_factors for
// field q's matrix; wface[q] selects w on the interior faces 1..nz-1,
// otherwise the nz centres.  Needs bounded z and nz <= 256.
// Eddy-viscosity LES closure of one substage (les.hip): inputs, the
// viscosity (and AMD's per-tracer diffusivity) buffers written with halo
// images, and the closure tendencies gc[f] (padded layout, interior).
template <class T>
struct LesArgs {
  const T* u;
  const T* v;
  const T* w;
  const T* c0;               // T and S (Smagorinsky-Lilly buoyancy)
  const T* c1;
  const T* tr[OC_MAX_TRACERS];
  int ntr;
  T* nu;
  T* kap[OC_MAX_TRACERS];    // AMD; null for Smagorinsky-Lilly (kappa = nu/Pr)
  T* gc[MAXF];
  T rdx, rdy;
  const T* rdzc;             // as in TendParams
  const T* rdzf;
  const T* delta2;           // Smagorinsky-Lilly: (C_s Delta_k)^2 per level
  T cb, camd, rpr;
  int buoyancy;
  T g_alpha, g_beta, t_ref, s_ref;
};
template <class T>
hipError_t launch_les(const Dims& d, const LesArgs<T>& a, int kind, hipStream_t s);

template <class T>
struct VImplicitArgs {
  T* f[MAXF];
  const T* fac[MAXF];
  int wface[MAXF];
};
template <class T>
hipError_t launch_vertical_implicit(const Dims& d, const VImplicitArgs<T>& a, int nfields,
                                    hipStream_t s);
// Host: the tables of the implicit solve of 1 - dt L for the vertical
// diffusion operator L with coefficient K (no flux through the walls for
// centred fields; w = 0 on the walls for wface): A, I, P, B, Q rows of n
// values (n = nz, or nz - 1 for wface) and the per-chunk products PE, QS;
// vertical_factors_len(nz) values in all.
void vertical_factors(const double* dzc, const double* dzf, int nz, double K, double dt,
                      int wface, double* out);
int vertical_factors_len(int nz);
template <class T>
hipError_t launch_pack(const Dims& d, int nzf, int nyf, const T* padded, void* dense, int dtype,
                       int to_dense, double offset, hipStream_t s);
// Diagnostics partials per workgroup or level, and the levels the
// allocation-free variant's scratch array holds.
constexpr int DIAG_NPART = 12;
constexpr int DIAG_MAX_LEVELS = 256;
// Host constants that finish the diagnostics on the device.
struct DiagFinish {
  double hmin, area, rdx, rdy, rdzmin;
  double toff[4];   // storage offset x cells x dz per tracer (0 if absent)
};
template <class T>
hipError_t launch_diagnostics_noalloc(const Dims& d, T* const* fields, int nf, double rdx,
                                      double rdy, const double* rdzc, const double* dzc,
                                      const double* dzf, const DiagFinish& f, double* out,
                                      hipStream_t s);
template <class T>
hipError_t launch_diagnostics(const Dims& d, T* const* fields, int nf, double rdx, double rdy,
                              const double* rdzc, const double* dzc, const double* dzf,
                              double* scratch, int nblocks, hipStream_t s);

bool fft_length_supported(int n);

}  // namespace oc
