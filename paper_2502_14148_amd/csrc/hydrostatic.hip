// Baroclinic part of the hydrostatic model on a latitude-longitude grid
// (hydrostatic-model subsection and hydrostatic time-discretisation appendix
// of arXiv 2502.14148) on gfx950.
//
// Discretisation (C-grid on the thin spherical shell, uniform dz, periodic
// longitude, walls at the latitude edges and in z):
//   * w at z faces from the floor up, w_{k+1} = w_k - dz div_h(u_h)_k;
//   * hydrostatic pressure p_k = -dz (b_k / 2 + sum_{m > k} b_m) (dp/dz = b,
//     p = 0 at the surface); only its horizontal differences enter, so the
//     columns integrate differences of b;
//   * vector-invariant momentum advection: vertical vorticity zeta at cell
//     corners from the metric circulation of the dual cell; + zeta_hat Vbar at
//     u points (zeta reconstructed by WENO along y, upwinded by the
//     four-point average Vbar of v), - zeta_hat Ubar at v points (along x);
//     kinetic energy at centres differenced to the faces; vertical advection
//     d(W q)/dz - q dW/dz with W = w averaged to the column and q
//     reconstructed by WENO along z;
//   * tracers in flux form with the shell's face areas and cell volumes,
//     WENO in every direction;
//   * f = 2 Omega sin(latitude of the point) times the four-point average of
//     the other component; explicit vertical viscosity/diffusivity with the
//     kinematic wind stress as surface momentum flux;
//   * advective fluxes vanish on the floor; through the moving surface they
//     carry the top cell's own value (a uniform tracer stays uniform);
//   * QAB2: X~ = X + dt [(3/2 + chi) G^n - (1/2 + chi) G^{n-1}], chi = 0.1
//     (chi = -1/2 on a first step), and the slow forcing of the barotropic
//     mode Gbar = sum_k dz [...] accumulated in FP64 per column.
//
// Layout: halo-padded fields (halo width h = 3), x fastest; v on the ny + 1 y faces (face
// ny in the first upper halo row), w on the nz + 1 z faces (face nz in the
// first upper halo plane).  Kernels: the column scans (zeta, w, pressure
// gradients), the tendency + QAB2 kernel (column tiles marching up the
// levels with horizontally staged planes in LDS and register windows along
// z), and the halo fill of the prognostic fields.
#include "oc_internal.h"
#include "weno_dev.h"
#include "gaddr.h"

namespace oc {

namespace {

constexpr int HTX = 64, HTY = 4;
// Levels whose loads the column scans issue together (the scans store
// between levels, so without batching every level would wait on its own
// loads).
constexpr int DKB = 8;

// Column scans over the columns i, j in [-2, n + 2] (what the tendency
// kernel reads of zeta and w).  Workgroups are renumbered XCD-contiguous
// (x fastest), so the neighbouring rows a column reads were fetched into the
// same L2 by the workgroups just before it.
template <class T>
__global__ void __launch_bounds__(HTX * HTY) hydro_diag_kernel(HydroBufs<T> a) {
  const Dims d = a.d;
  const int nbx = (d.nx + 5 + HTX - 1) / HTX;
  const int n = (int)gridDim.x, b = (int)blockIdx.x;
  const int q = n / 8, r = n % 8, x8 = b % 8;
  const int t = x8 * q + min(x8, r) + b / 8;
  const int i = -2 + (t % nbx) * HTX + (int)threadIdx.x;
  const int j = -2 + (t / nbx) * HTY + (int)threadIdx.y;
  if (i > d.nx + 2 || j > d.ny + 2) return;
  const HydroMetric& m = a.m;
  const T dy = (T)m.dy;
  const double dz = m.dz;
  const long sy = d.sy, sz = d.sz;
  const long c0 = pidx(d, i, j, 0);

  // vertical vorticity at corner (x face i, y face j) and, on the columns
  // i in [-1, nx), j in [0, ny), w on the faces from the floor up: one pass
  // over the levels, so that u and v are fetched once for both
  {
    const T dxj = (T)m.dxc[j + d.h], dxjm = (T)m.dxc[j - 1 + d.h];
    const T rza = T(1) / (T)m.areaz[j + d.h];
    const bool wcol = i >= -1 && i < d.nx && j >= 0 && j < d.ny;
    const int jw = wcol ? j : 0;   // metric row of w (any valid row elsewhere)
    const T dxf0 = (T)m.dxf[jw + d.h], dxf1 = (T)m.dxf[jw + 1 + d.h];
    const T rar = T(1) / (T)m.areac[jw + d.h];
    double wacc = 0.0;
    if (wcol) a.w[c0] = T(0);
    for (int k0 = 0; k0 < d.nz; k0 += DKB) {
      T v0[DKB], v1[DKB], u0[DKB], u1[DKB], ue[DKB], vn[DKB];
#pragma unroll
      for (int q = 0; q < DKB; ++q) {
        const long c = c0 + (long)min(k0 + q, d.nz - 1) * sz;
        v0[q] = a.v[c]; v1[q] = a.v[c - 1]; u0[q] = a.u[c]; u1[q] = a.u[c - sy];
        ue[q] = wcol ? a.u[c + 1] : T(0);
        vn[q] = wcol ? a.v[c + sy] : T(0);
      }
#pragma unroll
      for (int q = 0; q < DKB; ++q) {
        if (k0 + q < d.nz) {
          const T circ = dy * (v0[q] - v1[q]) - (dxj * u0[q] - dxjm * u1[q]);
          a.zeta[c0 + (long)(k0 + q) * sz] = circ * rza;
          if (wcol) {
            const T div = (dy * (ue[q] - u0[q]) + (dxf1 * vn[q] - dxf0 * v0[q])) * rar;
            wacc -= dz * (double)div;
            a.w[c0 + (long)(k0 + q + 1) * sz] = (T)wacc;
          }
        }
      }
    }
  }

  // pressure-gradient terms, integrated from the surface down:
  //   px = (p_i - p_{i-1}) / dx at u points, py = (p_j - p_{j-1}) / dy at v points
  if (i >= 0 && i < d.nx && j >= 0 && j < d.ny) {
    const T rdx = T(1) / (T)m.dxc[j + d.h];
    const T rdy = T(1) / dy;
    const bool vpt = j > 0;
    double sx = 0.0, sy_ = 0.0;
    for (int k1 = d.nz - 1; k1 >= 0; k1 -= DKB) {
      T tc[DKB], sc[DKB], tw[DKB], sw[DKB], ts[DKB], ss[DKB];
#pragma unroll
      for (int q = 0; q < DKB; ++q) {
        const long c = c0 + (long)max(k1 - q, 0) * sz;
        tc[q] = a.t[c]; sc[q] = a.s[c]; tw[q] = a.t[c - 1]; sw[q] = a.s[c - 1];
        ts[q] = a.t[c - sy]; ss[q] = a.s[c - sy];
      }
#pragma unroll
      for (int q = 0; q < DKB; ++q) {
        if (k1 - q >= 0) {
          const long c = c0 + (long)(k1 - q) * sz;
          const T b = a.ga * (tc[q] - a.tref) - a.gb * (sc[q] - a.sref);
          const T bw = a.ga * (tw[q] - a.tref) - a.gb * (sw[q] - a.sref);
          const double dbx = (double)(b - bw);
          a.px[c] = (T)(-dz * (0.5 * dbx + sx)) * rdx;
          sx += dbx;
          if (vpt) {
            const T bs = a.ga * (ts[q] - a.tref) - a.gb * (ss[q] - a.sref);
            const double dby = (double)(b - bs);
            a.py[c] = (T)(-dz * (0.5 * dby + sy_)) * rdy;
            sy_ += dby;
          }
        }
      }
    }
  }
}

template <class T, int SCHEME>
__device__ inline T rec(T m3, T m2, T m1, T p0, T p1, T p2, T vel, T eps) {
  if (SCHEME == tz::SCHEME_NONE) return T(0);
  return tz::rec6<T, SCHEME>(m3, m2, m1, p0, p1, p2, vel, eps);
}

// Tendency + QAB2 kernel: 32 x 8 column tiles marching up the levels.  At
// each level the workgroup stages the planes it reads horizontally (T, S
// with three halo cells, zeta, u, v and w on face k + 1) in LDS (two
// buffers: the next level's planes are copied in by the buffer unit while
// this level computes), computes every tracer face flux of the tile once (the
// east and north edge faces in a second round by the first wavefront) and
// then the cell, u-point and v-point tendencies.  Vertical reconstructions
// use per-thread register windows along z, and the fluxes through the lower
// face are carried up from the level below.
constexpr int TTX = 32, TTY = 8;
constexpr int P_TX = TTX + 6, P_TY = TTY + 6;       // T, S: x, y in [-3, T + 2]
constexpr int P_ZX = TTX + 5, P_ZY = TTY + 5;       // zeta: [-2, T + 2]
constexpr int P_UX = TTX + 2, P_UY = TTY + 1;       // u: x in [-1, TTX], y in [-1, TTY)
constexpr int P_VX = TTX + 1, P_VY = TTY + 2;       // v: x in [-1, TTX), y in [-1, TTY]
constexpr int P_WX = TTX + 1, P_WY = TTY + 1;       // w: x, y in [-1, T)
constexpr int F_X = (TTX + 1) * TTY, F_Y = TTX * (TTY + 1);   // per tracer

// Tile of workgroup blockIdx.x: workgroups are dealt round-robin to the 8
// XCDs; renumbering gives each XCD a contiguous run of tiles (x fastest),
// so the halo rows shared by neighbouring tiles stay in one L2.
__device__ inline int hydro_tile_index() {
  const int n = (int)gridDim.x, b = (int)blockIdx.x;
  const int q = n / 8, r = n % 8, x = b % 8;
  return x * q + min(x, r) + b / 8;
}

constexpr int TNT = TTX * TTY;

// Load-to-LDS copy of a W x H box of a padded field (NT = TNT threads,
// elements of ES bytes): dword j of the box lands in LDS dword j, copied by
// the buffer unit itself (one dword per lane, 64 consecutive dwords per
// wave), so the staging costs neither registers nor vector instructions
// after the per-lane offsets are set up once per tile.  Full rounds of TNT
// dwords, then 64-dword chunks dealt to the waves; points past the padded
// upper edges copy the last valid point into entries that are never read.
// LEN: the box's padded length in elements.
template <int W, int H, int ES>
struct BoxCopy {
  static constexpr int DPE = ES / 4, D = W * H * DPE;
  static constexpr int NR = D / TNT, REM = D - NR * TNT, NCH = (REM + 63) / 64;
  static constexpr int NWV = TNT / 64, MAXC = (NCH + NWV - 1) / NWV;
  static constexpr int LEN = (NR * TNT + NCH * 64) / DPE;
  uint32_t off[NR + MAXC];

  // x <= imax and y <= jmax: the box points inside the padded field
  __device__ inline void init(int sy, int imax, int jmax, int tid, int wave, int lane) {
    auto at_dword = [&](int j) -> uint32_t {
      if (j > D - 1) j = D - 1;
      const int e = j / DPE, half = j - e * DPE;
      const int y = min(e / W, jmax), x = min(e % W, imax);
      return (uint32_t)((y * sy + x) * ES + half * 4);
    };
#pragma unroll
    for (int r = 0; r < NR; ++r) off[r] = at_dword(r * TNT + tid);
#pragma unroll
    for (int c = 0; c < MAXC; ++c) off[NR + c] = at_dword(NR * TNT + (wave + c * NWV) * 64 + lane);
  }

  // copy the box whose first point is at `base` into LDS at dst
  template <class T>
  __device__ inline void issue(const T* base, T* dst, int wave) const {
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)0xFFFFFFFF, 0x00020000);
#pragma unroll
    for (int q = 0; q < NR; ++q)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (void*)(dst + (q * TNT + wave * 64) / DPE), 4,
                                               off[q], 0, 0, 0);
#pragma unroll
    for (int c = 0; c < MAXC; ++c) {
      const int ch = wave + c * NWV;
      if (ch < NCH)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (void*)(dst + (NR * TNT + ch * 64) / DPE), 4,
                                                 off[NR + c], 0, 0, 0);
    }
  }
};

// The copies of one level's staged planes (T, S share a shape) and their
// places in an LDS level buffer.
template <class T>
struct StageCopy {
  static constexpr int ES = (int)sizeof(T);
  BoxCopy<P_TX, P_TY, ES> ts;
  BoxCopy<P_ZX, P_ZY, ES> z;
  BoxCopy<P_UX, P_UY, ES> u;
  BoxCopy<P_VX, P_VY, ES> v;
  BoxCopy<P_WX, P_WY, ES> w;
  static constexpr int L_T = 0, L_S = L_T + BoxCopy<P_TX, P_TY, ES>::LEN;
  static constexpr int L_Z = L_S + BoxCopy<P_TX, P_TY, ES>::LEN;
  static constexpr int L_U = L_Z + BoxCopy<P_ZX, P_ZY, ES>::LEN;
  static constexpr int L_V = L_U + BoxCopy<P_UX, P_UY, ES>::LEN;
  static constexpr int L_W = L_V + BoxCopy<P_VX, P_VY, ES>::LEN;
  static constexpr int LEN = L_W + BoxCopy<P_WX, P_WY, ES>::LEN;
};

// Wait for this wave's outstanding vector-memory operations (the
// load-to-LDS copies among them).
__device__ inline void wait_vm() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// FP32: registers capped for five wavefronts per SIMD (a few spilled values,
// 4 % faster than four wavefronts); FP64 keeps its registers.
#ifndef OC_HYDRO_WAVES32
#define OC_HYDRO_WAVES32 5
#endif
#ifndef OC_HYDRO_CHUNKS
#define OC_HYDRO_CHUNKS 2
#endif
template <class T>
constexpr int hydro_tend_waves() { return sizeof(T) == 4 ? OC_HYDRO_WAVES32 : 1; }

template <class T, int SCHEME>
__global__ void __launch_bounds__(TTX * TTY, hydro_tend_waves<T>())
    hydro_tend_kernel(HydroBufs<T> a, HydroStep<T> st) {
  using SC = StageCopy<T>;
  __shared__ T P[2][SC::LEN];
  __shared__ T FX[2][F_X];
  __shared__ T FY[2][F_Y];
  const Dims d = a.d;
  const int nbx = (d.nx + TTX - 1) / TTX, nby = (d.ny + TTY - 1) / TTY;
  const int item = hydro_tile_index();            // chunk-major over (chunk, tile)
  const int tile = item % (nbx * nby), chunk = item / (nbx * nby);
  const int i0 = (tile % nbx) * TTX, j0 = (tile / nbx) * TTY;
  const int kb = chunk * st.kc, ke = min(kb + st.kc, d.nz);
  const int tx = (int)threadIdx.x, ty = (int)threadIdx.y, tid = ty * TTX + tx;
  const int i = i0 + tx, j = j0 + ty;
  const bool active = i < d.nx && j < d.ny;
  const HydroMetric& m = a.m;
  const long sz = d.sz;
  const bool vpt = j > 0;     // v point on y face j (face 0 is a wall)
  const T eps = a.eps;
  const T dy = (T)m.dy, rdy = T(1) / dy;
  const T dz = (T)m.dz, rdz = T(1) / dz;
  const int jm = min(j, d.ny - 1) + d.h;
  const T rdxc = T(1) / (T)m.dxc[jm];
  const T fc = (T)m.fc[jm], ff = (T)m.ff[jm];
  const T Ax = dy * dz;
  const T Ay0 = (T)m.dxf[jm] * dz;
  const T Az = (T)m.areac[jm];
  const T rvol = T(1) / (Az * dz);
  const T nu = a.nu, kappa = a.kappa;
  const T dt = st.dt, a1 = st.a1, a0 = st.a0;
  const bool first = st.first != 0;

  // own column: field pointers advanced by whole levels (uniform) plus a
  // 32-bit per-thread byte offset
  const unsigned cb = (unsigned)pidx(d, min(i, d.nx - 1), min(j, d.ny - 1), 0) * (unsigned)sizeof(T);
  // register windows along z: q[o] = q_{k-2+o}, from level kb - 3 (one
  // below the window, for the bottom face of an upper chunk)
  T uw[6], vw[6], tw[6], sw[6];
  T u3, v3, t3, s3;
#pragma unroll
  for (int o = -1; o < 6; ++o) {
    const long kz = (long)(kb + o - 2) * sz;
    const T uu = at(uniform_ptr(a.u + kz), cb), vv = at(uniform_ptr(a.v + kz), cb);
    const T tt = at(uniform_ptr(a.t + kz), cb), ss = at(uniform_ptr(a.s + kz), cb);
    if (o < 0) {
      u3 = uu; v3 = vv; t3 = tt; s3 = ss;
    } else {
      uw[o] = uu; vw[o] = vv; tw[o] = tt; sw[o] = ss;
    }
  }
  // quantities on face k carried up from the level below (floor: zero; the
  // bottom face of an upper chunk is computed here as the chunk below
  // computes its top face)
  T Fu = T(0), Fv = T(0), Ft = T(0), Fs = T(0), Nu = T(0), Nv = T(0);
  T Wu = T(0), Wv = T(0);
  if (kb > 0 && active) {
    const long kf = (long)kb * sz;   // face kb
    const T w_c = at(uniform_ptr(a.w + kf), cb);
    Wu = T(0.5) * (at(uniform_ptr(a.w + kf - 1), cb) + w_c);
    Wv = vpt ? T(0.5) * (at(uniform_ptr(a.w + kf - d.sy), cb) + w_c) : T(0);
    Fu = Wu * rec<T, SCHEME>(u3, uw[0], uw[1], uw[2], uw[3], uw[4], Wu, eps);
    Fv = Wv * rec<T, SCHEME>(v3, vw[0], vw[1], vw[2], vw[3], vw[4], Wv, eps);
    Ft = (w_c * rec<T, SCHEME>(t3, tw[0], tw[1], tw[2], tw[3], tw[4], w_c, eps) -
          kappa * (tw[2] - tw[1]) * rdz) * Az;
    Fs = (w_c * rec<T, SCHEME>(s3, sw[0], sw[1], sw[2], sw[3], sw[4], w_c, eps) -
          kappa * (sw[2] - sw[1]) * rdz) * Az;
    Nu = nu * (uw[2] - uw[1]) * rdz;
    Nv = nu * (vw[2] - vw[1]) * rdz;
  }
  double gu = 0.0, gv = 0.0;
  const long c2 = (long)min(j, d.ny - 1) * d.nx + min(i, d.nx - 1);

  // own positions in the staged planes
  const int lt = (ty + 3) * P_TX + tx + 3;
  const int lz = (ty + 2) * P_ZX + tx + 2;
  const int lu = (ty + 1) * P_UX + tx + 1;
  const int lv = (ty + 1) * P_VX + tx + 1;
  const int lw = (ty + 1) * P_WX + tx + 1;

  // load-to-LDS copies of the staged planes: per-lane offsets for this tile
  // (clamped at the last padded point), then the planes of level kb
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  SC cp;
  {
    const int ix = d.nx + d.h - 1 - i0, jy = d.ny + d.h - 1 - j0;   // last padded point
    const int sy = (int)d.sy;
    cp.ts.init(sy, ix + 3, jy + 3, tid, wave, lane);
    cp.z.init(sy, ix + 2, jy + 2, tid, wave, lane);
    cp.u.init(sy, ix + 1, jy + 1, tid, wave, lane);
    cp.v.init(sy, ix + 1, jy + 1, tid, wave, lane);
    cp.w.init(sy, ix + 1, jy + 1, tid, wave, lane);
  }
  const long b3 = pidx(d, i0 - 3, j0 - 3, 0), b2 = pidx(d, i0 - 2, j0 - 2, 0);
  const long b1 = pidx(d, i0 - 1, j0 - 1, 0);
  auto copy_level = [&](int kk) {
    T* S = P[kk & 1];
    const long kz = (long)kk * sz;
    cp.ts.issue(a.t + b3 + kz, S + SC::L_T, wave);
    cp.ts.issue(a.s + b3 + kz, S + SC::L_S, wave);
    cp.z.issue(a.zeta + b2 + kz, S + SC::L_Z, wave);
    cp.u.issue(a.u + b1 + kz, S + SC::L_U, wave);
    cp.v.issue(a.v + b1 + kz, S + SC::L_V, wave);
    cp.w.issue(a.w + b1 + kz + sz, S + SC::L_W, wave);   // w on face k + 1
  };
  copy_level(kb);
  wait_vm();
  __syncthreads();
  for (int k = kb; k < ke; ++k) {
    T* S = P[k & 1];
    const long kz = (long)k * sz;
    // the next level's planes are copied while this level computes (into the
    // other buffer, whose last readers finished before the previous barrier)
    if (k + 1 < ke) copy_level(k + 1);

    // ---- tracer fluxes through the x faces (west of each column) and the
    // y faces (south of each row) of the tile; then the east and north edge
    // faces by the first wavefront
    {
      const T* St = S + SC::L_T;
      const T* Ss = S + SC::L_S;
      if (i <= d.nx && j < d.ny) {
        const T uf = S[SC::L_U + lu];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const T* f = q ? Ss : St;
          FX[q][ty * (TTX + 1) + tx] =
              uf * rec<T, SCHEME>(f[lt - 3], f[lt - 2], f[lt - 1], f[lt], f[lt + 1], f[lt + 2], uf,
                                  eps) * Ax;
        }
      }
      if (i < d.nx && j <= d.ny) {
        const T vf = S[SC::L_V + lv];
        const bool open = j > 0 && j < d.ny;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const T* f = q ? Ss : St;
          FY[q][ty * TTX + tx] =
              open ? vf * rec<T, SCHEME>(f[lt - 3 * P_TX], f[lt - 2 * P_TX], f[lt - P_TX], f[lt],
                                         f[lt + P_TX], f[lt + 2 * P_TX], vf, eps) * Ay0
                   : T(0);
        }
      }
      if (tid < TTY + TTX) {
        if (tid < TTY) {           // x face i0 + TTX of row j0 + tid
          const int ey = tid;
          if (i0 + TTX <= d.nx && j0 + ey < d.ny) {
            const T uf = S[SC::L_U + (ey + 1) * P_UX + TTX + 1];
            const int le = (ey + 3) * P_TX + TTX + 3;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
              const T* f = q ? Ss : St;
              FX[q][ey * (TTX + 1) + TTX] =
                  uf * rec<T, SCHEME>(f[le - 3], f[le - 2], f[le - 1], f[le], f[le + 1], f[le + 2],
                                      uf, eps) * Ax;
            }
          }
        } else {                   // y face j0 + TTY of column i0 + ex
          const int ex = tid - TTY;
          const int jf = j0 + TTY;
          if (jf <= d.ny && i0 + ex < d.nx) {
            const T vf = S[SC::L_V + (TTY + 1) * P_VX + ex + 1];
            const int le = (TTY + 3) * P_TX + ex + 3;
            const bool open = jf < d.ny;
            const T Ay = (T)m.dxf[jf + d.h] * dz;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
              const T* f = q ? Ss : St;
              FY[q][TTY * TTX + ex] =
                  open ? vf * rec<T, SCHEME>(f[le - 3 * P_TX], f[le - 2 * P_TX], f[le - P_TX],
                                             f[le], f[le + P_TX], f[le + 2 * P_TX], vf, eps) * Ay
                       : T(0);
            }
          }
        }
      }
    }
    __syncthreads();

    if (active) {
      const T* U = S + SC::L_U;
      const T* V = S + SC::L_V;
      const T* Z = S + SC::L_Z;
      const T* Wp = S + SC::L_W;
      const T w_c = Wp[lw];
      const T Wu1 = T(0.5) * (Wp[lw - 1] + w_c);
      const T Wv1 = vpt ? T(0.5) * (Wp[lw - P_WX] + w_c) : T(0);
      // fluxes through face k + 1
      T Fu1, Fv1, Ft1, Fs1, Nu1, Nv1;
      if (k + 1 < d.nz) {
        Fu1 = Wu1 * rec<T, SCHEME>(uw[0], uw[1], uw[2], uw[3], uw[4], uw[5], Wu1, eps);
        Fv1 = Wv1 * rec<T, SCHEME>(vw[0], vw[1], vw[2], vw[3], vw[4], vw[5], Wv1, eps);
        Ft1 = (w_c * rec<T, SCHEME>(tw[0], tw[1], tw[2], tw[3], tw[4], tw[5], w_c, eps) -
               kappa * (tw[3] - tw[2]) * rdz) * Az;
        Fs1 = (w_c * rec<T, SCHEME>(sw[0], sw[1], sw[2], sw[3], sw[4], sw[5], w_c, eps) -
               kappa * (sw[3] - sw[2]) * rdz) * Az;
        Nu1 = nu * (uw[3] - uw[2]) * rdz;
        Nv1 = nu * (vw[3] - vw[2]) * rdz;
      } else {
        Fu1 = Wu1 * uw[2];
        Fv1 = Wv1 * vw[2];
        Ft1 = w_c * tw[2] * Az;
        Fs1 = w_c * sw[2] * Az;
        Nu1 = (T)a.taux[c2];
        Nv1 = (T)a.tauy[c2];
      }

      const T u_c = uw[2], v_c = vw[2];
      const T u_e = U[lu + 1], u_w = U[lu - 1];
      const T v_w = V[lv - 1], v_n = V[lv + P_VX], v_nw = V[lv - 1 + P_VX];
      const T ke = T(0.25) * (u_c * u_c + u_e * u_e + v_c * v_c + v_n * v_n);

      // ---- u point (x face i, row j)
      {
        const T vb = T(0.25) * (v_w + v_c + v_nw + v_n);
        const T zh = rec<T, SCHEME>(Z[lz - 2 * P_ZX], Z[lz - P_ZX], Z[lz], Z[lz + P_ZX],
                                    Z[lz + 2 * P_ZX], Z[lz + 3 * P_ZX], vb, eps);
        const T ke_w = T(0.25) * (u_w * u_w + u_c * u_c + v_w * v_w + v_nw * v_nw);
        T G = zh * vb + fc * vb;
        G -= (ke - ke_w) * rdxc;
        G -= at(uniform_ptr(a.px + kz), cb);
        G -= (Fu1 - Fu) * rdz - u_c * (Wu1 - Wu) * rdz;
        G += (Nu1 - Nu) * rdz;
        T comb = a1 * G;
        if (!first) comb -= a0 * at(uniform_ptr(a.Gu + kz), cb);
        at(uniform_ptr(a.Gu + kz), cb) = G;
        at(uniform_ptr(a.uo + kz), cb) = u_c + dt * comb;
        gu += (double)comb;
      }
      // ---- v point (x centre i, y face j)
      if (vpt) {
        const T u_s = U[lu - P_UX], u_se = U[lu - P_UX + 1];
        const T v_s = V[lv - P_VX];
        const T ub = T(0.25) * (u_s + u_se + u_c + u_e);
        const T zh = rec<T, SCHEME>(Z[lz - 2], Z[lz - 1], Z[lz], Z[lz + 1], Z[lz + 2], Z[lz + 3],
                                    ub, eps);
        const T ke_s = T(0.25) * (u_s * u_s + u_se * u_se + v_s * v_s + v_c * v_c);
        T G = -(zh * ub) - ff * ub;
        G -= (ke - ke_s) * rdy;
        G -= at(uniform_ptr(a.py + kz), cb);
        G -= (Fv1 - Fv) * rdz - v_c * (Wv1 - Wv) * rdz;
        G += (Nv1 - Nv) * rdz;
        T comb = a1 * G;
        if (!first) comb -= a0 * at(uniform_ptr(a.Gv + kz), cb);
        at(uniform_ptr(a.Gv + kz), cb) = G;
        at(uniform_ptr(a.vo + kz), cb) = v_c + dt * comb;
        gv += (double)comb;
      } else {
        at(uniform_ptr(a.Gv + kz), cb) = T(0);
        at(uniform_ptr(a.vo + kz), cb) = T(0);
      }
      // ---- tracers at centre (i, j)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const T cc = q ? sw[2] : tw[2];
        const T fx0 = FX[q][ty * (TTX + 1) + tx], fx1 = FX[q][ty * (TTX + 1) + tx + 1];
        const T fy0 = FY[q][ty * TTX + tx], fy1 = FY[q][(ty + 1) * TTX + tx];
        const T Fz0 = q ? Fs : Ft, Fz1 = q ? Fs1 : Ft1;
        const T G = -((fx1 - fx0) + (fy1 - fy0) + (Fz1 - Fz0)) * rvol;
        global_ptr<T> Gq = uniform_ptr((q ? a.Gs : a.Gt) + kz);
        T comb = a1 * G;
        if (!first) comb -= a0 * at(Gq, cb);
        at(Gq, cb) = G;
        at(uniform_ptr((q ? a.so : a.to) + kz), cb) = cc + dt * comb;
      }

      // ---- carry face k + 1 up; shift the windows
      Fu = Fu1; Fv = Fv1; Ft = Ft1; Fs = Fs1; Nu = Nu1; Nv = Nv1; Wu = Wu1; Wv = Wv1;
#pragma unroll
      for (int o = 0; o < 5; ++o) {
        uw[o] = uw[o + 1];
        vw[o] = vw[o + 1];
        tw[o] = tw[o + 1];
        sw[o] = sw[o + 1];
      }
      if (k + 1 < d.nz) {
        const long kn = kz + 4 * sz;  // level k + 4 (at most nz + 2, inside the halo)
        uw[5] = at(uniform_ptr(a.u + kn), cb);
        vw[5] = at(uniform_ptr(a.v + kn), cb);
        tw[5] = at(uniform_ptr(a.t + kn), cb);
        sw[5] = at(uniform_ptr(a.s + kn), cb);
      }
    }
    // the copies of level k + 1 have landed (this wave's), and every wave is
    // done with this level's planes and flux arrays
    wait_vm();
    __syncthreads();
  }
  if (active) {
    // partial column sums of this chunk (the lower chunk's into gub, gvb)
    (chunk == 0 ? a.gub : a.gub1)[c2] = gu;
    (chunk == 0 ? a.gvb : a.gvb1)[c2] = vpt ? gv : 0.0;
  }
}

// Slow forcing of the barotropic mode from the chunks' partial column sums
// (added in chunk order), times dz.
__global__ void hydro_gsum_kernel(double* __restrict__ gub, double* __restrict__ gvb,
                                  const double* __restrict__ gub1,
                                  const double* __restrict__ gvb1, long n, int nchunks,
                                  double dz) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  double su = gub[c], sv = gvb[c];
  if (nchunks > 1) {
    su += gub1[c];
    sv += gvb1[c];
  }
  gub[c] = su * dz;
  gvb[c] = sv * dz;
}

// Halo images of the prognostic fields: x periodic; y walls with even
// mirrors for u, T, S and an odd mirror about the wall faces for v (whose
// wall faces are set to zero); z walls with even mirrors.
template <class T>
__device__ inline void hydro_halo_point(const Dims& d, T* u, T* v, T* t, T* s, int i, int j,
                                        int k) {
  const bool xin = i >= 0 && i < d.nx, yin = j >= 0 && j < d.ny, zin = k >= 0 && k < d.nz;
  const bool vwall = (j == 0 || j == d.ny);
  const bool c_interior = xin && yin && zin;
  const bool v_interior = xin && zin && j > 0 && j < d.ny;
  if (c_interior && v_interior) return;
  const long p = pidx(d, i, j, k);
  const int si = (i < 0) ? i + d.nx : (i >= d.nx ? i - d.nx : i);
  const int sk = (k < 0) ? -1 - k : (k >= d.nz ? 2 * d.nz - 1 - k : k);
  if (!c_interior) {
    const int sj = (j < 0) ? -1 - j : (j >= d.ny ? 2 * d.ny - 1 - j : j);
    const long src = pidx(d, si, sj, sk);
    u[p] = u[src];
    t[p] = t[src];
    s[p] = s[src];
  }
  if (!v_interior) {
    if (vwall) {
      v[p] = T(0);
    } else {
      const int sj = (j < 0) ? -j : (j > d.ny ? 2 * d.ny - j : j);
      const T sg = (j < 0 || j > d.ny) ? T(-1) : T(1);
      v[p] = sg * v[pidx(d, si, sj, sk)];
    }
  }
}

// One workgroup per padded row (j, k): rows outside the interior, and the
// rows of v's wall faces (j = 0, ny), are filled across their whole length;
// the other rows have only their x halos.
template <class T>
__global__ void __launch_bounds__(64) hydro_halo_kernel(Dims d, T* u, T* v, T* t, T* s) {
  const int j = (int)(blockIdx.x % (unsigned)d.py) - d.h;
  const int k = (int)(blockIdx.x / (unsigned)d.py) - d.h;
  const bool full = j <= 0 || j >= d.ny || k < 0 || k >= d.nz;
  if (full) {
    for (int i = (int)threadIdx.x - d.h; i < d.nx + d.h; i += 64)
      hydro_halo_point(d, u, v, t, s, i, j, k);
  } else if ((int)threadIdx.x < 2 * d.h) {
    const int x = (int)threadIdx.x;
    const int i = x < d.h ? x - d.h : d.nx + (x - d.h);
    hydro_halo_point(d, u, v, t, s, i, j, k);
  }
}

}  // namespace

template <class T>
hipError_t launch_hydro_diag(const HydroBufs<T>& a, hipStream_t s) {
  const unsigned nb =
      (unsigned)(((a.d.nx + 5 + HTX - 1) / HTX) * ((a.d.ny + 5 + HTY - 1) / HTY));
  hipLaunchKernelGGL(hydro_diag_kernel<T>, dim3(nb), dim3(HTX, HTY), 0, s, a);
  return hipGetLastError();
}

template <class T>
hipError_t launch_hydro_tendency(const HydroBufs<T>& a, const HydroStep<T>& st, int scheme,
                                 hipStream_t s) {
  // two chunks of levels (when there are at least 16): the grid then holds
  // twice the workgroups of one march, so its last round of resident
  // workgroups is fuller
  HydroStep<T> sc = st;
  const int nchunks = a.d.nz >= 16 ? OC_HYDRO_CHUNKS : 1;
  sc.kc = (a.d.nz + nchunks - 1) / nchunks;
  const dim3 grid((unsigned)(((a.d.nx + TTX - 1) / TTX) * ((a.d.ny + TTY - 1) / TTY) * nchunks));
  const dim3 block(TTX, TTY);
  switch (scheme) {
    case tz::SCHEME_NONE:
      hipLaunchKernelGGL((hydro_tend_kernel<T, tz::SCHEME_NONE>), grid, block, 0, s, a, sc);
      break;
    case tz::SCHEME_LINEAR:
      hipLaunchKernelGGL((hydro_tend_kernel<T, tz::SCHEME_LINEAR>), grid, block, 0, s, a, sc);
      break;
    default:
      hipLaunchKernelGGL((hydro_tend_kernel<T, tz::SCHEME_WENOZ>), grid, block, 0, s, a, sc);
  }
  const long n2 = (long)a.d.nx * a.d.ny;
  hipLaunchKernelGGL(hydro_gsum_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s,
                     a.gub, a.gvb, (const double*)a.gub1, (const double*)a.gvb1, n2, nchunks,
                     a.m.dz);
  return hipGetLastError();
}

template <class T>
hipError_t launch_hydro_halo(const Dims& d, T* u, T* v, T* t, T* sf, hipStream_t s) {
  const unsigned rows = (unsigned)((long)d.py * d.pz);
  hipLaunchKernelGGL(hydro_halo_kernel<T>, dim3(rows), dim3(64), 0, s, d, u, v, t, sf);
  return hipGetLastError();
}

template hipError_t launch_hydro_diag<float>(const HydroBufs<float>&, hipStream_t);
template hipError_t launch_hydro_diag<double>(const HydroBufs<double>&, hipStream_t);
template hipError_t launch_hydro_tendency<float>(const HydroBufs<float>&, const HydroStep<float>&,
                                                 int, hipStream_t);
template hipError_t launch_hydro_tendency<double>(const HydroBufs<double>&,
                                                  const HydroStep<double>&, int, hipStream_t);
template hipError_t launch_hydro_halo<float>(const Dims&, float*, float*, float*, float*,
                                             hipStream_t);
template hipError_t launch_hydro_halo<double>(const Dims&, double*, double*, double*, double*,
                                              hipStream_t);

}  // namespace oc
