// Eddy-viscosity LES closures on gfx950 (closure paragraph of the
// nonhydrostatic model section of arXiv 2502.14148: the closure flux
// divergence d_m tau_nm with the SmagorinskyLilly eddy viscosity; the
// AnisotropicMinimumDissipation closure named beside it).
//
//   Smagorinsky-Lilly: nu_e = (C_s Delta)^2 |S| sqrt(max(0, 1 - C_b N^2/|S|^2)),
//     |S|^2 = 2 S_ij S_ij, Delta = (dx dy dzc)^(1/3), kappa_e = nu_e / Pr;
//   AMD (Rozema et al. 2015, Vreugdenhil & Taylor 2018):
//     nu_e = max(0, -C sum_k Delta_k^2 d_k u_i d_k u_j S_ij / |grad u|^2),
//     kappa_e = max(0, -C sum_k Delta_k^2 d_k u_i d_k c d_i c / |grad c|^2).
//
// Two kernels per substage; each workgroup owns a column tile and marches
// up a chunk of levels, keeping three levels (k-1, k, k+1, with a one-cell
// halo) of every field it reads in LDS rings, so each value is fetched from
// memory once per tile instead of once per neighbour that reads it:
//   1. the eddy viscosity (and AMD's per-tracer diffusivity) at the centres
//      from the resolved gradients: diagonal strain at the centre, the
//      off-diagonal components on the twelve surrounding edges (squared then
//      averaged for |S|, averaged for AMD's gradient tensor), N^2 from the
//      two z faces; written with their halo images;
//   2. the closure tendencies d_j(2 nu_e S_ij) of u, v, w (stresses at their
//      C-grid locations, edge viscosities the mean of four centres) and
//      d_i(kappa_e d_i c) of the tracers (face diffusivities the mean of two
//      centres); no flux through the walls.  The tendency kernel adds them.
#include "oc_internal.h"

namespace oc {

namespace {

// Tiles: TX x TY columns, chunks of LES_KC levels.  Workgroups are dealt
// round-robin to the 8 XCDs; renumbering them gives each XCD a contiguous
// run of tiles, so the halo rows shared by neighbouring tiles stay in one L2.
constexpr int LES_KC = 16;

struct LesTile {
  int i0, j0, kb, ke;
};

__device__ inline LesTile les_tile(const Dims& d, int tx, int ty) {
  const unsigned nb = gridDim.x;
  unsigned b = blockIdx.x;
  if (nb % 8 == 0) b = (b % 8) * (nb / 8) + b / 8;
  const int nbx = d.nx / tx, nby = d.ny / ty;
  LesTile t;
  t.i0 = (int)(b % nbx) * tx;
  t.j0 = (int)((b / nbx) % nby) * ty;
  t.kb = (int)(b / (nbx * nby)) * LES_KC;
  t.ke = min(t.kb + LES_KC, d.nz);
  return t;
}

// Values of field f around the own cell, read from the LDS rings: level
// k + dk sits at ring offset off[dk + 1] of the field's three planes.
template <class T, int PX, int PL>
struct Ring {
  const T* S;      // ring planes of all fields, 3 PL each
  int L;           // own position in a plane
  int off[3];      // plane offsets of levels k-1, k, k+1
  __device__ T operator()(int f, int di, int dj, int dk) const {
    return S[f * 3 * PL + off[dk + 1] + L + dj * PX + di];
  }
};

// Load level kk of nf <= NFMAX fields into ring slot `slot` (tile plus a
// one-cell halo).  Every load of the level is issued before the first LDS
// store, so the fetches overlap.  goff: the thread's element offsets within
// a level, relative to the tile corner.
template <class T, int TX, int TY, int NFMAX>
__device__ inline void les_fill(T* S, const T* const* fld, int nf, const Dims& d, const LesTile& t,
                                const int* goff, int slot, int kk) {
  constexpr int PX = TX + 2, PY = TY + 2, PL = PX * PY, NT = TX * TY;
  constexpr int NR = (PL + NT - 1) / NT;
  const long base = (long)(kk + d.h) * d.sz + (long)(t.j0 - 1 + d.h) * d.sy + (t.i0 - 1 + d.h);
  T v[NFMAX][NR];
#pragma unroll
  for (int f = 0; f < NFMAX; ++f)
    if (f < nf) {
      const auto src = glb(fld[f]) + base;
#pragma unroll
      for (int r = 0; r < NR; ++r)
        if (PL % NT == 0 || threadIdx.x + r * NT < PL) v[f][r] = src[goff[r]];
    }
#pragma unroll
  for (int f = 0; f < NFMAX; ++f)
    if (f < nf) {
      T* dst = S + f * 3 * PL + slot * PL;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int e = threadIdx.x + r * NT;
        if (PL % NT == 0 || e < PL) dst[e] = v[f][r];
      }
    }
}

// The z-march of a tile: cell(i, j, k, ring) runs for every cell of every
// level, with the rings holding levels k-1, k, k+1.
template <class T, int TX, int TY, int NFMAX, class Cell>
__device__ inline void les_march(const Dims& d, const T* const* fld, int nf, Cell cell) {
  constexpr int PX = TX + 2, PY = TY + 2, PL = PX * PY;
  __shared__ T S[NFMAX * 3 * PL];
  constexpr int NT = TX * TY, NR = (PL + NT - 1) / NT;
  const LesTile t = les_tile(d, TX, TY);
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  int goff[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    const int e = threadIdx.x + q * NT;
    const int ly = e / PX, lx = e - ly * PX;
    goff[q] = (int)(ly * d.sy) + lx;
  }
  les_fill<T, TX, TY, NFMAX>(S, fld, nf, d, t, goff, (t.kb + 2) % 3, t.kb - 1);
  les_fill<T, TX, TY, NFMAX>(S, fld, nf, d, t, goff, t.kb % 3, t.kb);
  Ring<T, PX, PL> r;
  r.S = S;
  r.L = (ty + 1) * PX + (tx + 1);
  for (int k = t.kb; k < t.ke; ++k) {
    __syncthreads();  // the slot of level k-2 is free
    les_fill<T, TX, TY, NFMAX>(S, fld, nf, d, t, goff, (k + 1) % 3, k + 1);
    __syncthreads();
    r.off[0] = ((k + 2) % 3) * PL;
    r.off[1] = (k % 3) * PL;
    r.off[2] = ((k + 1) % 3) * PL;
    cell(t.i0 + tx, t.j0 + ty, k, r);
  }
}

// Ring fields of the viscosity pass: 0 u, 1 v, 2 w, then the tracers
// (Smagorinsky-Lilly: T and S when buoyant; AMD: every tracer).
template <class T, int KIND, class R>
__device__ inline void les_viscosity_cell(const Dims& d, const LesArgs<T>& a, int i, int j, int k,
                                          const R& r) {
  auto U = [&](int di, int dj, int dk) { return r(0, di, dj, dk); };
  auto V = [&](int di, int dj, int dk) { return r(1, di, dj, dk); };
  auto W = [&](int di, int dj, int dk) { return r(2, di, dj, dk); };
  const T rdx = a.rdx, rdy = a.rdy, rzc = glb(a.rdzc)[k];
  const T rzf0 = glb(a.rdzf)[k], rzf1 = glb(a.rdzf)[k + 1];
  const bool wall0 = d.zb && k == 0, wall1 = d.zb && k + 1 == d.nz;
  const T ux = (U(1, 0, 0) - U(0, 0, 0)) * rdx;
  const T vy = (V(0, 1, 0) - V(0, 0, 0)) * rdy;
  const T wz = (W(0, 0, 1) - W(0, 0, 0)) * rzc;
  // off-diagonal gradients on the edges around the centre
  T uy[2][2], vx[2][2], uz[2][2], wx[2][2], vz[2][2], wy[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      // (F,F,C): x face i + p, y face j + q
      uy[p][q] = (U(p, q, 0) - U(p, q - 1, 0)) * rdy;
      vx[p][q] = (V(p, q, 0) - V(p - 1, q, 0)) * rdx;
      // (F,C,F): x face i + p, z face k + q; (C,F,F): y face j + p, z face k + q
      const bool wl = q ? wall1 : wall0;
      const T rzf = q ? rzf1 : rzf0;
      uz[p][q] = wl ? T(0) : (U(p, 0, q) - U(p, 0, q - 1)) * rzf;
      wx[p][q] = wl ? T(0) : (W(p, 0, q) - W(p - 1, 0, q)) * rdx;
      vz[p][q] = wl ? T(0) : (V(0, p, q) - V(0, p, q - 1)) * rzf;
      wy[p][q] = wl ? T(0) : (W(0, p, q) - W(0, p - 1, q)) * rdy;
    }
  T nu;
  if (KIND == OC_LES_SMAGORINSKY) {
    T sxy2 = 0, sxz2 = 0, syz2 = 0;
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const T e1 = T(0.5) * (uy[p][q] + vx[p][q]);
        const T e2 = T(0.5) * (uz[p][q] + wx[p][q]);
        const T e3 = T(0.5) * (vz[p][q] + wy[p][q]);
        sxy2 += e1 * e1;
        sxz2 += e2 * e2;
        syz2 += e3 * e3;
      }
    const T s2 = T(2) * (ux * ux + vy * vy + wz * wz) + (sxy2 + sxz2 + syz2);  // 4 x (1/4) sums
    T n2 = T(0);
    if (a.buoyancy) {
      auto b = [&](int dk) {
        return a.g_alpha * (r(3, 0, 0, dk) - a.t_ref) - a.g_beta * (r(4, 0, 0, dk) - a.s_ref);
      };
      const T b0 = b(0);
      const T g0 = wall0 ? T(0) : (b0 - b(-1)) * rzf0;
      const T g1 = wall1 ? T(0) : (b(1) - b0) * rzf1;
      n2 = T(0.5) * (g0 + g1);
    }
    T fac = T(0);
    if (s2 > T(0)) fac = fmax(T(0), T(1) - a.cb * n2 / s2);
    nu = glb(a.delta2)[k] * sqrt(s2) * sqrt(fac);
  } else {
    // AMD: the gradient tensor at the centre (edge values averaged)
    T G[3][3];
    G[0][0] = ux;
    G[1][1] = vy;
    G[2][2] = wz;
    G[0][1] = T(0.25) * (uy[0][0] + uy[0][1] + uy[1][0] + uy[1][1]);
    G[1][0] = T(0.25) * (vx[0][0] + vx[0][1] + vx[1][0] + vx[1][1]);
    G[0][2] = T(0.25) * (uz[0][0] + uz[0][1] + uz[1][0] + uz[1][1]);
    G[2][0] = T(0.25) * (wx[0][0] + wx[0][1] + wx[1][0] + wx[1][1]);
    G[1][2] = T(0.25) * (vz[0][0] + vz[0][1] + vz[1][0] + vz[1][1]);
    G[2][1] = T(0.25) * (wy[0][0] + wy[0][1] + wy[1][0] + wy[1][1]);
    const T D2[3] = {T(1) / (rdx * rdx), T(1) / (rdy * rdy), T(1) / (rzc * rzc)};
    T num = 0, den = 0;
#pragma unroll
    for (int kk = 0; kk < 3; ++kk)
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) {
        den += G[ii][kk] * G[ii][kk];
#pragma unroll
        for (int jj = 0; jj < 3; ++jj)
          num += D2[kk] * G[ii][kk] * G[jj][kk] * (T(0.5) * (G[ii][jj] + G[jj][ii]));
      }
    nu = (den > T(0)) ? fmax(T(0), -a.camd * num / den) : T(0);
    // per-tracer diffusivities
    for (int q = 0; q < a.ntr; ++q) {
      auto C = [&](int di, int dj, int dk) { return r(3 + q, di, dj, dk); };
      const T c0 = C(0, 0, 0);
      const T gx = T(0.5) * (C(1, 0, 0) - C(-1, 0, 0)) * rdx;
      const T gy = T(0.5) * (C(0, 1, 0) - C(0, -1, 0)) * rdy;
      const T gz0 = wall0 ? T(0) : (c0 - C(0, 0, -1)) * rzf0;
      const T gz1 = wall1 ? T(0) : (C(0, 0, 1) - c0) * rzf1;
      const T gc[3] = {gx, gy, T(0.5) * (gz0 + gz1)};
      T kn = 0;
#pragma unroll
      for (int kk = 0; kk < 3; ++kk)
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) kn += D2[kk] * G[ii][kk] * gc[kk] * gc[ii];
      const T kd = gc[0] * gc[0] + gc[1] * gc[1] + gc[2] * gc[2];
      const T kap = (kd > T(0)) ? fmax(T(0), -a.camd * kn / kd) : T(0);
      store_with_images(a.kap[q], d, i, j, k, kap, false);
    }
  }
  store_with_images(a.nu, d, i, j, k, nu, false);
}

template <class T, int KIND, int TX, int TY>
__global__ void __launch_bounds__(TX * TY) les_viscosity_kernel(Dims d, LesArgs<T> a) {
  const T* fld[3 + OC_MAX_TRACERS] = {a.u, a.v, a.w};
  int nf = 3;
  if (KIND == OC_LES_SMAGORINSKY) {
    if (a.buoyancy) { fld[3] = a.c0; fld[4] = a.c1; nf = 5; }
  } else {
    for (int q = 0; q < a.ntr; ++q) fld[3 + q] = a.tr[q];
    nf = 3 + a.ntr;
  }
  les_march<T, TX, TY, 3 + OC_MAX_TRACERS>(
      d, fld, nf, [&](int i, int j, int k, const auto& r) {
        les_viscosity_cell<T, KIND>(d, a, i, j, k, r);
      });
}

// The closure tendencies of the cell index (i, j, k): u at x face i, v at y
// face j, w at z face k, tracers at the centre.  Ring fields: 0 u, 1 v, 2 w,
// 3 nu, 4 + q tracer q, 4 + ntr + q AMD's kappa of tracer q.
template <class T, class R>
__device__ inline void les_flux_cell(const Dims& d, const LesArgs<T>& a, int i, int j, int k,
                                     const R& r) {
  const long c = pidx(d, i, j, k);
  auto U = [&](int di, int dj, int dk) { return r(0, di, dj, dk); };
  auto V = [&](int di, int dj, int dk) { return r(1, di, dj, dk); };
  auto W = [&](int di, int dj, int dk) { return r(2, di, dj, dk); };
  auto N = [&](int di, int dj, int dk) { return r(3, di, dj, dk); };
  const T rdx = a.rdx, rdy = a.rdy;
  const T rzc = glb(a.rdzc)[k], rzf0 = glb(a.rdzf)[k], rzf1 = glb(a.rdzf)[k + 1];
  const bool wall0 = d.zb && k == 0, wall1 = d.zb && k + 1 == d.nz;
  // edge viscosities: means of the four surrounding centres
  auto n_ffc = [&](int p, int q) {  // x face i + p, y face j + q
    return T(0.25) * (N(p - 1, q - 1, 0) + N(p, q - 1, 0) + N(p - 1, q, 0) + N(p, q, 0));
  };
  auto n_fcf = [&](int p, int q) {  // x face i + p, z face k + q
    return T(0.25) * (N(p - 1, 0, q - 1) + N(p, 0, q - 1) + N(p - 1, 0, q) + N(p, 0, q));
  };
  auto n_cff = [&](int p, int q) {  // y face j + p, z face k + q
    return T(0.25) * (N(0, p - 1, q - 1) + N(0, p, q - 1) + N(0, p - 1, q) + N(0, p, q));
  };
  // stresses 2 nu S at their locations
  auto txy = [&](int p, int q) {
    return n_ffc(p, q) * ((U(p, q, 0) - U(p, q - 1, 0)) * rdy + (V(p, q, 0) - V(p - 1, q, 0)) * rdx);
  };
  auto txz = [&](int p, int q) {
    if (q ? wall1 : wall0) return T(0);
    const T rzf = q ? rzf1 : rzf0;
    return n_fcf(p, q) * ((U(p, 0, q) - U(p, 0, q - 1)) * rzf + (W(p, 0, q) - W(p - 1, 0, q)) * rdx);
  };
  auto tyz = [&](int p, int q) {
    if (q ? wall1 : wall0) return T(0);
    const T rzf = q ? rzf1 : rzf0;
    return n_cff(p, q) * ((V(0, p, q) - V(0, p, q - 1)) * rzf + (W(0, p, q) - W(0, p - 1, q)) * rdy);
  };
  // u at x face i: txx at the centres i-1, i
  {
    const T t0 = T(2) * N(-1, 0, 0) * (U(0, 0, 0) - U(-1, 0, 0)) * rdx;
    const T t1 = T(2) * N(0, 0, 0) * (U(1, 0, 0) - U(0, 0, 0)) * rdx;
    const T g = (t1 - t0) * rdx + (txy(0, 1) - txy(0, 0)) * rdy + (txz(0, 1) - txz(0, 0)) * rzc;
    glb(a.gc[0])[c] = g;
  }
  // v at y face j
  {
    const T t0 = T(2) * N(0, -1, 0) * (V(0, 0, 0) - V(0, -1, 0)) * rdy;
    const T t1 = T(2) * N(0, 0, 0) * (V(0, 1, 0) - V(0, 0, 0)) * rdy;
    const T g = (txy(1, 0) - txy(0, 0)) * rdx + (t1 - t0) * rdy + (tyz(0, 1) - tyz(0, 0)) * rzc;
    glb(a.gc[1])[c] = g;
  }
  // w at z face k (the w cell spans the centres k-1, k: thickness dzf_k);
  // txz and tyz on face k are the q = 0 stresses of the edges with x face
  // i, i+1 (y face j, j+1)
  {
    T g = T(0);
    if (!wall0) {
      const T t0 = T(2) * N(0, 0, -1) * (W(0, 0, 0) - W(0, 0, -1)) * glb(a.rdzc)[k - 1];
      const T t1 = T(2) * N(0, 0, 0) * (W(0, 0, 1) - W(0, 0, 0)) * rzc;
      g = (txz(1, 0) - txz(0, 0)) * rdx + (tyz(1, 0) - tyz(0, 0)) * rdy + (t1 - t0) * rzf0;
    }
    glb(a.gc[2])[c] = g;
  }
  // tracers: d_i(kappa d_i c), face diffusivities the mean of two centres
  for (int q = 0; q < a.ntr; ++q) {
    const int fk = a.kap[q] ? 4 + a.ntr + q : 3;
    auto C = [&](int di, int dj, int dk) { return r(4 + q, di, dj, dk); };
    auto K = [&](int di, int dj, int dk) { return r(fk, di, dj, dk); };
    const T s = a.kap[q] ? T(1) : a.rpr;
    const T c0 = C(0, 0, 0), k0 = K(0, 0, 0);
    const T fxm = T(0.5) * (K(-1, 0, 0) + k0) * (c0 - C(-1, 0, 0)) * rdx;
    const T fxp = T(0.5) * (k0 + K(1, 0, 0)) * (C(1, 0, 0) - c0) * rdx;
    const T fym = T(0.5) * (K(0, -1, 0) + k0) * (c0 - C(0, -1, 0)) * rdy;
    const T fyp = T(0.5) * (k0 + K(0, 1, 0)) * (C(0, 1, 0) - c0) * rdy;
    const T fzm = wall0 ? T(0) : T(0.5) * (K(0, 0, -1) + k0) * (c0 - C(0, 0, -1)) * rzf0;
    const T fzp = wall1 ? T(0) : T(0.5) * (k0 + K(0, 0, 1)) * (C(0, 0, 1) - c0) * rzf1;
    glb(a.gc[3 + q])[c] = s * ((fxp - fxm) * rdx + (fyp - fym) * rdy + (fzp - fzm) * rzc);
  }
}

template <class T, int TX, int TY>
__global__ void __launch_bounds__(TX * TY) les_flux_kernel(Dims d, LesArgs<T> a) {
  const T* fld[4 + 2 * OC_MAX_TRACERS] = {a.u, a.v, a.w, a.nu};
  int nf = 4;
  for (int q = 0; q < a.ntr; ++q) fld[nf++] = a.tr[q];
  if (a.kap[0])
    for (int q = 0; q < a.ntr; ++q) fld[nf++] = a.kap[q];
  les_march<T, TX, TY, 4 + 2 * OC_MAX_TRACERS>(
      d, fld, nf, [&](int i, int j, int k, const auto& r) { les_flux_cell<T>(d, a, i, j, k, r); });
}

}  // namespace

template <class T, int TX, int TY>
hipError_t launch_les_tiles(const Dims& d, const LesArgs<T>& a, int kind, hipStream_t s) {
  const dim3 grid((d.nx / TX) * (d.ny / TY) * ((d.nz + LES_KC - 1) / LES_KC));
  if (kind == OC_LES_SMAGORINSKY)
    hipLaunchKernelGGL((les_viscosity_kernel<T, OC_LES_SMAGORINSKY, TX, TY>), grid, dim3(TX * TY), 0,
                       s, d, a);
  else if (kind == OC_LES_AMD)
    hipLaunchKernelGGL((les_viscosity_kernel<T, OC_LES_AMD, TX, TY>), grid, dim3(TX * TY), 0, s, d,
                       a);
  else
    return hipErrorInvalidValue;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((les_flux_kernel<T, TX, TY>), grid, dim3(TX * TY), 0, s, d, a);
  return hipGetLastError();
}

template <class T>
hipError_t launch_les(const Dims& d, const LesArgs<T>& a, int kind, hipStream_t s) {
  if (a.ntr < 1 || a.ntr > OC_MAX_TRACERS || d.h < 1) return hipErrorInvalidValue;
  if (d.nx % 32 == 0 && d.ny % 8 == 0) return launch_les_tiles<T, 32, 8>(d, a, kind, s);
  if (d.nx % 8 == 0 && d.ny % 8 == 0) return launch_les_tiles<T, 8, 8>(d, a, kind, s);
  return hipErrorInvalidValue;
}

template hipError_t launch_les<float>(const Dims&, const LesArgs<float>&, int, hipStream_t);
template hipError_t launch_les<double>(const Dims&, const LesArgs<double>&, int, hipStream_t);

}  // namespace oc
