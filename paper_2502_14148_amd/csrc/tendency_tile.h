// Fused tendency + RK3 kernel of the nonhydrostatic model on gfx950, for a
// reconstruction of stencil radius R (WENO5: R = 3, WENO7: 4, WENO9: 5).
//
// Method (finite-volume appendix of arXiv 2502.14148): conservative flux
// divergence of advective + diffusive fluxes for tracers; flux-form momentum
// advection with a centred advecting velocity of order 2R - 2 and a WENO-Z
// reconstruction of order 2R - 1 of the advected component; f-plane Coriolis
// (four-point averages); buoyancy b = g(alpha(T-T0) - beta(S-S0)) averaged
// to w faces; RK3 substage X~ = X + dt(gamma G^m - zeta G^{m-1}) (rk3
// equation).
//
// Vertically stretched grids: z flux differences are divided by the
// thickness of the control volume (cell k, or the w cell about face k) and
// vertical diffusive fluxes by the distance between the differenced values,
// from per-level tables read once per level; reconstructions and the
// advecting-velocity interpolation keep their index-space coefficients.
// Implicit vertical diffusion zeroes the explicit vertical coefficients.
//
// Schedule: a workgroup owns a TX x TY column tile and marches up a chunk of
// k levels.  Every face flux is computed exactly once:
//   * z fluxes per column from a 2R-level register window (the flux through
//     the top face of level k is the bottom flux of level k+1);
//   * x and y fluxes from LDS planes (tile + R-cell halo) of the current
//     level; the (TX+1)TY x-faces and TX(TY+1) y-faces are dealt out to the
//     threads as "slots" whose strides are per-lane values, so x and y faces
//     run the same instruction stream with no divergence;
//   * the advecting velocities of the x and y fluxes of w need u and v
//     interpolated in z to face k: each thread interpolates its own column
//     from its register window; the threads owning the right x faces of the
//     last column and the top y faces of the last row keep a short private
//     LDS ring of those columns' values.
// Tiles are mapped XCD-major so that neighbouring tiles (which share halo
// loads) land on the same XCD and its L2.
#pragma once

#include "oc_internal.h"
#include "weno_dev.h"

#ifndef OC_TEND_FLUXBAR
#define OC_TEND_FLUXBAR 0
#endif
#ifndef OC_TEND_KC_DIV
#define OC_TEND_KC_DIV 1024
#endif
#ifndef OC_TEND_WAVES
#define OC_TEND_WAVES 4
#endif

namespace oc {
namespace tz {

// advective flux vel * W(q) with q read from LDS at q[L + o*s], o = -R..R-1
template <class T, int SCHEME, int R>
__device__ inline T flux_lds(const T* q, int L, int s, T vel, T eps) {
  if (SCHEME == SCHEME_NONE) return T(0);
  if constexpr (R == 3) {
    return vel * rec6<T, SCHEME>(q[L - 3 * s], q[L - 2 * s], q[L - s], q[L], q[L + s],
                                 q[L + 2 * s], vel, eps);
  } else {
    T v[2 * R];
#pragma unroll
    for (int o = 0; o < 2 * R; ++o) v[o] = q[L + (o - R) * s];
    return vel * recw<T, SCHEME, R>(v, vel, eps);
  }
}

// advective flux from a register window w[0 .. 2R-1]
template <class T, int SCHEME, int R>
__device__ inline T flux_reg(const T* w, T vel, T eps) {
  if (SCHEME == SCHEME_NONE) return T(0);
  if constexpr (R == 3)
    return vel * rec6<T, SCHEME>(w[0], w[1], w[2], w[3], w[4], w[5], vel, eps);
  else
    return vel * recw<T, SCHEME, R>(w, vel, eps);
}

// centred interpolation of order 2R - 2 to the midpoint of q[L - s], q[L]
template <class T, int R>
__device__ inline T interp_lds(const T* q, int L, int s) {
  T a[2 * R - 2];
#pragma unroll
  for (int o = 0; o < 2 * R - 2; ++o) a[o] = q[L + (o - (R - 1)) * s];
  return interpc<T, R>(a);
}

// Fluxes of one x or y face slot at LDS position L.  All LDS planes are
// offsets into one shared array S (so every access stays an LDS access).
// sd/se are the strides along and across the flux direction (compile-time
// constants in the main rounds, per lane in the edge round).
struct SlotOff {
  int vd, ve;             // normal and tangential velocity planes (level k)
  int az;                 // normal velocity interpolated in z to face k, per slot
  int wk;                 // w plane (level k)
  int c0;                 // first tracer plane (level k); tracers are PL apart
  int Fself, Fcross, Fw;  // flux arrays (already for this direction)
  int Fc0, Fstride;       // first tracer flux array and the array pitch
};

// IMM: no diffusive tracer flux through a face next to an immersed cell (the
// mask plane at S + om).
template <class T, int SCHEME, int NTR, int PL, int R, bool IMM = false>
__device__ inline void slot_fluxes(T* S, const SlotOff& o, int L, int sd, int se, int fi, T rd,
                                   T nu, T kappa, T eps, int om = 0) {
  {
    const T* vd = S + o.vd;
    const T adv = interp_lds<T, R>(vd, L, sd);
    S[o.Fself + fi] = flux_lds<T, SCHEME, R>(vd, L, sd, adv, eps) - nu * (vd[L] - vd[L - sd]) * rd;
  }
#if OC_TEND_FLUXBAR
  __builtin_amdgcn_sched_barrier(0);
#endif
  {
    const T* vd = S + o.vd;
    const T* ve = S + o.ve;
    const T adv = interp_lds<T, R>(vd, L, se);
    S[o.Fcross + fi] = flux_lds<T, SCHEME, R>(ve, L, sd, adv, eps) - nu * (ve[L] - ve[L - sd]) * rd;
  }
#if OC_TEND_FLUXBAR
  __builtin_amdgcn_sched_barrier(0);
#endif
  {
    const T adv = S[o.az + fi];
    const T* wk = S + o.wk;
    S[o.Fw + fi] = flux_lds<T, SCHEME, R>(wk, L, sd, adv, eps) - nu * (wk[L] - wk[L - sd]) * rd;
  }
  const T un = S[o.vd + L];
  const T kap = IMM ? kappa * (S[om + L] * S[om + L - sd]) : kappa;
#pragma unroll
  for (int q = 0; q < NTR; ++q) {
#if OC_TEND_FLUXBAR
    __builtin_amdgcn_sched_barrier(0);
#endif
    const T* c = S + o.c0 + q * PL;
    S[o.Fc0 + q * o.Fstride + fi] =
        flux_lds<T, SCHEME, R>(c, L, sd, un, eps) - kap * (c[L] - c[L - sd]) * rd;
  }
}

// One column tile: tile b of an nbx x nby x nbz decomposition (k chunks of
// kc levels) of the grid d, whose halo width d.h is at least R.
// CLO: add the closure tendencies computed beforehand (fs.closure; learned
// closure: u, v, w and tracer 0, LES closure: every field).  A separate
// instantiation keeps the plain kernel's registers free of them.
// IMM: grid-fitted immersed boundary (fs.mask, 1 in fluid cells): zero
// velocity tendencies on faces next to an immersed cell, no diffusive tracer
// flux through them, no top flux into an immersed top cell.
template <class T, int SCHEME, int NTR, int TX, int TY, int R, bool CLO = false,
          bool IMM = false>
__device__ __attribute__((always_inline)) inline void tendency_tile(
    const Dims& d, const FieldSet<T>& fs, const TendParams<T>& P, int nbx, int nby, int nbz,
    int kc, int b) {
  constexpr int NT = TX * TY;
  constexpr int PX = TX + 2 * R, PY = TY + 2 * R, PL = PX * PY;
  constexpr int NXS = (TX + 1) * TY, NYS = TX * (TY + 1);
  constexpr int NF = 3 + NTR;
  constexpr int NFILL = (PL + NT - 1) / NT;
  constexpr int NW = 2 * R;            // register window: levels k-R+1 .. k+R
  constexpr int NI = 2 * R - 2;        // levels of the z interpolation to face k
  constexpr int NE = TX + TY;          // edge columns (x) and rows (y)
  constexpr int NRING = (R == 3) ? 4 : 8;
  static_assert(NRING >= NI, "edge ring too short");
  // LDS map: u, v (level k), w (levels k, k+1), tracers (level k), the
  // z-interpolated u at x faces and v at y faces, the edge rings, then the
  // x-face fluxes (NF arrays of NXS) and y-face fluxes (NF arrays of NYS)
  constexpr int OU = 0, OV = PL, OW = 2 * PL, OC = 4 * PL;
  constexpr int OM = (4 + NTR) * PL;   // mask plane (level k), IMM only
  constexpr int OAX = (4 + NTR + (IMM ? 1 : 0)) * PL, OAY = OAX + NXS;
  constexpr int OER = OAY + NYS;
  constexpr int OFX = OER + NRING * NE, OFY = OFX + NF * NXS;
  constexpr int NLDS = OFY + NF * NYS;
  __shared__ T S[NLDS];

  const int bx = b % nbx;
  const int by = (b / nbx) % nby;
  const int bz = b / (nbx * nby);
  const int i0 = bx * TX, j0 = by * TY;
  const int kb = bz * kc;
  const int ke = min(kb + kc, d.nz);

  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;
  const int gi = i0 + tx, gj = j0 + ty;
  const int Lc = (ty + R) * PX + (tx + R);  // own position in an LDS plane
  const T eps = P.eps;
  const long sz = d.sz;
  const int sy = (int)d.sy;
  const int hh = d.h;

  // 32-bit offsets of the plane elements this thread loads, relative to the
  // tile corner (i0-R, j0-R) of a level; the same for every level
  int goff[NFILL];
#pragma unroll
  for (int r = 0; r < NFILL; ++r) {
    const int e = tid + r * NT;
    const int ly = e / PX, lx = e - ly * PX;
    goff[r] = ly * sy + lx;
  }
  const long corner = (long)(j0 - R + hh) * sy + (i0 - R + hh);
  auto fill = [&](int dst, const T* __restrict__ src, int kk) {
    const T* __restrict__ base = src + (long)(kk + hh) * sz + corner;
#pragma unroll
    for (int r = 0; r < NFILL; ++r) {
      const int e = tid + r * NT;
      if (PL % NT == 0 || e < PL) S[dst + e] = base[goff[r]];
    }
  };
  auto rw = [](int kk) { return OW + (kk & 1) * PL; };

  const T* __restrict__ gu = fs.in[0];
  const T* __restrict__ gv = fs.in[1];
  const T* __restrict__ gw = fs.in[2];

  // ---- edge rings: thread e < TY owns the u column right of the tile (row
  // j0+e), thread TY <= e < NE the v row above it (column i0+e-TY); each
  // keeps levels k-R+1 .. k+R-2 of it in a private LDS ring
  const bool edge = tid < NE;
  const T* __restrict__ ecol = nullptr;
  if (edge) {
    ecol = (tid < TY) ? gu + ((long)(j0 + tid + hh) * sy + (i0 + TX + hh))
                      : gv + ((long)(j0 + TY + hh) * sy + (i0 + tid - TY + hh));
  }
  auto ering = [&](int kk) { return OER + (kk & (NRING - 1)) * NE + tid; };

  // ---- register windows: levels k-R+1..k+R of the own column (index o is
  // level k-R+1+o)
  const int col = (gj + hh) * sy + (gi + hh);   // offset within a level
  T wu[NW], wv[NW], ww[NW], wc[NTR][NW];
#pragma unroll
  for (int o = 0; o < NW; ++o) {
    const long lv = (long)(kb - R + 1 + o + hh) * sz;
    wu[o] = (gu + lv)[col];
    wv[o] = (gv + lv)[col];
    ww[o] = (gw + lv)[col];
#pragma unroll
    for (int q = 0; q < NTR; ++q) wc[q][o] = (fs.in[3 + q] + lv)[col];
  }
  if (edge) {
#pragma unroll
    for (int o = 0; o < NI - 1; ++o) {
      const int kk = kb - R + 1 + o;
      S[ering(kk)] = ecol[(long)(kk + hh) * sz];
    }
  }
  // immersed boundary: the own column's mask at levels k-1, k, k+1
  T mkm = T(1), mk0 = T(1), mkp = T(1);
  if (IMM) {
    mkm = (fs.mask + (long)(kb - 1 + hh) * sz)[col];
    mk0 = (fs.mask + (long)(kb + hh) * sz)[col];
    mkp = (fs.mask + (long)(kb + 1 + hh) * sz)[col];
  }

  // ---- prologue: w at level kb
  fill(rw(kb), gw, kb);
  __syncthreads();

  // bottom z fluxes of the first level (face kb; w: centre kb-1), from the
  // levels kb-R..kb+R-1
  T fzb_u, fzb_v, fzb_w, fzb_c[NTR];
  {
    const long lv = (long)(kb - R + hh) * sz;
    const T* wp = S + rw(kb);
    const bool wall = d.zb && kb == 0;
    T z[NW];
    const T wt_u = interp_lds<T, R>(wp, Lc, 1);
    const T wt_v = interp_lds<T, R>(wp, Lc, PX);
    const T rzb = P.rdzf[kb];  // face kb
    z[0] = (gu + lv)[col];
#pragma unroll
    for (int o = 1; o < NW; ++o) z[o] = wu[o - 1];
    fzb_u = wall ? T(0) : flux_reg<T, SCHEME, R>(z, wt_u, eps) - P.nuz * (z[R] - z[R - 1]) * rzb;
    z[0] = (gv + lv)[col];
#pragma unroll
    for (int o = 1; o < NW; ++o) z[o] = wv[o - 1];
    fzb_v = wall ? T(0) : flux_reg<T, SCHEME, R>(z, wt_v, eps) - P.nuz * (z[R] - z[R - 1]) * rzb;
    z[0] = (gw + lv)[col];
#pragma unroll
    for (int o = 1; o < NW; ++o) z[o] = ww[o - 1];
    const T wb = interpc<T, R>(z + 1);
    fzb_w = flux_reg<T, SCHEME, R>(z, wb, eps) - P.nuz * (z[R] - z[R - 1]) * P.rdzc[kb - 1];
    const T wface = z[R];
#pragma unroll
    for (int q = 0; q < NTR; ++q) {
      z[0] = (fs.in[3 + q] + lv)[col];
#pragma unroll
      for (int o = 1; o < NW; ++o) z[o] = wc[q][o - 1];
      fzb_c[q] = wall ? T(0)
                      : flux_reg<T, SCHEME, R>(z, wface, eps) -
                            (IMM ? P.kappaz * (mkm * mk0) : P.kappaz) * (z[R] - z[R - 1]) * rzb;
    }
  }

  for (int k = kb; k < ke; ++k) {
    __syncthreads();  // consumers of the previous level are done
    fill(OU, gu, k);
    fill(OV, gv, k);
    fill(rw(k + 1), gw, k + 1);
#pragma unroll
    for (int q = 0; q < NTR; ++q) fill(OC + q * PL, fs.in[3 + q], k);
    if (IMM) fill(OM, fs.mask, k);
    // u and v interpolated in z to face k (levels k-R+1 .. k+R-2): own
    // column from the register window, edge columns from their rings
    S[OAX + ty * (TX + 1) + tx] = interpc<T, R>(wu);
    S[OAY + ty * TX + tx] = interpc<T, R>(wv);
    if (edge) {
      S[ering(k + R - 2)] = ecol[(long)(k + R - 2 + hh) * sz];
      T a[NI];
#pragma unroll
      for (int o = 0; o < NI; ++o) a[o] = S[ering(k - R + 1 + o)];
      const int fi = (tid < TY) ? OAX + tid * (TX + 1) + TX : OAY + TY * TX + (tid - TY);
      S[fi] = interpc<T, R>(a);
    }
    __syncthreads();

    // ---- x and y face fluxes
    SlotOff ox, oy;
    ox.vd = OU; ox.ve = OV; ox.az = OAX;
    ox.wk = rw(k); ox.c0 = OC;
    ox.Fself = OFX + 0 * NXS; ox.Fcross = OFX + 1 * NXS; ox.Fw = OFX + 2 * NXS;
    ox.Fc0 = OFX + 3 * NXS; ox.Fstride = NXS;
    oy.vd = OV; oy.ve = OU; oy.az = OAY;
    oy.wk = rw(k); oy.c0 = OC;
    oy.Fself = OFY + 1 * NYS; oy.Fcross = OFY + 0 * NYS; oy.Fw = OFY + 2 * NYS;
    oy.Fc0 = OFY + 3 * NYS; oy.Fstride = NYS;
    // main rounds: the left x face and the bottom y face of the own cell
    slot_fluxes<T, SCHEME, NTR, PL, R, IMM>(S, ox, Lc, 1, PX, ty * (TX + 1) + tx, P.rdx, P.nu,
                                            P.kappa, eps, OM);
    __builtin_amdgcn_sched_barrier(0);
    slot_fluxes<T, SCHEME, NTR, PL, R, IMM>(S, oy, Lc, PX, 1, ty * TX + tx, P.rdy, P.nu, P.kappa,
                                            eps, OM);
    __builtin_amdgcn_sched_barrier(0);
    // edge round: right x faces of the last column, top y faces of the last row
    if (edge) {
      const bool xs = tid < TY;
      const int L = xs ? (tid + R) * PX + (TX + R) : (TY + R) * PX + (tid - TY + R);
      const int fi = xs ? tid * (TX + 1) + TX : TY * TX + (tid - TY);
      SlotOff oe;
      oe.vd = xs ? ox.vd : oy.vd; oe.ve = xs ? ox.ve : oy.ve; oe.az = xs ? ox.az : oy.az;
      oe.wk = ox.wk; oe.c0 = OC;
      oe.Fself = xs ? ox.Fself : oy.Fself; oe.Fcross = xs ? ox.Fcross : oy.Fcross;
      oe.Fw = xs ? ox.Fw : oy.Fw; oe.Fc0 = xs ? ox.Fc0 : oy.Fc0;
      oe.Fstride = xs ? NXS : NYS;
      slot_fluxes<T, SCHEME, NTR, PL, R, IMM>(S, oe, L, xs ? 1 : PX, xs ? PX : 1, fi,
                                              xs ? P.rdx : P.rdy, P.nu, P.kappa, eps, OM);
    }

    // ---- z fluxes through the top face of level k (w: at centre k)
    const bool top_wall = d.zb && (k + 1 == d.nz);
    // inverse spacings of this level (uniform across the workgroup): the top
    // face k+1, the cell k, and face k (the thickness of the w cell)
    const T rzft = P.rdzf[k + 1], rzc = P.rdzc[k], rzf = P.rdzf[k];
    T fzt_u, fzt_v, fzt_w, fzt_c[NTR];
    {
      const T* wp = S + rw(k + 1);
      const T wt_u = interp_lds<T, R>(wp, Lc, 1);
      const T wt_v = interp_lds<T, R>(wp, Lc, PX);
      fzt_u = top_wall ? T(0)
                       : flux_reg<T, SCHEME, R>(wu, wt_u, eps) - P.nuz * (wu[R] - wu[R - 1]) * rzft;
      fzt_v = top_wall ? T(0)
                       : flux_reg<T, SCHEME, R>(wv, wt_v, eps) - P.nuz * (wv[R] - wv[R - 1]) * rzft;
      const T wb = interpc<T, R>(ww + 1);
      fzt_w = flux_reg<T, SCHEME, R>(ww, wb, eps) - P.nuz * (ww[R] - ww[R - 1]) * rzc;
      const T kapz = IMM ? P.kappaz * (mk0 * mkp) : P.kappaz;
#pragma unroll
      for (int q = 0; q < NTR; ++q)
        fzt_c[q] = top_wall ? (IMM ? P.top_flux[q] * mk0 : P.top_flux[q])
                            : flux_reg<T, SCHEME, R>(wc[q], ww[R], eps) -
                                  kapz * (wc[q][R] - wc[q][R - 1]) * rzft;
    }
    __syncthreads();  // all x/y fluxes of level k are in LDS

    // ---- tendencies of the own cell and the RK3 combine
    {
      const int ix = ty * (TX + 1) + tx;
      const int iy = ty * TX + tx;
      T G[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f)
        G[f] = -(S[OFX + f * NXS + ix + 1] - S[OFX + f * NXS + ix]) * P.rdx -
               (S[OFY + f * NYS + iy + TX] - S[OFY + f * NYS + iy]) * P.rdy;
      const T* uk = S + OU;
      const T* vk = S + OV;
      G[0] += -(fzt_u - fzb_u) * rzc +
              P.f * T(0.25) * (vk[Lc - 1] + vk[Lc] + vk[Lc - 1 + PX] + vk[Lc + PX]);
      G[1] += -(fzt_v - fzb_v) * rzc -
              P.f * T(0.25) * (uk[Lc - PX] + uk[Lc + 1 - PX] + uk[Lc] + uk[Lc + 1]);
      G[2] += -(fzt_w - fzb_w) * rzf;
      if (NTR >= 2 && P.buoyancy) {
        const T bl = P.g_alpha * (wc[0][R - 2] - P.t_ref) - P.g_beta * (wc[1][R - 2] - P.s_ref);
        const T bu = P.g_alpha * (wc[0][R - 1] - P.t_ref) - P.g_beta * (wc[1][R - 1] - P.s_ref);
        G[2] += T(0.5) * (bl + bu);
      }
      const bool bottom_wall = d.zb && k == 0;
      if (bottom_wall) G[2] = T(0);
      if (IMM) {
        // velocities on faces next to an immersed cell do not change
        const T* mk = S + OM;
        G[0] *= mk[Lc - 1] * mk[Lc];
        G[1] *= mk[Lc - PX] * mk[Lc];
        G[2] *= mkm * mk0;
      }
      const T divu = (uk[Lc + 1] - uk[Lc]) * P.rdx + (vk[Lc + PX] - vk[Lc]) * P.rdy +
                     (ww[R] - ww[R - 1]) * rzc;
#pragma unroll
      for (int q = 0; q < NTR; ++q) G[3 + q] += -(fzt_c[q] - fzb_c[q]) * rzc - P.toff[q] * divu;

      const long lv = (long)(k + hh) * sz;
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        // plus the closure tendency computed beforehand
        const T g = (CLO && fs.closure[f]) ? G[f] + (fs.closure[f] + lv)[col] : G[f];
        T* __restrict__ Gf = fs.G[f] + lv;
        if (P.combine) {
          T x;
          if (f == 0) x = wu[R - 1];
          else if (f == 1) x = wv[R - 1];
          else if (f == 2) x = ww[R - 1];
          else x = wc[f - 3][R - 1];
          T incr = P.gam * g;
          if (P.stage > 0) incr -= P.zet * Gf[col];
          x = x + P.dt * incr;
          if (f == 2 && bottom_wall) x = T(0);
          if (f >= 3 && P.images)
            store_with_images(fs.out[f], d, gi, gj, k, x, false);  // tracers: final values
          else
            (fs.out[f] + lv)[col] = x;
          if (P.stage < 2) Gf[col] = g;
        } else {
          Gf[col] = g;
        }
      }
    }

    // ---- advance: top fluxes become bottom fluxes, windows shift up
    fzb_u = fzt_u;
    fzb_v = fzt_v;
    fzb_w = fzt_w;
#pragma unroll
    for (int q = 0; q < NTR; ++q) fzb_c[q] = fzt_c[q];
    if (IMM && k + 1 < ke) {
      mkm = mk0;
      mk0 = mkp;
      mkp = (fs.mask + (long)(k + 2 + hh) * sz)[col];
    }
    if (k + 1 < ke) {
      const long lv = (long)(k + R + 1 + hh) * sz;
#pragma unroll
      for (int o = 0; o < NW - 1; ++o) {
        wu[o] = wu[o + 1];
        wv[o] = wv[o + 1];
        ww[o] = ww[o + 1];
#pragma unroll
        for (int q = 0; q < NTR; ++q) wc[q][o] = wc[q][o + 1];
      }
      wu[NW - 1] = (gu + lv)[col];
      wv[NW - 1] = (gv + lv)[col];
      ww[NW - 1] = (gw + lv)[col];
#pragma unroll
      for (int q = 0; q < NTR; ++q) wc[q][NW - 1] = (fs.in[3 + q] + lv)[col];
    }
  }
}

// Waves per SIMD the kernel is compiled for: the WENO7/9 windows and
// reconstructions need more registers than WENO5's.
template <class T, int R>
struct TendWaves {
  static constexpr int value = sizeof(T) == 8 ? 2 : (R == 3 ? OC_TEND_WAVES : 3);
};

// One model; tiles are mapped XCD-major, so neighbouring tiles (which share
// halo loads) land on the same XCD and its L2.
template <class T, int SCHEME, int NTR, int TX, int TY, int R, bool CLO, bool IMM = false>
__global__ void __launch_bounds__(TX * TY)
    __attribute__((amdgpu_waves_per_eu(TendWaves<T, R>::value)))
    tendency_zmarch(Dims d, FieldSet<T> fs, TendParams<T> P, int nbx, int nby, int nbz, int kc) {
  const int nblk = nbx * nby * nbz;
  int b = blockIdx.x;
  if ((nblk & 7) == 0) b = (b & 7) * (nblk >> 3) + (b >> 3);
  tendency_tile<T, SCHEME, NTR, TX, TY, R, CLO, IMM>(d, fs, P, nbx, nby, nbz, kc, b);
}

}  // namespace tz

// Launch the single-model kernel of radius R; scheme is tz::SCHEME_*.
template <class T, int R, int WTX, int WTY>
hipError_t launch_tendency_radius(const Dims& d, const FieldSet<T>& fs, const TendParams<T>& p,
                                  int scheme, hipStream_t s) {
  const bool wide = (d.nx % WTX == 0) && (d.ny % WTY == 0);
  const int TX = wide ? WTX : 8, TY = wide ? WTY : 8;
  if (d.nx % TX || d.ny % TY || d.h < R) return hipErrorInvalidValue;
  const int nbx = d.nx / TX, nby = d.ny / TY;
  int kc = (int)((long)d.nz * nbx * nby / OC_TEND_KC_DIV);
  kc = kc < 4 ? 4 : (kc > 64 ? 64 : kc);
  if (kc > d.nz) kc = d.nz;
  const int nbz = (d.nz + kc - 1) / kc;
  const dim3 grid(nbx * nby * nbz);
  bool clo = false;
  for (int f = 0; f < MAXF; ++f) clo = clo || fs.closure[f] != nullptr;
  const bool imm = fs.mask != nullptr;
  if (imm && (R != 3 || clo)) return hipErrorInvalidValue;
#define OC_TZ(SCH, NTR_, TX_, TY_)                                                            \
  if (imm) {                                                                                  \
    if constexpr (R == 3)                                                                     \
      hipLaunchKernelGGL((tz::tendency_zmarch<T, SCH, NTR_, TX_, TY_, R, false, true>), grid,  \
                         dim3(TX_ * TY_), 0, s, d, fs, p, nbx, nby, nbz, kc);                 \
  } else if (clo)                                                                             \
    hipLaunchKernelGGL((tz::tendency_zmarch<T, SCH, NTR_, TX_, TY_, R, true>), grid,           \
                       dim3(TX_ * TY_), 0, s, d, fs, p, nbx, nby, nbz, kc);                   \
  else                                                                                        \
    hipLaunchKernelGGL((tz::tendency_zmarch<T, SCH, NTR_, TX_, TY_, R, false>), grid,          \
                       dim3(TX_ * TY_), 0, s, d, fs, p, nbx, nby, nbz, kc)
#define OC_TZ_NTR(SCH, TX_, TY_)                \
  switch (p.ntr) {                              \
    case 1: OC_TZ(SCH, 1, TX_, TY_); break;     \
    case 2: OC_TZ(SCH, 2, TX_, TY_); break;     \
    case 3: OC_TZ(SCH, 3, TX_, TY_); break;     \
    default: OC_TZ(SCH, 4, TX_, TY_); break;    \
  }
#define OC_TZ_TX(SCH)                                        \
  if (wide) { OC_TZ_NTR(SCH, WTX, WTY) } else { OC_TZ_NTR(SCH, 8, 8) }
  switch (scheme) {
    case tz::SCHEME_NONE:
      if constexpr (R == 3) { OC_TZ_TX(tz::SCHEME_NONE); break; }
      return hipErrorInvalidValue;
    case tz::SCHEME_WENOZ: OC_TZ_TX(tz::SCHEME_WENOZ); break;
    default: OC_TZ_TX(tz::SCHEME_LINEAR); break;
  }
#undef OC_TZ_TX
#undef OC_TZ_NTR
#undef OC_TZ
  return hipGetLastError();
}

template <class T>
hipError_t launch_tendency_r4(const Dims& d, const FieldSet<T>& fs, const TendParams<T>& p,
                              int scheme, hipStream_t s);
template <class T>
hipError_t launch_tendency_r5(const Dims& d, const FieldSet<T>& fs, const TendParams<T>& p,
                              int scheme, hipStream_t s);

}  // namespace oc
