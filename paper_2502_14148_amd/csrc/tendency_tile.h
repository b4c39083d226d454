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

// ---- buffer addressing -----------------------------------------------------
// One buffer resource spans all fields of a model (byte offsets below 4 GiB
// from FieldSet::base): loads and stores take a per-lane 32-bit offset (the
// column, fixed over the march) and a wave-uniform one (field and level), so
// no per-lane 64-bit address arithmetic is spent on them.  Whole planes of a
// level are copied into LDS by the buffer unit itself (load-to-LDS), one
// dword per lane, 64 consecutive dwords per wave, while the previous level is
// being computed.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const char* base) {
  // raw buffer, no stride, the whole 32-bit range; word 3 as for every gfx9
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(base), (short)0, (int)0xFFFFFFFF,
                                           0x00020000);
}

template <class T>
__device__ inline T bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

template <class T>
__device__ inline void bstore(T v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(T) == 4)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, voff, soff, 0);
  else
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
}

// Wait for this wave's outstanding vector-memory operations (the load-to-LDS
// copies among them).
__device__ inline void wait_vm() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

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
  {
    const T* vd = S + o.vd;
    const T* ve = S + o.ve;
    const T adv = interp_lds<T, R>(vd, L, se);
    S[o.Fcross + fi] = flux_lds<T, SCHEME, R>(ve, L, sd, adv, eps) - nu * (ve[L] - ve[L - sd]) * rd;
  }
  {
    const T adv = S[o.az + fi];
    const T* wk = S + o.wk;
    S[o.Fw + fi] = flux_lds<T, SCHEME, R>(wk, L, sd, adv, eps) - nu * (wk[L] - wk[L - sd]) * rd;
  }
  const T un = S[o.vd + L];
  const T kap = IMM ? kappa * (S[om + L] * S[om + L - sd]) : kappa;
#pragma unroll
  for (int q = 0; q < NTR; ++q) {
    const T* c = S + o.c0 + q * PL;
    S[o.Fc0 + q * o.Fstride + fi] =
        flux_lds<T, SCHEME, R>(c, L, sd, un, eps) - kap * (c[L] - c[L - sd]) * rd;
  }
}

// Shape of the load-to-LDS copy of one (TX + 2R) x (TY + 2R) plane of
// elements of ES bytes by NT threads: NR rounds in which every lane copies one
// dword, then NCH chunks of 64 dwords, chunk c copied by wave c % (NT / 64)
// (lanes past the plane copy its last dword into the padding).  PLP: the
// plane's padded length in elements.
template <int PX, int PY, int NT, int ES>
struct PlaneCopy {
  static constexpr int DPE = ES / 4;
  static constexpr int PLD = PX * PY * DPE;
  static constexpr int NR = PLD / NT;
  static constexpr int REM = PLD - NR * NT;
  static constexpr int NCH = (REM + 63) / 64;
  static constexpr int NWV = NT / 64;
  static constexpr int MAXC = (NCH + NWV - 1) / NWV;   // chunks per wave, at most
  static constexpr int PLP = (NR * NT + NCH * 64) / DPE;
  static_assert(NT % 64 == 0, "whole wavefronts");
  static_assert((NR * NT + NCH * 64) % DPE == 0, "whole elements");
};

// One column tile: tile b of an nbx x nby x nbz decomposition (k chunks of
// kc levels) of the grid d, whose halo width d.h is at least R.
// CLO: add the closure tendencies computed beforehand (fs.closure; learned
// closure: u, v, w and tracer 0, LES closure: every field).  A separate
// instantiation keeps the plain kernel's registers free of them.
// IMM: grid-fitted immersed boundary (fs.mask, 1 in fluid cells): zero
// velocity tendencies on faces next to an immersed cell, no diffusive tracer
// flux through them, no top flux into an immersed top cell.
//
// LDS: the planes of level k (u, v, the tracers, the mask) in one of two
// buffers by the parity of k, w in a ring of three (levels k, k + 1 in use,
// k + 2 being copied), the z-interpolated u at x faces and v at y faces, the
// edge rings, and the x- and y-face flux arrays.  The copies of level k + 1
// (w: k + 2) are issued when level k starts and are waited for at its end,
// where the face velocities of level k + 1 are also written: two barriers
// per level (fluxes -> tendencies, level -> next level).
template <class T, int SCHEME, int NTR, int TX, int TY, int R, bool CLO = false,
          bool IMM = false>
__device__ __attribute__((always_inline)) inline void tendency_tile(
    const Dims& d, const FieldSet<T>& fs, const TendParams<T>& P, int nbx, int nby, int nbz,
    int kc, int b) {
  constexpr int NT = TX * TY;
  constexpr int ES = (int)sizeof(T);
  constexpr int PX = TX + 2 * R, PY = TY + 2 * R;
  using PC = PlaneCopy<PX, PY, NT, ES>;
  constexpr int PLP = PC::PLP;
  constexpr int NXS = (TX + 1) * TY, NYS = TX * (TY + 1);
  constexpr int NF = 3 + NTR;
  constexpr int NW = 2 * R;            // register window: levels k-R+1 .. k+R
  constexpr int NI = 2 * R - 2;        // levels of the z interpolation to face k
  constexpr int NE = TX + TY;          // edge columns (x) and rows (y)
  constexpr int NRING = (R == 3) ? 4 : 8;
  static_assert(NRING >= NI, "edge ring too short");
  constexpr int NPL = 2 + NTR + (IMM ? 1 : 0);   // planes per level buffer
  // LDS map (elements)
  constexpr int OLB = 0;                         // 2 level buffers of NPL planes
  constexpr int OWR = 2 * NPL * PLP;             // w ring of 3 planes
  constexpr int OAX = OWR + 3 * PLP, OAY = OAX + NXS;
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
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int tx = tid % TX, ty = tid / TX;
  const int gi = i0 + tx, gj = j0 + ty;
  const int Lc = (ty + R) * PX + (tx + R);  // own position in an LDS plane
  const T eps = P.eps;
  const int sy = (int)d.sy;
  const int hh = d.h;
  const uint32_t lvb = (uint32_t)d.sz * ES;     // bytes per level
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(fs.base);

  // per-lane byte offsets of the copied plane dwords, relative to the tile
  // corner (i0-R, j0-R) of a level: the same for every field and level
  auto dword_off = [&](int j) -> uint32_t {
    if (j > PC::PLD - 1) j = PC::PLD - 1;
    const int e = j / PC::DPE, half = j - e * PC::DPE;
    const int ly = e / PX, lx = e - ly * PX;
    return (uint32_t)((ly * sy + lx) * ES + half * 4);
  };
  uint32_t goff[PC::NR + PC::MAXC];
#pragma unroll
  for (int r = 0; r < PC::NR; ++r) goff[r] = dword_off(r * NT + tid);
#pragma unroll
  for (int c = 0; c < PC::MAXC; ++c)
    goff[PC::NR + c] = dword_off(PC::NR * NT + (wave + c * PC::NWV) * 64 + lane);
  const uint32_t corner = (uint32_t)(((j0 - R + hh) * sy + (i0 - R + hh)) * ES);
  // copy plane `src` (byte offset of the field) at level kk into LDS plane dst
  auto copy_plane = [&](int dst, uint32_t src, int kk) {
    const uint32_t so = src + (uint32_t)(kk + hh) * lvb + corner;
#pragma unroll
    for (int r = 0; r < PC::NR; ++r)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (void*)(S + dst + (r * NT + wave * 64) / PC::DPE),
                                               4, goff[r], so, 0, 0);
#pragma unroll
    for (int c = 0; c < PC::MAXC; ++c) {
      const int ch = wave + c * PC::NWV;
      if (ch < PC::NCH)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rs, (void*)(S + dst + (PC::NR * NT + ch * 64) / PC::DPE), 4, goff[PC::NR + c], so, 0,
            0);
    }
  };
  auto lbuf = [](int kk) { return OLB + (kk & 1) * NPL * PLP; };
  auto wring = [](int kk) { return OWR + (kk % 3) * PLP; };
  // planes of level kk (u, v, tracers, mask) into its buffer
  auto copy_level = [&](int kk) {
    const int lb = lbuf(kk);
    copy_plane(lb, fs.oin[0], kk);
    copy_plane(lb + PLP, fs.oin[1], kk);
#pragma unroll
    for (int q = 0; q < NTR; ++q) copy_plane(lb + (2 + q) * PLP, fs.oin[3 + q], kk);
    if (IMM) copy_plane(lb + (2 + NTR) * PLP, fs.omask, kk);
  };

  // own column: byte offset within a level
  const uint32_t col = (uint32_t)(((gj + hh) * sy + (gi + hh)) * ES);
  auto lvl = [&](int kk) { return (uint32_t)(kk + hh) * lvb; };

  // ---- edge rings: thread e < TY owns the u column right of the tile (row
  // j0+e), thread TY <= e < NE the v row above it (column i0+e-TY); each
  // keeps levels k-R+1 .. k+R-2 of it in a private LDS ring
  const bool edge = tid < NE;
  uint32_t ecol = 0;   // field and column byte offset (per lane), level 0
  if (edge) {
    ecol = (tid < TY) ? fs.oin[0] + (uint32_t)(((j0 + tid + hh) * sy + (i0 + TX + hh)) * ES)
                      : fs.oin[1] + (uint32_t)(((j0 + TY + hh) * sy + (i0 + tid - TY + hh)) * ES);
  }
  auto ering = [&](int kk) { return OER + (kk & (NRING - 1)) * NE + tid; };

  // ---- register windows: levels k-R+1..k+R of the own column (index o is
  // level k-R+1+o)
  T wu[NW], wv[NW], ww[NW], wc[NTR][NW];
#pragma unroll
  for (int o = 0; o < NW; ++o) {
    const uint32_t lv = lvl(kb - R + 1 + o);
    wu[o] = bload<T>(rs, col, fs.oin[0] + lv);
    wv[o] = bload<T>(rs, col, fs.oin[1] + lv);
    ww[o] = bload<T>(rs, col, fs.oin[2] + lv);
#pragma unroll
    for (int q = 0; q < NTR; ++q) wc[q][o] = bload<T>(rs, col, fs.oin[3 + q] + lv);
  }
  if (edge) {
#pragma unroll
    for (int o = 0; o < NI - 1; ++o) {
      const int kk = kb - R + 1 + o;
      S[ering(kk)] = bload<T>(rs, ecol, lvl(kk));
    }
  }
  // immersed boundary: the own column's mask at levels k-1, k, k+1
  T mkm = T(1), mk0 = T(1), mkp = T(1);
  if (IMM) {
    mkm = bload<T>(rs, col, fs.omask + lvl(kb - 1));
    mk0 = bload<T>(rs, col, fs.omask + lvl(kb));
    mkp = bload<T>(rs, col, fs.omask + lvl(kb + 1));
  }

  // u and v interpolated in z to face kk (levels kk-R+1 .. kk+R-2): own
  // column from the register window, edge columns from their rings (the
  // ring already holds level kk+R-2)
  auto face_velocities = [&](int kk) {
    S[OAX + ty * (TX + 1) + tx] = interpc<T, R>(wu);
    S[OAY + ty * TX + tx] = interpc<T, R>(wv);
    if (edge) {
      T a[NI];
#pragma unroll
      for (int o = 0; o < NI; ++o) a[o] = S[ering(kk - R + 1 + o)];
      const int fi = (tid < TY) ? OAX + tid * (TX + 1) + TX : OAY + TY * TX + (tid - TY);
      S[fi] = interpc<T, R>(a);
    }
  };

  // ---- prologue: the planes of level kb, w at kb and kb + 1, and the
  // face velocities of level kb
  copy_level(kb);
  copy_plane(wring(kb), fs.oin[2], kb);
  copy_plane(wring(kb + 1), fs.oin[2], kb + 1);
  if (edge) S[ering(kb + R - 2)] = bload<T>(rs, ecol, lvl(kb + R - 2));
  face_velocities(kb);
  wait_vm();
  __syncthreads();

  // bottom z fluxes of the first level (face kb; w: centre kb-1), from the
  // levels kb-R..kb+R-1
  T fzb_u, fzb_v, fzb_w, fzb_c[NTR];
  {
    const uint32_t lv = lvl(kb - R);
    const T* wp = S + wring(kb);
    const bool wall = d.zb && kb == 0;
    T z[NW];
    const T wt_u = interp_lds<T, R>(wp, Lc, 1);
    const T wt_v = interp_lds<T, R>(wp, Lc, PX);
    const T rzb = glb(P.rdzf)[kb];  // face kb
    z[0] = bload<T>(rs, col, fs.oin[0] + lv);
#pragma unroll
    for (int o = 1; o < NW; ++o) z[o] = wu[o - 1];
    fzb_u = wall ? T(0) : flux_reg<T, SCHEME, R>(z, wt_u, eps) - P.nuz * (z[R] - z[R - 1]) * rzb;
    z[0] = bload<T>(rs, col, fs.oin[1] + lv);
#pragma unroll
    for (int o = 1; o < NW; ++o) z[o] = wv[o - 1];
    fzb_v = wall ? T(0) : flux_reg<T, SCHEME, R>(z, wt_v, eps) - P.nuz * (z[R] - z[R - 1]) * rzb;
    z[0] = bload<T>(rs, col, fs.oin[2] + lv);
#pragma unroll
    for (int o = 1; o < NW; ++o) z[o] = ww[o - 1];
    const T wb = interpc<T, R>(z + 1);
    fzb_w = flux_reg<T, SCHEME, R>(z, wb, eps) - P.nuz * (z[R] - z[R - 1]) * glb(P.rdzc)[kb - 1];
    const T wface = z[R];
#pragma unroll
    for (int q = 0; q < NTR; ++q) {
      z[0] = bload<T>(rs, col, fs.oin[3 + q] + lv);
#pragma unroll
      for (int o = 1; o < NW; ++o) z[o] = wc[q][o - 1];
      fzb_c[q] = wall ? T(0)
                      : flux_reg<T, SCHEME, R>(z, wface, eps) -
                            (IMM ? P.kappaz * (mkm * mk0) : P.kappaz) * (z[R] - z[R - 1]) * rzb;
    }
  }

  for (int k = kb; k < ke; ++k) {
    // The planes of level k and w at k, k + 1 are in LDS (waited for at the
    // end of the previous level).  Loads are issued in the order they are
    // needed (vector-memory loads complete in issue order): the edge column
    // of this level, the previous tendencies and closure tendencies of this
    // level, the own column's next level, then the copies for level k + 1.
    const bool more = k + 1 < ke;
    const uint32_t lv = lvl(k);
    T enext = T(0);
    if (edge && more) enext = bload<T>(rs, ecol, lvl(k + R - 1));
    T gprev[NF], gclo[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      gprev[f] = (P.combine && P.stage > 0) ? bload<T>(rs, col, fs.oG[f] + lv) : T(0);
      gclo[f] = (CLO && fs.closure[f]) ? bload<T>(rs, col, fs.oclo[f] + lv) : T(0);
    }
    T nu_ = T(0), nv_ = T(0), nw_ = T(0), nc_[NTR];
    T nmk = T(1);
    if (more) {
      const uint32_t ln = lvl(k + R + 1);
      nu_ = bload<T>(rs, col, fs.oin[0] + ln);
      nv_ = bload<T>(rs, col, fs.oin[1] + ln);
      nw_ = bload<T>(rs, col, fs.oin[2] + ln);
#pragma unroll
      for (int q = 0; q < NTR; ++q) nc_[q] = bload<T>(rs, col, fs.oin[3 + q] + ln);
      if (IMM) nmk = bload<T>(rs, col, fs.omask + lvl(k + 2));
      copy_level(k + 1);
      copy_plane(wring(k + 2), fs.oin[2], k + 2);
    }
    const int lb = lbuf(k);
    const int OU = lb, OV = lb + PLP, OC = lb + 2 * PLP, OM = lb + (2 + NTR) * PLP;
    const int OWk = wring(k), OWk1 = wring(k + 1);
    // ---- x and y face fluxes (the face velocities of level k were written
    // before the barrier that ended the previous level)
    SlotOff ox, oy;
    ox.vd = OU; ox.ve = OV; ox.az = OAX;
    ox.wk = OWk; ox.c0 = OC;
    ox.Fself = OFX + 0 * NXS; ox.Fcross = OFX + 1 * NXS; ox.Fw = OFX + 2 * NXS;
    ox.Fc0 = OFX + 3 * NXS; ox.Fstride = NXS;
    oy.vd = OV; oy.ve = OU; oy.az = OAY;
    oy.wk = OWk; oy.c0 = OC;
    oy.Fself = OFY + 1 * NYS; oy.Fcross = OFY + 0 * NYS; oy.Fw = OFY + 2 * NYS;
    oy.Fc0 = OFY + 3 * NYS; oy.Fstride = NYS;
    // main rounds: the left x face and the bottom y face of the own cell
    slot_fluxes<T, SCHEME, NTR, PLP, R, IMM>(S, ox, Lc, 1, PX, ty * (TX + 1) + tx, P.rdx, P.nu,
                                             P.kappa, eps, OM);
    __builtin_amdgcn_sched_barrier(0);
    slot_fluxes<T, SCHEME, NTR, PLP, R, IMM>(S, oy, Lc, PX, 1, ty * TX + tx, P.rdy, P.nu,
                                             P.kappa, eps, OM);
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
      slot_fluxes<T, SCHEME, NTR, PLP, R, IMM>(S, oe, L, xs ? 1 : PX, xs ? PX : 1, fi,
                                               xs ? P.rdx : P.rdy, P.nu, P.kappa, eps, OM);
    }

    // ---- z fluxes through the top face of level k (w: at centre k)
    const bool top_wall = d.zb && (k + 1 == d.nz);
    // inverse spacings of this level (uniform across the workgroup): the top
    // face k+1, the cell k, and face k (the thickness of the w cell)
    const T rzft = glb(P.rdzf)[k + 1], rzc = glb(P.rdzc)[k], rzf = glb(P.rdzf)[k];
    T fzt_u, fzt_v, fzt_w, fzt_c[NTR];
    {
      const T* wp = S + OWk1;
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

#pragma unroll
      for (int f = 0; f < NF; ++f) {
        // plus the closure tendency computed beforehand
        const T g = (CLO && fs.closure[f]) ? G[f] + gclo[f] : G[f];
        if (P.combine) {
          T x;
          if (f == 0) x = wu[R - 1];
          else if (f == 1) x = wv[R - 1];
          else if (f == 2) x = ww[R - 1];
          else x = wc[f - 3][R - 1];
          T incr = P.gam * g;
          if (P.stage > 0) incr -= P.zet * gprev[f];
          x = x + P.dt * incr;
          if (f == 2 && bottom_wall) x = T(0);
          bstore<T>(x, rs, col, fs.oout[f] + lv);
          // tracers: final values, so their halo images too
          if (f >= 3 && P.images)
            store_with_images((T*)(fs.base + fs.oout[f]), d, gi, gj, k, x, false, false);
          if (P.stage < 2) bstore<T>(g, rs, col, fs.oG[f] + lv);
        } else {
          bstore<T>(g, rs, col, fs.oG[f] + lv);
        }
      }
    }

    // ---- advance: top fluxes become bottom fluxes, windows shift up
    fzb_u = fzt_u;
    fzb_v = fzt_v;
    fzb_w = fzt_w;
#pragma unroll
    for (int q = 0; q < NTR; ++q) fzb_c[q] = fzt_c[q];
    if (more) {
      if (IMM) {
        mkm = mk0;
        mk0 = mkp;
        mkp = nmk;
      }
#pragma unroll
      for (int o = 0; o < NW - 1; ++o) {
        wu[o] = wu[o + 1];
        wv[o] = wv[o + 1];
        ww[o] = ww[o + 1];
#pragma unroll
        for (int q = 0; q < NTR; ++q) wc[q][o] = wc[q][o + 1];
      }
      wu[NW - 1] = nu_;
      wv[NW - 1] = nv_;
      ww[NW - 1] = nw_;
#pragma unroll
      for (int q = 0; q < NTR; ++q) wc[q][NW - 1] = nc_[q];
      // the face velocities of level k + 1 (every reader of level k's passed
      // the barrier before the tendencies)
      if (edge) S[ering(k + R - 1)] = enext;
      face_velocities(k + 1);
    }
    // the copies of level k + 1 have landed (this wave's), and every wave is
    // done with the planes of level k
    wait_vm();
    __syncthreads();
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
// Tracer counts above MAXNTR are not instantiated (refused).
template <class T, int R, int WTX, int WTY, int MAXNTR = 4>
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
  FieldSet<T> fb = fs;
  if (!fieldset_offsets(fb, (uint64_t)padded_elems(d) * sizeof(T))) return hipErrorInvalidValue;
  bool clo = false;
  for (int f = 0; f < MAXF; ++f) clo = clo || fs.closure[f] != nullptr;
  const bool imm = fs.mask != nullptr;
  if (imm && (R != 3 || clo)) return hipErrorInvalidValue;
  if (p.ntr > MAXNTR) return hipErrorInvalidValue;
#define OC_TZ(SCH, NTR_, TX_, TY_)                                                            \
  if (imm) {                                                                                  \
    if constexpr (R == 3)                                                                     \
      hipLaunchKernelGGL((tz::tendency_zmarch<T, SCH, NTR_, TX_, TY_, R, false, true>), grid,  \
                         dim3(TX_ * TY_), 0, s, d, fb, p, nbx, nby, nbz, kc);                 \
  } else if (clo)                                                                             \
    hipLaunchKernelGGL((tz::tendency_zmarch<T, SCH, NTR_, TX_, TY_, R, true>), grid,           \
                       dim3(TX_ * TY_), 0, s, d, fb, p, nbx, nby, nbz, kc);                   \
  else                                                                                        \
    hipLaunchKernelGGL((tz::tendency_zmarch<T, SCH, NTR_, TX_, TY_, R, false>), grid,          \
                       dim3(TX_ * TY_), 0, s, d, fb, p, nbx, nby, nbz, kc)
#define OC_TZ_NTR(SCH, TX_, TY_)                                  \
  switch (p.ntr) {                                                \
    case 1: OC_TZ(SCH, 1, TX_, TY_); break;                       \
    case 2: if constexpr (MAXNTR >= 2) { OC_TZ(SCH, 2, TX_, TY_); } break; \
    case 3: if constexpr (MAXNTR >= 3) { OC_TZ(SCH, 3, TX_, TY_); } break; \
    default: if constexpr (MAXNTR >= 4) { OC_TZ(SCH, 4, TX_, TY_); } break; \
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
