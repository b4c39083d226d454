// Fused tendency + RK3 kernel of the nonhydrostatic model on gfx950.
//
// Method (finite-volume appendix of arXiv 2502.14148): conservative flux
// divergence of advective + diffusive fluxes for tracers; flux-form momentum
// advection with a centred fourth-order advecting velocity and a WENO5-Z
// reconstruction of the advected component; f-plane Coriolis (four-point
// averages); buoyancy b = g(alpha(T-T0) - beta(S-S0)) averaged to w faces;
// RK3 substage X~ = X + dt(gamma G^m - zeta G^{m-1}) (rk3 equation).
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
//   * z fluxes per column from a 7-level register window (the flux through
//     the top face of level k is the bottom flux of level k+1);
//   * x and y fluxes from LDS planes (tile + 3-cell halo) of the current
//     level; the (TX+1)TY x-faces and TX(TY+1) y-faces are dealt out to the
//     threads as "slots" whose strides are per-lane values, so x and y faces
//     run the same instruction stream with no divergence;
//   * the advecting velocities of the w fluxes need u, v on the four levels
//     k-2..k+1, kept as LDS rings.
// Tiles are mapped XCD-major so that neighbouring tiles (which share halo
// loads) land on the same XCD and its L2.
#include "oc_internal.h"
#include "weno_dev.h"

// Column tile of the tendency kernel (x by y); 8 x 8 tiles serve grids whose
// sizes the wide tile does not divide.
#ifndef OC_TEND_TX
#define OC_TEND_TX 32
#endif
#ifndef OC_TEND_TY
#define OC_TEND_TY 8
#endif
#ifndef OC_TEND_FLUXBAR
#define OC_TEND_FLUXBAR 0
#endif
#ifndef OC_TEND_KC_DIV
#define OC_TEND_KC_DIV 1024
#endif

namespace oc {

namespace tz {

// advective flux vel * W(q) with q read from LDS at q[L + o*s], o = -3..2
template <class T, int SCHEME>
__device__ inline T flux_lds(const T* q, int L, int s, T vel, T eps) {
  if (SCHEME == SCHEME_NONE) return T(0);
  return vel * rec6<T, SCHEME>(q[L - 3 * s], q[L - 2 * s], q[L - s], q[L], q[L + s], q[L + 2 * s],
                               vel, eps);
}

// advective flux from a register window w[o0 .. o0+5]
template <class T, int SCHEME>
__device__ inline T flux_reg(const T* w, T vel, T eps) {
  if (SCHEME == SCHEME_NONE) return T(0);
  return vel * rec6<T, SCHEME>(w[0], w[1], w[2], w[3], w[4], w[5], vel, eps);
}

// Fluxes of one x or y face slot at LDS position L.  All LDS planes are
// offsets into one shared array S (so every access stays an LDS access).
// sd/se are the strides along and across the flux direction (compile-time
// constants in the main rounds, per lane in the edge round).
struct SlotOff {
  int vd, ve;             // normal and tangential velocity planes (level k)
  int r0, r1, r2, r3;     // normal velocity at levels k-2, k-1, k, k+1
  int wk;                 // w plane (level k)
  int c0;                 // first tracer plane (level k); tracers are PL apart
  int Fself, Fcross, Fw;  // flux arrays (already for this direction)
  int Fc0, Fstride;       // first tracer flux array and the array pitch
};

template <class T, int SCHEME, int NTR, int PL>
__device__ inline void slot_fluxes(T* S, const SlotOff& o, int L, int sd, int se, int fi, T rd,
                                   T nu, T kappa, T eps) {
  {
    const T* vd = S + o.vd;
    const T adv = interp4(vd[L - 2 * sd], vd[L - sd], vd[L], vd[L + sd]);
    S[o.Fself + fi] = flux_lds<T, SCHEME>(vd, L, sd, adv, eps) - nu * (vd[L] - vd[L - sd]) * rd;
  }
#if OC_TEND_FLUXBAR
  __builtin_amdgcn_sched_barrier(0);
#endif
  {
    const T* vd = S + o.vd;
    const T* ve = S + o.ve;
    const T adv = interp4(vd[L - 2 * se], vd[L - se], vd[L], vd[L + se]);
    S[o.Fcross + fi] = flux_lds<T, SCHEME>(ve, L, sd, adv, eps) - nu * (ve[L] - ve[L - sd]) * rd;
  }
#if OC_TEND_FLUXBAR
  __builtin_amdgcn_sched_barrier(0);
#endif
  {
    const T adv = interp4(S[o.r0 + L], S[o.r1 + L], S[o.r2 + L], S[o.r3 + L]);
    const T* wk = S + o.wk;
    S[o.Fw + fi] = flux_lds<T, SCHEME>(wk, L, sd, adv, eps) - nu * (wk[L] - wk[L - sd]) * rd;
  }
  const T un = S[o.vd + L];
#pragma unroll
  for (int q = 0; q < NTR; ++q) {
#if OC_TEND_FLUXBAR
    __builtin_amdgcn_sched_barrier(0);
#endif
    const T* c = S + o.c0 + q * PL;
    S[o.Fc0 + q * o.Fstride + fi] =
        flux_lds<T, SCHEME>(c, L, sd, un, eps) - kappa * (c[L] - c[L - sd]) * rd;
  }
}

#ifndef OC_TEND_WAVES
#define OC_TEND_WAVES 4
#endif

// One column tile: tile b of an nbx x nby x nbz decomposition (k chunks of
// kc levels) of the grid d.
// CLO: add the closure tendencies computed beforehand (fs.closure; learned
// closure: u, v, w and tracer 0, LES closure: every field).  A separate
// instantiation keeps the plain kernel's registers free of them.
template <class T, int SCHEME, int NTR, int TX, int TY, bool CLO = false>
__device__ __attribute__((always_inline)) inline void tendency_tile(
    const Dims& d, const FieldSet<T>& fs, const TendParams<T>& P, int nbx, int nby, int nbz,
    int kc, int b) {
  constexpr int NT = TX * TY;
  constexpr int PX = TX + 6, PY = TY + 6, PL = PX * PY;
  constexpr int NXS = (TX + 1) * TY, NYS = TX * (TY + 1);
  constexpr int NF = 3 + NTR;
  constexpr int NFILL = (PL + NT - 1) / NT;
  // LDS map: u ring (4 planes), v ring (4), w ring (2), tracers (NTR),
  // x-face fluxes (NF arrays of NXS), y-face fluxes (NF arrays of NYS)
  constexpr int OU = 0, OV = 4 * PL, OW = 8 * PL, OC = 10 * PL;
  constexpr int OFX = (10 + NTR) * PL, OFY = OFX + NF * NXS;
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
  const int Lc = (ty + 3) * PX + (tx + 3);  // own position in an LDS plane
  const T eps = P.eps;
  const long sz = d.sz;
  const int sy = (int)d.sy;

  // 32-bit offsets of the plane elements this thread loads, relative to the
  // tile corner (i0-3, j0-3) of a level; the same for every level
  int goff[NFILL];
#pragma unroll
  for (int r = 0; r < NFILL; ++r) {
    const int e = tid + r * NT;
    const int ly = e / PX, lx = e - ly * PX;
    goff[r] = ly * sy + lx;
  }
  const long corner = (long)(j0 - 3 + H) * sy + (i0 - 3 + H);
  auto fill = [&](int dst, const T* __restrict__ src, int kk) {
    const T* __restrict__ base = src + (long)(kk + H) * sz + corner;
#pragma unroll
    for (int r = 0; r < NFILL; ++r) {
      const int e = tid + r * NT;
      if (PL % NT == 0 || e < PL) S[dst + e] = base[goff[r]];
    }
  };
  auto ru = [](int kk) { return OU + (kk & 3) * PL; };
  auto rv = [](int kk) { return OV + (kk & 3) * PL; };
  auto rw = [](int kk) { return OW + (kk & 1) * PL; };

  const T* __restrict__ gu = fs.in[0];
  const T* __restrict__ gv = fs.in[1];
  const T* __restrict__ gw = fs.in[2];

  // ---- register windows: levels k-2..k+3 of the own column (index o is
  // level k-2+o)
  const int col = (gj + H) * sy + (gi + H);   // offset within a level
  T wu[6], wv[6], ww[6], wc[NTR][6];
#pragma unroll
  for (int o = 0; o < 6; ++o) {
    const long lv = (long)(kb - 2 + o + H) * sz;
    wu[o] = (gu + lv)[col];
    wv[o] = (gv + lv)[col];
    ww[o] = (gw + lv)[col];
#pragma unroll
    for (int q = 0; q < NTR; ++q) wc[q][o] = (fs.in[3 + q] + lv)[col];
  }

  // ---- prologue: rings for levels kb-2..kb (u, v) and kb (w)
  fill(ru(kb - 2), gu, kb - 2);
  fill(ru(kb - 1), gu, kb - 1);
  fill(ru(kb), gu, kb);
  fill(rv(kb - 2), gv, kb - 2);
  fill(rv(kb - 1), gv, kb - 1);
  fill(rv(kb), gv, kb);
  fill(rw(kb), gw, kb);
  __syncthreads();

  // bottom z fluxes of the first level (face kb; w: centre kb-1), from the
  // levels kb-3..kb+2
  T fzb_u, fzb_v, fzb_w, fzb_c[NTR];
  {
    const long lv = (long)(kb - 3 + H) * sz;
    const T* wp = S + rw(kb);
    const bool wall = d.zb && kb == 0;
    T z[6];
    const T wt_u = interp4(wp[Lc - 2], wp[Lc - 1], wp[Lc], wp[Lc + 1]);
    const T wt_v = interp4(wp[Lc - 2 * PX], wp[Lc - PX], wp[Lc], wp[Lc + PX]);
    z[0] = (gu + lv)[col];
#pragma unroll
    for (int o = 1; o < 6; ++o) z[o] = wu[o - 1];
    const T rzb = P.rdzf[kb];  // face kb
    fzb_u = wall ? T(0) : flux_reg<T, SCHEME>(z, wt_u, eps) - P.nuz * (z[3] - z[2]) * rzb;
    z[0] = (gv + lv)[col];
#pragma unroll
    for (int o = 1; o < 6; ++o) z[o] = wv[o - 1];
    fzb_v = wall ? T(0) : flux_reg<T, SCHEME>(z, wt_v, eps) - P.nuz * (z[3] - z[2]) * rzb;
    z[0] = (gw + lv)[col];
#pragma unroll
    for (int o = 1; o < 6; ++o) z[o] = ww[o - 1];
    const T wb = interp4(z[1], z[2], z[3], z[4]);
    fzb_w = flux_reg<T, SCHEME>(z, wb, eps) - P.nuz * (z[3] - z[2]) * P.rdzc[kb - 1];
    const T wface = z[3];
#pragma unroll
    for (int q = 0; q < NTR; ++q) {
      z[0] = (fs.in[3 + q] + lv)[col];
#pragma unroll
      for (int o = 1; o < 6; ++o) z[o] = wc[q][o - 1];
      fzb_c[q] = wall ? T(0)
                      : flux_reg<T, SCHEME>(z, wface, eps) - P.kappaz * (z[3] - z[2]) * rzb;
    }
  }

  for (int k = kb; k < ke; ++k) {
    __syncthreads();  // consumers of the previous level are done
    fill(ru(k + 1), gu, k + 1);
    fill(rv(k + 1), gv, k + 1);
    fill(rw(k + 1), gw, k + 1);
#pragma unroll
    for (int q = 0; q < NTR; ++q) fill(OC + q * PL, fs.in[3 + q], k);
    __syncthreads();

    // ---- x and y face fluxes
    SlotOff ox, oy;
    ox.vd = ru(k); ox.ve = rv(k);
    ox.r0 = ru(k - 2); ox.r1 = ru(k - 1); ox.r2 = ru(k); ox.r3 = ru(k + 1);
    ox.wk = rw(k); ox.c0 = OC;
    ox.Fself = OFX + 0 * NXS; ox.Fcross = OFX + 1 * NXS; ox.Fw = OFX + 2 * NXS;
    ox.Fc0 = OFX + 3 * NXS; ox.Fstride = NXS;
    oy.vd = rv(k); oy.ve = ru(k);
    oy.r0 = rv(k - 2); oy.r1 = rv(k - 1); oy.r2 = rv(k); oy.r3 = rv(k + 1);
    oy.wk = rw(k); oy.c0 = OC;
    oy.Fself = OFY + 1 * NYS; oy.Fcross = OFY + 0 * NYS; oy.Fw = OFY + 2 * NYS;
    oy.Fc0 = OFY + 3 * NYS; oy.Fstride = NYS;
    // main rounds: the left x face and the bottom y face of the own cell
    slot_fluxes<T, SCHEME, NTR, PL>(S, ox, Lc, 1, PX, ty * (TX + 1) + tx, P.rdx, P.nu, P.kappa, eps);
    __builtin_amdgcn_sched_barrier(0);
    slot_fluxes<T, SCHEME, NTR, PL>(S, oy, Lc, PX, 1, ty * TX + tx, P.rdy, P.nu, P.kappa, eps);
    __builtin_amdgcn_sched_barrier(0);
    // edge round: right x faces of the last column, top y faces of the last row
    if (tid < TY + TX) {
      const bool xs = tid < TY;
      const int L = xs ? (tid + 3) * PX + (TX + 3) : (TY + 3) * PX + (tid - TY + 3);
      const int fi = xs ? tid * (TX + 1) + TX : TY * TX + (tid - TY);
      SlotOff oe;
      oe.vd = xs ? ox.vd : oy.vd; oe.ve = xs ? ox.ve : oy.ve;
      oe.r0 = xs ? ox.r0 : oy.r0; oe.r1 = xs ? ox.r1 : oy.r1;
      oe.r2 = xs ? ox.r2 : oy.r2; oe.r3 = xs ? ox.r3 : oy.r3;
      oe.wk = ox.wk; oe.c0 = OC;
      oe.Fself = xs ? ox.Fself : oy.Fself; oe.Fcross = xs ? ox.Fcross : oy.Fcross;
      oe.Fw = xs ? ox.Fw : oy.Fw; oe.Fc0 = xs ? ox.Fc0 : oy.Fc0;
      oe.Fstride = xs ? NXS : NYS;
      slot_fluxes<T, SCHEME, NTR, PL>(S, oe, L, xs ? 1 : PX, xs ? PX : 1, fi, xs ? P.rdx : P.rdy,
                                      P.nu, P.kappa, eps);
    }

    // ---- z fluxes through the top face of level k (w: at centre k)
    const bool top_wall = d.zb && (k + 1 == d.nz);
    // inverse spacings of this level (uniform across the workgroup): the top
    // face k+1, the cell k, and face k (the thickness of the w cell)
    const T rzft = P.rdzf[k + 1], rzc = P.rdzc[k], rzf = P.rdzf[k];
    T fzt_u, fzt_v, fzt_w, fzt_c[NTR];
    {
      const T* wp = S + rw(k + 1);
      const T wt_u = interp4(wp[Lc - 2], wp[Lc - 1], wp[Lc], wp[Lc + 1]);
      const T wt_v = interp4(wp[Lc - 2 * PX], wp[Lc - PX], wp[Lc], wp[Lc + PX]);
      fzt_u = top_wall ? T(0) : flux_reg<T, SCHEME>(wu, wt_u, eps) - P.nuz * (wu[3] - wu[2]) * rzft;
      fzt_v = top_wall ? T(0) : flux_reg<T, SCHEME>(wv, wt_v, eps) - P.nuz * (wv[3] - wv[2]) * rzft;
      const T wb = interp4(ww[1], ww[2], ww[3], ww[4]);
      fzt_w = flux_reg<T, SCHEME>(ww, wb, eps) - P.nuz * (ww[3] - ww[2]) * rzc;
#pragma unroll
      for (int q = 0; q < NTR; ++q)
        fzt_c[q] = top_wall ? P.top_flux[q]
                            : flux_reg<T, SCHEME>(wc[q], ww[3], eps) -
                                  P.kappaz * (wc[q][3] - wc[q][2]) * rzft;
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
      const T* uk = S + ru(k);
      const T* vk = S + rv(k);
      G[0] += -(fzt_u - fzb_u) * rzc +
              P.f * T(0.25) * (vk[Lc - 1] + vk[Lc] + vk[Lc - 1 + PX] + vk[Lc + PX]);
      G[1] += -(fzt_v - fzb_v) * rzc -
              P.f * T(0.25) * (uk[Lc - PX] + uk[Lc + 1 - PX] + uk[Lc] + uk[Lc + 1]);
      G[2] += -(fzt_w - fzb_w) * rzf;
      if (NTR >= 2 && P.buoyancy) {
        const T bl = P.g_alpha * (wc[0][1] - P.t_ref) - P.g_beta * (wc[1][1] - P.s_ref);
        const T bu = P.g_alpha * (wc[0][2] - P.t_ref) - P.g_beta * (wc[1][2] - P.s_ref);
        G[2] += T(0.5) * (bl + bu);
      }
      const bool bottom_wall = d.zb && k == 0;
      if (bottom_wall) G[2] = T(0);
      const T divu = (uk[Lc + 1] - uk[Lc]) * P.rdx + (vk[Lc + PX] - vk[Lc]) * P.rdy +
                     (ww[3] - ww[2]) * rzc;
#pragma unroll
      for (int q = 0; q < NTR; ++q) G[3 + q] += -(fzt_c[q] - fzb_c[q]) * rzc - P.toff[q] * divu;

      const long lv = (long)(k + H) * sz;
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        // plus the closure tendency computed beforehand
        const T g = (CLO && fs.closure[f]) ? G[f] + (fs.closure[f] + lv)[col] : G[f];
        T* __restrict__ Gf = fs.G[f] + lv;
        if (P.combine) {
          T x;
          if (f == 0) x = wu[2];
          else if (f == 1) x = wv[2];
          else if (f == 2) x = ww[2];
          else x = wc[f - 3][2];
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
    if (k + 1 < ke) {
      const long lv = (long)(k + 4 + H) * sz;
#pragma unroll
      for (int o = 0; o < 5; ++o) {
        wu[o] = wu[o + 1];
        wv[o] = wv[o + 1];
        ww[o] = ww[o + 1];
#pragma unroll
        for (int q = 0; q < NTR; ++q) wc[q][o] = wc[q][o + 1];
      }
      wu[5] = (gu + lv)[col];
      wv[5] = (gv + lv)[col];
      ww[5] = (gw + lv)[col];
#pragma unroll
      for (int q = 0; q < NTR; ++q) wc[q][5] = (fs.in[3 + q] + lv)[col];
    }
  }
}

#define OC_TEND_ATTRS(T, TX, TY)   \
  __launch_bounds__(TX * TY)      \
  __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? OC_TEND_WAVES : 2)))

// One model; tiles are mapped XCD-major, so neighbouring tiles (which share
// halo loads) land on the same XCD and its L2.
template <class T, int SCHEME, int NTR, int TX, int TY, bool CLO>
__global__ void OC_TEND_ATTRS(T, TX, TY)
tendency_zmarch(Dims d, FieldSet<T> fs, TendParams<T> P, int nbx, int nby, int nbz, int kc) {
  const int nblk = nbx * nby * nbz;
  int b = blockIdx.x;
  if ((nblk & 7) == 0) b = (b & 7) * (nblk >> 3) + (b >> 3);
  tendency_tile<T, SCHEME, NTR, TX, TY, CLO>(d, fs, P, nbx, nby, nbz, kc, b);
}

// An ensemble of models in one launch.  Work items (member, tile) come from
// `items`; PERSIST = false: one workgroup per item; PERSIST = true: a grid of
// resident workgroups takes items from the atomic counter until the list is
// exhausted (every workgroup leaves the loop once the counter passes nitems).
template <class T, int SCHEME, int NTR, int TX, int TY, bool PERSIST>
__global__ void OC_TEND_ATTRS(T, TX, TY)
tendency_ensemble(const EnsMember<T>* __restrict__ mem, const int2* __restrict__ items,
                  int nitems, int* __restrict__ counter, int parity, int stage) {
  if (!PERSIST) {
    const int2 it = items[blockIdx.x];
    const EnsMember<T>& M = mem[it.x];
    tendency_tile<T, SCHEME, NTR, TX, TY>(M.d, M.fs[parity], M.P[stage], M.nbx, M.nby, M.nbz,
                                          M.kc, it.y);
    return;
  }
  __shared__ int s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(s_item);
    if (item >= nitems) break;
    const int2 it = items[item];
    const EnsMember<T>& M = mem[it.x];
    tendency_tile<T, SCHEME, NTR, TX, TY>(M.d, M.fs[parity], M.P[stage], M.nbx, M.nby, M.nbz,
                                          M.kc, it.y);
    __syncthreads();  // LDS and s_item are reused by the next item
  }
}

__global__ void reset_counter_kernel(int* counter) { counter[0] = 0; }

}  // namespace tz

template <class T>
hipError_t launch_tendency_fast(const Dims& d, const FieldSet<T>& fs, const TendParams<T>& p,
                                int scheme, hipStream_t s) {
  constexpr int WTX = OC_TEND_TX, WTY = OC_TEND_TY;
  const bool wide = (d.nx % WTX == 0) && (d.ny % WTY == 0);
  const int TX = wide ? WTX : 8, TY = wide ? WTY : 8;
  if (d.nx % TX || d.ny % TY) return hipErrorInvalidValue;
  const int nbx = d.nx / TX, nby = d.ny / TY;
  int kc = (int)((long)d.nz * nbx * nby / OC_TEND_KC_DIV);
  kc = kc < 4 ? 4 : (kc > 64 ? 64 : kc);
  if (kc > d.nz) kc = d.nz;
  const int nbz = (d.nz + kc - 1) / kc;
  const dim3 grid(nbx * nby * nbz);
  bool clo = false;
  for (int f = 0; f < MAXF; ++f) clo = clo || fs.closure[f] != nullptr;
#define OC_TZ(SCH, NTR_, TX_, TY_)                                                            \
  if (clo)                                                                                    \
    hipLaunchKernelGGL((tz::tendency_zmarch<T, SCH, NTR_, TX_, TY_, true>), grid,              \
                       dim3(TX_ * TY_), 0, s, d, fs, p, nbx, nby, nbz, kc);                   \
  else                                                                                        \
    hipLaunchKernelGGL((tz::tendency_zmarch<T, SCH, NTR_, TX_, TY_, false>), grid,             \
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
    case tz::SCHEME_NONE: OC_TZ_TX(tz::SCHEME_NONE); break;
    case tz::SCHEME_WENOZ: OC_TZ_TX(tz::SCHEME_WENOZ); break;
    default: OC_TZ_TX(tz::SCHEME_LINEAR); break;
  }
#undef OC_TZ_TX
#undef OC_TZ_NTR
#undef OC_TZ
  return hipGetLastError();
}

template <class T>
hipError_t launch_tendency_ensemble(const EnsMember<T>* mem, const int2* items, int nitems,
                                   int* counter, int parity, int stage, const EnsTuning& tn,
                                   hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  if (tn.persistent) hipLaunchKernelGGL(tz::reset_counter_kernel, dim3(1), dim3(1), 0, s, counter);
  const int nblk = tn.persistent ? tn.nblocks : nitems;
#define OC_TE(TX_, TY_, P_)                                                                  \
  hipLaunchKernelGGL((tz::tendency_ensemble<T, tz::SCHEME_WENOZ, 2, TX_, TY_, P_>),          \
                     dim3(nblk), dim3(TX_ * TY_), 0, s, mem, items, nitems, counter, parity, \
                     stage)
#define OC_TE_P(TX_, TY_) \
  if (tn.persistent) { OC_TE(TX_, TY_, true); } else { OC_TE(TX_, TY_, false); }
  switch (tn.tile) {
    case 0: OC_TE_P(32, 8); break;
    case 1: OC_TE_P(16, 8); break;
    default: OC_TE_P(8, 8); break;
  }
#undef OC_TE_P
#undef OC_TE
  return hipGetLastError();
}

// Resident workgroups per CU of the persistent ensemble kernel of a tile
// shape (from the kernel's registers and LDS).
template <class T>
int ensemble_blocks_per_cu(int tile) {
  int n = 0;
  hipError_t e;
  switch (tile) {
    case 0:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &n, tz::tendency_ensemble<T, tz::SCHEME_WENOZ, 2, 32, 8, true>, 256, 0);
      break;
    case 1:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &n, tz::tendency_ensemble<T, tz::SCHEME_WENOZ, 2, 16, 8, true>, 128, 0);
      break;
    default:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &n, tz::tendency_ensemble<T, tz::SCHEME_WENOZ, 2, 8, 8, true>, 64, 0);
  }
  return (e == hipSuccess && n > 0) ? n : 1;
}
template int ensemble_blocks_per_cu<float>(int);
template int ensemble_blocks_per_cu<double>(int);

template hipError_t launch_tendency_ensemble<float>(const EnsMember<float>*, const int2*, int,
                                                    int*, int, int, const EnsTuning&,
                                                    hipStream_t);
template hipError_t launch_tendency_ensemble<double>(const EnsMember<double>*, const int2*, int,
                                                     int*, int, int, const EnsTuning&,
                                                     hipStream_t);

template hipError_t launch_tendency_fast<float>(const Dims&, const FieldSet<float>&,
                                                const TendParams<float>&, int, hipStream_t);
template hipError_t launch_tendency_fast<double>(const Dims&, const FieldSet<double>&,
                                                 const TendParams<double>&, int, hipStream_t);

}  // namespace oc
