// Internal state of a model (the opaque oc_model of the C ABI), shared by
// the translation units that orchestrate kernels on a model's buffers.
#pragma once

#include <vector>

#include "oc_internal.h"

namespace oc {

// RK3 coefficients (rk3 equation): gamma = (8/15, 5/12, 3/4),
// zeta = (0, 17/60, 5/12).
constexpr double RK_GAMMA[3] = {8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0};
constexpr double RK_ZETA[3] = {0.0, 17.0 / 60.0, 5.0 / 12.0};

// Offsets of the FP64 vertical tables in oc_model::zt64, and table lengths.
inline int zt_dzc(int)       { return 0; }
inline int zt_dzf(int nz)    { return nz; }
inline int zt_rdzc(int nz)   { return 2 * nz + 1; }
inline int zt_rdzf(int nz)   { return 3 * nz + 1; }
inline int zt_lo(int nz)     { return 4 * nz + 2; }
inline int zt_up(int nz)     { return 5 * nz + 2; }
inline int zt64_len(int nz)  { return 6 * nz + 2; }
inline int ztT_len(int nz)   { return 2 * nz + 3; }
inline int vfac_len(int nz)  { return 9 * vertical_factors_len(nz); }

}  // namespace oc

using namespace oc;

struct oc_grid {
  oc_grid_desc d;
  std::vector<double> zf;   // stretched z: the nz + 1 faces (empty: uniform)
};

struct oc_model {
  oc_grid_desc gd;
  oc_model_desc md;
  Dims dims;
  int nf;
  int esz;
  int kinds[MAXF];
  char* ws;
  uint64_t ws_bytes;
  void* state[2][MAXF];
  void* G[MAXF];
  int cur;
  SpecBufs sb;
  double offset[MAXF];  // storage offset per field: stored = value - offset
  void* staging;
  double* diag_part;
  double dx, dy, dz;      // dz: lz / nz (the mean thickness on a stretched grid)
  int kind;              // OC_NONHYDROSTATIC or OC_HYDROSTATIC
  // vertical grid tables (device, in the workspace).  zt64 (FP64): dzc[nz],
  // dzf[nz+1], rdzc[nz], rdzf[nz+1], the pressure operator's off-diagonals
  // lo[nz], up[nz].  ztT (state precision): rdzc for k = -1..nz, then rdzf.
  // vfac: implicit-diffusion tables [stage][u/v, w, tracer] of
  // vertical_factors_len(nz) values (state precision) for the step vfac_dt.
  int stretched;
  double dzmin;          // thinnest cell
  std::vector<double> hdzc, hdzf;   // host copies of dzc, dzf
  double* zt64;
  void* ztT;
  void* vfac;
  double vfac_dt;
  std::vector<char> vfac_host;
  // hydrostatic model: 2D barotropic state (FP64), ping-pong (eta, U, V)
  double* eta[2];
  double* ubt[2];
  double* vbt[2];
  double* gubt;
  double* gvbt;
  double* gub1;   // partial column sums of the upper levels (two-chunk tendency)
  double* gvb1;
  double* etab;
  double* ubar;
  double* vbar;
  double* metric;        // len_u | dx_u | len_v | dy_v | area
  int bcur;
  // hydrostatic baroclinic step: diagnostic fields (state precision,
  // padded), row tables, surface stress, and the QAB2 / refresh flags
  void* hzeta;
  void* hpx;
  void* hpy;
  double* hmet;
  double* taux;
  double* tauy;
  int hfirst;            // the next step is a first (Euler) step
  int hstale;            // halos and diagnostic fields need a refresh
  // learned closure: network, statistics, tendency buffers (u, v, w, T)
  oc_mlp* net;
  ClosureStats cst;
  void* gc[MAXF];
  // LES closure: viscosity at the centres, AMD's per-tracer diffusivities
  // (padded, state precision) and the (C_s Delta_k)^2 table
  void* les_nu;
  void* les_kap[OC_MAX_TRACERS];
  void* les_d2;
  // immersed boundary: the padded mask (state precision, 1 = fluid), the
  // conjugate-gradient vectors and scalars, pinned host copy of the scalars,
  // the number of fluid cells and the last solve's statistics
  void* mask;
  uint8_t* ibits;        // per-cell geometry bytes (IB_*), dense
  CgBufs cg;
  double* cg_host;
  double nfluid;
  int cg_iterations;
  double cg_residual;
  // per-kernel-class event timing
  int prof_on;
  uint32_t prof_mask;         // classes that record events (bit OC_PROF_*)
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used;
  std::vector<int> prof_cls;  // class of each recorded (start, stop) pair
  // whole RK3 steps captured as HIP graphs, one per starting buffer parity,
  // for the time step gdt[p] (the kernels take both as arguments); gcap is
  // the capture stream, which never runs work
  hipStream_t gcap = nullptr;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  double gdt[2] = {0.0, 0.0};
  // the last solve's p is still only in sb.spec (the fused inverse x pass
  // and projection does not write it); oc_get_pressure transforms it first
  bool p_pending = false;
};

namespace oc {

// Physics of the tendency kernel of a nonhydrostatic model (the substage
// fields dt, gam, zet, stage, combine, images are left zero).
template <class T>
inline TendParams<T> tend_params(const oc_model* m) {
  TendParams<T> p;
  const oc_model_desc& d = m->md;
  p.rdx = (T)(1.0 / m->dx);
  p.rdy = (T)(1.0 / m->dy);
  p.rdzc = (const T*)m->ztT + 1;
  p.rdzf = (const T*)m->ztT + (m->dims.nz + 2);
  p.nu = (T)d.nu;
  p.kappa = (T)d.kappa;
  p.nuz = d.implicit_z ? T(0) : (T)d.nu;
  p.kappaz = d.implicit_z ? T(0) : (T)d.kappa;
  p.f = (T)d.f;
  p.g_alpha = (T)(d.g * d.alpha);
  p.g_beta = (T)(d.g * d.beta);
  // FP32 storage keeps T and S as anomalies about (t_ref, s_ref)
  p.t_ref = (T)(d.t_ref - m->offset[OC_TRACER0]);
  p.s_ref = (T)(d.s_ref - m->offset[OC_TRACER0 + 1]);
  p.buoyancy = d.buoyancy ? 1 : 0;
  p.ntr = d.ntracers;
  for (int q = 0; q < OC_MAX_TRACERS; ++q) {
    p.top_flux[q] = (T)(m->dims.zb ? d.top_flux[q] : 0.0);
    p.toff[q] = (T)((OC_TRACER0 + q < m->nf) ? m->offset[OC_TRACER0 + q] : 0.0);
  }
  p.eps = (T)d.weno_eps;
  p.dt = 0;
  p.gam = 0;
  p.zet = 0;
  p.stage = 0;
  p.combine = 0;
  p.images = 0;
  return p;
}

}  // namespace oc
