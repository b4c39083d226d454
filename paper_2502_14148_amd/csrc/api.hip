// C ABI of liboc (declared in include/oc.h): argument validation, workspace
// carving, FFT tables, and the orchestration of the RK3 / pressure-correction
// step on a caller-provided HIP stream.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "model.h"

namespace oc {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

static const int DIAG_BLOCKS = 1024;
static const int DIAG_PARTS = 12;

}  // namespace oc

using namespace oc;


namespace {

#define OC_CHECK_HIP(expr)                                                       \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess) {                                                      \
      set_error("%s failed: %s", #expr, hipGetErrorString(e_));                  \
      return OC_ERR_DEVICE;                                                      \
    }                                                                            \
  } while (0)

struct Layout {
  uint64_t state[2][MAXF], G[MAXF];
  uint64_t spec, p, twx, twy, twz, dctz, lamx, lamy, lamz, staging, diag;
  uint64_t baro[15], metric, hzeta, hpx, hpy, hmet;
  uint64_t gc[MAXF];
  uint64_t les_nu, les_kap[OC_MAX_TRACERS], les_d2;
  uint64_t mask, ibits, cg_x, cg_r, cg_q, cg_aq, cg_part, cg_scal;
  uint64_t zt64, ztT, vfac;
  uint64_t total;
};

uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

Layout make_layout(const oc_grid_desc& g, const oc_model_desc& m) {
  Layout L;
  std::memset(&L, 0, sizeof(L));
  Dims d = make_dims(g.nx, g.ny, g.nz, g.topology_z == OC_BOUNDED, halo_width(m.advection));
  const int nf = 3 + m.ntracers;
  const uint64_t esz = (m.precision == OC_FP64) ? 8 : 4;
  const uint64_t fb = align256((uint64_t)padded_elems(d) * esz);
  uint64_t off = 0;
  for (int s = 0; s < 2; ++s)
    for (int q = 0; q < MAXF; ++q) {
      L.state[s][q] = off;
      if (q < nf) off += fb;
    }
  for (int q = 0; q < MAXF; ++q) {
    L.G[q] = off;
    if (q < nf) off += fb;
  }
  if (m.kind == OC_NONHYDROSTATIC) {
    L.spec = off; off += align256((uint64_t)g.nz * g.ny * spec_pitch(g.nx) * 16);
    L.p = off; off += align256((uint64_t)g.nz * g.ny * g.nx * 8);
    L.twx = off; off += align256((uint64_t)g.nx * 16);
    L.twy = off; off += align256((uint64_t)g.ny * 16);
    L.twz = off; off += align256((uint64_t)g.nz * 16);
    L.dctz = off; off += align256((uint64_t)g.nz * 16);
    L.lamx = off; off += align256((uint64_t)g.nx * 8);
    L.lamy = off; off += align256((uint64_t)g.ny * 8);
    L.lamz = off; off += align256((uint64_t)g.nz * 8);
  } else {
    // eta[2], U[2], V[2], GU, GV, etabar, Ubar, Vbar, tau_x, tau_y, and the
    // upper levels' partial column sums of GU, GV (V-like: ny + 1 rows)
    const uint64_t a2 = align256((uint64_t)(g.ny + 1) * g.nx * 8);
    for (int q = 0; q < 15; ++q) { L.baro[q] = off; off += a2; }
    L.metric = off; off += align256((uint64_t)(5 * (g.ny + 1)) * 8);
    L.hzeta = off; off += fb;
    L.hpx = off; off += fb;
    L.hpy = off; off += fb;
    L.hmet = off; off += align256((uint64_t)HYDRO_NMET * (g.ny + 2 * d.h + 1) * 8);
  }
  // closure tendencies: u, v, w, T for the learned closure, every field for LES
  const int ngc = m.closure ? 4 : (m.les ? nf : 0);
  for (int q = 0; q < ngc; ++q) { L.gc[q] = off; off += fb; }
  if (m.les) {
    L.les_nu = off; off += fb;
    if (m.les == OC_LES_AMD)
      for (int q = 0; q < m.ntracers; ++q) { L.les_kap[q] = off; off += fb; }
    L.les_d2 = off; off += align256((uint64_t)g.nz * esz);
  }
  if (m.immersed) {
    const uint64_t nv = align256((uint64_t)g.nx * g.ny * g.nz * 8);
    L.mask = off; off += fb;
    L.ibits = off; off += align256((uint64_t)g.nx * g.ny * g.nz);
    L.cg_x = off; off += nv;
    L.cg_r = off; off += nv;
    L.cg_q = off; off += nv;
    L.cg_aq = off; off += nv;
    L.cg_part = off; off += align256((uint64_t)IB_PART_CAP * 8);
    L.cg_scal = off; off += align256((uint64_t)CG_NSCAL * 8);
  }
  L.zt64 = off; off += align256((uint64_t)zt64_len(g.nz) * 8);
  L.ztT = off; off += align256((uint64_t)ztT_len(g.nz) * esz);
  L.vfac = off; off += align256((uint64_t)vfac_len(g.nz) * esz);
  L.staging = off; off += align256((uint64_t)(g.nz + 1) * (g.ny + 1) * g.nx * 8);
  L.diag = off; off += align256((uint64_t)DIAG_BLOCKS * DIAG_PARTS * 8);
  L.total = off;
  return L;
}

int validate_grid(const oc_grid_desc* d) {
  if (!d) { set_error("grid descriptor is NULL"); return OC_ERR_ARG; }
  if (d->topology_z != OC_PERIODIC && d->topology_z != OC_BOUNDED) {
    set_error("topology_z must be OC_PERIODIC or OC_BOUNDED");
    return OC_ERR_ARG;
  }
  if (!(d->lx > 0) || !(d->ly > 0) || !(d->lz > 0) || !std::isfinite(d->lx) ||
      !std::isfinite(d->ly) || !std::isfinite(d->lz)) {
    set_error("domain extents must be positive and finite");
    return OC_ERR_ARG;
  }
  if (d->z_faces && d->coord != OC_RECTILINEAR) {
    set_error("z_faces are supported on rectilinear grids only");
    return OC_ERR_UNSUPPORTED;
  }
  if (d->z_faces) {
    if (d->topology_z != OC_BOUNDED || d->nz < 8 || d->nz > 256) {
      set_error("a stretched z needs topology_z = OC_BOUNDED and 8 <= nz <= 256");
      return OC_ERR_UNSUPPORTED;
    }
    const double tol = 1e-9 * d->lz;
    for (int k = 0; k <= d->nz; ++k)
      if (!std::isfinite(d->z_faces[k]) || (k > 0 && !(d->z_faces[k] > d->z_faces[k - 1]))) {
        set_error("z_faces must be finite and strictly increasing (face %d)", k);
        return OC_ERR_ARG;
      }
    if (std::fabs(d->z_faces[0] - d->z0) > tol || std::fabs(d->z_faces[d->nz] - (d->z0 + d->lz)) > tol) {
      set_error("z_faces must run from z0 to z0 + lz");
      return OC_ERR_ARG;
    }
  }
  if (d->coord == OC_RECTILINEAR) {
    if (!fft_length_supported(d->nx) || !fft_length_supported(d->ny) ||
        (!d->z_faces && !fft_length_supported(d->nz))) {
      set_error("unsupported grid size %d x %d x %d (each of 8,16,32,64,96,128,256; a "
                "stretched z any 8..256)", d->nx, d->ny, d->nz);
      return OC_ERR_UNSUPPORTED;
    }
    if (d->ny % 2) { set_error("ny must be even"); return OC_ERR_UNSUPPORTED; }
  } else if (d->coord == OC_LATLON) {
    if (d->nx < 8 || d->ny < 8 || d->nz < 8 || d->nx % 8 || d->ny % 8) {
      set_error("lat-lon grids need nx, ny multiples of 8 and nz >= 8");
      return OC_ERR_UNSUPPORTED;
    }
    if (!(d->radius > 0) || d->y0 < -90.0 || d->y0 + d->ly > 90.0 || d->topology_z != OC_BOUNDED) {
      set_error("lat-lon grid needs radius > 0, latitudes within [-90, 90] and walls in z");
      return OC_ERR_ARG;
    }
  } else {
    set_error("coord must be OC_RECTILINEAR or OC_LATLON");
    return OC_ERR_ARG;
  }
  return OC_OK;
}

int validate_model(const oc_model_desc* m) {
  if (!m) { set_error("model descriptor is NULL"); return OC_ERR_ARG; }
  if (m->kind != OC_NONHYDROSTATIC && m->kind != OC_HYDROSTATIC) {
    set_error("kind must be OC_NONHYDROSTATIC or OC_HYDROSTATIC");
    return OC_ERR_ARG;
  }
  if (m->precision != OC_FP64 && m->precision != OC_FP32_MIXED) {
    set_error("precision must be OC_FP64 or OC_FP32_MIXED");
    return OC_ERR_ARG;
  }
  if (m->advection < OC_ADV_NONE || m->advection > OC_ADV_WENO9_LINEAR) {
    set_error("unknown advection scheme %d", m->advection);
    return OC_ERR_ARG;
  }
  if (m->kind == OC_HYDROSTATIC && m->advection > OC_ADV_WENO5_LINEAR) {
    set_error("the hydrostatic model supports WENO5 advection only");
    return OC_ERR_UNSUPPORTED;
  }
  const bool wenoz = m->advection == OC_ADV_WENO5Z || m->advection == OC_ADV_WENO7Z ||
                     m->advection == OC_ADV_WENO9Z;
  if (wenoz && (!(m->weno_eps > 0) || m->weno_q != 2)) {
    set_error("WENO-Z needs weno_eps > 0 and weno_q == 2");
    return OC_ERR_UNSUPPORTED;
  }
  if (m->ntracers < 1 || m->ntracers > OC_MAX_TRACERS) {
    set_error("ntracers must be in 1..%d", OC_MAX_TRACERS);
    return OC_ERR_ARG;
  }
  if (m->buoyancy && m->ntracers < 2) {
    set_error("buoyancy needs tracers 0 and 1 (T and S)");
    return OC_ERR_ARG;
  }
  if (!(m->nu >= 0) || !(m->kappa >= 0)) {
    set_error("nu and kappa must be >= 0");
    return OC_ERR_ARG;
  }
  if (m->kind == OC_HYDROSTATIC && !(m->depth > 0)) {
    set_error("hydrostatic model needs depth > 0");
    return OC_ERR_ARG;
  }
  if (m->les < OC_LES_NONE || m->les > OC_LES_AMD) {
    set_error("unknown LES closure %d", m->les);
    return OC_ERR_ARG;
  }
  if (m->les && (!(m->les_c > 0) || !(m->les_cb >= 0) ||
                 (m->les == OC_LES_SMAGORINSKY && !(m->les_pr > 0)))) {
    set_error("LES constants: les_c > 0, les_cb >= 0, les_pr > 0");
    return OC_ERR_ARG;
  }
  if (m->implicit_z != 0 && m->implicit_z != 1) {
    set_error("implicit_z must be 0 or 1");
    return OC_ERR_ARG;
  }
  if (m->kind == OC_HYDROSTATIC && m->ntracers != 2) {
    set_error("the hydrostatic model carries exactly T and S (ntracers = 2)");
    return OC_ERR_ARG;
  }
  if (m->immersed != 0 && m->immersed != 1) {
    set_error("immersed must be 0 or 1");
    return OC_ERR_ARG;
  }
  if (m->immersed) {
    if (!(m->cg_tol > 0) || !std::isfinite(m->cg_tol) || m->cg_maxiter < 1 ||
        m->cg_maxiter > 10000) {
      set_error("immersed boundary: cg_tol > 0 and 1 <= cg_maxiter <= 10000");
      return OC_ERR_ARG;
    }
    if (m->kind != OC_NONHYDROSTATIC || m->advection > OC_ADV_WENO5_LINEAR || m->implicit_z ||
        m->les || m->closure) {
      set_error("an immersed boundary needs the nonhydrostatic model with WENO5 or no advection "
                "and no implicit_z, LES or learned closure");
      return OC_ERR_UNSUPPORTED;
    }
  }
  return OC_OK;
}

int validate_pair(const oc_grid_desc& g, const oc_model_desc& m) {
  if (m.kind == OC_NONHYDROSTATIC && g.coord != OC_RECTILINEAR) {
    set_error("the nonhydrostatic model runs on rectilinear grids");
    return OC_ERR_UNSUPPORTED;
  }
  if (m.kind == OC_HYDROSTATIC && g.coord != OC_LATLON) {
    set_error("the hydrostatic model runs on lat-lon grids");
    return OC_ERR_UNSUPPORTED;
  }
  if (m.kind == OC_HYDROSTATIC) {
    // its tendency kernel addresses a field by 32-bit byte offsets
    const Dims hd = make_dims(g.nx, g.ny, g.nz, true, halo_width(m.advection));
    const long esz = m.precision == OC_FP64 ? 8 : 4;
    if ((long)hd.px * hd.py * hd.pz * esz >= (1L << 32)) {
      set_error("the hydrostatic model needs fields of fewer than 2^32 bytes with halos");
      return OC_ERR_UNSUPPORTED;
    }
  }
  if (m.kind == OC_NONHYDROSTATIC) {
    // the tendency kernel addresses the state, tendency, closure and mask
    // fields by 32-bit byte offsets from the lowest of them
    const Layout L = make_layout(g, m);
    const Dims nd = make_dims(g.nx, g.ny, g.nz, g.topology_z == OC_BOUNDED,
                              halo_width(m.advection));
    const uint64_t fb = (uint64_t)padded_elems(nd) * (m.precision == OC_FP64 ? 8 : 4);
    const int nf = 3 + m.ntracers;
    uint64_t hi = L.G[nf - 1] + fb;
    const int ngc = m.closure ? 4 : (m.les ? nf : 0);
    if (ngc) hi = std::max(hi, L.gc[ngc - 1] + fb);
    if (m.immersed) hi = std::max(hi, L.mask + fb);
    if (hi > 0xFFFFFFFFull) {
      set_error("the fields of the tendency kernel span %llu bytes; at most 2^32 - 1 are "
                "addressable", (unsigned long long)hi);
      return OC_ERR_UNSUPPORTED;
    }
  }
  if (m.implicit_z && (m.kind != OC_NONHYDROSTATIC || g.topology_z != OC_BOUNDED)) {
    set_error("implicit vertical diffusion needs the nonhydrostatic model with walls in z");
    return OC_ERR_UNSUPPORTED;
  }
  if (m.les && (m.kind != OC_NONHYDROSTATIC || m.closure)) {
    set_error("the LES closure needs the nonhydrostatic model without a learned closure");
    return OC_ERR_UNSUPPORTED;
  }
  if (m.closure && g.z_faces) {
    set_error("the learned closure needs a uniform z");
    return OC_ERR_UNSUPPORTED;
  }
  if (m.immersed && g.z_faces) {
    set_error("an immersed boundary needs a uniform z");
    return OC_ERR_UNSUPPORTED;
  }
  return OC_OK;
}

bool is_2d_field(int field) { return field >= OC_ETA && field <= OC_TAUY; }

int nzf_of(const oc_model* m, int field) {
  if (is_2d_field(field)) return 1;
  return (field == OC_W && m->dims.zb) ? m->dims.nz + 1 : m->dims.nz;
}

// rows of a field: v-like fields of the hydrostatic model include the
// northern wall face
int nyf_of(const oc_model* m, int field) {
  const bool vlike = field == OC_VBT || field == OC_GVBT || field == OC_TAUY ||
                     (m->kind == OC_HYDROSTATIC && field == OC_V);
  return vlike ? m->dims.ny + 1 : m->dims.ny;
}

int check_field_io(const oc_model* m, int field, const void* buf, int dtype,
                   const int64_t shape[3]) {
  if (!m || !buf || !shape) { set_error("NULL argument"); return OC_ERR_ARG; }
  const bool f2 = is_2d_field(field) && m->kind == OC_HYDROSTATIC;
  if (!f2 && (field < 0 || field >= m->nf)) {
    set_error("field %d is not a field of this model", field);
    return OC_ERR_ARG;
  }
  if (dtype != OC_F32 && dtype != OC_F64) { set_error("dtype must be OC_F32 or OC_F64"); return OC_ERR_DTYPE; }
  if (f2 && dtype != OC_F64) { set_error("barotropic fields are FP64"); return OC_ERR_DTYPE; }
  if (shape[0] != nzf_of(m, field) || shape[1] != nyf_of(m, field) || shape[2] != m->dims.nx) {
    set_error("shape (%lld, %lld, %lld) does not match (%d, %d, %d)", (long long)shape[0],
              (long long)shape[1], (long long)shape[2], nzf_of(m, field), nyf_of(m, field),
              m->dims.nx);
    return OC_ERR_SHAPE;
  }
  return OC_OK;
}

double* baro_field(oc_model* m, int field) {
  switch (field) {
    case OC_ETA: return m->eta[m->bcur];
    case OC_UBT: return m->ubt[m->bcur];
    case OC_VBT: return m->vbt[m->bcur];
    case OC_GUBT: return m->gubt;
    case OC_TAUX: return m->taux;
    case OC_TAUY: return m->tauy;
    default: return m->gvbt;
  }
}

int baro_io(oc_model* m, int field, void* buf, int on_device, int to_host, hipStream_t s) {
  double* f = baro_field(m, field);
  const size_t bytes = (size_t)nyf_of(m, field) * m->dims.nx * 8;
  if (to_host) {
    OC_CHECK_HIP(hipMemcpyAsync(buf, f, bytes,
                                on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
  } else {
    OC_CHECK_HIP(hipMemcpyAsync(f, buf, bytes,
                                on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
  }
  if (!on_device) OC_CHECK_HIP(hipStreamSynchronize(s));
  return OC_OK;
}

// Event pair around a launch group when profiling is on.
struct ProfScope {
  oc_model* m;
  hipStream_t s;
  bool on;
  ProfScope(oc_model* m_, int cls, hipStream_t s_)
      : m(m_), s(s_), on(m_->prof_on != 0 && ((m_->prof_mask >> cls) & 1u)) {
    if (!on) return;
    while (m->ev_pool.size() < m->ev_used + 2) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) { on = false; return; }
      m->ev_pool.push_back(e);
    }
    m->prof_cls.push_back(cls);
    (void)hipEventRecord(m->ev_pool[m->ev_used], s);
  }
  ~ProfScope() {
    if (!on) return;
    (void)hipEventRecord(m->ev_pool[m->ev_used + 1], s);
    m->ev_used += 2;
  }
};

template <class T>
int halo_one(oc_model* m, int which, int field, hipStream_t s) {
  T* f[1] = {(T*)m->state[which][field]};
  int kind[1] = {m->kinds[field]};
  OC_CHECK_HIP(launch_halo_fill<T>(m->dims, f, kind, 1, s));
  return OC_OK;
}


// The immersed-boundary mask in the padded layout, state precision: 1 in
// fluid cells, 0 in immersed ones (solid: nz * ny * nx bytes, nonzero =
// immersed; NULL: all fluid), with periodic images in x, y (and a periodic
// z) and mirror images below and above walls.
std::vector<char> padded_mask(const oc_model* m, const uint8_t* solid) {
  const Dims& d = m->dims;
  std::vector<char> out((size_t)padded_elems(d) * m->esz);
  for (int pk = 0; pk < d.pz; ++pk)
    for (int pj = 0; pj < d.py; ++pj)
      for (int pi = 0; pi < d.px; ++pi) {
        const int i = ((pi - d.h) % d.nx + d.nx) % d.nx;
        const int j = ((pj - d.h) % d.ny + d.ny) % d.ny;
        int k = pk - d.h;
        if (d.zb) k = (k < 0) ? -1 - k : (k >= d.nz ? 2 * d.nz - 1 - k : k);
        else k = (k % d.nz + d.nz) % d.nz;
        const bool imm = solid && solid[((size_t)k * d.ny + j) * d.nx + i] != 0;
        const double v = imm ? 0.0 : 1.0;
        const size_t at = (((size_t)pk * d.py + pj) * d.px + pi) * m->esz;
        if (m->esz == 8) std::memcpy(&out[at], &v, 8);
        else { const float f = (float)v; std::memcpy(&out[at], &f, 4); }
      }
  return out;
}

// The per-cell geometry bytes of the conjugate-gradient kernels (IB_*):
// fluid, and which faces are open (both neighbours fluid; walls closed).
std::vector<uint8_t> geometry_bits(const oc_model* m, const uint8_t* solid) {
  const Dims& d = m->dims;
  const long n = (long)d.nx * d.ny * d.nz;
  std::vector<uint8_t> out(n, 0);
  auto fluid = [&](int i, int j, int k) {
    i = (i + d.nx) % d.nx;
    j = (j + d.ny) % d.ny;
    k = (k + d.nz) % d.nz;
    return !solid || solid[((size_t)k * d.ny + j) * d.nx + i] == 0;
  };
  for (int k = 0; k < d.nz; ++k)
    for (int j = 0; j < d.ny; ++j)
      for (int i = 0; i < d.nx; ++i) {
        if (!fluid(i, j, k)) continue;
        uint8_t b = IB_FLUID;
        if (fluid(i - 1, j, k)) b |= IB_XM;
        if (fluid(i + 1, j, k)) b |= IB_XP;
        if (fluid(i, j - 1, k)) b |= IB_YM;
        if (fluid(i, j + 1, k)) b |= IB_YP;
        if ((!d.zb || k > 0) && fluid(i, j, k - 1)) b |= IB_ZM;
        if ((!d.zb || k + 1 < d.nz) && fluid(i, j, k + 1)) b |= IB_ZP;
        out[((size_t)k * d.ny + j) * d.nx + i] = b;
      }
  return out;
}

template <class T>
int tendency_call(oc_model* m, int in, int out, int stage, double dt, int combine,
                  hipStream_t s) {
  FieldSet<T> fs;
  for (int q = 0; q < MAXF; ++q) {
    fs.in[q] = (q < m->nf) ? (const T*)m->state[in][q] : nullptr;
    fs.out[q] = (q < m->nf) ? (T*)m->state[out][q] : nullptr;
    fs.G[q] = (q < m->nf) ? (T*)m->G[q] : nullptr;
  }
  for (int q = 0; q < MAXF; ++q) fs.closure[q] = (m->net && q < 4) ? (const T*)m->gc[q] : nullptr;
  fs.mask = m->md.immersed ? (const T*)m->mask : nullptr;
  if (m->net) {
    // learned closure of the current state: the fused gather + network, then
    // the flux divergence of its outputs
    ProfScope pc(m, OC_PROF_CLOSURE, s);
    const T* const* x = fs.in;
    OC_CHECK_HIP(launch_closure_mlp_fused<T>(m->dims, x[0], x[1], x[2], x[3], x[4], m->cst,
                                             mlp_params(m->net), mlp_output_rw(m->net), s));
    OC_CHECK_HIP(launch_closure_apply<T>(m->dims, mlp_output(m->net), m->cst, 1.0 / m->dz,
                                         (T*)m->gc[0], (T*)m->gc[1], (T*)m->gc[2], (T*)m->gc[3],
                                         s));
  }
  TendParams<T> p = tend_params<T>(m);
  if (m->md.les) {
    // eddy-viscosity closure of the current state: viscosity at the centres,
    // then the closure tendencies of every field, added by the tendency kernel
    ProfScope pl(m, OC_PROF_LES, s);
    LesArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    a.u = fs.in[0];
    a.v = fs.in[1];
    a.w = fs.in[2];
    a.c0 = fs.in[3];
    a.c1 = (m->nf > 4) ? fs.in[4] : fs.in[3];
    a.ntr = m->nf - 3;
    for (int q = 0; q < a.ntr; ++q) {
      a.tr[q] = fs.in[3 + q];
      a.kap[q] = (T*)m->les_kap[q];
    }
    a.nu = (T*)m->les_nu;
    for (int q = 0; q < m->nf; ++q) a.gc[q] = (T*)m->gc[q];
    a.rdx = p.rdx;
    a.rdy = p.rdy;
    a.rdzc = p.rdzc;
    a.rdzf = p.rdzf;
    a.delta2 = (const T*)m->les_d2;
    a.cb = (T)m->md.les_cb;
    a.camd = (T)m->md.les_c;
    a.rpr = (T)(m->md.les == OC_LES_SMAGORINSKY ? 1.0 / m->md.les_pr : 1.0);
    a.buoyancy = (m->md.buoyancy && m->nf > 4) ? 1 : 0;
    a.g_alpha = p.g_alpha;
    a.g_beta = p.g_beta;
    a.t_ref = p.t_ref;
    a.s_ref = p.s_ref;
    OC_CHECK_HIP(launch_les<T>(m->dims, a, m->md.les, s));
    for (int q = 0; q < m->nf; ++q) fs.closure[q] = (const T*)m->gc[q];
  }
  ProfScope ps(m, OC_PROF_TENDENCY, s);
  p.dt = (T)dt;
  p.gam = (T)RK_GAMMA[stage];
  p.zet = (T)RK_ZETA[stage];
  p.stage = stage;
  p.combine = combine;
  p.images = combine;  // substage outputs are final for tracers
  OC_CHECK_HIP(launch_tendency_fast<T>(m->dims, fs, p, m->md.advection, s));
  return OC_OK;
}

// The FFT/DCT solve of the whole box applied to a dense FP64 field: sb.p =
// L^-1 src (the preconditioner of the immersed-boundary iteration); the last
// pass also leaves the partial sums of src . sb.p in cg.part (*npart).  The
// passes do nothing once the iteration's stop flag is set.
int fft_solve_dense(oc_model* m, const double* src, int* npart, hipStream_t s) {
  SpecBufs sb = m->sb;
  sb.stop = m->cg.scal + CG_DONE;
  {
    ProfScope ps(m, OC_PROF_FFT_X_FWD, s);
    OC_CHECK_HIP(launch_poisson_x_forward_dense(m->dims, src, sb, s));
  }
  {
    ProfScope ps(m, OC_PROF_FFT_Y_FWD, s);
    OC_CHECK_HIP(launch_poisson_y(m->dims, sb, -1, s));
  }
  {
    ProfScope ps(m, OC_PROF_Z_SOLVE, s);
    OC_CHECK_HIP(launch_poisson_spectral(m->dims, sb, s));
  }
  {
    ProfScope ps(m, OC_PROF_FFT_Y_INV, s);
    OC_CHECK_HIP(launch_poisson_y(m->dims, sb, 1, s));
  }
  {
    ProfScope ps(m, OC_PROF_FFT_X_INV, s);
    OC_CHECK_HIP(launch_poisson_x_inverse_dot(m->dims, sb, src, m->cg.part, IB_PART_CAP, npart,
                                              s));
  }
  return OC_OK;
}

// Pressure correction with an immersed boundary: conjugate gradients on the
// masked Poisson equation, preconditioned by the FFT solve of the whole box
// (the residual is zero in immersed cells; the result is masked), until
// |r| <= cg_tol |b| or cg_maxiter iterations.  The scalars of an iteration
// stay on the device, and every kernel of an iteration does nothing once the
// stop flag is set, so the host need not look at the flag after every
// iteration: it first looks after one iteration fewer than the previous
// solve took, then after every iteration (solves of successive substeps
// take similar counts).  Queued iterations past convergence cost launches
// only.
template <class T>
int pressure_call_immersed(oc_model* m, int which, double dt_eff, hipStream_t s) {
  T* u = (T*)m->state[which][0];
  T* v = (T*)m->state[which][1];
  T* w = (T*)m->state[which][2];
  const T* mask = (const T*)m->mask;
  const Dims& d = m->dims;
  const CgBufs& cg = m->cg;
  const double tol2 = m->md.cg_tol * m->md.cg_tol;
  const int maxit = m->md.cg_maxiter;
  const double* z = m->sb.p;
  m->p_pending = false;   // sb.p is the iteration's work vector, then the solution
  {
    ProfScope pc(m, OC_PROF_CG, s);
    OC_CHECK_HIP(launch_ib_rhs<T>(d, u, v, w, m->ibits, 1.0 / dt_eff, 1.0 / m->dx,
                                  1.0 / m->dy, 1.0 / m->dz, cg, s));
    OC_CHECK_HIP(launch_ib_finalize(cg, CG_FIN_BNORM, tol2, maxit, s));
  }
  int npart = 0;
  int rc = fft_solve_dense(m, cg.r, &npart, s);
  if (rc) return rc;
  {
    ProfScope pc(m, OC_PROF_CG, s);
    OC_CHECK_HIP(launch_ib_finalize(cg, CG_FIN_RZ0, tol2, maxit, s, npart));
    OC_CHECK_HIP(launch_ib_dir(d, m->ibits, cg, z, s));
  }
  const double rdx2 = 1.0 / (m->dx * m->dx), rdy2 = 1.0 / (m->dy * m->dy);
  const double rdz2 = 1.0 / (m->dz * m->dz);
  const int first_look = std::max(1, m->cg_iterations - 1);
  for (int it = 0; it < maxit; ++it) {
    {
      ProfScope pc(m, OC_PROF_CG, s);
      OC_CHECK_HIP(launch_ib_apply(d, m->ibits, rdx2, rdy2, rdz2, cg, s));
      OC_CHECK_HIP(launch_ib_finalize(cg, CG_FIN_ALPHA, tol2, maxit, s));
      OC_CHECK_HIP(launch_ib_update(d, cg, s));
      OC_CHECK_HIP(launch_ib_finalize(cg, CG_FIN_RES, tol2, maxit, s));
    }
    if (it + 1 >= first_look || it + 1 == maxit) {   // the last iteration always looks
      OC_CHECK_HIP(hipMemcpyAsync(m->cg_host, cg.scal, CG_NSCAL * sizeof(double),
                                  hipMemcpyDeviceToHost, s));
      OC_CHECK_HIP(hipStreamSynchronize(s));
      if (m->cg_host[CG_DONE] != 0.0) break;
    }
    rc = fft_solve_dense(m, cg.r, &npart, s);
    if (rc) return rc;
    {
      ProfScope pc(m, OC_PROF_CG, s);
      OC_CHECK_HIP(launch_ib_finalize(cg, CG_FIN_BETA, tol2, maxit, s, npart));
      OC_CHECK_HIP(launch_ib_dir(d, m->ibits, cg, z, s));
    }
  }
  {
    ProfScope pc(m, OC_PROF_CG, s);
    OC_CHECK_HIP(launch_ib_xfinal(d, cg, s));
  }
  m->cg_iterations = (int)m->cg_host[CG_IT];
  m->cg_residual = m->cg_host[CG_BNORM2] > 0
                       ? std::sqrt(m->cg_host[CG_RNORM2] / m->cg_host[CG_BNORM2]) : 0.0;
  Spacing sp{1.0 / m->dx, 1.0 / m->dy, m->zt64 + zt_rdzc(d.nz), m->zt64 + zt_rdzf(d.nz)};
  {
    ProfScope pc(m, OC_PROF_CG, s);
    OC_CHECK_HIP(launch_ib_gauge(d, m->ibits, cg, m->nfluid, s));
    OC_CHECK_HIP(hipMemcpyAsync(m->sb.p, cg.x, (size_t)d.nx * d.ny * d.nz * sizeof(double),
                                hipMemcpyDeviceToDevice, s));
  }
  {
    ProfScope ps(m, OC_PROF_PROJECT, s);
    OC_CHECK_HIP(launch_project<T>(d, u, v, w, dt_eff, sp, cg.x, s, nullptr, 1, mask));
  }
  return OC_OK;
}

template <class T>
int pressure_call(oc_model* m, int which, double dt_eff, hipStream_t s) {
  if (m->md.immersed) return pressure_call_immersed<T>(m, which, dt_eff, s);
  const T* u = (const T*)m->state[which][0];
  const T* v = (const T*)m->state[which][1];
  const T* w = (const T*)m->state[which][2];
  const int nz = m->dims.nz;
  Spacing sp{1.0 / m->dx, 1.0 / m->dy, m->zt64 + zt_rdzc(nz), m->zt64 + zt_rdzf(nz)};
  {
    ProfScope ps(m, OC_PROF_FFT_X_FWD, s);
    OC_CHECK_HIP(launch_poisson_x_forward<T>(m->dims, u, v, w, 1.0 / dt_eff, sp, m->sb, s));
  }
  {
    ProfScope ps(m, OC_PROF_FFT_Y_FWD, s);
    OC_CHECK_HIP(launch_poisson_y(m->dims, m->sb, -1, s));
  }
  {
    ProfScope ps(m, OC_PROF_Z_SOLVE, s);
    if (m->stretched)
      OC_CHECK_HIP(launch_poisson_tridiag(m->dims, m->sb, m->zt64 + zt_lo(nz), m->zt64 + zt_up(nz),
                                          m->zt64 + zt_dzc(nz), m->zt64 + zt_dzf(nz), s));
    else
      OC_CHECK_HIP(launch_poisson_spectral(m->dims, m->sb, s));
  }
  {
    ProfScope ps(m, OC_PROF_FFT_Y_INV, s);
    OC_CHECK_HIP(launch_poisson_y(m->dims, m->sb, 1, s));
  }
  {
    ProfScope ps(m, OC_PROF_PROJECT, s);
    OC_CHECK_HIP(launch_poisson_x_inverse_project<T>(m->dims, m->sb, (T*)m->state[which][0],
                                                     (T*)m->state[which][1],
                                                     (T*)m->state[which][2], dt_eff, sp, s));
  }
  m->p_pending = true;
  return OC_OK;
}

// Elimination factors of the implicit vertical diffusion (FP64 on the host,
// stored in state precision).  stage >= 0: the three RK3 substages of a step
// dt (slot = substage, dt_eff = (gamma - zeta) dt), kept while dt repeats;
// stage < 0: one solve with dt_eff = dt in slot 0.  The upload is ordered on
// the stream after the work that used the previous factors.
template <class T>
int implicit_factors(oc_model* m, double dt, int stage, hipStream_t s) {
  if (stage >= 0 && m->vfac_dt == dt) return OC_OK;
  const int nz = m->dims.nz;
  std::vector<double> f64(vfac_len(nz), 0.0);
  const int nstage = stage < 0 ? 1 : 3;
  const int L = vertical_factors_len(nz);
  for (int st = 0; st < nstage; ++st) {
    const double dte = stage < 0 ? dt : (RK_GAMMA[st] - RK_ZETA[st]) * dt;
    double* base = f64.data() + (size_t)st * 3 * L;
    vertical_factors(m->hdzc.data(), m->hdzf.data(), nz, m->md.nu, dte, 0, base);
    vertical_factors(m->hdzc.data(), m->hdzf.data(), nz, m->md.nu, dte, 1, base + L);
    vertical_factors(m->hdzc.data(), m->hdzf.data(), nz, m->md.kappa, dte, 0, base + 2 * L);
  }
  m->vfac_host.resize(f64.size() * m->esz);
  for (size_t q = 0; q < f64.size(); ++q) {
    if (m->esz == 8) std::memcpy(&m->vfac_host[q * 8], &f64[q], 8);
    else { const float f = (float)f64[q]; std::memcpy(&m->vfac_host[q * 4], &f, 4); }
  }
  OC_CHECK_HIP(hipMemcpyAsync(m->vfac, m->vfac_host.data(), m->vfac_host.size(),
                              hipMemcpyHostToDevice, s));
  // the host buffer is rewritten by the next change of dt
  OC_CHECK_HIP(hipStreamSynchronize(s));
  m->vfac_dt = stage < 0 ? std::nan("") : dt;
  return OC_OK;
}

// Implicit vertical diffusion of state `which` with the factors of slot st.
template <class T>
int implicit_call(oc_model* m, int which, int st, hipStream_t s) {
  ProfScope ps(m, OC_PROF_IMPLICIT_Z, s);
  const int L = vertical_factors_len(m->dims.nz);
  const T* base = (const T*)m->vfac + (size_t)st * 3 * L;
  VImplicitArgs<T> a;
  for (int q = 0; q < m->nf; ++q) {
    const int cls = (q < 2) ? 0 : (q == 2 ? 1 : 2);  // u, v | w | tracers
    a.f[q] = (T*)m->state[which][q];
    a.fac[q] = base + (size_t)L * cls;
    a.wface[q] = (q == 2) ? 1 : 0;
  }
  OC_CHECK_HIP(launch_vertical_implicit<T>(m->dims, a, m->nf, s));
  return OC_OK;
}

template <class T>
int rk3_step_enqueue(oc_model* m, double dt, hipStream_t s) {
  for (int st = 0; st < 3; ++st) {
    const int in = m->cur, out = 1 - m->cur;
    int rc = tendency_call<T>(m, in, out, st, dt, 1, s);
    if (rc) return rc;
    if (m->md.implicit_z) {
      rc = implicit_call<T>(m, out, st, s);
      if (rc) return rc;
    }
    // the projection writes the velocity halos, the tendency kernel those
    // of the tracers
    rc = pressure_call<T>(m, out, (RK_GAMMA[st] - RK_ZETA[st]) * dt, s);
    if (rc) return rc;
    m->cur = out;
  }
  return OC_OK;
}

// Graphs are replaced only after the device has finished every launch of
// them (a replaced graph may still be running on the caller's stream).
void drop_step_graph(oc_model* m, int p) {
  if (!m->gexec[p]) return;
  (void)hipDeviceSynchronize();
  (void)hipGraphExecDestroy(m->gexec[p]);
  m->gexec[p] = nullptr;
}
void drop_step_graphs(oc_model* m) {
  drop_step_graph(m, 0);
  drop_step_graph(m, 1);
}

// Capture one RK3 step from buffer parity p as a graph (nothing runs).
template <class T>
int capture_step_graph(oc_model* m, double dt, int p) {
  drop_step_graph(m, p);
  if (!m->gcap && hipStreamCreateWithFlags(&m->gcap, hipStreamNonBlocking) != hipSuccess) {
    m->gcap = nullptr;
    set_error("capture stream creation failed");
    return OC_ERR_DEVICE;
  }
  hipGraph_t g;
  OC_CHECK_HIP(hipStreamBeginCapture(m->gcap, hipStreamCaptureModeThreadLocal));
  const int cur0 = m->cur;
  m->cur = p;
  const int rc = rk3_step_enqueue<T>(m, dt, m->gcap);
  m->cur = cur0;
  const hipError_t ce = hipStreamEndCapture(m->gcap, &g);
  if (rc) {
    if (ce == hipSuccess) (void)hipGraphDestroy(g);
    return rc;
  }
  if (ce != hipSuccess) {
    set_error("graph capture failed: %s", hipGetErrorString(ce));
    return OC_ERR_DEVICE;
  }
  const hipError_t ie = hipGraphInstantiate(&m->gexec[p], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) {
    m->gexec[p] = nullptr;
    set_error("graph instantiation failed: %s", hipGetErrorString(ie));
    return OC_ERR_DEVICE;
  }
  m->gdt[p] = dt;
  return OC_OK;
}

// Several steps in one call replay a captured step (one graph launch instead
// of 21 or more kernel launches); a single step, a profiled run and the
// immersed-boundary path (its iteration reads its residual on the host) are
// launched directly.
template <class T>
int rk3_steps(oc_model* m, double dt, int nsteps, hipStream_t s) {
  if (m->md.implicit_z) {
    int rc = implicit_factors<T>(m, dt, 0, s);
    if (rc) return rc;
  }
  const bool graphs = nsteps >= 2 && !m->prof_on && !m->md.immersed;
  for (int n = 0; n < nsteps; ++n) {
    if (graphs) {
      const int p = m->cur;
      if (!m->gexec[p] || m->gdt[p] != dt) {
        int rc = capture_step_graph<T>(m, dt, p);
        if (rc) return rc;
      }
      OC_CHECK_HIP(hipGraphLaunch(m->gexec[p], s));
      m->cur ^= 1;   // three substages
      m->p_pending = true;   // the replayed solves leave p as a spectrum
    } else {
      int rc = rk3_step_enqueue<T>(m, dt, s);
      if (rc) return rc;
    }
  }
  return OC_OK;
}

template <class T>
int field_io(oc_model* m, void* fieldbuf, int nzf, int nyf, void* buf, int dtype, int on_device,
             int to_dense, double offset, hipStream_t s) {
  const uint64_t bytes = (uint64_t)nzf * nyf * m->dims.nx * (dtype == OC_F32 ? 4 : 8);
  if (to_dense) {
    void* dst = on_device ? buf : m->staging;
    OC_CHECK_HIP(launch_pack<T>(m->dims, nzf, nyf, (const T*)fieldbuf, dst, dtype, 1, offset, s));
    if (!on_device) {
      OC_CHECK_HIP(hipMemcpyAsync(buf, m->staging, bytes, hipMemcpyDeviceToHost, s));
      OC_CHECK_HIP(hipStreamSynchronize(s));
    }
  } else {
    const void* src = buf;
    if (!on_device) {
      OC_CHECK_HIP(hipMemcpyAsync(m->staging, buf, bytes, hipMemcpyHostToDevice, s));
      OC_CHECK_HIP(hipStreamSynchronize(s));
      src = m->staging;
    }
    OC_CHECK_HIP(launch_pack<T>(m->dims, nzf, nyf, (const T*)fieldbuf, const_cast<void*>(src),
                                dtype, 0, offset, s));
  }
  return OC_OK;
}

template <class T>
int diagnostics_call(oc_model* m, double* out, hipStream_t s) {
  T* f[MAXF];
  for (int q = 0; q < m->nf; ++q) f[q] = (T*)m->state[m->cur][q];
  const int nz = m->dims.nz;
  OC_CHECK_HIP(launch_diagnostics<T>(m->dims, f, m->nf, 1.0 / m->dx, 1.0 / m->dy,
                                     m->zt64 + zt_rdzc(nz), m->zt64 + zt_dzc(nz),
                                     m->zt64 + zt_dzf(nz), m->diag_part, DIAG_BLOCKS, s));
  std::vector<double> part((size_t)DIAG_BLOCKS * DIAG_PARTS);
  OC_CHECK_HIP(hipMemcpyAsync(part.data(), m->diag_part, part.size() * 8, hipMemcpyDeviceToHost, s));
  OC_CHECK_HIP(hipStreamSynchronize(s));
  double acc[DIAG_PARTS] = {0};
  for (int b = 0; b < DIAG_BLOCKS; ++b)
    for (int q = 0; q < DIAG_PARTS; ++q) {
      double x = part[(size_t)b * DIAG_PARTS + q];
      acc[q] = (q < 4) ? std::fmax(acc[q], x) : acc[q] + x;
    }
  // sums are already weighted by the layer thickness
  const double area = m->dx * m->dy;
  out[0] = acc[0] * std::fmin(m->dx, std::fmin(m->dy, m->dzmin));
  out[1] = acc[1];
  out[2] = acc[2];
  out[3] = acc[3];
  const double ncell = (double)m->dims.nx * m->dims.ny * m->dims.nz;
  for (int q = 0; q < 4; ++q) {
    const double off = (OC_TRACER0 + q < m->nf) ? m->offset[OC_TRACER0 + q] : 0.0;
    out[4 + q] = (acc[4 + q] + off * ncell * m->dz) * area;
  }
  for (int q = 0; q < 3; ++q) out[8 + q] = acc[9 + q] * area;
  out[11] = std::fmax(acc[1] / m->dx, std::fmax(acc[2] / m->dy, acc[3] / m->dzmin));
  if (acc[8] > 0) {
    set_error("state holds %g non-finite cells", acc[8]);
    return OC_ERR_NONFINITE;
  }
  return OC_OK;
}

// Vertical tables of a grid (uniform or stretched z), in the layout of
// oc_model::zt64 (FP64) and oc_model::ztT (state precision, esz bytes).
void fill_z_tables(const oc_grid_desc& g, const std::vector<double>& zf, int esz,
                   std::vector<double>& z64, std::vector<char>& zT) {
  const int nz = g.nz;
  const bool bounded = g.topology_z == OC_BOUNDED;
  std::vector<double> dzc(nz), dzf(nz + 1);
  if (zf.empty()) {
    for (int k = 0; k < nz; ++k) dzc[k] = g.lz / nz;
    for (int k = 0; k <= nz; ++k) dzf[k] = g.lz / nz;
  } else {
    for (int k = 0; k < nz; ++k) dzc[k] = zf[k + 1] - zf[k];
    for (int k = 1; k < nz; ++k) dzf[k] = 0.5 * (zf[k + 1] - zf[k - 1]);
    dzf[0] = dzc[0];        // mirror image of the first centre below the wall
    dzf[nz] = dzc[nz - 1];
  }
  z64.assign(zt64_len(nz), 0.0);
  for (int k = 0; k < nz; ++k) {
    z64[zt_dzc(nz) + k] = dzc[k];
    z64[zt_rdzc(nz) + k] = 1.0 / dzc[k];
  }
  for (int k = 0; k <= nz; ++k) {
    z64[zt_dzf(nz) + k] = dzf[k];
    z64[zt_rdzf(nz) + k] = 1.0 / dzf[k];
  }
  // off-diagonals of the vertical part of the Laplacian (no flux at walls)
  for (int k = 0; k < nz; ++k) {
    z64[zt_lo(nz) + k] = (k > 0) ? 1.0 / (dzc[k] * dzf[k]) : 0.0;
    z64[zt_up(nz) + k] = (k < nz - 1) ? 1.0 / (dzc[k] * dzf[k + 1]) : 0.0;
  }
  // state precision: rdzc for k = -1..nz (images below and above), rdzf
  std::vector<double> t(ztT_len(nz));
  t[0] = 1.0 / (bounded ? dzc[0] : dzc[nz - 1]);
  for (int k = 0; k < nz; ++k) t[1 + k] = 1.0 / dzc[k];
  t[nz + 1] = 1.0 / (bounded ? dzc[nz - 1] : dzc[0]);
  for (int k = 0; k <= nz; ++k) t[nz + 2 + k] = 1.0 / dzf[k];
  zT.assign(t.size() * esz, 0);
  for (size_t q = 0; q < t.size(); ++q) {
    if (esz == 8) std::memcpy(&zT[q * 8], &t[q], 8);
    else { const float f = (float)t[q]; std::memcpy(&zT[q * 4], &f, 4); }
  }
}

void fill_tables(const oc_grid_desc& g, std::vector<double>& twx, std::vector<double>& twy,
                 std::vector<double>& twz, std::vector<double>& dctz, std::vector<double>& lamx,
                 std::vector<double>& lamy, std::vector<double>& lamz, double dx, double dy,
                 double dz) {
  const double pi = 3.14159265358979323846;
  auto tw = [&](std::vector<double>& t, int n) {
    t.resize(2 * n);
    for (int m = 0; m < n; ++m) {
      t[2 * m] = std::cos(2.0 * pi * m / n);
      t[2 * m + 1] = -std::sin(2.0 * pi * m / n);
    }
  };
  tw(twx, g.nx);
  tw(twy, g.ny);
  tw(twz, g.nz);
  dctz.resize(2 * g.nz);
  for (int k = 0; k < g.nz; ++k) {
    dctz[2 * k] = std::cos(pi * k / (2.0 * g.nz));
    dctz[2 * k + 1] = -std::sin(pi * k / (2.0 * g.nz));
  }
  auto lam = [&](std::vector<double>& t, int n, double h, bool neumann) {
    t.resize(n);
    for (int k = 0; k < n; ++k) {
      double s = std::sin(pi * k / (neumann ? 2.0 * n : (double)n));
      t[k] = -(4.0 / (h * h)) * s * s;
    }
  };
  lam(lamx, g.nx, dx, false);
  lam(lamy, g.ny, dy, false);
  lam(lamz, g.nz, dz, g.topology_z == OC_BOUNDED);
}

// Thin-shell metrics of a lat-lon grid, packed as len_u | dx_u | len_v |
// dy_v | area, each padded to ny + 1 entries.
void fill_latlon_metrics(const oc_grid_desc& g, std::vector<double>& met) {
  const double pi = 3.14159265358979323846;
  const int ny = g.ny;
  const double dlam = g.lx / g.nx * pi / 180.0;
  const double dphi = g.ly / ny * pi / 180.0;
  const double phi0 = g.y0 * pi / 180.0;
  const double R = g.radius;
  met.assign(5 * (size_t)(ny + 1), 0.0);
  double* len_u = met.data();
  double* dx_u = len_u + (ny + 1);
  double* len_v = dx_u + (ny + 1);
  double* dy_v = len_v + (ny + 1);
  double* area = dy_v + (ny + 1);
  for (int j = 0; j <= ny; ++j) {
    const double phf = phi0 + j * dphi;
    len_v[j] = R * std::cos(phf) * dlam;
    dy_v[j] = R * dphi;
    if (j < ny) {
      const double phc = phf + 0.5 * dphi;
      len_u[j] = R * dphi;
      dx_u[j] = R * std::cos(phc) * dlam;
      area[j] = R * R * dlam * (std::sin(phf + dphi) - std::sin(phf));
    }
  }
}

// Row tables of the baroclinic step (HydroMetric), rows j = -h .. ny + h
// for halo width h.
void fill_hydro_metrics(const oc_grid_desc& g, double omega, int H, std::vector<double>& met) {
  const double pi = 3.14159265358979323846;
  const int ny = g.ny, nt = ny + 2 * H + 1;
  const double dlam = g.lx / g.nx * pi / 180.0;
  const double dphi = g.ly / ny * pi / 180.0;
  const double phi0 = g.y0 * pi / 180.0;
  const double R = g.radius;
  met.assign((size_t)HYDRO_NMET * nt, 0.0);
  for (int r = 0; r < nt; ++r) {
    const int j = r - H;
    const double phf = phi0 + j * dphi, phc = phi0 + (j + 0.5) * dphi;
    const double phf1 = phi0 + (j + 1) * dphi, phcm = phi0 + (j - 0.5) * dphi;
    met[0 * (size_t)nt + r] = R * std::cos(phc) * dlam;
    met[1 * (size_t)nt + r] = R * std::cos(phf) * dlam;
    met[2 * (size_t)nt + r] = R * R * dlam * (std::sin(phf1) - std::sin(phf));
    met[3 * (size_t)nt + r] = R * R * dlam * (std::sin(phc) - std::sin(phcm));
    met[4 * (size_t)nt + r] = 2.0 * omega * std::sin(phc);
    met[5 * (size_t)nt + r] = 2.0 * omega * std::sin(phf);
  }
}

BaroBufs baro_bufs(oc_model* m) {
  BaroBufs b;
  const int ny = m->dims.ny;
  const int in = m->bcur, out = 1 - m->bcur;
  b.eta = m->eta[in];
  b.U = m->ubt[in];
  b.V = m->vbt[in];
  b.eta1 = m->eta[out];
  b.U1 = m->ubt[out];
  b.V1 = m->vbt[out];
  b.GU = m->gubt;
  b.GV = m->gvbt;
  b.etab = m->etab;
  b.Ub = m->ubar;
  b.Vb = m->vbar;
  b.len_u = m->metric;
  b.dx_u = m->metric + (ny + 1);
  b.len_v = m->metric + 2 * (ny + 1);
  b.dy_v = m->metric + 3 * (ny + 1);
  b.area = m->metric + 4 * (ny + 1);
  b.nx = m->dims.nx;
  b.ny = ny;
  return b;
}

ClosureStats closure_stats(const oc_model* m, const double* stats) {
  ClosureStats c;
  for (int q = 0; q < 4; ++q) {
    c.in_mean[q] = (float)stats[q];
    c.in_std[q] = (float)stats[4 + q];
    c.in_rstd[q] = (float)(1.0 / stats[4 + q]);
    c.out_mean[q] = (float)stats[8 + q];
    c.out_std[q] = (float)stats[12 + q];
  }
  c.g_alpha = (float)(m->md.g * m->md.alpha);
  c.g_beta = (float)(m->md.g * m->md.beta);
  c.t_ref = (float)(m->md.t_ref - m->offset[OC_TRACER0]);
  c.s_ref = (float)(m->md.s_ref - m->offset[OC_TRACER0 + 1]);
  c.inv_galpha = (float)(1.0 / (m->md.g * m->md.alpha));
  return c;
}

template <class T>
int coarse_grain_call(oc_model* fine, oc_model* coarse, int r, float* fluxes, hipStream_t s) {
  CoarseArgs<T> a;
  a.df = fine->dims;
  a.dc = coarse->dims;
  a.r = r;
  T* const* fs = (T* const*)fine->state[fine->cur];
  T* const* cs = (T* const*)coarse->state[coarse->cur];
  a.u = fs[0]; a.v = fs[1]; a.w = fs[2]; a.t = fs[3]; a.s = fs[4];
  a.U = cs[0]; a.V = cs[1]; a.W = cs[2]; a.Tc = cs[3]; a.Sc = cs[4];
  a.flux = fluxes;
  const oc_model_desc& d = fine->md;
  a.ga = d.g * d.alpha;
  a.gb = d.g * d.beta;
  a.tref = d.t_ref - fine->offset[OC_TRACER0];
  a.sref = d.s_ref - fine->offset[OC_TRACER0 + 1];
  OC_CHECK_HIP(launch_coarse_grain<T>(a, s));
  // halos (and the wall faces of w) of every coarse field
  int kinds[MAXF];
  for (int q = 0; q < coarse->nf; ++q) kinds[q] = coarse->kinds[q];
  OC_CHECK_HIP(launch_halo_fill<T>(coarse->dims, cs, kinds, coarse->nf, s));
  return OC_OK;
}

template <class T>
HydroBufs<T> hydro_bufs(oc_model* m, int in, int out) {
  HydroBufs<T> a;
  a.d = m->dims;
  const int nt = m->dims.ny + 2 * m->dims.h + 1;
  // tables of nt rows each; the kernels index them with j + h
  a.m.dxc = m->hmet + 0 * nt;
  a.m.dxf = m->hmet + 1 * nt;
  a.m.areac = m->hmet + 2 * nt;
  a.m.areaz = m->hmet + 3 * nt;
  a.m.fc = m->hmet + 4 * nt;
  a.m.ff = m->hmet + 5 * nt;
  const double pi = 3.14159265358979323846;
  a.m.dy = m->gd.radius * (m->gd.ly / m->gd.ny * pi / 180.0);
  a.m.dz = m->gd.lz / m->gd.nz;
  const oc_model_desc& d = m->md;
  a.eps = (T)d.weno_eps;
  a.nu = (T)d.nu;
  a.kappa = (T)d.kappa;
  a.ga = d.buoyancy ? (T)(d.g * d.alpha) : T(0);
  a.gb = d.buoyancy ? (T)(d.g * d.beta) : T(0);
  a.tref = (T)(d.t_ref - m->offset[OC_TRACER0]);
  a.sref = (T)(d.s_ref - m->offset[OC_TRACER0 + 1]);
  a.u = (const T*)m->state[in][OC_U];
  a.v = (const T*)m->state[in][OC_V];
  a.t = (const T*)m->state[in][OC_TRACER0];
  a.s = (const T*)m->state[in][OC_TRACER0 + 1];
  a.uo = (T*)m->state[out][OC_U];
  a.vo = (T*)m->state[out][OC_V];
  a.to = (T*)m->state[out][OC_TRACER0];
  a.so = (T*)m->state[out][OC_TRACER0 + 1];
  a.Gu = (T*)m->G[OC_U];
  a.Gv = (T*)m->G[OC_V];
  a.Gt = (T*)m->G[OC_TRACER0];
  a.Gs = (T*)m->G[OC_TRACER0 + 1];
  a.w = (T*)m->state[in][OC_W];
  a.zeta = (T*)m->hzeta;
  a.px = (T*)m->hpx;
  a.py = (T*)m->hpy;
  a.taux = m->taux;
  a.tauy = m->tauy;
  a.gub = m->gubt;
  a.gvb = m->gvbt;
  a.gub1 = m->gub1;
  a.gvb1 = m->gvb1;
  return a;
}

// Halos of the current state, then w, zeta and the pressure gradients.
template <class T>
int hydro_refresh(oc_model* m, hipStream_t s) {
  T* const* st = (T* const*)m->state[m->cur];
  {
    ProfScope ps(m, OC_PROF_HALO, s);
    OC_CHECK_HIP(launch_hydro_halo<T>(m->dims, st[OC_U], st[OC_V], st[OC_TRACER0],
                                      st[OC_TRACER0 + 1], s));
  }
  {
    ProfScope ps(m, OC_PROF_HYDRO_DIAG, s);
    OC_CHECK_HIP(launch_hydro_diag<T>(hydro_bufs<T>(m, m->cur, m->cur), s));
  }
  m->hstale = 0;
  return OC_OK;
}

template <class T>
int free_surface_call(oc_model* m, double dt, int N, int M, const double* a, hipStream_t s);

// QAB2 baroclinic steps coupled to the split-explicit barotropic mode.
template <class T>
int hydro_steps(oc_model* m, double dt, int N, int M, const double* a, int nsteps, hipStream_t s) {
  const double chi = 0.1;
  const int scheme = m->md.advection == OC_ADV_NONE ? 0
                     : (m->md.advection == OC_ADV_WENO5_LINEAR ? 2 : 1);
  for (int n = 0; n < nsteps; ++n) {
    if (m->hstale) {
      int rc = hydro_refresh<T>(m, s);
      if (rc) return rc;
    }
    HydroStep<T> st;
    st.dt = (T)dt;
    st.first = m->hfirst;
    st.a1 = m->hfirst ? T(1) : (T)(1.5 + chi);
    st.a0 = m->hfirst ? T(0) : (T)(0.5 + chi);
    {
      ProfScope ps(m, OC_PROF_HYDRO_TEND, s);
      OC_CHECK_HIP(launch_hydro_tendency<T>(hydro_bufs<T>(m, m->cur, 1 - m->cur), st, scheme, s));
    }
    m->cur = 1 - m->cur;
    m->hfirst = 0;
    {
      ProfScope ps(m, OC_PROF_BAROTROPIC, s);
      int rc = free_surface_call<T>(m, dt, N, M, a, s);
      if (rc) return rc;
    }
    int rc = hydro_refresh<T>(m, s);
    if (rc) return rc;
  }
  return OC_OK;
}

template <class T>
int free_surface_call(oc_model* m, double dt, int N, int M, const double* a, hipStream_t s) {
  const long n2 = (long)(m->dims.ny + 1) * m->dims.nx;
  OC_CHECK_HIP(launch_baro_fill(m->etab, 0.0, n2, s));
  OC_CHECK_HIP(launch_baro_fill(m->ubar, 0.0, n2, s));
  OC_CHECK_HIP(launch_baro_fill(m->vbar, 0.0, n2, s));
  const double dtau = dt / N;
  const double gH = m->md.g * m->md.depth;
  for (int n = 0; n < M;) {
    const int ns = std::min(baro_max_fused(), M - n);
    BaroBufs b = baro_bufs(m);
    OC_CHECK_HIP(launch_baro_substeps(b, dtau, gH, a + n, ns, s));
    m->bcur = 1 - m->bcur;
    n += ns;
  }
  // correction of the baroclinic velocity: its depth integral becomes Ubar
  const double dz = m->gd.lz / m->gd.nz;
  OC_CHECK_HIP(launch_baro_correct<T>(m->dims, (T*)m->state[m->cur][OC_U], m->ubar, 0,
                                      m->dims.ny, dz, m->md.depth, s));
  OC_CHECK_HIP(launch_baro_correct<T>(m->dims, (T*)m->state[m->cur][OC_V], m->vbar, 1,
                                      m->dims.ny, dz, m->md.depth, s));
  // restart of the barotropic state from the averages
  OC_CHECK_HIP(launch_baro_copy(m->eta[m->bcur], m->etab, (long)m->dims.ny * m->dims.nx, s));
  OC_CHECK_HIP(launch_baro_copy(m->ubt[m->bcur], m->ubar, (long)m->dims.ny * m->dims.nx, s));
  OC_CHECK_HIP(launch_baro_copy(m->vbt[m->bcur], m->vbar, n2, s));
  return OC_OK;
}

// Zero the current velocities on closed faces and refill their halos.
template <class T>
int mask_velocities_call(oc_model* m, hipStream_t s) {
  const int c = m->cur;
  OC_CHECK_HIP(launch_ib_mask_velocity<T>(m->dims, (T*)m->state[c][0], (T*)m->state[c][1],
                                          (T*)m->state[c][2], (const T*)m->mask, s));
  for (int q = 0; q < 3; ++q) {
    int rc = halo_one<T>(m, c, q, s);
    if (rc) return rc;
  }
  return OC_OK;
}

template <class T>
int set_immersed_call(oc_model* m, const uint8_t* solid, hipStream_t s) {
  std::vector<char> host = padded_mask(m, solid);
  const long n = (long)m->dims.nx * m->dims.ny * m->dims.nz;
  long nfluid = 0;
  for (long c = 0; c < n; ++c) nfluid += solid[c] == 0;
  if (nfluid == 0) {
    set_error("oc_set_immersed: no fluid cell left");
    return OC_ERR_UNSUPPORTED;
  }
  OC_CHECK_HIP(hipMemcpyAsync(m->mask, host.data(), host.size(), hipMemcpyHostToDevice, s));
  std::vector<uint8_t> bits = geometry_bits(m, solid);
  OC_CHECK_HIP(hipMemcpyAsync(m->ibits, bits.data(), bits.size(), hipMemcpyHostToDevice, s));
  const int rc = mask_velocities_call<T>(m, s);
  if (rc) return rc;
  OC_CHECK_HIP(hipStreamSynchronize(s));  // the host copy of the mask goes out of scope
  m->nfluid = (double)nfluid;
  return OC_OK;
}

}  // namespace

extern "C" {

const char* oc_last_error(void) { return g_err; }

int oc_grid_create(const oc_grid_desc* d, oc_grid** out) {
  if (!out) { set_error("out is NULL"); return OC_ERR_ARG; }
  int rc = validate_grid(d);
  if (rc) return rc;
  oc_grid* g = new (std::nothrow) oc_grid;
  if (!g) { set_error("out of host memory"); return OC_ERR_ARG; }
  g->d = *d;
  if (d->z_faces) {
    g->zf.assign(d->z_faces, d->z_faces + d->nz + 1);
    g->d.z_faces = g->zf.data();  // the grid's own copy
  }
  *out = g;
  return OC_OK;
}

int oc_grid_destroy(oc_grid* g) {
  delete g;
  return OC_OK;
}

int oc_model_workspace_size(const oc_grid* g, const oc_model_desc* m, uint64_t* bytes) {
  if (!g || !bytes) { set_error("NULL argument"); return OC_ERR_ARG; }
  int rc = validate_model(m);
  if (rc) return rc;
  rc = validate_pair(g->d, *m);
  if (rc) return rc;
  *bytes = make_layout(g->d, *m).total;
  return OC_OK;
}

int oc_model_create(const oc_grid* g, const oc_model_desc* md, void* workspace,
                    uint64_t workspace_bytes, oc_model** out) {
  if (!g || !out || !workspace) { set_error("NULL argument"); return OC_ERR_ARG; }
  int rc = validate_model(md);
  if (rc) return rc;
  rc = validate_pair(g->d, *md);
  if (rc) return rc;
  if (((uintptr_t)workspace) % 256) { set_error("workspace must be 256-byte aligned"); return OC_ERR_ARG; }
  const Layout L = make_layout(g->d, *md);
  if (workspace_bytes < L.total) {
    set_error("workspace has %llu bytes, needs %llu", (unsigned long long)workspace_bytes,
              (unsigned long long)L.total);
    return OC_ERR_ARG;
  }
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, workspace) != hipSuccess || attr.type != hipMemoryTypeDevice) {
    (void)hipGetLastError();
    set_error("workspace is not device memory");
    return OC_ERR_ARG;
  }
  oc_model* m = new (std::nothrow) oc_model;
  if (!m) { set_error("out of host memory"); return OC_ERR_ARG; }
  m->gd = g->d;
  m->gd.z_faces = nullptr;  // the model keeps only the device tables
  m->stretched = g->zf.empty() ? 0 : 1;
  m->md = *md;
  m->dims = make_dims(g->d.nx, g->d.ny, g->d.nz, g->d.topology_z == OC_BOUNDED,
                      halo_width(md->advection));
  m->nf = 3 + md->ntracers;
  m->esz = md->precision == OC_FP64 ? 8 : 4;
  for (int q = 0; q < MAXF; ++q) m->kinds[q] = (q == OC_W) ? 1 : 0;
  for (int q = 0; q < MAXF; ++q) m->offset[q] = 0.0;
  if (md->precision == OC_FP32_MIXED && md->buoyancy) {
    // FP32 resolves ~1e-6 of T ~ 20: store T and S as anomalies about the
    // equation-of-state reference.  The flux form is unchanged except for
    // offset * div(u), which vanishes for the projected velocity.
    m->offset[OC_TRACER0] = md->t_ref;
    m->offset[OC_TRACER0 + 1] = md->s_ref;
  }
  m->ws = (char*)workspace;
  m->ws_bytes = workspace_bytes;
  for (int s = 0; s < 2; ++s)
    for (int q = 0; q < MAXF; ++q) m->state[s][q] = m->ws + L.state[s][q];
  for (int q = 0; q < MAXF; ++q) m->G[q] = m->ws + L.G[q];
  m->cur = 0;
  m->prof_on = 0;
  m->prof_mask = (1u << OC_NPROF) - 1;
  m->ev_used = 0;
  m->dx = g->d.lx / g->d.nx;
  m->dy = g->d.ly / g->d.ny;
  m->dz = g->d.lz / g->d.nz;
  m->sb.spec = (double2*)(m->ws + L.spec);
  m->sb.p = (double*)(m->ws + L.p);
  m->sb.twx = (const double2*)(m->ws + L.twx);
  m->sb.twy = (const double2*)(m->ws + L.twy);
  m->sb.twz = (const double2*)(m->ws + L.twz);
  m->sb.dctz = (const double2*)(m->ws + L.dctz);
  m->sb.lamx = (const double*)(m->ws + L.lamx);
  m->sb.lamy = (const double*)(m->ws + L.lamy);
  m->sb.lamz = (const double*)(m->ws + L.lamz);
  m->sb.nxh = g->d.nx / 2 + 1;
  m->sb.nxp = spec_pitch(g->d.nx);
  m->staging = m->ws + L.staging;
  m->diag_part = (double*)(m->ws + L.diag);
  m->zt64 = (double*)(m->ws + L.zt64);
  m->ztT = m->ws + L.ztT;
  m->vfac = m->ws + L.vfac;
  m->vfac_dt = std::nan("");

  m->kind = md->kind;
  for (int q = 0; q < 2; ++q) {
    m->eta[q] = (double*)(m->ws + L.baro[0 + q]);
    m->ubt[q] = (double*)(m->ws + L.baro[2 + q]);
    m->vbt[q] = (double*)(m->ws + L.baro[4 + q]);
  }
  m->gubt = (double*)(m->ws + L.baro[6]);
  m->gvbt = (double*)(m->ws + L.baro[7]);
  m->etab = (double*)(m->ws + L.baro[8]);
  m->ubar = (double*)(m->ws + L.baro[9]);
  m->vbar = (double*)(m->ws + L.baro[10]);
  m->metric = (double*)(m->ws + L.metric);
  m->bcur = 0;
  m->hzeta = m->ws + L.hzeta;
  m->hpx = m->ws + L.hpx;
  m->hpy = m->ws + L.hpy;
  m->hmet = (double*)(m->ws + L.hmet);
  m->taux = (double*)(m->ws + L.baro[11]);
  m->tauy = (double*)(m->ws + L.baro[12]);
  m->gub1 = (double*)(m->ws + L.baro[13]);
  m->gvb1 = (double*)(m->ws + L.baro[14]);
  m->hfirst = 1;
  m->hstale = 1;
  m->net = nullptr;
  {
    const int ngc = md->closure ? 4 : (md->les ? m->nf : 0);
    for (int q = 0; q < MAXF; ++q) m->gc[q] = (q < ngc) ? (void*)(m->ws + L.gc[q]) : nullptr;
    m->les_nu = md->les ? (void*)(m->ws + L.les_nu) : nullptr;
    for (int q = 0; q < OC_MAX_TRACERS; ++q)
      m->les_kap[q] = (md->les == OC_LES_AMD && q < md->ntracers) ? (void*)(m->ws + L.les_kap[q])
                                                                   : nullptr;
    m->les_d2 = md->les ? (void*)(m->ws + L.les_d2) : nullptr;
  }
  m->mask = md->immersed ? (void*)(m->ws + L.mask) : nullptr;
  m->ibits = md->immersed ? (uint8_t*)(m->ws + L.ibits) : nullptr;
  m->cg.x = (double*)(m->ws + L.cg_x);
  m->cg.r = (double*)(m->ws + L.cg_r);
  m->cg.q = (double*)(m->ws + L.cg_q);
  m->cg.aq = (double*)(m->ws + L.cg_aq);
  m->cg.part = (double*)(m->ws + L.cg_part);
  m->cg.scal = (double*)(m->ws + L.cg_scal);
  m->cg_host = nullptr;
  m->cg_iterations = 0;
  m->cg_residual = 0.0;
  m->nfluid = (double)g->d.nx * g->d.ny * g->d.nz;

  hipError_t e = hipMemset(m->ws, 0, L.total);
  {
    std::vector<double> z64;
    std::vector<char> zT;
    fill_z_tables(g->d, g->zf, m->esz, z64, zT);
    const int nz = g->d.nz;
    m->hdzc.assign(z64.begin() + zt_dzc(nz), z64.begin() + zt_dzc(nz) + nz);
    m->hdzf.assign(z64.begin() + zt_dzf(nz), z64.begin() + zt_dzf(nz) + nz + 1);
    m->dzmin = *std::min_element(m->hdzc.begin(), m->hdzc.end());
    if (e == hipSuccess) e = hipMemcpy(m->zt64, z64.data(), z64.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->ztT, zT.data(), zT.size(), hipMemcpyHostToDevice);
    if (md->les) {
      // Smagorinsky-Lilly: (C_s Delta_k)^2, Delta_k = (dx dy dzc_k)^(1/3)
      std::vector<char> d2((size_t)nz * m->esz);
      for (int k = 0; k < nz; ++k) {
        const double v = std::pow(md->les_c * std::cbrt(m->dx * m->dy * m->hdzc[k]), 2.0);
        if (m->esz == 8) std::memcpy(&d2[(size_t)k * 8], &v, 8);
        else { const float f = (float)v; std::memcpy(&d2[(size_t)k * 4], &f, 4); }
      }
      if (e == hipSuccess) e = hipMemcpy(m->les_d2, d2.data(), d2.size(), hipMemcpyHostToDevice);
    }
  }
  if (md->kind == OC_NONHYDROSTATIC) {
    std::vector<double> twx, twy, twz, dctz, lamx, lamy, lamz;
    fill_tables(g->d, twx, twy, twz, dctz, lamx, lamy, lamz, m->dx, m->dy, m->dz);
    if (e == hipSuccess) e = hipMemcpy(m->ws + L.twx, twx.data(), twx.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->ws + L.twy, twy.data(), twy.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->ws + L.twz, twz.data(), twz.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->ws + L.dctz, dctz.data(), dctz.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->ws + L.lamx, lamx.data(), lamx.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->ws + L.lamy, lamy.data(), lamy.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->ws + L.lamz, lamz.data(), lamz.size() * 8, hipMemcpyHostToDevice);
  } else {
    std::vector<double> met;
    fill_latlon_metrics(g->d, met);
    if (e == hipSuccess) e = hipMemcpy(m->metric, met.data(), met.size() * 8, hipMemcpyHostToDevice);
    std::vector<double> hmet;
    fill_hydro_metrics(g->d, md->omega, m->dims.h, hmet);
    if (e == hipSuccess) e = hipMemcpy(m->hmet, hmet.data(), hmet.size() * 8, hipMemcpyHostToDevice);
  }
  if (md->immersed) {
    // every cell fluid until oc_set_immersed; pinned host room for the
    // iteration's scalars
    std::vector<char> ones = padded_mask(m, nullptr);
    if (e == hipSuccess) e = hipMemcpy(m->mask, ones.data(), ones.size(), hipMemcpyHostToDevice);
    std::vector<uint8_t> bits = geometry_bits(m, nullptr);
    if (e == hipSuccess) e = hipMemcpy(m->ibits, bits.data(), bits.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipHostMalloc((void**)&m->cg_host, CG_NSCAL * sizeof(double));
  }
  if (e != hipSuccess) {
    set_error("model setup failed: %s", hipGetErrorString(e));
    if (m->cg_host) (void)hipHostFree(m->cg_host);
    delete m;
    return OC_ERR_DEVICE;
  }
  *out = m;
  return OC_OK;
}

int oc_model_destroy(oc_model* m) {
  if (m) {
    for (hipEvent_t e : m->ev_pool) (void)hipEventDestroy(e);
    if (m->cg_host) (void)hipHostFree(m->cg_host);
    drop_step_graphs(m);
    if (m->gcap) (void)hipStreamDestroy(m->gcap);
  }
  delete m;
  return OC_OK;
}

int oc_profile(oc_model* m, int32_t enable) {
  if (!m) { set_error("model is NULL"); return OC_ERR_ARG; }
  if (enable) {
    m->ev_used = 0;
    m->prof_cls.clear();
  }
  m->prof_on = enable ? 1 : 0;
  return OC_OK;
}

int oc_profile_classes(oc_model* m, uint32_t classes) {
  if (!m) { set_error("model is NULL"); return OC_ERR_ARG; }
  if (classes >> OC_NPROF) { set_error("unknown profiling class bit"); return OC_ERR_ARG; }
  m->prof_mask = classes;
  return OC_OK;
}

int oc_profile_read(oc_model* m, double* ms, int64_t* launches) {
  if (!m || !ms || !launches) { set_error("NULL argument"); return OC_ERR_ARG; }
  for (int c = 0; c < OC_NPROF; ++c) { ms[c] = 0.0; launches[c] = 0; }
  if (m->ev_used == 0) return OC_OK;
  OC_CHECK_HIP(hipEventSynchronize(m->ev_pool[m->ev_used - 1]));
  for (size_t r = 0; r < m->prof_cls.size(); ++r) {
    float t = 0.f;
    OC_CHECK_HIP(hipEventElapsedTime(&t, m->ev_pool[2 * r], m->ev_pool[2 * r + 1]));
    ms[m->prof_cls[r]] += t;
    launches[m->prof_cls[r]] += 1;
  }
  return OC_OK;
}

int oc_set_state(oc_model* m, int32_t field, const void* buf, int32_t dtype, int32_t on_device,
                 const int64_t shape[3], void* stream) {
  int rc = check_field_io(m, field, buf, dtype, shape);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (is_2d_field(field)) {
    rc = baro_io(m, field, const_cast<void*>(buf), on_device, 0, s);
    if (rc) return rc;
    if (field == OC_VBT || field == OC_GVBT || field == OC_TAUY) {
      // the wall faces carry no transport
      double* f = baro_field(m, field);
      OC_CHECK_HIP(launch_baro_fill(f, 0.0, m->dims.nx, s));
      OC_CHECK_HIP(launch_baro_fill(f + (size_t)m->dims.ny * m->dims.nx, 0.0, m->dims.nx, s));
    }
    return OC_OK;
  }
  if (m->kind == OC_HYDROSTATIC && field == OC_W) {
    set_error("w is diagnosed from continuity in the hydrostatic model");
    return OC_ERR_ARG;
  }
  void* fb = m->state[m->cur][field];
  const int nzf = nzf_of(m, field), nyf = nyf_of(m, field);
  const double off = m->offset[field];
  if (m->esz == 8)
    rc = field_io<double>(m, fb, nzf, nyf, const_cast<void*>(buf), dtype, on_device, 0, off, s);
  else
    rc = field_io<float>(m, fb, nzf, nyf, const_cast<void*>(buf), dtype, on_device, 0, off, s);
  if (rc) return rc;
  if (field == OC_W && m->dims.zb) {
    // the bottom wall face carries no flow
    OC_CHECK_HIP(hipMemsetAsync((char*)fb + (size_t)m->dims.h * m->dims.sz * m->esz, 0,
                                (size_t)m->dims.sz * m->esz, s));
  }
  if (m->kind == OC_HYDROSTATIC) {
    // a new initial condition: halos and diagnostics are refreshed, and the
    // next baroclinic step starts the QAB2 history afresh
    m->hstale = 1;
    m->hfirst = 1;
    return OC_OK;
  }
  if (m->md.immersed && field <= OC_W)  // no flow through closed faces
    return (m->esz == 8) ? mask_velocities_call<double>(m, s) : mask_velocities_call<float>(m, s);
  return (m->esz == 8) ? halo_one<double>(m, m->cur, field, s) : halo_one<float>(m, m->cur, field, s);
}

int oc_get_state(oc_model* m, int32_t field, void* buf, int32_t dtype, int32_t on_device,
                 const int64_t shape[3], void* stream) {
  int rc = check_field_io(m, field, buf, dtype, shape);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (is_2d_field(field)) return baro_io(m, field, buf, on_device, 1, s);
  if (m->kind == OC_HYDROSTATIC && field == OC_W && m->hstale) {
    rc = (m->esz == 8) ? hydro_refresh<double>(m, s) : hydro_refresh<float>(m, s);
    if (rc) return rc;
  }
  void* fb = m->state[m->cur][field];
  const int nzf = nzf_of(m, field), nyf = nyf_of(m, field);
  const double off = m->offset[field];
  return (m->esz == 8) ? field_io<double>(m, fb, nzf, nyf, buf, dtype, on_device, 1, off, s)
                       : field_io<float>(m, fb, nzf, nyf, buf, dtype, on_device, 1, off, s);
}

int oc_tendencies(oc_model* m, void* stream) {
  if (!m) { set_error("model is NULL"); return OC_ERR_ARG; }
  if (m->kind != OC_NONHYDROSTATIC) { set_error("nonhydrostatic model only"); return OC_ERR_UNSUPPORTED; }
  hipStream_t s = (hipStream_t)stream;
  return (m->esz == 8) ? tendency_call<double>(m, m->cur, m->cur, 0, 0.0, 0, s)
                       : tendency_call<float>(m, m->cur, m->cur, 0, 0.0, 0, s);
}

int oc_get_tendency(oc_model* m, int32_t field, void* buf, int32_t dtype, int32_t on_device,
                    const int64_t shape[3], void* stream) {
  int rc = check_field_io(m, field, buf, dtype, shape);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (is_2d_field(field)) { set_error("barotropic fields have no tendency buffer"); return OC_ERR_ARG; }
  const int nzf = nzf_of(m, field), nyf = nyf_of(m, field);
  return (m->esz == 8)
             ? field_io<double>(m, m->G[field], nzf, nyf, buf, dtype, on_device, 1, 0.0, s)
             : field_io<float>(m, m->G[field], nzf, nyf, buf, dtype, on_device, 1, 0.0, s);
}

int oc_pressure_solve(oc_model* m, double dt_eff, void* stream) {
  if (!m) { set_error("model is NULL"); return OC_ERR_ARG; }
  if (m->kind != OC_NONHYDROSTATIC) { set_error("nonhydrostatic model only"); return OC_ERR_UNSUPPORTED; }
  if (!(dt_eff > 0) || !std::isfinite(dt_eff)) { set_error("dt_eff must be positive"); return OC_ERR_ARG; }
  hipStream_t s = (hipStream_t)stream;
  // the projection also refills the velocity halos
  return (m->esz == 8) ? pressure_call<double>(m, m->cur, dt_eff, s)
                       : pressure_call<float>(m, m->cur, dt_eff, s);
}

int oc_get_pressure(oc_model* m, double* buf, int32_t on_device, void* stream) {
  if (!m || !buf) { set_error("NULL argument"); return OC_ERR_ARG; }
  if (m->kind != OC_NONHYDROSTATIC) { set_error("nonhydrostatic model only"); return OC_ERR_UNSUPPORTED; }
  hipStream_t s = (hipStream_t)stream;
  const size_t bytes = (size_t)m->dims.nz * m->dims.ny * m->dims.nx * 8;
  if (m->p_pending) {
    OC_CHECK_HIP(launch_poisson_x_inverse(m->dims, m->sb, s));
    m->p_pending = false;
  }
  OC_CHECK_HIP(hipMemcpyAsync(buf, m->sb.p, bytes,
                              on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
  if (!on_device) OC_CHECK_HIP(hipStreamSynchronize(s));
  return OC_OK;
}

int oc_rk3_step(oc_model* m, double dt, int32_t nsteps, void* stream) {
  if (!m) { set_error("model is NULL"); return OC_ERR_ARG; }
  if (m->kind != OC_NONHYDROSTATIC) { set_error("nonhydrostatic model only"); return OC_ERR_UNSUPPORTED; }
  if (!(dt > 0) || !std::isfinite(dt)) { set_error("dt must be positive"); return OC_ERR_ARG; }
  if (nsteps < 0) { set_error("nsteps must be >= 0"); return OC_ERR_ARG; }
  hipStream_t s = (hipStream_t)stream;
  return (m->esz == 8) ? rk3_steps<double>(m, dt, nsteps, s) : rk3_steps<float>(m, dt, nsteps, s);
}

int oc_implicit_vertical_diffusion(oc_model* m, double dt_eff, void* stream) {
  if (!m) { set_error("model is NULL"); return OC_ERR_ARG; }
  if (m->kind != OC_NONHYDROSTATIC || !m->dims.zb) {
    set_error("implicit vertical diffusion needs a nonhydrostatic model with walls in z");
    return OC_ERR_UNSUPPORTED;
  }
  if (!(dt_eff > 0) || !std::isfinite(dt_eff)) { set_error("dt_eff must be positive"); return OC_ERR_ARG; }
  hipStream_t s = (hipStream_t)stream;
  int rc = (m->esz == 8) ? implicit_factors<double>(m, dt_eff, -1, s)
                         : implicit_factors<float>(m, dt_eff, -1, s);
  if (rc) return rc;
  return (m->esz == 8) ? implicit_call<double>(m, m->cur, 0, s)
                       : implicit_call<float>(m, m->cur, 0, s);
}

int oc_set_immersed(oc_model* m, const uint8_t* solid, void* stream) {
  if (!m || !solid) { set_error("NULL argument"); return OC_ERR_ARG; }
  if (!m->md.immersed) {
    set_error("the model was created without an immersed boundary (immersed = 0)");
    return OC_ERR_UNSUPPORTED;
  }
  hipStream_t s = (hipStream_t)stream;
  return m->esz == 8 ? set_immersed_call<double>(m, solid, s) : set_immersed_call<float>(m, solid, s);
}

int oc_pressure_stats(oc_model* m, int32_t* iterations, double* rel_residual, void* stream) {
  if (!m || !iterations || !rel_residual) { set_error("NULL argument"); return OC_ERR_ARG; }
  if (!m->md.immersed) {
    set_error("the model has no immersed boundary (no iterative solve)");
    return OC_ERR_UNSUPPORTED;
  }
  OC_CHECK_HIP(hipStreamSynchronize((hipStream_t)stream));
  *iterations = m->cg_iterations;
  *rel_residual = m->cg_residual;
  return OC_OK;
}

int oc_diagnostics(oc_model* m, double* out, void* stream) {
  if (!m || !out) { set_error("NULL argument"); return OC_ERR_ARG; }
  if (m->kind != OC_NONHYDROSTATIC) {
    set_error("diagnostics are defined for the nonhydrostatic (rectilinear) model");
    return OC_ERR_UNSUPPORTED;
  }
  hipStream_t s = (hipStream_t)stream;
  return (m->esz == 8) ? diagnostics_call<double>(m, out, s) : diagnostics_call<float>(m, out, s);
}

int oc_diagnostics_noalloc(oc_model* m, double* out, void* stream) {
  if (!m || !out) { set_error("NULL argument"); return OC_ERR_ARG; }
  if (m->kind != OC_NONHYDROSTATIC) {
    set_error("diagnostics are defined for the nonhydrostatic (rectilinear) model");
    return OC_ERR_UNSUPPORTED;
  }
  if (m->dims.nz > DIAG_MAX_LEVELS) {
    set_error("nz = %d exceeds the %d levels of the diagnostics scratch", m->dims.nz,
              DIAG_MAX_LEVELS);
    return OC_ERR_SHAPE;
  }
  hipStream_t s = (hipStream_t)stream;
  const int nz = m->dims.nz;
  DiagFinish f;
  f.hmin = std::fmin(m->dx, std::fmin(m->dy, m->dzmin));
  f.area = m->dx * m->dy;
  f.rdx = 1.0 / m->dx;
  f.rdy = 1.0 / m->dy;
  f.rdzmin = 1.0 / m->dzmin;
  const double ncell = (double)m->dims.nx * m->dims.ny * nz;
  for (int q = 0; q < 4; ++q)
    f.toff[q] = (OC_TRACER0 + q < m->nf) ? m->offset[OC_TRACER0 + q] * ncell * m->dz : 0.0;
  hipError_t e;
  if (m->esz == 8) {
    double* fl[MAXF];
    for (int q = 0; q < m->nf; ++q) fl[q] = (double*)m->state[m->cur][q];
    e = launch_diagnostics_noalloc<double>(m->dims, fl, m->nf, 1.0 / m->dx, 1.0 / m->dy,
                                           m->zt64 + zt_rdzc(nz), m->zt64 + zt_dzc(nz),
                                           m->zt64 + zt_dzf(nz), f, out, s);
  } else {
    float* fl[MAXF];
    for (int q = 0; q < m->nf; ++q) fl[q] = (float*)m->state[m->cur][q];
    e = launch_diagnostics_noalloc<float>(m->dims, fl, m->nf, 1.0 / m->dx, 1.0 / m->dy,
                                          m->zt64 + zt_rdzc(nz), m->zt64 + zt_dzc(nz),
                                          m->zt64 + zt_dzf(nz), f, out, s);
  }
  if (e != hipSuccess) {
    set_error("diagnostics launch failed: %s", hipGetErrorString(e));
    return OC_ERR_DEVICE;
  }
  return OC_OK;
}

int oc_sync_check(oc_model* m, void* stream) {
  if (!m) { set_error("model is NULL"); return OC_ERR_ARG; }
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("device error: %s", hipGetErrorString(e));
    return OC_ERR_DEVICE;
  }
  if (m->kind != OC_NONHYDROSTATIC) return OC_OK;
  double out[OC_NDIAG];
  return (m->esz == 8) ? diagnostics_call<double>(m, out, s) : diagnostics_call<float>(m, out, s);
}

int oc_free_surface_substeps(oc_model* m, double dt, int32_t N, int32_t M, const double* a,
                             void* stream) {
  if (!m || !a) { set_error("NULL argument"); return OC_ERR_ARG; }
  if (m->kind != OC_HYDROSTATIC) { set_error("hydrostatic model only"); return OC_ERR_UNSUPPORTED; }
  if (!(dt > 0) || N < 1 || M < 1 || M > 4096) {
    set_error("need dt > 0, N >= 1 and 1 <= M <= 4096");
    return OC_ERR_ARG;
  }
  for (int n = 0; n < M; ++n)
    if (!std::isfinite(a[n])) { set_error("weight %d is not finite", n); return OC_ERR_ARG; }
  hipStream_t s = (hipStream_t)stream;
  m->hstale = 1;  // the correction changes u and v
  return (m->esz == 8) ? free_surface_call<double>(m, dt, N, M, a, s)
                       : free_surface_call<float>(m, dt, N, M, a, s);
}

int oc_hydrostatic_step(oc_model* m, double dt, int32_t N, int32_t M, const double* a,
                        int32_t nsteps, void* stream) {
  if (!m || !a) { set_error("NULL argument"); return OC_ERR_ARG; }
  if (m->kind != OC_HYDROSTATIC) { set_error("hydrostatic model only"); return OC_ERR_UNSUPPORTED; }
  if (!(dt > 0) || !std::isfinite(dt) || N < 1 || M < 1 || M > 4096 || nsteps < 0) {
    set_error("need dt > 0, N >= 1, 1 <= M <= 4096 and nsteps >= 0");
    return OC_ERR_ARG;
  }
  for (int n = 0; n < M; ++n)
    if (!std::isfinite(a[n])) { set_error("weight %d is not finite", n); return OC_ERR_ARG; }
  hipStream_t s = (hipStream_t)stream;
  return (m->esz == 8) ? hydro_steps<double>(m, dt, N, M, a, nsteps, s)
                       : hydro_steps<float>(m, dt, N, M, a, nsteps, s);
}

int oc_model_set_closure(oc_model* m, oc_mlp* net, const double* stats, void* stream) {
  if (!m) { set_error("model is NULL"); return OC_ERR_ARG; }
  drop_step_graphs(m);   // captured steps launch the closure kernels with these arguments
  if (!net) { m->net = nullptr; return OC_OK; }
  if (m->kind != OC_NONHYDROSTATIC || !m->dims.zb || !m->md.buoyancy || !m->md.closure ||
      m->stretched) {
    set_error("the closure needs a wall-bounded, uniformly spaced nonhydrostatic model with T, S "
              "created with closure = 1");
    return OC_ERR_UNSUPPORTED;
  }
  if (!stats) { set_error("stats is NULL"); return OC_ERR_ARG; }
  const long ncell = (long)m->dims.nx * m->dims.ny * m->dims.nz;
  if (ncell % 32 || ncell > mlp_max_batch(net)) {
    set_error("the network's max_batch (%d) must cover the model's %ld cells", mlp_max_batch(net), ncell);
    return OC_ERR_ARG;
  }
  for (int q = 0; q < 4; ++q)
    if (!(stats[4 + q] > 0) || !(stats[12 + q] > 0)) { set_error("standard deviations must be > 0"); return OC_ERR_ARG; }
  hipStream_t s = (hipStream_t)stream;
  const int fin = mlp_params_finite(net, s);
  if (fin < 0) return fin;
  if (!fin) {
    m->net = nullptr;
    set_error("network parameters are not finite: the diffusive closure alone stays in use");
    return OC_ERR_NONFINITE;
  }
  m->cst = closure_stats(m, stats);
  m->net = net;
  return OC_OK;
}

int oc_closure_features(oc_model* m, const double* stats, float* x, void* stream) {
  if (!m || !stats || !x) { set_error("NULL argument"); return OC_ERR_ARG; }
  if (m->kind != OC_NONHYDROSTATIC || !m->dims.zb || !m->md.buoyancy || m->stretched) {
    set_error("features need a wall-bounded, uniformly spaced nonhydrostatic model with T, S");
    return OC_ERR_UNSUPPORTED;
  }
  for (int q = 0; q < 4; ++q)
    if (!(stats[4 + q] > 0)) { set_error("standard deviations must be > 0"); return OC_ERR_ARG; }
  const ClosureStats c = closure_stats(m, stats);
  hipStream_t s = (hipStream_t)stream;
  void* const* st = m->state[m->cur];
  if (m->esz == 8)
    OC_CHECK_HIP(launch_closure_features_f32<double>(
        m->dims, (const double*)st[0], (const double*)st[1], (const double*)st[2],
        (const double*)st[3], (const double*)st[4], c, x, s));
  else
    OC_CHECK_HIP(launch_closure_features_f32<float>(
        m->dims, (const float*)st[0], (const float*)st[1], (const float*)st[2],
        (const float*)st[3], (const float*)st[4], c, x, s));
  return OC_OK;
}

int oc_coarse_grain(oc_model* fine, oc_model* coarse, float* fluxes, void* stream) {
  if (!fine || !coarse) { set_error("NULL argument"); return OC_ERR_ARG; }
  if (fine->kind != OC_NONHYDROSTATIC || coarse->kind != OC_NONHYDROSTATIC ||
      !fine->dims.zb || !coarse->dims.zb || fine->nf < 5 || coarse->nf < 5 ||
      !fine->md.buoyancy || fine->stretched || coarse->stretched) {
    set_error("coarse-graining takes wall-bounded, uniformly spaced nonhydrostatic models with T, S");
    return OC_ERR_UNSUPPORTED;
  }
  if (fine->esz != coarse->esz) { set_error("both models need the same precision"); return OC_ERR_ARG; }
  const int r = fine->dims.nx / coarse->dims.nx;
  const Dims& f = fine->dims;
  const Dims& c = coarse->dims;
  if (r < 1 || f.nx != r * c.nx || f.ny != r * c.ny || f.nz != r * c.nz) {
    set_error("fine grid must be the coarse grid refined by one integer factor in x, y and z");
    return OC_ERR_SHAPE;
  }
  auto close = [](double a, double b) { return std::fabs(a - b) <= 1e-12 * std::fabs(b); };
  if (!close(fine->gd.lx, coarse->gd.lx) || !close(fine->gd.ly, coarse->gd.ly) ||
      !close(fine->gd.lz, coarse->gd.lz) || fine->offset[OC_TRACER0] != coarse->offset[OC_TRACER0] ||
      fine->offset[OC_TRACER0 + 1] != coarse->offset[OC_TRACER0 + 1]) {
    set_error("the models must cover the same domain with the same tracer storage");
    return OC_ERR_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  return fine->esz == 8 ? coarse_grain_call<double>(fine, coarse, r, fluxes, s)
                        : coarse_grain_call<float>(fine, coarse, r, fluxes, s);
}

}  // extern "C"
