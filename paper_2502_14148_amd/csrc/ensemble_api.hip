// Ensembles of nonhydrostatic models advanced together (C ABI declared in
// include/oc.h).  The paper runs many small simulations side by side (its
// motivation for GPU throughput, and ensembles for parameter studies); here
// one RK3 substage of every member is
//   * one launch of the fused tendency + RK3 kernel over all members' column
//     tiles (flat grid, or a persistent grid draining an atomic work queue),
//   * per class of members with equal grids, one launch per Poisson pass
//     with the member in blockIdx.z,
// and a whole RK3 step is captured once as a HIP graph per buffer parity and
// replayed.  An autotuner times the tile shape, the grid mode and the k
// chunking of the tendency launch and keeps the choice in a JSON-lines cache.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "model.h"

using namespace oc;

struct oc_ensemble {
  std::vector<oc_model*> mem;
  int esz;
  int flags;
  char* ws;
  uint64_t ws_bytes;
  void* dmem;              // EnsMember<T>[n]
  int2* items;
  int nitems;
  int max_items;
  int* counter;
  struct Class {
    std::vector<int> idx;  // members of this class
    PoissonSlots* slots[2];
  };
  std::vector<Class> classes;
  EnsTuning tn;
  int tuned;               // 0 default, 1 timed, 2 from the cache, 3 set by the caller
  double tune_ms;
  std::vector<int> cur0;
  int phase;
  double table_dt;
  hipStream_t cap;         // capture stream (never runs work)
  hipGraphExec_t exec[2];
  bool have_graphs;
  double graph_dt;
};

namespace {

#define OC_CHECK_HIP(expr)                                                       \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess) {                                                      \
      set_error("%s failed: %s", #expr, hipGetErrorString(e_));                  \
      return OC_ERR_DEVICE;                                                      \
    }                                                                            \
  } while (0)

uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

const int KC_DIVS[3] = {256, 1024, 4096};

int member_kc(const Dims& d, int nbx, int nby, int kc_div) {
  int kc = (int)((long)d.nz * nbx * nby / kc_div);
  kc = kc < 4 ? 4 : (kc > 64 ? 64 : kc);
  if (kc > d.nz) kc = d.nz;
  return kc;
}

bool tile_fits(const oc_model* m, int tile) {
  return m->dims.nx % ENS_TILE_X[tile] == 0 && m->dims.ny % ENS_TILE_Y[tile] == 0;
}

int validate_members(oc_model* const* members, int count) {
  if (!members || count < 1 || count > 4096) {
    set_error("need 1..4096 members");
    return OC_ERR_ARG;
  }
  for (int i = 0; i < count; ++i) {
    const oc_model* m = members[i];
    if (!m) { set_error("member %d is NULL", i); return OC_ERR_ARG; }
    if (m->kind != OC_NONHYDROSTATIC || m->md.advection != OC_ADV_WENO5Z ||
        m->md.ntracers != 2 || m->net || m->stretched || m->md.implicit_z || m->md.les ||
        m->md.immersed) {
      set_error("member %d: ensembles take nonhydrostatic WENO5-Z models with tracers T, S, "
                "uniform grids, explicit diffusion, no learned closure and no immersed "
                "boundary", i);
      return OC_ERR_UNSUPPORTED;
    }
    if (m->esz != members[0]->esz) {
      set_error("member %d: all members need the same precision", i);
      return OC_ERR_ARG;
    }
    if (!tile_fits(m, 2)) {
      set_error("member %d: nx and ny must be multiples of 8", i);
      return OC_ERR_UNSUPPORTED;
    }
    for (int j = 0; j < i; ++j)
      if (members[j] == m) { set_error("member %d appears twice", i); return OC_ERR_ARG; }
  }
  return OC_OK;
}

// Upper bound of the work items of any tuning candidate (8 x 8 tiles, the
// shortest k chunk).
int max_items_of(oc_model* const* members, int count) {
  long n = 0;
  for (int i = 0; i < count; ++i) {
    const Dims& d = members[i]->dims;
    n += (long)(d.nx / 8) * (d.ny / 8) * ((d.nz + 3) / 4);
  }
  return (int)n;
}

bool same_class(const oc_model* a, const oc_model* b) {
  return a->dims.nx == b->dims.nx && a->dims.ny == b->dims.ny && a->dims.nz == b->dims.nz &&
         a->dims.zb == b->dims.zb && a->dx == b->dx && a->dy == b->dy && a->dz == b->dz;
}

struct EnsLayout {
  uint64_t dmem, items, counter, slots, total;
  int nclass_max;
};

template <class T>
EnsLayout ens_layout(int count, int max_items) {
  EnsLayout L;
  uint64_t off = 0;
  L.dmem = off; off += align256(sizeof(EnsMember<T>) * (uint64_t)count);
  L.items = off; off += align256(sizeof(int2) * (uint64_t)max_items);
  L.counter = off; off += 256;
  L.nclass_max = count;  // at most one class per member
  L.slots = off; off += align256(sizeof(PoissonSlots)) * 2 * (uint64_t)count;
  L.total = off;
  return L;
}

// Work items (member, tile) of a tuning: members with longer k chunks first
// (the longest items start first); for the flat grid the order is permuted
// so that workgroups on one XCD (dispatched round-robin over the 8 XCDs)
// take consecutive tiles.
template <class T>
void build_items(const oc_ensemble* e, const EnsTuning& tn, std::vector<EnsMember<T>>& hm,
                 std::vector<int2>& items) {
  const int n = (int)e->mem.size();
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) {
    const oc_model* m = e->mem[i];
    EnsMember<T>& M = hm[i];
    M.d = m->dims;
    M.nbx = m->dims.nx / ENS_TILE_X[tn.tile];
    M.nby = m->dims.ny / ENS_TILE_Y[tn.tile];
    M.kc = member_kc(m->dims, M.nbx, M.nby, tn.kc_div);
    M.nbz = (m->dims.nz + M.kc - 1) / M.kc;
    order[i] = i;
  }
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return hm[a].kc > hm[b].kc; });
  std::vector<int2> nat;
  for (int i : order) {
    const int nt = hm[i].nbx * hm[i].nby * hm[i].nbz;
    for (int b = 0; b < nt; ++b) nat.push_back(make_int2(i, b));
  }
  const int ni = (int)nat.size();
  items.resize(ni);
  if (!tn.persistent && ni % 8 == 0) {
    for (int q = 0; q < ni; ++q) items[q] = nat[(q & 7) * (ni >> 3) + (q >> 3)];
  } else {
    items = nat;
  }
}

// Member tables for the current buffer assignment and dt.
template <class T>
void fill_member_params(const oc_ensemble* e, std::vector<EnsMember<T>>& hm, double dt) {
  const int n = (int)e->mem.size();
  for (int i = 0; i < n; ++i) {
    oc_model* m = e->mem[i];
    EnsMember<T>& M = hm[i];
    const int A = e->cur0[i], B = 1 - A;
    for (int par = 0; par < 2; ++par) {
      const int in = par ? B : A, out = par ? A : B;
      FieldSet<T>& fs = M.fs[par];
      for (int q = 0; q < MAXF; ++q) {
        fs.in[q] = (q < m->nf) ? (const T*)m->state[in][q] : nullptr;
        fs.out[q] = (q < m->nf) ? (T*)m->state[out][q] : nullptr;
        fs.G[q] = (q < m->nf) ? (T*)m->G[q] : nullptr;
      }
      for (int q = 0; q < MAXF; ++q) fs.closure[q] = nullptr;
      fs.mask = nullptr;
      // within 4 GiB: every member passed the model checks
      (void)fieldset_offsets(fs, (uint64_t)padded_elems(m->dims) * sizeof(T));
    }
    for (int st = 0; st < 3; ++st) {
      TendParams<T> p = tend_params<T>(m);
      p.dt = (T)dt;
      p.gam = (T)RK_GAMMA[st];
      p.zet = (T)RK_ZETA[st];
      p.stage = st;
      p.combine = 1;
      p.images = 1;
      M.P[st] = p;
    }
  }
}

template <class T>
int upload_tables(oc_ensemble* e, const EnsTuning& tn, double dt) {
  const int n = (int)e->mem.size();
  std::vector<EnsMember<T>> hm(n);
  std::vector<int2> items;
  build_items<T>(e, tn, hm, items);
  fill_member_params<T>(e, hm, dt);
  if ((int)items.size() > e->max_items) { set_error("work list overflow"); return OC_ERR_ARG; }
  OC_CHECK_HIP(hipMemcpy(e->dmem, hm.data(), sizeof(EnsMember<T>) * n, hipMemcpyHostToDevice));
  OC_CHECK_HIP(hipMemcpy(e->items, items.data(), sizeof(int2) * items.size(),
                         hipMemcpyHostToDevice));
  e->nitems = (int)items.size();
  // Poisson slots: parity par acts on the output buffer of that parity
  for (auto& c : e->classes) {
    for (int par = 0; par < 2; ++par) {
      PoissonSlots hs;
      std::memset(&hs, 0, sizeof(hs));
      for (size_t z = 0; z < c.idx.size(); ++z) {
        oc_model* m = e->mem[c.idx[z]];
        const int A = e->cur0[c.idx[z]], B = 1 - A;
        const int out = par ? A : B;
        hs.u[z] = m->state[out][0];
        hs.v[z] = m->state[out][1];
        hs.w[z] = m->state[out][2];
        hs.spec[z] = m->sb.spec;
        hs.p[z] = m->sb.p;
      }
      OC_CHECK_HIP(hipMemcpy(c.slots[par], &hs, sizeof(hs), hipMemcpyHostToDevice));
    }
  }
  e->table_dt = dt;
  return OC_OK;
}

// One RK3 step starting from buffer parity p (substages alternate parity).
template <class T>
int enqueue_step(oc_ensemble* e, int p, double dt, hipStream_t s) {
  for (int st = 0; st < 3; ++st) {
    const int par = p ^ (st & 1);
    OC_CHECK_HIP(launch_tendency_ensemble<T>((const EnsMember<T>*)e->dmem, e->items, e->nitems,
                                             e->counter, par, st, e->tn, s));
    const double dt_eff = (RK_GAMMA[st] - RK_ZETA[st]) * dt;
    for (auto& c : e->classes) {
      const oc_model* m0 = e->mem[c.idx[0]];
      const int ns = (int)c.idx.size();
      const PoissonSlots* bs = c.slots[par];
      // members of a class share their uniform spacings, so member 0's
      // vertical tables serve all of them
      const int nz = m0->dims.nz;
      Spacing sp{1.0 / m0->dx, 1.0 / m0->dy, m0->zt64 + zt_rdzc(nz), m0->zt64 + zt_rdzf(nz)};
      OC_CHECK_HIP(launch_poisson_x_forward<T>(m0->dims, nullptr, nullptr, nullptr, 1.0 / dt_eff,
                                               sp, m0->sb, s, bs, ns));
      OC_CHECK_HIP(launch_poisson_y(m0->dims, m0->sb, -1, s, bs, ns));
      OC_CHECK_HIP(launch_poisson_spectral(m0->dims, m0->sb, s, bs, ns));
      OC_CHECK_HIP(launch_poisson_y(m0->dims, m0->sb, 1, s, bs, ns));
      OC_CHECK_HIP(launch_poisson_x_inverse_project<T>(m0->dims, m0->sb, (T*)nullptr,
                                                       (T*)nullptr, (T*)nullptr, dt_eff, sp, s,
                                                       bs, ns));
    }
  }
  return OC_OK;
}

// ---- autotuner -------------------------------------------------------------

std::string tune_key(const oc_ensemble* e) {
  hipDeviceProp_t prop;
  int dev = 0;
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  std::vector<std::string> sizes;
  for (const oc_model* m : e->mem) {
    char b[64];
    snprintf(b, sizeof(b), "%dx%dx%d", m->dims.nx, m->dims.ny, m->dims.nz);
    sizes.push_back(b);
  }
  std::sort(sizes.begin(), sizes.end());
  std::string key = arch + (e->esz == 4 ? "|fp32|" : "|fp64|");
  for (size_t i = 0; i < sizes.size();) {
    size_t j = i;
    while (j < sizes.size() && sizes[j] == sizes[i]) ++j;
    key += sizes[i] + "*" + std::to_string(j - i) + (j < sizes.size() ? "," : "");
    i = j;
  }
  return key;
}

// Cache file: one JSON object per line,
// {"key": "...", "tile": t, "persistent": p, "kc_div": k, "ms": x}
bool cache_lookup(const char* path, const std::string& key, EnsTuning& tn, double& ms) {
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char line[1024];
  bool found = false;
  while (fgets(line, sizeof(line), f)) {
    char k[768];
    int t, p, kd;
    double x;
    if (sscanf(line, " {\"key\": \"%767[^\"]\", \"tile\": %d, \"persistent\": %d, \"kc_div\": %d, "
                     "\"ms\": %lf}", k, &t, &p, &kd, &x) == 5 &&
        key == k && t >= 0 && t <= 2 && (p == 0 || p == 1) && kd > 0) {
      tn.tile = t;
      tn.persistent = p;
      tn.kc_div = kd;
      ms = x;
      found = true;  // the last matching line wins
    }
  }
  fclose(f);
  return found;
}

void cache_store(const char* path, const std::string& key, const EnsTuning& tn, double ms) {
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "{\"key\": \"%s\", \"tile\": %d, \"persistent\": %d, \"kc_div\": %d, \"ms\": %.6f}\n",
          key.c_str(), tn.tile, tn.persistent, tn.kc_div, ms);
  fclose(f);
}

template <class T>
int persistent_blocks(const EnsTuning& tn) {
  hipDeviceProp_t prop;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return 256;
  return prop.multiProcessorCount * ensemble_blocks_per_cu<T>(tn.tile);
}

// Time the tendency launch (substage 1, parity 0: reads only the current
// state, writes the other buffer and G, which the next step overwrites).
template <class T>
int time_candidate(oc_ensemble* e, const EnsTuning& tn, double& ms) {
  int rc = upload_tables<T>(e, tn, 1.0);
  if (rc) return rc;
  hipEvent_t a, b;
  OC_CHECK_HIP(hipEventCreate(&a));
  OC_CHECK_HIP(hipEventCreate(&b));
  double best = 1e30;
  for (int r = 0; r < 4; ++r) {
    OC_CHECK_HIP(hipEventRecord(a, 0));
    OC_CHECK_HIP(launch_tendency_ensemble<T>((const EnsMember<T>*)e->dmem, e->items, e->nitems,
                                             e->counter, 0, 0, tn, 0));
    OC_CHECK_HIP(hipEventRecord(b, 0));
    OC_CHECK_HIP(hipEventSynchronize(b));
    float t = 0.f;
    OC_CHECK_HIP(hipEventElapsedTime(&t, a, b));
    if (r > 0) best = std::min(best, (double)t);  // the first run warms up
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  ms = best;
  return OC_OK;
}

template <class T>
EnsTuning default_tuning(const oc_ensemble* e) {
  EnsTuning def;
  def.tile = 0;
  for (const oc_model* m : e->mem)
    if (!tile_fits(m, 0)) def.tile = tile_fits(m, 1) ? std::max(def.tile, 1) : 2;
  def.persistent = 0;
  def.kc_div = 1024;
  def.nblocks = persistent_blocks<T>(def);
  return def;
}

// Time every candidate launch configuration and keep the fastest, or take the
// choice recorded under this ensemble's key in the cache file `path` (NULL:
// no cache).  A timed choice is appended to the cache.
template <class T>
int tune(oc_ensemble* e, const char* path) {
  const std::string key = tune_key(e);
  EnsTuning c;
  double ms = 0.0;
  if (path && cache_lookup(path, key, c, ms)) {
    bool ok = true;
    for (const oc_model* m : e->mem) ok = ok && tile_fits(m, c.tile);
    if (ok) {
      c.nblocks = persistent_blocks<T>(c);
      e->tn = c;
      e->tuned = 2;
      e->tune_ms = ms;
      return OC_OK;
    }
  }
  double best = 1e30;
  EnsTuning bt = default_tuning<T>(e);
  for (int tile = 0; tile < 3; ++tile) {
    bool ok = true;
    for (const oc_model* m : e->mem) ok = ok && tile_fits(m, tile);
    if (!ok) continue;
    for (int pers = 0; pers < 2; ++pers)
      for (int kd : KC_DIVS) {
        EnsTuning t;
        t.tile = tile;
        t.persistent = pers;
        t.kc_div = kd;
        t.nblocks = persistent_blocks<T>(t);
        double x = 0.0;
        int rc = time_candidate<T>(e, t, x);
        if (rc) return rc;
        if (x < best) { best = x; bt = t; }
      }
  }
  e->tn = bt;
  e->tuned = 1;
  e->tune_ms = best;
  if (path) cache_store(path, key, bt, best);
  return OC_OK;
}

template <class T>
int ens_setup(oc_ensemble* e) {
  e->tn = default_tuning<T>(e);
  e->tuned = 0;
  e->tune_ms = 0.0;
  if (e->flags & OC_ENS_TUNE) {
    int rc = tune<T>(e, nullptr);
    if (rc) return rc;
  }
  return upload_tables<T>(e, e->tn, e->table_dt);
}

void drop_graphs(oc_ensemble* e) {
  if (!e->have_graphs) return;
  (void)hipGraphExecDestroy(e->exec[0]);
  (void)hipGraphExecDestroy(e->exec[1]);
  e->have_graphs = false;
}

template <class T>
int capture_graphs(oc_ensemble* e, double dt) {
  drop_graphs(e);
  for (int p = 0; p < 2; ++p) {
    hipGraph_t g;
    OC_CHECK_HIP(hipStreamBeginCapture(e->cap, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_step<T>(e, p, dt, e->cap);
    hipError_t ce = hipStreamEndCapture(e->cap, &g);
    if (rc) {
      if (ce == hipSuccess) (void)hipGraphDestroy(g);
      if (p == 1) (void)hipGraphExecDestroy(e->exec[0]);
      return rc;
    }
    if (ce != hipSuccess) {
      set_error("graph capture failed: %s", hipGetErrorString(ce));
      if (p == 1) (void)hipGraphExecDestroy(e->exec[0]);
      return OC_ERR_DEVICE;
    }
    hipError_t ie = hipGraphInstantiate(&e->exec[p], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
      set_error("graph instantiation failed: %s", hipGetErrorString(ie));
      if (p == 1) (void)hipGraphExecDestroy(e->exec[0]);
      return OC_ERR_DEVICE;
    }
  }
  e->have_graphs = true;
  e->graph_dt = dt;
  return OC_OK;
}

template <class T>
int ens_step(oc_ensemble* e, double dt, int nsteps, hipStream_t s) {
  // members stepped on their own since the last call: restart the parities
  bool moved = false;
  for (size_t i = 0; i < e->mem.size(); ++i)
    moved = moved || (e->mem[i]->cur != (e->cur0[i] ^ e->phase));
  const bool redo = moved || dt != e->table_dt;
  if (redo) {
    // the tables are rewritten while earlier work on s may still read them
    OC_CHECK_HIP(hipStreamSynchronize(s));
    if (moved) {
      for (size_t i = 0; i < e->mem.size(); ++i) e->cur0[i] = e->mem[i]->cur;
      e->phase = 0;
    }
    int rc = upload_tables<T>(e, e->tn, dt);
    if (rc) return rc;
  }
  const bool graphs = (e->flags & OC_ENS_GRAPH) != 0;
  if (graphs && (!e->have_graphs || e->graph_dt != dt)) {
    int rc = capture_graphs<T>(e, dt);
    if (rc) return rc;
  }
  for (int n = 0; n < nsteps; ++n) {
    if (graphs) {
      OC_CHECK_HIP(hipGraphLaunch(e->exec[e->phase], s));
    } else {
      int rc = enqueue_step<T>(e, e->phase, dt, s);
      if (rc) return rc;
    }
    e->phase ^= 1;
  }
  for (size_t i = 0; i < e->mem.size(); ++i) {
    e->mem[i]->cur = e->cur0[i] ^ e->phase;
    if (nsteps > 0) e->mem[i]->p_pending = true;   // p left as a spectrum
  }
  return OC_OK;
}

// A new launch configuration: wait for queued work (the tables and the
// timing launches write device memory that it may still read), restart the
// buffer parities from where the members stand, then either time the
// candidates (`set` == NULL) or take `set`, and rebuild the tables; graphs
// are captured again on the next step.
template <class T>
int ens_retune(oc_ensemble* e, const char* path, const EnsTuning* set) {
  OC_CHECK_HIP(hipDeviceSynchronize());
  for (size_t i = 0; i < e->mem.size(); ++i) e->cur0[i] = e->mem[i]->cur;
  e->phase = 0;
  drop_graphs(e);
  if (set) {
    e->tn = *set;
    e->tn.nblocks = persistent_blocks<T>(e->tn);
    e->tuned = 3;
    e->tune_ms = 0.0;
  } else {
    int rc = tune<T>(e, path);
    if (rc) return rc;
  }
  return upload_tables<T>(e, e->tn, e->table_dt);
}

}  // namespace

extern "C" {

int oc_ensemble_workspace_size(oc_model* const* members, int32_t count, uint64_t* bytes) {
  if (!bytes) { set_error("bytes is NULL"); return OC_ERR_ARG; }
  int rc = validate_members(members, count);
  if (rc) return rc;
  const int mi = max_items_of(members, count);
  *bytes = members[0]->esz == 8 ? ens_layout<double>(count, mi).total
                                : ens_layout<float>(count, mi).total;
  return OC_OK;
}

int oc_ensemble_create(oc_model* const* members, int32_t count, void* workspace, uint64_t bytes,
                       int32_t flags, oc_ensemble** out) {
  if (!out) { set_error("out is NULL"); return OC_ERR_ARG; }
  int rc = validate_members(members, count);
  if (rc) return rc;
  if (flags & ~(OC_ENS_TUNE | OC_ENS_GRAPH)) { set_error("unknown flags"); return OC_ERR_ARG; }
  const int esz = members[0]->esz;
  const int mi = max_items_of(members, count);
  const EnsLayout L = esz == 8 ? ens_layout<double>(count, mi) : ens_layout<float>(count, mi);
  if (!workspace || bytes < L.total) {
    set_error("workspace has %llu bytes, needs %llu", (unsigned long long)bytes,
              (unsigned long long)L.total);
    return OC_ERR_ARG;
  }
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, workspace) != hipSuccess || attr.type != hipMemoryTypeDevice) {
    (void)hipGetLastError();
    set_error("workspace is not device memory");
    return OC_ERR_ARG;
  }
  oc_ensemble* e = new (std::nothrow) oc_ensemble;
  if (!e) { set_error("out of host memory"); return OC_ERR_ARG; }
  e->mem.assign(members, members + count);
  e->esz = esz;
  e->flags = flags;
  e->ws = (char*)workspace;
  e->ws_bytes = bytes;
  e->dmem = e->ws + L.dmem;
  e->items = (int2*)(e->ws + L.items);
  e->nitems = 0;
  e->max_items = mi;
  e->counter = (int*)(e->ws + L.counter);
  // classes: members with equal grids share the Poisson launches
  uint64_t soff = L.slots;
  for (int i = 0; i < count; ++i) {
    bool placed = false;
    for (auto& c : e->classes)
      if ((int)c.idx.size() < ENS_MAX_SLOTS && same_class(e->mem[c.idx[0]], e->mem[i])) {
        c.idx.push_back(i);
        placed = true;
        break;
      }
    if (!placed) {
      oc_ensemble::Class c;
      c.idx.push_back(i);
      for (int par = 0; par < 2; ++par) {
        c.slots[par] = (PoissonSlots*)(e->ws + soff);
        soff += align256(sizeof(PoissonSlots));
      }
      e->classes.push_back(c);
    }
  }
  e->cur0.resize(count);
  for (int i = 0; i < count; ++i) e->cur0[i] = members[i]->cur;
  e->phase = 0;
  e->table_dt = 1.0;
  e->have_graphs = false;
  e->graph_dt = 0.0;
  e->cap = nullptr;
  if (hipStreamCreateWithFlags(&e->cap, hipStreamNonBlocking) != hipSuccess) {
    set_error("capture stream creation failed");
    delete e;
    return OC_ERR_DEVICE;
  }
  rc = esz == 8 ? ens_setup<double>(e) : ens_setup<float>(e);
  if (rc) {
    (void)hipStreamDestroy(e->cap);
    delete e;
    return rc;
  }
  *out = e;
  return OC_OK;
}

int oc_ensemble_step(oc_ensemble* e, double dt, int32_t nsteps, void* stream) {
  if (!e) { set_error("ensemble is NULL"); return OC_ERR_ARG; }
  if (!(dt > 0) || !std::isfinite(dt) || nsteps < 0) {
    set_error("need dt > 0 and nsteps >= 0");
    return OC_ERR_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  return e->esz == 8 ? ens_step<double>(e, dt, nsteps, s) : ens_step<float>(e, dt, nsteps, s);
}

int oc_ensemble_tuning(const oc_ensemble* e, int32_t* out, double* ms) {
  if (!e || !out) { set_error("NULL argument"); return OC_ERR_ARG; }
  out[0] = e->tn.tile;
  out[1] = e->tn.persistent;
  out[2] = e->tn.nblocks;
  out[3] = e->tn.kc_div;
  out[4] = e->tuned;
  out[5] = e->nitems;
  if (ms) *ms = e->tune_ms;
  return OC_OK;
}

int oc_autotune(oc_ensemble* e, const char* cache_path) {
  if (!e) { set_error("ensemble is NULL"); return OC_ERR_ARG; }
  return e->esz == 8 ? ens_retune<double>(e, cache_path, nullptr)
                     : ens_retune<float>(e, cache_path, nullptr);
}

int oc_ensemble_set_tuning(oc_ensemble* e, const int32_t* tuning) {
  if (!e || !tuning) { set_error("NULL argument"); return OC_ERR_ARG; }
  EnsTuning t;
  t.tile = tuning[0];
  t.persistent = tuning[1];
  t.kc_div = tuning[2];
  t.nblocks = 0;
  if (t.tile < 0 || t.tile > 2 || (t.persistent != 0 && t.persistent != 1) || t.kc_div < 1) {
    set_error("need tile in 0..2, persistent 0 or 1 and kc_div >= 1");
    return OC_ERR_ARG;
  }
  for (const oc_model* m : e->mem)
    if (!tile_fits(m, t.tile)) {
      set_error("tile %d does not divide every member's nx and ny", t.tile);
      return OC_ERR_ARG;
    }
  return e->esz == 8 ? ens_retune<double>(e, nullptr, &t) : ens_retune<float>(e, nullptr, &t);
}

int oc_ensemble_destroy(oc_ensemble* e) {
  if (e) {
    drop_graphs(e);
    if (e->cap) (void)hipStreamDestroy(e->cap);
  }
  delete e;
  return OC_OK;
}

}  // extern "C"
