// C ABI of the MLP subgrid closure (declared in include/oc.h): workspace
// carving, parameter upload, and the forward / backward / Adam sequences
// built from the BF16 MFMA GEMM kernel of mlp.hip.
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "oc_internal.h"

using namespace oc;

#define OC_CHECK_HIP(expr)                                        \
  do {                                                            \
    hipError_t e_ = (expr);                                       \
    if (e_ != hipSuccess) {                                       \
      set_error("%s failed: %s", #expr, hipGetErrorString(e_));   \
      return OC_ERR_DEVICE;                                       \
    }                                                             \
  } while (0)

static const int LOSS_BLOCKS = 256;

struct oc_mlp {
  int max_batch;
  MlpParams p;
  float* m1;
  float* m2;
  float* grad;
  __bf16* xb;       // B x 512
  float* z1;        // B x 256 pre-activations
  __bf16* h1;       // B x 256
  float* z2;
  __bf16* h2;
  float* y;         // B x 4
  float* dy;        // B x 32
  __bf16* dyb;
  float* dz2;       // B x 256
  __bf16* dz2b;
  float* dz1;
  __bf16* dz1b;
  double* partial;  // LOSS_BLOCKS
  float* part;      // split-K and column-sum partials (MLP_PART_FLOATS)
  int step;
};

namespace {

struct MlpLayout {
  uint64_t master, m1, m2, grad, w1b, w2b, w2bt, w3b, xb, z1, h1, z2, h2, y, dy, dyb, dz2, dz2b, dz1,
      dz1b, partial, part, total;
};

uint64_t a256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

MlpLayout mlp_layout(int B) {
  MlpLayout L;
  uint64_t o = 0;
  auto take = [&](uint64_t bytes) { uint64_t r = o; o += a256(bytes); return r; };
  L.master = take((uint64_t)MLP_NPARAM * 4);
  L.m1 = take((uint64_t)MLP_NPARAM * 4);
  L.m2 = take((uint64_t)MLP_NPARAM * 4);
  L.grad = take((uint64_t)MLP_NPARAM * 4);
  L.w1b = take((uint64_t)MLP_NH * MLP_KIN * 2);
  L.w2b = take((uint64_t)MLP_NH * MLP_NH * 2);
  L.w2bt = take((uint64_t)MLP_NH * MLP_NH * 2);
  L.w3b = take((uint64_t)MLP_NOUTP * MLP_NH * 2);
  L.xb = take((uint64_t)B * MLP_KIN * 2);
  L.z1 = take((uint64_t)B * MLP_NH * 4);
  L.h1 = take((uint64_t)B * MLP_NH * 2);
  L.z2 = take((uint64_t)B * MLP_NH * 4);
  L.h2 = take((uint64_t)B * MLP_NH * 2);
  L.y = take((uint64_t)B * MLP_NOUT * 4);
  L.dy = take((uint64_t)B * MLP_NOUTP * 4);
  L.dyb = take((uint64_t)B * MLP_NOUTP * 2);
  L.dz2 = take((uint64_t)B * MLP_NH * 4);
  L.dz2b = take((uint64_t)B * MLP_NH * 2);
  L.dz1 = take((uint64_t)B * MLP_NH * 4);
  L.dz1b = take((uint64_t)B * MLP_NH * 2);
  L.partial = take((uint64_t)LOSS_BLOCKS * 8);
  L.part = take((uint64_t)MLP_PART_FLOATS * 4);
  L.total = o;
  return L;
}

GemmArgs gemm(const __bf16* A, int lda, int ta, const __bf16* B, int ldb, int tb, int M, int N,
              int K, int epi, float* C, int ldc, const float* bias = nullptr,
              const float* Z = nullptr, __bf16* Hh = nullptr, int ldh = 0) {
  GemmArgs g;
  g.A = A; g.lda = lda; g.transA = ta;
  g.B = B; g.ldb = ldb; g.transB = tb;
  g.M = M; g.N = N; g.K = K;
  g.epi = epi; g.C = C; g.ldc = ldc; g.bias = bias; g.Z = Z; g.H = Hh; g.ldh = ldh;
  g.ksplit = 1; g.part = nullptr;
  return g;
}

// A weight-gradient GEMM (K = batch) split over K until the grid has about
// 1024 workgroups, each split covering at least two 32-deep k blocks.
GemmArgs split_k(GemmArgs g, float* part) {
  const int tiles = ((g.M + 63) / 64) * ((g.N + 63) / 64);
  int ks = 1;
  while (tiles * ks < 1024 && ks < MLP_MAX_KSPLIT && g.K % (64 * ks * 2) == 0 &&
         (long)2 * ks * g.M * g.N <= MLP_PART_FLOATS)
    ks *= 2;
  g.ksplit = ks;
  g.part = part;
  return g;
}

int check_batch(const oc_mlp* m, int B) {
  if (!m) { set_error("mlp is NULL"); return OC_ERR_ARG; }
  if (B < 32 || B > m->max_batch || B % 32) {
    set_error("batch must be a multiple of 32 in [32, %d]", m->max_batch);
    return OC_ERR_ARG;
  }
  return OC_OK;
}

// forward pass on the BF16 features already in m->xb
int forward_from_xb(oc_mlp* m, int B, hipStream_t s) {
  const float* mp = m->p.master;
  OC_CHECK_HIP(launch_gemm_bf16(gemm(m->xb, MLP_KIN, 0, m->p.W1b, MLP_KIN, 1, B, MLP_NH, MLP_KIN,
                                     EPI_BIAS_GELU, m->z1, MLP_NH, mp + MLP_OFF_B1, nullptr, m->h1,
                                     MLP_NH), s));
  OC_CHECK_HIP(launch_gemm_bf16(gemm(m->h1, MLP_NH, 0, m->p.W2b, MLP_NH, 1, B, MLP_NH, MLP_NH,
                                     EPI_BIAS_GELU, m->z2, MLP_NH, mp + MLP_OFF_B2, nullptr, m->h2,
                                     MLP_NH), s));
  OC_CHECK_HIP(launch_gemm_bf16(gemm(m->h2, MLP_NH, 0, m->p.W3b, MLP_NH, 1, B, MLP_NOUT, MLP_NH,
                                     EPI_BIAS, m->y, MLP_NOUT, mp + MLP_OFF_B3), s));
  return OC_OK;
}

// gradients of the mean squared error into m->grad (packed like the
// parameters); the per-block squared-error partials into m->partial
int backward(oc_mlp* m, const float* target, int B, hipStream_t s) {
  float* g = m->grad;
  OC_CHECK_HIP(launch_loss_grad(m->y, MLP_NOUT, target, B, m->dy, m->dyb, MLP_NOUTP, m->partial,
                                LOSS_BLOCKS, s));
  // layer 3: dW3 = dY^T H2, db3 = colsum dY, dZ2 = (dY W3) * gelu'(Z2)
  OC_CHECK_HIP(launch_gemm_bf16(split_k(gemm(m->dyb, MLP_NOUTP, 1, m->h2, MLP_NH, 0, MLP_NOUT,
                                             MLP_NH, B, EPI_STORE, g + MLP_OFF_W3, MLP_NH),
                                        m->part), s));
  OC_CHECK_HIP(launch_colsum(m->dy, B, MLP_NOUT, MLP_NOUTP, g + MLP_OFF_B3, m->part, s));
  OC_CHECK_HIP(launch_gemm_bf16(gemm(m->dyb, MLP_NOUTP, 0, m->p.W3b, MLP_NH, 0, B, MLP_NH,
                                     MLP_NOUTP, EPI_GELU_BWD, m->dz2, MLP_NH, nullptr, m->z2,
                                     m->dz2b, MLP_NH), s));
  // layer 2
  OC_CHECK_HIP(launch_gemm_bf16(split_k(gemm(m->dz2b, MLP_NH, 1, m->h1, MLP_NH, 0, MLP_NH,
                                             MLP_NH, B, EPI_STORE, g + MLP_OFF_W2, MLP_NH),
                                        m->part), s));
  OC_CHECK_HIP(launch_colsum(m->dz2, B, MLP_NH, MLP_NH, g + MLP_OFF_B2, m->part, s));
  OC_CHECK_HIP(launch_gemm_bf16(gemm(m->dz2b, MLP_NH, 0, m->p.W2bT, MLP_NH, 1, B, MLP_NH, MLP_NH,
                                     EPI_GELU_BWD, m->dz1, MLP_NH, nullptr, m->z1, m->dz1b,
                                     MLP_NH), s));
  // layer 1
  OC_CHECK_HIP(launch_gemm_bf16(split_k(gemm(m->dz1b, MLP_NH, 1, m->xb, MLP_KIN, 0, MLP_NH,
                                             MLP_NIN, B, EPI_STORE, g + MLP_OFF_W1, MLP_NIN),
                                        m->part), s));
  OC_CHECK_HIP(launch_colsum(m->dz1, B, MLP_NH, MLP_NH, g + MLP_OFF_B1, m->part, s));
  return OC_OK;
}

int read_loss(oc_mlp* m, int B, double* loss, hipStream_t s) {
  if (!loss) return OC_OK;
  double part[LOSS_BLOCKS];
  OC_CHECK_HIP(hipMemcpyAsync(part, m->partial, sizeof(part), hipMemcpyDeviceToHost, s));
  OC_CHECK_HIP(hipStreamSynchronize(s));
  double acc = 0.0;
  for (int b = 0; b < LOSS_BLOCKS; ++b) acc += part[b];
  *loss = acc / ((double)B * MLP_NOUT);
  return OC_OK;
}

}  // namespace

namespace oc {

__bf16* mlp_input(oc_mlp* net) { return net->xb; }
const float* mlp_output(oc_mlp* net) { return net->y; }
float* mlp_output_rw(oc_mlp* net) { return net->y; }
const MlpParams& mlp_params(const oc_mlp* net) { return net->p; }
int mlp_max_batch(const oc_mlp* net) { return net->max_batch; }
int mlp_run_forward(oc_mlp* net, int batch, hipStream_t s) { return forward_from_xb(net, batch, s); }

int mlp_params_finite(oc_mlp* net, hipStream_t s) {
  std::vector<float> p(MLP_NPARAM);
  OC_CHECK_HIP(hipMemcpyAsync(p.data(), net->p.master, p.size() * 4, hipMemcpyDeviceToHost, s));
  OC_CHECK_HIP(hipStreamSynchronize(s));
  for (float x : p)
    if (!std::isfinite(x)) return 0;
  return 1;
}

}  // namespace oc

extern "C" {

int oc_mlp_workspace_size(int32_t max_batch, uint64_t* bytes) {
  if (!bytes || max_batch < 32 || max_batch % 32) {
    set_error("max_batch must be a positive multiple of 32");
    return OC_ERR_ARG;
  }
  *bytes = mlp_layout(max_batch).total;
  return OC_OK;
}

int oc_mlp_create(int32_t max_batch, void* workspace, uint64_t bytes, oc_mlp** out) {
  if (!out || !workspace || max_batch < 32 || max_batch % 32) {
    set_error("need a workspace, an output handle and max_batch a multiple of 32");
    return OC_ERR_ARG;
  }
  if ((uintptr_t)workspace % 256) { set_error("workspace must be 256-byte aligned"); return OC_ERR_ARG; }
  const MlpLayout L = mlp_layout(max_batch);
  if (bytes < L.total) {
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
  oc_mlp* m = new (std::nothrow) oc_mlp;
  if (!m) { set_error("out of host memory"); return OC_ERR_ARG; }
  char* w = (char*)workspace;
  m->max_batch = max_batch;
  m->p.master = (float*)(w + L.master);
  m->p.W1b = (__bf16*)(w + L.w1b);
  m->p.W2b = (__bf16*)(w + L.w2b);
  m->p.W2bT = (__bf16*)(w + L.w2bt);
  m->p.W3b = (__bf16*)(w + L.w3b);
  m->m1 = (float*)(w + L.m1);
  m->m2 = (float*)(w + L.m2);
  m->grad = (float*)(w + L.grad);
  m->xb = (__bf16*)(w + L.xb);
  m->z1 = (float*)(w + L.z1);
  m->h1 = (__bf16*)(w + L.h1);
  m->z2 = (float*)(w + L.z2);
  m->h2 = (__bf16*)(w + L.h2);
  m->y = (float*)(w + L.y);
  m->dy = (float*)(w + L.dy);
  m->dyb = (__bf16*)(w + L.dyb);
  m->dz2 = (float*)(w + L.dz2);
  m->dz2b = (__bf16*)(w + L.dz2b);
  m->dz1 = (float*)(w + L.dz1);
  m->dz1b = (__bf16*)(w + L.dz1b);
  m->partial = (double*)(w + L.partial);
  m->part = (float*)(w + L.part);
  m->step = 0;
  // zero everything: padded weight rows/columns stay zero for good
  if (hipMemset(workspace, 0, L.total) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    set_error("mlp setup failed");
    delete m;
    return OC_ERR_DEVICE;
  }
  *out = m;
  return OC_OK;
}

int oc_mlp_destroy(oc_mlp* m) {
  delete m;
  return OC_OK;
}

int oc_mlp_set_params(oc_mlp* m, const float* params, void* stream) {
  if (!m || !params) { set_error("NULL argument"); return OC_ERR_ARG; }
  for (int i = 0; i < MLP_NPARAM; ++i)
    if (!std::isfinite(params[i])) { set_error("parameter %d is not finite", i); return OC_ERR_NONFINITE; }
  hipStream_t s = (hipStream_t)stream;
  OC_CHECK_HIP(hipMemcpyAsync(m->p.master, params, (size_t)MLP_NPARAM * 4, hipMemcpyHostToDevice, s));
  OC_CHECK_HIP(launch_refresh_bf16(m->p, MLP_NPARAM, s));
  // a fresh optimiser state
  OC_CHECK_HIP(hipMemsetAsync(m->m1, 0, (size_t)MLP_NPARAM * 4, s));
  OC_CHECK_HIP(hipMemsetAsync(m->m2, 0, (size_t)MLP_NPARAM * 4, s));
  OC_CHECK_HIP(hipStreamSynchronize(s));
  m->step = 0;
  return OC_OK;
}

int oc_mlp_get_params(oc_mlp* m, float* params, void* stream) {
  if (!m || !params) { set_error("NULL argument"); return OC_ERR_ARG; }
  hipStream_t s = (hipStream_t)stream;
  OC_CHECK_HIP(hipMemcpyAsync(params, m->p.master, (size_t)MLP_NPARAM * 4, hipMemcpyDeviceToHost, s));
  OC_CHECK_HIP(hipStreamSynchronize(s));
  return OC_OK;
}

int oc_mlp_forward(oc_mlp* m, const float* x, int32_t batch, float* y, void* stream) {
  int rc = check_batch(m, batch);
  if (rc) return rc;
  if (!x || !y) { set_error("NULL argument"); return OC_ERR_ARG; }
  hipStream_t s = (hipStream_t)stream;
  OC_CHECK_HIP(launch_features_to_bf16(x, batch, m->xb, s));
  rc = forward_from_xb(m, batch, s);
  if (rc) return rc;
  OC_CHECK_HIP(hipMemcpyAsync(y, m->y, (size_t)batch * MLP_NOUT * 4, hipMemcpyDeviceToDevice, s));
  return OC_OK;
}

int oc_mlp_gradients(oc_mlp* m, const float* x, const float* target, int32_t batch, float* grad,
                     double* loss, void* stream) {
  int rc = check_batch(m, batch);
  if (rc) return rc;
  if (!x || !target || !grad) { set_error("NULL argument"); return OC_ERR_ARG; }
  hipStream_t s = (hipStream_t)stream;
  OC_CHECK_HIP(launch_features_to_bf16(x, batch, m->xb, s));
  rc = forward_from_xb(m, batch, s);
  if (rc) return rc;
  rc = backward(m, target, batch, s);
  if (rc) return rc;
  OC_CHECK_HIP(hipMemcpyAsync(grad, m->grad, (size_t)MLP_NPARAM * 4, hipMemcpyDeviceToDevice, s));
  return read_loss(m, batch, loss, s);
}

int oc_mlp_train_step(oc_mlp* m, const float* x, const float* target, int32_t batch, float lr,
                      double* loss, void* stream) {
  int rc = check_batch(m, batch);
  if (rc) return rc;
  if (!x || !target || !(lr > 0)) { set_error("need inputs, targets and lr > 0"); return OC_ERR_ARG; }
  hipStream_t s = (hipStream_t)stream;
  OC_CHECK_HIP(launch_features_to_bf16(x, batch, m->xb, s));
  rc = forward_from_xb(m, batch, s);
  if (rc) return rc;
  rc = backward(m, target, batch, s);
  if (rc) return rc;
  m->step += 1;
  OC_CHECK_HIP(launch_adam(m->p, m->grad, m->m1, m->m2, MLP_NPARAM, lr, m->step, s));
  return read_loss(m, batch, loss, s);
}

}  // extern "C"
