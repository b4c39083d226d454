// MLP subgrid closure on gfx950: BF16 MFMA GEMMs with FP32 accumulation
// for the forward and backward passes, fused bias/GELU epilogues, loss and
// bias-gradient reductions, Adam on FP32 master weights, and the gather of
// the standardised 5x5x5 (u, v, w, b) neighbourhood of every coarse cell.
//
// Network: 500 -> 256 -> 256 -> 4 with exact-erf GELU.  On the device the
// input width is padded to 512 and the output width to 32 with zero weights
// so every GEMM dimension is a multiple of the 32-deep MFMA k step.
#include "oc_internal.h"

namespace oc {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ void mlp_write_bf16(const MlpParams& p, int t, float w) {
  // master layout: W1 (256 x 500) | b1 | W2 (256 x 256) | b2 | W3 (4 x 256) | b3
  if (t < MLP_OFF_B1) {
    const int r = t / 500, c = t % 500;
    p.W1b[r * 512 + c] = (__bf16)w;
  } else if (t >= MLP_OFF_W2 && t < MLP_OFF_B2) {
    const int r = (t - MLP_OFF_W2) / MLP_NH, c = (t - MLP_OFF_W2) % MLP_NH;
    p.W2b[r * MLP_NH + c] = (__bf16)w;
    p.W2bT[c * MLP_NH + r] = (__bf16)w;   // transposed copy for the backward pass
  } else if (t >= MLP_OFF_W3 && t < MLP_OFF_B3) {
    p.W3b[t - MLP_OFF_W3] = (__bf16)w;
  }
}


namespace {

constexpr int BM = 64, BN = 64, BK = 32, LDP = BK + 8;  // LDS rows padded by 8 bf16

// erf(z / sqrt 2) and exp(-z^2 / 2) by Abramowitz & Stegun, formula 7.1.26
// (absolute error of erf at most 1.5e-7, far below the BF16 rounding the
// activations get next): for x >= 0, erf x = 1 - t P(t) exp(-x^2),
// t = 1 / (1 + p x), P a quartic; erf is odd.  About a dozen full-rate
// instructions, a reciprocal and an exponential: the activation epilogues
// are the bulk of the fused kernel's vector instructions.
struct ErfGauss {
  float erf, g;
};
__device__ inline ErfGauss erf_gauss(float z) {
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f * 0.70710678118654752f, fabsf(z), 1.0f));
  float q = fmaf(1.061405429f, t, -1.453152027f);
  q = fmaf(q, t, 1.421413741f);
  q = fmaf(q, t, -0.284496736f);
  q = fmaf(q, t, 0.254829592f);
  const float g = __builtin_amdgcn_exp2f(z * z * (-0.5f * 1.44269504088896341f));
  return {copysignf(fmaf(-(q * t), g, 1.0f), z), g};
}
// erf(z / sqrt 2) alone by Abramowitz & Stegun, formula 7.1.28 (absolute
// error at most 3e-7): for x >= 0, erf x = 1 - (1 + a1 x + ... + a6 x^6)^-16,
// here with the 1/sqrt 2 folded into the coefficients.  One reciprocal and
// no exponential.
__device__ inline float erf_sqrt2(float z) {
  const float az = fabsf(z);
  float q = fmaf(0.0000430638f / 8.0f, az, 0.0002765672f / 5.65685424949238f);
  q = fmaf(q, az, 0.0001520143f / 4.0f);
  q = fmaf(q, az, 0.0092705272f / 2.82842712474619f);
  q = fmaf(q, az, 0.0422820123f / 2.0f);
  q = fmaf(q, az, 0.0705230784f / 1.41421356237310f);
  float r = __builtin_amdgcn_rcpf(fmaf(q, az, 1.0f));
  r *= r;
  r *= r;
  r *= r;
  r *= r;
  return copysignf(1.0f - r, z);
}
// exact-erf GELU, z Phi(z), and its derivative
__device__ inline float gelu(float z) {
  const float h = 0.5f * z;
  return fmaf(h, erf_sqrt2(z), h);
}
__device__ inline float gelu_prime(float z) {
  const ErfGauss r = erf_gauss(z);
  return fmaf(0.5f, r.erf, 0.5f) + z * r.g * 0.39894228040143268f;
}

// Epilogue of one output element (m, n) of a GEMM.
__device__ inline void epilogue(const GemmArgs& g, int m, int n, float v) {
  const long o = (long)m * g.ldc + n;
  switch (g.epi) {
    case EPI_STORE:
      g.C[o] = v;
      break;
    case EPI_BIAS:
      g.C[o] = v + g.bias[n];
      break;
    case EPI_BIAS_GELU: {
      const float z = v + g.bias[n];
      g.C[o] = z;                                   // pre-activation (for backward)
      g.H[(long)m * g.ldh + n] = (__bf16)gelu(z);    // activation (next layer)
      break;
    }
    case EPI_GELU_BWD: {
      const float dz = v * gelu_prime(g.Z[o]);
      g.C[o] = dz;
      g.H[(long)m * g.ldh + n] = (__bf16)dz;
      break;
    }
  }
}

// C[m][n] = sum_k A[m][k] B[k][n].  transA = 0: A[m][k] at A[m*lda + k];
// 1: at A[k*lda + m].  transB = 0: B[k][n] at B[k*ldb + n]; 1: at B[n*ldb + k].
// Tiles are staged in LDS with k contiguous, the order the MFMA operands
// need: lane l holds 8 consecutive k of row (or column) l % 16, k block l / 16.
__global__ void __launch_bounds__(256) gemm_bf16_kernel(GemmArgs g) {
  __shared__ __bf16 As[BM][LDP];
  __shared__ __bf16 Bs[BN][LDP];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  // split K: this workgroup's range of the reduction
  const int kspan = g.K / g.ksplit;
  const int kbeg = blockIdx.z * kspan, kend = kbeg + kspan;
  f32x4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    // ---- stage A (BM x BK) and B (BN x BK)
    if (!g.transA) {
      const int r = tid >> 2, ks = (tid & 3) * 8;
      const int m = m0 + r;
      bf16x8 v;
      if (m < g.M) v = *(const bf16x8*)(g.A + (long)m * g.lda + k0 + ks);
      else for (int e = 0; e < 8; ++e) v[e] = (__bf16)0.0f;
      *(bf16x8*)&As[r][ks] = v;
    } else {
      const int kk = tid >> 3, ms = (tid & 7) * 8;
      const __bf16* src = g.A + (long)(k0 + kk) * g.lda + m0 + ms;
      for (int e = 0; e < 8; ++e) As[ms + e][kk] = (m0 + ms + e < g.M) ? src[e] : (__bf16)0.0f;
    }
    if (g.transB) {
      const int r = tid >> 2, ks = (tid & 3) * 8;
      const int n = n0 + r;
      bf16x8 v;
      if (n < g.N) v = *(const bf16x8*)(g.B + (long)n * g.ldb + k0 + ks);
      else for (int e = 0; e < 8; ++e) v[e] = (__bf16)0.0f;
      *(bf16x8*)&Bs[r][ks] = v;
    } else {
      const int kk = tid >> 3, ns = (tid & 7) * 8;
      const __bf16* src = g.B + (long)(k0 + kk) * g.ldb + n0 + ns;
      for (int e = 0; e < 8; ++e) Bs[ns + e][kk] = (n0 + ns + e < g.N) ? src[e] : (__bf16)0.0f;
    }
    __syncthreads();
    // ---- 2 x 2 MFMA tiles of 16 x 16 per wave
    bf16x8 a[2], b[2];
    for (int i = 0; i < 2; ++i)
      a[i] = *(const bf16x8*)&As[wm * 32 + i * 16 + (lane & 15)][8 * (lane >> 4)];
    for (int j = 0; j < 2; ++j)
      b[j] = *(const bf16x8*)&Bs[wn * 32 + j * 16 + (lane & 15)][8 * (lane >> 4)];
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }

  // ---- epilogue: lane holds rows 4*(lane/16) + e of column lane % 16
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + wn * 32 + j * 16 + (lane & 15);
      if (n >= g.N) continue;
      for (int e = 0; e < 4; ++e) {
        const int m = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + e;
        if (m >= g.M) continue;
        const float v = acc[i][j][e];
        if (g.ksplit > 1) {
          g.part[((long)blockIdx.z * g.M + m) * g.N + n] = v;
          continue;
        }
        epilogue(g, m, n, v);
      }
    }
}

// dY = 2 (Y - T) / (B * 4) on the 4 real outputs (FP32 and BF16, padded
// columns zero); per-block partial sums of the squared error.
// C = A B with both operands k-contiguous (A[m][k] at A[m*lda + k], B[k][n]
// at B[n*ldb + k]), M any multiple of 32, N a multiple of 128, K a multiple
// of 64.  Workgroup tile 128 x 128, k step 64, four waves of 64 x 64 (4 x 4
// MFMA 16x16x32 tiles); 16-byte global loads into registers for the next
// k step while the current one is multiplied out of double-buffered LDS.
constexpr int NT_BM = 128, NT_BN = 128, NT_BK = 64, NT_LDP = NT_BK + 8;

__global__ void __launch_bounds__(256) gemm_bf16_nt_kernel(GemmArgs g) {
  __shared__ __bf16 As[2][NT_BM][NT_LDP];
  __shared__ __bf16 Bs[2][NT_BN][NT_LDP];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  const int m0 = blockIdx.y * NT_BM, n0 = blockIdx.x * NT_BN;
  // each thread moves 4 chunks of 8 bf16 per operand and k step: rows
  // (tid >> 3) + 32 c, k offset 8 (tid & 7)
  const int lr = tid >> 3, lk = (tid & 7) * 8;
  bf16x8 ra[4], rb[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int m = m0 + lr + 32 * c;
      if (m < g.M) ra[c] = *(const bf16x8*)(g.A + (long)m * g.lda + k0 + lk);
      else for (int e = 0; e < 8; ++e) ra[c][e] = (__bf16)0.0f;
      const int n = n0 + lr + 32 * c;
      rb[c] = *(const bf16x8*)(g.B + (long)n * g.ldb + k0 + lk);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      *(bf16x8*)&As[buf][lr + 32 * c][lk] = ra[c];
      *(bf16x8*)&Bs[buf][lr + 32 * c][lk] = rb[c];
    }
  };
  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int nk = g.K / NT_BK;
  load(0);
  stash(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) load((kt + 1) * NT_BK);
#pragma unroll
    for (int ks = 0; ks < NT_BK; ks += 32) {
      bf16x8 a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        a[i] = *(const bf16x8*)&As[buf][wm * 64 + i * 16 + (lane & 15)][ks + 8 * (lane >> 4)];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        b[j] = *(const bf16x8*)&Bs[buf][wn * 64 + j * 16 + (lane & 15)][ks + 8 * (lane >> 4)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < nk) stash(buf ^ 1);
    __syncthreads();
  }
  // lane holds rows 4 (lane / 16) + e of column lane % 16 of each 16 x 16 tile
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + wn * 64 + j * 16 + (lane & 15);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + e;
        if (m < g.M) epilogue(g, m, n, acc[i][j][e]);
      }
    }
}

__global__ void __launch_bounds__(256) loss_grad_kernel(const float* Y, int ldy, const float* T,
                                                        int B, float* dY, __bf16* dYb, int ldd,
                                                        double* partial) {
  __shared__ double red[256];
  double acc = 0.0;
  const float scale = 2.0f / (float)(B * 4);
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < (long)B * ldd;
       t += (long)gridDim.x * blockDim.x) {
    const int r = (int)(t / ldd), c = (int)(t % ldd);
    float d = 0.f;
    if (c < 4) {
      const float e = Y[(long)r * ldy + c] - T[(long)r * 4 + c];
      acc += (double)e * e;
      d = scale * e;
    }
    dY[t] = d;
    dYb[t] = (__bf16)d;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// column sums of a (rows x cols) FP32 matrix into out (bias gradients)
// Sum of the split-K partials in z order: C[m][n] = sum_z part[z][m][n].
__global__ void splitk_reduce_kernel(const float* part, int ksplit, int M, int N, float* C,
                                     int ldc) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)M * N) return;
  const long mn = (long)M * N;
  float s = 0.f;
  for (int z = 0; z < ksplit; ++z) s += part[z * mn + t];
  C[(t / N) * ldc + t % N] = s;
}

// Column sums in two levels: chunk q of the rows gives part[q][c] (a block
// of 64 columns x 4 row lanes, combined in LDS), then the chunks are added
// in order.
__global__ void __launch_bounds__(256) colsum_partial_kernel(const float* a, int rows, int cols,
                                                             int lda, int chunk, float* part) {
  __shared__ float red[4][64];
  const int cl = threadIdx.x & 63, rl = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + cl;
  const int r0 = blockIdx.y * chunk, r1 = min(r0 + chunk, rows);
  float s = 0.f;
  if (c < cols)
    for (int r = r0 + rl; r < r1; r += 4) s += a[(long)r * lda + c];
  red[rl][cl] = s;
  __syncthreads();
  if (rl == 0 && c < cols)
    part[(long)blockIdx.y * cols + c] = ((red[0][cl] + red[1][cl]) + red[2][cl]) + red[3][cl];
}

__global__ void colsum_final_kernel(const float* part, int nchunk, int cols, float* out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  float s = 0.f;
  for (int q = 0; q < nchunk; ++q) s += part[(long)q * cols + c];
  out[c] = s;
}

// FP32 features (B x 500) -> BF16 (B x 512), zero padding
__global__ void features_to_bf16_kernel(const float* x, int B, __bf16* xb) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)B * 512) return;
  const int r = (int)(t / 512), c = (int)(t % 512);
  xb[t] = (c < 500) ? (__bf16)x[(long)r * 500 + c] : (__bf16)0.0f;
}

// Adam (Kingma & Ba) on the FP32 master parameters; refreshes the padded
// BF16 copies used by the GEMMs.
__global__ void adam_kernel(MlpParams p, const float* grad, float* m1, float* m2, int n,
                            float lr, float b1, float b2, float eps, float c1, float c2) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float g = grad[t];
  const float mm = b1 * m1[t] + (1.f - b1) * g;
  const float vv = b2 * m2[t] + (1.f - b2) * g * g;
  m1[t] = mm;
  m2[t] = vv;
  const float w = p.master[t] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  p.master[t] = w;
  mlp_write_bf16(p, t, w);
}

__global__ void refresh_bf16_kernel(MlpParams p, int n) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) mlp_write_bf16(p, t, p.master[t]);
}

}  // namespace

hipError_t launch_gemm_bf16(const GemmArgs& g, hipStream_t s) {
  const int ks = g.ksplit > 1 ? g.ksplit : 1;
  if (ks > 1 && (g.epi != EPI_STORE || g.K % (ks * BK) || !g.part ||
                 (long)ks * g.M * g.N > MLP_PART_FLOATS))
    return hipErrorInvalidValue;
  GemmArgs a = g;
  a.ksplit = ks;
  if (ks == 1 && !g.transA && g.transB && g.N % NT_BN == 0 && g.K % NT_BK == 0) {
    dim3 grid(g.N / NT_BN, (g.M + NT_BM - 1) / NT_BM);
    hipLaunchKernelGGL(gemm_bf16_nt_kernel, grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  dim3 grid((g.N + BN - 1) / BN, (g.M + BM - 1) / BM, ks);
  hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(256), 0, s, a);
  if (ks > 1) {
    const long n = (long)g.M * g.N;
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       g.part, ks, g.M, g.N, g.C, g.ldc);
  }
  return hipGetLastError();
}

hipError_t launch_loss_grad(const float* Y, int ldy, const float* T, int B, float* dY, __bf16* dYb,
                            int ldd, double* partial, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(loss_grad_kernel, dim3(nblocks), dim3(256), 0, s, Y, ldy, T, B, dY, dYb, ldd,
                     partial);
  return hipGetLastError();
}

hipError_t launch_colsum(const float* a, int rows, int cols, int lda, float* out, float* part,
                         hipStream_t s) {
  int chunk = 128;
  while ((rows + chunk - 1) / chunk > COLSUM_MAX_CHUNKS) chunk *= 2;
  const int nchunk = (rows + chunk - 1) / chunk;
  hipLaunchKernelGGL(colsum_partial_kernel, dim3((cols + 63) / 64, nchunk), dim3(256), 0, s, a,
                     rows, cols, lda, chunk, part);
  hipLaunchKernelGGL(colsum_final_kernel, dim3((cols + 127) / 128), dim3(128), 0, s, part, nchunk,
                     cols, out);
  return hipGetLastError();
}

hipError_t launch_features_to_bf16(const float* x, int B, __bf16* xb, hipStream_t s) {
  const long n = (long)B * 512;
  hipLaunchKernelGGL(features_to_bf16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     x, B, xb);
  return hipGetLastError();
}

hipError_t launch_adam(const MlpParams& p, const float* grad, float* m1, float* m2, int n, float lr,
                       int step, hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, grad, m1, m2, n, lr,
                     b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_refresh_bf16(const MlpParams& p, int n, hipStream_t s) {
  hipLaunchKernelGGL(refresh_bf16_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Closure inside the model: features from the halo-padded state, and the
// conservative flux divergence of the predicted vertical fluxes.
// ---------------------------------------------------------------------------

// xb[cell][f], f = var * 125 + (dk+2)*25 + (dj+2)*5 + (di+2), var = u, v, w, b
// Standardised input f (0..499) of the cell `cell`: variable f / 125 of
// (u, v, w, b) at offset (dk, dj, di) = digits of f % 125 in base 5, minus 2.
template <class T>
__device__ inline float feature_value(const Dims& d, const T* u, const T* v, const T* w,
                                      const T* tt, const T* ss, const ClosureStats& st, long cell,
                                      int f) {
  const int i = (int)(cell % d.nx);
  const int j = (int)((cell / d.nx) % d.ny);
  const int k = (int)(cell / ((long)d.nx * d.ny));
  const int var = f / 125, o = f % 125;
  const int dk = o / 25 - 2, dj = (o / 5) % 5 - 2, di = o % 5 - 2;
  const long p = pidx(d, i + di, j + dj, k + dk);
  float x;
  if (var == 0) x = (float)u[p];
  else if (var == 1) x = (float)v[p];
  else if (var == 2) x = (float)w[p];
  else x = st.g_alpha * ((float)tt[p] - st.t_ref) - st.g_beta * ((float)ss[p] - st.s_ref);
  return (x - st.in_mean[var]) / st.in_std[var];
}

// BF16 rows of 512 (the GEMM's padded K) for the model's own closure.
template <class T>
__global__ void __launch_bounds__(256) closure_features_kernel(Dims d, const T* u, const T* v,
                                                               const T* w, const T* tt,
                                                               const T* ss, ClosureStats st,
                                                               __bf16* xb) {
  const long ncell = (long)d.nx * d.ny * d.nz;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ncell * 512) return;
  const long cell = t >> 9;
  const int f = (int)(t & 511);
  xb[t] = (f < 500) ? (__bf16)feature_value(d, u, v, w, tt, ss, st, cell, f) : (__bf16)0.0f;
}

// The closure network on every cell of a model, fused.  A workgroup (4
// waves) takes 64 consecutive cells, gathers their standardised 5x5x5
// (u, v, w, b) neighbourhoods 64 features at a time (im2col: the walk over
// (variable, offset) is uniform per wave and runs on the scalar unit) and
// multiplies them by W1 with MFMA.  The 64 x 256 activations stay in LDS as
// the A operand of the second layer; the third layer is one MFMA column
// block (outputs padded to 16).  The next k chunk's features and weights are
// loaded into registers while the current one is multiplied.  Only y (4 per
// cell) goes to memory.  Operand rounding matches the unfused path: BF16
// inputs, weights and activations, FP32 accumulation.
constexpr int FZ_BM = 64, FZ_BK = 64, FZ_LDP = FZ_BK + 8, FZ_HP = MLP_NH + 8;

template <class T>
__global__ void __launch_bounds__(256) closure_mlp_fused_kernel(Dims d, const T* u, const T* v,
                                                               const T* w, const T* tt,
                                                               const T* ss, ClosureStats st,
                                                               MlpParams p, float* y) {
  __shared__ __bf16 Ws[MLP_NH][FZ_LDP];      // weight chunk, rows = outputs
  __shared__ __bf16 Hs[FZ_BM][FZ_HP];        // layer activations; layer 1 uses its
                                             // first FZ_LDP columns for the features
  const long ncell = (long)d.nx * d.ny * d.nz;
  const long c0 = (long)blockIdx.x * FZ_BM;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;   // wave wv: output columns [64 wv, +64)
  const float* b1 = p.master + MLP_OFF_B1;
  const float* b2 = p.master + MLP_OFF_B2;
  const float* b3 = p.master + MLP_OFF_B3;

  f32x4 acc[4][4];
  auto zero = [&]() {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  };
  // acc += A[64 rows][ka .. ka + 64) * Ws^T (A = Hs, pitch FZ_HP)
  auto mma = [&](int ka) {
#pragma unroll
    for (int ks = 0; ks < FZ_BK; ks += 32) {
      bf16x8 a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        a[i] = *(const bf16x8*)&Hs[i * 16 + (lane & 15)][ka + ks + 8 * (lane >> 4)];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        b[j] = *(const bf16x8*)&Ws[wv * 64 + j * 16 + (lane & 15)][ks + 8 * (lane >> 4)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  };
  // weight chunk in registers: rows (tid >> 3) + 32 c, k offset 8 (tid & 7)
  bf16x8 wreg[8];
  auto load_w = [&](const __bf16* W, int ldw, int k0) {
#pragma unroll
    for (int c = 0; c < 8; ++c)
      wreg[c] = *(const bf16x8*)(W + (long)((tid >> 3) + 32 * c) * ldw + k0 + (tid & 7) * 8);
  };
  auto stash_w = [&]() {
#pragma unroll
    for (int c = 0; c < 8; ++c) *(bf16x8*)&Ws[(tid >> 3) + 32 * c][(tid & 7) * 8] = wreg[c];
  };
  auto store_h = [&](const float* bias) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int n = wv * 64 + j * 16 + (lane & 15);
        const float bn = bias[n];
#pragma unroll
        for (int e = 0; e < 4; ++e)
          Hs[i * 16 + 4 * (lane >> 4) + e][n] = (__bf16)gelu(acc[i][j][e] + bn);
      }
  };

  // ---- gather: cell gc (lane), features gf .. gf + 15 (gf uniform per wave)
  const int gc = lane;
  const int gf = __builtin_amdgcn_readfirstlane(wv * 16);
  const long cell = c0 + gc;
  const bool live = cell < ncell;
  int corner = 0;   // padded offset of the neighbourhood corner (i-2, j-2, k-2)
  if (live) {
    const int ci = (int)(cell % d.nx);
    const int cj = (int)((cell / d.nx) % d.ny);
    const int ck = (int)(cell / ((long)d.nx * d.ny));
    corner = (int)pidx(d, ci - 2, cj - 2, ck - 2);
  }
  const int sy = (int)d.sy, sz = (int)d.sz;
  float graw[16], sraw[16];
  bf16x8 xreg[2];
  auto gather_load = [&](int k0) {
    int f = k0 + gf;   // uniform: the walk below is scalar
    int var = f / 125, o = f - var * 125;
    int dk = o / 25, dj = (o - dk * 25) / 5, di = o - dk * 25 - dj * 5;
#pragma unroll
    for (int q = 0; q < 16; ++q, ++f) {
      const int off = dk * sz + dj * sy + di;
      graw[q] = 0.f;
      sraw[q] = 0.f;
      if (f < MLP_NIN) {
        if (var == 0) graw[q] = (float)u[corner + off];
        else if (var == 1) graw[q] = (float)v[corner + off];
        else if (var == 2) graw[q] = (float)w[corner + off];
        else { graw[q] = (float)tt[corner + off]; sraw[q] = (float)ss[corner + off]; }
      }
      if (++di == 5) { di = 0; if (++dj == 5) { dj = 0; if (++dk == 5) { dk = 0; ++var; } } }
    }
  };
  auto gather_convert = [&](int k0) {
    int f = k0 + gf;
    int var = f / 125;
    int o = f - var * 125;
#pragma unroll
    for (int q = 0; q < 16; ++q, ++f) {
      const int vq = var < 4 ? var : 3;
      const float raw = vq == 3 ? st.g_alpha * (graw[q] - st.t_ref) - st.g_beta * (sraw[q] - st.s_ref)
                                : graw[q];
      const float x = (live && f < MLP_NIN) ? (raw - st.in_mean[vq]) * st.in_rstd[vq] : 0.f;
      xreg[q >> 3][q & 7] = (__bf16)x;
      if (++o == 125) { o = 0; ++var; }
    }
  };

  // ---- layer 1: 8 chunks of 64 features (500 real, zero padding to 512),
  // staged in the first FZ_BK columns of Hs
  zero();
  gather_load(0);
  gather_convert(0);
  load_w(p.W1b, MLP_KIN, 0);
  for (int k0 = 0; k0 < MLP_KIN; k0 += FZ_BK) {
    *(bf16x8*)&Hs[gc][gf] = xreg[0];
    *(bf16x8*)&Hs[gc][gf + 8] = xreg[1];
    stash_w();
    __syncthreads();
    const bool more = k0 + FZ_BK < MLP_KIN;
    if (more) {                   // next chunk's loads in flight during the multiply
      gather_load(k0 + FZ_BK);
      load_w(p.W1b, MLP_KIN, k0 + FZ_BK);
    }
    mma(0);
    if (more) gather_convert(k0 + FZ_BK);
    __syncthreads();
  }
  store_h(b1);

  // ---- layer 2: A = the layer-1 activations in Hs, 4 chunks of W2
  zero();
  load_w(p.W2b, MLP_NH, 0);
  for (int k0 = 0; k0 < MLP_NH; k0 += FZ_BK) {
    stash_w();
    __syncthreads();    // (first chunk: also orders the Hs writes above)
    if (k0 + FZ_BK < MLP_NH) load_w(p.W2b, MLP_NH, k0 + FZ_BK);
    mma(k0);
    __syncthreads();
  }
  store_h(b2);          // every wave has finished reading Hs (barrier above)
  __syncthreads();

  // ---- layer 3: wave wv takes rows [16 wv, +16) against W3 rows 0..15
  // (rows >= 4 are zero): 8 MFMAs over k
  {
    f32x4 c3 = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < MLP_NH; ks += 32) {
      const bf16x8 a = *(const bf16x8*)&Hs[wv * 16 + (lane & 15)][ks + 8 * (lane >> 4)];
      const bf16x8 b = *(const bf16x8*)(p.W3b + (long)(lane & 15) * MLP_NH + ks + 8 * (lane >> 4));
      c3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c3, 0, 0, 0);
    }
    const int o = lane & 15;
    if (o < MLP_NOUT)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const long c = c0 + wv * 16 + 4 * (lane >> 4) + e;
        if (c < ncell) y[c * MLP_NOUT + o] = c3[e] + b3[o];
      }
  }
}

// The same network for grids whose x rows hold a multiple of 64 cells: the
// 64 cells of a workgroup share one x row, so the standardised BF16 values
// of (u, v, w, b) over their whole 5 x 5 x 68 neighbourhood region are
// loaded once (coalesced along x) into LDS, and every 32-deep k chunk of
// features is copied out of that region (im2col in LDS, double-buffered
// column blocks, one barrier per chunk).  Each wave's B operands (its 64
// output rows of the weights, k contiguous) go from global memory (L2)
// straight into registers in the MFMA operand layout, RG_D chunks ahead of
// their use: no weight staging in LDS, and the second layer runs without
// barriers.  The weight prefetch crosses from the first layer into the
// second.
constexpr int RG_X = FZ_BM + 4, RG_P = RG_X + 4, RG_D = 2;
constexpr int RG_S1 = MLP_KIN / 32, RG_S2 = MLP_NH / 32;   // k chunks per layer
constexpr int RG_ROWS = 4 * 25 + 1;                         // + a row of zeros
// k chunks of features staged per barrier (two blocks alternate in the
// first 4 RG_BLK 32 columns of the activation buffer): 16 -> 8 barriers
// per layer, 0.259 -> 0.252 ms per substage at 64^3; four chunks per
// barrier measured 0.256 ms
constexpr int RG_BLK = 2;
static_assert(2 * RG_BLK * 32 <= MLP_NH && RG_S1 % RG_BLK == 0, "staging blocks");

// Element offset in the region buffer of input feature f: variable f / 125
// (u, v, w, b), row 25 var + 5 dk + dj and column di, where (dk, dj, di) are
// the base-5 digits of f % 125; the padding features past the 500 inputs
// read the row of zeros.
struct RgOffsets {
  unsigned short v[MLP_KIN];
};
constexpr RgOffsets make_rg_offsets() {
  RgOffsets t{};
  for (int f = 0; f < MLP_KIN; ++f) {
    if (f >= MLP_NIN) {
      t.v[f] = (unsigned short)((RG_ROWS - 1) * RG_P);
      continue;
    }
    const int var = f / 125, o = f % 125;
    t.v[f] = (unsigned short)((var * 25 + o / 5) * RG_P + o % 5);
  }
  return t;
}
__constant__ RgOffsets kRgOff = make_rg_offsets();

template <class T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
closure_mlp_region_kernel(Dims d, const T* u, const T* v,
                                                                const T* w, const T* tt,
                                                                const T* ss, ClosureStats st,
                                                                MlpParams p, float* y) {
  __shared__ __bf16 Rg[RG_ROWS][RG_P];       // (25 var + 5 dk + dj, x - (i0 - 2)); zero row
  __shared__ __bf16 Hs[FZ_BM][FZ_HP];        // activations; layer 1 stages features here
  const long c0 = (long)blockIdx.x * FZ_BM;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int i0 = (int)(c0 % d.nx);
  const int j0 = (int)((c0 / d.nx) % d.ny);
  const int k0c = (int)(c0 / ((long)d.nx * d.ny));
  const float* b1 = p.master + MLP_OFF_B1;
  const float* b2 = p.master + MLP_OFF_B2;
  const float* b3 = p.master + MLP_OFF_B3;

  // this wave's B operands of k chunk s (s < RG_S1: W1; then W2): lane
  // holds 8 consecutive k of output row wv 64 + 16 j + lane % 16
  auto load_b = [&](int s, bf16x8* b) {
    const bool l1 = s < RG_S1;
    const __bf16* W = l1 ? p.W1b : p.W2b;
    const int ldw = l1 ? MLP_KIN : MLP_NH;
    const int kk = (l1 ? s : s - RG_S1) * 32;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      b[j] = *(const __attribute__((address_space(1))) bf16x8*)(
          W + (long)(wv * 64 + j * 16 + (lane & 15)) * ldw + kk + 8 * (lane >> 4));
  };
  bf16x8 wb[RG_D][4];
#pragma unroll
  for (int s = 0; s < RG_D; ++s) load_b(s, wb[s]);

  // ---- the neighbourhood region, standardised, in BF16 (compile-time trip
  // count: every load of the region is in flight before the first is used)
#pragma unroll
  for (int q = 0; q < (25 * RG_X + 255) / 256; ++q) {
    const int e = tid + q * 256;
    if (e >= 25 * RG_X) break;
    const int row = e / RG_X, x = e - row * RG_X;
    const int dk = row / 5, dj = row - dk * 5;
    const long pp = pidx(d, i0 - 2 + x, j0 - 2 + dj, k0c - 2 + dk);
    Rg[row][x] = (__bf16)(((float)u[pp] - st.in_mean[0]) * st.in_rstd[0]);
    Rg[25 + row][x] = (__bf16)(((float)v[pp] - st.in_mean[1]) * st.in_rstd[1]);
    Rg[50 + row][x] = (__bf16)(((float)w[pp] - st.in_mean[2]) * st.in_rstd[2]);
    const float b = st.g_alpha * ((float)tt[pp] - st.t_ref) - st.g_beta * ((float)ss[pp] - st.s_ref);
    Rg[75 + row][x] = (__bf16)((b - st.in_mean[3]) * st.in_rstd[3]);
  }
  if (tid < RG_P) Rg[RG_ROWS - 1][tid] = (__bf16)0.0f;

  f32x4 acc[4][4];
  auto zero = [&]() {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  };
  // one 32-deep k chunk, computed transposed: C^T = W H^T, weights (from
  // registers) as the first operand and the cells' features or
  // activations (Hs columns [ka, ka + 32)) as the second, so that a lane's
  // four results are four consecutive outputs of one cell
  auto mma = [&](int ka, const bf16x8* b) {
    bf16x8 a[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
      a[i] = *(const bf16x8*)&Hs[i * 16 + (lane & 15)][ka + 8 * (lane >> 4)];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[j], a[i], acc[i][j], 0, 0, 0);
  };
  // acc[i][j][e]: cell 16 i + lane % 16, output wv 64 + 16 j + 4 (lane / 16) + e
  auto store_h = [&](const float* bias) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = wv * 64 + j * 16 + 4 * (lane >> 4);
      const f32x4 bn = *(const __attribute__((address_space(1))) f32x4*)(bias + n);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        bf16x4 h;
#pragma unroll
        for (int e = 0; e < 4; ++e) h[e] = (__bf16)gelu(acc[i][j][e] + bn[e]);
        *(bf16x4*)&Hs[i * 16 + (lane & 15)][n] = h;
      }
    }
  };
  // features [kk, kk + 32) of cell `lane`: wave wv writes features kk + 8 wv .. + 7
  auto stage_x = [&](int kk) {
    const int f0 = __builtin_amdgcn_readfirstlane(kk + 8 * wv);
    const __bf16* rg = &Rg[0][0] + lane;
    bf16x8 xv;
#pragma unroll
    for (int q = 0; q < 8; ++q) xv[q] = rg[kRgOff.v[f0 + q]];
    *(bf16x8*)&Hs[lane][kk % (2 * RG_BLK * 32) + 8 * wv] = xv;
  };

  // ---- layer 1: 16 chunks of 32 features in blocks of RG_BLK chunks, one
  // barrier per block.  Block b is staged in half b % 2 of the first
  // 2 RG_BLK 32 columns of Hs.  A wave writes a half only after the barrier
  // of the block in between, which every wave reaches after its products
  // of the block that last read the half.
  zero();
  __syncthreads();                  // the region is complete
#pragma unroll
  for (int s0 = 0; s0 < RG_S1; s0 += RG_BLK) {
#pragma unroll
    for (int q = 0; q < RG_BLK; ++q) stage_x((s0 + q) * 32);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RG_BLK; ++q) {
      const int s = s0 + q;
      mma((s * 32) % (2 * RG_BLK * 32), wb[s % RG_D]);
      if (s + RG_D < RG_S1 + RG_S2) load_b(s + RG_D, wb[s % RG_D]);
    }
  }
  __syncthreads();                  // every wave's last feature reads are done
  store_h(b1);
  __syncthreads();

  // ---- layer 2: A = the activations in Hs, no barriers
  zero();
#pragma unroll
  for (int s = RG_S1; s < RG_S1 + RG_S2; ++s) {
    mma((s - RG_S1) * 32, wb[s % RG_D]);
    if (s + RG_D < RG_S1 + RG_S2) load_b(s + RG_D, wb[s % RG_D]);
  }
  __syncthreads();                  // every wave's reads of the layer-1 activations are done
  store_h(b2);
  __syncthreads();

  // ---- layer 3 (outputs padded to 16 columns)
  {
    f32x4 c3 = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < MLP_NH; ks += 32) {
      const bf16x8 a = *(const bf16x8*)&Hs[wv * 16 + (lane & 15)][ks + 8 * (lane >> 4)];
      const bf16x8 b = *(const bf16x8*)(p.W3b + (long)(lane & 15) * MLP_NH + ks + 8 * (lane >> 4));
      c3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c3, 0, 0, 0);
    }
    const int o = lane & 15;
    if (o < MLP_NOUT)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const long c = c0 + wv * 16 + 4 * (lane >> 4) + e;
        y[c * MLP_NOUT + o] = c3[e] + b3[o];
      }
  }
}

// FP32 rows of 500: the network input of oc_mlp_* (training data).
template <class T>
__global__ void __launch_bounds__(256) closure_features_f32_kernel(Dims d, const T* u,
                                                                   const T* v, const T* w,
                                                                   const T* tt, const T* ss,
                                                                   ClosureStats st, float* x) {
  const long ncell = (long)d.nx * d.ny * d.nz;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ncell * 500) return;
  x[t] = feature_value(d, u, v, w, tt, ss, st, t / 500, (int)(t % 500));
}

// Physical fluxes F_q = y_q std_q + mean_q at cell centres; u takes the
// flux at (x face, z face) as the mean of the four adjacent centres, v the
// same in y, tracers the mean of the two centres about each z face (J_b
// turned into a temperature flux), w the difference of tau_ww across its
// face.  Wall fluxes are zero.
template <class T>
__global__ void __launch_bounds__(256) closure_apply_kernel(Dims d, const float* y, ClosureStats st,
                                                            double rdz, T* gu, T* gv, T* gw,
                                                            T* gt) {
  const long ncell = (long)d.nx * d.ny * d.nz;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ncell) return;
  const int i = (int)(t % d.nx);
  const int j = (int)((t / d.nx) % d.ny);
  const int k = (int)(t / ((long)d.nx * d.ny));
  auto F = [&](int q, int ii, int jj, int kk) -> float {
    ii = (ii + d.nx) % d.nx;
    jj = (jj + d.ny) % d.ny;
    const long c = ((long)kk * d.ny + jj) * d.nx + ii;
    return y[c * 4 + q] * st.out_std[q] + st.out_mean[q];
  };
  // flux through the z face kk (0..nz) of quantity q averaged over x or y
  auto zface = [&](int q, int ax, int kk) -> float {
    if (kk <= 0 || kk >= d.nz) return 0.f;
    if (ax == 0) return 0.25f * (F(q, i - 1, j, kk - 1) + F(q, i, j, kk - 1) + F(q, i - 1, j, kk) +
                                 F(q, i, j, kk));
    if (ax == 1) return 0.25f * (F(q, i, j - 1, kk - 1) + F(q, i, j, kk - 1) + F(q, i, j - 1, kk) +
                                 F(q, i, j, kk));
    return 0.5f * (F(q, i, j, kk - 1) + F(q, i, j, kk));
  };
  const long p = pidx(d, i, j, k);
  const float rz = (float)rdz;
  gu[p] = (T)(-(zface(0, 0, k + 1) - zface(0, 0, k)) * rz);
  gv[p] = (T)(-(zface(1, 1, k + 1) - zface(1, 1, k)) * rz);
  gt[p] = (T)(-(zface(3, 2, k + 1) - zface(3, 2, k)) * rz * st.inv_galpha);
  gw[p] = (k == 0) ? (T)0 : (T)(-(F(2, i, j, k) - F(2, i, j, k - 1)) * rz);
}

template <class T>
hipError_t launch_closure_features(const Dims& d, const T* u, const T* v, const T* w, const T* t,
                                   const T* s, ClosureStats st, __bf16* xb, hipStream_t stream) {
  const long n = (long)d.nx * d.ny * d.nz * 512;
  hipLaunchKernelGGL(closure_features_kernel<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     stream, d, u, v, w, t, s, st, xb);
  return hipGetLastError();
}

template <class T>
hipError_t launch_closure_mlp_fused(const Dims& d, const T* u, const T* v, const T* w, const T* t,
                                    const T* s, ClosureStats st, const MlpParams& p, float* y,
                                    hipStream_t stream) {
  const long n = (long)d.nx * d.ny * d.nz;
  if (d.nx % FZ_BM == 0)
    hipLaunchKernelGGL(closure_mlp_region_kernel<T>, dim3((unsigned)(n / FZ_BM)), dim3(256), 0,
                       stream, d, u, v, w, t, s, st, p, y);
  else
    hipLaunchKernelGGL(closure_mlp_fused_kernel<T>, dim3((unsigned)((n + FZ_BM - 1) / FZ_BM)),
                       dim3(256), 0, stream, d, u, v, w, t, s, st, p, y);
  return hipGetLastError();
}
template hipError_t launch_closure_mlp_fused<float>(const Dims&, const float*, const float*,
                                                    const float*, const float*, const float*,
                                                    ClosureStats, const MlpParams&, float*,
                                                    hipStream_t);
template hipError_t launch_closure_mlp_fused<double>(const Dims&, const double*, const double*,
                                                     const double*, const double*, const double*,
                                                     ClosureStats, const MlpParams&, float*,
                                                     hipStream_t);

template <class T>
hipError_t launch_closure_features_f32(const Dims& d, const T* u, const T* v, const T* w,
                                       const T* t, const T* s, ClosureStats st, float* x,
                                       hipStream_t stream) {
  const long n = (long)d.nx * d.ny * d.nz * 500;
  hipLaunchKernelGGL(closure_features_f32_kernel<T>, dim3((unsigned)((n + 255) / 256)), dim3(256),
                     0, stream, d, u, v, w, t, s, st, x);
  return hipGetLastError();
}
template hipError_t launch_closure_features_f32<float>(const Dims&, const float*, const float*,
                                                       const float*, const float*, const float*,
                                                       ClosureStats, float*, hipStream_t);
template hipError_t launch_closure_features_f32<double>(const Dims&, const double*,
                                                        const double*, const double*,
                                                        const double*, const double*,
                                                        ClosureStats, float*, hipStream_t);

template <class T>
hipError_t launch_closure_apply(const Dims& d, const float* y, ClosureStats st, double rdz, T* gu,
                                T* gv, T* gw, T* gt, hipStream_t stream) {
  const long n = (long)d.nx * d.ny * d.nz;
  hipLaunchKernelGGL(closure_apply_kernel<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     stream, d, y, st, rdz, gu, gv, gw, gt);
  return hipGetLastError();
}

template hipError_t launch_closure_features<float>(const Dims&, const float*, const float*,
                                                   const float*, const float*, const float*,
                                                   ClosureStats, __bf16*, hipStream_t);
template hipError_t launch_closure_features<double>(const Dims&, const double*, const double*,
                                                    const double*, const double*, const double*,
                                                    ClosureStats, __bf16*, hipStream_t);
template hipError_t launch_closure_apply<float>(const Dims&, const float*, ClosureStats, double,
                                                float*, float*, float*, float*, hipStream_t);
template hipError_t launch_closure_apply<double>(const Dims&, const float*, ClosureStats, double,
                                                 double*, double*, double*, double*, hipStream_t);

}  // namespace oc
