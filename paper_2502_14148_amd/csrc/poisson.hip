// FFT/DCT eigenfunction solve of the discrete pressure Poisson equation and
// the projection of the predictor velocity (pressure-correction appendix of
// arXiv 2502.14148: lap p = div(u~)/dt, u = u~ - dt grad p; the 7-point
// Laplacian is diagonalised by Fourier modes in periodic directions and by
// cosine modes (DCT-II) between no-normal-flow walls).
//
// Five passes over a half spectrum held in FP64, kx fastest:
//   1. x: divergence of the predictor (fused) and a real-to-complex FFT
//      (two real lines packed into one complex line);
//   2. y: complex FFT;
//   3. z: DCT-II (Makhoul's N-point FFT reordering) or FFT, division by the
//      eigenvalue, and the inverse transform, all in LDS; on a stretched z a
//      tridiagonal solve per (kx, ky) mode instead;
//   4. y: inverse FFT;
//   5. x: complex-to-real inverse FFT -> p.
// Then a projection kernel applies u -= dt_eff grad p.
//
// Transforms are radix-8/4/2/3 Stockham passes in LDS, one radix-R butterfly
// per thread per pass, twiddles from FP64 tables.
#include "oc_internal.h"

#include <algorithm>

namespace oc {

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ inline double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// multiply by +i (SIGN = +1) or -i (SIGN = -1)
template <int SIGN>
__device__ inline double2 mul_i(double2 a) {
  return SIGN > 0 ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}

// In-register DFT of length R; DIR = -1 forward (exp(-2 pi i/R)), +1 inverse.
template <int R, int DIR>
__device__ inline void dft(double2* v) {
  if (R == 2) {
    double2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if (R == 4) {
    double2 a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
    double2 c = cadd(v[1], v[3]), d = csub(v[1], v[3]);
    v[0] = cadd(a, c);
    v[2] = csub(a, c);
    v[1] = cadd(b, mul_i<DIR>(d));
    v[3] = csub(b, mul_i<DIR>(d));
  } else if (R == 8) {
    // two length-4 DFTs of the even and odd terms, combined with the
    // eighth roots of unity w^k, w = exp(DIR 2 pi i / 8)
    double2 e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
    dft<4, DIR>(e);
    dft<4, DIR>(o);
    const double h = 0.70710678118654752440, s = DIR;  // sqrt(2)/2
    const double2 o1 = make_double2(h * (o[1].x - s * o[1].y), h * (o[1].y + s * o[1].x));
    const double2 o2 = mul_i<DIR>(o[2]);
    const double2 o3 = make_double2(h * (-o[3].x - s * o[3].y), h * (-o[3].y + s * o[3].x));
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  } else {  // R == 3
    const double h = 0.86602540378443864676;  // sqrt(3)/2
    double2 t = cadd(v[1], v[2]), s = csub(v[1], v[2]);
    double2 m = csub(v[0], cscale(t, 0.5));
    double2 r = cscale(mul_i<DIR>(s), h);
    v[0] = cadd(v[0], t);
    v[1] = cadd(m, r);
    v[2] = csub(m, r);
  }
}

// One Stockham pass of radix R over L lines of length N held in LDS at
// buf[line * ls + n * es].  NS is the length of the sub-transforms already
// done.  LINE_FAST maps consecutive threads to consecutive lines (used when
// lines are interleaved, es = L) to avoid LDS bank conflicts.
template <int N, int R, int NS, int L, int NT, int DIR, bool LINE_FAST>
__device__ inline void stockham_pass(double2* buf, int ls, int es, const double2* __restrict__ tw) {
  constexpr int M = N / R;
  constexpr int NB = L * M;
  constexpr int BPT = (NB + NT - 1) / NT;
  double2 v[BPT][R];
  int line_[BPT], jj_[BPT];
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int b = threadIdx.x + q * NT;
    line_[q] = LINE_FAST ? (b % L) : (b / M);
    jj_[q] = LINE_FAST ? (b / L) : (b % M);
    if (NB % NT == 0 || b < NB) {
      const int k = jj_[q] % NS;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double2 x = buf[line_[q] * ls + (jj_[q] + r * M) * es];
        if (r > 0 && NS > 1) {
          double2 w = tw[(r * k) * (N / (NS * R))];
          if (DIR > 0) w = cconj(w);
          x = cmul(x, w);
        }
        v[q][r] = x;
      }
      dft<R, DIR>(v[q]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int b = threadIdx.x + q * NT;
    if (NB % NT == 0 || b < NB) {
      const int k = jj_[q] % NS;
      const int d = (jj_[q] / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[line_[q] * ls + (d + r * NS) * es] = v[q][r];
    }
  }
  __syncthreads();
}

// Radix MAXR (4 or 8) while it divides what remains, then 4, 2, 3.  Radix 8
// saves a quarter of the LDS round trips; it pays in the y and z passes
// (eight interleaved lines: one butterfly per thread) and not in the x
// passes, whose few lines leave half the threads idle at radix 8.
template <int REM, int MAXR>
constexpr int pass_radix() {
  return (MAXR >= 8 && REM % 8 == 0) ? 8 : ((REM % 4 == 0) ? 4 : ((REM % 2 == 0) ? 2 : 3));
}

template <int N, int NS, int L, int NT, int DIR, bool LINE_FAST, int MAXR = 4>
__device__ inline void fft_lines(double2* buf, int ls, int es, const double2* __restrict__ tw) {
  if constexpr (NS < N) {
    constexpr int R = pass_radix<N / NS, MAXR>();
    stockham_pass<N, R, NS, L, NT, DIR, LINE_FAST>(buf, ls, es, tw);
    fft_lines<N, NS * R, L, NT, DIR, LINE_FAST, MAXR>(buf, ls, es, tw);
  }
}

// Interleaved lines (buf[n * L + line], consecutive threads on consecutive
// lines) whose first pass takes its inputs from global memory, load(line, n),
// instead of from a staged copy in LDS: the tile's load and the first pass
// share one trip, and only the pass's outputs go to LDS.  (The first pass
// has no twiddles; the barrier after it also covers the twiddle staging.)
template <int N, int L, int NT, int DIR, int MAXR, class Load>
__device__ inline void first_pass_from(double2* buf, const Load& load) {
  constexpr int R = pass_radix<N, MAXR>();
  constexpr int M = N / R, NB = L * M, BPT = (NB + NT - 1) / NT;
  double2 v[BPT][R];
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int b = threadIdx.x + q * NT;
    if (NB % NT == 0 || b < NB) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = load(b % L, b / L + r * M);
      dft<R, DIR>(v[q]);
    }
  }
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int b = threadIdx.x + q * NT;
    if (NB % NT == 0 || b < NB) {
#pragma unroll
      for (int r = 0; r < R; ++r) buf[((b / L) * R + r) * L + b % L] = v[q][r];
    }
  }
  __syncthreads();
}
template <int N, int L, int NT, int DIR, int MAXR, class Load>
__device__ inline void fft_lines_from(double2* buf, const double2* __restrict__ tw,
                                      const Load& load) {
  first_pass_from<N, L, NT, DIR, MAXR>(buf, load);
  fft_lines<N, pass_radix<N, MAXR>(), L, NT, DIR, true, MAXR>(buf, 1, L, tw);
}

// The same lines whose last pass hands its outputs to store(line, n, value)
// (global memory) instead of writing them back to LDS.
template <int N, int NS, int L, int NT, int DIR, int MAXR, class Store>
__device__ inline void fft_lines_to(double2* buf, const double2* __restrict__ tw,
                                    const Store& store) {
  constexpr int R = pass_radix<N / NS, MAXR>();
  if constexpr (NS * R < N) {
    stockham_pass<N, R, NS, L, NT, DIR, true>(buf, 1, L, tw);
    fft_lines_to<N, NS * R, L, NT, DIR, MAXR>(buf, tw, store);
  } else {
    constexpr int M = N / R, NB = L * M, BPT = (NB + NT - 1) / NT;
#pragma unroll
    for (int q = 0; q < BPT; ++q) {
      const int b = threadIdx.x + q * NT;
      if (NB % NT == 0 || b < NB) {
        const int line = b % L, jj = b / L, k = jj % NS;
        double2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          double2 x = buf[(jj + r * M) * L + line];
          if (r > 0 && NS > 1) {
            double2 w = tw[(r * k) * (N / (NS * R))];
            if (DIR > 0) w = cconj(w);
            x = cmul(x, w);
          }
          v[r] = x;
        }
        dft<R, DIR>(v);
        const int d = (jj / NS) * NS * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) store(line, d + r * NS, v[r]);
      }
    }
  }
}

// Both: the first pass from global memory, the last one to it.
template <int N, int L, int NT, int DIR, int MAXR, class Load, class Store>
__device__ inline void fft_lines_io(double2* buf, const double2* __restrict__ tw, const Load& load,
                                    const Store& store) {
  constexpr int R = pass_radix<N, MAXR>();
  if constexpr (R == N) {   // one pass
    constexpr int NB = L, BPT = (NB + NT - 1) / NT;
#pragma unroll
    for (int q = 0; q < BPT; ++q) {
      const int b = threadIdx.x + q * NT;
      if (NB % NT == 0 || b < NB) {
        double2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = load(b, r);
        dft<R, DIR>(v);
#pragma unroll
        for (int r = 0; r < R; ++r) store(b, r, v[r]);
      }
    }
  } else {
    first_pass_from<N, L, NT, DIR, MAXR>(buf, load);
    fft_lines_to<N, R, L, NT, DIR, MAXR>(buf, tw, store);
  }
}

constexpr int NT = 256;
// Twiddle table staged in LDS by the whole workgroup (made visible by the
// barrier that follows the tile load), so that the Stockham passes read
// their factors from LDS instead of waiting on global memory between barriers.
template <int N>
__device__ inline void stage_twiddles(double2* tws, const double2* __restrict__ tw) {
#pragma unroll
  for (int q = 0; q < (N + NT - 1) / NT; ++q) {
    const int t = threadIdx.x + q * NT;
    if (N % NT == 0 || t < N) tws[t] = ld2(tw, t);
  }
}
template <int N> struct XCfg { static constexpr int LP = (N >= 1024) ? 1 : 1024 / N; };
template <int N> struct YZCfg { static constexpr int W = (N >= 512) ? 4 : (N >= 256 ? 8 : 16); };

// ---------------------------------------------------------------------------
// Pass 1: rhs = div(u~) * inv_dt on line pairs (j, j+1), packed FFT along x.
// ---------------------------------------------------------------------------
// dense != null: transform that dense FP64 (nz, ny, nx) field instead (the
// preconditioner of the immersed-boundary solve).
template <class T, int N>
__global__ void __launch_bounds__(NT) fwd_x_kernel(Dims d, const T* __restrict__ u,
                                                   const T* __restrict__ v,
                                                   const T* __restrict__ w, double inv_dt,
                                                   double rdx, double rdy,
                                                   const double* __restrict__ rdzc, SpecBufs sb,
                                                   const PoissonSlots* __restrict__ bs,
                                                   const double* __restrict__ dense) {
  if (sb.stop && *glb(sb.stop) != 0.0) return;
  if (bs) {
    const int z = blockIdx.z;
    u = (const T*)bs->u[z];
    v = (const T*)bs->v[z];
    w = (const T*)bs->w[z];
    sb.spec = bs->spec[z];
  }
  constexpr int LP = XCfg<N>::LP;
  __shared__ double2 buf[LP * N];
  __shared__ double2 tws[N];
  stage_twiddles<N>(tws, sb.twx);
  const int k = blockIdx.y;
  const int npairs = d.ny / 2;
  const int pair0 = blockIdx.x * LP;
  // A thread takes four consecutive points of both lines of a pair (16-byte
  // row loads; rows carry no alignment, the loads need none) and stores
  // the packed values (line 2pr, line 2pr+1) at buf[l N + i .. + 3].
  // Compile-time trip counts, so that every load is in flight before the
  // first one is used.
  constexpr int NQ = N / 4, QUADS = LP * NQ, QPT = (QUADS + NT - 1) / NT;
  static_assert(N % 4 == 0, "four points per thread");
#pragma unroll
  for (int q = 0; q < QPT; ++q) {
    const int t = threadIdx.x + q * NT;
    if (QUADS % NT != 0 && t >= QUADS) break;
    const int l = t / NQ, i = 4 * (t % NQ);
    const int pr = pair0 + l;
    double de[4] = {0.0, 0.0, 0.0, 0.0}, dod[4] = {0.0, 0.0, 0.0, 0.0};
    if (pr < npairs && dense) {
      const long o = ((long)k * d.ny + 2 * pr) * d.nx + i;
      const v4u<double> xe = ld4(dense, o), xo = ld4(dense, o + d.nx);
#pragma unroll
      for (int m = 0; m < 4; ++m) { de[m] = xe[m]; dod[m] = xo[m]; }
    } else if (pr < npairs) {
      const double rdz = rdzc[k];
      const int j = 2 * pr;
      const long c = pidx(d, i, j, k);
      // x neighbour of the fourth point, the line above the pair and the
      // level above (periodic wraps; above a top wall w is 0)
      const long ie = (i + 4 == d.nx) ? 4 - d.nx : 4;
      const long jn = (j + 2 == d.ny) ? -(long)(d.ny - 2) * d.sy : 2 * d.sy;
      const bool top_wall = d.zb && k + 1 == d.nz;
      const long kn = (k + 1 == d.nz) ? -(long)(d.nz - 1) * d.sz : d.sz;
      const long co = c + d.sy;
      const v4u<T> ue = ld4(u, c), uo = ld4(u, co);
      const T uee = glb(u)[c + ie], uoe = glb(u)[co + ie];
      const v4u<T> ve = ld4(v, c), vo = ld4(v, co), vn = ld4(v, c + jn);
      const v4u<T> we = ld4(w, c), wo = ld4(w, co);
      v4u<T> wte = {T(0), T(0), T(0), T(0)}, wto = wte;
      if (!top_wall) { wte = ld4(w, c + kn); wto = ld4(w, co + kn); }
      const bool bottom_wall = d.zb && k == 0;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const double upe = (double)(m < 3 ? ue[m + 1] : uee);
        const double upo = (double)(m < 3 ? uo[m + 1] : uoe);
        const double wbe = bottom_wall ? 0.0 : (double)we[m];
        const double wbo = bottom_wall ? 0.0 : (double)wo[m];
        de[m] = ((upe - (double)ue[m]) * rdx + ((double)vo[m] - (double)ve[m]) * rdy +
                 ((double)wte[m] - wbe) * rdz) * inv_dt;
        dod[m] = ((upo - (double)uo[m]) * rdx + ((double)vn[m] - (double)vo[m]) * rdy +
                  ((double)wto[m] - wbo) * rdz) * inv_dt;
      }
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) buf[l * N + i + m] = make_double2(de[m], dod[m]);
  }
  __syncthreads();
  fft_lines<N, 1, LP, NT, -1, false>(buf, N, 1, tws);
  // unpack the two real spectra: X1 = (Z_k + conj Z_{N-k})/2, X2 = -i (Z_k - conj Z_{N-k})/2
  const int nxh = sb.nxh;
  for (int t = threadIdx.x; t < LP * nxh; t += NT) {
    const int l = t / nxh, kx = t % nxh;
    const int pr = pair0 + l;
    if (pr >= npairs) continue;
    double2 a = buf[l * N + kx];
    double2 b = cconj(buf[l * N + ((N - kx) % N)]);
    double2 x1 = cscale(cadd(a, b), 0.5);
    double2 x2 = cscale(mul_i<-1>(csub(a, b)), 0.5);
    const long base = ((long)k * d.ny + 2 * pr) * sb.nxp + kx;
    st2(sb.spec, base, x1);
    st2(sb.spec, base + sb.nxp, x2);
  }
}

// ---------------------------------------------------------------------------
// Passes 2 and 4: complex FFT along y for W consecutive kx columns.
// ---------------------------------------------------------------------------
template <int N, int DIR>
__global__ void __launch_bounds__(NT) y_kernel(Dims d, SpecBufs sb,
                                               const PoissonSlots* __restrict__ bs) {
  if (sb.stop && *glb(sb.stop) != 0.0) return;
  if (bs) sb.spec = bs->spec[blockIdx.z];
  constexpr int W = YZCfg<N>::W;
  __shared__ double2 buf[W * N];
  __shared__ double2 tws[N];
  stage_twiddles<N>(tws, sb.twy);
  // the forward pass takes the planes in the reverse of the order the x pass
  // wrote them, so it starts on the ones most likely still in the caches
  const int k = DIR < 0 ? (int)gridDim.y - 1 - (int)blockIdx.y : (int)blockIdx.y;
  const int kx0 = blockIdx.x * W;
  const int nxh = sb.nxh, nxp = sb.nxp;
  double2* plane = sb.spec + (long)k * d.ny * nxp + kx0;
  const int ncol = nxh - kx0;   // valid columns of this block (W or fewer)
  fft_lines_io<N, W, NT, DIR, 8>(
      buf, tws,
      [&](int c, int y) {
        return c < ncol ? ld2(plane, (long)y * nxp + c) : make_double2(0.0, 0.0);
      },
      [&](int c, int y, double2 x) {
        if (c < ncol) st2(plane, (long)y * nxp + c, x);
      });
}

// ---------------------------------------------------------------------------
// Pass 3: along z, forward transform, division by the eigenvalue (with the
// 1/(nx ny nz) normalisation of the unnormalised inverses), inverse.
// ---------------------------------------------------------------------------
// DCT-II via an N-point FFT (Makhoul): v[n'] = x[2n'], v[N-1-n'] = x[2n'+1];
// the source level of position p
__device__ inline int makhoul_src(int p, int n) {
  return (p < n / 2) ? 2 * p : 2 * (n - 1 - p) + 1;
}

// The division, and on walls the DCT post- and pre-processing around it,
// in place and without a barrier: the post-processing of mode k reads V_k
// and V_{N-k}, and the pre-processing of the inverse writes the same two, so
// one thread owns the pair (k, N-k); the first pair of a column is the two
// self-paired modes k = 0 and k = N/2.  On periodic z the pair is (k, k+N/2).
//   X_k = (e_k V_k + conj(e_k) V_{N-k}) / 2,  e_k = exp(-i pi k / 2N)
//   Y_k = X_k norm / lam_k  (0 for the singular mode)
//   V'_k = conj(e_k) (Y_k - i Y_{N-k}),  Y_N = 0
// The factors norm / lam and e_k of a thread's pairs are fetched and formed
// before the forward transform, so that their latency hides behind the tile
// load; e_{N-k} = -i conj(e_k).
template <int N, bool BOUNDED>
struct ZPairs {
  static constexpr int W = YZCfg<N>::W;
  static constexpr int NU = W * N / 2;          // pairs per column block
  static constexpr int UPT = (NU + NT - 1) / NT;  // pairs per thread
  static_assert(NT % W == 0, "a thread keeps one column");
  double sa[UPT], sb[UPT];

  __device__ inline void load(const SpecBufs& b, int j, int kx0, double norm) {
    const int c = (int)threadIdx.x % W;
    const double lxy = (kx0 + c < b.nxh ? glb(b.lamx)[kx0 + c] : 1.0) + glb(b.lamy)[j];
#pragma unroll
    for (int q = 0; q < UPT; ++q) {
      const int u = min(((int)threadIdx.x + q * NT) / W, N / 2 - 1);
      const int kb = BOUNDED ? (u == 0 ? N / 2 : N - u) : u + N / 2;
      const double la = lxy + glb(b.lamz)[u], lb = lxy + glb(b.lamz)[kb];
      sa[q] = (la == 0.0) ? 0.0 : norm / la;
      sb[q] = (lb == 0.0) ? 0.0 : norm / lb;
    }
  }

  __device__ inline void apply(double2* buf, const double2* __restrict__ dctz) const {
    const double h = 0.70710678118654752440;
#pragma unroll
    for (int q = 0; q < UPT; ++q) {
      const int t = (int)threadIdx.x + q * NT;
      if (NU % NT != 0 && t >= NU) break;
      const int c = t % W, u = t / W;
      const bool self = (u == 0);
      const int kb = BOUNDED ? (self ? N / 2 : N - u) : u + N / 2;
      const double2 va = buf[u * W + c], vb = buf[kb * W + c];
      double2 ra, rb;
      if (BOUNDED) {
        const double2 ea = ld2(dctz, u);
        const double2 eb = self ? make_double2(h, -h) : make_double2(-ea.y, -ea.x);
        const double2 pa = self ? va : vb, pb = self ? vb : va;
        const double2 xa = cscale(cadd(cmul(ea, va), cmul(cconj(ea), pa)), 0.5);
        const double2 xb = cscale(cadd(cmul(eb, vb), cmul(cconj(eb), pb)), 0.5);
        const double2 ya = cscale(xa, sa[q]), yb = cscale(xb, sb[q]);
        const double2 qa = self ? make_double2(0.0, 0.0) : yb, qb = self ? yb : ya;
        ra = cmul(cconj(ea), csub(ya, mul_i<1>(qa)));
        rb = cmul(cconj(eb), csub(yb, mul_i<1>(qb)));
      } else {
        ra = cscale(va, sa[q]);
        rb = cscale(vb, sb[q]);
      }
      buf[u * W + c] = ra;
      buf[kb * W + c] = rb;
    }
  }
};

// Four waves per SIMD: four blocks per CU, as many as the LDS holds.
template <int N, bool BOUNDED>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4)))
    z_kernel(Dims d, SpecBufs sb, double norm, const PoissonSlots* __restrict__ bs) {
  if (sb.stop && *glb(sb.stop) != 0.0) return;
  if (bs) sb.spec = bs->spec[blockIdx.z];
  constexpr int W = YZCfg<N>::W;
  __shared__ double2 buf[W * N];
  __shared__ double2 tws[N];
  const int j = blockIdx.y;
  const int kx0 = blockIdx.x * W;
  const int nxh = sb.nxh, nxp = sb.nxp;
  ZPairs<N, BOUNDED> pairs;
  pairs.load(sb, j, kx0, norm);
  stage_twiddles<N>(tws, sb.twz);
  const long zs = (long)d.ny * nxp;
  double2* col = sb.spec + (long)j * nxp + kx0;
  const int ncol = nxh - kx0;   // valid columns of this block (W or fewer)
  // transform position n holds level makhoul_src(n) (DCT-II by Makhoul's
  // reordering) on walls, level n when periodic
  auto level = [](int n) { return BOUNDED ? makhoul_src(n, N) : n; };
  fft_lines_from<N, W, NT, -1, 8>(buf, tws, [&](int c, int n) {
    return c < ncol ? ld2(col, (long)level(n) * zs + c) : make_double2(0.0, 0.0);
  });
  pairs.apply(buf, sb.dctz);
  __syncthreads();
  fft_lines_to<N, 1, W, NT, 1, 8>(buf, tws, [&](int c, int n, double2 x) {
    if (c < ncol) st2(col, (long)level(n) * zs + c, x);
  });
}

// ---------------------------------------------------------------------------
// Pass 3 on a stretched z (the mixed FFT-tridiagonal solver): every (kx, ky)
// mode solves along z
//   lo_k p_{k-1} + (lam_x + lam_y - lo_k - up_k) p_k + up_k p_{k+1} = r_k / (nx ny)
// with each equation scaled to a unit diagonal, a_k x_{k-1} + x_k + c_k x_{k+1}
// = d_k.  PCR_W modes per workgroup and 32 threads per mode, each owning a
// chunk of TD_M consecutive levels (levels past nz are rows x = 0, which
// leave the others unchanged).  Partition method: a thread eliminates its
// chunk's interior in registers, downwards and then upwards, until every
// row reads  a''_i x_first + x_i + c''_i x_last = d''_i  and the chunk's
// first and last rows couple only to the neighbouring chunks' last and
// first unknowns.  Those two rows per chunk form a tridiagonal system of
// 64 unknowns per mode, solved by parallel cyclic reduction in LDS; then
// every thread substitutes its chunk's interior.  The systems are strictly
// diagonally dominant (lam_x + lam_y < 0): no pivoting.  The horizontally
// uniform mode is singular (no-flux walls) and is integrated directly: the
// face gradient obeys g_{k+1} = g_k + dzc_k r_k from g_0 = 0, then p_k =
// p_{k-1} + dzf_k g_k, and the volume-weighted mean is removed.
// ---------------------------------------------------------------------------
constexpr int PCR_W = 8, PCR_NMAX = 256;
constexpr int TD_P = NT / PCR_W, TD_M = PCR_NMAX / TD_P, TD_R = 2 * TD_P;
static_assert(TD_M >= 3, "the partition method needs three rows per chunk");
static_assert(PCR_W * TD_R >= PCR_NMAX && PCR_W * TD_R == 2 * NT, "reduced-row layout");

__global__ void __launch_bounds__(NT) z_tridiag_kernel(Dims d, SpecBufs sb, double norm,
                                                       const double* __restrict__ lo,
                                                       const double* __restrict__ up,
                                                       const double* __restrict__ dzc,
                                                       const double* __restrict__ dzf) {
  // reduced rows, mode-major: row 2p (chunk p's first) and 2p + 1 (its last)
  __shared__ double sa[PCR_W * TD_R], sc[PCR_W * TD_R];
  __shared__ double2 sr[PCR_W * TD_R];   // also the uniform mode's column
  const int nz = d.nz;
  const int j = blockIdx.y, kx0 = blockIdx.x * PCR_W;
  const int nxh = sb.nxh, nxp = sb.nxp;
  const long zs = (long)d.ny * nxp;
  // consecutive threads on consecutive modes: a wave loads eight 128-byte
  // level rows per instruction
  const int c = (int)threadIdx.x % PCR_W, pc = (int)threadIdx.x / PCR_W;
  const int kx = kx0 + c, z0 = pc * TD_M;
  const bool live = kx < nxh && (kx | j) != 0;
  const double lam = live ? sb.lamx[kx] + sb.lamy[j] : 0.0;
  const long col = (long)j * nxp + kx;
  double a[TD_M], cc[TD_M];
  double2 r[TD_M];
#pragma unroll
  for (int i = 0; i < TD_M; ++i) {
    const int z = z0 + i;
    a[i] = 0.0;
    cc[i] = 0.0;
    r[i] = make_double2(0.0, 0.0);
    if (live && z < nz) {
      const double l = lo[z], u = up[z];
      const double ib = 1.0 / (lam - l - u);
      a[i] = l * ib;
      cc[i] = u * ib;
      r[i] = cscale(ld2(sb.spec, z * zs + col), norm * ib);
    }
  }
  // downwards: rows i >= 1 become a_i x_first + x_i + c_i x_{i+1} = r_i
#pragma unroll
  for (int i = 2; i < TD_M; ++i) {
    const double ib = 1.0 / (1.0 - a[i] * cc[i - 1]);
    r[i] = cscale(csub(r[i], cscale(r[i - 1], a[i])), ib);
    a[i] = -a[i] * a[i - 1] * ib;
    cc[i] *= ib;
  }
  // upwards: rows 1 .. TD_M - 2 become a_i x_first + x_i + c_i x_last = r_i
#pragma unroll
  for (int i = TD_M - 3; i >= 1; --i) {
    r[i] = csub(r[i], cscale(r[i + 1], cc[i]));
    a[i] -= cc[i] * a[i + 1];
    cc[i] = -cc[i] * cc[i + 1];
  }
  // the first row: a_0 x_{first-1} + x_first + c_0 x_last = r_0
  {
    const double ib = 1.0 / (1.0 - cc[0] * a[1]);
    r[0] = cscale(csub(r[0], cscale(r[1], cc[0])), ib);
    a[0] *= ib;
    cc[0] = -cc[0] * cc[1] * ib;
  }
  const int e0 = c * TD_R + 2 * pc;
  sa[e0] = a[0];
  sc[e0] = cc[0];
  sr[e0] = r[0];
  sa[e0 + 1] = a[TD_M - 1];
  sc[e0 + 1] = cc[TD_M - 1];
  sr[e0 + 1] = r[TD_M - 1];
  __syncthreads();
  // cyclic reduction of the reduced systems: thread t takes rows t and
  // t + NT (both of mode t / TD_R resp. t / TD_R + NT / TD_R)
  for (int st = 1; st < TD_R; st <<= 1) {
    double na[2], nc[2];
    double2 nr[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = (int)threadIdx.x + h * NT, q = e % TD_R;
      const double ae = sa[e], ce = sc[e];
      double am = 0.0, cm = 0.0, ap = 0.0, cp = 0.0;
      double2 rm = make_double2(0.0, 0.0), rp = rm;
      if (q >= st) { am = sa[e - st]; cm = sc[e - st]; rm = sr[e - st]; }
      if (q + st < TD_R) { ap = sa[e + st]; cp = sc[e + st]; rp = sr[e + st]; }
      const double ib = 1.0 / (1.0 - ae * cm - ce * ap);
      na[h] = -ae * am * ib;
      nc[h] = -ce * cp * ib;
      nr[h] = cscale(csub(csub(sr[e], cscale(rm, ae)), cscale(rp, ce)), ib);
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = (int)threadIdx.x + h * NT;
      sa[e] = na[h];
      sc[e] = nc[h];
      sr[e] = nr[h];
    }
    __syncthreads();
  }
  // the chunk's first and last unknowns, then its interior
  const double2 xf = sr[e0], xl = sr[e0 + 1];
#pragma unroll
  for (int i = 0; i < TD_M; ++i) {
    const int z = z0 + i;
    double2 x = xf;
    if (i == TD_M - 1) x = xl;
    else if (i > 0) x = csub(csub(r[i], cscale(xf, a[i])), cscale(xl, cc[i]));
    if (live && z < nz) st2(sb.spec, z * zs + col, x);
  }
  if (blockIdx.x != 0 || j != 0) return;  // uniform within the workgroup
  // ---- the horizontally uniform mode (kx = 0, ky = 0)
  __syncthreads();
  for (int z = threadIdx.x; z < nz; z += NT) sr[z] = sb.spec[z * zs];
  __syncthreads();
  if (threadIdx.x == 0) {
    double2 g = make_double2(0.0, 0.0), pk = make_double2(0.0, 0.0), acc = make_double2(0.0, 0.0);
    double vol = 0.0;
    for (int z = 0; z < nz; ++z) {
      if (z > 0) pk = cadd(pk, cscale(g, dzf[z]));
      g = cadd(g, cscale(sr[z], dzc[z] * norm));
      sr[z] = pk;
      acc = cadd(acc, cscale(pk, dzc[z]));
      vol += dzc[z];
    }
    sa[0] = acc.x / vol;
    sa[1] = acc.y / vol;
  }
  __syncthreads();
  const double2 mean = make_double2(sa[0], sa[1]);
  for (int z = threadIdx.x; z < nz; z += NT) sb.spec[z * zs] = csub(sr[z], mean);
}

// ---------------------------------------------------------------------------
// Pass 5: complex-to-real inverse FFT along x for line pairs -> p.
// ---------------------------------------------------------------------------
// rdot != null: also the partial sum of rdot . p over the values this
// workgroup writes, into part[blockIdx.y * gridDim.x + blockIdx.x] (the r . z
// of the immersed-boundary iteration).
template <int N>
__global__ void __launch_bounds__(NT) inv_x_kernel(Dims d, SpecBufs sb,
                                                   const PoissonSlots* __restrict__ bs,
                                                   const double* __restrict__ rdot,
                                                   double* __restrict__ part) {
  if (sb.stop && *glb(sb.stop) != 0.0) return;
  if (bs) {
    sb.spec = bs->spec[blockIdx.z];
    sb.p = bs->p[blockIdx.z];
  }
  const auto pout = glb(sb.p);
  const auto grdot = glb(rdot);
  constexpr int LP = XCfg<N>::LP;
  __shared__ double2 buf[LP * N];
  __shared__ double2 tws[N];
  stage_twiddles<N>(tws, sb.twx);
  const int k = blockIdx.y;
  const int npairs = d.ny / 2;
  const int pair0 = blockIdx.x * LP;
  constexpr int LOADS = (LP * N + NT - 1) / NT;
#pragma unroll
  for (int q = 0; q < LOADS; ++q) {
    const int t = threadIdx.x + q * NT;
    if ((LP * N) % NT != 0 && t >= LP * N) break;
    const int l = t / N, n = t % N;
    const int pr = pair0 + l;
    double2 z = make_double2(0.0, 0.0);
    if (pr < npairs) {
      const long base = ((long)k * d.ny + 2 * pr) * sb.nxp;
      const bool lo = n <= N / 2;
      const int m = lo ? n : N - n;
      double2 x1 = ld2(sb.spec, base + m), x2 = ld2(sb.spec, base + sb.nxp + m);
      if (!lo) { x1 = cconj(x1); x2 = cconj(x2); }
      z = cadd(x1, mul_i<1>(x2));  // Z = X1 + i X2
    }
    buf[t] = z;
  }
  __syncthreads();
  fft_lines<N, 1, LP, NT, 1, false>(buf, N, 1, tws);
  double acc = 0.0;
  for (int t = threadIdx.x; t < LP * N; t += NT) {
    const int l = t / N, i = t % N;
    const int pr = pair0 + l;
    if (pr >= npairs) continue;
    const long base = ((long)k * d.ny + 2 * pr) * d.nx + i;
    pout[base] = buf[t].x;
    pout[base + d.nx] = buf[t].y;
    if (rdot) acc += grdot[base] * buf[t].x + grdot[base + d.nx] * buf[t].y;
  }
  if (rdot) {
    __shared__ double red[NT];
    red[threadIdx.x] = acc;
    __syncthreads();
#pragma unroll
    for (int h = NT / 2; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) glb(part)[blockIdx.y * gridDim.x + blockIdx.x] = red[0];
  }
}

// ---------------------------------------------------------------------------
// Projection u -= scale grad p at interior faces (wall faces of w untouched).
// A workgroup covers 64 x 4 columns and marches up PJ_KC planes, keeping the
// pressure of the plane below in a register, so p is fetched once per cell
// (plus one plane per chunk).
// ---------------------------------------------------------------------------
constexpr int PJ_X = 64, PJ_Y = 4, PJ_KC = 8;

// mask != null (immersed boundary): velocities on closed faces are set to 0.
template <class T>
__global__ void __launch_bounds__(PJ_X * PJ_Y) project_kernel(
    Dims d, T* __restrict__ u, T* __restrict__ v, T* __restrict__ w, double scale, double rdx,
    double rdy, const double* __restrict__ rdzf, const double* __restrict__ p,
    const PoissonSlots* __restrict__ bs, const T* __restrict__ mask) {
  if (bs) {
    const int z = blockIdx.z;
    u = (T*)bs->u[z];
    v = (T*)bs->v[z];
    w = (T*)bs->w[z];
    p = bs->p[z];
  }
  // Workgroups are dealt round-robin to the 8 XCDs; renumber them so that
  // each XCD takes a contiguous run of tiles (x fastest, then y, then the z
  // chunk), and the cache lines shared by neighbouring tiles stay in one L2.
  const int nbx = (d.nx + PJ_X - 1) / PJ_X;
  const int ntile = (int)(gridDim.x * gridDim.y);
  int lin = (int)(blockIdx.x + blockIdx.y * gridDim.x);
  if (ntile % 8 == 0) lin = (lin % 8) * (ntile / 8) + lin / 8;
  const int txy = lin % (int)gridDim.x;
  const int i = (txy % nbx) * PJ_X + (int)(threadIdx.x % PJ_X);
  const int j = (txy / nbx) * PJ_Y + (int)(threadIdx.x / PJ_X);
  if (i >= d.nx || j >= d.ny) return;
  const int k0 = (lin / (int)gridDim.x) * PJ_KC;
  const int k1 = min(k0 + PJ_KC, d.nz);
  const long plane = (long)d.nx * d.ny;
  const auto pc = glb(p) + (long)j * d.nx + i;
  const auto gu = glb(u), gv = glb(v), gw = glb(w);
  const auto gmask = glb(mask);
  const long oxm = ((i == 0) ? d.nx - 1 : i - 1) - i;
  const long oym = (long)(((j == 0) ? d.ny - 1 : j - 1) - j) * d.nx;
  // pressure below the first plane of the chunk (periodic wrap in z)
  double pb = 0.0;
  if (k0 > 0) pb = pc[(long)(k0 - 1) * plane];
  else if (!d.zb) pb = pc[(long)(d.nz - 1) * plane];
  // planes in batches of PJ_B: all loads of a batch are issued before its
  // stores (the stores may alias later loads of the same field)
  constexpr int PJ_B = 4;
  for (int kb = k0; kb < k1; kb += PJ_B) {
    double p0[PJ_B], pxm[PJ_B], pym[PJ_B];
    T uu[PJ_B], vv[PJ_B], ww[PJ_B];
#pragma unroll
    for (int q = 0; q < PJ_B; ++q) {
      if (kb + q < k1) {
        const long t = (long)(kb + q) * plane;
        p0[q] = pc[t];
        pxm[q] = pc[t + oxm];
        pym[q] = pc[t + oym];
        const long c = pidx(d, i, j, kb + q);
        uu[q] = gu[c];
        vv[q] = gv[c];
        ww[q] = gw[c];
      }
    }
#pragma unroll
    for (int q = 0; q < PJ_B; ++q) {
      const int k = kb + q;
      if (k < k1) {
        T un = (T)((double)uu[q] - scale * (p0[q] - pxm[q]) * rdx);
        T vn = (T)((double)vv[q] - scale * (p0[q] - pym[q]) * rdy);
        T wn = ww[q];
        if (!d.zb || k > 0) wn = (T)((double)wn - scale * (p0[q] - pb) * rdzf[k]);
        pb = p0[q];
        if (mask) {
          const long c = pidx(d, i, j, k);
          const T m0 = gmask[c];
          un = un * (m0 * gmask[c - 1]);
          vn = vn * (m0 * gmask[c - d.sy]);
          if (!d.zb || k > 0) wn = wn * (m0 * gmask[c - d.sz]);
        }
        // the final velocities, with their halo images
        store_with_images(u, d, i, j, k, un, false);
        store_with_images(v, d, i, j, k, vn, false);
        store_with_images(w, d, i, j, k, wn, true);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Pass 5 fused with the projection (the FFT/DCT solve of the whole box).  A
// workgroup takes rb <= RB = 2 L - 1 rows, j0 .. j0 + rb - 1 (the rows are
// dealt evenly to the fewest blocks of at most RB; a block of one member is
// a column), and a chunk of the column's levels.  At every level it
// transforms L packed lines back to p: line l holds rows j0 - 1 + 2l and
// j0 + 2l (Z = X_a + i X_b of their Hermitian half rows), so the row below
// the block (periodic in y) comes along in line 0.
// It then subtracts scale * grad p from u, v and w of its rows: p at i - 1
// and j - 1 come from the lines in LDS, p of the level below from registers
// (the level below the chunk is transformed once more first).  p is not
// written: the spectrum stays in its buffer, and the stand-alone pass 5
// turns it into p when p is asked for.  Every column has the same number of
// chunks (chosen at launch against the resident workgroups), each column's
// levels dealt evenly to them.
// ---------------------------------------------------------------------------

// Lines per level and levels per transform of the fused pass: four lines
// (7 rows) at length 256, about 512 / N at the shorter lengths, which keeps
// a thread's cells per level at four or fewer and its registers near 150
// (three waves per SIMD).  Length 96 transforms two levels at once: with
// one, fewer than half of the threads have a first-pass butterfly, and two
// cost no resident wave there (measured in the 48-member ensemble: 223 ->
// 200 us per launch; at 128 and 64 the second level costs a wave and time).
template <int N> struct PXCfg {
  static constexpr int L = N >= 256 ? 4 : (512 / N > 2 ? 512 / N : 2);
  static constexpr int LV = N == 96 ? 2 : 1;
};

template <class T, int N>
__global__ void __launch_bounds__(NT) inv_x_project_kernel(
    Dims d, SpecBufs sb, T* __restrict__ u, T* __restrict__ v, T* __restrict__ w, double scale,
    double rdx, double rdy, const double* __restrict__ rdzf, int rb, int nblk, int nch,
    const PoissonSlots* __restrict__ bs) {
  // Workgroups are dealt round-robin to the 8 XCDs: XCD x takes workgroups
  // x, x + 8, ...; renumber them so that each XCD works on a contiguous run
  // (the chunks of a column, then the next column), whose shared rows and
  // levels stay in its L2
  const int nwg = (int)gridDim.x, bid = (int)blockIdx.x, xcd = bid % 8;
  const int wg = xcd * (nwg / 8) + min(xcd, nwg % 8) + bid / 8;
  // nch chunks per column, each column's levels dealt evenly to them
  const int colm = wg / nch, ch = wg % nch;
  if (bs) {
    const int z = colm / nblk;
    u = (T*)bs->u[z];
    v = (T*)bs->v[z];
    w = (T*)bs->w[z];
    sb.spec = bs->spec[z];
  }
  constexpr int L = PXCfg<N>::L, LV = PXCfg<N>::LV, LT = L * LV;
  constexpr int RB = 2 * L - 1, CELLS = RB * N;
  constexpr int R0 = pass_radix<N, 4>();
  __shared__ double2 buf[LT * N];
  __shared__ double2 tws[N];
  stage_twiddles<N>(tws, sb.twx);
  const int j0 = (colm % nblk) * rb;   // rb <= RB rows per block
  const int k0 = (int)((long)ch * d.nz / nch), k1 = (int)((long)(ch + 1) * d.nz / nch);
  const int nxp = sb.nxp, ny = d.ny, jend = min(ny, j0 + rb);
  const auto gu = glb(u), gv = glb(v), gw = glb(w);
  // The chunk's levels as a stream: the level below the chunk (if there is
  // one), then k0 .. k1 - 1.  An iteration transforms LV consecutive ones
  // and projects those that belong to the chunk.
  const bool below = !d.zb || k0 > 0;
  const int kb = k0 > 0 ? k0 - 1 : d.nz - 1;
  const int ns = k1 - k0 + (below ? 1 : 0);
  auto lev = [&](int sv) { return below ? (sv == 0 ? kb : k0 + sv - 1) : k0 + sv; };
  // The first Stockham pass, one radix-R0 butterfly per thread (LT N / R0 <=
  // NT), takes its points from registers: fetch(s) issues the loads of the
  // iteration starting at stream index s, first() combines each row pair
  // (with the Hermitian extension) and writes the pass's outputs.  The next
  // iteration's loads are issued right after this one's first pass, so they
  // travel while this one is transformed and projected.
  constexpr int M0 = N / R0;
  static_assert(LT * M0 <= NT, "one first-pass butterfly per thread");
  const int bl = (int)threadIdx.x / M0, bj = (int)threadIdx.x % M0;
  const bool bact = (int)threadIdx.x < LT * M0;
  const int bv = bl / L, blv = bl % L;   // the line's level in the iteration, its index
  const int ja = (blv == 0 && j0 == 0) ? ny - 1 : j0 - 1 + 2 * blv, jb = j0 + 2 * blv;
  const bool has_a = bact && (blv == 0 || ja < jend), has_b = bact && jb < jend;
  double2 fa[R0], fb[R0];
  auto fetch = [&](int s) {
    const bool ok = s + bv < ns;
    const long lvl = (long)(ok ? lev(s + bv) : 0) * ny;
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const int n = bj + r * M0, m = n <= N / 2 ? n : N - n;
      fa[r] = (ok && has_a) ? ld2(sb.spec, (lvl + ja) * nxp + m) : make_double2(0.0, 0.0);
      fb[r] = (ok && has_b) ? ld2(sb.spec, (lvl + jb) * nxp + m) : make_double2(0.0, 0.0);
    }
  };
  auto first = [&]() {
    if (bact) {
      double2 x[R0];
#pragma unroll
      for (int r = 0; r < R0; ++r) {
        const bool lo = bj + r * M0 <= N / 2;
        x[r] = cadd(lo ? fa[r] : cconj(fa[r]), mul_i<1>(lo ? fb[r] : cconj(fb[r])));
      }
      dft<R0, 1>(x);
#pragma unroll
      for (int r = 0; r < R0; ++r) buf[bl * N + bj * R0 + r] = x[r];
    }
    __syncthreads();
  };
  auto rest = [&]() { fft_lines<N, R0, LT, NT, 1, false>(buf, N, 1, tws); };
  // p of the iteration's level vv at row r of the block (r = -1: the row
  // below) and column i
  auto pat = [&](int vv, int r, int i) -> double {
    const double2 z = buf[(vv * L + ((r + 1) >> 1)) * N + i];
    return (r & 1) ? z.x : z.y;
  };
  // a thread's cells of a level: c = tid + q NT
  constexpr int CPL = (CELLS + NT - 1) / NT;
  double pb[CPL];   // p of the level below the iteration's first level
  fetch(0);
  for (int s = 0; s < ns; s += LV) {
    // the velocities of the projected levels, in flight during the transform
    T uu[LV][CPL], vv[LV][CPL], ww[LV][CPL];
#pragma unroll
    for (int lv = 0; lv < LV; ++lv) {
      const int sv = s + lv;
      if (sv < ns && !(below && sv == 0)) {
        const int k = lev(sv);
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
          const int c = threadIdx.x + q * NT, j = j0 + c / N;
          if ((CELLS % NT == 0 || c < CELLS) && j < jend) {
            const long o = pidx(d, c % N, j, k);
            uu[lv][q] = gu[o];
            vv[lv][q] = gv[o];
            ww[lv][q] = gw[o];
          }
        }
      }
    }
    if (s > 0) __syncthreads();   // the lines of the previous iteration are read
    first();
    if (s + LV < ns) fetch(s + LV);
    rest();
#pragma unroll
    for (int lv = 0; lv < LV; ++lv) {
      const int sv = s + lv;
      if (sv < ns && !(below && sv == 0)) {
        const int k = lev(sv);
        const double rz = rdzf[k];
        const bool wk = !d.zb || k > 0;
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
          const int c = threadIdx.x + q * NT;
          const int r = c / N, i = c % N, j = j0 + r;
          if ((CELLS % NT == 0 || c < CELLS) && j < jend) {
            const double p0 = pat(lv, r, i);
            const double pxm = pat(lv, r, i == 0 ? N - 1 : i - 1);
            const double pym = pat(lv, r - 1, i);
            const double pzm = lv == 0 ? pb[q] : pat(lv - 1, r, i);
            const T un = (T)((double)uu[lv][q] - scale * (p0 - pxm) * rdx);
            const T vn = (T)((double)vv[lv][q] - scale * (p0 - pym) * rdy);
            const T wn = wk ? (T)((double)ww[lv][q] - scale * (p0 - pzm) * rz) : ww[lv][q];
            store_with_images(u, d, i, j, k, un, false);
            store_with_images(v, d, i, j, k, vn, false);
            store_with_images(w, d, i, j, k, wn, true);
          }
        }
      }
    }
    // p of the iteration's last level, below the next iteration's first
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      const int c = threadIdx.x + q * NT;
      if (CELLS % NT == 0 || c < CELLS) pb[q] = pat(LV - 1, c / N, c % N);
    }
  }
}

// ---------------------------------------------------------------------------
// Launchers: dispatch on the (compile-time) transform lengths.
// ---------------------------------------------------------------------------
bool fft_length_supported(int n) {
  switch (n) {
    case 8: case 16: case 32: case 64: case 96: case 128: case 256: return true;
    default: return false;
  }
}

#define OC_FFT_DISPATCH(n, MACRO) \
  switch (n) {                    \
    case 8: MACRO(8); break;      \
    case 16: MACRO(16); break;    \
    case 32: MACRO(32); break;    \
    case 64: MACRO(64); break;    \
    case 96: MACRO(96); break;    \
    case 128: MACRO(128); break;  \
    case 256: MACRO(256); break;  \
    default: return hipErrorInvalidValue; \
  }

template <class T>
hipError_t launch_poisson_x_forward(const Dims& d, const T* u, const T* v, const T* w,
                                   double inv_dt, Spacing sp, const SpecBufs& sb, hipStream_t s,
                                   const PoissonSlots* bs, int nslots) {
#define OC_LAUNCH_FX(N)                                                                    \
  {                                                                                        \
    dim3 grid((d.ny / 2 + XCfg<N>::LP - 1) / XCfg<N>::LP, d.nz, nslots);                  \
    hipLaunchKernelGGL((fwd_x_kernel<T, N>), grid, dim3(NT), 0, s, d, u, v, w, inv_dt,    \
                       sp.rdx, sp.rdy, sp.rdzc, sb, bs, (const double*)nullptr);           \
  }
  OC_FFT_DISPATCH(d.nx, OC_LAUNCH_FX)
#undef OC_LAUNCH_FX
  return hipGetLastError();
}

hipError_t launch_poisson_x_forward_dense(const Dims& d, const double* src, const SpecBufs& sb,
                                          hipStream_t s) {
#define OC_LAUNCH_FXD(N)                                                                   \
  {                                                                                        \
    dim3 grid((d.ny / 2 + XCfg<N>::LP - 1) / XCfg<N>::LP, d.nz, 1);                       \
    hipLaunchKernelGGL((fwd_x_kernel<double, N>), grid, dim3(NT), 0, s, d,                \
                       (const double*)nullptr, (const double*)nullptr,                     \
                       (const double*)nullptr, 0.0, 0.0, 0.0, (const double*)nullptr, sb,  \
                       (const PoissonSlots*)nullptr, src);                                 \
  }
  OC_FFT_DISPATCH(d.nx, OC_LAUNCH_FXD)
#undef OC_LAUNCH_FXD
  return hipGetLastError();
}

hipError_t launch_poisson_y(const Dims& d, const SpecBufs& sb, int dir, hipStream_t s,
                            const PoissonSlots* bs, int nslots) {
#define OC_LAUNCH_Y(N)                                                                     \
  {                                                                                        \
    dim3 grid((sb.nxh + YZCfg<N>::W - 1) / YZCfg<N>::W, d.nz, nslots);                    \
    if (dir < 0)                                                                           \
      hipLaunchKernelGGL((y_kernel<N, -1>), grid, dim3(NT), 0, s, d, sb, bs);             \
    else                                                                                   \
      hipLaunchKernelGGL((y_kernel<N, 1>), grid, dim3(NT), 0, s, d, sb, bs);              \
  }
  OC_FFT_DISPATCH(d.ny, OC_LAUNCH_Y)
#undef OC_LAUNCH_Y
  return hipGetLastError();
}

hipError_t launch_poisson_spectral(const Dims& d, const SpecBufs& sb, hipStream_t s,
                                   const PoissonSlots* bs, int nslots) {
  const double norm = 1.0 / ((double)d.nx * d.ny * d.nz);
#define OC_LAUNCH_Z(N)                                                                     \
  {                                                                                        \
    dim3 grid((sb.nxh + YZCfg<N>::W - 1) / YZCfg<N>::W, d.ny, nslots);                    \
    if (d.zb)                                                                              \
      hipLaunchKernelGGL((z_kernel<N, true>), grid, dim3(NT), 0, s, d, sb, norm, bs);     \
    else                                                                                   \
      hipLaunchKernelGGL((z_kernel<N, false>), grid, dim3(NT), 0, s, d, sb, norm, bs);    \
  }
  OC_FFT_DISPATCH(d.nz, OC_LAUNCH_Z)
#undef OC_LAUNCH_Z
  return hipGetLastError();
}

hipError_t launch_poisson_tridiag(const Dims& d, const SpecBufs& sb, const double* lo,
                                  const double* up, const double* dzc, const double* dzf,
                                  hipStream_t s) {
  if (d.nz > PCR_NMAX || !d.zb) return hipErrorInvalidValue;
  const double norm = 1.0 / ((double)d.nx * d.ny);
  dim3 grid((sb.nxh + PCR_W - 1) / PCR_W, d.ny);
  hipLaunchKernelGGL(z_tridiag_kernel, grid, dim3(NT), 0, s, d, sb, norm, lo, up, dzc, dzf);
  return hipGetLastError();
}

hipError_t launch_poisson_x_inverse(const Dims& d, const SpecBufs& sb, hipStream_t s,
                                    const PoissonSlots* bs, int nslots) {
#define OC_LAUNCH_XI(N)                                                                    \
  {                                                                                        \
    dim3 grid((d.ny / 2 + XCfg<N>::LP - 1) / XCfg<N>::LP, d.nz, nslots);                  \
    hipLaunchKernelGGL((inv_x_kernel<N>), grid, dim3(NT), 0, s, d, sb, bs,                \
                       (const double*)nullptr, (double*)nullptr);                          \
  }
  OC_FFT_DISPATCH(d.nx, OC_LAUNCH_XI)
#undef OC_LAUNCH_XI
  return hipGetLastError();
}

// Chunks per column of the fused inverse pass: a workgroup's time grows
// with its levels (one more than its chunk holds: the level below), and
// the grid runs in rounds of `slots` resident workgroups, so take the
// count that minimises rounds x (levels per chunk + 1).
static int px_chunks(int nz, int ncol, int slots) {
  if (slots <= 0) return 1;
  int best = 1;
  long best_cost = -1;
  for (int n = 1; n <= nz; ++n) {
    const long rounds = ((long)ncol * n + slots - 1) / slots;
    const long cost = rounds * ((nz + n - 1) / n + 1);
    if (best_cost < 0 || cost < best_cost) { best = n; best_cost = cost; }
  }
  return best;
}

// Workgroups of a kernel (NT threads) resident on the whole device at once
// (0 if the runtime cannot say).
static int resident_slots(const void* kernel) {
  int dev = 0, ncu = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, NT, 0) != hipSuccess)
    return 0;
  return std::max(0, ncu * per_cu);
}

template <class T>
hipError_t launch_poisson_x_inverse_project(const Dims& d, const SpecBufs& sb, T* u, T* v, T* w,
                                            double scale, const Spacing& sp, hipStream_t s,
                                            const PoissonSlots* bs, int nslots) {
#define OC_LAUNCH_XIP(N)                                                                   \
  {                                                                                        \
    constexpr int RB = 2 * PXCfg<N>::L - 1;                                                \
    const int nblk = (d.ny + RB - 1) / RB, rb = (d.ny + nblk - 1) / nblk;                  \
    static const int slots = resident_slots((const void*)inv_x_project_kernel<T, N>);     \
    const int ncol = nblk * nslots, nch = px_chunks(d.nz, ncol, slots);                    \
    hipLaunchKernelGGL((inv_x_project_kernel<T, N>), dim3(ncol * nch), dim3(NT), 0, s, d, sb, \
                       u, v, w, scale, sp.rdx, sp.rdy, sp.rdzf, rb, nblk, nch, bs);        \
  }
  OC_FFT_DISPATCH(d.nx, OC_LAUNCH_XIP)
#undef OC_LAUNCH_XIP
  return hipGetLastError();
}

hipError_t launch_poisson_x_inverse_dot(const Dims& d, const SpecBufs& sb, const double* rdot,
                                        double* part, int part_cap, int* npart, hipStream_t s) {
#define OC_LAUNCH_XID(N)                                                                   \
  {                                                                                        \
    dim3 grid((d.ny / 2 + XCfg<N>::LP - 1) / XCfg<N>::LP, d.nz, 1);                       \
    *npart = (int)(grid.x * grid.y);                                                       \
    if (*npart > part_cap) return hipErrorInvalidValue;                                    \
    hipLaunchKernelGGL((inv_x_kernel<N>), grid, dim3(NT), 0, s, d, sb,                    \
                       (const PoissonSlots*)nullptr, rdot, part);                          \
  }
  OC_FFT_DISPATCH(d.nx, OC_LAUNCH_XID)
#undef OC_LAUNCH_XID
  return hipGetLastError();
}

template <class T>
hipError_t launch_project(const Dims& d, T* u, T* v, T* w, double scale, const Spacing& sp,
                          const double* p, hipStream_t s, const PoissonSlots* bs, int nslots,
                          const T* mask) {
  const unsigned nb = (unsigned)(((d.nx + PJ_X - 1) / PJ_X) * ((d.ny + PJ_Y - 1) / PJ_Y));
  hipLaunchKernelGGL(project_kernel<T>, dim3(nb, (d.nz + PJ_KC - 1) / PJ_KC, nslots),
                     dim3(PJ_X * PJ_Y), 0, s, d, u, v, w, scale, sp.rdx, sp.rdy, sp.rdzf, p, bs,
                     mask);
  return hipGetLastError();
}

template hipError_t launch_poisson_x_forward<float>(const Dims&, const float*, const float*,
                                                    const float*, double, Spacing,
                                                    const SpecBufs&, hipStream_t,
                                                    const PoissonSlots*, int);
template hipError_t launch_poisson_x_forward<double>(const Dims&, const double*, const double*,
                                                     const double*, double, Spacing,
                                                     const SpecBufs&, hipStream_t,
                                                     const PoissonSlots*, int);
template hipError_t launch_poisson_x_inverse_project<float>(const Dims&, const SpecBufs&, float*,
                                                            float*, float*, double,
                                                            const Spacing&, hipStream_t,
                                                            const PoissonSlots*, int);
template hipError_t launch_poisson_x_inverse_project<double>(const Dims&, const SpecBufs&,
                                                             double*, double*, double*, double,
                                                             const Spacing&, hipStream_t,
                                                             const PoissonSlots*, int);
template hipError_t launch_project<float>(const Dims&, float*, float*, float*, double,
                                          const Spacing&, const double*, hipStream_t,
                                          const PoissonSlots*, int, const float*);
template hipError_t launch_project<double>(const Dims&, double*, double*, double*, double,
                                           const Spacing&, const double*, hipStream_t,
                                           const PoissonSlots*, int, const double*);

}  // namespace oc
