// Baroclinic part of the hydrostatic model on a latitude-longitude grid
// (hydrostatic-model subsection and hydrostatic time-discretisation appendix
// of arXiv 2502.14148) on gfx950.
//
// Discretisation (C-grid on the thin spherical shell, uniform dz, periodic
// longitude, walls at the latitude edges and in z):
//   * w at z faces from the floor up, w_{k+1} = w_k - dz div_h(u_h)_k;
//   * hydrostatic pressure p_k = -dz (b_k / 2 + sum_{m > k} b_m) (dp/dz = b,
//     p = 0 at the surface); only its horizontal differences enter, so the
//     columns integrate differences of b;
//   * vector-invariant momentum advection: vertical vorticity zeta at cell
//     corners from the metric circulation of the dual cell; + zeta_hat Vbar at
//     u points (zeta reconstructed by WENO along y, upwinded by the
//     four-point average Vbar of v), - zeta_hat Ubar at v points (along x);
//     kinetic energy at centres differenced to the faces; vertical advection
//     d(W q)/dz - q dW/dz with W = w averaged to the column and q
//     reconstructed by WENO along z;
//   * tracers in flux form with the shell's face areas and cell volumes,
//     WENO in every direction;
//   * f = 2 Omega sin(latitude of the point) times the four-point average of
//     the other component; explicit vertical viscosity/diffusivity with the
//     kinematic wind stress as surface momentum flux;
//   * advective fluxes vanish on the floor; through the moving surface they
//     carry the top cell's own value (a uniform tracer stays uniform);
//   * QAB2: X~ = X + dt [(3/2 + chi) G^n - (1/2 + chi) G^{n-1}], chi = 0.1
//     (chi = -1/2 on a first step), and the slow forcing of the barotropic
//     mode Gbar = sum_k dz [...] accumulated in FP64 per column.
//
// Layout: halo-padded fields (halo width h = 3), x fastest; v on the ny + 1 y faces (face
// ny in the first upper halo row), w on the nz + 1 z faces (face nz in the
// first upper halo plane).  Kernels: the column scans (zeta, w, pressure
// gradients), the tendency + QAB2 kernel (one thread per column, register
// windows along z), and the halo fill of the prognostic fields.
#include "oc_internal.h"
#include "weno_dev.h"

namespace oc {

namespace {

constexpr int HTX = 64, HTY = 4;

template <class T>
__global__ void __launch_bounds__(HTX * HTY) hydro_diag_kernel(HydroBufs<T> a) {
  const Dims d = a.d;
  const int i = -2 + (int)(blockIdx.x * HTX + threadIdx.x);
  const int j = -2 + (int)(blockIdx.y * HTY + threadIdx.y);
  if (i > d.nx + 2 || j > d.ny + 2) return;
  const HydroMetric& m = a.m;
  const T dy = (T)m.dy;
  const double dz = m.dz;
  const long sy = d.sy, sz = d.sz;
  const long c0 = pidx(d, i, j, 0);

  // vertical vorticity at corner (x face i, y face j)
  {
    const T dxj = (T)m.dxc[j + d.h], dxjm = (T)m.dxc[j - 1 + d.h];
    const T rza = T(1) / (T)m.areaz[j + d.h];
    long c = c0;
    for (int k = 0; k < d.nz; ++k, c += sz) {
      const T circ = dy * (a.v[c] - a.v[c - 1]) - (dxj * a.u[c] - dxjm * a.u[c - sy]);
      a.zeta[c] = circ * rza;
    }
  }

  // w on the faces of columns i in [-1, nx), j in [0, ny)
  if (i >= -1 && i < d.nx && j >= 0 && j < d.ny) {
    const T dxf0 = (T)m.dxf[j + d.h], dxf1 = (T)m.dxf[j + 1 + d.h];
    const T rar = T(1) / (T)m.areac[j + d.h];
    double wacc = 0.0;
    long c = c0;
    a.w[c] = T(0);
    for (int k = 0; k < d.nz; ++k, c += sz) {
      const T div = (dy * (a.u[c + 1] - a.u[c]) + (dxf1 * a.v[c + sy] - dxf0 * a.v[c])) * rar;
      wacc -= dz * (double)div;
      a.w[c + sz] = (T)wacc;
    }
  }

  // pressure-gradient terms, integrated from the surface down:
  //   px = (p_i - p_{i-1}) / dx at u points, py = (p_j - p_{j-1}) / dy at v points
  if (i >= 0 && i < d.nx && j >= 0 && j < d.ny) {
    const T rdx = T(1) / (T)m.dxc[j + d.h];
    const T rdy = T(1) / dy;
    const bool vpt = j > 0;
    double sx = 0.0, sy_ = 0.0;
    long c = c0 + (long)(d.nz - 1) * sz;
    for (int k = d.nz - 1; k >= 0; --k, c -= sz) {
      const T b = a.ga * (a.t[c] - a.tref) - a.gb * (a.s[c] - a.sref);
      const T bw = a.ga * (a.t[c - 1] - a.tref) - a.gb * (a.s[c - 1] - a.sref);
      const double dbx = (double)(b - bw);
      a.px[c] = (T)(-dz * (0.5 * dbx + sx)) * rdx;
      sx += dbx;
      if (vpt) {
        const T bs = a.ga * (a.t[c - sy] - a.tref) - a.gb * (a.s[c - sy] - a.sref);
        const double dby = (double)(b - bs);
        a.py[c] = (T)(-dz * (0.5 * dby + sy_)) * rdy;
        sy_ += dby;
      }
    }
  }
}

template <class T, int SCHEME>
__device__ inline T rec(T m3, T m2, T m1, T p0, T p1, T p2, T vel, T eps) {
  if (SCHEME == tz::SCHEME_NONE) return T(0);
  return tz::rec6<T, SCHEME>(m3, m2, m1, p0, p1, p2, vel, eps);
}

template <class T, int SCHEME>
__global__ void __launch_bounds__(HTX * HTY) hydro_tend_kernel(HydroBufs<T> a, HydroStep<T> st) {
  const Dims d = a.d;
  const int i = (int)(blockIdx.x * HTX + threadIdx.x);
  const int j = (int)(blockIdx.y * HTY + threadIdx.y);
  if (i >= d.nx || j >= d.ny) return;
  const HydroMetric& m = a.m;
  const long sy = d.sy, sz = d.sz;
  const bool vpt = j > 0;     // v point on y face j (face 0 is a wall)
  const T eps = a.eps;
  const T dy = (T)m.dy, rdy = T(1) / dy;
  const T dz = (T)m.dz, rdz = T(1) / dz;
  const T rdxc = T(1) / (T)m.dxc[j + d.h];
  const T fc = (T)m.fc[j + d.h], ff = (T)m.ff[j + d.h];
  const T Ax = dy * dz;
  const T Ay0 = (T)m.dxf[j + d.h] * dz, Ay1 = (T)m.dxf[j + 1 + d.h] * dz;
  const T Az = (T)m.areac[j + d.h];
  const T rvol = T(1) / (Az * dz);
  const T nu = a.nu, kappa = a.kappa;
  const T dt = st.dt, a1 = st.a1, a0 = st.a0;
  const bool first = st.first != 0;

  const long c0 = pidx(d, i, j, 0);
  // register windows along z: q[o] = q_{k-2+o}
  T uw[6], vw[6], tw[6], sw[6];
#pragma unroll
  for (int o = 0; o < 6; ++o) {
    const long c = c0 + (long)(o - 2) * sz;
    uw[o] = a.u[c];
    vw[o] = a.v[c];
    tw[o] = a.t[c];
    sw[o] = a.s[c];
  }
  // quantities on face k carried up from the level below (floor: zero)
  T Fu = T(0), Fv = T(0), Ft = T(0), Fs = T(0), Nu = T(0), Nv = T(0);
  T Wu = T(0), Wv = T(0);
  double gu = 0.0, gv = 0.0;
  const long c2 = (long)j * d.nx + i;

  for (int k = 0; k < d.nz; ++k) {
    const long c = c0 + (long)k * sz;
    const long cf = c + sz;  // face k + 1
    const T w_c = a.w[cf];
    const T Wu1 = T(0.5) * (a.w[cf - 1] + w_c);
    const T Wv1 = vpt ? T(0.5) * (a.w[cf - sy] + w_c) : T(0);
    // fluxes through face k + 1
    T Fu1, Fv1, Ft1, Fs1, Nu1, Nv1;
    if (k + 1 < d.nz) {
      Fu1 = Wu1 * rec<T, SCHEME>(uw[0], uw[1], uw[2], uw[3], uw[4], uw[5], Wu1, eps);
      Fv1 = Wv1 * rec<T, SCHEME>(vw[0], vw[1], vw[2], vw[3], vw[4], vw[5], Wv1, eps);
      Ft1 = (w_c * rec<T, SCHEME>(tw[0], tw[1], tw[2], tw[3], tw[4], tw[5], w_c, eps) -
             kappa * (tw[3] - tw[2]) * rdz) * Az;
      Fs1 = (w_c * rec<T, SCHEME>(sw[0], sw[1], sw[2], sw[3], sw[4], sw[5], w_c, eps) -
             kappa * (sw[3] - sw[2]) * rdz) * Az;
      Nu1 = nu * (uw[3] - uw[2]) * rdz;
      Nv1 = nu * (vw[3] - vw[2]) * rdz;
    } else {
      Fu1 = Wu1 * uw[2];
      Fv1 = Wv1 * vw[2];
      Ft1 = w_c * tw[2] * Az;
      Fs1 = w_c * sw[2] * Az;
      Nu1 = (T)a.taux[c2];
      Nv1 = (T)a.tauy[c2];
    }

    const T u_c = uw[2], v_c = vw[2];
    const T u_e = a.u[c + 1], u_w = a.u[c - 1];
    const T v_w = a.v[c - 1], v_n = a.v[c + sy], v_nw = a.v[c - 1 + sy];
    const T ke = T(0.25) * (u_c * u_c + u_e * u_e + v_c * v_c + v_n * v_n);

    // ---- u point (x face i, row j)
    {
      const T vb = T(0.25) * (v_w + v_c + v_nw + v_n);
      const T zh = rec<T, SCHEME>(a.zeta[c - 2 * sy], a.zeta[c - sy], a.zeta[c], a.zeta[c + sy],
                                  a.zeta[c + 2 * sy], a.zeta[c + 3 * sy], vb, eps);
      const T ke_w = T(0.25) * (u_w * u_w + u_c * u_c + v_w * v_w + v_nw * v_nw);
      T G = zh * vb + fc * vb;
      G -= (ke - ke_w) * rdxc;
      G -= a.px[c];
      G -= (Fu1 - Fu) * rdz - u_c * (Wu1 - Wu) * rdz;
      G += (Nu1 - Nu) * rdz;
      T comb = a1 * G;
      if (!first) comb -= a0 * a.Gu[c];
      a.Gu[c] = G;
      a.uo[c] = u_c + dt * comb;
      gu += (double)comb;
    }
    // ---- v point (x centre i, y face j)
    if (vpt) {
      const T u_s = a.u[c - sy], u_se = a.u[c - sy + 1];
      const T v_s = a.v[c - sy];
      const T ub = T(0.25) * (u_s + u_se + u_c + u_e);
      const T zh = rec<T, SCHEME>(a.zeta[c - 2], a.zeta[c - 1], a.zeta[c], a.zeta[c + 1],
                                  a.zeta[c + 2], a.zeta[c + 3], ub, eps);
      const T ke_s = T(0.25) * (u_s * u_s + u_se * u_se + v_s * v_s + v_c * v_c);
      T G = -(zh * ub) - ff * ub;
      G -= (ke - ke_s) * rdy;
      G -= a.py[c];
      G -= (Fv1 - Fv) * rdz - v_c * (Wv1 - Wv) * rdz;
      G += (Nv1 - Nv) * rdz;
      T comb = a1 * G;
      if (!first) comb -= a0 * a.Gv[c];
      a.Gv[c] = G;
      a.vo[c] = v_c + dt * comb;
      gv += (double)comb;
    } else {
      a.Gv[c] = T(0);
      a.vo[c] = T(0);
    }
    // ---- tracers at centre (i, j)
    {
      const bool south = j > 0, north = j + 1 < d.ny;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const T* f = q ? a.s : a.t;
        const T cc = q ? sw[2] : tw[2];
        const T cm3 = f[c - 3], cm2 = f[c - 2], cm1 = f[c - 1];
        const T cp1 = f[c + 1], cp2 = f[c + 2], cp3 = f[c + 3];
        const T fx0 = u_c * rec<T, SCHEME>(cm3, cm2, cm1, cc, cp1, cp2, u_c, eps) * Ax;
        const T fx1 = u_e * rec<T, SCHEME>(cm2, cm1, cc, cp1, cp2, cp3, u_e, eps) * Ax;
        const T sm3 = f[c - 3 * sy], sm2 = f[c - 2 * sy], sm1 = f[c - sy];
        const T sp1 = f[c + sy], sp2 = f[c + 2 * sy], sp3 = f[c + 3 * sy];
        const T fy0 = south ? v_c * rec<T, SCHEME>(sm3, sm2, sm1, cc, sp1, sp2, v_c, eps) * Ay0
                            : T(0);
        const T fy1 = north ? v_n * rec<T, SCHEME>(sm2, sm1, cc, sp1, sp2, sp3, v_n, eps) * Ay1
                            : T(0);
        const T Fz0 = q ? Fs : Ft, Fz1 = q ? Fs1 : Ft1;
        const T G = -((fx1 - fx0) + (fy1 - fy0) + (Fz1 - Fz0)) * rvol;
        T* Gq = q ? a.Gs : a.Gt;
        T comb = a1 * G;
        if (!first) comb -= a0 * Gq[c];
        Gq[c] = G;
        (q ? a.so : a.to)[c] = cc + dt * comb;
      }
    }

    // ---- carry face k + 1 up; shift the windows
    Fu = Fu1; Fv = Fv1; Ft = Ft1; Fs = Fs1; Nu = Nu1; Nv = Nv1; Wu = Wu1; Wv = Wv1;
#pragma unroll
    for (int o = 0; o < 5; ++o) {
      uw[o] = uw[o + 1];
      vw[o] = vw[o + 1];
      tw[o] = tw[o + 1];
      sw[o] = sw[o + 1];
    }
    if (k + 1 < d.nz) {
      const long cn = c + 4 * sz;  // level k + 4 (at most nz + 2, inside the halo)
      uw[5] = a.u[cn];
      vw[5] = a.v[cn];
      tw[5] = a.t[cn];
      sw[5] = a.s[cn];
    }
  }
  a.gub[c2] = gu * m.dz;
  a.gvb[c2] = vpt ? gv * m.dz : 0.0;
}

// Halo images of the prognostic fields: x periodic; y walls with even
// mirrors for u, T, S and an odd mirror about the wall faces for v (whose
// wall faces are set to zero); z walls with even mirrors.  One thread per
// padded point; interior points return at once.
template <class T>
__global__ void hydro_halo_kernel(Dims d, T* u, T* v, T* t, T* s) {
  const long n = (long)d.px * d.py * d.pz;
  const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int pi = (int)(p % d.px);
  const int pj = (int)((p / d.px) % d.py);
  const int pk = (int)(p / ((long)d.px * d.py));
  const int i = pi - d.h, j = pj - d.h, k = pk - d.h;
  const bool xin = i >= 0 && i < d.nx, yin = j >= 0 && j < d.ny, zin = k >= 0 && k < d.nz;
  const bool vwall = (j == 0 || j == d.ny);
  const bool c_interior = xin && yin && zin;
  const bool v_interior = xin && zin && j > 0 && j < d.ny;
  if (c_interior && v_interior) return;
  const int si = (i < 0) ? i + d.nx : (i >= d.nx ? i - d.nx : i);
  const int sk = (k < 0) ? -1 - k : (k >= d.nz ? 2 * d.nz - 1 - k : k);
  if (!c_interior) {
    const int sj = (j < 0) ? -1 - j : (j >= d.ny ? 2 * d.ny - 1 - j : j);
    const long src = pidx(d, si, sj, sk);
    u[p] = u[src];
    t[p] = t[src];
    s[p] = s[src];
  }
  if (!v_interior) {
    if (vwall) {
      v[p] = T(0);
    } else {
      const int sj = (j < 0) ? -j : (j > d.ny ? 2 * d.ny - j : j);
      const T sg = (j < 0 || j > d.ny) ? T(-1) : T(1);
      v[p] = sg * v[pidx(d, si, sj, sk)];
    }
  }
}

}  // namespace

template <class T>
hipError_t launch_hydro_diag(const HydroBufs<T>& a, hipStream_t s) {
  dim3 grid((a.d.nx + 5 + HTX - 1) / HTX, (a.d.ny + 5 + HTY - 1) / HTY);
  hipLaunchKernelGGL(hydro_diag_kernel<T>, grid, dim3(HTX, HTY), 0, s, a);
  return hipGetLastError();
}

template <class T>
hipError_t launch_hydro_tendency(const HydroBufs<T>& a, const HydroStep<T>& st, int scheme,
                                 hipStream_t s) {
  dim3 grid((a.d.nx + HTX - 1) / HTX, (a.d.ny + HTY - 1) / HTY);
  switch (scheme) {
    case tz::SCHEME_NONE:
      hipLaunchKernelGGL((hydro_tend_kernel<T, tz::SCHEME_NONE>), grid, dim3(HTX, HTY), 0, s, a, st);
      break;
    case tz::SCHEME_LINEAR:
      hipLaunchKernelGGL((hydro_tend_kernel<T, tz::SCHEME_LINEAR>), grid, dim3(HTX, HTY), 0, s, a,
                         st);
      break;
    default:
      hipLaunchKernelGGL((hydro_tend_kernel<T, tz::SCHEME_WENOZ>), grid, dim3(HTX, HTY), 0, s, a,
                         st);
  }
  return hipGetLastError();
}

template <class T>
hipError_t launch_hydro_halo(const Dims& d, T* u, T* v, T* t, T* sf, hipStream_t s) {
  const long n = (long)d.px * d.py * d.pz;
  hipLaunchKernelGGL(hydro_halo_kernel<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d, u,
                     v, t, sf);
  return hipGetLastError();
}

template hipError_t launch_hydro_diag<float>(const HydroBufs<float>&, hipStream_t);
template hipError_t launch_hydro_diag<double>(const HydroBufs<double>&, hipStream_t);
template hipError_t launch_hydro_tendency<float>(const HydroBufs<float>&, const HydroStep<float>&,
                                                 int, hipStream_t);
template hipError_t launch_hydro_tendency<double>(const HydroBufs<double>&,
                                                  const HydroStep<double>&, int, hipStream_t);
template hipError_t launch_hydro_halo<float>(const Dims&, float*, float*, float*, float*,
                                             hipStream_t);
template hipError_t launch_hydro_halo<double>(const Dims&, double*, double*, double*, double*,
                                              hipStream_t);

}  // namespace oc
