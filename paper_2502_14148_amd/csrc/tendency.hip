// Launchers of the fused tendency + RK3 kernel (tendency_tile.h): WENO5
// (stencil radius 3) for single models and for ensembles of models in one
// launch; WENO7 and WENO9 are instantiated in tendency_r4.hip and
// tendency_r5.hip.
#include "tendency_tile.h"

// Column tile of the tendency kernel (x by y); 8 x 8 tiles serve grids whose
// sizes the wide tile does not divide.
#ifndef OC_TEND_TX
#define OC_TEND_TX 32
#endif
#ifndef OC_TEND_TY
#define OC_TEND_TY 8
#endif


namespace oc {

namespace tz {

// An ensemble of models in one launch.  Work items (member, tile) come from
// `items`; PERSIST = false: one workgroup per item; PERSIST = true: a grid of
// resident workgroups takes items from the atomic counter until the list is
// exhausted (every workgroup leaves the loop once the counter passes nitems).
template <class T, int SCHEME, int NTR, int TX, int TY, bool PERSIST>
__global__ void __launch_bounds__(TX * TY)
    __attribute__((amdgpu_waves_per_eu(TendWaves<T, 3>::value)))
    tendency_ensemble(const EnsMember<T>* __restrict__ mem, const int2* __restrict__ items,
                  int nitems, int* __restrict__ counter, int parity, int stage) {
  if (!PERSIST) {
    const int2 it = items[blockIdx.x];
    const EnsMember<T>& M = mem[it.x];
    tendency_tile<T, SCHEME, NTR, TX, TY, 3>(M.d, M.fs[parity], M.P[stage], M.nbx, M.nby, M.nbz,
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
    tendency_tile<T, SCHEME, NTR, TX, TY, 3>(M.d, M.fs[parity], M.P[stage], M.nbx, M.nby, M.nbz,
                                             M.kc, it.y);
    __syncthreads();  // LDS and s_item are reused by the next item
  }
}

__global__ void reset_counter_kernel(int* counter) { counter[0] = 0; }

}  // namespace tz

// FP32 WENO5 with at most two tracers on rows that hold whole 64-column
// tiles: 64 x 8 tiles (fewer edge faces and halo columns per cell than
// 32 x 8: 2.8 % faster at 256^3).  With more tracers, or in FP64, the
// planes of a 64 x 8 tile leave room for only one workgroup per CU, so those
// keep 32 x 8.
template <class T, int TX, int TY>
hipError_t launch_weno5(const Dims& d, const FieldSet<T>& fs, const TendParams<T>& p, int scheme,
                        hipStream_t s) {
  if constexpr (sizeof(T) == 4) {
    if (p.ntr <= 2 && d.nx % 64 == 0 && d.ny % 8 == 0)
      return launch_tendency_radius<T, 3, 64, 8, 2>(d, fs, p, scheme, s);
  }
  return launch_tendency_radius<T, 3, TX, TY>(d, fs, p, scheme, s);
}

template <class T>
hipError_t launch_tendency_fast(const Dims& d, const FieldSet<T>& fs, const TendParams<T>& p,
                                int advection, hipStream_t s) {
  constexpr int TX = OC_TEND_TX, TY = OC_TEND_TY;
  switch (advection) {
    case OC_ADV_NONE:
      return launch_weno5<T, TX, TY>(d, fs, p, tz::SCHEME_NONE, s);
    case OC_ADV_WENO5Z:
      return launch_weno5<T, TX, TY>(d, fs, p, tz::SCHEME_WENOZ, s);
    case OC_ADV_WENO5_LINEAR:
      return launch_weno5<T, TX, TY>(d, fs, p, tz::SCHEME_LINEAR, s);
    case OC_ADV_WENO7Z: return launch_tendency_r4<T>(d, fs, p, tz::SCHEME_WENOZ, s);
    case OC_ADV_WENO7_LINEAR: return launch_tendency_r4<T>(d, fs, p, tz::SCHEME_LINEAR, s);
    case OC_ADV_WENO9Z: return launch_tendency_r5<T>(d, fs, p, tz::SCHEME_WENOZ, s);
    case OC_ADV_WENO9_LINEAR: return launch_tendency_r5<T>(d, fs, p, tz::SCHEME_LINEAR, s);
    default: return hipErrorInvalidValue;
  }
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
