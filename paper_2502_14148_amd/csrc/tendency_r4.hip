// Fused tendency + RK3 kernel with a stencil of radius 4 (WENO7; centred
// order-6 advecting velocity), single models.
#include "tendency_tile.h"

namespace oc {

template <class T>
hipError_t launch_tendency_r4(const Dims& d, const FieldSet<T>& fs, const TendParams<T>& p,
                              int scheme, hipStream_t s) {
  return launch_tendency_radius<T, 4, 32, 8>(d, fs, p, scheme, s);
}

template hipError_t launch_tendency_r4<float>(const Dims&, const FieldSet<float>&,
                                              const TendParams<float>&, int, hipStream_t);
template hipError_t launch_tendency_r4<double>(const Dims&, const FieldSet<double>&,
                                               const TendParams<double>&, int, hipStream_t);

}  // namespace oc
