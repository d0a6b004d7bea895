// Fused s-stage RKL tau-step (placeholder until the LDS-tiled kernel lands).
#include "kernels.h"

namespace rkl {

template <typename T>
bool launch_fused_tau(const LevelView<T>&, const T*, const T*, T*, int, const StageCoef*, double*,
                      hipStream_t) {
  return false;
}

template bool launch_fused_tau<double>(const LevelView<double>&, const double*, const double*, double*,
                                       int, const StageCoef*, double*, hipStream_t);
template bool launch_fused_tau<float>(const LevelView<float>&, const float*, const float*, float*, int,
                                      const StageCoef*, double*, hipStream_t);

}  // namespace rkl
