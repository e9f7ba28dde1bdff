// Double-double subset-engine kernels (the accuracy mode): classes kClsDd + T - 1 for subsets with
// 2|Z| <= 16 T, T = 1, 2, 3, any k.
#include <hip/hip_runtime.h>

#include "gbs_dd_engine.h"

namespace gbs {

void register_dd_engines(EngineVariant* tab) {
  tab[kClsDd + 0] = EngineVariant{reinterpret_cast<const void*>(&dd_engine_kernel<1>), kDdThreads, kDdKind, 1};
  tab[kClsDd + 1] = EngineVariant{reinterpret_cast<const void*>(&dd_engine_kernel<2>), kDdThreads, kDdKind, 2};
  tab[kClsDd + 2] = EngineVariant{reinterpret_cast<const void*>(&dd_engine_kernel<3>), kDdThreads, kDdKind, 3};
}

}  // namespace gbs
