// Subset-engine kernels: quad engine on a 4x4 tile grid for |Z| = 7, 8 (classes kClsGrid4 + k - 5,
// k = 5..23).
#include <hip/hip_runtime.h>

#include <utility>

#include "gbs_engine_common.h"
#include "gbs_quad_engine.h"

namespace gbs {

template <int... I>
static void fill_grid4(EngineVariant* tab, std::integer_sequence<int, I...>) {
  ((tab[kClsGrid4 + I] = EngineVariant{reinterpret_cast<const void*>(&quad_grid_kernel<I + 5, 4>), kThreads,
                                       kQuadKind, 4}),
   ...);
}

void register_grid4_engines(EngineVariant* tab) { fill_grid4(tab, std::make_integer_sequence<int, 19>{}); }

}  // namespace gbs
