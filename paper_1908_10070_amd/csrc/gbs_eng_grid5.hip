// Subset-engine kernels: quad engine on a 5x5 tile grid for |Z| = 9, 10 (classes kClsGrid5 + k - 9,
// k = 9..23).
#include <hip/hip_runtime.h>

#include <utility>

#include "gbs_engine_common.h"
#include "gbs_quad_engine.h"

namespace gbs {

template <int... I>
static void fill_grid5(EngineVariant* tab, std::integer_sequence<int, I...>) {
  ((tab[kClsGrid5 + I] = EngineVariant{reinterpret_cast<const void*>(&quad_grid_kernel<I + 9, 5>), kThreads,
                                       kQuadKind, 5}),
   ...);
}

void register_grid5_engines(EngineVariant* tab) { fill_grid5(tab, std::make_integer_sequence<int, 15>{}); }

}  // namespace gbs
