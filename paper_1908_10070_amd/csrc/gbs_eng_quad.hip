// Subset-engine kernels: quad engine for |Z| <= 6 (classes kClsQuad + k - 1, k = 1..23).
#include <hip/hip_runtime.h>

#include <utility>

#include "gbs_engine_common.h"
#include "gbs_quad_engine.h"

namespace gbs {

template <int... I>
static void fill_quad(EngineVariant* tab, std::integer_sequence<int, I...>) {
  ((tab[kClsQuad + I] = EngineVariant{reinterpret_cast<const void*>(&quad_engine_kernel<I + 1>), kThreads,
                                      kQuadKind, 3}),
   ...);
}

void register_quad_engines(EngineVariant* tab) { fill_quad(tab, std::make_integer_sequence<int, 23>{}); }

}  // namespace gbs
