// Subset-engine kernels: strip engine (6 tile rows) for |Z| = 11, 12 and k = 11..16 (classes
// kClsStrip + k - 11).
#include <hip/hip_runtime.h>

#include <utility>

#include "gbs_engine_common.h"
#include "gbs_strip_engine.h"

namespace gbs {

template <int... I>
static void fill_strip(EngineVariant* tab, std::integer_sequence<int, I...>) {
  ((tab[kClsStrip + I] = EngineVariant{reinterpret_cast<const void*>(&strip_engine_kernel<I + 11, 6, 6>), kThreads,
                                       kStripKind, 1}),
   ...);
}

void register_strip_engines(EngineVariant* tab) { fill_strip(tab, std::make_integer_sequence<int, 6>{}); }

}  // namespace gbs
