// Symmetric quad-tile engine kernels on a 6x6 tile grid: |Z| = 9..12 (d <= 24) at k = 11..23,
// classes kClsSqt + k - 11.
#include <hip/hip_runtime.h>

#include <utility>

#include "gbs_sqt_engine.h"

namespace gbs {

template <int... I>
static void fill_sqt(EngineVariant* tab, std::integer_sequence<int, I...>) {
  ((tab[kClsSqt + I] = EngineVariant{reinterpret_cast<const void*>(&sqt_engine_kernel<I + 11, 6>), kThreads, kSqtKind,
                                     6}),
   ...);
}

void register_sqt_engines(EngineVariant* tab) { fill_sqt(tab, std::make_integer_sequence<int, 13>{}); }

}  // namespace gbs
