// Symmetric quad-tile engine kernels on a 7x7 tile grid: |Z| = 13, 14 (d <= 28) at k = 13..23,
// classes kClsSqt7 + k - 13.
#include <hip/hip_runtime.h>

#include <utility>

#include "gbs_sqt_engine.h"

namespace gbs {

template <int... I>
static void fill_sqt7(EngineVariant* tab, std::integer_sequence<int, I...>) {
  ((tab[kClsSqt7 + I] = EngineVariant{reinterpret_cast<const void*>(&sqt_engine_kernel<I + 13, 7>), kThreads,
                                      kSqtKind, 7}),
   ...);
}

void register_sqt7_engines(EngineVariant* tab) { fill_sqt7(tab, std::make_integer_sequence<int, 11>{}); }

}  // namespace gbs
