// Subset-engine kernels for the largest subsets: quad-tile engine for |Z| = 11, 12 at k = 17..23
// (classes kClsQtile + k - 17), tile engine with 2x2 16x16 tiles for |Z| = 13..16 (and 9..12 where
// the engine shape asks for it) at k = 9..23 (kClsTile2 + k - 9) and with the six stored tiles of a 3x3
// grid for |Z| >= 17 at k = 17..23 (kClsTile3 + k - 17).
#include <hip/hip_runtime.h>

#include <utility>

#include "gbs_engine_common.h"
#include "gbs_quad_engine.h"
#include "gbs_qtile_engine.h"
#include "gbs_tile_engine.h"

namespace gbs {

template <int... I>
static void fill_qtile(EngineVariant* tab, std::integer_sequence<int, I...>) {
  ((tab[kClsQtile + I] = EngineVariant{reinterpret_cast<const void*>(&qtile_engine_kernel<I + 17>), kThreads,
                                       kQtileKind, 1}),
   ...);
}

// The 3x3 grid stores only the six tiles on and above the diagonal (six waves per subset, two per SIMD
// without spills, a third fewer products; nine full tiles needed three waves per SIMD and spilled:
// n = 46, 2 hafnians, 222 -> 214 ms). The 2x2 grid keeps all four tiles: three-wave workgroups of the
// stored tiles measured slower (n = 44, 4 hafnians: 167.5 -> 171.6 ms).
constexpr bool kTile2Sym = false, kTile3Sym = true;

template <int... I>
static void fill_tile2(EngineVariant* tab, std::integer_sequence<int, I...>) {
  ((tab[kClsTile2 + I] = EngineVariant{reinterpret_cast<const void*>(&tile_engine_kernel<2, I + 9, kTile2Sym>),
                                       tile_waves(2, kTile2Sym) * 64, kTile2Sym ? kTileSymKind : kTileKind, 2}),
   ...);
}

template <int... I>
static void fill_tile3(EngineVariant* tab, std::integer_sequence<int, I...>) {
  ((tab[kClsTile3 + I] = EngineVariant{reinterpret_cast<const void*>(&tile_engine_kernel<3, I + 17, kTile3Sym>),
                                       tile_waves(3, kTile3Sym) * 64, kTile3Sym ? kTileSymKind : kTileKind, 3}),
   ...);
}

void register_tile_engines(EngineVariant* tab) {
  fill_qtile(tab, std::make_integer_sequence<int, 7>{});
  fill_tile2(tab, std::make_integer_sequence<int, 15>{});
  fill_tile3(tab, std::make_integer_sequence<int, 7>{});
}

}  // namespace gbs
