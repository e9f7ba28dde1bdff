// Internal types shared by the HIP kernels and the host runtime of libgbs.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "gbs.h"

namespace gbs {

constexpr int kMaxK = GBS_N_MAX / 2;  // largest pair count k = n/2
constexpr int kMaxOps = 64;           // ops in one chain program
constexpr int kThreads = 256;         // workgroup size of the engines that give each wave its own subsets

enum OpType : uint8_t { OP_MUL = 1, OP_TDIAG = 2, OP_TPAIR = 3 };

// One step of the per-subset program. MUL: slot x = slot a * slot b (x may equal a dying operand).
// TDIAG: t_x = tr(slot a). TPAIR: t_x = tr(slot a * slot b), read as sum_{i,c} a[i][c] b[c][i].
struct Op {
  uint8_t type, x, a, b;
};

// Power-trace schedule for one k: the powers of M_Z to form (an addition chain) and, for every
// j = 1..k, where t_j = tr(M_Z^j) comes from.
struct ChainProgram {
  int32_t nops;
  int32_t nslots;
  int32_t nmul;
  int32_t npair;
  Op ops[kMaxOps];
};

// One pattern (a matrix to take the hafnian of).
struct PatternDesc {
  int64_t src;      // haf path: element offset of the row-major n x n matrix; prob path: offset into modes
  int32_t n;
  int32_t pad;
};

// A contiguous range [lo, hi) of the canonical subset order of one pattern, summed into one partial.
struct WorkItem {
  int64_t lo, hi;
  int32_t pattern;
  int32_t partial;
};

// Arguments of the subset engine.
struct EngineArgs {
  const double2* A;           // haf path: matrices (complex128); prob path: B (m x m)
  const int32_t* modes;       // prob path: staged mode lists; nullptr on the haf path
  int32_t m;                  // prob path: row length of B
  int32_t n_items;
  const PatternDesc* pats;
  const WorkItem* items;
  gbs_partial* partials;
  int32_t* counter;           // work counter for the persistent launch
  int32_t persistent;
  int32_t stage_A;            // copy each pattern matrix into LDS (n <= 32)
  int32_t nmax;               // largest n among the items (LDS sizing)
  int32_t kmax;               // largest k among the items
};

struct FinalizeArgs {
  const gbs_partial* partials;
  const int64_t* part_lo;     // pattern b sums partials[part_lo[b] .. part_hi[b])
  const int64_t* part_hi;
  const int32_t* n;           // photon number per pattern
  const double* sfact;        // prod_j s_j! per pattern (prob path)
  const double* prefactor;    // 1 / prod cosh r_i (device scalar), or nullptr
  int64_t batch;
  double* prob_out;           // nullable
  double2* haf_out;           // nullable
  gbs_partial* partial_out;   // nullable: write the combined compensated partial instead
  const int64_t* out_idx;     // nullable: result b goes to index out_idx[b] of the output it writes
};

// Marginal probabilities (Theorem 1, regrouped). Per prefix p of k positions (modes x), h[mask] is
// the hafnian of W restricted to the positions in mask (every even-size mask over k bits), built
// size by size from h(S) = sum_{j in S, j > i0} W(x_i0, x_j) h(S minus {i0, j}), i0 = lowest of S.
// Position sets A with the same mode multiset form a class; for class c (all members of size mu)
//   H_j = sum over members A of sum over 2j-subsets a of C = [k] minus A of h[a] h[C minus a],
//   v_c = w_c * Re sum_{j1, j2} F[mu][j1][j2] H_{j1} conj(H_{j2}),
// and q_p = sum of v_c over the prefix's classes in class order. A collision-free prefix has one
// class per A with |A| = k mod 2, numbered implicitly (class i <-> A = 2i + parity bit, w = 1);
// other prefixes list their classes explicitly.
struct MargArgs {
  const double2* W;          // m x m, row-major
  int32_t m;
  const int32_t* x;          // prefix modes, prefix p at x_off[p]
  const int64_t* x_off;
  double2* h;                // hafnian tables; prefix p's starts at h_off[p] (2^k entries)
  const int64_t* h_off;
  const int32_t* k;          // prefix lengths
  const double* F;           // per prefix (k + 1) x jdim x jdim weights at F_off[p]
  const int64_t* F_off;
  const int64_t* pre_cls;    // per prefix: classes pre_cls[p] .. pre_cls[p + 1] (global numbering)
  const int64_t* ex_base;    // per prefix: first explicit class, or -1 if the prefix is collision-free
  const int64_t* cls_mem;    // explicit class e: members cls_mem[e] .. cls_mem[e + 1] of mem
  const double* cls_w;       // explicit class e: Per(S_{A,B}) for A, B in the class
  const uint32_t* mem;       // member masks A
  int64_t n_classes;         // total (implicit + explicit)
  double* v;                 // per class value
  int64_t batch;
  int32_t jdim;              // kmax / 2 + 1
  double* q_out;             // per prefix marginal
};

// Subset-engine kernel variants, one kernel per (engine, k) so each carries only its own k's
// registers and chain program. Class numbers (k = n/2, s = |Z|):
//   0..22   quad engine, |Z| <= 6, k = 1..23                        (gbs_eng_quad.hip)
//   23..41  quad engine on a 4x4 tile grid, |Z| = 7, 8, k = 5..23    (gbs_eng_grid4.hip)
//   42..56  quad engine on a 5x5 tile grid, |Z| = 9, 10, k = 9..23   (gbs_eng_grid5.hip)
//   57..62  strip engine, 6 tile rows, |Z| = 11, 12, k = 11..16      (gbs_eng_strip.hip)
//   63..69  quad-tile engine, |Z| = 11, 12, k = 17..23               (gbs_eng_tile.hip)
//   70..84  tile engine, 2x2 16x16 tiles, |Z| = 13..16 (and 9..12 where the engine shape asks for
//           it), k = 9..23                                             (gbs_eng_tile.hip)
//   85..91  tile engine, 3x3 16x16 tiles (the six on and above the diagonal), |Z| >= 17, k = 17..23
//                                                                      (gbs_eng_tile.hip)
//   92..94  double-double engine (accuracy mode), 2|Z| <= 16, 32, 48; any k (gbs_eng_dd.hip)
//   95..107 symmetric quad-tile engine, 6x6 grid, |Z| = 11, 12 (and 9, 10), k = 11..23 (gbs_eng_sqt.hip)
//   108..118 symmetric quad-tile engine, 7x7 grid, |Z| = 13, 14, k = 13..23 (gbs_eng_sqt7.hip)
constexpr int kEngineClasses = 119;
constexpr int kClsQuad = 0, kClsGrid4 = 23, kClsGrid5 = 42, kClsStrip = 57, kClsQtile = 63, kClsTile2 = 70,
              kClsTile3 = 85, kClsDd = 92, kClsSqt = 95, kClsSqt7 = 108;

// Engine shape bits (per photon number, chosen by the autotuner): which engine takes the middle
// subset sizes instead of the default (the 5x5 quad grid for |Z| = 9, 10; the strip engine at k <= 16
// and the quad-tile engine above for |Z| = 11, 12; the 2x2 16x16-tile engine for |Z| = 13..16). The
// symmetric quad-tile bits win over the tile bits and need k >= 11.
constexpr int kShapeTile910 = 1;   // |Z| = 9, 10: 16x16 tile engine (2x2 tiles)
constexpr int kShapeTile1112 = 2;  // |Z| = 11, 12: 16x16 tile engine
constexpr int kShapeSqt1112 = 4;   // |Z| = 11, 12: symmetric quad-tile engine
constexpr int kShapeSqt910 = 8;    // |Z| = 9, 10: symmetric quad-tile engine
constexpr int kShapeSqt1314 = 16;  // |Z| = 13, 14: symmetric quad-tile engine on a 7x7 grid
constexpr int kShapeMask = 31;

enum EngineKind {
  kQuadKind = 0, kStripKind = 1, kQtileKind = 2, kTileKind = 3, kDdKind = 4, kSqtKind = 5,
  kTileSymKind = 6  // the 16x16 tile engine storing only the tiles on and above the diagonal
};

// Arithmetic of the subset engines: FP64 (MFMA) or double-double (VALU, error-free transformations).
enum Precision { kPrecFp64 = 0, kPrecDd = 1 };

// One kernel variant: its entry point, workgroup size, engine kind and tile count per side (tile
// engines) or largest grid side (quad engines).
struct EngineVariant {
  const void* fn;
  int threads;
  int kind;
  int tiles;
};

// Each engine translation unit fills its classes of the variant table.
void register_quad_engines(EngineVariant* tab);
void register_grid4_engines(EngineVariant* tab);
void register_grid5_engines(EngineVariant* tab);
void register_strip_engines(EngineVariant* tab);
void register_tile_engines(EngineVariant* tab);
void register_dd_engines(EngineVariant* tab);
void register_sqt_engines(EngineVariant* tab);
void register_sqt7_engines(EngineVariant* tab);

// No-allocation hafnian path (haf_batch_noalloc): a uniform-n batch's plan is built on the device in
// a static scratch array. Per engine launch g, every pattern has count items: item j of pattern p
// covers [a + j chunk, min(b, a + (j + 1) chunk)) of the canonical subset order and writes partial
// p * ipp + local_base + j; the launch's items are stored pattern by pattern from index first.
constexpr int kNoallocMaxGroups = 8;
struct NoallocGroup {
  int64_t first;       // first item of this launch in the item array
  int64_t a, b;        // the launch's range of one pattern's canonical subset order
  int64_t chunk;       // subsets per item
  int32_t count;       // items per pattern in this launch
  int32_t local_base;  // partial index of the launch's first item within its pattern
};
struct NoallocPlanArgs {
  NoallocGroup g[kNoallocMaxGroups];
  int32_t n_groups;
  int32_t n;
  int32_t ipp;             // items (partials) per pattern
  int32_t pad;
  int64_t batch;
  int64_t stride;          // elements between consecutive matrices
  int64_t total_items;
  PatternDesc* pats;
  WorkItem* items;
  int64_t* part_off;       // batch + 1
  int32_t* nvec;
  double* sfact;
};
// Device address of the no-allocation scratch on `device` (hipGetSymbolAddress, taken once per
// device with that device current); nullptr with *err set if the lookup failed.
void* noalloc_scratch(int device, hipError_t* err);
size_t noalloc_scratch_bytes();
void launch_noalloc_plan(const NoallocPlanArgs& a, hipStream_t s);

// Output-space sweep (gbs_sweep.hip): hafnians of every pattern of n photons in m modes from the
// stored hafnians of all patterns two photons shorter, and the brute-force sampler over them.
constexpr int kSweepMaxN = 32;
struct SweepArgs {
  const double2* B;          // m x m
  int32_t m;
  int32_t n;
  int32_t collisions;        // 1: multisets (modes may repeat); 0: sets
  int32_t bstride;           // binom row length (n + 1)
  const uint64_t* binom;     // C(v, i) at binom[v * bstride + i], v < m + n, i <= n
  int64_t count;             // patterns of size n
  const double* prefactor;   // device scalar 1 / prod cosh r_i
  double* prob_out;          // nullable, count entries, lexicographic order
  double2* haf_out;          // nullable
};
void launch_sweep(const SweepArgs& a, double2* tab0, double2* tab1, const int64_t* level_count, hipStream_t s);
int64_t cdf_blocks(int64_t count);
void launch_cdf(const double* p, int64_t count, double* cdf, double* bsum, double* total, hipStream_t s);
void launch_cdf_draw(const double* cdf, int64_t count, const double* total, const double* u, int64_t nsamples,
                     int64_t* idx, hipStream_t s);

// Host-side launchers (defined in gbs_kernels.hip).
int engine_class(int s, int k, int shape = 0);  // variant for subsets of size s, k pairs, engine shape bits
int engine_class_dd(int s);        // double-double variant for subsets of size s
size_t engine_lds_bytes(int cls, int nmax, int kmax, int stage_A);
int engine_blocks_per_cu(int cls, size_t lds);
void launch_engine(int cls, const EngineArgs& a, int grid, size_t lds, hipStream_t s);
void launch_reset(int32_t* counter, int n, hipStream_t s);
void launch_sym_check(const double2* A, const PatternDesc* pats, int64_t batch, double tol, int32_t* flags,
                      hipStream_t s);
void launch_finalize(const FinalizeArgs& a, hipStream_t s);
void launch_state(const double2* U, const double* r, int m, double2* B, double2* W, double* prefactor, hipStream_t s);
void launch_marginal(const MargArgs& a, int kmax, int64_t h_total, hipStream_t s);
// next[b] = smallest l in [0, m) with w[b][0] + ... + w[b][l] >= u[b] * (w[b][0] + ... + w[b][m-1])
void launch_draw(const double* w, int64_t batch, int m, const double* u, int32_t* next, hipStream_t s);

}  // namespace gbs
