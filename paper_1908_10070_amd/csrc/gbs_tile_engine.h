// Tile-per-wave subset engine for subsets with 16 < d = 2|Z| <= 16 T (T = 2 or 3), gfx950.
//
// A workgroup evaluates one subset at a time, one 16x16 tile of M_Z and of every power per wave, in
// registers in the v_mfma_f64_16x16x4f64 accumulator layout (lane x + 16y, register r holds element
// (y + 4r, x)). Without SYM there are T*T waves, wave (I, J) holding tile (I, J); with SYM only the
// T(T+1)/2 tiles with I <= J exist, one per wave in row-major order (every power Q has
// Q[a][c] = Q[c^1][a^1], so tile (J, I) is a permutation of tile (I, J)). A product Z = X Y publishes
// each wave's tiles of X and Y to LDS once; wave (I, J) then accumulates Z(I, J) = sum_K X(I, K) Y(K, J)
// with the A operand X(I, K) read from tile (K, I) at lane l ^ 17 and the B operand from tile (K, J);
// under SYM a tile below the diagonal is read out of its stored mirror with the permuted addresses
// of tile_a_addr / tile_b_addr. Trace inner products pair a tile with the same tile of the other
// factor, so they stay local (under SYM an off-diagonal tile counts twice, for its mirror); each wave
// reduces its partial traces with the shared VALU lane exchanges, four traces at a time, and the wave
// results are added in wave order.
// Coefficient recursion, compensated summation and partials are the shared ones (gbs_engine_common.h).
#pragma once
#include "gbs_engine_common.h"

namespace gbs {

// waves (= stored tiles) per subset
__host__ __device__ constexpr int tile_waves(int T, bool sym) { return sym ? T * (T + 1) / 2 : T * T; }

namespace {

// stored index of tile (I, J) (I <= J under SYM)
template <int T, bool SYM>
__device__ __forceinline__ int tile_slot(int I, int J) {
  return SYM ? I * T - I * (I - 1) / 2 + (J - I) : I * T + J;
}
// the tile wave w holds
template <int T, bool SYM>
__device__ __forceinline__ void tile_of_wave(int w, int& I, int& J) {
  if constexpr (!SYM) {
    I = w / T;
    J = w % T;
  } else {
    I = 0;
    while (w >= T - I) {
      w -= T - I;
      ++I;
    }
    J = I + w;
  }
}
// A published tile is four register planes of kTilePlane 16-byte slots; lane l's register r sits at
// r * kTilePlane + tile_pos(l), tile_pos folding lane bits 4..5 into bits 0..1. Both choices serve the
// transposed operand reads below, whose 16 lanes of a row would otherwise all hit one 16-byte bank
// group (lane bits 0..1 select the source row of 16, bits 2..3 the plane): the fold spreads the rows,
// the 4-slot pad per plane spreads the planes. Every offset stays a sum of a per-lane base and a
// constant, so the reads keep immediate offsets.
constexpr int kTilePlane = 68, kTileSlots = 4 * kTilePlane;
__device__ __forceinline__ int tile_pos(int l) { return l ^ ((l >> 4) & 3); }

// LDS slot (in double2 units, inside the stored tile) of the A operand of step r for tile (I, K),
// K > I, read from the stored tile (I, K): the operand wants element (x, y + 4r) of X(I, K) at lane
// x + 16y, i.e. register x >> 2 at lane (y + 4r) + 16 (x & 3). The fold there leaves bits 2..3 (4r)
// alone, so the slot is that of step 0 plus 4r (written so, for the immediate offset).
__device__ __forceinline__ int tile_a_addr(int lane, int r) {
  const int x = lane & 15, y = lane >> 4;
  return (x >> 2) * kTilePlane + tile_pos(y + 16 * (x & 3)) + 4 * r;
}
// The B operand of step r for tile (K, J), K > J, from the stored tile (J, K): element (y + 4r, x) of
// Y(K, J) is element (x^1, (y + 4r)^1) of Y(J, K): register (x^1) >> 2 at lane ((y^1) + 4r) + 16 ((x^1) & 3).
__device__ __forceinline__ int tile_b_addr(int lane, int r) {
  const int x = lane & 15, y = lane >> 4;
  return ((x ^ 1) >> 2) * kTilePlane + tile_pos((y ^ 1) + 16 * ((x ^ 1) & 3)) + 4 * r;
}

template <int T, bool SYM>
__device__ __forceinline__ void tile_mul(const CMat<1>& X, const CMat<1>& Y, CMat<1>& Z, int d, int lane, int w,
                                         int I, int J, double2* xbuf) {
  constexpr int NT = tile_waves(T, SYM);
  // every wave done reading the previous product's factors before they are overwritten; waiting here
  // rather than at the end of that product lets the waves whose tiles lie outside d, or finish early,
  // form their traces while the others still multiply
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    xbuf[(0 * NT + w) * kTileSlots + r * kTilePlane + tile_pos(lane)] = make_double2(X.r[0][0][r], X.i[0][0][r]);
    xbuf[(1 * NT + w) * kTileSlots + r * kTilePlane + tile_pos(lane)] = make_double2(Y.r[0][0][r], Y.i[0][0][r]);
  }
  __syncthreads();
  // operand r of k-tile K: A from X(I, K), B from Y(K, J)
  auto opA = [&](int K, int r) -> double2 {
    if (!SYM || K <= I)
      return xbuf[(0 * NT + tile_slot<T, SYM>(K, I)) * kTileSlots + r * kTilePlane + tile_pos(lane ^ 17)];
    return xbuf[(0 * NT + tile_slot<T, SYM>(I, K)) * kTileSlots + tile_a_addr(lane, r)];
  };
  auto opB = [&](int K, int r) -> double2 {
    if (!SYM || K <= J) return xbuf[(1 * NT + tile_slot<T, SYM>(K, J)) * kTileSlots + r * kTilePlane + tile_pos(lane)];
    return xbuf[(1 * NT + tile_slot<T, SYM>(J, K)) * kTileSlots + tile_b_addr(lane, r)];
  };
  // The first step (K = 0, r = 0) always runs for a tile inside d and starts the accumulators; three
  // real products per step (Gauss, gbs_engine_common.h).
  const d4 zero = d4{0.0, 0.0, 0.0, 0.0};
  d4 accr, acci, t3;
  if (16 * I < d && 16 * J < d) {
#pragma unroll
    for (int K = 0; K < T; ++K)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const bool first = K == 0 && r == 0;
        if (first || 16 * K + 4 * r < d) {
          const double2 a = opA(K, r);
          const double2 b = opB(K, r);
          accr = mfma(a.x, b.x, first ? zero : accr);
          acci = mfma(a.y, b.y, first ? zero : acci);
          t3 = mfma(a.x + a.y, b.x + b.y, first ? zero : t3);
        }
      }
  } else {
    accr = zero;
    acci = zero;
    t3 = zero;
  }
  Z.r[0][0] = accr - acci;
  Z.i[0][0] = t3 - accr - acci;
}

// Traces are reduced over the wave four at a time as the chain forms them (the q-th trace operation
// goes to slot q % 4; full buffers, and the last, go through reduce_folded), so no k registers are held
// across the products: that lets the kernel run three waves per SIMD (168 registers; at k = 22 about
// 300 bytes of spills per lane) instead of two (n = 46, 2 hafnians: 212 -> 205 ms; n <= 36 unchanged).
template <int KK, int OI, typename Store>
__device__ __forceinline__ void push_trace_tile(double (&tb)[4], double v, int lane, Store store) {
  constexpr int ord = chain_trace_ord(kChainTable[KK], OI), slot = ord % 4, first = ord - slot;
  tb[slot] = v;
  if constexpr (slot == 3 || ord == KK - 1) {
#pragma unroll
    for (int q = slot + 1; q < 4; ++q) tb[q] = 0.0;
    constexpr int j0 = chain_trace_at(kChainTable[KK], first), j1 = chain_trace_at(kChainTable[KK], first + 1),
                  j2 = chain_trace_at(kChainTable[KK], first + 2), j3 = chain_trace_at(kChainTable[KK], first + 3);
    reduce_folded<4>(tb, lane, [&](int q, int part, double x) {
      const int j = q == 1 ? j0 : (q == 2 ? j1 : (q == 3 ? j2 : j3));
      if (q - 1 <= slot) store(j, part, x);
    });
  }
}

template <int K, int T, bool SYM, int OI, int NS, typename Store>
__device__ __forceinline__ void run_ops_tile(CMat<1> (&S)[NS], double (&tb)[4], int d, int lane, int w, int I, int J,
                                             double2* xbuf, Store store) {
  if constexpr (OI < kChainTable[K].nops) {
    constexpr Op op = kChainTable[K].ops[OI];
    if constexpr (op.type == OP_MUL) {
      tile_mul<T, SYM>(S[op.a], S[op.b], S[op.x], d, lane, w, I, J, xbuf);
    } else {
      double2 p = op.type == OP_TDIAG ? (I == J ? tdiag<1>(S[op.a], lane) : make_double2(0.0, 0.0))
                                      : tpair<1>(S[op.a], S[op.b]);
      if (op.type != OP_TDIAG && SYM && I != J) p = make_double2(2.0 * p.x, 2.0 * p.y);
      push_trace_tile<K, OI>(tb, fold32(p.x, p.y), lane, store);
    }
    run_ops_tile<K, T, SYM, OI + 1, NS>(S, tb, d, lane, w, I, J, xbuf, store);
  }
}

// One subset on the whole workgroup; the wave sums of the traces land in tred[w][component].
template <int K, int T, bool SYM>
__device__ __forceinline__ void eval_subset_tile(const PatternView& P, const int32_t* pl, int d, int lane, int w,
                                                 double2* xbuf, double* tred) {
  constexpr int NS = kChainTable[K].nslots;
  int I, J;
  tile_of_wave<T, SYM>(w, I, J);
  CMat<1> S[NS];
  const int x = lane & 15, y = lane >> 4;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int a = 16 * I + y + 4 * r;
    const int c = 16 * J + x;
    double vr = 0.0, vi = 0.0;
    if (a < d && c < d) {
      const int b = a ^ 1;
      const double2 e = P.at(2 * pl[b >> 1] + (b & 1), 2 * pl[c >> 1] + (c & 1));
      vr = e.x;
      vi = e.y;
    }
    S[0].r[0][0][r] = vr;
    S[0].i[0][0][r] = vi;
  }
  // each wave's share of every trace, summed over the wave; added across waves in wave order later
  double tb[4];
  run_ops_tile<K, T, SYM, 0, NS>(S, tb, d, lane, w, I, J, xbuf,
                                 [&](int j, int part, double v) { tred[w * 2 * K + 2 * (j - 1) + part] = v; });
}

template <int K, int T, bool SYM>
__device__ void tile_range(const PatternView& P, int64_t lo, int64_t hi, int32_t* pl, double2* xbuf, double* tred,
                           double* trw, int32_t* sz, double2* terms, int tid, double& sr, double& si, double& cr,
                           double& ci) {
  constexpr int NT = tile_waves(T, SYM);
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  int s = 1;
  uint32_t mask = lo < hi ? unrank(K, lo, &s) : 0u;
  for (int64_t g0 = lo; g0 < hi; g0 += kWaveG) {
    const int cnt = (int)((hi - g0) < kWaveG ? (hi - g0) : kWaveG);
    for (int u = 0; u < cnt; ++u) {
      if (u > 0 || g0 > lo) mask = next_subset(mask, K, &s);
      __syncthreads();  // previous subset done with the pair list and tred
      if (tid < K && ((mask >> tid) & 1u)) pl[__popc(mask & ((1u << tid) - 1u))] = tid;
      if (tid == 0) sz[u] = s;
      __syncthreads();
      eval_subset_tile<K, T, SYM>(P, pl, 2 * s, lane, w, xbuf, tred);
      __syncthreads();
      if (tid < 2 * K) {
        double v = tred[tid];
#pragma unroll
        for (int q = 1; q < NT; ++q) v += tred[q * 2 * K + tid];
        trw[((tid >> 1) + 1) * (2 * kWaveG) + 2 * u + (tid & 1)] = 0.5 * v;
      }
    }
    __syncthreads();
    if (w == 0) combine_batch<K>(trw, sz, cnt, lane, sr, si, cr, ci);
    __syncthreads();
  }
}

}  // namespace

struct TileLds {
  size_t A, modes, pl, xbuf, tred, trw, sz, terms, item, total;
};

__host__ __device__ inline TileLds tile_lds_layout(int T, bool sym, int nmax, int kmax, int stage_A) {
  const int NT = tile_waves(T, sym);
  TileLds L;
  size_t off = 0;
  L.A = off;
  off += stage_A ? wal16(sizeof(double) * 2 * nmax * nmax) : 0;
  L.modes = off;
  off += wal16(sizeof(int32_t) * GBS_N_MAX);
  L.pl = off;
  off += wal16(sizeof(int32_t) * kMaxK);
  L.xbuf = off;
  off += wal16(sizeof(double) * 2 * 2 * NT * kTileSlots);
  L.tred = off;
  off += wal16(sizeof(double) * NT * 2 * kmax);
  L.trw = off;
  off += wal16(sizeof(double) * (kmax + 1) * 2 * kWaveG);
  L.sz = off;
  off += wal16(sizeof(int32_t) * kWaveG);
  L.terms = off;
  off += wal16(sizeof(double) * 2 * kWaveG);
  L.item = off;
  off += 16;
  L.total = off;
  return L;
}

template <int T, int K, bool SYM = false>
__global__ __launch_bounds__(tile_waves(T, SYM) * 64) __attribute__((amdgpu_waves_per_eu(3, 8))) void
tile_engine_kernel(EngineArgs args) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NTH = tile_waves(T, SYM) * 64;
  const TileLds L = tile_lds_layout(T, SYM, args.nmax, args.kmax, args.stage_A);
  double2* Alds = reinterpret_cast<double2*>(smem + L.A);
  int32_t* mlds = reinterpret_cast<int32_t*>(smem + L.modes);
  int32_t* pl = reinterpret_cast<int32_t*>(smem + L.pl);
  double2* xbuf = reinterpret_cast<double2*>(smem + L.xbuf);
  double* tred = reinterpret_cast<double*>(smem + L.tred);
  double* trw = reinterpret_cast<double*>(smem + L.trw);
  int32_t* sz = reinterpret_cast<int32_t*>(smem + L.sz);
  double2* terms = reinterpret_cast<double2*>(smem + L.terms);
  int32_t* item_sh = reinterpret_cast<int32_t*>(smem + L.item);
  const int tid = threadIdx.x;

  int it = args.persistent ? 0 : (int)blockIdx.x;
  for (;;) {
    if (args.persistent) {
      __syncthreads();
      if (tid == 0) item_sh[0] = atomicAdd(args.counter, 1);
      __syncthreads();
      it = item_sh[0];
    }
    if (it >= args.n_items) break;
    const WorkItem item = args.items[it];
    const PatternDesc pd = args.pats[item.pattern];
    const int n = pd.n, k = n >> 1;
    const bool prob = args.modes != nullptr;
    if (prob && tid < n) mlds[tid] = args.modes[pd.src + tid];
    __syncthreads();
    const bool staged = args.stage_A && n <= 32;
    if (staged) {
      for (int e = tid; e < n * n; e += NTH) {
        const int i = e / n, j = e - (e / n) * n;
        Alds[e] = prob ? args.A[(int64_t)mlds[i] * args.m + mlds[j]] : args.A[pd.src + e];
      }
    }
    __syncthreads();
    PatternView P;
    P.lds = staged ? Alds : nullptr;
    P.A = args.A;
    P.modes = prob ? mlds : nullptr;
    P.src = pd.src;
    P.n = n;
    P.m = args.m;
    P.ld = n;
    double sr = 0.0, si = 0.0, cr = 0.0, ci = 0.0;
    if (k == K) tile_range<K, T, SYM>(P, item.lo, item.hi, pl, xbuf, tred, trw, sz, terms, tid, sr, si, cr, ci);
    if (tid == 0) {
      gbs_partial p;
      p.s_re = sr;
      p.s_im = si;
      p.c_re = cr;
      p.c_im = ci;
      args.partials[item.partial] = p;
    }
    if (!args.persistent) break;
  }
}

}  // namespace gbs
