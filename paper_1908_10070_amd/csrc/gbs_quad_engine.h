// Quad subset engine for subsets with d = 2|Z| <= 20, gfx950.
//
// v_mfma_f64_4x4x4_4b_f64 computes four independent 4x4x4 products, one per block b = (lane >> 2) & 3.
// Here each block carries a different subset: a wave evaluates four consecutive subsets of the
// canonical order at once. A d x d complex matrix is a T4 x T4 grid (T4 = ceil(d/4) <= 5) of 4x4
// tiles; one double register per tile holds, for block b, element (row y, column x) of that tile at
// lane x + 4b + 16y -- the instruction's output (and B-operand) layout. As in every engine,
// every power Q of M_Z has Q[i][c] = Q[c^1][i^1], so the A operand of a product is the transposed
// tile read from lane l ^ 17 (block bits untouched), and tr(P Q) pairs each tile with the same tile of
// Q read from lane l ^ 17. The same symmetry makes tile (J, I) a lane permutation of tile (I, J), so
// only the tiles with I <= J are stored and computed (qmul: 6 of 9 tile products at T4 = 3, 10 of 16
// at T4 = 4). The k traces of the four subsets are reduced over the 16 lanes of each
// block with the shared VALU lane exchanges (fold over bit 5 per trace, then transposed
// over bits 4 and 1, plain over bit 0); half the lanes store a share of the results.
#pragma once
#include "gbs_engine_common.h"

namespace gbs {
namespace {

// occupancy: up to k = kQuad3WavesKMax the |Z| <= 6 kernels run three waves per SIMD (168 registers,
// about 100 bytes of spills per lane) with their traces reduced four at a time instead of parked in
// LDS, which is what lets three workgroups fit a CU (4096 hafnians of n = 24: 18.5 -> 18.0 ms;
// probabilities of 100,000 twenty-photon patterns: 73.4 -> 67.9 ms; at k = 14, 16 it measured within
// 1%; a fourth wave up to k = 10 spilled 244 bytes per lane and ran 24% slower); above, two waves up
// to k = 20 and one beyond (where two would spill). Up to kQuadWaves2KMax the 4x4-grid kernels run two
// waves per SIMD (one above; three spilled 132 registers and ran 35% slower).
constexpr int kQuad3WavesKMax = 12;
constexpr int kQuadWaves2KMax = 12;

template <int T4>
struct QMat {
  double r[T4][T4];
  double i[T4][T4];
};

__device__ __forceinline__ double mfma4(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

// Only the tiles (I, J) with I <= J of a power are stored and computed: every power Q of M_Z has
// Q[a][c] = Q[c^1][a^1], so tile (J, I) holds at lane (x, y) what tile (I, J) holds at lane
// (y^1, x^1). Per-lane byte addresses of the two lane permutations used (inside each block):
//   tr: lane (x, y) <- (y, x)          (tile (I, K) read by rows, as an A operand, from tile (I, K))
//   tf: lane (x, y) <- (y^1, x^1)      (tile (K, J), K > J, as a B operand, from tile (J, K))
struct QPerm {
  int tr, tf;
};

__device__ __forceinline__ QPerm qperm(int lane) {
  const int x = lane & 3, b = (lane >> 2) & 3, y = lane >> 4;
  QPerm q;
  q.tr = (y + 4 * b + 16 * x) * 4;
  q.tf = ((y ^ 1) + 4 * b + 16 * (x ^ 1)) * 4;
  return q;
}

// Z = X Y on the stored tiles (I <= J); three real products per step (Gauss, gbs_engine_common.h).
// The A operand of (I, K) is tile (K, I) read at lane l ^ 17 when K <= I (the symmetry above), else
// stored tile (I, K) transposed; the B operand of (K, J) is stored when K <= J, else tile (J, K)
// through tf. Z may alias X or Y: it is written after the last product.
template <int T4>
__device__ __forceinline__ void qmul(const QMat<T4>& X, const QMat<T4>& Y, QMat<T4>& Z, const QPerm& pm) {
  double t1[T4][T4], t2[T4][T4], t3[T4][T4];
#pragma unroll
  for (int K = 0; K < T4; ++K) {
    double br[T4], bi[T4], bs[T4];
#pragma unroll
    for (int J = 0; J < T4; ++J) {
      if (K <= J) {
        br[J] = Y.r[K][J];
        bi[J] = Y.i[K][J];
      } else {
        br[J] = bperm(pm.tf, Y.r[J][K]);
        bi[J] = bperm(pm.tf, Y.i[J][K]);
      }
      bs[J] = br[J] + bi[J];
    }
#pragma unroll
    for (int I = 0; I < T4; ++I) {
      double ar, ai;
      if (K <= I) {
        ar = swap17(X.r[K][I]);
        ai = swap17(X.i[K][I]);
      } else {
        ar = bperm(pm.tr, X.r[I][K]);
        ai = bperm(pm.tr, X.i[I][K]);
      }
      const double as = ar + ai;
#pragma unroll
      for (int J = I; J < T4; ++J) {
        t1[I][J] = mfma4(ar, br[J], K == 0 ? 0.0 : t1[I][J]);
        t2[I][J] = mfma4(ai, bi[J], K == 0 ? 0.0 : t2[I][J]);
        t3[I][J] = mfma4(as, bs[J], K == 0 ? 0.0 : t3[I][J]);
      }
    }
  }
#pragma unroll
  for (int I = 0; I < T4; ++I)
#pragma unroll
    for (int J = I; J < T4; ++J) {
      Z.r[I][J] = t1[I][J] - t2[I][J];
      Z.i[I][J] = t3[I][J] - t1[I][J] - t2[I][J];
    }
}

template <int T4>
__device__ __forceinline__ double2 qdiag(const QMat<T4>& X, int lane) {
  double2 t = make_double2(0.0, 0.0);
  if ((lane & 3) == (lane >> 4)) {
#pragma unroll
    for (int I = 0; I < T4; ++I) {
      t.x += X.r[I][I];
      t.y += X.i[I][I];
    }
  }
  return t;
}

// per-lane partial of tr(X Y) = sum X[i][c] Y[i^1][c^1]: tile (I, C) pairs with itself read at lane
// l ^ 17, and a tile (C, I) below the diagonal contributes what its mirror (I, C) does (both factors
// have the symmetry above), so off-diagonal stored tiles count twice
template <int T4>
__device__ __forceinline__ double2 qpair(const QMat<T4>& X, const QMat<T4>& Y) {
  double2 d = make_double2(0.0, 0.0), o = make_double2(0.0, 0.0);
#pragma unroll
  for (int I = 0; I < T4; ++I)
#pragma unroll
    for (int C = I; C < T4; ++C) {
      double2& t = C == I ? d : o;
      const double yr = swap17(Y.r[I][C]);
      const double yi = swap17(Y.i[I][C]);
      t.x = fma(X.r[I][C], yr, t.x);
      t.x = fma(-X.i[I][C], yi, t.x);
      t.y = fma(X.r[I][C], yi, t.y);
      t.y = fma(X.i[I][C], yr, t.y);
    }
  return make_double2(fma(2.0, o.x, d.x), fma(2.0, o.y, d.y));
}

// One tile's contribution to the partial of tr(X S[s]) with S[s]'s lane-exchanged tile (yr, yi).
template <int T4, int NS, int X>
__device__ __forceinline__ void qpair_acc(const QMat<T4> (&S)[NS], int I, int C, double yr, double yi, double2& t) {
  t.x = fma(S[X].r[I][C], yr, t.x);
  t.x = fma(-S[X].i[I][C], yi, t.x);
  t.y = fma(S[X].r[I][C], yi, t.y);
  t.y = fma(S[X].i[I][C], yr, t.y);
}

// The per-lane partials of the run of inner products starting at operation OI of program KK
// (pair_run): the shared slot is exchanged (lane l ^ 17) once per tile for all of them.
template <int KK, int T4, int OI, int NS>
__device__ __forceinline__ void qpair_run(const QMat<T4> (&S)[NS], double2 (&out)[4]) {
  constexpr PairRun run = pair_run(kChainTable[KK], OI);
  constexpr int s = run.s, x0 = pair_other(kChainTable[KK], OI, s), x1 = pair_other(kChainTable[KK], OI + 1, s),
                x2 = pair_other(kChainTable[KK], OI + 2, s), x3 = pair_other(kChainTable[KK], OI + 3, s);
  double2 d[4], o[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) d[r] = o[r] = make_double2(0.0, 0.0);
#pragma unroll
  for (int I = 0; I < T4; ++I)
#pragma unroll
    for (int C = I; C < T4; ++C) {
      const double yr = swap17(S[s].r[I][C]);
      const double yi = swap17(S[s].i[I][C]);
      qpair_acc<T4, NS, x0>(S, I, C, yr, yi, C == I ? d[0] : o[0]);
      if constexpr (run.len > 1) qpair_acc<T4, NS, x1>(S, I, C, yr, yi, C == I ? d[1] : o[1]);
      if constexpr (run.len > 2) qpair_acc<T4, NS, x2>(S, I, C, yr, yi, C == I ? d[2] : o[2]);
      if constexpr (run.len > 3) qpair_acc<T4, NS, x3>(S, I, C, yr, yi, C == I ? d[3] : o[3]);
    }
#pragma unroll
  for (int r = 0; r < 4; ++r) out[r] = make_double2(fma(2.0, o[r].x, d[r].x), fma(2.0, o[r].y, d[r].y));
}

// Traces of 3x3 and larger tile grids are parked in LDS (park[(j - 1) * 64 + lane]) until the chain
// ends instead of holding k registers through every product; smaller grids keep them in registers.
// (The |Z| <= 6 kernel up to k = kQuad3WavesKMax reduces them four at a time instead: push_trace.)
constexpr int kQuadParkT4 = 3;
// parking rows per wave: a kernel whose grids have at most T4 tiles per side forms min(k, 4 T4) traces
__host__ __device__ constexpr int quad_park_k(int t4max, int k) { return k < 4 * t4max ? k : 4 * t4max; }

template <int K, int T4, int OI, int NS>
__device__ __forceinline__ void run_ops_quad(QMat<T4> (&S)[NS], double (&w)[K], double* park, int lane,
                                             const QPerm& pm) {
  if constexpr (OI < kChainTable[K].nops) {
    constexpr Op op = kChainTable[K].ops[OI];
    auto put = [&](int j, const double2& p) {
      if constexpr (T4 >= kQuadParkT4)
        park[(j - 1) * 64 + lane] = fold32(p.x, p.y);
      else
        w[j - 1] = fold32(p.x, p.y);
    };
    if constexpr (op.type == OP_MUL) {
      qmul<T4>(S[op.a], S[op.b], S[op.x], pm);
      run_ops_quad<K, T4, OI + 1, NS>(S, w, park, lane, pm);
    } else if constexpr (op.type == OP_TDIAG) {
      put(op.x, qdiag<T4>(S[op.a], lane));
      run_ops_quad<K, T4, OI + 1, NS>(S, w, park, lane, pm);
    } else {
      constexpr int len = pair_run(kChainTable[K], OI).len;
      double2 p[4];
      qpair_run<K, T4, OI, NS>(S, p);
      put(op.x, p[0]);
      if constexpr (len > 1) put(kChainTable[K].ops[OI + 1].x, p[1]);
      if constexpr (len > 2) put(kChainTable[K].ops[OI + 2].x, p[2]);
      if constexpr (len > 3) put(kChainTable[K].ops[OI + 3].x, p[3]);
      run_ops_quad<K, T4, OI + len, NS>(S, w, park, lane, pm);
    }
  }
}

// Rest of the reduction over the 16 lanes of each block (lane bits 5, 4, 1, 0; the block is bits
// 3..2) after the fold over bit 5: transposed over bits 4 and 1, plain over bit 0. Afterwards the
// lanes with bit 0 clear call store(j, part, total) for their share of the block's (trace, part) pairs.
template <int K, typename Store>
__device__ __forceinline__ void reduce_folded_quad(const double (&w)[K], int lane, Store store) {
  constexpr int KP = (K + 3) / 4 * 4, H2 = KP / 2, H3 = KP / 4;
  double v[KP];
#pragma unroll
  for (int q = 0; q < KP; ++q) v[q] = q < K ? w[q] : 0.0;
  double u[H2];
#pragma unroll
  for (int q = 0; q < H2; ++q) u[q] = fold16(v[q], v[q + H2]);
  const bool b1 = lane & 2;
  double z[H3];
#pragma unroll
  for (int q = 0; q < H3; ++q) {
    z[q] = fold_row<kDppXor2>(u[q], u[q + H3], b1);
    z[q] += dpp<kDppXor1>(z[q]);
  }
  if ((lane & 1) == 0) {
    const int base = ((lane & 16) ? H2 : 0) + (b1 ? H3 : 0);
    const int part = lane >> 5;
#pragma unroll
    for (int q = 0; q < H3; ++q)
      if (base + q < K) store(base + q + 1, part, z[q]);
  }
}

// Batched trace reduction for engines whose occupancy a parking area would limit: the q-th trace
// operation of a chain program goes to slot q % 4 of a four-value buffer, and each full buffer (and
// the last, partial one) is reduced over the 16 lanes of every block at once (reduce_folded_quad) and
// handed to store(j, part, value) with its trace index j. The exchanges per trace are those of one
// reduction at the end; the buffer's registers stay live across the products in between, which is why
// the quad grids, whose occupancy registers bound, park their traces instead (the 4x4 grid spilled).
template <int KK, int OI, typename Store>
__device__ __forceinline__ void push_trace(double (&tb)[4], double v, int lane, Store store) {
  static_assert(chain_trace_ord(kChainTable[KK], kChainTable[KK].nops) == KK, "one operation per trace");
  constexpr int ord = chain_trace_ord(kChainTable[KK], OI), slot = ord % 4, first = ord - slot;
  tb[slot] = v;
  if constexpr (slot == 3 || ord == KK - 1) {
#pragma unroll
    for (int q = slot + 1; q < 4; ++q) tb[q] = 0.0;
    constexpr int j0 = chain_trace_at(kChainTable[KK], first), j1 = chain_trace_at(kChainTable[KK], first + 1),
                  j2 = chain_trace_at(kChainTable[KK], first + 2), j3 = chain_trace_at(kChainTable[KK], first + 3);
    reduce_folded_quad<4>(tb, lane, [&](int q, int part, double x) {
      const int j = q == 1 ? j0 : (q == 2 ? j1 : (q == 3 ? j2 : j3));
      if (q - 1 <= slot) store(j, part, x);
    });
  }
}

// Four subsets (one per block) with matrices of at most 4*T4 rows; forms the first KK of the K
// traces (KK >= 2|Z| for all four, so the combine step extends the rest exactly).
template <int K, int T4, int OI, int NS, typename Store>
__device__ __forceinline__ void run_ops_quad_b(QMat<T4> (&S)[NS], double (&tb)[4], int lane, const QPerm& pm,
                                               Store store) {
  if constexpr (OI < kChainTable[K].nops) {
    constexpr Op op = kChainTable[K].ops[OI];
    if constexpr (op.type == OP_MUL) {
      qmul<T4>(S[op.a], S[op.b], S[op.x], pm);
      run_ops_quad_b<K, T4, OI + 1, NS>(S, tb, lane, pm, store);
    } else if constexpr (op.type == OP_TDIAG) {
      const double2 p = qdiag<T4>(S[op.a], lane);
      push_trace<K, OI>(tb, fold32(p.x, p.y), lane, store);
      run_ops_quad_b<K, T4, OI + 1, NS>(S, tb, lane, pm, store);
    } else {
      constexpr int len = pair_run(kChainTable[K], OI).len;
      double2 p[4];
      qpair_run<K, T4, OI, NS>(S, p);
      push_trace<K, OI>(tb, fold32(p[0].x, p[0].y), lane, store);
      if constexpr (len > 1) push_trace<K, OI + 1>(tb, fold32(p[1].x, p[1].y), lane, store);
      if constexpr (len > 2) push_trace<K, OI + 2>(tb, fold32(p[2].x, p[2].y), lane, store);
      if constexpr (len > 3) push_trace<K, OI + 3>(tb, fold32(p[3].x, p[3].y), lane, store);
      run_ops_quad_b<K, T4, OI + len, NS>(S, tb, lane, pm, store);
    }
  }
}

template <int K, int T4, int KK, bool PARK = true>
__device__ __forceinline__ void eval_quad(const PatternView& P, const int32_t* pl4, int d_b, bool valid_b, double* trw,
                                          double* park, int u_b, int lane) {
  static_assert(KK <= K, "trace count");
  constexpr int NS = kChainTable[KK].nslots;
  const int b = (lane >> 2) & 3;
  const int x = lane & 3, y = lane >> 4;
  const int32_t* pl = pl4 + b * kMaxK;
  QMat<T4> S[NS];
  if (P.lds) {
    // blocks past the last subset (stale pair lists) gather as d = 0: every entry the zero one
    const int dv = valid_b ? d_b : 0;
    int cix[T4];
#pragma unroll
    for (int J = 0; J < T4; ++J) cix[J] = mz_col(P, pl, 4 * J + x, dv);
#pragma unroll
    for (int I = 0; I < T4; ++I) {
      const int ro = mz_row(P, pl, 4 * I + y, dv);
#pragma unroll
      for (int J = I; J < T4; ++J) {  // stored tiles only
        const double2 e = mz_at(P, ro + cix[J]);
        S[0].r[I][J] = e.x;
        S[0].i[I][J] = e.y;
      }
    }
  } else {
#pragma unroll
    for (int I = 0; I < T4; ++I)
#pragma unroll
      for (int J = I; J < T4; ++J) {  // stored tiles only
        const int a = 4 * I + y, c = 4 * J + x;
        double vr = 0.0, vi = 0.0;
        if (valid_b && a < d_b && c < d_b) {
          const int bb = a ^ 1;
          const double2 e = P.at(2 * pl[bb >> 1] + (bb & 1), 2 * pl[c >> 1] + (c & 1));
          vr = e.x;
          vi = e.y;
        }
        S[0].r[I][J] = vr;
        S[0].i[I][J] = vi;
      }
  }
  if constexpr (!PARK) {
    double tb[4];
    run_ops_quad_b<KK, T4, 0, NS>(S, tb, lane, qperm(lane), [&](int j, int part, double v) {
      if (valid_b) trw[j * (2 * kWaveG) + 2 * u_b + part] = 0.5 * v;
    });
    return;
  }
  double w[KK];
  run_ops_quad<KK, T4, 0, NS>(S, w, park, lane, qperm(lane));
  if constexpr (T4 >= kQuadParkT4) {
    static_assert(KK <= quad_park_k(T4, K), "park size");
#pragma unroll
    for (int j = 0; j < KK; ++j) w[j] = park[j * 64 + lane];  // each lane reads only what it wrote
  }
  reduce_folded_quad<KK>(w, lane, [&](int j, int part, double v) {
    if (valid_b) trw[j * (2 * kWaveG) + 2 * u_b + part] = 0.5 * v;
  });
}

// Subsets [lo, hi) of one pattern on one wave, four at a time: all with |Z| <= 6 (grids of up to
// 3x3 tiles), or, with T4F > 0, all with |Z| = 2 T4F - 1 or 2 T4F (a T4F x T4F grid).
template <int K, int T4F = 0, bool PARK = true>
__device__ void quad_range(const PatternView& P, int64_t lo, int64_t hi, int32_t* pl4, double* trw, double* park,
                           int32_t* sz,
                           double2* terms, int lane, double& sr, double& si, double& cr, double& ci) {
  const int b = (lane >> 2) & 3;
  int s = 1;
  uint32_t mask = lo < hi ? unrank(K, lo, &s) : 0u;
  for (int64_t g0 = lo; g0 < hi; g0 += kWaveG) {
    const int cnt = (int)((hi - g0) < kWaveG ? (hi - g0) : kWaveG);
    for (int u0 = 0; u0 < cnt; u0 += 4) {
      // masks and sizes of the four subsets u0 .. u0+3 (uniform across the wave)
      uint32_t m4[4];
      int s4[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (u0 + q > 0 || g0 > lo) {
          if (u0 + q < cnt) mask = next_subset(mask, K, &s);
        }
        m4[q] = mask;
        s4[q] = s;
      }
      const int nv = cnt - u0 < 4 ? cnt - u0 : 4;
      wave_sync();
      // pair lists: element e < 4K of the (list, pair) grid is list e / K, pair e % K (4K may exceed 64)
      for (int e = lane; e < 4 * K; e += 64) {
        const int q = e / K, t = e - (e / K) * K;
        const uint32_t mq = m4[0] * (q == 0) + m4[1] * (q == 1) + m4[2] * (q == 2) + m4[3] * (q == 3);
        if (q < nv && ((mq >> t) & 1u)) pl4[q * kMaxK + __popc(mq & ((1u << t) - 1u))] = t;
      }
      if (lane < nv) sz[u0 + lane] = lane == 0 ? s4[0] : (lane == 1 ? s4[1] : (lane == 2 ? s4[2] : s4[3]));
      wave_sync();
      int smax = s4[0];
#pragma unroll
      for (int q = 1; q < 4; ++q)
        if (q < nv && s4[q] > smax) smax = s4[q];
      const int d_b = 2 * (b == 0 ? s4[0] : (b == 1 ? s4[1] : (b == 2 ? s4[2] : s4[3])));
      const bool valid_b = b < nv;
      const int u_b = u0 + b;
      // traces formed: min(K, 2 smax), the rest follow from them (extend_traces)
      if constexpr (T4F > 0) {  // a kernel for one grid size: |Z| = 2 T4F - 1 or 2 T4F
        if (smax <= 2 * T4F - 1)
          eval_quad<K, T4F, cmin(K, 4 * T4F - 2), PARK>(P, pl4, d_b, valid_b, trw, park, u_b, lane);
        else
          eval_quad<K, T4F, cmin(K, 4 * T4F), PARK>(P, pl4, d_b, valid_b, trw, park, u_b, lane);
      } else if (smax <= 2)
        eval_quad<K, 1, cmin(K, 4), PARK>(P, pl4, d_b, valid_b, trw, park, u_b, lane);
      else if (smax <= 3)
        eval_quad<K, 2, cmin(K, 6), PARK>(P, pl4, d_b, valid_b, trw, park, u_b, lane);
      else if (smax <= 4)
        eval_quad<K, 2, cmin(K, 8), PARK>(P, pl4, d_b, valid_b, trw, park, u_b, lane);
      else if (smax <= 5)
        eval_quad<K, 3, cmin(K, 10), PARK>(P, pl4, d_b, valid_b, trw, park, u_b, lane);
      else
        eval_quad<K, 3, cmin(K, 12), PARK>(P, pl4, d_b, valid_b, trw, park, u_b, lane);
    }
    wave_sync();
    combine_batch<K, (K > 4)>(trw, sz, cnt, lane, sr, si, cr, ci);
    wave_sync();
  }
}

}  // namespace

// LDS: the shared item-loop layout (wave_lds_layout), then one trace-parking area per wave (park_k
// rows; none for the |Z| <= 6 kernel up to k = kQuad3WavesKMax).
__host__ __device__ inline size_t quad_lds_bytes(int nmax, int kmax, int stage_A, int park_k) {
  return wave_lds_layout(nmax, kmax, stage_A).total + sizeof(double) * 4 * park_k * 64;
}

// |Z| = 2 T4 - 1, 2 T4 on a T4 x T4 grid of 4x4 tiles, a kernel per grid size so that each runs at the
// occupancy its registers allow: T4 = 4 (10 stored tiles, two waves per SIMD), T4 = 5 (15 stored
// tiles, 380-512 VGPRs and AGPRs, one wave per SIMD)
template <int K, int T4>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(T4 >= 5 || K > kQuadWaves2KMax ? 1 : 2, 8))) void
quad_grid_kernel(EngineArgs args) {
  extern __shared__ __align__(16) unsigned char smem[];
  const WaveLds L = wave_lds_layout(args.nmax, args.kmax, args.stage_A);
  wave_items<K>(args, smem, [&](const PatternView& P, int64_t lo, int64_t hi, int wave, int lane, double& sr,
                                double& si, double& cr, double& ci) {
    int32_t* pl4 = reinterpret_cast<int32_t*>(smem + L.pl) + wave * 4 * kMaxK;
    double* trw = reinterpret_cast<double*>(smem + L.trw) + (size_t)wave * (args.kmax + 1) * 2 * kWaveG;
    int32_t* sz = reinterpret_cast<int32_t*>(smem + L.sz) + wave * kWaveG;
    double2* terms = reinterpret_cast<double2*>(smem + L.terms) + wave * kWaveG;
    double* park = reinterpret_cast<double*>(smem + L.total) + wave * quad_park_k(T4, K) * 64;
    quad_range<K, T4>(P, lo, hi, pl4, trw, park, sz, terms, lane, sr, si, cr, ci);
  });
}

template <int K>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(
    K <= kQuad3WavesKMax ? 3 : (K <= 20 ? 2 : 1), 8))) void
quad_engine_kernel(EngineArgs args) {
  extern __shared__ __align__(16) unsigned char smem[];
  const WaveLds L = wave_lds_layout(args.nmax, args.kmax, args.stage_A);
  wave_items<K>(args, smem, [&](const PatternView& P, int64_t lo, int64_t hi, int wave, int lane, double& sr,
                                double& si, double& cr, double& ci) {
    int32_t* pl4 = reinterpret_cast<int32_t*>(smem + L.pl) + wave * 4 * kMaxK;
    double* trw = reinterpret_cast<double*>(smem + L.trw) + (size_t)wave * (args.kmax + 1) * 2 * kWaveG;
    int32_t* sz = reinterpret_cast<int32_t*>(smem + L.sz) + wave * kWaveG;
    double2* terms = reinterpret_cast<double2*>(smem + L.terms) + wave * kWaveG;
    double* park = K > kQuad3WavesKMax ? reinterpret_cast<double*>(smem + L.total) + wave * quad_park_k(3, K) * 64
                                       : nullptr;  // no park area (traces reduced four at a time)
    quad_range<K, 0, (K > kQuad3WavesKMax)>(P, lo, hi, pl4, trw, park, sz, terms, lane, sr, si, cr, ci);
  });
}

}  // namespace gbs
