// Quad-tile subset engine for 8 < |Z| <= 12 (16 < d = 2|Z| <= 24) at k >= 17, gfx950.
//
// A workgroup of four waves evaluates four subsets at a time, one per block of
// v_mfma_f64_4x4x4_4b_f64 (block b = (lane >> 2) & 3, as in the quad engine). M_Z and its powers are
// 6x6 grids of 4x4 tiles; wave w = 2 WI + WJ keeps the 3x3 quadrant of tiles (3 WI + I, 3 WJ + J) of
// every power in registers, one double per tile and component, in the quad engine's layout (lane
// x + 4b + 16y holds element (y, x) of the tile for block b). The 4x4x4 FP64 MFMA sustains about
// 1.5x the rate of the 16x16x4 one on this device, and 4-wide tiles pad d = 18..24 to 20 or 24
// instead of 32.
//
// A product Z = X Y publishes both factors' quadrants to LDS (a square publishes once). Each wave
// then accumulates its quadrant over the k-tiles inside d: the A operand, X's tile (gi, K) by rows,
// is X's tile (K, gi) read at lane l ^ 17 (every power Q satisfies Q[i][c] = Q[c^1][i^1]); the B
// operand is Y's tile (K, gj) as stored. Complex products use three real products per step. Traces
// need no exchange: diagonal tiles for tr(M^j), and tr(P Q) pairs every tile of P with the same tile
// of Q read at lane l ^ 17. Each wave reduces its partial traces over the 16 lanes of every block;
// the four waves' values are added in wave order through LDS, and the coefficient recursion and the
// compensated sum are those of the other engines.
#pragma once
#include "gbs_engine_common.h"
#include "gbs_quad_engine.h"

namespace gbs {
namespace {

constexpr int kQtG = 6;        // tiles per matrix side (d <= 24)
constexpr int kQtQ = 3;        // tiles per wave side
constexpr int kQtTiles = kQtG * kQtG;

// Z = X Y for the wave's quadrant; T4 = ceil(max d / 4) over the four subsets (uniform).
template <bool SAME>
__device__ __forceinline__ void qt_mul(const QMat<kQtQ>& X, const QMat<kQtQ>& Y, QMat<kQtQ>& Z, int T4, int WI,
                                       int WJ, int lane, double2* xq) {
#pragma unroll
  for (int I = 0; I < kQtQ; ++I)
#pragma unroll
    for (int J = 0; J < kQtQ; ++J) {
      const int t = (kQtQ * WI + I) * kQtG + kQtQ * WJ + J;
      xq[t * 64 + lane] = make_double2(X.r[I][J], X.i[I][J]);
      if (!SAME) xq[(kQtTiles + t) * 64 + lane] = make_double2(Y.r[I][J], Y.i[I][J]);
    }
  __syncthreads();
  const double2* yq = SAME ? xq : xq + kQtTiles * 64;
  bool act[kQtQ][kQtQ];
#pragma unroll
  for (int I = 0; I < kQtQ; ++I)
#pragma unroll
    for (int J = 0; J < kQtQ; ++J) act[I][J] = kQtQ * WI + I < T4 && kQtQ * WJ + J < T4;
  double t1[kQtQ][kQtQ], t2[kQtQ][kQtQ], t3[kQtQ][kQtQ];
#pragma unroll
  for (int K = 0; K < kQtG; ++K) {
    if (K < T4) {  // k-tiles beyond d hold zeros
      double2 a[kQtQ], b[kQtQ];
      double as[kQtQ], bs[kQtQ];
#pragma unroll
      for (int I = 0; I < kQtQ; ++I) {
        a[I] = xq[(K * kQtG + kQtQ * WI + I) * 64 + (lane ^ 17)];
        as[I] = a[I].x + a[I].y;
      }
#pragma unroll
      for (int J = 0; J < kQtQ; ++J) {
        b[J] = yq[(K * kQtG + kQtQ * WJ + J) * 64 + lane];
        bs[J] = b[J].x + b[J].y;
      }
#pragma unroll
      for (int I = 0; I < kQtQ; ++I)
#pragma unroll
        for (int J = 0; J < kQtQ; ++J) {
          if (act[I][J]) {
            t1[I][J] = mfma4(a[I].x, b[J].x, K == 0 ? 0.0 : t1[I][J]);
            t2[I][J] = mfma4(a[I].y, b[J].y, K == 0 ? 0.0 : t2[I][J]);
            t3[I][J] = mfma4(as[I], bs[J], K == 0 ? 0.0 : t3[I][J]);
          }
        }
    }
  }
  __syncthreads();  // every wave done reading before the next publish
#pragma unroll
  for (int I = 0; I < kQtQ; ++I)
#pragma unroll
    for (int J = 0; J < kQtQ; ++J) {
      Z.r[I][J] = act[I][J] ? t1[I][J] - t2[I][J] : 0.0;
      Z.i[I][J] = act[I][J] ? t3[I][J] - t1[I][J] - t2[I][J] : 0.0;
    }
}

// per-lane partial of tr(X) over the wave's quadrant (diagonal tiles only on waves with WI == WJ)
__device__ __forceinline__ double2 qt_diag(const QMat<kQtQ>& X, int lane, bool diag_wave) {
  double2 t = make_double2(0.0, 0.0);
  if (diag_wave && (lane & 3) == (lane >> 4)) {
#pragma unroll
    for (int I = 0; I < kQtQ; ++I) {
      t.x += X.r[I][I];
      t.y += X.i[I][I];
    }
  }
  return t;
}

template <int K, int OI, int NS>
__device__ __forceinline__ void run_ops_qt(QMat<kQtQ> (&S)[NS], double (&w)[K], int T4, int WI, int WJ, int lane,
                                           double2* xq) {
  if constexpr (OI < kChainTable[K].nops) {
    constexpr Op op = kChainTable[K].ops[OI];
    if constexpr (op.type == OP_MUL) {
      qt_mul<op.a == op.b>(S[op.a], S[op.b], S[op.x], T4, WI, WJ, lane, xq);
    } else if constexpr (op.type == OP_TDIAG) {
      const double2 p = qt_diag(S[op.a], lane, WI == WJ);
      w[op.x - 1] = fold32(p.x, p.y);
    } else {
      const double2 p = qpair<kQtQ>(S[op.a], S[op.b]);
      w[op.x - 1] = fold32(p.x, p.y);
    }
    run_ops_qt<K, OI + 1, NS>(S, w, T4, WI, WJ, lane, xq);
  }
}

// Four subsets (one per block): gather the wave's quadrant of M_Z, run the chain program, leave the
// wave's block-reduced partial traces in tred[((w * 4 + b) * K + j - 1) * 2 + part].
template <int K>
__device__ __forceinline__ void eval_qtile(const PatternView& P, const int32_t* pl4, int T4, int d_b, bool valid_b,
                                           int w, int lane, double2* xq, double* tred) {
  constexpr int NS = kChainTable[K].nslots;
  const int WI = w >> 1, WJ = w & 1;
  const int b = (lane >> 2) & 3;
  const int x = lane & 3, y = lane >> 4;
  const int32_t* pl = pl4 + b * kMaxK;
  QMat<kQtQ> S[NS];
#pragma unroll
  for (int I = 0; I < kQtQ; ++I)
#pragma unroll
    for (int J = 0; J < kQtQ; ++J) {
      const int a = 4 * (kQtQ * WI + I) + y, c = 4 * (kQtQ * WJ + J) + x;
      double vr = 0.0, vi = 0.0;
      if (valid_b && a < d_b && c < d_b) {
        const int bb = a ^ 1;  // M = X A_Z: row a of M is row a^1 of A_Z
        const double2 e = P.at(2 * pl[bb >> 1] + (bb & 1), 2 * pl[c >> 1] + (c & 1));
        vr = e.x;
        vi = e.y;
      }
      S[0].r[I][J] = vr;
      S[0].i[I][J] = vi;
    }
  double wt[K];
  run_ops_qt<K, 0, NS>(S, wt, T4, WI, WJ, lane, xq);
  reduce_folded_quad<K>(wt, lane, [&](int j, int part, double v) { tred[((w * 4 + b) * K + j - 1) * 2 + part] = v; });
}

// Subsets [lo, hi) of one pattern on the workgroup, four at a time.
template <int K>
__device__ void qtile_range(const PatternView& P, int64_t lo, int64_t hi, int32_t* pl4, double2* xq, double* tred,
                            double* trw, int32_t* sz, double2* terms, int tid, double& sr, double& si, double& cr,
                            double& ci) {
  const int w = tid >> 6, lane = tid & 63;
  const int b = (lane >> 2) & 3;
  int s = 1;
  uint32_t mask = lo < hi ? unrank(K, lo, &s) : 0u;
  for (int64_t g0 = lo; g0 < hi; g0 += kWaveG) {
    const int cnt = (int)((hi - g0) < kWaveG ? (hi - g0) : kWaveG);
    for (int u0 = 0; u0 < cnt; u0 += 4) {
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
      __syncthreads();  // previous group done with the pair lists and tred
      for (int e = tid; e < 4 * K; e += kThreads) {
        const int q = e / K, t = e - (e / K) * K;
        const uint32_t mq = m4[0] * (q == 0) + m4[1] * (q == 1) + m4[2] * (q == 2) + m4[3] * (q == 3);
        if (q < nv && ((mq >> t) & 1u)) pl4[q * kMaxK + __popc(mq & ((1u << t) - 1u))] = t;
      }
      if (tid < nv) sz[u0 + tid] = tid == 0 ? s4[0] : (tid == 1 ? s4[1] : (tid == 2 ? s4[2] : s4[3]));
      __syncthreads();
      int smax = s4[0];
#pragma unroll
      for (int q = 1; q < 4; ++q)
        if (q < nv && s4[q] > smax) smax = s4[q];
      const int T4 = (smax + 1) >> 1;  // ceil(2 smax / 4)
      const int d_b = 2 * (b == 0 ? s4[0] : (b == 1 ? s4[1] : (b == 2 ? s4[2] : s4[3])));
      eval_qtile<K>(P, pl4, T4, d_b, b < nv, w, lane, xq, tred);
      __syncthreads();
      if (tid < 4 * 2 * K) {
        const int q = tid / (2 * K), jj = tid - q * (2 * K);
        double v = tred[(0 * 4 + q) * 2 * K + jj];
#pragma unroll
        for (int ww = 1; ww < 4; ++ww) v += tred[(ww * 4 + q) * 2 * K + jj];
        if (q < nv) trw[((jj >> 1) + 1) * (2 * kWaveG) + 2 * (u0 + q) + (jj & 1)] = 0.5 * v;
      }
    }
    __syncthreads();
    if (w == 0) combine_batch<K>(trw, sz, cnt, lane, sr, si, cr, ci);
    __syncthreads();
  }
}

}  // namespace

struct QtileLds {
  size_t A, modes, pl, xq, tred, trw, sz, terms, item, total;
};

__host__ __device__ inline QtileLds qtile_lds_layout(int nmax, int kmax, int stage_A) {
  QtileLds L;
  size_t off = 0;
  L.A = off;
  off += stage_A ? wal16(sizeof(double) * 2 * nmax * nmax) : 0;
  L.modes = off;
  off += wal16(sizeof(int32_t) * GBS_N_MAX);
  L.pl = off;
  off += wal16(sizeof(int32_t) * 4 * kMaxK);
  L.xq = off;
  off += wal16(sizeof(double) * 2 * 2 * kQtTiles * 64);
  L.tred = off;
  off += wal16(sizeof(double) * 4 * 4 * 2 * kmax);
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

template <int K>
__global__ __launch_bounds__(kThreads) void qtile_engine_kernel(EngineArgs args) {
  extern __shared__ __align__(16) unsigned char smem[];
  const QtileLds L = qtile_lds_layout(args.nmax, args.kmax, args.stage_A);
  double2* Alds = reinterpret_cast<double2*>(smem + L.A);
  int32_t* mlds = reinterpret_cast<int32_t*>(smem + L.modes);
  int32_t* pl4 = reinterpret_cast<int32_t*>(smem + L.pl);
  double2* xq = reinterpret_cast<double2*>(smem + L.xq);
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
      for (int e = tid; e < n * n; e += kThreads) {
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
    if (k == K) qtile_range<K>(P, item.lo, item.hi, pl4, xq, tred, trw, sz, terms, tid, sr, si, cr, ci);
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
