// Symmetric quad-tile subset engine, gfx950: a G x G grid of 4x4 tiles for d = 2|Z| <= 4G; built for
// G = 6 (|Z| = 9..12) and G = 7 (|Z| = 13, 14), both at two waves per SIMD. (An 8x8 grid for
// |Z| = 15, 16 needs more than 256 registers per wave and 74 KB of LDS for the published factors, so it
// runs at one wave per SIMD; it measured within 1% of the 16x16 tile engine there and is not built.)
//
// A workgroup of four waves evaluates four subsets at a time, one per block of
// v_mfma_f64_4x4x4_4b_f64 (block b = (lane >> 2) & 3, as in the quad engine); M_Z and its powers are
// G x G grids of 4x4 tiles in the quad engine's lane layout (lane x + 4b + 16y holds element (y, x) of
// the tile for block b). Every power Q satisfies Q[i][c] = Q[c^1][i^1], so tile (J, I) is a lane
// permutation of tile (I, J) and only the G(G+1)/2 tiles with I <= J are stored and multiplied; they
// are dealt to the waves in row-major order (G = 6: 6 / 5 / 5 / 5 tiles; G = 7: 7 each):
//   G = 6: wave 0: (0,0)..(0,5)   wave 1: (1,1)..(1,5)   wave 2: (2,2)..(2,5), (3,3)
//          wave 3: (3,4), (3,5), (4,4), (4,5), (5,5)
// Each wave's code is specialised for its tile set (rows and columns are compile-time constants), so
// every register index is static.
//
// A product Z = X Y publishes the stored tiles of both factors to LDS (a square publishes once). Each
// wave then accumulates its tiles over the k-tiles inside d; per k-tile it reads the A operands of its
// rows and the B operands of its columns once: A(I, K) by rows is stored tile (K, I) read at lane
// l ^ 17 when K <= I, else stored tile (I, K) transposed; B(K, J) is stored tile (K, J) when K <= J,
// else tile (J, K) read through (x, y) <- (y^1, x^1). Complex products use three real products per
// step. Traces need no exchange: tr(M^j) from the diagonal tiles, tr(P Q) pairs every stored tile of P
// with the same tile of Q at lane l ^ 17 (off-diagonal tiles count twice). Each wave reduces its
// partial traces over the 16 lanes of every block; the four waves' values are added in wave order
// through LDS, and the coefficient recursion and the compensated sum are those of the other engines.
#pragma once
#include "gbs_engine_common.h"
#include "gbs_quad_engine.h"

namespace gbs {
namespace {

__host__ __device__ constexpr int sqt_stored(int G) { return G * (G + 1) / 2; }
__host__ __device__ constexpr int sqt_q(int G) { return (sqt_stored(G) + 3) / 4; }  // most tiles per wave
__host__ __device__ constexpr int sqt_idx(int G, int I, int J) { return I * G - I * (I - 1) / 2 + (J - I); }

// The tile set of wave W: slot q holds tile (I[q], J[q]); rows / cols list the distinct ones, and slot q
// uses row ri[q] and column ci[q] of those lists.
template <int G>
struct SqtPlan {
  int nq, nr, nc;
  int I[sqt_q(G)], J[sqt_q(G)], ri[sqt_q(G)], ci[sqt_q(G)];
  int rows[G], cols[G];
};

template <int G>
constexpr SqtPlan<G> make_sqt_plan(int W) {
  SqtPlan<G> p{};
  // row-major order of the stored tiles, dealt in contiguous runs (the first waves take the remainder)
  constexpr int S = sqt_stored(G), base = S / 4, extra = S % 4;
  const int count = base + (W < extra ? 1 : 0);
  const int first = W * base + (W < extra ? W : extra);
  int t = 0;
  for (int I = 0; I < G; ++I)
    for (int J = I; J < G; ++J, ++t)
      if (t >= first && t < first + count) {
        const int q = p.nq++;
        p.I[q] = I;
        p.J[q] = J;
        int r = 0;
        while (r < p.nr && p.rows[r] != I) ++r;
        if (r == p.nr) p.rows[p.nr++] = I;
        p.ri[q] = r;
        int c = 0;
        while (c < p.nc && p.cols[c] != J) ++c;
        if (c == p.nc) p.cols[p.nc++] = J;
        p.ci[q] = c;
      }
  return p;
}

template <int G, int W>
struct SqtPlanOf {
  static constexpr SqtPlan<G> p = make_sqt_plan<G>(W);
};

template <int G>
struct SqtMat {
  double r[sqt_q(G)];
  double i[sqt_q(G)];
};

// A published tile keeps lane l's element at position sqt_pos(l) of its 64 (16-byte) slots: the lane
// number with bits 4..5 folded into bits 0..1. The transposed reads (lane (x, y) <- (y, x) and
// (y^1, x^1)) then hit eight different 16-byte bank groups in every run of eight lanes, as the direct
// and lane ^ 17 reads do, instead of four lanes sharing one (measured as LDS bank conflicts).
__host__ __device__ constexpr int sqt_pos(int l) { return l ^ ((l >> 4) & 3); }

// Per-lane slot positions of the own element and of the three permutations read (inside each block):
// lane ^ 17, transpose, flipped transpose.
struct SqtLanes {
  int self, l17, tr, tf;
};

__device__ __forceinline__ SqtLanes sqt_lanes(int lane) {
  const int x = lane & 3, b = (lane >> 2) & 3, y = lane >> 4;
  SqtLanes s;
  s.self = sqt_pos(lane);
  s.l17 = sqt_pos(lane ^ 17);
  s.tr = sqt_pos(y + 4 * b + 16 * x);
  s.tf = sqt_pos((y ^ 1) + 4 * b + 16 * (x ^ 1));
  return s;
}

// Z = X Y for wave W's tiles; T4 = ceil(max d / 4) over the four subsets (uniform). Z may alias X or Y.
template <int G, int W, bool SAME>
__device__ __forceinline__ void sqt_mul(const SqtMat<G>& X, const SqtMat<G>& Y, SqtMat<G>& Z, int T4, int lane,
                                        const SqtLanes& ln, double2* xq) {
  constexpr SqtPlan<G> P = SqtPlanOf<G, W>::p;
  constexpr int Q = sqt_q(G);
  double2* yq = SAME ? xq : xq + sqt_stored(G) * 64;
  // every wave done reading the previous product's factors before they are overwritten; waiting here
  // rather than at the end of that product lets a wave that finished its tiles early form its traces
  // while the others still multiply
  __syncthreads();
#pragma unroll
  for (int q = 0; q < P.nq; ++q)
    if (P.J[q] < T4) {
      const int t = sqt_idx(G, P.I[q], P.J[q]);
      lds_st2(xq, t * 64 + ln.self, make_double2(X.r[q], X.i[q]));
      if (!SAME) lds_st2(yq, t * 64 + ln.self, make_double2(Y.r[q], Y.i[q]));
    }
  __syncthreads();
  double t1[Q], t2[Q], t3[Q];
#pragma unroll
  for (int K = 0; K < G; ++K) {
    if (K < T4) {  // k-tiles beyond d hold zeros
      double2 b[G];
      double bs[G];
#pragma unroll
      for (int c = 0; c < P.nc; ++c) {
        const int J = P.cols[c];
        b[c] = K <= J ? lds_ld2(yq, sqt_idx(G, K, J) * 64 + ln.self) : lds_ld2(yq, sqt_idx(G, J, K) * 64 + ln.tf);
        bs[c] = b[c].x + b[c].y;
      }
      // one A operand (a row of the wave's tiles) at a time
#pragma unroll
      for (int r = 0; r < P.nr; ++r) {
        const int I = P.rows[r];
        const double2 a = K <= I ? lds_ld2(xq, sqt_idx(G, K, I) * 64 + ln.l17) : lds_ld2(xq, sqt_idx(G, I, K) * 64 + ln.tr);
        const double as = a.x + a.y;
#pragma unroll
        for (int q = 0; q < P.nq; ++q) {
          if (P.ri[q] == r && P.J[q] < T4) {
            const double2 bb = b[P.ci[q]];
            t1[q] = mfma4(a.x, bb.x, K == 0 ? 0.0 : t1[q]);
            t2[q] = mfma4(a.y, bb.y, K == 0 ? 0.0 : t2[q]);
            t3[q] = mfma4(as, bs[P.ci[q]], K == 0 ? 0.0 : t3[q]);
          }
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < P.nq; ++q) {
    const bool act = P.J[q] < T4;
    Z.r[q] = act ? t1[q] - t2[q] : 0.0;
    Z.i[q] = act ? t3[q] - t1[q] - t2[q] : 0.0;
  }
}

// per-lane partial of tr(X) over wave W's diagonal tiles
template <int G, int W>
__device__ __forceinline__ double2 sqt_diag(const SqtMat<G>& X, int lane) {
  constexpr SqtPlan<G> P = SqtPlanOf<G, W>::p;
  double2 t = make_double2(0.0, 0.0);
  if ((lane & 3) == (lane >> 4)) {
#pragma unroll
    for (int q = 0; q < P.nq; ++q)
      if (P.I[q] == P.J[q]) {
        t.x += X.r[q];
        t.y += X.i[q];
      }
  }
  return t;
}

// per-lane partial of tr(X Y) over wave W's tiles (off-diagonal tiles twice, for their mirrors)
template <int G, int W>
__device__ __forceinline__ double2 sqt_pair(const SqtMat<G>& X, const SqtMat<G>& Y) {
  constexpr SqtPlan<G> P = SqtPlanOf<G, W>::p;
  double2 d = make_double2(0.0, 0.0), o = make_double2(0.0, 0.0);
#pragma unroll
  for (int q = 0; q < P.nq; ++q) {
    double2& t = P.I[q] == P.J[q] ? d : o;
    const double yr = swap17(Y.r[q]);
    const double yi = swap17(Y.i[q]);
    t.x = fma(X.r[q], yr, t.x);
    t.x = fma(-X.i[q], yi, t.x);
    t.y = fma(X.r[q], yi, t.y);
    t.y = fma(X.i[q], yr, t.y);
  }
  return make_double2(fma(2.0, o.x, d.x), fma(2.0, o.y, d.y));
}

// Traces are block-reduced four at a time as the chain forms them (push_trace).
template <int K, int G, int W, int OI, int NS>
__device__ __forceinline__ void run_ops_sqt(SqtMat<G> (&S)[NS], double (&tb)[4], double* tred_b, int T4, int lane,
                                            const SqtLanes& ln, double2* xq) {
  if constexpr (OI < kChainTable[K].nops) {
    constexpr Op op = kChainTable[K].ops[OI];
    if constexpr (op.type == OP_MUL) {
      sqt_mul<G, W, op.a == op.b>(S[op.a], S[op.b], S[op.x], T4, lane, ln, xq);
    } else {
      const double2 p = op.type == OP_TDIAG ? sqt_diag<G, W>(S[op.a], lane) : sqt_pair<G, W>(S[op.a], S[op.b]);
      push_trace<K, OI>(tb, fold32(p.x, p.y), lane, [&](int j, int part, double v) { lds_st(tred_b, (j - 1) * 2 + part, v); });
    }
    run_ops_sqt<K, G, W, OI + 1, NS>(S, tb, tred_b, T4, lane, ln, xq);
  }
}

// Four subsets (one per block): gather wave W's tiles of M_Z, run the chain program, leave the wave's
// block-reduced partial traces in tred[((W * 4 + b) * K + j - 1) * 2 + part].
// Not inlined: with the four wave-specialised copies in one body the register allocator spills; as
// separate functions each fits two waves per SIMD.
template <int K, int G, int W>
__device__ __noinline__ void eval_sqt(const PatternView& Pv, const int32_t* pl4, int T4, int d_b, bool valid_b,
                                         int lane, double2* xq, double* tred) {
  constexpr SqtPlan<G> P = SqtPlanOf<G, W>::p;
  constexpr int NS = kChainTable[K].nslots;
  T4 = __builtin_amdgcn_readfirstlane(T4);  // uniform: the k-tile and output-tile tests become scalar branches
  const int b = (lane >> 2) & 3;
  const int x = lane & 3, y = lane >> 4;
  const int32_t* pl = pl4 + b * kMaxK;
  SqtMat<G> S[NS];
  const int dv = valid_b ? d_b : 0;  // blocks past the last subset gather zeros
#pragma unroll
  for (int q = 0; q < P.nq; ++q) {
    const int a = 4 * P.I[q] + y, c = 4 * P.J[q] + x;
    double vr = 0.0, vi = 0.0;
    if (a < dv && c < dv) {
      const int bb = a ^ 1;  // M = X A_Z: row a of M is row a^1 of A_Z
      const int i = 2 * ((lds_i32*)pl)[bb >> 1] + (bb & 1), j = 2 * ((lds_i32*)pl)[c >> 1] + (c & 1);
      const double2 e = Pv.at_as(i, j);
      vr = e.x;
      vi = e.y;
    }
    S[0].r[q] = vr;
    S[0].i[q] = vi;
  }
  double tb[4];
  run_ops_sqt<K, G, W, 0, NS>(S, tb, tred + (W * 4 + b) * K * 2, T4, lane, sqt_lanes(lane), xq);
}

// Subsets [lo, hi) of one pattern on the workgroup, four at a time.
template <int K, int G>
__device__ void sqt_range(const PatternView& Pv, int64_t lo, int64_t hi, int32_t* pl4, double2* xq, double* tred,
                          double* trw, int32_t* sz, int tid, double& sr, double& si, double& cr,
                          double& ci) {
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
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
      switch (w) {
        case 0: eval_sqt<K, G, 0>(Pv, pl4, T4, d_b, b < nv, lane, xq, tred); break;
        case 1: eval_sqt<K, G, 1>(Pv, pl4, T4, d_b, b < nv, lane, xq, tred); break;
        case 2: eval_sqt<K, G, 2>(Pv, pl4, T4, d_b, b < nv, lane, xq, tred); break;
        default: eval_sqt<K, G, 3>(Pv, pl4, T4, d_b, b < nv, lane, xq, tred); break;
      }
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

struct SqtLds {
  size_t A, modes, pl, xq, tred, trw, sz, item, total;
};

__host__ __device__ inline SqtLds sqt_lds_layout(int G, int nmax, int kmax, int stage_A) {
  SqtLds L;
  size_t off = 0;
  L.A = off;
  off += stage_A ? wal16(sizeof(double) * 2 * nmax * nmax) : 0;
  L.modes = off;
  off += wal16(sizeof(int32_t) * GBS_N_MAX);
  L.pl = off;
  off += wal16(sizeof(int32_t) * 4 * kMaxK);
  L.xq = off;  // the stored tiles of both factors of a product
  off += wal16(sizeof(double) * 2 * 2 * sqt_stored(G) * 64);
  L.tred = off;
  off += wal16(sizeof(double) * 4 * 4 * 2 * kmax);
  L.trw = off;
  off += wal16(sizeof(double) * (kmax + 1) * 2 * kWaveG);
  L.sz = off;
  off += wal16(sizeof(int32_t) * kWaveG);
  L.item = off;
  off += 16;
  L.total = off;
  return L;
}

template <int K, int G>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(G <= 7 ? 2 : 1, 8))) void sqt_engine_kernel(
    EngineArgs args) {
  extern __shared__ __align__(16) unsigned char smem[];
  const SqtLds L = sqt_lds_layout(G, args.nmax, args.kmax, args.stage_A);
  double2* Alds = reinterpret_cast<double2*>(smem + L.A);
  int32_t* mlds = reinterpret_cast<int32_t*>(smem + L.modes);
  int32_t* pl4 = reinterpret_cast<int32_t*>(smem + L.pl);
  double2* xq = reinterpret_cast<double2*>(smem + L.xq);
  double* tred = reinterpret_cast<double*>(smem + L.tred);
  double* trw = reinterpret_cast<double*>(smem + L.trw);
  int32_t* sz = reinterpret_cast<int32_t*>(smem + L.sz);
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
    if (k == K) sqt_range<K, G>(P, item.lo, item.hi, pl4, xq, tred, trw, sz, tid, sr, si, cr, ci);
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
