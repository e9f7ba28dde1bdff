// Strip subset engine for 8 < |Z| <= 12 (16 < d = 2|Z| <= 24), gfx950.
//
// One wave evaluates one subset at a time on v_mfma_f64_4x4x4_4b_f64, whose four blocks here hold
// four neighbouring column tiles of one tile row: a d x d complex matrix is T4 tile rows
// (T4 = ceil(d/4) <= 6) of NR = ceil(T4/4) registers per component, and block b of register (I, R)
// holds tile (I, 4R + b) in the quad engine's tile layout (lane x + 4b + 16y: element (y, x)). Both
// FP64 MFMA shapes run at the same 32 flops per cycle per SIMD; 4-wide tiles pad d to a multiple of
// 4 instead of 16.
//
// For Z = X Y, output register (I, R) accumulates over the k-tiles K inside d the product of X's
// tile (I, K) -- broadcast to all four blocks and put into A-operand order (element (x, y) at lane
// x + 4b + 16y) by one ds_bpermute per 32-bit half -- with Y's register (K, R) as the B operand.
// Row I of Z needs only row I of X, so Z may take X's registers row by row; powers of M_Z commute,
// so a product that overwrites its second factor swaps the factors. Complex products use three real
// products per step. Traces are tile-local as in the other engines (tr(P Q) pairs each register of
// P with Q's register read at lane l ^ 17); their reduction, the coefficient recursion and the
// compensated sum are the shared ones (gbs_engine_common.h). No LDS traffic besides lane exchanges, no barriers.
#pragma once
#include "gbs_engine_common.h"
#include "gbs_quad_engine.h"

namespace gbs {
namespace {

template <int T4>
struct SMat {
  static constexpr int NR = (T4 + 3) / 4;
  double r[T4][NR];
  double i[T4][NR];
};


// Z = X Y. addr[c]: byte address of the lane holding, in block c of a register, the element that
// lane needs as A operand (row x, column y of that block's tile).
template <int T4>
__device__ __forceinline__ void strip_mul(const SMat<T4>& X, const SMat<T4>& Y, SMat<T4>& Z, const int (&addr)[4],
                                          int T4d) {
  constexpr int NR = SMat<T4>::NR;
  SMat<T4> acc;
#pragma unroll
  for (int I = 0; I < T4; ++I) {
    double t1[NR], t2[NR], t3[NR];
#pragma unroll
    for (int K = 0; K < T4; ++K) {
      if (K == 0 || K < T4d) {  // k-tiles beyond d hold zeros
        const double ar = bperm(addr[K & 3], X.r[I][K >> 2]);
        const double ai = bperm(addr[K & 3], X.i[I][K >> 2]);
        const double as = ar + ai;
#pragma unroll
        for (int R = 0; R < NR; ++R) {
          t1[R] = mfma4(ar, Y.r[K][R], K == 0 ? 0.0 : t1[R]);
          t2[R] = mfma4(ai, Y.i[K][R], K == 0 ? 0.0 : t2[R]);
          t3[R] = mfma4(as, Y.r[K][R] + Y.i[K][R], K == 0 ? 0.0 : t3[R]);
        }
      }
    }
#pragma unroll
    for (int R = 0; R < NR; ++R) {
      acc.r[I][R] = t1[R] - t2[R];
      acc.i[I][R] = t3[R] - t1[R] - t2[R];
    }
  }
  Z = acc;
}

// per-lane partial of tr(X): diagonal tile (I, I) is block I % 4 of register (I, I / 4)
template <int T4>
__device__ __forceinline__ double2 strip_diag(const SMat<T4>& X, int lane) {
  double2 t = make_double2(0.0, 0.0);
  if ((lane & 3) == (lane >> 4)) {
    const int b = (lane >> 2) & 3;
#pragma unroll
    for (int I = 0; I < T4; ++I)
      if (b == (I & 3)) {
        t.x += X.r[I][I >> 2];
        t.y += X.i[I][I >> 2];
      }
  }
  return t;
}

// per-lane partial of tr(X Y) = sum X[i][c] Y[i^1][c^1]
template <int T4>
__device__ __forceinline__ double2 strip_pair(const SMat<T4>& X, const SMat<T4>& Y) {
  constexpr int NR = SMat<T4>::NR;
  double2 t = make_double2(0.0, 0.0);
#pragma unroll
  for (int I = 0; I < T4; ++I)
#pragma unroll
    for (int R = 0; R < NR; ++R) {
      const double yr = swap17(Y.r[I][R]);
      const double yi = swap17(Y.i[I][R]);
      t.x = fma(X.r[I][R], yr, t.x);
      t.x = fma(-X.i[I][R], yi, t.x);
      t.y = fma(X.r[I][R], yi, t.y);
      t.y = fma(X.i[I][R], yr, t.y);
    }
  return t;
}

// Runs the chain program; trace t_j's per-lane partial, folded over lane bit 5, is parked in LDS at
// park[(j - 1) * 64 + lane] until the chain is done (it would otherwise hold k registers while the
// powers are live).
template <int K, int T4, int OI, int NS>
__device__ __forceinline__ void run_ops_strip(SMat<T4> (&S)[NS], double* park, const int (&addr)[4], int T4d,
                                              int lane) {
  if constexpr (OI < kChainTable[K].nops) {
    constexpr Op op = kChainTable[K].ops[OI];
    if constexpr (op.type == OP_MUL) {
      if constexpr (op.x == op.b && op.a != op.b)
        strip_mul<T4>(S[op.b], S[op.a], S[op.x], addr, T4d);  // powers commute: overwrite the first factor
      else
        strip_mul<T4>(S[op.a], S[op.b], S[op.x], addr, T4d);
    } else if constexpr (op.type == OP_TDIAG) {
      const double2 p = strip_diag<T4>(S[op.a], lane);
      park[(op.x - 1) * 64 + lane] = fold32(p.x, p.y);
    } else {
      const double2 p = strip_pair<T4>(S[op.a], S[op.b]);
      park[(op.x - 1) * 64 + lane] = fold32(p.x, p.y);
    }
    run_ops_strip<K, T4, OI + 1, NS>(S, park, addr, T4d, lane);
  }
}

// One subset with d <= 4 T4: build M_Z, run the chain program, reduce the traces into slot u.
template <int K, int T4>
__device__ __forceinline__ void eval_strip(const PatternView& P, const int32_t* pl, int d, double* trw, int u,
                                           double* park, int lane) {
  constexpr int NS = kChainTable[K].nslots;
  constexpr int NR = SMat<T4>::NR;
  const int x = lane & 3, b = (lane >> 2) & 3, y = lane >> 4;
  int addr[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) addr[c] = (y + 4 * c + 16 * x) * 4;
  {
    SMat<T4> S[NS];
    if (P.lds) {
      int cix[NR];
#pragma unroll
      for (int R = 0; R < NR; ++R) cix[R] = mz_col(P, pl, 4 * (4 * R + b) + x, d);
#pragma unroll
      for (int I = 0; I < T4; ++I) {
        const int ro = mz_row(P, pl, 4 * I + y, d);
#pragma unroll
        for (int R = 0; R < NR; ++R) {
          const double2 e = mz_at(P, ro + cix[R]);
          S[0].r[I][R] = e.x;
          S[0].i[I][R] = e.y;
        }
      }
    } else {
#pragma unroll
      for (int I = 0; I < T4; ++I)
#pragma unroll
        for (int R = 0; R < NR; ++R) {
          const int a = 4 * I + y, c = 4 * (4 * R + b) + x;
          double vr = 0.0, vi = 0.0;
          if (a < d && c < d) {
            const int bb = a ^ 1;  // M = X A_Z: row a of M is row a^1 of A_Z
            const double2 e = P.at(2 * pl[bb >> 1] + (bb & 1), 2 * pl[c >> 1] + (c & 1));
            vr = e.x;
            vi = e.y;
          }
          S[0].r[I][R] = vr;
          S[0].i[I][R] = vi;
        }
    }
    run_ops_strip<K, T4, 0, NS>(S, park, addr, (d + 3) >> 2, lane);
  }
  double w[K];
#pragma unroll
  for (int j = 0; j < K; ++j) w[j] = park[j * 64 + lane];  // each lane reads only what it wrote
  reduce_folded<K>(w, lane, [&](int j, int part, double v) { trw[j * (2 * kWaveG) + 2 * u + part] = 0.5 * v; });
}

// Five tile rows (16 < d <= 20) without the padded second register per row: main register I
// holds tiles (I, 0..3) in blocks 0..3 as above; side register g holds column tile 4 of rows
// 4g + b in block b (side register 1 has only row 4, its blocks 1..3 stay zero). For Z = X Y:
//  * A operands use the pair symmetry: X's tile (I, K) by rows is X's tile (K, I) read at
//    (x^1, y^1), broadcast from the block that holds it (main register K for I < 4, side register
//    K / 4 for I = 4) -- one ds_swizzle per 32-bit half, within each 32-lane half of the wave;
//  * side outputs, rows 0..3: block b needs X's tile (b, K) by rows, which is main register K read
//    at lane l ^ 17 (no broadcast); B is Y's tile (K, 4), broadcast from its side register; row 4
//    as for the main outputs, masked to block 0.
// 105 instead of 150 MFMAs per product and 7 instead of 10 registers per component.
struct S5Mat {
  double mr[5], mi[5];  // main registers, rows 0..4
  double sr[2], si[2];  // side registers
};

// Lane exchanges within each 32-lane half by ds_swizzle (bit mode: source lane bits 0..4 are
// ((lane & AND) | OR) ^ XOR), no address registers. swz_tr(c, v): the tile in block c read at
// (x^1, y^1) -- by the pair symmetry of powers, the transposed neighbour tile in A order;
// swz_bc(c, v): the tile in block c as stored (B order).
template <int AND, int OR, int XOR>
__device__ __forceinline__ double swz(double v) {
  constexpr int pat = AND | (OR << 5) | (XOR << 10);
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_swizzle((int)(unsigned)b, pat);
  const int hi = __builtin_amdgcn_ds_swizzle((int)(unsigned)(b >> 32), pat);
  return join((unsigned)lo, (unsigned)hi);
}
// c is a constant after unrolling; the switch folds to one exchange
__device__ __forceinline__ double swz_tr(int c, double v) {
  switch (c & 3) {
    case 0: return swz<0x13, 0 << 2, 0x11>(v);
    case 1: return swz<0x13, 1 << 2, 0x11>(v);
    case 2: return swz<0x13, 2 << 2, 0x11>(v);
    default: return swz<0x13, 3 << 2, 0x11>(v);
  }
}
__device__ __forceinline__ double swz_bc(int c, double v) {
  switch (c & 3) {
    case 0: return swz<0x13, 0 << 2, 0>(v);
    case 1: return swz<0x13, 1 << 2, 0>(v);
    case 2: return swz<0x13, 2 << 2, 0>(v);
    default: return swz<0x13, 3 << 2, 0>(v);
  }
}

__device__ __forceinline__ void strip5_mul(const S5Mat& X, const S5Mat& Y, S5Mat& Z, const int (&addr)[4],
                                           const int (&baddr)[4], bool block0) {
  (void)addr;
  (void)baddr;
  S5Mat acc;
#pragma unroll
  for (int I = 0; I < 5; ++I) {
    double t1, t2, t3;
#pragma unroll
    for (int K = 0; K < 5; ++K) {
      // X's tile (I, K) by rows = X's tile (K, I) read at (x^1, y^1), broadcast from its block
      double ar, ai;
      if (I < 4) {
        ar = swz_tr(I, X.mr[K]);
        ai = swz_tr(I, X.mi[K]);
      } else {
        ar = swz_tr(K, X.sr[K >> 2]);
        ai = swz_tr(K, X.si[K >> 2]);
      }
      t1 = mfma4(ar, Y.mr[K], K == 0 ? 0.0 : t1);
      t2 = mfma4(ai, Y.mi[K], K == 0 ? 0.0 : t2);
      t3 = mfma4(ar + ai, Y.mr[K] + Y.mi[K], K == 0 ? 0.0 : t3);
    }
    acc.mr[I] = t1 - t2;
    acc.mi[I] = t3 - t1 - t2;
  }
  double u1[2], u2[2], u3[2];
#pragma unroll
  for (int K = 0; K < 5; ++K) {
    const double br = swz_bc(K, Y.sr[K >> 2]);
    const double bi = swz_bc(K, Y.si[K >> 2]);
    const double bs = br + bi;
    // rows 0..3
    {
      const double ar = swz<0x1f, 0, 0x11>(X.mr[K]);
      const double ai = swz<0x1f, 0, 0x11>(X.mi[K]);
      u1[0] = mfma4(ar, br, K == 0 ? 0.0 : u1[0]);
      u2[0] = mfma4(ai, bi, K == 0 ? 0.0 : u2[0]);
      u3[0] = mfma4(ar + ai, bs, K == 0 ? 0.0 : u3[0]);
    }
    // row 4 (block 0 only): X's tile (4, K) by rows = X's tile (K, 4), in side register K / 4;
    // blocks 1..3 compute a product that is discarded below (one select per result register)
    {
      const double ar = swz_tr(K, X.sr[K >> 2]);
      const double ai = swz_tr(K, X.si[K >> 2]);
      u1[1] = mfma4(ar, br, K == 0 ? 0.0 : u1[1]);
      u2[1] = mfma4(ai, bi, K == 0 ? 0.0 : u2[1]);
      u3[1] = mfma4(ar + ai, bs, K == 0 ? 0.0 : u3[1]);
    }
  }
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    acc.sr[g] = u1[g] - u2[g];
    acc.si[g] = u3[g] - u1[g] - u2[g];
  }
  acc.sr[1] = block0 ? acc.sr[1] : 0.0;  // tiles (5..7, 4) do not exist
  acc.si[1] = block0 ? acc.si[1] : 0.0;
  Z = acc;
}

__device__ __forceinline__ double2 strip5_diag(const S5Mat& X, int lane) {
  double2 t = make_double2(0.0, 0.0);
  if ((lane & 3) == (lane >> 4)) {
    const int b = (lane >> 2) & 3;
#pragma unroll
    for (int I = 0; I < 4; ++I)
      if (b == I) {
        t.x += X.mr[I];
        t.y += X.mi[I];
      }
    if (b == 0) {  // tile (4, 4)
      t.x += X.sr[1];
      t.y += X.si[1];
    }
  }
  return t;
}

__device__ __forceinline__ double2 strip5_pair(const S5Mat& X, const S5Mat& Y) {
  double2 t = make_double2(0.0, 0.0);
  auto acc = [&](double xr, double xi, double yr0, double yi0) {
    const double yr = swap17(yr0), yi = swap17(yi0);
    t.x = fma(xr, yr, t.x);
    t.x = fma(-xi, yi, t.x);
    t.y = fma(xr, yi, t.y);
    t.y = fma(xi, yr, t.y);
  };
#pragma unroll
  for (int I = 0; I < 5; ++I) acc(X.mr[I], X.mi[I], Y.mr[I], Y.mi[I]);
#pragma unroll
  for (int g = 0; g < 2; ++g) acc(X.sr[g], X.si[g], Y.sr[g], Y.si[g]);
  return t;
}

template <int K, int OI, int NS>
__device__ __forceinline__ void run_ops_strip5(S5Mat (&S)[NS], double* park, const int (&addr)[4],
                                               const int (&baddr)[4], bool block0, int lane) {
  if constexpr (OI < kChainTable[K].nops) {
    constexpr Op op = kChainTable[K].ops[OI];
    if constexpr (op.type == OP_MUL) {
      if constexpr (op.x == op.b && op.a != op.b)
        strip5_mul(S[op.b], S[op.a], S[op.x], addr, baddr, block0);  // powers commute
      else
        strip5_mul(S[op.a], S[op.b], S[op.x], addr, baddr, block0);
    } else if constexpr (op.type == OP_TDIAG) {
      const double2 p = strip5_diag(S[op.a], lane);
      park[(op.x - 1) * 64 + lane] = fold32(p.x, p.y);
    } else {
      const double2 p = strip5_pair(S[op.a], S[op.b]);
      park[(op.x - 1) * 64 + lane] = fold32(p.x, p.y);
    }
    run_ops_strip5<K, OI + 1, NS>(S, park, addr, baddr, block0, lane);
  }
}

template <int K>
__device__ __forceinline__ void eval_strip5(const PatternView& P, const int32_t* pl, int d, double* trw, int u,
                                            double* park, int lane) {
  constexpr int NS = kChainTable[K].nslots;
  const int x = lane & 3, b = (lane >> 2) & 3, y = lane >> 4;
  int addr[4], baddr[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    addr[c] = (y + 4 * c + 16 * x) * 4;   // tile in block c, transposed (A order)
    baddr[c] = (x + 4 * c + 16 * y) * 4;  // tile in block c, as stored (B order)
  }
  auto at = [&](int a, int c) -> double2 {
    if (a < d && c < d) {
      const int bb = a ^ 1;  // M = X A_Z: row a of M is row a^1 of A_Z
      return P.at(2 * pl[bb >> 1] + (bb & 1), 2 * pl[c >> 1] + (c & 1));
    }
    return make_double2(0.0, 0.0);
  };
  {
    S5Mat S[NS];
    if (P.lds) {
      const int cm = mz_col(P, pl, 4 * b + x, d), cs = mz_col(P, pl, 16 + x, d);
#pragma unroll
      for (int I = 0; I < 5; ++I) {
        const double2 e = mz_at(P, mz_row(P, pl, 4 * I + y, d) + cm);
        S[0].mr[I] = e.x;
        S[0].mi[I] = e.y;
      }
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        const double2 e = mz_at(P, mz_row(P, pl, 4 * (4 * g + b) + y, d) + cs);
        S[0].sr[g] = e.x;
        S[0].si[g] = e.y;
      }
    } else {
#pragma unroll
      for (int I = 0; I < 5; ++I) {
        const double2 e = at(4 * I + y, 4 * b + x);
        S[0].mr[I] = e.x;
        S[0].mi[I] = e.y;
      }
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        const double2 e = at(4 * (4 * g + b) + y, 16 + x);
        S[0].sr[g] = e.x;
        S[0].si[g] = e.y;
      }
    }
    run_ops_strip5<K, 0, NS>(S, park, addr, baddr, b == 0, lane);
  }
  double w[K];
#pragma unroll
  for (int j = 0; j < K; ++j) w[j] = park[j * 64 + lane];  // each lane reads only what it wrote
  reduce_folded<K>(w, lane, [&](int j, int part, double v) { trw[j * (2 * kWaveG) + 2 * u + part] = 0.5 * v; });
}

// The subsets [lo, hi) of one pattern on one wave; each subset uses the tile-row count TL or TH.
template <int K, int TL, int TH>
__device__ void strip_range(const PatternView& P, int64_t lo, int64_t hi, int32_t* pl, double* trw, int32_t* sz,
                            double2* terms, double* park, int lane, double& sr, double& si, double& cr, double& ci) {
  int s = 1;
  uint32_t mask = lo < hi ? unrank(K, lo, &s) : 0u;
  for (int64_t g0 = lo; g0 < hi; g0 += kWaveG) {
    const int cnt = (int)((hi - g0) < kWaveG ? (hi - g0) : kWaveG);
    for (int u = 0; u < cnt; ++u) {
      if (u > 0 || g0 > lo) mask = next_subset(mask, K, &s);
      wave_sync();  // previous subset's pair list no longer read
      if (lane < K && ((mask >> lane) & 1u)) pl[__popc(mask & ((1u << lane) - 1u))] = lane;
      if (lane == 0) sz[u] = s;
      wave_sync();
      if constexpr (TL == 5 && TH == 5)
        eval_strip5<K>(P, pl, 2 * s, trw, u, park, lane);
      else if (2 * s <= 4 * TL)
        eval_strip<K, TL>(P, pl, 2 * s, trw, u, park, lane);
      else
        eval_strip<K, TH>(P, pl, 2 * s, trw, u, park, lane);
    }
    wave_sync();
    combine_batch<K>(trw, sz, cnt, lane, sr, si, cr, ci);
    wave_sync();
  }
}

}  // namespace

// LDS: the shared item-loop layout (wave_lds_layout), then one trace-parking area of kmax x 64 doubles per wave.
__host__ __device__ inline size_t strip_lds_bytes(int nmax, int kmax, int stage_A) {
  return wave_lds_layout(nmax, kmax, stage_A).total + sizeof(double) * 4 * kmax * 64;
}

// Kernels: subsets with 4 (TL - 1) < 2|Z| <= 4 TH, one wave per subset.
template <int K, int TL, int TH>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 8))) void
strip_engine_kernel(EngineArgs args) {
  extern __shared__ __align__(16) unsigned char smem[];
  const WaveLds L = wave_lds_layout(args.nmax, args.kmax, args.stage_A);
  wave_items<K>(args, smem, [&](const PatternView& P, int64_t lo, int64_t hi, int wave, int lane, double& sr,
                                double& si, double& cr, double& ci) {
    int32_t* pl = reinterpret_cast<int32_t*>(smem + L.pl) + wave * kMaxK;
    double* trw = reinterpret_cast<double*>(smem + L.trw) + (size_t)wave * (args.kmax + 1) * 2 * kWaveG;
    int32_t* sz = reinterpret_cast<int32_t*>(smem + L.sz) + wave * kWaveG;
    double2* terms = reinterpret_cast<double2*>(smem + L.terms) + wave * kWaveG;
    double* park = reinterpret_cast<double*>(smem + L.total) + (size_t)wave * args.kmax * 64;
    strip_range<K, TL, TH>(P, lo, hi, pl, trw, sz, terms, park, lane, sr, si, cr, ci);
  });
}

}  // namespace gbs
