// Strip subset engine for 8 < |Z| <= 12 (16 < d = 2|Z| <= 24), gfx950.
//
// One wave evaluates one subset at a time on v_mfma_f64_4x4x4_4b_f64, whose four blocks here hold
// four neighbouring column tiles of one tile row: a d x d complex matrix is T4 tile rows
// (T4 = ceil(d/4) <= 6) of NR = ceil(T4/4) registers per component, and block b of register (I, R)
// holds tile (I, 4R + b) in the quad engine's tile layout (lane x + 4b + 16y: element (y, x)). The
// 4x4x4 FP64 MFMA sustains about 1.5x the rate of the 16x16x4 one on this device, and 4-wide tiles
// pad d to a multiple of 4 instead of 16.
//
// For Z = X Y, output register (I, R) accumulates over the k-tiles K inside d the product of X's
// tile (I, K) -- broadcast to all four blocks and put into A-operand order (element (x, y) at lane
// x + 4b + 16y) by one ds_bpermute per 32-bit half -- with Y's register (K, R) as the B operand.
// Row I of Z needs only row I of X, so Z may take X's registers row by row; powers of M_Z commute,
// so a product that overwrites its second factor swaps the factors. Complex products use three real
// products per step. Traces are tile-local as in the other engines (tr(P Q) pairs each register of
// P with Q's register read at lane l ^ 17); their reduction, the coefficient recursion and the
// compensated sum are the register engine's. No LDS traffic besides lane exchanges, no barriers.
#pragma once

namespace gbs {
namespace {

template <int T4>
struct SMat {
  static constexpr int NR = (T4 + 3) / 4;
  double r[T4][NR];
  double i[T4][NR];
};

__device__ __forceinline__ double bperm(int addr, double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)(unsigned)b);
  const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(unsigned)(b >> 32));
  return join((unsigned)lo, (unsigned)hi);
}

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
    run_ops_strip<K, T4, 0, NS>(S, park, addr, (d + 3) >> 2, lane);
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
      if (2 * s <= 4 * TL)
        eval_strip<K, TL>(P, pl, 2 * s, trw, u, park, lane);
      else
        eval_strip<K, TH>(P, pl, 2 * s, trw, u, park, lane);
    }
    wave_sync();
    combine_batch<K>(trw, sz, terms, cnt, lane, sr, si, cr, ci);
    wave_sync();
  }
}

}  // namespace

// LDS: the register engine's layout, then one trace-parking area of kmax x 64 doubles per wave.
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
