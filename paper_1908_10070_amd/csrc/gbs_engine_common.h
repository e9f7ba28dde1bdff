// Pieces shared by the subset engines (gfx950): tile layouts of the 16x16x4 FP64 MFMA, lane
// exchanges, the wave reduction of per-lane trace partials, the gather of M_Z from the staged pattern
// matrix, subset enumeration, the trace extension by Newton's identities, the coefficient recursion
// with compensated summation, and the persistent item loop of the engines that give each wave its
// own subsets.
//
// Conventions used by every engine:
//   * A d x d complex matrix in the v_mfma_f64_16x16x4f64 layout is a grid of 16x16 FP64 tiles, each
//     a pair (re, im) of 4-double registers; lane l = x + 16 y, register r of a tile holds element
//     (row y + 4 r, column x). Entries beyond d are zero.
//   * Every power Q of M_Z = X A_Z satisfies Q^t = X Q X (X swaps the two indices of each pair, and
//     A_Z is symmetric), so Q[i][c] = Q[c^1][i^1]: the A operand of a product -- Q by rows where the
//     output layout holds it by columns -- is the same register of the transposed tile read from
//     lane l ^ 17 (x^1, y^1), and tr(P Q) = sum_{i,c} P[i][c] Q[i^1][c^1] pairs each register of P
//     with the same register of Q at lane l ^ 17.
//   * Each trace's per-lane partial is folded over lane bit 5 (v_permlane32_swap, real part kept in
//     the low half, imaginary in the high half) as soon as it is formed; the folded traces are then
//     reduced together by a transposed butterfly on permlane16 swaps and DPP row moves.
//   * A workgroup of 4 waves takes one work item -- a range of one pattern's canonical subset order
//     -- stages the pattern matrix in LDS once (n <= 32) and gives each wave a contiguous quarter.
//     Traces of 32 subsets are buffered per wave; 32 lanes then run the coefficient recursion and one
//     lane adds the signed terms into a compensated running sum. The four wave partials are combined
//     in wave order, so an item's partial depends only on its range.
#pragma once
#include <hip/hip_runtime.h>

#include "gbs_chain_table.h"
#include "gbs_internal.h"
#include "gbs_tables.h"

namespace gbs {

namespace {

constexpr int cmin(int a, int b) { return a < b ? a : b; }

// s + c += x with Neumaier's compensation (per component, fixed order).
__device__ __forceinline__ void neumaier(double& s, double& c, double x) {
  double t = s + x;
  if (fabs(s) >= fabs(x))
    c += (s - t) + x;
  else
    c += (x - t) + s;
  s = t;
}

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kWaveG = 32;  // subsets buffered per wave before the coefficient step

template <int T>
struct CMat {
  d4 r[T][T];
  d4 i[T][T];
};

// lane l ^ 17 (x ^ 1, y ^ 1 within a tile): ds_swizzle in bit mode (xor 0x11 inside each 32-lane
// half), no address register
__device__ __forceinline__ double swap17(double v) {
  constexpr int pat = 0x1f | (0 << 5) | (0x11 << 10);
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_swizzle((int)(unsigned)b, pat);
  const int hi = __builtin_amdgcn_ds_swizzle((int)(unsigned)(b >> 32), pat);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Complex products use three real products per step (Gauss): with T1 = Xr Yr, T2 = Xi Yi,
// T3 = (Xr + Xi)(Yr + Yi), Re = T1 - T2 and Im = T3 - T1 - T2. That is 3/4 of the MFMA work for two
// extra additions per step. The imaginary part's rounding bound is about twice the four-product one;
// measured hafnian errors at n = 36..44 against the long-double oracle were no larger, so every engine
// uses it at every k.

// per-lane partial of tr(X): the diagonal element this lane holds, if any
template <int T>
__device__ __forceinline__ double2 tdiag(const CMat<T>& X, int lane) {
  // the lane's diagonal element, if it holds one, is register r = (x - y) / 4 of each diagonal
  // tile; 0/1 weights pick it without a branch (exact for finite entries: the rest adds zeros)
  const int x = lane & 15, y = lane >> 4;
  const bool on = x >= y && ((x - y) & 3) == 0;
  const int r = (x - y) >> 2;
  double wgt[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) wgt[q] = on && r == q ? 1.0 : 0.0;
  double2 t = make_double2(0.0, 0.0);
#pragma unroll
  for (int I = 0; I < T; ++I)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      t.x = fma(wgt[q], X.r[I][I][q], t.x);
      t.y = fma(wgt[q], X.i[I][I][q], t.y);
    }
  return t;
}

// per-lane partial of tr(X Y) = sum X[i][c] Y[i^1][c^1]
template <int T>
__device__ __forceinline__ double2 tpair(const CMat<T>& X, const CMat<T>& Y) {
  double2 t = make_double2(0.0, 0.0);
#pragma unroll
  for (int I = 0; I < T; ++I)
#pragma unroll
    for (int C = 0; C < T; ++C)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double yr = swap17(Y.r[I][C][r]);
        const double yi = swap17(Y.i[I][C][r]);
        const double xr = X.r[I][C][r], xi = X.i[I][C][r];
        t.x = fma(xr, yr, t.x);
        t.x = fma(-xi, yi, t.x);
        t.y = fma(xr, yi, t.y);
        t.y = fma(xi, yr, t.y);
      }
  return t;
}

// Lane exchanges of 64-bit values on the VALU (no LDS traffic): DPP moves within a row of 16
// lanes, v_permlane{16,32}_swap across rows. The two 32-bit halves move separately.
__device__ __forceinline__ double join(unsigned lo, unsigned hi) {
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// v from the lane whose byte address is addr (ds_bpermute, one per 32-bit half)
__device__ __forceinline__ double bperm(int addr, double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)(unsigned)b);
  const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(unsigned)(b >> 32));
  return join((unsigned)lo, (unsigned)hi);
}

template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
  return join((unsigned)lo, (unsigned)hi);
}

constexpr int kDppXor1 = 0xB1;         // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;         // quad_perm [2,3,0,1]
constexpr int kDppXor8 = 0x128;        // row_ror:8
constexpr int kDppHalfMirror = 0x141;  // lane i of each 8-lane half <- lane 7 - i

// Transposed butterfly steps. From per-lane x and y: x summed over the lane pair (l, l ^ 32) in
// lanes 0..31 and y summed over it in lanes 32..63 (fold32); the same over (l, l ^ 16) with x in
// rows 0 and 2, y in rows 1 and 3 (fold16).
__device__ __forceinline__ double fold32(double x, double y) {
  const unsigned long long bx = (unsigned long long)__double_as_longlong(x);
  const unsigned long long by = (unsigned long long)__double_as_longlong(y);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)bx, (unsigned)by, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(bx >> 32), (unsigned)(by >> 32), false, false);
  return join(lo[0], hi[0]) + join(lo[1], hi[1]);
}

__device__ __forceinline__ double fold16(double x, double y) {
  const unsigned long long bx = (unsigned long long)__double_as_longlong(x);
  const unsigned long long by = (unsigned long long)__double_as_longlong(y);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)bx, (unsigned)by, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(bx >> 32), (unsigned)(by >> 32), false, false);
  return join(lo[0], hi[0]) + join(lo[1], hi[1]);
}

// The same within a row, for the lane bit that CTRL exchanges: x where the bit is clear, y where set.
template <int CTRL>
__device__ __forceinline__ double fold_row(double x, double y, bool bit) {
  const double send = bit ? x : y;
  const double keep = bit ? y : x;
  return keep + dpp<CTRL>(send);
}

// Rest of the wave reduction of the folded traces: transposed over lane bits 4 and 3, plain over
// bits 2..0. Afterwards the lanes with (lane & 7) == 0 call store(j, part, total) for their share
// of the (trace, real/imaginary part) pairs.
template <int K, typename Store>
__device__ __forceinline__ void reduce_folded(const double (&w)[K], int lane, Store store) {
  constexpr int KP = (K + 3) / 4 * 4, H2 = KP / 2, H3 = KP / 4;
  double v[KP];
#pragma unroll
  for (int q = 0; q < KP; ++q) v[q] = q < K ? w[q] : 0.0;
  double u[H2];
#pragma unroll
  for (int q = 0; q < H2; ++q) u[q] = fold16(v[q], v[q + H2]);
  const bool b3 = lane & 8;
  double z[H3];
#pragma unroll
  for (int q = 0; q < H3; ++q) {
    z[q] = fold_row<kDppXor8>(u[q], u[q + H3], b3);
    z[q] += dpp<kDppHalfMirror>(z[q]);
    z[q] += dpp<kDppXor1>(z[q]);
    z[q] += dpp<kDppXor2>(z[q]);
  }
  if ((lane & 7) == 0) {
    const int base = ((lane & 16) ? H2 : 0) + (b3 ? H3 : 0);
    const int part = lane >> 5;
#pragma unroll
    for (int q = 0; q < H3; ++q)
      if (base + q < K) store(base + q + 1, part, z[q]);
  }
}

// Trace operations of a chain program in program order (for engines that reduce traces in batches):
// the ordinal of operation oi among them, and the trace index j of the ord-th one.
__host__ __device__ constexpr int chain_trace_ord(const ChainProgram& p, int oi) {
  int c = 0;
  for (int i = 0; i < oi; ++i) c += p.ops[i].type != OP_MUL;
  return c;
}
// trace index j of the ord-th trace operation (0 past the last)
__host__ __device__ constexpr int chain_trace_at(const ChainProgram& p, int ord) {
  int c = 0;
  for (int i = 0; i < p.nops; ++i)
    if (p.ops[i].type != OP_MUL) {
      if (c == ord) return p.ops[i].x;
      ++c;
    }
  return 0;
}

// Inner products tr(P Q) are sums of P[l] Q[l ^ 17]-style lane pairs, symmetric in the two factors,
// so a run of consecutive OP_TPAIR operations that all name one slot s exchanges that slot's lanes
// once for the whole run. pair_run gives the run starting at operation oi (len 0 if it is not an
// inner product; at most 4; the slot that makes it longest), pair_other the other factor of one.
struct PairRun {
  int len, s;
};
__host__ __device__ constexpr PairRun pair_run(const ChainProgram& p, int oi) {
  if (oi >= p.nops || p.ops[oi].type != OP_TPAIR) return {0, 0};
  PairRun best{1, p.ops[oi].b};
  for (int c = 0; c < 2; ++c) {
    const int s = c == 0 ? p.ops[oi].b : p.ops[oi].a;
    int len = 1;
    while (len < 4 && oi + len < p.nops && p.ops[oi + len].type == OP_TPAIR &&
           (p.ops[oi + len].a == s || p.ops[oi + len].b == s))
      ++len;
    if (len > best.len) best = {len, s};
  }
  return best;
}
__host__ __device__ constexpr int pair_other(const ChainProgram& p, int oi, int s) {
  return oi >= p.nops ? 0 : (p.ops[oi].a == s ? p.ops[oi].b : p.ops[oi].a);
}

typedef const __attribute__((address_space(3))) double lds_d;  // LDS-qualified, for direct ds_read
typedef __attribute__((address_space(3))) double lds_dw;       // the same, writable

// Element e of an LDS array of double2 / double through LDS-qualified pointers: in a function that is
// not inlined into the kernel the compiler cannot see that a pointer is into LDS and would use flat
// accesses with 64-bit address arithmetic; these give ds_read / ds_write with 32-bit addresses. The
// pointer must point into LDS.
typedef double d2v __attribute__((ext_vector_type(2)));  // 16-byte aligned: ds_read_b128 / ds_write_b128
__device__ __forceinline__ double2 lds_ld2(const double2* p, int e) {
  const d2v v = ((const __attribute__((address_space(3))) d2v*)p)[e];
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ void lds_st2(double2* p, int e, double2 v) {
  ((__attribute__((address_space(3))) d2v*)p)[e] = d2v{v.x, v.y};
}
__device__ __forceinline__ void lds_st(double* p, int e, double v) { ((lds_dw*)p)[e] = v; }

struct PatternView {
  const double2* lds;     // staged matrix in LDS, row-major with leading dimension ld, or nullptr
  const double2* A;       // global matrix (haf path) or B (prob path)
  const int32_t* modes;   // LDS mode list (prob path) or nullptr
  int64_t src;
  int n, m;
  int ld;                 // n + 1 where row n and column n of the staged copy are zero, else n
  __device__ __forceinline__ double2 at(int i, int j) const {
    if (lds) return lds[i * ld + j];
    if (modes) return A[(int64_t)modes[i] * m + modes[j]];
    return A[src + (int64_t)i * n + j];
  }
  // at() with the address spaces spelled out (LDS copy and mode list, global matrix), for functions
  // that are not inlined into the kernel and would otherwise use flat accesses
  __device__ __forceinline__ double2 at_as(int i, int j) const;
};

typedef const __attribute__((address_space(1))) double gbl_d;
__device__ __forceinline__ double2 PatternView::at_as(int i, int j) const {
  if (lds) return lds_ld2(lds, i * ld + j);
  typedef const __attribute__((address_space(3))) int32_t lds_mode;
  const int64_t off = modes ? (int64_t)((lds_mode*)modes)[i] * m + ((lds_mode*)modes)[j] : src + (int64_t)i * n + j;
  gbl_d* g = (gbl_d*)A;
  return make_double2(g[2 * off], g[2 * off + 1]);
}

// Gather from the zero-padded staged copy that the item loop below writes (ld = n + 1, row n and
// column n zero): offset of row a and index of column c of M_Z = X A_Z (d x d) for the pair list
// pl; rows and columns at or beyond d map to the zero row / column, so every read is unconditional.
// The pair list is read through an LDS-qualified pointer: 32-bit addresses, direct ds_read.
typedef const __attribute__((address_space(3))) int32_t lds_i32;
__device__ __forceinline__ int mz_row(const PatternView& P, const int32_t* pl, int a, int d) {
  const int b = a ^ 1;  // row a of M is row a^1 of A_Z
  return (a < d ? 2 * ((lds_i32*)pl)[b >> 1] + (b & 1) : P.n) * P.ld;
}
__device__ __forceinline__ int mz_col(const PatternView& P, const int32_t* pl, int c, int d) {
  return c < d ? 2 * ((lds_i32*)pl)[c >> 1] + (c & 1) : P.n;
}
__device__ __forceinline__ double2 mz_at(const PatternView& P, int off) {
  lds_d* Al = (lds_d*)P.lds;
  return make_double2(Al[2 * off], Al[2 * off + 1]);
}

__device__ __forceinline__ uint32_t unrank(int k, int64_t g, int* s_out) {
  int s = 1;
  uint64_t rem = (uint64_t)g;
  while (s < k && rem >= kBinom.v[k][s]) {
    rem -= kBinom.v[k][s];
    ++s;
  }
  uint32_t mask = 0;
  int c = k - 1;
  for (int i = s; i >= 1; --i) {
    while (kBinom.v[c][i] > rem) --c;
    mask |= 1u << c;
    rem -= kBinom.v[c][i];
    --c;
  }
  *s_out = s;
  return mask;
}

// Next subset in canonical order: the next larger bitmask with the same popcount (Gosper's
// construction), or the smallest mask of the next size once the current size is exhausted.
__device__ __forceinline__ uint32_t next_subset(uint32_t mask, int k, int* s) {
  const uint32_t low = mask & (0u - mask);
  const uint32_t ripple = mask + low;
  const uint32_t nxt = (((ripple ^ mask) >> 2) >> __builtin_ctz(mask)) | ripple;
  if (ripple != 0u && nxt < (1u << k)) return nxt;
  *s += 1;
  return (1u << *s) - 1u;
}

// Halved traces t_j = tr(M^j) / 2 for j > d from t_1..t_d, for a d x d matrix M (d = 2|Z| < K),
// in place in the lane's column of the trace buffer (t_j at tw[j * 2 kWaveG], imaginary part next).
// The characteristic polynomial of M has degree d, so with a_i = (-1)^(i-1) e_i (e_i the elementary
// symmetric functions of the eigenvalues, zero for i > d), Newton's identities give
//   i a_i = 2 (t_i - sum_{j<i} a_{i-j} t_j)   (i <= d)   and   t_q = sum_{i<=d} a_i t_{q-i}   (q > d).
// Exact in exact arithmetic; an engine may therefore form only the first min(K, d) traces.
template <int K>
__device__ __forceinline__ void extend_traces(double* tw, int d) {
  constexpr int S = 2 * kWaveG;
  double2 a[K];
#pragma unroll
  for (int i = 1; i < K; ++i) {
    double vr = 0.0, vi = 0.0;
    if (i <= d) {
      vr = tw[i * S];
      vi = tw[i * S + 1];
#pragma unroll
      for (int j = 1; j < i; ++j) {
        const double tr = tw[j * S], ti = tw[j * S + 1];
        vr = fma(-a[i - j].x, tr, vr);
        vr = fma(a[i - j].y, ti, vr);
        vi = fma(-a[i - j].x, ti, vi);
        vi = fma(-a[i - j].y, tr, vi);
      }
      const double f = 2.0 / i;  // a constant once the loop is unrolled
      vr *= f;
      vi *= f;
    }
    a[i] = make_double2(vr, vi);
  }
#pragma unroll
  for (int q = 2; q <= K; ++q) {
    if (q > d) {
      double vr = 0.0, vi = 0.0;
#pragma unroll
      for (int i = 1; i < q; ++i) {
        const double tr = tw[(q - i) * S], ti = tw[(q - i) * S + 1];
        vr = fma(a[i].x, tr, vr);
        vr = fma(-a[i].y, ti, vr);
        vi = fma(a[i].x, ti, vi);
        vi = fma(a[i].y, tr, vi);
      }
      tw[q * S] = vr;
      tw[q * S + 1] = vi;
    }
  }
}

// a + b = s + e exactly (Knuth's TwoSum); the same (s, e) whichever operand comes first.
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bp = s - a;
  e = (a - (s - bp)) + (b - bp);
}

// One level of the compensated lane tree: (s, c) += the partner lane's (ps, pc). Both lanes of a pair
// end with the same values.
__device__ __forceinline__ void tree_add(double& s, double& c, double ps, double pc) {
  double t, e;
  two_sum(s, ps, t, e);
  c = (c + pc) + e;
  s = t;
}

// Partner exchange across the two rows of 16 lanes in each half-wave (lane l ^ 16), by
// v_permlane16_swap of the value with itself.
__device__ __forceinline__ double xrow16(double v, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)b, (unsigned)b, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
  const bool odd_row = (lane >> 4) & 1;
  return odd_row ? join(lo[0], hi[0]) : join(lo[1], hi[1]);
}

// Compensated sum over lanes 0..31 of the per-lane pairs (s, c): a fixed tree of TwoSum steps
// (partners lane ^ 1, lane ^ 2, the mirror lane within 8, the other half of the row of 16, the other
// row); lanes 0..31 end with the total. The order depends only on the lane numbers.
__device__ __forceinline__ void lane_tree_sum32(double& s, double& c, int lane) {
  tree_add(s, c, dpp<kDppXor1>(s), dpp<kDppXor1>(c));
  tree_add(s, c, dpp<kDppXor2>(s), dpp<kDppXor2>(c));
  tree_add(s, c, dpp<kDppHalfMirror>(s), dpp<kDppHalfMirror>(c));
  tree_add(s, c, dpp<kDppXor8>(s), dpp<kDppXor8>(c));
  tree_add(s, c, xrow16(s, lane), xrow16(c, lane));
}

// Coefficient recursion for the buffered subsets (one lane each) and the compensated sum of their
// signed terms, added to the running sum (sr + cr, si + ci) held by every lane. With EXT, traces
// beyond 2|Z| (which the engine leaves unformed) are first extended from the first 2|Z|.
template <int K, bool EXT = false>
__device__ __forceinline__ void combine_batch(double* trw, const int32_t* sz, int cnt, int lane, double& sr,
                                              double& si, double& cr, double& ci) {
  double2 ck = make_double2(0.0, 0.0);
  if (lane < cnt) {
    if constexpr (EXT) {
      const int d = 2 * sz[lane];
      if (d < K) extend_traces<K>(trw + 2 * lane, d);
    }
    double2 c[K + 1];
    c[0] = make_double2(1.0, 0.0);
#pragma unroll
    for (int q = 1; q <= K; ++q) {
      double ar = 0.0, ai = 0.0;
#pragma unroll
      for (int j = 1; j <= q; ++j) {
        const double tr = trw[j * (2 * kWaveG) + 2 * lane];
        const double ti = trw[j * (2 * kWaveG) + 2 * lane + 1];
        ar = fma(tr, c[q - j].x, ar);
        ar = fma(-ti, c[q - j].y, ar);
        ai = fma(tr, c[q - j].y, ai);
        ai = fma(ti, c[q - j].x, ai);
      }
      const double iq = kInv.v[q];
      c[q] = make_double2(ar * iq, ai * iq);
    }
    ck = c[K];
    if ((K - sz[lane]) & 1) {
      ck.x = -ck.x;
      ck.y = -ck.y;
    }
  }
  // the batch's terms (zero beyond cnt) summed over lanes 0..31 with compensation, then added to the
  // running sums (lanes 0..31 hold the same values; the engines read lane 0's)
  static_assert(kWaveG == 32, "the lane tree covers 32 lanes");
  double br = ck.x, bcr = 0.0, bi = ck.y, bci = 0.0;
  lane_tree_sum32(br, bcr, lane);
  lane_tree_sum32(bi, bci, lane);
  neumaier(sr, cr, br);
  neumaier(si, ci, bi);
  cr += bcr;
  ci += bci;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace

struct WaveLds {
  size_t A, modes, pl, trw, sz, terms, part, item, total;
};

__host__ __device__ inline size_t wal16(size_t x) { return (x + 15) & ~size_t(15); }

__host__ __device__ inline WaveLds wave_lds_layout(int nmax, int kmax, int stage_A) {
  WaveLds L;
  size_t off = 0;
  L.A = off;
  off += stage_A ? wal16(sizeof(double) * 2 * (nmax + 1) * (nmax + 1)) : 0;
  L.modes = off;
  off += wal16(sizeof(int32_t) * GBS_N_MAX);
  L.pl = off;
  off += wal16(sizeof(int32_t) * 16 * kMaxK);  // four pair lists per wave (quad engine)
  L.trw = off;
  off += wal16(sizeof(double) * 4 * (kmax + 1) * 2 * kWaveG);
  L.sz = off;
  off += wal16(sizeof(int32_t) * 4 * kWaveG);
  L.terms = off;
  off += wal16(sizeof(double) * 2 * 4 * kWaveG);
  L.part = off;
  off += wal16(sizeof(double) * 4 * 4);
  L.item = off;
  off += 16;
  L.total = off;
  return L;
}

// Persistent item loop of the engines that give each wave its own subsets: stage the pattern
// matrix (n <= 32) and mode list in LDS, give each of the four waves a contiguous quarter of the
// item, and combine the four wave partials in wave order, so an item's partial depends only on its
// range. range(P, lo, hi, wave, lane, sr, si, cr, ci) evaluates the wave's quarter.
template <int K, typename Range>
__device__ __forceinline__ void wave_items(const EngineArgs& args, unsigned char* smem, Range range) {
  const WaveLds L = wave_lds_layout(args.nmax, args.kmax, args.stage_A);
  double2* Alds = reinterpret_cast<double2*>(smem + L.A);
  int32_t* mlds = reinterpret_cast<int32_t*>(smem + L.modes);
  double* part = reinterpret_cast<double*>(smem + L.part);
  int32_t* item_sh = reinterpret_cast<int32_t*>(smem + L.item);
  // the wave index is uniform across the wave: readfirstlane lets the compiler keep everything
  // derived from it (the wave's subset range, masks, sizes) in scalar registers
  const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;

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
    const int ld = n + 1;  // staged copy: (n + 1) x (n + 1), row n and column n zero
    if (staged) {
      for (int e = tid; e < ld * ld; e += kThreads) {
        const int i = e / ld, j = e - (e / ld) * ld;
        double2 v = make_double2(0.0, 0.0);
        if (i < n && j < n) v = prob ? args.A[(int64_t)mlds[i] * args.m + mlds[j]] : args.A[pd.src + (int64_t)i * n + j];
        Alds[e] = v;
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
    P.ld = ld;

    // this wave's quarter of the item
    const int64_t len = item.hi - item.lo;
    const int64_t q = (len + 3) / 4;
    const int64_t lo = item.lo + q * wave < item.hi ? item.lo + q * wave : item.hi;
    const int64_t hi = lo + q < item.hi ? lo + q : item.hi;
    double sr = 0.0, si = 0.0, cr = 0.0, ci = 0.0;
    if (lo < hi && k == K) range(P, lo, hi, wave, lane, sr, si, cr, ci);
    if (lane == 0) {
      part[wave * 4 + 0] = sr;
      part[wave * 4 + 1] = si;
      part[wave * 4 + 2] = cr;
      part[wave * 4 + 3] = ci;
    }
    __syncthreads();
    if (tid == 0) {
      double r0 = part[0], i0 = part[1], c0 = part[2], d0 = part[3];
      for (int w = 1; w < 4; ++w) {
        neumaier(r0, c0, part[w * 4 + 0]);
        neumaier(i0, d0, part[w * 4 + 1]);
        c0 += part[w * 4 + 2];
        d0 += part[w * 4 + 3];
      }
      gbs_partial p;
      p.s_re = r0;
      p.s_im = i0;
      p.c_re = c0;
      p.c_im = d0;
      args.partials[item.partial] = p;
    }
    if (!args.persistent) break;
  }
}

}  // namespace gbs
