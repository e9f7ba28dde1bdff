// Double-double subset engine (the accuracy mode), gfx950.
//
// Same method as the FP64 engines -- for every pair subset Z the traces t_j = tr(M_Z^j), j <= k,
// then c_0 = 1, q c_q = sum_j (t_j / 2) c_{q-j} and the signed term (-1)^(k-|Z|) c_k summed over Z
// (the hafnian algorithm cited in Sec. II C) -- but every value is carried as a double-double, an
// unevaluated sum hi + lo of two doubles (~106 significant bits). A term's rounding error is then ~u^2
// instead of ~u relative to its size, so the cancellation of the subset sum (sum |term| / |Haf| ~
// 1e7..1e12 at n = 36..46) no longer limits the result; the pattern matrix itself, given in FP64, is
// exact input.
// The arithmetic is error-free transformations on the VALU: the FP64 MFMA rounds every product and
// has no error-free form.
//
// Powers. Instead of the per-k chain programs of the FP64 engines (up to six stored powers) the
// engine climbs one power at a time and reads two traces per product: holding Q = M^i, it forms
// Y = Q M, then t_{2i+1} = tr(Q Y) and, with Q = Y, t_{2i+2} = tr(Q Q). From t_1 = tr(M) and
// t_2 = tr(M M) that is ceil(k/2) - 1 products for all k traces, with one power in registers.
// Every power of M = X A_Z satisfies Q^t = X Q X (X swaps the two indices of each pair; A_Z is
// symmetric), so tr(P Q) = sum_{i,c} P[i][c] Q[i^1][c^1]: each entry of P meets one entry of Q.
//
// Layout. A workgroup of 256 threads evaluates one subset at a time, with M_Z (d = 2|Z|) padded to
// D = 16 T, T <= 3 a template parameter. Thread (rb, cb) = (tid / 16, tid % 16) owns the T x T
// entries (rb + 16 r, cb + 16 c) of the current power, so the partner entry (i^1, c^1) sits in
// thread tid ^ 17 of the same wave, at the same (r, c). The product Q M reads M's entries straight
// from the pattern matrix staged in LDS (they are exact doubles: row l of M is row l^1 of A_Z) and
// Q's columns through LDS, 16 at a time. Sums of products accumulate as s + c, the running sum by
// TwoSum and every rounding error (fma for products) into c -- the compensated dot product of Ogita,
// Rump and Oishi (SIAM J. Sci. Comput. 26, 2005), as accurate as double-double arithmetic. Each trace
// is reduced over the wave with a shuffle tree and over the four waves in LDS, in fixed order. The
// traces of 16 subsets are buffered; 16 threads then run the coefficient recursion in double-double,
// and a shuffle tree adds their terms to the item's running sum.
//
// Every helper below is an error-free transformation or built on one: this header must be compiled
// with -ffp-contract=off (a contracted a * b + c changes the rounding the transformations recover).
#pragma once
#include "gbs_engine_common.h"

namespace gbs {
namespace {

struct dd {
  double hi, lo;
};
struct zdd {
  dd re, im;
};

// |a| >= |b| or a == 0: a + b = s + e exactly
__device__ __forceinline__ dd quick_two_sum(double a, double b) {
  const double s = a + b;
  return dd{s, b - (s - a)};
}

__device__ __forceinline__ dd dd_norm(double s, double c) {
  double h, l;
  two_sum(s, c, h, l);
  return dd{h, l};
}

// a + b, accurate (both parts added with TwoSum)
__device__ __forceinline__ dd dd_add(dd a, dd b) {
  double s, e;
  two_sum(a.hi, b.hi, s, e);
  double t, f;
  two_sum(a.lo, b.lo, t, f);
  e += t;
  dd r = quick_two_sum(s, e);
  r.lo += f;
  return quick_two_sum(r.hi, r.lo);
}

__device__ __forceinline__ dd dd_neg(dd a) { return dd{-a.hi, -a.lo}; }

// a * b with the product's rounding error recovered by fma
__device__ __forceinline__ dd dd_mul(dd a, dd b) {
  const double p = a.hi * b.hi;
  double e = fma(a.hi, b.hi, -p);
  e = fma(a.hi, b.lo, e);
  e = fma(a.lo, b.hi, e);
  return quick_two_sum(p, e);
}

// a / q for a small positive integer q
__device__ __forceinline__ dd dd_div_int(dd a, double q) {
  const double q1 = a.hi / q;
  const double p = q1 * q;
  const double pe = fma(q1, q, -p);            // q1 q = p + pe exactly
  const double r = ((a.hi - p) - pe) + a.lo;   // a - q1 q (a.hi - p is exact: p is within u of a.hi)
  return quick_two_sum(q1, r / q);
}

__device__ __forceinline__ zdd zdd_zero() { return zdd{dd{0.0, 0.0}, dd{0.0, 0.0}}; }
__device__ __forceinline__ zdd zdd_add(zdd a, zdd b) { return zdd{dd_add(a.re, b.re), dd_add(a.im, b.im)}; }

// acc + x y (complex), every step accurate
__device__ __forceinline__ zdd zdd_mac(zdd acc, zdd x, zdd y) {
  acc.re = dd_add(acc.re, dd_mul(x.re, y.re));
  acc.re = dd_add(acc.re, dd_neg(dd_mul(x.im, y.im)));
  acc.im = dd_add(acc.im, dd_mul(x.re, y.im));
  acc.im = dd_add(acc.im, dd_mul(x.im, y.re));
  return acc;
}

// Compensated dot-product accumulator: value s + c.
struct acc2 {
  double s, c;
};

// a += (xh + xl) m for a double m
__device__ __forceinline__ void acc_dm(acc2& a, double xh, double xl, double m) {
  const double p = xh * m;
  const double e = fma(xh, m, -p);
  double s, t;
  two_sum(a.s, p, s, t);
  a.s = s;
  a.c += t + fma(xl, m, e);
}

// a += (xh + xl)(yh + yl)
__device__ __forceinline__ void acc_dd(acc2& a, double xh, double xl, double yh, double yl) {
  const double p = xh * yh;
  const double e = fma(xh, yh, -p);
  double s, t;
  two_sum(a.s, p, s, t);
  a.s = s;
  a.c += t + fma(xh, yl, fma(xl, yh, e));
}

constexpr int kDdThreads = 256;
constexpr int kDdBuf = 16;  // subsets whose traces are buffered before the recursion

__device__ __forceinline__ double shfl_d(double v, int lane_mask) { return __shfl_xor(v, lane_mask, 64); }

__device__ __forceinline__ zdd shfl_zdd(zdd v, int lane_mask) {
  zdd o;
  o.re.hi = shfl_d(v.re.hi, lane_mask);
  o.re.lo = shfl_d(v.re.lo, lane_mask);
  o.im.hi = shfl_d(v.im.hi, lane_mask);
  o.im.lo = shfl_d(v.im.lo, lane_mask);
  return o;
}

// Sum of one zdd per lane over the wave (every lane ends with the total: dd_add is commutative).
__device__ __forceinline__ zdd wave_sum(zdd v) {
#pragma unroll
  for (int w = 1; w < 64; w <<= 1) v = zdd_add(v, shfl_zdd(v, w));
  return v;
}

template <int T>
struct DdPow {
  zdd e[T][T];  // entry (rb + 16 r, cb + 16 c)
};

// This thread's part of tr(P Q) = sum P[i][c] Q[i^1][c^1]; Q's entries come from thread tid ^ 17.
template <int T>
__device__ __forceinline__ zdd dd_trace_pair_part(const DdPow<T>& P, const DdPow<T>& Q) {
  acc2 re{0.0, 0.0}, im{0.0, 0.0};
#pragma unroll
  for (int r = 0; r < T; ++r)
#pragma unroll
    for (int c = 0; c < T; ++c) {
      const zdd p = P.e[r][c];
      const zdd q = shfl_zdd(Q.e[r][c], 17);
      acc_dd(re, p.re.hi, p.re.lo, q.re.hi, q.re.lo);
      acc_dd(re, -p.im.hi, -p.im.lo, q.im.hi, q.im.lo);
      acc_dd(im, p.re.hi, p.re.lo, q.im.hi, q.im.lo);
      acc_dd(im, p.im.hi, p.im.lo, q.re.hi, q.re.lo);
    }
  return zdd{dd_norm(re.s, re.c), dd_norm(im.s, im.c)};
}

// Reduce this thread's part of trace t_j over its wave; the wave's total goes to wpart[(j-1) 4 + w].
__device__ __forceinline__ void dd_trace_out(zdd part, zdd* wpart, int j, int tid) {
  const zdd w = wave_sum(part);
  if ((tid & 63) == 0) wpart[(j - 1) * 4 + (tid >> 6)] = w;
}

// Q <- Q M. M[l][c] = A_Z[l^1][c] is read from the staged pattern matrix: rowoff[l] is the offset of
// A_Z's row l^1, cid[c] that of this thread's column cb + 16 c (negative beyond d). Xs stages 16
// columns of Q at a time (16 T rows x 16).
template <int T>
__device__ __forceinline__ void dd_mul_M(DdPow<T>& Q, const double2* Alds, const int32_t* rowoff, const int (&cid)[T],
                                         zdd* Xs, int d, int rb, int cb) {
  acc2 ar[T][T], ai[T][T];
#pragma unroll
  for (int r = 0; r < T; ++r)
#pragma unroll
    for (int c = 0; c < T; ++c) {
      ar[r][c] = acc2{0.0, 0.0};
      ai[r][c] = acc2{0.0, 0.0};
    }
#pragma unroll
  for (int c0 = 0; c0 < T; ++c0) {
    if (16 * c0 < d) {
      __syncthreads();
#pragma unroll
      for (int r = 0; r < T; ++r) Xs[(rb + 16 * r) * 16 + cb] = Q.e[r][c0];
      __syncthreads();
      const int lend = d - 16 * c0 < 16 ? d - 16 * c0 : 16;
      for (int l = 0; l < lend; ++l) {
        const int ro = rowoff[16 * c0 + l];
        double2 m[T];
#pragma unroll
        for (int c = 0; c < T; ++c) m[c] = cid[c] >= 0 ? Alds[ro + cid[c]] : make_double2(0.0, 0.0);
#pragma unroll
        for (int r = 0; r < T; ++r) {
          const zdd x = Xs[(rb + 16 * r) * 16 + l];
#pragma unroll
          for (int c = 0; c < T; ++c) {
            acc_dm(ar[r][c], x.re.hi, x.re.lo, m[c].x);
            acc_dm(ar[r][c], -x.im.hi, -x.im.lo, m[c].y);
            acc_dm(ai[r][c], x.re.hi, x.re.lo, m[c].y);
            acc_dm(ai[r][c], x.im.hi, x.im.lo, m[c].x);
          }
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < T; ++r)
#pragma unroll
    for (int c = 0; c < T; ++c) Q.e[r][c] = zdd{dd_norm(ar[r][c].s, ar[r][c].c), dd_norm(ai[r][c].s, ai[r][c].c)};
}

}  // namespace

struct DdLds {
  size_t A, modes, rowoff, cidx, sz, wpart, work, tbuf, item, total;
};

// LDS of the double-double engine for tile count T (padded size 16 T), patterns up to nmax.
__host__ __device__ inline DdLds dd_lds_layout(int T, int nmax, int kmax) {
  DdLds L;
  size_t off = 0;
  L.A = off;
  off += wal16(sizeof(double) * 2 * (size_t)nmax * nmax);
  L.modes = off;
  off += wal16(sizeof(int32_t) * GBS_N_MAX);
  L.rowoff = off;  // per row l < d of M: offset of A_Z's row l^1 in the staged matrix
  off += wal16(sizeof(int32_t) * GBS_N_MAX);
  L.cidx = off;    // per column c < d: offset of A_Z's column c
  off += wal16(sizeof(int32_t) * GBS_N_MAX);
  L.sz = off;
  off += wal16(sizeof(int32_t) * kDdBuf);
  L.wpart = off;
  off += wal16(sizeof(double) * 4 * 4 * (size_t)(kmax > 0 ? kmax : 1));
  // columns of the current power during a product (16 T x 16), coefficients during the recursion
  L.work = off;
  const size_t cols = (size_t)16 * T * 16, coef = (size_t)(kmax + 1) * kDdBuf;
  off += wal16(sizeof(double) * 4 * (cols > coef ? cols : coef));
  L.tbuf = off;
  off += wal16(sizeof(double) * 4 * (size_t)(kmax > 0 ? kmax : 1) * kDdBuf);
  L.item = off;
  off += 16;
  L.total = off;
  return L;
}

// Engine kernel for subsets with 2|Z| <= 16 T; any k, and a launch may mix patterns of different n
// (LDS sized for the largest, args.nmax and args.kmax).
template <int T>
__global__ __launch_bounds__(kDdThreads, 2) void dd_engine_kernel(EngineArgs args) {
  extern __shared__ __align__(16) unsigned char smem[];
  const DdLds Ly = dd_lds_layout(T, args.nmax, args.kmax);
  double2* Alds = reinterpret_cast<double2*>(smem + Ly.A);
  int32_t* mlds = reinterpret_cast<int32_t*>(smem + Ly.modes);
  int32_t* rowoff = reinterpret_cast<int32_t*>(smem + Ly.rowoff);
  int32_t* cidx = reinterpret_cast<int32_t*>(smem + Ly.cidx);
  int32_t* szb = reinterpret_cast<int32_t*>(smem + Ly.sz);
  zdd* wpart = reinterpret_cast<zdd*>(smem + Ly.wpart);
  zdd* work = reinterpret_cast<zdd*>(smem + Ly.work);
  zdd* tbuf = reinterpret_cast<zdd*>(smem + Ly.tbuf);
  int32_t* item_sh = reinterpret_cast<int32_t*>(smem + Ly.item);
  const int tid = threadIdx.x;
  const int rb = tid >> 4, cb = tid & 15;

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
    __syncthreads();
    if (prob && tid < n) mlds[tid] = args.modes[pd.src + tid];
    __syncthreads();
    for (int e = tid; e < n * n; e += kDdThreads) {
      const int i = e / n, j = e - (e / n) * n;
      Alds[e] = prob ? args.A[(int64_t)mlds[i] * args.m + mlds[j]] : args.A[pd.src + e];
    }
    dd sre{0.0, 0.0}, sim{0.0, 0.0};
    if (item.lo < item.hi) {
      int s = 1;
      uint32_t mask = unrank(k, item.lo, &s);
      for (int64_t g0 = item.lo; g0 < item.hi; g0 += kDdBuf) {
        const int cnt = (int)((item.hi - g0) < kDdBuf ? (item.hi - g0) : kDdBuf);
        for (int u = 0; u < cnt; ++u) {
          if (u > 0 || g0 > item.lo) mask = next_subset(mask, k, &s);
          const int d = 2 * s;
          __syncthreads();
          // pair p of the pattern is pair q of Z (q = rank of bit p in the mask): rows/columns 2q, 2q + 1
          if (tid < k && ((mask >> tid) & 1u)) {
            const int q = __popc(mask & ((1u << tid) - 1u));
            rowoff[2 * q] = (2 * tid + 1) * n;  // row 2q of M is row 2q + 1 of A_Z
            rowoff[2 * q + 1] = (2 * tid) * n;
            cidx[2 * q] = 2 * tid;
            cidx[2 * q + 1] = 2 * tid + 1;
          }
          if (tid == 0) szb[u] = s;
          __syncthreads();
          int cid[T];
#pragma unroll
          for (int c = 0; c < T; ++c) cid[c] = cb + 16 * c < d ? cidx[cb + 16 * c] : -1;
          DdPow<T> Q;
          zdd t1 = zdd_zero();
#pragma unroll
          for (int r = 0; r < T; ++r)
#pragma unroll
            for (int c = 0; c < T; ++c) {
              const int i = rb + 16 * r;
              double2 v = make_double2(0.0, 0.0);
              if (i < d && cid[c] >= 0) v = Alds[rowoff[i] + cid[c]];
              Q.e[r][c] = zdd{dd{v.x, 0.0}, dd{v.y, 0.0}};
              if (r == c && rb == cb) t1 = zdd_add(t1, Q.e[r][c]);
            }
          dd_trace_out(t1, wpart, 1, tid);
          if (k >= 2) dd_trace_out(dd_trace_pair_part<T>(Q, Q), wpart, 2, tid);
          for (int i = 1; 2 * i < k; ++i) {
            DdPow<T> Y = Q;
            dd_mul_M<T>(Y, Alds, rowoff, cid, work, d, rb, cb);
            dd_trace_out(dd_trace_pair_part<T>(Q, Y), wpart, 2 * i + 1, tid);
            Q = Y;
            if (2 * i + 2 <= k) dd_trace_out(dd_trace_pair_part<T>(Q, Q), wpart, 2 * i + 2, tid);
          }
          __syncthreads();
          if (tid < k) {
            const zdd* w = wpart + tid * 4;
            tbuf[tid * kDdBuf + u] = zdd_add(zdd_add(w[0], w[1]), zdd_add(w[2], w[3]));
          }
        }
        __syncthreads();
        // coefficient recursion, one thread per buffered subset; c_q at work[q * kDdBuf + u]
        zdd term = zdd_zero();
        if (tid < cnt) {
          const int u = tid;
          work[u] = zdd{dd{1.0, 0.0}, dd{0.0, 0.0}};
          zdd cq = work[u];
          for (int q = 1; q <= k; ++q) {
            zdd a = zdd_zero();
            for (int j = 1; j <= q; ++j) {
              zdd t = tbuf[(j - 1) * kDdBuf + u];
              t.re = dd{0.5 * t.re.hi, 0.5 * t.re.lo};
              t.im = dd{0.5 * t.im.hi, 0.5 * t.im.lo};
              a = zdd_mac(a, t, work[(q - j) * kDdBuf + u]);
            }
            cq = zdd{dd_div_int(a.re, (double)q), dd_div_int(a.im, (double)q)};
            work[q * kDdBuf + u] = cq;
          }
          term = ((k - szb[u]) & 1) ? zdd{dd_neg(cq.re), dd_neg(cq.im)} : cq;
        }
        if (tid < 64) {
          // threads 0..15 hold the terms (zero past cnt); a fixed tree over them
#pragma unroll
          for (int w = 1; w < kDdBuf; w <<= 1) term = zdd_add(term, shfl_zdd(term, w));
          if (tid == 0) {
            sre = dd_add(sre, term.re);
            sim = dd_add(sim, term.im);
          }
        }
        __syncthreads();
      }
    }
    if (tid == 0) {
      gbs_partial p;
      p.s_re = sre.hi;
      p.s_im = sim.hi;
      p.c_re = sre.lo;
      p.c_im = sim.lo;
      args.partials[item.partial] = p;
    }
    if (!args.persistent) break;
  }
}

}  // namespace gbs
