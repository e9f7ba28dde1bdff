// HIP kernels of libgbs for gfx950 (MI355X) other than the subset engines, and the dispatch of the
// engine variants.
//
// Hafnian by the power-trace formula the paper cites for its O(n^3 2^(n/2)) cost (Sec. II C):
// with k = n/2, pairs (2i, 2i+1) and X the within-pair row swap,
//   Haf(A) = sum_{Z subset [k], Z != {}} (-1)^(k-|Z|) c_k(M_Z),   M_Z = X A_Z,
//   c_0 = 1,  q c_q = sum_{j=1..q} (tr(M_Z^j) / 2) c_{q-j}        (c_k = [lambda^k] det(I - lambda M_Z)^(-1/2)).
//
// A call's subsets are cut into work items (ranges of one pattern's canonical subset order: by |Z|,
// then bitmask). Each item runs on the engine kernel for its subset sizes and k (gbs_eng_*.hip; the
// class table is in gbs_internal.h) and writes one compensated partial sum; finalize_kernel adds a
// pattern's partials in a fixed order (64 strided lane sums, then a lane tree), so a result depends
// only on n and the launch shape, never on the batch around it. This file also holds the state setup (B, W, prefactor), the Theorem-1 marginal
// kernels, the inverse-CDF draw of the sampler and the work-counter reset.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <utility>

#include "gbs_engine_common.h"
#include "gbs_quad_engine.h"
#include "gbs_qtile_engine.h"
#include "gbs_strip_engine.h"
#include "gbs_tile_engine.h"
#include "gbs_dd_engine.h"
#include "gbs_sqt_engine.h"

namespace gbs {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// ---------------------------------------------------------------- finalize

// One wave per pattern: lane l adds partials lo + l, lo + l + 64, ... (Neumaier), then a fixed tree of
// TwoSum steps over the 64 lanes; the order depends only on the pattern's partial range.
__global__ __launch_bounds__(256) void finalize_kernel(FinalizeArgs a) {
  const int lane = threadIdx.x & 63;
  for (int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); b < a.batch; b += (int64_t)gridDim.x * 4) {
    double sr = 0.0, si = 0.0, cr = 0.0, ci = 0.0;
    for (int64_t q = a.part_lo[b] + lane; q < a.part_hi[b]; q += 64) {
      const gbs_partial p = a.partials[q];
      neumaier(sr, cr, p.s_re);
      neumaier(si, ci, p.s_im);
      cr += p.c_re;
      ci += p.c_im;
    }
#pragma unroll
    for (int w = 1; w < 64; w <<= 1) {
      tree_add(sr, cr, __shfl_xor(sr, w, 64), __shfl_xor(cr, w, 64));
      tree_add(si, ci, __shfl_xor(si, w, 64), __shfl_xor(ci, w, 64));
    }
    if (lane != 0) continue;
    if (a.partial_out) {
      gbs_partial o;
      o.s_re = sr;
      o.s_im = si;
      o.c_re = cr;
      o.c_im = ci;
      a.partial_out[a.out_idx ? a.out_idx[b] : b] = o;
      continue;
    }
    const int n = a.n[b];
    double hr = sr + cr, hi = si + ci;
    if (n == 0) {
      hr = 1.0;
      hi = 0.0;
    } else if (n & 1) {
      hr = 0.0;
      hi = 0.0;
    }
    const int64_t o = a.out_idx ? a.out_idx[b] : b;
    if (a.haf_out) a.haf_out[o] = make_double2(hr, hi);
    if (a.prob_out) a.prob_out[o] = (*a.prefactor) * (hr * hr + hi * hi) / a.sfact[b];
  }
}

// ---------------------------------------------------------------- debug symmetry check

// flags[b] = 1 if pattern b's matrix (haf path: row-major n x n at A + src) has a pair of entries with
// |A_ij - A_ji| > tol * max |A|, else 0. NaN entries compare false and are ignored (they propagate).
__global__ __launch_bounds__(256) void sym_check_kernel(const double2* A, const PatternDesc* pats, int64_t batch,
                                                        double tol, int32_t* flags) {
  __shared__ double red[256];
  __shared__ int bad;
  const int t = threadIdx.x;
  for (int64_t b = blockIdx.x; b < batch; b += gridDim.x) {
    const PatternDesc pd = pats[b];
    const int n = pd.n;
    const double2* M = A + pd.src;
    double mx = 0.0;
    for (int e = t; e < n * n; e += 256) {
      const double2 v = M[e];
      const double a = hypot(v.x, v.y);
      if (a > mx) mx = a;
    }
    red[t] = mx;
    if (t == 0) bad = 0;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (t < w) red[t] = fmax(red[t], red[t + w]);
      __syncthreads();
    }
    const double lim = tol * red[0];
    for (int e = t; e < n * n; e += 256) {
      const int i = e / n, j = e - (e / n) * n;
      if (j > i) {
        const double2 a = M[e], c = M[(int64_t)j * n + i];
        if (hypot(a.x - c.x, a.y - c.y) > lim) atomicOr(&bad, 1);
      }
    }
    __syncthreads();
    if (t == 0) flags[b] = bad;
    __syncthreads();
  }
}

void launch_sym_check(const double2* A, const PatternDesc* pats, int64_t batch, double tol, int32_t* flags,
                      hipStream_t s) {
  const int64_t g = batch < 4096 ? batch : 4096;
  if (g > 0) hipLaunchKernelGGL(sym_check_kernel, dim3((unsigned)g), dim3(256), 0, s, A, pats, batch, tol, flags);
}

// ---------------------------------------------------------------- state

// B = U diag(tanh r) U^t (transpose), W = U U^t, prefactor = prod_i 1/cosh r_i.
__global__ void state_kernel(const double2* U, const double* r, int m, double2* B, double2* W, double* prefactor) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < (int64_t)m * m) {
    const int i = (int)(e / m), j = (int)(e - (int64_t)(e / m) * m);
    double br = 0.0, bi = 0.0, wr = 0.0, wi = 0.0;
    for (int l = 0; l < m; ++l) {
      const double t = tanh(r[l]);
      const double2 p = cmul(U[(int64_t)i * m + l], U[(int64_t)j * m + l]);
      br = fma(t, p.x, br);
      bi = fma(t, p.y, bi);
      wr += p.x;
      wi += p.y;
    }
    B[e] = make_double2(br, bi);
    W[e] = make_double2(wr, wi);
  }
  if (e == 0) {
    double pf = 1.0;
    for (int l = 0; l < m; ++l) pf /= cosh(r[l]);
    *prefactor = pf;
  }
}

// ---------------------------------------------------------------- marginals (Theorem 1)

// Prefix holding global index t of a table with per-prefix starts off[0..batch] (binary search).
__device__ __forceinline__ int64_t owner(const int64_t* off, int64_t batch, int64_t t) {
  int64_t lo = 0, hi = batch;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (off[mid] <= t) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Subset hafnians of size `level` (even) for every prefix: the expansion of the matching sum along
// the lowest position of S (Eq. HafMatch), from the tables of size level - 2.
__global__ void subset_haf_kernel(MargArgs a, int level) {
  const int64_t total = a.h_off[a.batch];
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = owner(a.h_off, a.batch, t);
    const uint32_t S = (uint32_t)(t - a.h_off[p]);
    if (__popc(S) != level) continue;
    double2* h = a.h + a.h_off[p];
    if (level == 0) {
      h[0] = make_double2(1.0, 0.0);
      continue;
    }
    const int32_t* x = a.x + a.x_off[p];
    const int i0 = __builtin_ctz(S);
    const uint32_t R = S & (S - 1u);
    const double2* Wrow = a.W + (int64_t)x[i0] * a.m;
    double sr = 0.0, si = 0.0;
    for (uint32_t r = R; r; r &= r - 1u) {
      const int j = __builtin_ctz(r);
      const double2 w = Wrow[x[j]];
      const double2 g = h[R ^ (1u << j)];
      sr = fma(w.x, g.x, sr);
      sr = fma(-w.y, g.y, sr);
      si = fma(w.x, g.y, si);
      si = fma(w.y, g.x, si);
    }
    h[S] = make_double2(sr, si);
  }
}

// Deposit the low bits of t onto the set bits of mask, lowest first (bits of t beyond popc(mask)
// are ignored).
__device__ __forceinline__ uint32_t deposit(uint32_t t, uint32_t mask) {
  uint32_t out = 0;
  for (uint32_t m = mask; m && t; m &= m - 1u, t >>= 1)
    if (t & 1u) out |= m & (0u - m);
  return out;
}

constexpr int kMargLow = 7;                  // positions of C spread over the lanes
constexpr int kMargHigh = kMaxK - kMargLow;  // at most this many walked in the uniform loop
constexpr int kMargUnroll = 4;               // walk steps whose table reads are in flight together

// One wave per class. For each member A (in order) and C = [k] minus A, the even subsets a of C are
// split as a = low | high: low ranges over the subsets of C's lowest kMargLow positions -- lane l
// owns the l-th one of even and the l-th one of odd size, so every lane works on every step -- and
// high walks subsets of C's other positions in increasing order, the same for every lane (the
// wave reads neighbouring table entries). The parity of high picks the lane's even or odd low
// subset so that |a| is even; partial sums are kept per size of high (a uniform index) and moved to
// j = |a| / 2 at the end. The product h(a) h(C minus a) is the same for a and its complement, and
// exactly one of the two holds C's highest position: when that position is a high one, only the
// subsets a containing it are walked and each product is added to j = |a| / 2 and to
// j' = |C minus a| / 2 (half the table reads). Lane sums are combined in a fixed order, so results do
// not depend on timing.
__global__ __launch_bounds__(64) void marg_class_kernel(MargArgs a) {
  __shared__ double2 acc[(kMaxK / 2 + 1) * 64];
  __shared__ double2 H[kMaxK / 2 + 1];
  const int lane = threadIdx.x;
  for (int64_t c = blockIdx.x; c < a.n_classes; c += gridDim.x) {
    const int64_t p = owner(a.pre_cls, a.batch, c);
    const int k = a.k[p];
    const uint32_t full = k >= 32 ? 0xffffffffu : ((1u << k) - 1u);
    const double2* h = a.h + a.h_off[p];
    const int64_t eb = a.ex_base[p];
    int64_t m_lo = 0, m_hi = 1;
    uint32_t A_impl = 0;
    double w = 1.0;
    if (eb < 0) {  // collision-free: class i is the single set A = 2i + parity bit
      const uint32_t i = (uint32_t)(c - a.pre_cls[p]);
      A_impl = (i << 1) | ((uint32_t)(__popc(i) + k) & 1u);
    } else {
      const int64_t e = eb + (c - a.pre_cls[p]);
      m_lo = a.cls_mem[e];
      m_hi = a.cls_mem[e + 1];
      w = a.cls_w[e];
    }
    const uint32_t A0 = eb < 0 ? A_impl : a.mem[m_lo];
    const int mu = __popc(A0);
    const int cs = k - mu;  // |C|, even by construction
    const int J = cs / 2 + 1;
    if (lane < J) H[lane] = make_double2(0.0, 0.0);
    for (int64_t q = m_lo; q < m_hi; ++q) {
      const uint32_t C = full & ~(eb < 0 ? A_impl : a.mem[q]);
      for (int j = 0; j < J; ++j) acc[j * 64 + lane] = make_double2(0.0, 0.0);
      // low part: C's lowest nl positions; lane's even- and odd-size low subsets
      const int nl = cs < kMargLow ? cs : kMargLow;
      uint32_t L = 0;
      {
        uint32_t r = C;
        for (int t = 0; t < nl; ++t, r &= r - 1u) L |= r & (0u - r);
      }
      const uint32_t Hh = C & ~L;
      // pairs (a, C minus a) once each: walk only high parts holding C's top position (if it is high)
      const uint32_t top = Hh ? (0x80000000u >> __clz(Hh)) : 0u;
      const uint32_t Hw = Hh & ~top;
      const int half = nl > 0 ? 1 << (nl - 1) : 1;  // number of even (and of odd) low subsets
      const uint32_t te = ((uint32_t)lane << 1) | ((uint32_t)__popc((uint32_t)lane) & 1u);
      const uint32_t to = ((uint32_t)lane << 1) | ((~(uint32_t)__popc((uint32_t)lane)) & 1u);
      const bool ae = lane < half, ao = nl > 0 && lane < half;
      const uint32_t le = ae ? deposit(te, L) : 0u, lo = ao ? deposit(to, L) : 0u;
      const int pe = __popc(le), po = __popc(lo);
      double sr[kMargHigh + 1], si[kMargHigh + 1];
#pragma unroll
      for (int t = 0; t <= kMargHigh; ++t) sr[t] = si[t] = 0.0;
      // the walk in steps of kMargUnroll consecutive subsets: their table reads are issued together
      // (independent gathers in flight), then accumulated in walk order
      uint32_t sw = 0;  // walked subset of Hw; the high part is sw | top
      bool more = true;
      while (more) {
        uint32_t hq[kMargUnroll], sq[kMargUnroll];
        bool vq[kMargUnroll];  // uniform: the walk has not wrapped around to 0 yet
        sq[0] = sw;
        vq[0] = true;
#pragma unroll
        for (int u = 1; u < kMargUnroll; ++u) {
          sq[u] = (sq[u - 1] - Hw) & Hw;  // next subset of Hw in increasing order
          vq[u] = vq[u - 1] && sq[u] != 0;
        }
#pragma unroll
        for (int u = 0; u < kMargUnroll; ++u) hq[u] = sq[u] | top;
        sw = (sq[kMargUnroll - 1] - Hw) & Hw;
        more = vq[kMargUnroll - 1] && sw != 0;
        double2 xs[kMargUnroll], ys[kMargUnroll];
        bool act[kMargUnroll];
#pragma unroll
        for (int u = 0; u < kMargUnroll; ++u) {
          const bool even = (__popc(hq[u]) & 1) == 0;
          act[u] = vq[u] && (even ? ae : ao);
          xs[u] = ys[u] = make_double2(0.0, 0.0);
          if (act[u]) {
            const uint32_t sub = (even ? le : lo) | hq[u];
            xs[u] = h[sub];
            ys[u] = h[C ^ sub];
          }
        }
#pragma unroll
        for (int u = 0; u < kMargUnroll; ++u) {
          if (!act[u]) continue;
          const double2 x = xs[u], y = ys[u];
          const double pr = fma(x.x, y.x, -x.y * y.y), pi = fma(x.x, y.y, x.y * y.x);
          switch (__popc(hq[u])) {  // uniform index into registers
#define GBS_MARG_ACC(T) \
            case T:                \
              sr[T] += pr;         \
              si[T] += pi;         \
              break;
            GBS_MARG_ACC(0) GBS_MARG_ACC(1) GBS_MARG_ACC(2) GBS_MARG_ACC(3) GBS_MARG_ACC(4) GBS_MARG_ACC(5)
            GBS_MARG_ACC(6) GBS_MARG_ACC(7) GBS_MARG_ACC(8) GBS_MARG_ACC(9) GBS_MARG_ACC(10) GBS_MARG_ACC(11)
            GBS_MARG_ACC(12) GBS_MARG_ACC(13) GBS_MARG_ACC(14) GBS_MARG_ACC(15) GBS_MARG_ACC(16)
#undef GBS_MARG_ACC
            default: break;
          }
        }
      }
      // |a| = |low| + |high|: move each partial to j = |a| / 2 (one lane writes only its own slots)
#pragma unroll
      for (int t = 0; t <= kMargHigh; ++t) {
        if (t <= cs - nl) {
          const int pl = (t & 1) ? po : pe;
          const int j = (pl + t) >> 1;
          if ((t & 1) ? ao : ae) {
            acc[j * 64 + lane] = make_double2(acc[j * 64 + lane].x + sr[t], acc[j * 64 + lane].y + si[t]);
            if (top) {  // the complement's share
              const int j2 = (cs - pl - t) >> 1;
              acc[j2 * 64 + lane] = make_double2(acc[j2 * 64 + lane].x + sr[t], acc[j2 * 64 + lane].y + si[t]);
            }
          }
        }
      }
      __syncthreads();
      // fixed-order sum over lanes for each j (lane j adds column j; J <= 12 lanes busy)
      if (lane < J) {
        double xr = 0.0, xi = 0.0;
        for (int l = 0; l < 64; ++l) {
          xr += acc[lane * 64 + l].x;
          xi += acc[lane * 64 + l].y;
        }
        H[lane] = make_double2(H[lane].x + xr, H[lane].y + xi);
      }
      __syncthreads();
    }
    if (lane == 0) {
      const double* F = a.F + a.F_off[p] + (int64_t)mu * a.jdim * a.jdim;
      double v = 0.0;
      for (int j1 = 0; j1 < J; ++j1)
        for (int j2 = 0; j2 < J; ++j2) {
          const double f = F[j1 * a.jdim + j2];
          if (f != 0.0) v = fma(f, H[j1].x * H[j2].x + H[j1].y * H[j2].y, v);  // Re H_j1 conj(H_j2)
        }
      a.v[c] = w * v;
    }
    __syncthreads();
  }
}

// q_p = sum of the prefix's class values, in class order (one wave per prefix, fixed tree).
__global__ __launch_bounds__(64) void marg_sum_kernel(MargArgs a) {
  const int lane = threadIdx.x;
  for (int64_t p = blockIdx.x; p < a.batch; p += gridDim.x) {
    const int64_t lo = a.pre_cls[p], hi = a.pre_cls[p + 1];
    const int64_t per = (hi - lo + 63) / 64;
    const int64_t b0 = lo + per * lane, b1 = b0 + per < hi ? b0 + per : hi;
    double s = 0.0;
    for (int64_t c = b0; c < b1; ++c) s += a.v[c];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) a.q_out[p] = s;
  }
}

__global__ void reset_kernel(int32_t* counter, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) counter[i] = 0;
}

// ---------------------------------------------------------------- host launchers

void launch_reset(int32_t* counter, int n, hipStream_t s) {
  hipLaunchKernelGGL(reset_kernel, dim3((n + 63) / 64), dim3(64), 0, s, counter, n);
}

void launch_finalize(const FinalizeArgs& a, hipStream_t s) {
  int64_t blocks = (a.batch + 3) / 4;  // four patterns (waves) per block
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a);
}

void launch_state(const double2* U, const double* r, int m, double2* B, double2* W, double* prefactor, hipStream_t s) {
  int64_t total = (int64_t)m * m;
  hipLaunchKernelGGL(state_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, U, r, m, B, W, prefactor);
}

// Inverse-CDF draw from unnormalised weights, one thread per row, sums in index order.
__global__ void draw_kernel(const double* w, int64_t batch, int m, const double* u, int32_t* next) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= batch) return;
  const double* row = w + b * m;
  double tot = 0.0;
  for (int l = 0; l < m; ++l) tot += row[l];
  const double t = u[b] * tot;
  double acc = 0.0;
  int pick = m - 1;
  for (int l = 0; l < m; ++l) {
    acc += row[l];
    if (acc >= t && row[l] > 0.0) {
      pick = l;
      break;
    }
  }
  next[b] = pick;
}

void launch_draw(const double* w, int64_t batch, int m, const double* u, int32_t* next, hipStream_t s) {
  if (batch <= 0) return;
  hipLaunchKernelGGL(draw_kernel, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, s, w, batch, m, u, next);
}

void launch_marginal(const MargArgs& a, int kmax, int64_t h_total, hipStream_t s) {
  if (a.batch <= 0) return;
  // hafnian tables, size by size (each level reads the previous one)
  const int64_t blocks = std::min<int64_t>(4096, (h_total + 255) / 256);
  for (int level = 0; level <= kmax; level += 2)
    hipLaunchKernelGGL(subset_haf_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a, level);
  if (a.n_classes > 0) {
    const int64_t g = a.n_classes < 65536 ? a.n_classes : 65536;
    hipLaunchKernelGGL(marg_class_kernel, dim3((unsigned)g), dim3(64), 0, s, a);
  }
  const int64_t g = a.batch < 65536 ? a.batch : 65536;
  hipLaunchKernelGGL(marg_sum_kernel, dim3((unsigned)g), dim3(64), 0, s, a);
}

// ---------------------------------------------------------------- engine dispatch

static const EngineVariant* variants() {
  static EngineVariant tab[kEngineClasses] = {};
  static const bool filled = [] {
    register_quad_engines(tab);
    register_grid4_engines(tab);
    register_grid5_engines(tab);
    register_strip_engines(tab);
    register_tile_engines(tab);
    register_dd_engines(tab);
    register_sqt_engines(tab);
    register_sqt7_engines(tab);
    return true;
  }();
  (void)filled;
  return tab;
}

static EngineVariant variant(int cls) {
  if (cls < 0 || cls >= kEngineClasses) return EngineVariant{nullptr, 0, 0, 0};
  return variants()[cls];
}

// Engine per subset size: the quad engine's grids up to |Z| = 10 (four subsets per wave on the 4x4x4
// MFMA; only the tiles on and above the diagonal), the strip engine for |Z| = 11, 12 up to k = 16 and
// the quad-tile engine above (where the strip engine's registers spill), the 16x16 tile engines
// (2x2 and 3x3 tiles per workgroup) for larger subsets.
// The shape bits move |Z| = 9, 10 and |Z| = 11, 12 to the 2x2 tile engine (chosen per n by the
// autotuner).
int engine_class(int s, int k, int shape) {
  if (s <= 6) return kClsQuad + (k - 1);
  if (s <= 8) return kClsGrid4 + (k - 5);
  if (s <= 10) {
    if ((shape & kShapeSqt910) && k >= 11) return kClsSqt + (k - 11);
    return (shape & kShapeTile910) ? kClsTile2 + (k - 9) : kClsGrid5 + (k - 9);
  }
  if (s <= 12) {
    if (shape & kShapeSqt1112) return kClsSqt + (k - 11);
    if (shape & kShapeTile1112) return kClsTile2 + (k - 9);
    return k <= 16 ? kClsStrip + (k - 11) : kClsQtile + (k - 17);
  }
  if (s <= 16) return (shape & kShapeSqt1314) && s <= 14 ? kClsSqt7 + (k - 13) : kClsTile2 + (k - 9);
  return kClsTile3 + (k - 17);
}

// Double-double engine per subset size: the smallest padded size 16 T that holds M_Z (d = 2s).
int engine_class_dd(int s) { return kClsDd + (2 * s + 15) / 16 - 1; }

size_t engine_lds_bytes(int cls, int nmax, int kmax, int stage_A) {
  const EngineVariant v = variant(cls);
  if (v.kind == kQtileKind) return qtile_lds_layout(nmax, kmax, stage_A).total;
  if (v.kind == kStripKind) return strip_lds_bytes(nmax, kmax, stage_A);
  if (v.kind == kTileKind) return tile_lds_layout(v.tiles, false, nmax, kmax, stage_A).total;
  if (v.kind == kTileSymKind) return tile_lds_layout(v.tiles, true, nmax, kmax, stage_A).total;
  if (v.kind == kDdKind) return dd_lds_layout(v.tiles, nmax, kmax).total;
  if (v.kind == kSqtKind) return sqt_lds_layout(v.tiles, nmax, kmax, stage_A).total;
  // the |Z| <= 6 kernel (tiles 3) parks no traces up to k = kQuad3WavesKMax
  if (v.tiles == 3 && kmax <= kQuad3WavesKMax) return quad_lds_bytes(nmax, kmax, stage_A, 0);
  return quad_lds_bytes(nmax, kmax, stage_A, quad_park_k(v.tiles, kmax));
}

static void allow_lds(int cls) {
  static std::atomic<bool> done[kEngineClasses] = {};
  if (cls < 0 || cls >= kEngineClasses || done[cls].load(std::memory_order_acquire)) return;
  (void)hipFuncSetAttribute(variant(cls).fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  done[cls].store(true, std::memory_order_release);
}

// Workgroups per CU from the occupancy API, cached per (variant, LDS bytes): every call of the
// library sizes its persistent grids with it.
int engine_blocks_per_cu(int cls, size_t lds) {
  const EngineVariant v = variant(cls);
  if (!v.fn) return 1;
  static std::mutex mu;
  static std::map<std::pair<int, size_t>, int> cache;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find({cls, lds});
    if (it != cache.end()) return it->second;
  }
  allow_lds(cls);
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, v.fn, v.threads, lds) != hipSuccess) return 1;
  nb = nb > 0 ? nb : 1;
  std::lock_guard<std::mutex> lk(mu);
  cache[{cls, lds}] = nb;
  return nb;
}

void launch_engine(int cls, const EngineArgs& a, int grid, size_t lds, hipStream_t s) {
  const EngineVariant v = variant(cls);
  if (!v.fn) return;
  allow_lds(cls);
  EngineArgs arg = a;
  void* kargs[] = {&arg};
  (void)hipLaunchKernel(v.fn, dim3(grid), dim3(v.threads), kargs, lds, s);
}

}  // namespace gbs
