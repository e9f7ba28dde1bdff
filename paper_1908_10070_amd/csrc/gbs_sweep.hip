// Output-space sweep with stored sub-hafnians, and the brute-force sampler over it.
//
// Every output pattern of n photons in m modes is a sorted mode list a_0 <= ... <= a_{n-1}
// (a multiset; with collisions excluded, a set). Its hafnian Haf(B_a) is the sum over perfect
// matchings of its positions (Eq. HafMatch); pairing position 0 with each other position j,
//   Haf(B_a) = sum_{j=1..l-1} B(a_0, a_j) Haf(B_{a minus positions 0, j}),
// and the smaller pattern is again a sorted mode list, two photons shorter. Storing the hafnians of
// all patterns of every even size l <= n (the paper's exponential-space variant keeps sub-hafnians
// this way, App. D) makes each hafnian of size l a sum of l - 1 products of table entries, and
// every sub-pattern shared by many patterns is evaluated once.
//
// Indexing. A multiset of size l over [m] is the strictly increasing b_i = a_i + i over
// [m + l - 1] (a set is b = a over [m]); its colexicographic rank is sum_i C(b_i, i + 1). Tables of
// the intermediate sizes are stored at that rank. The last size is written in lexicographic order
// of the mode lists (the order of itertools.combinations / combinations_with_replacement), whose
// rank is N - 1 - colex(sorted(U - 1 - b)) for the universe size U and N = C(U, l).
//
// The sampler (App. I) divides [0, 1) into one interval per pattern of length p(pattern) / total:
// an inclusive prefix sum of the probabilities (fixed order, so a given uniform always picks the
// same pattern) and a binary search per uniform.
#include <hip/hip_runtime.h>

#include "gbs_internal.h"

namespace gbs {

__device__ __forceinline__ uint64_t bn(const SweepArgs& a, int v, int i) {
  return (v < 0 || i < 0) ? 0 : a.binom[(int64_t)v * a.bstride + i];
}

// Largest v in [i - 1, U - 1] with C(v, i) <= r (C(v, i) grows with v).
__device__ __forceinline__ int colex_digit(const SweepArgs& a, int U, int i, uint64_t r) {
  int lo = i - 1, hi = U - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (bn(a, mid, i) <= r) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Strictly increasing b_0 < ... < b_{l-1} over [U] with colex rank r.
__device__ __forceinline__ void colex_unrank(const SweepArgs& a, int U, int l, uint64_t r, int* b) {
  for (int i = l; i >= 1; --i) {
    const int v = colex_digit(a, U, i, r);
    b[i - 1] = v;
    r -= bn(a, v, i);
    U = v;
  }
}

// Hafnian of the pattern b (size l, universe encoding as above) from the table of size l - 2.
__device__ double2 sweep_haf(const SweepArgs& a, const int* b, int l, const double2* prev) {
  const int sh = a.collisions ? 1 : 0;  // b_i = a_i + i for multisets
  int md[kSweepMaxN];
  for (int i = 0; i < l; ++i) md[i] = b[i] - sh * i;
  // rank of the pattern without positions 0 and j: the entries before j move down one place and
  // those after it two places; P[t] sums the first kind over t < j - 1, S[t] the second from t on
  uint64_t S[kSweepMaxN + 1];
  S[l - 2] = 0;
  for (int t = l - 3; t >= 0; --t) S[t] = S[t + 1] + bn(a, b[t + 2] - 2 * sh, t + 1);
  const double2* Brow = a.B + (int64_t)md[0] * a.m;
  double sr = 0.0, si = 0.0;
  uint64_t P = 0;
  for (int j = 1; j < l; ++j) {
    const uint64_t r = P + S[j - 1];
    const double2 w = Brow[md[j]];
    const double2 h = prev[r];
    sr = fma(w.x, h.x, sr);
    sr = fma(-w.y, h.y, sr);
    si = fma(w.x, h.y, si);
    si = fma(w.y, h.x, si);
    P += bn(a, b[j] - sh, j);  // entry j moves to place j - 1 for the next position
  }
  return make_double2(sr, si);
}

// Table of size `level` (even, 2 <= level < n): one thread per pattern, stored at its colex rank.
__global__ void sweep_level_kernel(SweepArgs a, int level, const double2* prev, double2* cur, int64_t count) {
  const int U = a.collisions ? a.m + level - 1 : a.m;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x) {
    int b[kSweepMaxN];
    colex_unrank(a, U, level, (uint64_t)t, b);
    cur[t] = sweep_haf(a, b, level, prev);
  }
}

// Size n: one thread per pattern in lexicographic order; hafnian and probability
// p = prefactor |Haf|^2 / prod_j s_j! (Eq. ProOri; s_j the multiplicities).
__global__ void sweep_final_kernel(SweepArgs a, const double2* prev, int64_t count) {
  const int n = a.n;
  const int U = a.collisions ? a.m + n - 1 : a.m;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x) {
    // lexicographic rank t <-> colex rank count - 1 - t of the reflected set U - 1 - b
    int d[kSweepMaxN], b[kSweepMaxN];
    colex_unrank(a, U, n, (uint64_t)(count - 1 - t), d);
    for (int i = 0; i < n; ++i) b[i] = U - 1 - d[n - 1 - i];
    double2 h = make_double2(1.0, 0.0);
    if (n > 0) h = sweep_haf(a, b, n, prev);
    if (a.haf_out) a.haf_out[t] = h;
    if (a.prob_out) {
      double sf = 1.0, run = 1.0;
      const int sh = a.collisions ? 1 : 0;
      for (int i = 1; i < n; ++i) {
        if (b[i] - sh * i == b[i - 1] - sh * (i - 1)) {
          run += 1.0;
          sf *= run;
        } else {
          run = 1.0;
        }
      }
      a.prob_out[t] = (*a.prefactor) * (h.x * h.x + h.y * h.y) / sf;
    }
  }
}

__global__ void sweep_zero_kernel(SweepArgs a, int64_t count) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x) {
    if (a.haf_out) a.haf_out[t] = make_double2(0.0, 0.0);
    if (a.prob_out) a.prob_out[t] = 0.0;
  }
}

__global__ void sweep_one_kernel(double2* t) { t[0] = make_double2(1.0, 0.0); }

static unsigned grid_for(int64_t count) {
  int64_t g = (count + 255) / 256;
  if (g > 16384) g = 16384;
  return (unsigned)(g < 1 ? 1 : g);
}

void launch_sweep(const SweepArgs& a, double2* tab0, double2* tab1, const int64_t* level_count, hipStream_t s) {
  if (a.n & 1) {
    hipLaunchKernelGGL(sweep_zero_kernel, dim3(grid_for(a.count)), dim3(256), 0, s, a, a.count);
    return;
  }
  // level 0: the empty pattern, Haf = 1; then every even size below n, alternating two tables
  hipLaunchKernelGGL(sweep_one_kernel, dim3(1), dim3(1), 0, s, tab0);
  double2* prev = tab0;
  double2* cur = tab1;
  for (int l = 2; l < a.n; l += 2) {
    hipLaunchKernelGGL(sweep_level_kernel, dim3(grid_for(level_count[l])), dim3(256), 0, s, a, l, prev, cur,
                       level_count[l]);
    double2* t = prev;
    prev = cur;
    cur = t;
  }
  hipLaunchKernelGGL(sweep_final_kernel, dim3(grid_for(a.count)), dim3(256), 0, s, a, prev, a.count);
}

// ---------------------------------------------------------------- prefix sum and draw

constexpr int kCdfTile = 2048;  // elements per block: 256 threads x 8

// Block b: inclusive prefix sums of its tile into cdf (local), its total into bsum[b].
__global__ __launch_bounds__(256) void cdf_local_kernel(const double* p, int64_t count, double* cdf, double* bsum) {
  __shared__ double part[256];
  const int64_t base = (int64_t)blockIdx.x * kCdfTile;
  const int tid = threadIdx.x;
  double v[8];
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int64_t i = base + tid * 8 + q;
    s += i < count ? p[i] : 0.0;
    v[q] = s;
  }
  part[tid] = s;
  __syncthreads();
  if (tid == 0) {  // fixed-order exclusive scan of the 256 thread sums
    double acc = 0.0;
    for (int t = 0; t < 256; ++t) {
      const double x = part[t];
      part[t] = acc;
      acc += x;
    }
    bsum[blockIdx.x] = acc;
  }
  __syncthreads();
  const double off = part[tid];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int64_t i = base + tid * 8 + q;
    if (i < count) cdf[i] = off + v[q];
  }
}

// Exclusive scan of the block totals (one thread, in block order); total into *total.
__global__ void cdf_blocks_kernel(double* bsum, int64_t nblocks, double* total) {
  double acc = 0.0;
  for (int64_t b = 0; b < nblocks; ++b) {
    const double x = bsum[b];
    bsum[b] = acc;
    acc += x;
  }
  *total = acc;
}

__global__ void cdf_offset_kernel(double* cdf, int64_t count, const double* bsum) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    cdf[i] += bsum[i / kCdfTile];
}

// idx[s] = the first i with cdf[i] > u[s] * total (u in [0, 1)): the pattern whose interval holds u.
__global__ void cdf_draw_kernel(const double* cdf, int64_t count, const double* total, const double* u,
                                int64_t nsamples, int64_t* idx) {
  const double T = *total;
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < nsamples; s += (int64_t)gridDim.x * blockDim.x) {
    const double target = u[s] * T;
    int64_t lo = 0, hi = count - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (cdf[mid] > target) hi = mid;
      else lo = mid + 1;
    }
    idx[s] = lo;
  }
}

void launch_cdf(const double* p, int64_t count, double* cdf, double* bsum, double* total, hipStream_t s) {
  const int64_t nb = (count + kCdfTile - 1) / kCdfTile;
  hipLaunchKernelGGL(cdf_local_kernel, dim3((unsigned)nb), dim3(256), 0, s, p, count, cdf, bsum);
  hipLaunchKernelGGL(cdf_blocks_kernel, dim3(1), dim3(1), 0, s, bsum, nb, total);
  hipLaunchKernelGGL(cdf_offset_kernel, dim3(grid_for(count)), dim3(256), 0, s, cdf, count, (const double*)bsum);
}

void launch_cdf_draw(const double* cdf, int64_t count, const double* total, const double* u, int64_t nsamples,
                     int64_t* idx, hipStream_t s) {
  hipLaunchKernelGGL(cdf_draw_kernel, dim3(grid_for(nsamples)), dim3(256), 0, s, cdf, count, total, u, nsamples, idx);
}

int64_t cdf_blocks(int64_t count) { return (count + kCdfTile - 1) / kCdfTile; }

}  // namespace gbs
