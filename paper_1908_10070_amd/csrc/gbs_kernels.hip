// HIP kernels of libgbs for gfx950 (MI355X).
//
// Hafnian by the power-trace formula the paper cites for its O(n^3 2^(n/2)) cost (Sec. II C):
// with k = n/2, pairs (2i, 2i+1) and X the within-pair row swap,
//   Haf(A) = sum_{Z subset [k], Z != {}} (-1)^(k-|Z|) c_k(M_Z),   M_Z = X A_Z,
//   c_0 = 1,  q c_q = sum_{j=1..q} (tr(M_Z^j) / 2) c_{q-j}        (c_k = [lambda^k] det(I - lambda M_Z)^(-1/2)).
//
// Work layout (one workgroup = 4 waves):
//   * a work item is a range of the canonical subset order of one pattern (by |Z|, then bitmask);
//   * the pattern matrix (n <= 32) is staged in LDS once per item;
//   * "small" subsets (d = 2|Z| <= 16) run one per wave, "large" ones (d <= 48) on all four waves;
//   * per subset, a chain program forms a few powers of M_Z with FP64 MFMA (16x16x4 tiles, operands
//     read from LDS slots) and takes every t_j = tr(M_Z^j), j <= k, either from a diagonal or as an
//     inner product tr(M^a M^b);
//   * traces of 16 subsets are buffered, then 16 lanes run the coefficient recursion at once and
//     one lane adds the signed terms into a compensated (Neumaier) running sum;
//   * each item writes one compensated partial; a finalize kernel sums a pattern's partials in
//     item order, so the result depends only on n and the chunking, never on the batch around it.
#include <hip/hip_runtime.h>

#include "gbs_internal.h"

namespace gbs {

typedef double d4 __attribute__((ext_vector_type(4)));

__constant__ ConstTables c_tab;

struct __align__(16) C2 {
  double x, y;
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ void neumaier(double& s, double& c, double x) {
  double t = s + x;
  if (fabs(s) >= fabs(x))
    c += (s - t) + x;
  else
    c += (x - t) + s;
  s = t;
}

__device__ __forceinline__ double2 wave_sum(double2 v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    v.x += __shfl_xor(v.x, off, 64);
    v.y += __shfl_xor(v.y, off, 64);
  }
  return v;
}

// Canonical subset order for k pairs: all subsets of size 1, then size 2, ...; within a size,
// increasing bitmask (colexicographic order of the pair sets).
__device__ __forceinline__ uint32_t unrank_subset(int k, int64_t g, int* s_out) {
  int s = 1;
  uint64_t rem = (uint64_t)g;
  while (s < k && rem >= c_tab.binom[k][s]) {
    rem -= c_tab.binom[k][s];
    ++s;
  }
  uint32_t mask = 0;
  int c = k - 1;
  for (int i = s; i >= 1; --i) {
    while (c_tab.binom[c][i] > rem) --c;
    mask |= 1u << c;
    rem -= c_tab.binom[c][i];
    --c;
  }
  *s_out = s;
  return mask;
}

// LDS carve-up, computed identically on host and device.
struct LdsLayout {
  size_t A, modes, plist, slots, trbuf, cbuf, red, misc, total;
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

__host__ __device__ inline LdsLayout lds_layout(int nmax, int kmax, int slot_elems, int stage_A, int nslots) {
  LdsLayout L;
  size_t off = 0;
  L.A = off;
  off += stage_A ? align16(sizeof(double2) * nmax * nmax) : 0;
  L.modes = off;
  off += align16(sizeof(int32_t) * GBS_N_MAX);
  L.plist = off;
  off += align16(sizeof(int32_t) * 4 * kMaxK);
  L.slots = off;
  size_t small_slots = (size_t)4 * nslots * kSmallD * (kSmallD + 1);
  size_t large_slots = (size_t)nslots * slot_elems;
  off += align16(sizeof(double2) * (small_slots > large_slots ? small_slots : large_slots));
  L.trbuf = off;
  off += align16(sizeof(double2) * (kmax + 1) * kBatchG);
  L.cbuf = off;
  off += align16(sizeof(double2) * (kmax + 1) * kBatchG);
  L.red = off;
  off += align16(sizeof(double2) * (4 + kBatchG));
  L.misc = off;
  off += align16(sizeof(int32_t) * (kBatchG + 4));
  L.total = off;
  return L;
}

// ---------------------------------------------------------------- engine

__global__ __launch_bounds__(kThreads) void engine_kernel(EngineArgs args) {
  extern __shared__ __align__(16) unsigned char smem[];
  const LdsLayout L = lds_layout(args.nmax, args.kmax, args.slot_elems, args.stage_A, args.nslots);
  double2* Alds = reinterpret_cast<double2*>(smem + L.A);
  int32_t* mlds = reinterpret_cast<int32_t*>(smem + L.modes);
  int32_t* plist = reinterpret_cast<int32_t*>(smem + L.plist);
  double2* slots = reinterpret_cast<double2*>(smem + L.slots);
  double2* trbuf = reinterpret_cast<double2*>(smem + L.trbuf);  // [j][u] = t_j / 2
  double2* cbuf = reinterpret_cast<double2*>(smem + L.cbuf);    // [q][u]
  double2* red = reinterpret_cast<double2*>(smem + L.red);      // [4] cross-wave, then terms [kBatchG]
  double2* terms = red + 4;
  int32_t* misc = reinterpret_cast<int32_t*>(smem + L.misc);    // [0..kBatchG) subset sizes, [kBatchG] item

  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;

  int it = args.persistent ? 0 : (int)blockIdx.x;
  for (;;) {
    if (args.persistent) {
      __syncthreads();
      if (tid == 0) misc[kBatchG] = atomicAdd(args.counter, 1);
      __syncthreads();
      it = misc[kBatchG];
    }
    if (it >= args.n_items) break;

    const WorkItem item = args.items[it];
    const PatternDesc pd = args.pats[item.pattern];
    const int n = pd.n;
    const int k = n >> 1;
    const bool prob = args.modes != nullptr;

    // Stage the pattern: mode list (prob path) and, for n <= 32, the full n x n matrix.
    if (prob && tid < n) mlds[tid] = args.modes[pd.src + tid];
    __syncthreads();
    if (args.stage_A) {
      for (int e = tid; e < n * n; e += kThreads) {
        int i = e / n, j = e - i * n;
        Alds[e] = prob ? args.A[(int64_t)mlds[i] * args.m + mlds[j]] : args.A[pd.src + e];
      }
    }
    __syncthreads();

    int s_first;
    (void)unrank_subset(k, item.lo, &s_first);
    const bool small = 2 * s_first <= kSmallD;  // items never straddle the small/large boundary
    const int ngw = small ? 1 : 4;              // waves per subset group
    const int gw = small ? 0 : wave;            // wave index within the group
    const int grp = small ? wave : 0;           // group index
    const int gtid = gw * 64 + lane;            // thread index within the group
    const int gthreads = ngw * 64;
    const int S = small ? (kSmallD + 1) : args.slot_stride;
    double2* gslots = small ? slots + (size_t)grp * args.nslots * kSmallD * (kSmallD + 1) : slots;
    const int slot_sz = small ? kSmallD * (kSmallD + 1) : args.slot_elems;
    int32_t* gpl = plist + grp * kMaxK;
    const ChainProgram& prog = c_tab.prog[k];
    const int per_step = small ? 4 : 1;

    double run_sr = 0.0, run_si = 0.0, run_cr = 0.0, run_ci = 0.0;

    for (int64_t g0 = item.lo; g0 < item.hi; g0 += kBatchG) {
      const int cnt = (int)((item.hi - g0) < kBatchG ? (item.hi - g0) : kBatchG);
      for (int b0 = 0; b0 < cnt; b0 += per_step) {
        const int u = b0 + grp;  // batch slot of this group's subset
        const bool valid = u < cnt;
        int s = 0;
        uint32_t mask = 0;
        if (valid) mask = unrank_subset(k, g0 + u, &s);
        const int d = 2 * s;
        if (valid && gtid == 0) misc[u] = s;
        // pair list of the subset
        if (valid && gtid < k && ((mask >> gtid) & 1u)) gpl[__popc(mask & ((1u << gtid) - 1u))] = gtid;
        __syncthreads();
        // M_Z = X A_Z into slot 0: row a of M is row (a xor 1) of A_Z
        if (valid) {
          double2* M0 = gslots;
          for (int e = gtid; e < d * d; e += gthreads) {
            int a = e / d, c = e - a * d;
            int ia = 2 * gpl[(a ^ 1) >> 1] + ((a ^ 1) & 1);
            int ic = 2 * gpl[c >> 1] + (c & 1);
            double2 v;
            if (args.stage_A)
              v = Alds[ia * n + ic];
            else if (prob)
              v = args.A[(int64_t)mlds[ia] * args.m + mlds[ic]];
            else
              v = args.A[pd.src + (int64_t)ia * n + ic];
            M0[a * S + c] = v;
          }
        }
        __syncthreads();

        for (int oi = 0; oi < prog.nops; ++oi) {
          const Op op = prog.ops[oi];
          if (op.type == OP_MUL) {
            const double2* X = gslots + (size_t)op.a * slot_sz;
            const double2* Y = gslots + (size_t)op.b * slot_sz;
            double2* Z = gslots + (size_t)op.x * slot_sz;
            const int tiles = (d + 15) >> 4;
            const int nks = (d + 3) >> 2;
            d4 accr[3], acci[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
              accr[q] = d4{0.0, 0.0, 0.0, 0.0};
              acci[q] = d4{0.0, 0.0, 0.0, 0.0};
              const int tau = gw + 4 * q;
              if (valid && tau < tiles * tiles) {
                const int I = tau / tiles, J = tau - (tau / tiles) * tiles;
                const int row = 16 * I + (lane & 15);
                const int col = 16 * J + (lane & 15);
                for (int kk = 0; kk < nks; ++kk) {
                  const int kx = 4 * kk + (lane >> 4);
                  double2 xa = make_double2(0.0, 0.0), yb = make_double2(0.0, 0.0);
                  if (row < d && kx < d) xa = X[row * S + kx];
                  if (kx < d && col < d) yb = Y[kx * S + col];
                  accr[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa.x, yb.x, accr[q], 0, 0, 0);
                  accr[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(-xa.y, yb.y, accr[q], 0, 0, 0);
                  acci[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa.x, yb.y, acci[q], 0, 0, 0);
                  acci[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa.y, yb.x, acci[q], 0, 0, 0);
                }
              }
            }
            __syncthreads();  // the destination may be a dying operand
#pragma unroll
            for (int q = 0; q < 3; ++q) {
              const int tau = gw + 4 * q;
              if (valid && tau < tiles * tiles) {
                const int I = tau / tiles, J = tau - (tau / tiles) * tiles;
                const int col = 16 * J + (lane & 15);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                  const int row = 16 * I + (lane >> 4) + 4 * r;  // D[i][j]: lane j + 16 (i%4), reg i/4
                  if (row < d && col < d) Z[row * S + col] = make_double2(accr[q][r], acci[q][r]);
                }
              }
            }
            __syncthreads();
          } else {
            // trace: diagonal of one slot, or inner product of two
            double2 acc = make_double2(0.0, 0.0);
            if (valid) {
              const double2* X = gslots + (size_t)op.a * slot_sz;
              if (op.type == OP_TDIAG) {
                for (int i = gtid; i < d; i += gthreads) {
                  double2 v = X[i * S + i];
                  acc.x += v.x;
                  acc.y += v.y;
                }
              } else {
                const double2* Y = gslots + (size_t)op.b * slot_sz;
                for (int e = gtid; e < d * d; e += gthreads) {
                  int i = e / d, c = e - i * d;
                  double2 p = cmul(X[i * S + c], Y[c * S + i]);
                  acc.x += p.x;
                  acc.y += p.y;
                }
              }
            }
            acc = wave_sum(acc);
            if (small) {
              if (valid && lane == 0) trbuf[op.x * kBatchG + u] = make_double2(0.5 * acc.x, 0.5 * acc.y);
            } else {
              if (lane == 0) red[wave] = acc;
              __syncthreads();
              if (tid == 0) {
                double2 t = red[0];
                for (int w = 1; w < 4; ++w) {
                  t.x += red[w].x;
                  t.y += red[w].y;
                }
                if (valid) trbuf[op.x * kBatchG + u] = make_double2(0.5 * t.x, 0.5 * t.y);
              }
            }
            __syncthreads();
          }
        }
      }
      __syncthreads();

      // coefficient recursion, one lane per buffered subset
      if (tid < cnt) {
        const int u = tid;
        cbuf[u] = make_double2(1.0, 0.0);
        for (int q = 1; q <= k; ++q) {
          double ar = 0.0, ai = 0.0;
          for (int j = 1; j <= q; ++j) {
            double2 t = trbuf[j * kBatchG + u];
            double2 c = cbuf[(q - j) * kBatchG + u];
            ar = fma(t.x, c.x, ar);
            ar = fma(-t.y, c.y, ar);
            ai = fma(t.x, c.y, ai);
            ai = fma(t.y, c.x, ai);
          }
          const double iq = c_tab.inv[q];
          cbuf[q * kBatchG + u] = make_double2(ar * iq, ai * iq);
        }
        double2 ck = cbuf[k * kBatchG + u];
        if ((k - misc[u]) & 1) {
          ck.x = -ck.x;
          ck.y = -ck.y;
        }
        terms[u] = ck;
      }
      __syncthreads();
      if (tid == 0) {
        for (int u = 0; u < cnt; ++u) {
          neumaier(run_sr, run_cr, terms[u].x);
          neumaier(run_si, run_ci, terms[u].y);
        }
      }
      __syncthreads();
    }

    if (tid == 0) {
      gbs_partial p;
      p.s_re = run_sr;
      p.s_im = run_si;
      p.c_re = run_cr;
      p.c_im = run_ci;
      args.partials[item.partial] = p;
    }
    if (!args.persistent) break;
  }
}

// ---------------------------------------------------------------- finalize

__global__ void finalize_kernel(FinalizeArgs a) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < a.batch;
       b += (int64_t)gridDim.x * blockDim.x) {
    double sr = 0.0, si = 0.0, cr = 0.0, ci = 0.0;
    for (int64_t q = a.part_off[b]; q < a.part_off[b + 1]; ++q) {
      const gbs_partial p = a.partials[q];
      neumaier(sr, cr, p.s_re);
      neumaier(si, ci, p.s_im);
      cr += p.c_re;
      ci += p.c_im;
    }
    if (a.partial_out) {
      gbs_partial o;
      o.s_re = sr;
      o.s_im = si;
      o.c_re = cr;
      o.c_im = ci;
      a.partial_out[b] = o;
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
    if (a.haf_out) a.haf_out[b] = make_double2(hr, hi);
    if (a.prob_out) a.prob_out[b] = (*a.prefactor) * (hr * hr + hi * hi) / a.sfact[b];
  }
}

// ---------------------------------------------------------------- state

// B = U diag(tanh r) U^t (transpose), prefactor = prod_i 1/cosh r_i.
__global__ void state_kernel(const double2* U, const double* r, int m, double2* B, double* prefactor) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < (int64_t)m * m) {
    const int i = (int)(e / m), j = (int)(e - (int64_t)(e / m) * m);
    double br = 0.0, bi = 0.0;
    for (int l = 0; l < m; ++l) {
      const double t = tanh(r[l]);
      const double2 p = cmul(U[(int64_t)i * m + l], U[(int64_t)j * m + l]);
      br = fma(t, p.x, br);
      bi = fma(t, p.y, bi);
    }
    B[e] = make_double2(br, bi);
  }
  if (e == 0) {
    double pf = 1.0;
    for (int l = 0; l < m; ++l) pf /= cosh(r[l]);
    *prefactor = pf;
  }
}

__global__ void reset_kernel(int32_t* counter, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) counter[i] = 0;
}

// ---------------------------------------------------------------- host launchers

size_t engine_lds_bytes(int nmax, int kmax, int slot_elems, int stage_A, int nslots) {
  return lds_layout(nmax, kmax, slot_elems, stage_A, nslots).total;
}

static void allow_full_lds() {
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(engine_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr_set = true;
  }
}

int engine_blocks_per_cu(size_t lds_bytes) {
  allow_full_lds();
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, engine_kernel, kThreads, lds_bytes) != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}

void launch_reset(int32_t* counter, int n, hipStream_t s) {
  hipLaunchKernelGGL(reset_kernel, dim3((n + 63) / 64), dim3(64), 0, s, counter, n);
}

void launch_engine(const EngineArgs& a, int grid, size_t lds, hipStream_t s) {
  allow_full_lds();
  hipLaunchKernelGGL(engine_kernel, dim3(grid), dim3(kThreads), lds, s, a);
}

void launch_finalize(const FinalizeArgs& a, hipStream_t s) {
  int64_t blocks = (a.batch + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a);
}

void launch_state(const double2* U, const double* r, int m, double2* B, double* prefactor, hipStream_t s) {
  int64_t total = (int64_t)m * m;
  hipLaunchKernelGGL(state_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, U, r, m, B, prefactor);
}

int upload_tables(const ConstTables& t) {
  return hipMemcpyToSymbol(HIP_SYMBOL(c_tab), &t, sizeof(ConstTables)) == hipSuccess ? 0 : 1;
}

}  // namespace gbs
