/*
 * CPU oracle for hafnians -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library. The product path never calls it and shares no code
 * with it.
 *
 * Two independent routes to the same number:
 *
 *   orc_haf_enum*  Haf(V) = sum over perfect matchings sigma of [n] of
 *                  prod_j V(sigma_{2j-1}, sigma_{2j})          (Sec. II C, Eq. HafMatch)
 *                  written as the recursion "pair the lowest remaining index i
 *                  with every other remaining j", memoised on the bitmask of the
 *                  remaining indices for n <= 24 (same enumeration, shared
 *                  subtrees). Diagonal entries are never read.
 *
 *   orc_haf_pt*    The power-trace formula the paper cites for its O(n^3 2^(n/2))
 *                  hafnian (Sec. II C): with k = n/2, pairs (2i, 2i+1), and
 *                  X the matrix that swaps the two rows of every pair,
 *                    Haf(A) = sum_{Z subset of [k]} (-1)^(k-|Z|) c_k(X A_Z),
 *                  where A_Z keeps the rows/columns of the pairs in Z and
 *                  c_k(M) = [lambda^k] det(I - lambda M)^(-1/2)
 *                         = [lambda^k] exp( sum_j tr(M^j) lambda^j / (2j) ).
 *                  c_0 = 1, q c_q = sum_{j=1..q} (tr(M^j)/2) c_{q-j}
 *                  (differentiate the exponential). Powers are formed by plain
 *                  repeated multiplication M^j = M^(j-1) M, traces read off the
 *                  diagonal, the subset terms summed in increasing bitmask order.
 *                  A double and a long-double build are provided.
 *
 * Matrices are dense row-major n x n complex (re, im interleaved), any
 * (complex-)symmetric input. Odd n gives 0, n = 0 gives 1.
 */
#include <complex.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double _Complex cplx;
typedef long double _Complex lcplx;

/* ---------------------------------------------------------------- enum --- */

struct enum_ctx {
  const cplx* A;
  int n;
  cplx* memo;           /* indexed by remaining-set bitmask (n <= 24) */
  unsigned char* known;
};

static cplx enum_rec(struct enum_ctx* c, uint64_t rem) {
  if (rem == 0) return 1.0;
  if (c->memo && c->known[rem]) return c->memo[rem];
  int i = __builtin_ctzll(rem);
  uint64_t rest = rem & ~(1ull << i);
  cplx acc = 0.0;
  for (uint64_t r = rest; r; r &= r - 1) {
    int j = __builtin_ctzll(r);
    acc += c->A[(size_t)i * c->n + j] * enum_rec(c, rest & ~(1ull << j));
  }
  if (c->memo) {
    c->memo[rem] = acc;
    c->known[rem] = 1;
  }
  return acc;
}

/* Returns 0 on success, 1 on bad size, 2 on allocation failure. */
int orc_haf_enum(const double* A_ri, int n, double* out_ri) {
  if (n < 0 || n > 64) return 1;
  cplx res;
  if (n % 2) {
    res = 0.0;
  } else if (n == 0) {
    res = 1.0;
  } else {
    struct enum_ctx c = {(const cplx*)A_ri, n, NULL, NULL};
    if (n <= 24) {
      size_t sz = (size_t)1 << n;
      c.memo = (cplx*)malloc(sz * sizeof(cplx));
      c.known = (unsigned char*)calloc(sz, 1);
      if (!c.memo || !c.known) {
        free(c.memo);
        free(c.known);
        return 2;
      }
    }
    uint64_t full = (n == 64) ? ~0ull : ((1ull << n) - 1);
    res = enum_rec(&c, full);
    free(c.memo);
    free(c.known);
  }
  out_ri[0] = creal(res);
  out_ri[1] = cimag(res);
  return 0;
}

int orc_haf_enum_batch(const double* A_ri, int n, long batch, double* out_ri) {
  for (long b = 0; b < batch; ++b) {
    int rc = orc_haf_enum(A_ri + (size_t)b * n * n * 2, n, out_ri + 2 * b);
    if (rc) return rc;
  }
  return 0;
}

/* ---------------------------------------------------------- power trace --- */

/* One definition, instantiated for double and long double. NAME_kappa also returns, in
   stats[0], sum_Z |t_Z| and, in stats[1], sum_Z |t_Z|^2, where t_Z = (-1)^(k-|Z|) c_k(X A_Z)
   is the subset term: kappa = stats[0] / |Haf| measures the cancellation in the subset sum,
   and sqrt(stats[1]) / |Haf| its root-sum-square counterpart. */
#define DEFINE_HAF_PT(NAME, REAL, CPLX, CABS)                                    \
  int NAME##_kappa(const double* A_ri, int n, double* out_ri, double* stats);   \
  int NAME(const double* A_ri, int n, double* out_ri) {                         \
    return NAME##_kappa(A_ri, n, out_ri, NULL);                                 \
  }                                                                             \
  int NAME##_kappa(const double* A_ri, int n, double* out_ri, double* stats) {  \
    if (stats) { stats[0] = 0.0; stats[1] = 0.0; }                             \
    if (n < 0 || n > 64) return 1;                                              \
    if (n % 2) { out_ri[0] = 0.0; out_ri[1] = 0.0; return 0; }                  \
    int k = n / 2;                                                              \
    if (k == 0) {                                                               \
      out_ri[0] = 1.0; out_ri[1] = 0.0;                                         \
      if (stats) { stats[0] = 1.0; stats[1] = 1.0; }                            \
      return 0;                                                                 \
    }                                                                           \
    if (k > 40) return 1;                                                       \
    CPLX* A = (CPLX*)malloc(sizeof(CPLX) * n * n);                              \
    CPLX* M = (CPLX*)malloc(sizeof(CPLX) * n * n);                              \
    CPLX* P = (CPLX*)malloc(sizeof(CPLX) * n * n);                              \
    CPLX* Q = (CPLX*)malloc(sizeof(CPLX) * n * n);                              \
    CPLX* t = (CPLX*)malloc(sizeof(CPLX) * (k + 1));                            \
    CPLX* c = (CPLX*)malloc(sizeof(CPLX) * (k + 1));                            \
    int* idx = (int*)malloc(sizeof(int) * n);                                   \
    if (!A || !M || !P || !Q || !t || !c || !idx) {                             \
      free(A); free(M); free(P); free(Q); free(t); free(c); free(idx);          \
      return 2;                                                                 \
    }                                                                           \
    for (int i = 0; i < n * n; ++i)                                             \
      A[i] = (REAL)A_ri[2 * i] + (REAL)A_ri[2 * i + 1] * (CPLX)I;               \
    CPLX total = 0;                                                             \
    REAL mag = 0, mag2 = 0;                                                     \
    for (uint64_t Z = 1; Z < (1ull << k); ++Z) {                                \
      int d = 0;                                                                \
      for (int i = 0; i < k; ++i)                                               \
        if (Z >> i & 1) { idx[d++] = 2 * i; idx[d++] = 2 * i + 1; }             \
      int s = d / 2;                                                            \
      /* M = X A_Z: row a of M is row (a xor 1) of A_Z. */                      \
      for (int a = 0; a < d; ++a)                                               \
        for (int b = 0; b < d; ++b)                                             \
          M[a * d + b] = A[idx[a ^ 1] * n + idx[b]];                            \
      /* t_j = tr(M^j), j = 1..k, by repeated multiplication. */                \
      memcpy(P, M, sizeof(CPLX) * d * d);                                       \
      for (int j = 1; j <= k; ++j) {                                            \
        CPLX tr = 0;                                                            \
        for (int a = 0; a < d; ++a) tr += P[a * d + a];                         \
        t[j] = tr;                                                              \
        if (j == k) break;                                                      \
        for (int a = 0; a < d; ++a)                                             \
          for (int b = 0; b < d; ++b) {                                         \
            CPLX acc = 0;                                                       \
            for (int l = 0; l < d; ++l) acc += P[a * d + l] * M[l * d + b];     \
            Q[a * d + b] = acc;                                                 \
          }                                                                     \
        memcpy(P, Q, sizeof(CPLX) * d * d);                                     \
      }                                                                         \
      /* c_0 = 1, q c_q = sum_j (t_j / 2) c_{q-j}. */                           \
      c[0] = 1;                                                                 \
      for (int q = 1; q <= k; ++q) {                                            \
        CPLX acc = 0;                                                           \
        for (int j = 1; j <= q; ++j) acc += (t[j] / (REAL)2) * c[q - j];        \
        c[q] = acc / (REAL)q;                                                   \
      }                                                                         \
      if ((k - s) % 2) total -= c[k]; else total += c[k];                       \
      mag += CABS(c[k]);                                                        \
      mag2 += CABS(c[k]) * CABS(c[k]);                                          \
    }                                                                           \
    out_ri[0] = (double)creall(total);                                          \
    out_ri[1] = (double)cimagl(total);                                          \
    if (stats) { stats[0] = (double)mag; stats[1] = (double)mag2; }             \
    free(A); free(M); free(P); free(Q); free(t); free(c); free(idx);            \
    return 0;                                                                   \
  }

DEFINE_HAF_PT(orc_haf_pt, double, cplx, cabs)
DEFINE_HAF_PT(orc_haf_pt_ld, long double, lcplx, cabsl)

int orc_haf_pt_batch(const double* A_ri, int n, long batch, double* out_ri) {
  for (long b = 0; b < batch; ++b) {
    int rc = orc_haf_pt(A_ri + (size_t)b * n * n * 2, n, out_ri + 2 * b);
    if (rc) return rc;
  }
  return 0;
}

int orc_haf_pt_ld_batch(const double* A_ri, int n, long batch, double* out_ri) {
  for (long b = 0; b < batch; ++b) {
    int rc = orc_haf_pt_ld(A_ri + (size_t)b * n * n * 2, n, out_ri + 2 * b);
    if (rc) return rc;
  }
  return 0;
}
