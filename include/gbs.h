/*
 * gbs.h -- C ABI of the MI355X (gfx950) library for batched Gaussian-boson-
 * sampling probabilities and hafnians.
 *
 * What it computes (Wu, Cheng, Zhang, Yung, Sun, arXiv:1908.10070):
 *
 *   Haf(V) = sum over perfect matchings sigma of [n] of prod_j V(sigma_{2j-1}, sigma_{2j})
 *            (Sec. II C, Eq. HafMatch), evaluated with the power-trace formula the paper
 *            cites for its O(n^3 2^(n/2)) hafnian: with k = n/2, pairs (2i, 2i+1) and X the
 *            within-pair row swap,
 *              Haf(A) = sum_{Z subset of [k]} (-1)^(k-|Z|) [lambda^k] det(I - lambda X A_Z)^(-1/2).
 *
 *   p(x)   = |Haf(B_x)|^2 / (prod_j s_j! * prod_i cosh r_i),   B = U diag(tanh r_i) U^t,
 *            B_x(i, j) = B(x_i, x_j)        (Eq. ProOri with W = U U^t, Sec. II C; the
 *            position-sequence matrix W_x of Sec. III B and App. B). For identical r_i this is
 *            exactly Eq. ProOri; per-mode r_i are the natural generalisation.
 *
 * Conventions
 *   - gbs_c128 is bit-identical to C99 double _Complex, torch.complex128, hipDoubleComplex.
 *   - "_dev" pointers are device memory on the context's device; "_host" pointers are host memory.
 *   - Every entry point returns an int status (GBS_OK on success). Nothing throws or aborts
 *     across the ABI. On failure no work has been enqueued unless the status is GBS_EHIP (or
 *     GBS_EINVAL from the debug symmetry check, which runs its own kernel first).
 *   - Compute calls enqueue on `stream` (a hipStream_t passed as void*; NULL = legacy default
 *     stream) and return at once; outputs are valid once the stream reaches the work.
 *     Host arrays are read before the call returns and may be reused afterwards.
 *   - Device inputs must stay alive and unmodified until the stream reaches the work.
 *   - A context is not thread-safe: use one per host thread (and per stream if work on
 *     several streams must overlap). Calls on one context serialise on its internal staging.
 *     A context keeps the host storage of its largest work plan (about 50 bytes per work item
 *     and 40 per pattern: 32 MB for 100,000 twenty-photon patterns) so that later calls plan
 *     without reallocating; gbs_ctx_destroy releases it.
 *   - n (photon number, matrix size) must satisfy 0 <= n <= GBS_N_MAX. n = 0 gives Haf = 1;
 *     odd n gives Haf = 0 and p = 0 (P_n = 0 for odd n, Eq. Eqdistribution).
 *   - Input matrices are assumed complex symmetric; diagonal entries are never used
 *     (matchings pair distinct indices), so they may hold anything finite.
 *   - Non-finite inputs propagate as NaN; that is not an error.
 */
#ifndef GBS_H_
#define GBS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GBS_N_MAX 46

typedef struct {
  double re, im;
} gbs_c128;

/* Compensated partial sum of subset terms: value = (s_re + c_re) + i (s_im + c_im). */
typedef struct {
  double s_re, s_im, c_re, c_im;
} gbs_partial;

typedef struct gbs_ctx gbs_ctx;
typedef struct gbs_state gbs_state;

enum {
  GBS_OK = 0,
  GBS_EINVAL = 1,        /* null pointer, negative size, malformed offsets */
  GBS_ERANGE = 2,        /* a mode outside [0, m), n > GBS_N_MAX, subset range outside [0, 2^(n/2)-1] */
  GBS_ENOMEM = 3,        /* caller workspace or state memory too small (see gbs_ctx_workspace_needed) */
  GBS_EHIP = 4,          /* a HIP runtime call failed; gbs_last_error() has the text */
  GBS_EUNSUPPORTED = 5   /* device is not gfx950 */
};

/* ---------------------------------------------------------------- context */

/* Device memory. The library never allocates device memory: the caller owns every device buffer
 * (in the Python binding, PyTorch tensors), including each context's workspace and each state's
 * memory. Host-side, a context holds pinned staging buffers, the launch-shape table and cached HIP
 * graphs.
 *
 * Create a context on `device`. workspace_dev/workspace_bytes: the caller-owned device buffer the
 * library carves each call's scratch from (staged plan and patterns, work counters, partial sums,
 * marginal tables). It may be NULL/0 at creation. A call whose plan does not fit returns GBS_ENOMEM,
 * enqueues nothing, and records the size it needed (gbs_ctx_workspace_needed); the caller then
 * installs a larger buffer with gbs_ctx_set_workspace and repeats the call. */
int gbs_ctx_create(int device, void* workspace_dev, size_t workspace_bytes, gbs_ctx** out);
int gbs_ctx_destroy(gbs_ctx* ctx);
/* Replace the workspace. Waits until the work this context has enqueued is done (the old buffer
 * may be released afterwards) and drops the cached graphs, which refer to the old buffer. */
int gbs_ctx_set_workspace(gbs_ctx* ctx, void* workspace_dev, size_t workspace_bytes);
/* Bytes the last call that returned GBS_ENOMEM on this context needed (0 if none did). */
size_t gbs_ctx_workspace_needed(const gbs_ctx* ctx);

/* Static description of a status code. */
const char* gbs_status_str(int status);
/* Detail text of the last failure on this context (empty string if none). Valid until the next call. */
const char* gbs_last_error(const gbs_ctx* ctx);

/* Execution options.
 *   use_graph:   1 = capture the batch's kernels in a HIP graph and replay it (cached per launch
 *                shape); 0 = launch eagerly.
 *   persistent:  1 = persistent work-queue kernels (grid sized to the device, items taken from an
 *                atomic counter); 0 = one workgroup per work item.
 * Defaults: use_graph = 1, persistent = 1. */
int gbs_ctx_set_exec(gbs_ctx* ctx, int use_graph, int persistent);

/* Spread each call's engine kernels (one per kernel variant the call needs) round-robin over nstreams
 * internal streams, forked from the call's stream after its staging copy and joined back before the
 * final combine, so that the kernels of a mixed batch (a serving step: many sizes, each a few
 * patterns) run side by side instead of one after another. With use_graph the fork and join are
 * captured as graph edges. 1 = every kernel on the call's stream. Until this is called the context
 * holds 2 and a call whose patterns all have one size n takes the built-in count for that n (two,
 * so that a one-size batch's few kernels overlap their tails; one at n = 18 and 20, where two measured
 * slower); a call that mixes sizes takes 2. Once called, every call takes nstreams (a serving step's
 * many small kernels want about 4). Results are the same bit for bit. GBS_EINVAL outside [1, 8];
 * GBS_EHIP if a stream or event cannot be created. */
int gbs_ctx_set_streams(gbs_ctx* ctx, int32_t nstreams);
/* The context's stream count (*nstreams; 2 until gbs_ctx_set_streams). GBS_EINVAL for a null
 * argument. */
int gbs_ctx_get_streams(const gbs_ctx* ctx, int32_t* nstreams);

/* Debugging hooks (process-wide, any thread).
 * gbs_debug_fault_inject(N): the N-th library call from now on that would enqueue compute work
 *   (hafnians, probabilities, slices, finalize, marginals, sweeps, draws) returns GBS_EHIP with
 *   "injected launch failure" in gbs_last_error and enqueues nothing; N <= 0 turns it off. The
 *   environment variable GBS_FAULT_INJECT=launch:N sets the same at the first such call. For testing
 *   the failure handling of callers (a server must fail that request only and keep serving).
 * gbs_debug_check_symmetry(on): before haf_batch / haf_batch_varlen run, check every caller-provided
 *   matrix for |A_ij - A_ji| <= 1e-12 max|A| (the power-trace formula assumes a symmetric matrix and
 *   otherwise computes the hafnian of its symmetric part's pairing, silently); an asymmetric one makes
 *   the call return GBS_EINVAL after the check's own kernel and a stream synchronisation. Also
 *   GBS_CHECK_SYMMETRY=1 in the environment. Off by default: the check costs a synchronisation. */
int gbs_debug_fault_inject(int64_t launch_n);
int gbs_debug_check_symmetry(int32_t on);

/* Arithmetic of the subset sum (Sec. III, the power-trace formula), per context:
 *   GBS_PREC_FP64: FP64 on the matrix cores (default). Rounding error about n^2 u kappa relative,
 *                  u = 2^-53, kappa = sum_Z |term(Z)| / |Haf| the cancellation of the subset sum.
 *   GBS_PREC_DD:   double-double (about 106 bits) on the vector ALUs: the same sum with error about
 *                  n^2 u^2 kappa, so the result is correct to FP64 rounding unless kappa > ~1e25;
 *                  roughly 10-40x the FP64 cost. For the large-n patterns whose cancellation reaches
 *                  1e7..1e12 (n = 36..46).
 * Applies to every later hafnian and probability call on the context (haf_batch, haf_batch_varlen,
 * haf_batch_noalloc, gbs_prob_batch, gbs_haf_partial); GBS_EINVAL for another value. */
#define GBS_PREC_FP64 0
#define GBS_PREC_DD 1
int gbs_ctx_set_precision(gbs_ctx* ctx, int32_t precision);
int32_t gbs_ctx_get_precision(const gbs_ctx* ctx);

/* Launch-shape table (what the autotuner writes): for photon number n, the number of subsets per
 * work item for the small-subset engine (subsets with 2|Z| <= 16) and for the large-subset engine.
 * chunk <= 0 restores the built-in default. Results depend only on these values and n, never on
 * how patterns are batched together. */
int gbs_ctx_set_tuning(gbs_ctx* ctx, int32_t n, int64_t chunk_small, int64_t chunk_large);
int gbs_ctx_get_tuning(const gbs_ctx* ctx, int32_t n, int64_t* chunk_small, int64_t* chunk_large);

/* Engine shape (what the autotuner picks besides the chunk sizes): for photon number n, which
 * engine evaluates the middle subset sizes. Bits:
 *   GBS_SHAPE_TILE_9_10   |Z| = 9, 10 on the 16x16-tile engine (2x2 tiles) instead of the 4x4-tile
 *                         quad engine on a 5x5 grid;
 *   GBS_SHAPE_TILE_11_12  |Z| = 11, 12 on the 16x16-tile engine instead of the strip engine
 *                         (k <= 16) or the quad-tile engine (k >= 17).
 *   GBS_SHAPE_SQT_11_12   |Z| = 11, 12 on the symmetric quad-tile engine (4x4 tiles, only those on and
 *                         above the diagonal, spread over four waves); needs k = n/2 >= 11;
 *   GBS_SHAPE_SQT_9_10    |Z| = 9, 10 on the symmetric quad-tile engine (k >= 11);
 *   GBS_SHAPE_SQT_13_14   |Z| = 13, 14 on the symmetric quad-tile engine on a 7x7 grid instead of
 *                         the 16x16-tile engine (k >= 13).
 * The quad-tile bits win over the tile bits of the same band. -1 removes the entry (back to the
 * built-in table). Results differ only at the rounding level. GBS_ERANGE for n outside
 * [0, GBS_N_MAX], GBS_EINVAL for unknown bits. */
#define GBS_SHAPE_TILE_9_10 1
#define GBS_SHAPE_TILE_11_12 2
#define GBS_SHAPE_SQT_11_12 4
#define GBS_SHAPE_SQT_9_10 8
#define GBS_SHAPE_SQT_13_14 16
int gbs_ctx_set_shape(gbs_ctx* ctx, int32_t n, int32_t shape);
int gbs_ctx_get_shape(const gbs_ctx* ctx, int32_t n, int32_t* shape);

/* Algorithmic FP64 flop count of one hafnian of size n: the power-trace method as formulated, every
 * pair subset Z forming all n/2 traces with the library's chain program for n/2 (matrix products,
 * trace inner products, coefficient recursion; a complex multiply-add counts 8). The kernels do
 * less arithmetic than this (three-product complex multiplies, only the tiles on and above the
 * diagonal, short chains for 2|Z| < n/2), so flops/s against this count is throughput in method
 * flops, not executed hardware work. Padding and bookkeeping are not counted. */
double gbs_haf_flops(int32_t n);

/* ---------------------------------------------------------------- hafnians */

/* Hafnians of `batch` matrices of size n x n, row-major complex128, matrix b starting at
 * A_dev + b * stride_elems (stride_elems >= n*n). haf_out_dev[b] receives Haf(A_b).
 * A_dev may be NULL when n = 0 (every result is 1). */
int haf_batch(gbs_ctx* ctx, const gbs_c128* A_dev, int32_t n, int64_t batch, int64_t stride_elems,
              gbs_c128* haf_out_dev, void* stream);

/* Hafnians of matrices of mixed sizes: matrix b is n_host[b] x n_host[b], row-major, starting at
 * A_dev + elem_off_host[b]. */
int haf_batch_varlen(gbs_ctx* ctx, const gbs_c128* A_dev, const int64_t* elem_off_host,
                     const int32_t* n_host, int64_t batch, gbs_c128* haf_out_dev, void* stream);

/* haf_batch for callers that cannot allocate memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): the same arguments, work items, kernels and summation
 * order as haf_batch at the context's chunk sizes (so the same results, bit for bit), but the plan
 * is built on the device and the plan, work counters and partial sums live in a static 32 MiB
 * scratch array per device instead of the context's workspace; no device or pinned host memory is
 * allocated, nothing is staged from the host, and the launches are eager (no graph). The scratch needs about 56 bytes per work item
 * plus 36 per matrix (n = 24 at the built-in chunks: 11 items per matrix, so 4096 matrices take
 * 2.7 MB); a call that needs more returns GBS_ENOMEM and enqueues nothing. All calls on one GPU
 * share that GPU's scratch, which keeps the last call's contents (the work counters are cleared by
 * a kernel at the start of every call): calls that overlap on one GPU (other streams, other
 * contexts, other host threads) race and must be ordered by the caller. */
int haf_batch_noalloc(gbs_ctx* ctx, const gbs_c128* A_dev, int32_t n, int64_t batch, int64_t stride_elems,
                      gbs_c128* haf_out_dev, void* stream);

/* ------------------------------------------------------------ GBS state */

/* Device bytes a state on m modes needs (B and W, m*m complex128 each, the m squeezing values and
 * the prefactor, 256-byte aligned); 0 for m outside [1, 4096]. */
size_t gbs_state_bytes(int32_t m);
/* Build a resident GBS state from an m x m unitary U (device, row-major complex128) and per-mode
 * squeezing parameters r (host, m doubles). A kernel forms B = U diag(tanh r_i) U^t, W = U U^t
 * (the marginal probabilities' matrix) and the prefactor 1 / prod_i cosh r_i on the device
 * (Sec. II C: W = U U^t; Eq. ProOri) in state_mem_dev, caller-owned device memory of at least
 * gbs_state_bytes(m) bytes that must stay allocated until gbs_state_destroy. U_dev is read only by
 * that kernel: it may be freed once the stream has reached it. The state is bound to the context's
 * device and may be used with any context on that device. Errors: GBS_EINVAL for null pointers or
 * non-finite r, GBS_ERANGE for m outside [1, 4096], GBS_ENOMEM if state_mem_bytes is too small. */
int gbs_state_create(gbs_ctx* ctx, const gbs_c128* U_dev, int32_t m, const double* r_host,
                     void* state_mem_dev, size_t state_mem_bytes, void* stream, gbs_state** out);
/* Waits for the state's setup, then releases the host object (not state_mem_dev). */
int gbs_state_destroy(gbs_state* state);
/* Device pointer to the state's B (m x m row-major complex128), and m / the prefactor (host copy,
 * valid after the creating stream has been synced). */
int gbs_state_info(const gbs_state* state, const gbs_c128** B_dev, int32_t* m, double* prefactor);
/* Copy the state's B (m*m complex128) into caller device memory dst_dev, enqueued on `stream`. */
int gbs_state_copy_B(const gbs_state* state, gbs_c128* dst_dev, void* stream);

/* ------------------------------------------------------------ probabilities */

/* Probabilities of `batch` output patterns. Pattern b is the mode list (position sequence x)
 * modes_host[offsets_host[b] .. offsets_host[b+1]), modes in [0, m), repeats allowed (collisions
 * give the prod s_j! divisor), order irrelevant (App. B). offsets_host has batch+1 entries,
 * offsets_host[0] = 0 and non-decreasing.
 * prob_out_dev[b] = |Haf(B_x)|^2 / (prod_j s_j! prod_i cosh r_i); haf_out_dev (nullable)
 * receives Haf(B_x). */
int gbs_prob_batch(gbs_ctx* ctx, const gbs_state* state, const int32_t* modes_host,
                   const int64_t* offsets_host, int64_t batch, double* prob_out_dev,
                   gbs_c128* haf_out_dev, void* stream);

/* ------------------------------------------- split evaluation (for schedulers) */

/* The 2^k - 1 non-empty pair subsets Z of a size-n pattern (k = n/2) are ordered by |Z| and, within
 * one size, by increasing bitmask. gbs_subset_count(n) = 2^(n/2) - 1 for even n (0 for odd n or n=0). */
int64_t gbs_subset_count(int32_t n);

/* Partial sums of the subset terms over index ranges [lo_host[b], hi_host[b]) of pattern b
 * (0 <= lo <= hi <= gbs_subset_count(n)). Slice b's compensated partial is written to
 * partials_dev[out_idx_host ? out_idx_host[b] : b] (indices >= 0; the caller sizes partials_dev).
 * Summing the partials of consecutive ranges covering [0, count) with gbs_finalize gives the
 * pattern's hafnian; a slice's partial depends only on the pattern and its range, so a scheduler
 * may split one pattern over several calls. Patterns as in gbs_prob_batch. */
int gbs_prob_slices(gbs_ctx* ctx, const gbs_state* state, const int32_t* modes_host,
                    const int64_t* offsets_host, const int64_t* lo_host, const int64_t* hi_host,
                    int64_t batch, gbs_partial* partials_dev, const int64_t* out_idx_host, void* stream);

/* Combine partials: pattern b's partials are partials_dev[part_lo_host[b] .. part_hi_host[b]),
 * summed in that order with compensation (ranges may be anywhere in partials_dev and may differ in
 * length). Pattern b is the mode list modes_host[offsets_host[b] .. offsets_host[b+1]) as in
 * gbs_prob_batch: its length is the photon number n, and the library derives prod_j s_j! from its
 * repeated modes (Eq. ProOri). haf_out_dev[b] = sum (1 for n = 0, 0 for odd n);
 * prob_out_dev[b] = prefactor |haf|^2 / prod_j s_j! (prefactor from `state`). Either output may be
 * NULL; prob_out_dev needs a state, and then modes must lie in [0, m) (GBS_ERANGE otherwise).
 * modes_host may be NULL when every pattern is empty. Nothing is enqueued on a validation failure. */
int gbs_finalize(gbs_ctx* ctx, const gbs_state* state, const gbs_partial* partials_dev,
                 const int64_t* part_lo_host, const int64_t* part_hi_host, const int32_t* modes_host,
                 const int64_t* offsets_host, int64_t batch, double* prob_out_dev, gbs_c128* haf_out_dev,
                 void* stream);

/* ------------------------------------------- the whole output space (App. D, App. I) */

#define GBS_SWEEP_NMAX 32

/* Number of output patterns of n photons in m modes: C(m + n - 1, n) mode multisets with
 * collisions = 1 (every configuration s with |s| = n), C(m, n) mode sets with collisions = 0.
 * -1 if n is outside [0, GBS_SWEEP_NMAX], m <= 0, or the count exceeds 2^31 - 1. */
int64_t gbs_sweep_count(int32_t m, int32_t n, int32_t collisions);

/* Probabilities (Eq. ProOri) and hafnians of every output pattern of n photons against `state`, in
 * the lexicographic order of the sorted mode lists (the order of Python's
 * itertools.combinations_with_replacement(range(m), n), or combinations with collisions = 0):
 * prob_out_dev[i] = |Haf(B_x)|^2 / (prod_j s_j! prod_i cosh r_i), haf_out_dev[i] = Haf(B_x), either
 * nullable (not both), gbs_sweep_count(m, n, collisions) entries each.
 * The hafnians share their work across patterns: the hafnians of all patterns of every even size
 * l < n are kept (the stored sub-hafnians of the paper's exponential-space variant, App. D), and a
 * size-l hafnian is the matching sum expanded along its lowest position (Eq. HafMatch): l - 1
 * products of B entries with stored size-(l - 2) hafnians. Work ~ n x count products; workspace
 * 16 bytes x (the count at size n - 2) x 2. Odd n gives zeros, n = 0 the vacuum (Haf = 1).
 * Errors: GBS_ERANGE if gbs_sweep_count is -1; as gbs_prob_batch otherwise. */
int gbs_prob_sweep(gbs_ctx* ctx, const gbs_state* state, int32_t n, int32_t collisions, double* prob_out_dev,
                   gbs_c128* haf_out_dev, void* stream);

/* Brute-force sampling over a list of probabilities (App. I): [0, 1) is cut into one interval per
 * entry, of length prob_dev[i] / total (total = their sum, computed by a fixed-order prefix sum in
 * the workspace and written to total_out_dev if it is not NULL), and index_out_dev[s] receives the
 * entry whose interval holds uniforms_dev[s] (caller's uniforms in [0, 1), so draws are
 * reproducible). With the probabilities of gbs_prob_sweep this samples output patterns exactly from
 * p_n(s) / sum p_n. count <= 2^31 - 1; nsamples may be 0 (then only the total is computed). */
int gbs_sweep_sample(gbs_ctx* ctx, const double* prob_dev, int64_t count, const double* uniforms_dev,
                     int64_t nsamples, int64_t* index_out_dev, double* total_out_dev, void* stream);

/* ------------------------------------------- marginal probabilities (sequential sampling) */

#define GBS_MARGINAL_KMAX 20   /* longest prefix */
#define GBS_MARGINAL_NMAX 4096 /* largest total photon number */

/* Marginal probabilities of photon-position prefixes, Sec. III C-D (Eq. marginal_definition,
 * Theorem 1), for identical squeezing on every mode. The n photons' positions x = (x_1..x_n) in
 * [m]^n are distributed as q_n(x) = |Haf(W_x)|^2 / f_n with W = U U^t (the state's U; its squeezing
 * values do not enter) and f_n = n! C((m+n)/2 - 1, n/2); the marginal of a prefix is q_n summed over
 * all completions:
 *   q_out_dev[b] = q_n(x_1..x_k),  x = modes_host[offsets_host[b] .. offsets_host[b+1]),  k <= n.
 * Evaluated with Theorem 1 (B ranging over mu-subsets of X_k minus a'), regrouped: the hafnians of
 * W over all 2^(k-1) even-size position subsets of the prefix are built size by size from the
 * matching sum expanded along the lowest position (Eq. HafMatch; O(k 2^k) work), then for
 * every set A of positions the sums over the 2j-subsets a of the other positions of
 * Haf(W_a) Haf(W_{rest}) are combined with the weights F and Per(S_{A,B}) (A, B with equal mode
 * multisets) on the device; about 3^k / 2 products per prefix.
 * Repeated modes (collisions) are allowed. n must be even (q is defined for even n only);
 * 0 <= k <= min(n, GBS_MARGINAL_KMAX), modes in [0, m). k = 0 gives 1, k = 1 gives 1/m.
 * Results are deterministic. Work memory: 16 bytes x 2^k per prefix plus the hafnian plan, in the
 * context's workspace. Errors as for gbs_prob_batch; nothing is enqueued on a validation failure. */
int gbs_marginal_batch(gbs_ctx* ctx, const gbs_state* state, int32_t n, const int32_t* modes_host,
                       const int64_t* offsets_host, int64_t batch, double* q_out_dev, void* stream);

/* ------------------------------------------- sampling (Sec. III A-C, Alg. 1) */

/* Step 1: P_n = C((m+n)/2 - 1, n/2) tanh^n r / cosh^m r for n = 0..nmax (0 for odd n), identical
 * squeezing r >= 0 on m modes (Eq. Eqdistribution); host only. The caller truncates and
 * renormalises as the paper does. Returns GBS_EINVAL for m <= 0, nmax < 0, r < 0 or NULL. */
int gbs_photon_number_pmf(int32_t m, double r, int32_t nmax, double* pmf_host);

/* One step of the chain rule (Eq. ConPro): for each prefix b (k - 1 < n positions) the weights
 * w[b][l] = q_n(x_1..x_{k-1}, l), l in [0, m), are the marginals of gbs_marginal_batch, and
 * next_dev[b] = the smallest l with w[b][0] + .. + w[b][l] >= uniforms_dev[b] * sum_l w[b][l]
 * (inverse CDF; uniforms in [0, 1) are the caller's random numbers, so a draw is reproducible).
 * weights_dev (nullable, batch x m doubles) receives the weights. Limits and errors as for
 * gbs_marginal_batch with k = prefix length + 1; batch x m <= 2^24. */
int gbs_sample_step(gbs_ctx* ctx, const gbs_state* state, int32_t n, const int32_t* modes_host,
                    const int64_t* offsets_host, int64_t batch, const double* uniforms_dev,
                    double* weights_dev, int32_t* next_dev, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GBS_H_ */
