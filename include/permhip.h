/* permhip.h -- C ABI of the MI355X (gfx950) permanent library.
 *
 * What is computed.  The permanent of an n x n complex matrix,
 *   Per(A) = sum over permutations s of prod_i a_{i, s(i)},
 * the quantity whose modulus squared gives the boson-sampling output
 * probability of the paper's main-text Eq. (1).  Two exact formulas are
 * offered, both from the Supplementary section "Parallelization and
 * Optimization":
 *   PH_GLYNN  Eq. (S2) (BB/FG):  Per(A) = 2^-(n-1) sum_delta (prod_k delta_k)
 *             prod_i sum_j delta_j a_ij,  delta_0 = +1, delta_k = +-1;
 *   PH_RYSER  Eq. (S1):          Per(A) = (-1)^n sum_S (-1)^|S| prod_i sum_{j in S} a_ij.
 * Both are evaluated in Gray-code order (one column changes per term) in
 * binary64, with the outer sum accumulated either in compensated double-double
 * (PH_ACC_DD, default) or in plain binary64 (PH_ACC_PLAIN).  The Supplementary
 * "Analysis of the Precision Issue" explains why Ryser loses accuracy on some
 * inputs; PH_GLYNN is the default.
 *
 * Data layout.  complex128 = two binary64 {re, im}, interleaved (the layout of
 * C99 double _Complex, std::complex<double> and torch.complex128).  Matrices
 * are row-major: entry (i, j) of a matrix at A with row stride lda is
 * A[i * lda + j].
 *
 * Memory and streams.  Unless a parameter says "host", pointers are DEVICE
 * pointers on the current HIP device.  `stream` is a hipStream_t passed as
 * void* (NULL = the null stream).  Calls enqueue work on the stream and return
 * without synchronising; results are valid once the stream has reached them.
 * The caller owns every buffer it passes; the library keeps no reference to
 * caller memory after a call returns (plans excepted, see below).  The
 * library owns its workspace (per device and stream, grown on demand with
 * hipMalloc and kept until the process ends).
 *
 * Errors.  Every entry point returns PH_OK (0) or a negative PH_E* code and
 * never aborts.  Argument errors are detected on the host before anything is
 * enqueued.  A kernel fault is asynchronous and surfaces at the caller's next
 * synchronisation.  ph_last_error() describes the last failure of the calling
 * thread.
 *
 * Conventions.  n = 0 gives Per = 1 (empty product); n = 1 gives a_00.
 * NaN and Inf propagate and are not checked.
 */
#ifndef PERMHIP_H
#define PERMHIP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  double re, im;
} ph_c128;

enum { PH_GLYNN = 0, PH_RYSER = 1 };
enum { PH_ACC_DD = 0, PH_ACC_PLAIN = 1 };
#define PH_FLAG_UNGROUPED 1u
#define PH_FLAG_UNSORTED 2u
#define PH_FLAG_DU_FULL 4u

/* Options; pass NULL for the defaults (Glynn, double-double, tuned sizes; the
 * environment variable PERMHIP_ACCUM=plain or =dd sets the default
 * accumulation, any other value makes the call fail with PH_EINVAL).
 *   algo        PH_GLYNN or PH_RYSER
 *   accum       PH_ACC_DD or PH_ACC_PLAIN
 *   chunk_log2  log2 of the Gray-code chunk one lane walks between re-seeds
 *               of its row sums; 0 = library choice, < 0 is PH_EINVAL.
 *               Values above PH_CHUNK_LOG2_MAX, or outside the range the
 *               kernel supports for n (at least the few steps of one
 *               unrolled block, at most the whole term range), are clamped
 *               (ph_perm_chunk_log2 reports the value used).
 *   waves       wavefronts per SIMD to launch (1..8); 0 = library choice
 *   flags       0, or PH_FLAG_UNGROUPED (ph_boson_probs only: one full sweep
 *               per pattern instead of the multiplicity-grouped sweeps), or
 *               PH_FLAG_UNSORTED (ph_boson_sample only: out_modes in the
 *               order the photons were placed, r_1..r_n), or PH_FLAG_DU_FULL
 *               (ph_boson_probs_grad only: the gradient with respect to all
 *               of U, see there); flags combine with | */
typedef struct {
  int32_t algo;
  int32_t accum;
  int32_t chunk_log2;
  int32_t waves;
  uint32_t flags;
} ph_opts;

enum {
  PH_OK = 0,
  PH_EINVAL = -1,       /* bad pointer, size, stride or option */
  PH_ERANGE = -2,       /* n above the supported maximum */
  PH_ENOMEM = -3,       /* device allocation failed */
  PH_EHIP = -4,         /* HIP runtime error (message in ph_last_error) */
  PH_EUNSUPPORTED = -5  /* no usable gfx950 device */
};

#define PH_NMAX 52      /* largest n of ph_perm / batched plans */
/* Largest chunk_log2 any call uses: steps inside a chunk are counted in 32-bit
 * integers, and the incremental row sums drift by up to about 2^c roundings
 * between re-seeds, so longer chunks buy nothing. */
#define PH_CHUNK_LOG2_MAX 24
#define PH_NMAX_GRAD 32 /* largest n of ph_perm_grad and the boson layer */

/* Per(A) of one n x n matrix into *out (one complex128, device).
 * A: device, row stride lda >= n (elements).  0 <= n <= PH_NMAX.
 * The 2^(n-1) (Glynn) or 2^n (Ryser) terms are cut into contiguous Gray-code
 * chunks, one per GPU lane at a time (one per pair of lanes from n = 49, and
 * for n = 12..21 when there are at most 2^15 chunks, too few to give every
 * SIMD a wavefront); see the formulas above. */
int ph_perm(const ph_c128* A, int32_t n, int64_t lda, ph_c128* out, const ph_opts* opt, void* stream);

/* ph_perm_noalloc: ph_perm without any device allocation, for callers that
 * cannot allocate: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, errors and result bits as
 * ph_perm.  ph_perm keeps its per-wave partial sums in workspace it grows with
 * hipMalloc; this call keeps them in a fixed static device array of the
 * library (262,144 bytes per device, held until the process ends; room for
 * 8192 partial sums, every launch shape of a 256-CU MI355X), and fails with
 * PH_ERANGE where a device would need more.  It allocates nothing, on the
 * host's side or the device's, from its first call on.  All calls on one
 * device share that array: calls that overlap on a device (concurrent
 * streams) race and must be ordered by the caller. */
int ph_perm_noalloc(const ph_c128* A, int32_t n, int64_t lda, ph_c128* out, const ph_opts* opt, void* stream);

/* ph_perm_ryser_paired: *out (device, one complex128) = Per(A) by Ryser's
 * formula, Eq. (S1), in the load-balanced order of Supplementary
 * Algorithm S3: the loop runs over the 2^(n-1) subsets S of the first n - 1
 * columns (in Gray order here) and takes with each S the term of its
 * complement among all n columns, so every subset is summed once.  A as
 * ph_perm (device, lda >= n), 0 <= n <= 32.  opt: accum and chunk_log2 are
 * used (a chunk is 2^chunk_log2 loop indices, at least 16 from n = 19, where
 * two lanes share an index and step in blocks of 16); algo and waves are checked as
 * for ph_perm but do not change the computation.
 * Errors: PH_EINVAL (NULL pointer, lda < n, n < 0, bad options), PH_ERANGE
 * (n > 32), PH_EHIP.  Asynchronous on `stream`; deterministic. */
int ph_perm_ryser_paired(const ph_c128* A, int32_t n, int64_t lda, ph_c128* out, const ph_opts* opt, void* stream);

/* One share of a permanent's Gray-code sum, for sums split across devices or
 * run as resumable segments.  The parallel listings of the Supplementary
 * (Algorithms S1 and S2) give each process a contiguous range of the term
 * index k and reduce the partial sums at the end; these three calls are that
 * split.
 *
 * ph_perm_chunk_log2: *out (host) receives c, the log2 chunk length that
 * ph_perm and ph_perm_partial use for this n and these options.
 *
 * ph_perm_partial: the sum over terms k in [k_begin, k_end) of Eq. (S2)
 * (2^(n-1) terms in all) or Eq. (S1) (2^n), each term with its sign, before
 * the formula's scale (no 2^-(n-1), no (-1)^n).  Term k is the summand of
 * the Gray word w = k XOR (k >> 1): BB/FG takes delta_0 = +1 and
 * delta_{b+1} = -1 iff bit b of w is set; Ryser puts column b in S iff bit b
 * of w is set.  k_begin and k_end are multiples of 2^c, with
 * k_begin <= k_end <= the term count; an empty range gives 0.
 * partial (device) receives 4 doubles {re_hi, re_lo, im_hi, im_lo}:
 * a double-double per component (PH_ACC_PLAIN: the lo halves are 0).  A, n,
 * lda as ph_perm, 1 <= n <= PH_NMAX.  The result is deterministic for the
 * same inputs, range, options and device; the split of a range into shares
 * changes the rounding of the total, not its exactness bound.
 *
 * ph_perm_combine: out (device, one complex128) = the scaled sum of `count`
 * partials (device, 4 doubles each) added in a fixed order (contiguous
 * index-ordered slices, then a fixed tree over the slices), with the same
 * n and options (algo, accum) as the calls that made them.  Partials covering
 * the whole range [0, term count) give Per(A). */
int ph_perm_chunk_log2(int32_t n, const ph_opts* opt, int32_t* out);
int ph_perm_partial(const ph_c128* A, int32_t n, int64_t lda, uint64_t k_begin, uint64_t k_end, double* partial,
                    const ph_opts* opt, void* stream);
int ph_perm_combine(const double* partials, int64_t count, int32_t n, ph_c128* out, const ph_opts* opt,
                    void* stream);

/* Batched permanents in one launch sequence.  Matrix b is n_host[b] x
 * n_host[b], row-major and contiguous (lda = n), starting at
 * A_packed + offsets_host[b] (elements); offsets_host = NULL means the
 * matrices are packed back to back in order.  out[b] receives Per of matrix
 * b.  Host arrays n_host and offsets_host have `batch` entries.  Convenience
 * wrapper around the plans below: the library keeps the plans of the last
 * few (device, stream, options, sizes) combinations, so a repeated call costs
 * one graph launch; the first call for a new combination plans (and may time
 * chunk-length candidates) before it returns.  A plan evicted from this cache
 * is freed after its stream has finished with it. */
int ph_perm_batched(const ph_c128* A_packed, const int64_t* offsets_host, const int32_t* n_host, int64_t batch,
                    ph_c128* out, const ph_opts* opt, void* stream);

/* Plans for repeated batched calls with the same sizes.  ph_plan_create
 * sorts the matrices by size (largest first), splits each into work items of
 * 64-chunk groups, allocates the plan's workspace, picks chunk lengths (timing
 * candidates on `stream` when opt->chunk_log2 == 0 and no tuned value is
 * cached for this device), and records prep, sweep and finalize kernels in one
 * hipGraph.  ph_plan_execute replays the graph with the given input and output
 * (one hipGraphLaunch; the kernel arguments are updated in place when the
 * pointers differ from the last call); matrices of order >= 45 (2^44 terms or
 * more each) are then swept one at a time by the ph_perm kernels.  A plan is bound to the device that
 * was current at creation and may be used from one thread at a time.  Its
 * executions run one after another, also across streams: an execution on a
 * stream other than the previous one's first waits for that one (the plan's
 * counters and partial sums are its own, not per stream). */
int ph_plan_create(const int32_t* n_host, const int64_t* offsets_host, int64_t batch, const ph_opts* opt,
                   void* stream, void** plan);
int ph_plan_execute(void* plan, const ph_c128* A_packed, ph_c128* out, void* stream);
int ph_plan_destroy(void* plan);

/* ph_plan_shape: the sweep shape a plan uses for its matrices of order n --
 * *chunk_log2 (host) the log2 chunk length, *waves (host) the wavefronts per
 * SIMD of that size bucket's sweep (0 = as many as fit).  With
 * opt->chunk_log2 == 0 the plan takes both from the autotuner, which times
 * every (chunk length, waves) pair on a synthetic batch of about 2^27 terms
 * per order (orders of more than 2^27 terms take c = min(12, n - 9) and full
 * occupancy) and remembers the fastest per (library build, device, order,
 * formula, accumulation) for the process, and across processes in the file
 * named by the environment variable PERMHIP_TUNE_CACHE (entries of other
 * builds are ignored).  opt->waves > 0 overrides the tuned waves.
 * PH_EINVAL if the plan holds no matrix of order n. */
int ph_plan_shape(const void* plan, int32_t n, int32_t* chunk_log2, int32_t* waves);

/* Gradient of the permanent.  A holds `batch` contiguous n x n matrices
 * (batch * n * n complex128).  For each matrix the library forms
 *   M_ij = d Per(A) / d a_ij = Per(A with row i and column j removed)
 * by differentiating Eq. (S2) term by term inside one Gray-code sweep, and
 * writes grad_A[b] = g_b * conj(M) elementwise, with g_b = grad_out[b] (the
 * upstream gradient, PyTorch's conjugate-Wirtinger convention); grad_out =
 * NULL means g_b = 1, i.e. grad_A = conj(M).  perm_out (nullable) receives
 * Per(A[b]).  1 <= n <= PH_NMAX_GRAD.  opt->accum selects the accumulation of
 * the sums over terms; opt->algo must be PH_GLYNN. */
int ph_perm_grad(const ph_c128* A, int32_t n, int64_t batch, const ph_c128* grad_out, ph_c128* perm_out,
                 ph_c128* grad_A, const ph_opts* opt, void* stream);

/* Boson-sampling output probabilities, main-text Eq. (1):
 *   Pr[S -> T_p] = |Per(U_{S,T_p})|^2 / (prod_i s_i! prod_j t_j!),
 * U: m x m unitary (device, row stride ldu), indexed [output mode, input mode].
 * in_modes (host, n entries): input mode of each photon (a mode holding s
 * photons appears s times).  patterns (host, n_patterns x n): output mode of
 * each photon of pattern p, likewise with repeats.  U_{S,T} has rows =
 * pattern modes and columns = input modes, both in the given order.
 * probs (device, n_patterns doubles) receives the probabilities.
 * A pattern whose output modes repeat is evaluated through Eq. (S2) grouped by
 * multiplicity: with output mode l holding mu_l photons, the signs of its mu_l
 * copies enter only through their count k_l of -1 entries, so
 *   Per = 2^-(n-1) sum_{k} prod_l C(mu_l, k_l) (-1)^{k_l} prod_i sum_l (mu_l - 2 k_l) u_{l, s_i}
 * (one single-photon mode's sign fixed), i.e. one BB/FG sweep over the
 * single-photon modes per choice of k for the collided ones: prod_l (mu_l + 1)
 * / 2 terms in place of 2^(n-1).  Patterns with fewer than 5 single-photon
 * modes, and every pattern under PH_FLAG_UNGROUPED, take one sweep of
 * 2^(n-1) terms.  The host arrays are copied before the call returns.
 * 1 <= n <= PH_NMAX_GRAD for the gradient entry point, n <= PH_NMAX here. */
int ph_boson_probs(const ph_c128* U, int32_t m, int64_t ldu, const int32_t* in_modes, int32_t n,
                   const int32_t* patterns, int64_t n_patterns, double* probs, const ph_opts* opt, void* stream);

/* Gradient of L = sum_p w_p Pr[S -> T_p] with respect to the columns of U
 * used by the inputs: dU (device, m x n, row stride lddu >= n) receives
 * dL/dU[:, in_modes[k]] for k = 0..n-1 (column k of dU belongs to input
 * photon k; PyTorch's conjugate-Wirtinger convention), accumulated over all
 * patterns and repeated rows in a fixed order.  With PH_FLAG_DU_FULL in
 * opt->flags, dU is instead the m x m gradient with respect to all of U
 * (row stride lddu >= m): column j holds the sum, in increasing k, of the
 * per-photon columns of the photons k with in_modes[k] == j, and the columns
 * of modes without an input photon are 0.  weights (device, n_patterns
 * doubles) or NULL for w_p = 1.  probs (device, nullable) receives the
 * probabilities as a by-product.  dU is overwritten, not accumulated into. */
int ph_boson_probs_grad(const ph_c128* U, int32_t m, int64_t ldu, const int32_t* in_modes, int32_t n,
                        const int32_t* patterns, int64_t n_patterns, const double* weights, double* probs,
                        ph_c128* dU, int64_t lddu, const ph_opts* opt, void* stream);

/* Minors along one row: for each of `batch` contiguous row-major n x (n+1)
 * matrices B (device), minors[b][l] = Per(B without column l), l = 0..n, the
 * derivatives of Per([B; x]) in the entries of an added last row x.  They
 * come from differentiating Eq. (S2) of that (n+1) x (n+1) matrix in x: one
 * Gray-code sweep of B's n rows over its n + 1 columns that adds every term,
 * signed by delta_l, into one sum per column (n >= 12; smaller n go through
 * the gradient sweep of ph_perm_grad).  The sampler below expands along x
 * with them.  0 <= n <= PH_NMAX_GRAD - 1; minors (device, batch x (n+1)
 * complex128); opt->algo must be PH_GLYNN. */
int ph_perm_row_minors(const ph_c128* B, int32_t n, int64_t batch, ph_c128* minors, const ph_opts* opt,
                       void* stream);

/* Boson-sampling outputs, drawn by the chain rule over the output photons.
 * The paper's simulation serves sampling from main-text Eq. (1) but gives no
 * sampler; this is Clifford and Clifford's exact algorithm (2018).  With
 * A = U[:, in_modes] (rows = output modes) and the columns of A taken in the
 * order perms[s] (a permutation of 0..n-1 per sample), photon k = 1..n of
 * sample s goes to output mode r_k with probability proportional to
 *   w_k(i) = |Per(A[(r_1, ..., r_{k-1}, i), columns 1..k])|^2,
 * computed from the minors along the last row (one gradient sweep of k x k
 * matrices per step, for all samples at once); r_k is the first mode whose
 * running sum of weights (in mode order) exceeds uniforms[s][k-1] times their
 * total.  out_modes[s] (device, n int32) receives r sorted ascending (in
 * placement order under PH_FLAG_UNSORTED): for a unitary U and uniformly
 * random perms and uniforms, a draw from Eq. (1).
 *   U (device, m x m, row stride ldu), in_modes (host, n distinct modes),
 *   1 <= n <= PH_NMAX_GRAD; perms (host, nsamples x n int32) and uniforms
 *   (host, nsamples x n doubles in [0, 1)) are checked and copied before the
 *   call returns.  opt->accum selects the sweeps' accumulation; opt->algo must
 *   be PH_GLYNN.  Weights that are all zero or NaN put the photon in mode 0. */
int ph_boson_sample(const ph_c128* U, int32_t m, int64_t ldu, const int32_t* in_modes, int32_t n, int64_t nsamples,
                    const int32_t* perms, const double* uniforms, int32_t* out_modes, const ph_opts* opt,
                    void* stream);

/* Achieved FP64 FMA rate of this device (microbenchmark, the FMA-only
 * reference program of the paper's Supplementary efficiency section): every
 * lane of 8 wavefronts per SIMD runs 8 independent FMA chains for 32 * iters
 * FMAs.  *gflops (host) receives the rate; *sclk_mhz (host, nullable) the
 * shader clock sustained during the run, from the cycle and constant-rate
 * counters of one wavefront.  Synchronises the stream. */
int ph_fp64_peak(int64_t iters, double* gflops, double* sclk_mhz, void* stream);

/* Message for the last failure on the calling thread (never NULL). */
const char* ph_last_error(void);

/* Library version: major * 10000 + minor * 100 + patch. */
int ph_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PERMHIP_H */
