/*
 * rfr.h -- C ABI of the MI355X Real-Factors-Recombination (RFR) library.
 *
 * The library factors an integer polynomial p(x) into irreducible
 * factors over Z by the method of Iravanian, "Integer Polynomial Factorization
 * by Recombination of Real Factors" (arXiv 2410.15880):
 *
 *   1. the real linear and quadratic factors of p (Section 2, Eq 1) give the
 *      elements t_i = u_i (real roots) and z_j + conj(z_j) (conjugate pairs);
 *   2. each element becomes a 64-bit weight w_i = floor(frac(a_d t_i) 2^64)
 *      (Section 3.3, Eq 18, with the roots of the monic transform, Section 2);
 *   3. the subset-sum search over the weights runs on the GPU as a
 *      Horowitz-Sahni meet in the middle (Section 3.3, EXPAND + FIND): both
 *      halves are enumerated, radix-sorted and band-joined;
 *   4. every candidate pattern is confirmed by exact trial division on the
 *      host (Section 2, Algorithm FACTOR), and the irreducible factors are the
 *      atoms of the divisors found.
 * The method needs a square-free p (Section 2); a p with repeated factors is
 * first split into square-free parts by Yun's algorithm and each part is
 * factored in turn (rfr_squarefree exposes that decomposition).
 *
 * Conventions for every entry point:
 *   - Polynomials are int64 coefficient arrays in ascending order:
 *     coeffs[i] multiplies x^i, coeffs[degree] != 0.
 *   - The return value is the status; nothing is thrown across the ABI.
 *     rfr_last_error() gives a thread-local message for the last failure.
 *   - Input arrays are borrowed for the duration of the call only.
 *   - Results (rfr_result) are owned by the caller after a successful call and
 *     must be released with rfr_result_free().
 *   - A context is bound to one HIP device and is not thread-safe: use one
 *     context per host thread (the serving calls rfr_submit/rfr_poll are the
 *     exception: they may be called from any thread).
 */
#ifndef RFR_H
#define RFR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rfr_status {
    RFR_OK = 0,
    RFR_EINVAL = -1,       /* bad argument: degree < 1, zero leading coeff, NULL */
    RFR_ENOTSQFREE = -2,   /* p has a repeated factor: returned by the host-stage calls
                              (rfr_weights, rfr_prepare_batch); the factoring calls
                              decompose such p instead (rfr_squarefree) */
    RFR_ENOMEM = -3,       /* device or host allocation failed / over the memory budget */
    RFR_EPRECISION = -4,   /* roots could not be separated or the accept window is too wide */
    RFR_EOVERFLOW = -5,    /* a coefficient or element count exceeds the supported range */
    RFR_ECANDIDATES = -6,  /* more candidate patterns than the candidate capacity */
    RFR_EDEVICE = -7,      /* a HIP runtime call failed */
    RFR_EBUSY = -8         /* serving: the request is not finished yet */
} rfr_status;

/* Largest supported degree and element count (elements = real roots + pairs). */
#define RFR_MAX_DEGREE 256
#define RFR_MAX_ELEMENTS 128

typedef struct rfr_ctx rfr_ctx;

/*
 * Factorisation result: p = content * prod_k factor_k.
 * Factor k has degree degrees[k] and coefficients
 * coeffs[off_k .. off_k + degrees[k]] (ascending), off_k = sum_{i<k}(degrees[i]+1).
 * Factors are primitive, irreducible over Z, with positive leading
 * coefficient, sorted by (degree, coefficient tuple in ascending-power order).
 * A factor x is reported when p(0) = 0.  A factor of multiplicity m appears
 * m times (only when p is not square-free; the counters then sum over its
 * square-free parts and t_lo/t_hi are those of the part with most elements).
 */
typedef struct rfr_result {
    int64_t content;           /* signed integer content of p */
    int32_t nfactors;
    int32_t n_elements;        /* n = r + c (Section 2) */
    int32_t n_real;            /* r: real roots */
    int32_t trace_folded;      /* 1 if the search of the first trace overflowed the
                                  candidate capacity and was redone with the second
                                  trace folded into the weights (Section 2: the sum of
                                  squares of a factor's monic-transform roots is an
                                  integer too), which rejects inside the search every
                                  pattern whose second trace is not an integer */
    const int32_t *degrees;    /* [nfactors] */
    const int64_t *coeffs;     /* [sum(degrees[k]+1)] */
    uint64_t n_candidates;     /* candidate patterns the search returned */
    uint64_t n_confirmed;      /* candidates that divide p exactly */
    uint64_t t_lo, t_hi;       /* accept window: sum in [2^64 - t_lo, 2^64) U [0, t_hi] */
    double ms_roots;           /* wall time of normalisation, roots (device, or host when the
                                  device roots fail a check), single-element factors, weights
                                  and window */
    double ms_search;          /* wall time of the recombination search (device) and the
                                  candidate copy back */
    double ms_confirm;         /* wall time on the host: confirmation and atoms */
} rfr_result;

/* ------------------------------------------------------------------ context */

/* Create a context on HIP device `device`.  mem_budget_bytes caps the device
 * memory the context may hold for search tables (0 = 90% of free memory).
 * Returns RFR_EDEVICE if the device cannot be opened. */
rfr_status rfr_create(int device, size_t mem_budget_bytes, rfr_ctx **out);

/* Release a context and all device memory it holds (NULL is ignored). */
void rfr_destroy(rfr_ctx *ctx);

/* Search design of the plain and served paths: 0 (default) per size class as
 * the tuning table says (rfr_autotune times both), 1 always the Horowitz-Sahni
 * pipeline (Section 3.3, Algorithm C), 2 the query design (Section 3.5,
 * Algorithm E) wherever it applies (halves of at most 2^26 keys).  Results
 * are the same; only speed and workspace change.  Batches use Algorithm C. */
rfr_status rfr_set_design(rfr_ctx *ctx, int design);

/* Capacity of candidate patterns per polynomial (default 65536). */
rfr_status rfr_set_candidate_cap(rfr_ctx *ctx, uint64_t cap);

/* ------------------------------------------------------------------ plain */

/* Factor one polynomial (Algorithm FACTOR, Section 2).
 * coeffs: host array [degree + 1]; degree in [1, RFR_MAX_DEGREE].
 * The search runs on the context's device; the call blocks until done.
 * A p that is not square-free is factored through its square-free parts
 * (rfr_squarefree), each by the square-free path.
 * Errors: RFR_EINVAL, RFR_EPRECISION, RFR_EOVERFLOW, RFR_ECANDIDATES,
 * RFR_ENOMEM, RFR_EDEVICE. */
rfr_status rfr_factor(rfr_ctx *ctx, const int64_t *coeffs, int degree, rfr_result **out);

/* ------------------------------------------------------------------ batched */

/* Factor `count` polynomials in one device pass.
 * coeffs: all polynomials concatenated, polynomial i occupying
 *         coeffs[off_i .. off_i + degrees[i]], off_i = sum_{k<i}(degrees[k]+1).
 * out[i] receives a result (or NULL on failure) and status[i] its status.
 * The roots of all polynomials are found in one device launch (a workgroup
 * per polynomial); elements, weights and window on a host thread pool.  The
 * searches are split by size: those whose halves hold at most 2^11 keys run
 * in one persistent kernel (a workgroup per search, taken largest first from
 * an atomic queue, everything in LDS); mid-size ones run through the staged
 * pipeline with one launch per stage for all of them; searches with a half of
 * 2^23 keys or more (each fills the GPU) are queued one after another.  The
 * device pass of the small and mid searches is captured once per batch shape
 * into a HIP graph and replayed.  Confirmation runs on the thread pool.
 * Returns RFR_OK if the batch ran, even when some entries failed (see
 * status[]). */
rfr_status rfr_factor_batch(rfr_ctx *ctx, int count, const int64_t *coeffs,
                            const int32_t *degrees, rfr_result **out, rfr_status *status);

/* ------------------------------------------------------------------ served */

/* Start the serving loop on this context: up to `max_active` requests share
 * the device at once, each admitted when its search tables fit the memory
 * budget.  `host_threads` workers find roots and weights and confirm
 * candidates; with max_active > 1, searches with a half of 2^23 keys or more
 * run one at a time on slot 0 (on a stream of their own, driven by two
 * threads of the library) while the workers go on with other requests, whose
 * device work runs on a second stream.  Requests are factored exactly as by
 * rfr_factor.  Errors: RFR_EINVAL (max_active outside [1, 64], host_threads
 * outside [1, 256]), RFR_EBUSY (already serving), RFR_EDEVICE, RFR_ENOMEM. */
rfr_status rfr_serve_start(rfr_ctx *ctx, int max_active, int host_threads);

/* Queue a request; returns a ticket.  Thread-safe.  The coefficient array is
 * copied before the call returns. */
rfr_status rfr_submit(rfr_ctx *ctx, const int64_t *coeffs, int degree, uint64_t *ticket);

/* Collect a finished request: RFR_EBUSY while it runs, otherwise its status,
 * with *out set on RFR_OK.  A ticket can be collected once.  Thread-safe.
 * latency_ms (may be NULL) receives submit-to-completion wall time. */
rfr_status rfr_poll(rfr_ctx *ctx, uint64_t ticket, rfr_result **out, double *latency_ms);

/* Stop the serving loop after draining queued requests. */
rfr_status rfr_serve_stop(rfr_ctx *ctx);

/* ------------------------------------------------------------------ profiling */

/* Device time per search stage, accumulated from HIP events recorded on the
 * stream each stage runs on, while profiling is enabled on the context.
 * stage_ms: [0] K0 count, [1] scans, [2] K1 enumerate+partition,
 * [3] K2 tile sort, [4] K3 sort+join, [5] K4+K5 pattern recovery.
 * keys: sum of N_A + N_B over the profiled searches.  In a batch, one launch
 * of each stage serves all searches of the batch, so stage_ms is per launch
 * sequence, not per search. */
typedef struct rfr_profile_t {
    uint64_t searches;
    uint64_t keys;
    double stage_ms[6];
    uint64_t launches;         /* batched pipeline launches profiled (one per stage per batch) */
    uint64_t graph_captures;   /* batch HIP graphs captured / replayed on this context */
    uint64_t graph_replays;
} rfr_profile_t;

/* enable != 0 starts (and zeroes) accumulation, 0 stops it. */
rfr_status rfr_profile(rfr_ctx *ctx, int enable);
rfr_status rfr_profile_read(rfr_ctx *ctx, rfr_profile_t *out);

/* ------------------------------------------------------------------ tuning */

/* Time the device search for every radix split candidate of each size class
 * lg in [lg_lo, lg_hi] (halves of 2^lg keys; 8 <= lg_lo <= lg_hi <= 32; lg = 32
 * needs the tables of an n = 65 search, about 80 GB): the sub-bucket size
 * (2^9 or 2^10 keys) and the level-1 digit bits.  Installs
 * the fastest split per class for this process and, if path_out is not NULL,
 * writes the table ("lg b1 sub_log ms" lines).  Not concurrent with other
 * calls.  Contexts load RFR_TUNING or the package's tuning/mi355x.txt at
 * creation. */
rfr_status rfr_autotune(rfr_ctx *ctx, int lg_lo, int lg_hi, const char *path_out);

/* Install a table written by rfr_autotune ("lg b1 sub_log ms" lines; a line
 * "lg -1 -1 0" returns class lg to the fixed rule).  Affects the workspace
 * size and speed of later searches, never their results; not concurrent with
 * searches. */
rfr_status rfr_load_tuning(const char *path);

/* ------------------------------------------------------------------ square-free parts */

/* Square-free decomposition (Section 2: Yun's algorithm, the step that lets
 * the method take any p): p = content * prod_j part_j ^ mult_j with every part
 * primitive, square-free, lc > 0 and pairwise coprime; a power of x is the
 * part x.  Parts are sorted by (mult, degree, coefficients).  Host only.
 * parts_out receives the parts' coefficients back to back (ascending;
 * capacity 2 * degree + 2 suffices), degrees_out and mult_out one entry per
 * part (capacity degree + 1), *nparts the number of parts.  A square-free p
 * gives its primitive part (and x) with multiplicity 1.  Errors: RFR_EINVAL,
 * RFR_EOVERFLOW (a gcd or quotient leaves int64). */
rfr_status rfr_squarefree(const int64_t *coeffs, int degree, int64_t *content, int64_t *parts_out,
                          int32_t *degrees_out, int32_t *mult_out, int *nparts);

/* ------------------------------------------------------------------ results */

void rfr_result_free(rfr_result *res);

/* Flatten `count` results for callers that convert many at once (a batch):
 * content[i] and nfactors[i] per result, the degrees of all factors result
 * after result into degrees[0..), their coefficients (ascending, factor after
 * factor) into coeffs[0..).  A null res[i] counts as content 0 with no factors.
 * The totals are returned in *ndeg and *ncoef; with degrees or coeffs NULL
 * nothing else is written (a size query).  RFR_EINVAL if deg_cap or coef_cap
 * is below the totals (nothing written then).  The results stay owned by the
 * caller. */
rfr_status rfr_results_pack(rfr_result *const *res, int count, int64_t *content, int32_t *nfactors,
                            int32_t *degrees, size_t deg_cap, int64_t *coeffs, size_t coef_cap, size_t *ndeg,
                            size_t *ncoef);
/* rfr_result_free on res[0..count) (null entries are skipped). */
void rfr_results_free(rfr_result *const *res, int count);
const char *rfr_strerror(rfr_status st);
const char *rfr_last_error(void);

/* ------------------------------------------------------------------ host stages */

/* Elements, weights and window of p (Section 2 and Section 3.3, Eq 18-19):
 * w_out: host array of at least `degree` entries, receives n weights in
 * canonical element order (real roots ascending, then conjugate pairs by
 * (Re, Im)); n_out, n_real_out, t_lo, t_hi receive n, r and the accept
 * window.  Runs on the host only.  RFR_ENOTSQFREE for a p with a repeated
 * factor (its elements are not defined; see rfr_squarefree). */
rfr_status rfr_weights(const int64_t *coeffs, int degree, uint64_t *w_out, int32_t *n_out,
                       int32_t *n_real_out, uint64_t *t_lo, uint64_t *t_hi);

/* The host stages of rfr_factor_batch for `count` polynomials (same packing
 * as rfr_factor_batch): normalisation on the host, the roots of every
 * polynomial of degree >= 2 on the device (one workgroup per polynomial:
 * FP64 Aberth, double-double Newton polish, inclusion radii; Section 2, Eq 1),
 * then the disc checks, elements, weights and window (Section 3.3, Eq 18-19)
 * on the host, which finds the roots itself for a polynomial whose device
 * roots fail a check.  Per polynomial i: w_out[off_i .. off_i + n_i) with
 * off_i = sum of degrees[j] for j < i (room for degree weights each), n_out,
 * t_lo, t_hi, device_roots_out (1 if the device roots were used) and
 * status[i].  Returns RFR_OK unless the arguments or the device fail. */
rfr_status rfr_prepare_batch(rfr_ctx *ctx, int count, const int64_t *coeffs, const int32_t *degrees,
                             uint64_t *w_out, int32_t *n_out, uint64_t *t_lo, uint64_t *t_hi,
                             int32_t *device_roots_out, rfr_status *status);

/* ------------------------------------------------------------------ kernel level */

/* Device workspace for rfr_recombine_dev to search n elements in one pass
 * (for n = 70, whose half A is always streamed: in two chunks). */
size_t rfr_recombine_workspace_bytes(int n);

/* Smallest workspace rfr_recombine_dev accepts for n elements.  Between this
 * and rfr_recombine_workspace_bytes(n) the search streams half A in chunks:
 * half B' is built and sorted once and stays resident, and half A is
 * enumerated, sorted and joined 2^c times with its top c weights fixed per
 * chunk (c the smallest that fits, at most 8). */
size_t rfr_recombine_min_workspace_bytes(int n);

/*
 * The recombination search (Section 3.3, Algorithm C with a FIND that reports
 * every pair): all patterns s in [1, 2^(n-1)) over the first n-1 weights whose
 * sum mod 2^64 lies in [2^64 - t_lo, 2^64) U [0, t_hi].
 *   w_host     host array of n weights (borrowed for the call)
 *   workspace  device buffer of ws_bytes >= rfr_recombine_min_workspace_bytes(n)
 *              (less than rfr_recombine_workspace_bytes(n) streams half A)
 *   hip_stream hipStream_t the work is queued on (NULL = default stream)
 *   cand_dev   device array of 2*cap uint64: pattern k is split as
 *              cand_dev[2k] = bits of elements [0, n_a) and
 *              cand_dev[2k+1] = bits of elements [n_a, n-1) shifted down,
 *              with n_a = ceil((n-1)/2)
 *   count_dev  device uint64: number of patterns found; UINT64_MAX if the
 *              candidate capacity overflowed (then cand_dev is partial)
 * The call only enqueues work; read count_dev after synchronising the stream.
 * Requires 2 <= n <= 70 (from n = 70 on half A, 35 weights, is always
 * streamed) and t_lo + t_hi < 2^32; else RFR_EINVAL. */
rfr_status rfr_recombine_dev(const uint64_t *w_host, int n, uint64_t t_lo, uint64_t t_hi,
                             void *workspace, size_t ws_bytes, void *hip_stream,
                             uint64_t *cand_dev, uint64_t cap, uint64_t *count_dev);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the search
 * of rfr_recombine_dev with the same arguments and results, minus the
 * workspace, which is a fixed device array of
 * rfr_recombine_noalloc_scratch_bytes() = 64 MiB inside the library (one per
 * GPU, allocated with the library's code when it is first used on that GPU
 * and held until the process ends).  The call allocates no device or host
 * memory.  It searches up to n = 46 elements (larger n returns RFR_ENOMEM;
 * from n = 45 on, half A is streamed in chunks as in rfr_recombine_dev with a
 * small workspace).  hip_stream must belong to the current device.  All calls
 * on one GPU share its scratch array: calls whose work overlaps on that GPU
 * (other host threads, other streams) race and give wrong results; serialise
 * them, e.g. on one stream.  The kernels clear every counter they use, so a
 * call needs nothing cleared by the caller.
 */
rfr_status rfr_recombine_dev_noalloc(const uint64_t *w_host, int n, uint64_t t_lo, uint64_t t_hi,
                                     void *hip_stream, uint64_t *cand_dev, uint64_t cap, uint64_t *count_dev);

/* Size of the fixed device scratch of rfr_recombine_dev_noalloc. */
size_t rfr_recombine_noalloc_scratch_bytes(void);

/* Device workspace for rfr_recombine_e_dev over n elements (0 if n is out of
 * its range, 3 <= n <= 53). */
size_t rfr_recombine_e_workspace_bytes(int n);

/*
 * The same search by the paper's Algorithm E (Section 3.5: SPLAT, QUERY,
 * RECOMBINE_E; Section 4: the table stays on the device, only candidates
 * leave it): half B' (elements [n_a, n-1), negated) is expanded and sorted,
 * then laid out as the splat table (2 N_B cells, each value at or after its
 * estimated index, in ascending order); half A (elements [0, n_a)) is never
 * stored: each of its 2^n_a sums is generated and queried for every table
 * value inside the window.  Same arguments, outputs and window rules as
 * rfr_recombine_dev; ws_bytes >= rfr_recombine_e_workspace_bytes(n), about
 * 41 bytes per B' sum.  *count_dev = UINT64_MAX - 1 (not a valid count) when
 * B''s sums were too clustered for the expansion's sort: the search did not
 * run; use rfr_recombine_dev.  The call only enqueues work.
 */
rfr_status rfr_recombine_e_dev(const uint64_t *w_host, int n, uint64_t t_lo, uint64_t t_hi,
                               void *workspace, size_t ws_bytes, void *hip_stream,
                               uint64_t *cand_dev, uint64_t cap, uint64_t *count_dev);

/* Device workspace needed by rfr_expand_dev for m weights. */
size_t rfr_expand_workspace_bytes(int m);

/*
 * EXPAND (Section 3.3): the 2^m subset sums of m weights (negated first when
 * `negate` is nonzero), sorted ascending, written to sorted_dev[2^m].
 * Same kernels as the search (enumerate, partition, tile sort, final sort in
 * LDS).  Requires 1 <= m <= 30 (else RFR_EINVAL).  Synchronises hip_stream
 * before returning: the final sort holds at most 2048 keys sharing their top
 * partition bits, and sums more clustered than that (many equal sums, such as
 * from zero or repeated weights) return RFR_EOVERFLOW with sorted_dev only
 * partly written.
 */
rfr_status rfr_expand_dev(const uint64_t *w_host, int m, int negate, void *workspace,
                          size_t ws_bytes, void *hip_stream, uint64_t *sorted_dev);

#ifdef __cplusplus
}
#endif
#endif /* RFR_H */
