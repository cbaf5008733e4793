/*
 * tor.h -- C ABI of the MI355X Torontonian library (libtor.so).
 *
 * The library evaluates the exact Torontonian of Eq. 2 of Kaposi et al.,
 * "Polynomial speedup in Torontonian calculation by a scalable recursive
 * algorithm":
 *
 *     Tor(O) = sum over Z subset {0..n-1} of (-1)^(n-|Z|) / sqrt(det(I - O)_Z)
 *
 * where (I - O)_Z keeps rows and columns {i, i+n : i in Z}.  The sum is
 * evaluated the recursive way of Sec. 2 (Algorithm 2): the factorisation of a
 * parent subset is reused and a child subset only adds the two rows of its new
 * mode, here in right-looking form (the Schur complement of the included modes
 * is carried down the include/exclude tree, so each child costs one rank-2
 * update), on gfx950 in FP64 with double-double accumulation of the terms.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  * O is complex128, row-major, 2n x 2n, stored as interleaved (re, im)
 *    doubles; ld is the leading dimension in complex elements (ld >= 2n).
 *    Rows and columns are in block order a_1..a_n, a_1^dag..a_n^dag, so mode i
 *    owns rows {i, i+n} (the problem statement of Sec. 1).
 *  * Only the lower triangle of I - O is read, as in Algorithm 1; the upper
 *    triangle is taken as its conjugate transpose.
 *  * Every value read must be finite (else TOR_E_INVAL).  Staging runs on the
 *    GPU: a kernel validates the values, forms I - O, detects the
 *    Gaussian-state block structure and packs the matrix for its kernel.
 *  * I - O must be Hermitian positive definite.  The recursive kernels test
 *    every 2x2 pivot of the factorisation of I - O itself (the all-include
 *    subset): all of them positive is the block form of Sylvester's
 *    criterion, and every principal submatrix of an HPD matrix is HPD
 *    (Cauchy interlacing).  A failed pivot makes the result's status
 *    TOR_E_NOT_PD.  The paper takes |det| in Eq. 2; for HPD input det > 0
 *    and the two agree.
 *  * n = 0 gives Tor = 1 (the empty subset only).
 *  * Unless TOR_INPUT_DEVICE is set, O is a host pointer and is copied to the
 *    device as it is; with TOR_INPUT_DEVICE it is device memory, read in
 *    place by the staging kernel (the caller orders its writes to O before
 *    the call, e.g. by synchronising).  The caller owns its inputs; the
 *    library is done with them when the call returns (for tor_submit as
 *    well).  The context owns all device state.
 *  * A context is internally serialised: calls on one context from several
 *    threads are safe and run one at a time.
 *  * Every function returns TOR_OK (0) or a negative TOR_E_* code; the output
 *    structure is untouched on argument errors.
 */
#ifndef TOR_H
#define TOR_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define TOR_OK 0
#define TOR_PENDING 1          /* tor_poll: the request is still running            */
#define TOR_E_INVAL (-1)       /* null pointer, n < 0, n > max_n, ld < 2n, NaN/Inf  */
#define TOR_E_NOT_PD (-2)      /* I - O is not Hermitian positive definite (a
                                  tested pivot <= 0 or NaN)                         */
#define TOR_E_NUMERIC (-3)     /* a non-finite result with every tested pivot
                                  positive, still so after its failed roots ran
                                  once more (see tor_eval)                          */
#define TOR_E_BUSY (-4)        /* admission refused: serving queue is full          */
#define TOR_E_NOMEM (-5)       /* device or host allocation failed                  */
#define TOR_E_DEVICE (-6)      /* no usable GPU, or a HIP runtime error             */
#define TOR_E_TIMEOUT (-7)     /* a host-side deadline passed                       */
#define TOR_E_UNKNOWN (-8)     /* tor_poll on a ticket this context never issued    */
#define TOR_E_SCRATCH (-9)     /* tor_eval_static: the problem does not fit the
                                  static scratch (TOR_STATIC_SCRATCH_BYTES)          */

/* ---- options ------------------------------------------------------------- */
#define TOR_ACCUM_DD 0   /* double-double accumulation of the signed terms (default) */
#define TOR_ACCUM_FP64 1 /* plain FP64 accumulation, for comparison                   */

#define TOR_INPUT_DEVICE 0x1u    /* O points to device memory                          */
#define TOR_CHECK_HERMITIAN 0x2u /* reject O whose upper triangle is not the conjugate
                                    transpose of its lower triangle (rel. tol 1e-12)   */
#define TOR_FORCE_COMPLEX 0x4u   /* never take the real quadrature path               */
/* Factorise in double-double (about 104-bit significands) instead of FP64:
 * the higher-precision factor that the FP64 floor u R / sqrt(2^n) calls for
 * when the cancellation R = sum|t| / |Tor| is large (Sec. 5 keeps the
 * determinants in extended precision for the same reason).  Each term then
 * carries a relative error of a few units of 2^-104 per factorisation step,
 * and the terms are summed in double-double.  Runs on the real quadrature
 * form only: a matrix without the Gaussian-state block structure is rejected
 * with TOR_E_INVAL; tor_create rejects it together with TOR_FORCE_COMPLEX.
 * The input itself is FP64; I - O and the real form are formed from it in
 * double-double (exactly, or rounded to 2^-106).  About 9x the FP64 time. */
#define TOR_FACTOR_DD 0x8u
/* tor_click_all writes probs, tor_hi and tor_lo to device memory: the
 * caller's device pointers, on the context's device, ordered on its stream */
#define TOR_OUTPUT_DEVICE 0x10u

typedef struct tor_ctx tor_ctx;

typedef struct {
    int device;             /* HIP device ordinal                                     */
    void *stream;           /* hipStream_t to run on (NULL: the library creates one)  */
    void *workspace;        /* caller-owned device buffer, 256-byte aligned, or NULL  */
    size_t workspace_bytes; /* its size; see tor_workspace_size                       */
    int max_n;              /* largest n this context accepts (0: 40)                 */
    int split_k;            /* roots = 2^split_k per matrix (0: automatic)            */
    int waves_per_cu;       /* persistent waves per CU (0: automatic)                 */
    int accum;              /* TOR_ACCUM_DD or TOR_ACCUM_FP64                         */
    unsigned flags;         /* TOR_INPUT_DEVICE | TOR_CHECK_HERMITIAN | ...           */
} tor_options;

typedef struct {
    double tor;                /* Torontonian, high part                                */
    double tor_lo;             /* low part of the double-double value                   */
    double sum_abs;            /* sum of |term|; R = sum_abs / |tor| is the cancellation */
    double err_est;            /* typical relative error from the rounding of the
                                  terms: 2 u R / sqrt(2^n), u = 2^-53 (FP64 factor) or
                                  2^-102 (TOR_FACTOR_DD)                                */
    unsigned long long subsets;/* 2^n                                                   */
    int status;                /* TOR_OK or an error for this matrix                    */
    int path;                  /* 1 = real quadrature path, 2 = complex path,
                                  3 = real quadrature path with a double-double factor  */
    float device_ms;           /* device time of the launch that produced it (served
                                  requests: their share of the launches they ran in)    */
    int launches;              /* launches of the recursive kernel that computed it: 1,
                                  2 when failed roots ran once more (tor_eval), or for a
                                  served request the serving launches it took part in  */
} tor_result;

/* Defaults for every field (device 0, library stream and workspace, max_n 40). */
void tor_default_options(tor_options *opt);

/* Create a context on opt->device.  *out receives the handle.
 * Errors: TOR_E_INVAL (null out, an option out of range, a workspace not
 * aligned to 256 bytes), TOR_E_DEVICE (no GPU), TOR_E_NOMEM. */
int tor_create(tor_ctx **out, const tor_options *opt);

/* Stop the serving scheduler, cancel the served requests that have not
 * completed (their tickets are released), wait for the context's stream and
 * for the serving launches still on the GPU, then free every device and host
 * resource.  A request must not be polled after its context is destroyed. */
void tor_destroy(tor_ctx *ctx);

/* Device bytes a caller-provided workspace needs for matrices up to max_n
 * with up to max_inflight concurrent serving requests (serving stages its
 * requests there; its request pool, 256 MiB, and the workspaces of its two
 * launch streams it allocates itself on the first submission). */
size_t tor_workspace_size(int max_n, int split_k, int max_inflight);

/* Torontonian of one 2n x 2n matrix (Eq. 2), recursive GPU path.  Each of
 * the 2^k subtree roots writes its partial sum to a slot of its own, which a
 * later run of the same root overwrites.  A root whose partial sum comes out
 * non-finite while every pivot it tested was positive (a numeric failure, not
 * a property of the input) is therefore run once more: tor_eval, tor_eval_batch,
 * tor_eval_partials and tor_click_probs relaunch the range of failed roots of
 * each such matrix, then reduce its slots again in the same fixed order, so a
 * recovered result is bit for bit the result of a clean run and reports
 * launches = 2.  A root that fails again gives TOR_E_NUMERIC.  Serving and
 * tor_eval_static report TOR_E_NUMERIC without a second run. */
int tor_eval(tor_ctx *ctx, int n, const double *O, long ld, tor_result *out);

/* For callers that cannot allocate device or pinned memory -- code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc: the
 * same evaluation as tor_eval (same kernels, same split, the same value
 * bit for bit), using only a device array the library declares statically,
 * TOR_STATIC_SCRATCH_BYTES (128 MiB) per GPU, held from the first context
 * created on that GPU until the process ends.  It calls no hipMalloc,
 * hipFree, hipHostMalloc or host heap allocation, and uses neither the
 * context's workspace nor its pinned buffers, only its stream and events.
 * O is a host pointer (copied into the array) or, with TOR_INPUT_DEVICE,
 * device memory read in place.  The array holds the staged matrix, the
 * root slots and the per-wave stacks of one call at a time: every path fits
 * for n <= 30; beyond that the call returns TOR_E_SCRATCH when the launch's
 * stacks do not fit (the real quadrature path fits up to n = 34).  Calls on
 * one GPU share its array and keep the last call's contents; the library
 * serialises them with a per-device lock (calls that overlapped would race
 * on the array).  Errors: those of tor_eval, TOR_E_SCRATCH, and
 * TOR_E_DEVICE when the array's address could not be resolved. */
#define TOR_STATIC_SCRATCH_BYTES ((size_t)128 << 20)
int tor_eval_static(tor_ctx *ctx, int n, const double *O, long ld, tor_result *out);

/* Torontonians of count matrices of possibly different n in ONE persistent
 * launch: one work queue over (matrix, subtree root) items, largest n first.
 * out[i] corresponds to O[i] (input order).  Per-matrix failures are reported
 * in out[i].status and make the call return the first such error. */
int tor_eval_batch(tor_ctx *ctx, int count, const int *n, const double *const *O,
                   const long *ld, tor_result *out);

/* The comparison baseline (not the method): every subset gets a fresh Cholesky
 * (Algorithm 1) on the GPU, one wavefront per subset, in FP64 on the form the
 * recursive kernel would use (the real quadrature form of a Gaussian-state
 * matrix, else the complex matrix; TOR_FORCE_COMPLEX forces the latter).
 * Sums the subsets whose bitmask lies in [mask_begin, mask_end) (pass 0 and
 * 2^n for all of them); n <= 34.  The positive-definiteness test covers the
 * subsets of that range (the full I - O only when its mask 2^n - 1 is in it). */
int tor_eval_plain(tor_ctx *ctx, int n, const double *O, long ld,
                   unsigned long long mask_begin, unsigned long long mask_end,
                   tor_result *out);

/* The paper's own reuse order, as a second comparison (Sec. 2, Algorithm 2):
 * modes are removed in increasing order; a child keeps its parent's Cholesky
 * rows and columns of the kept modes below the removed mode (L11, L21) and
 * factorises the trailing block afresh, L22 = chol(A22 - L21 L21^H).  The
 * full Torontonian of the complex matrix (general Hermitian input; n <=
 * min(34, max_n)), one wavefront per depth-first walk below each of 2^k
 * roots (the removal decisions on the first k modes).  Same argument
 * conventions and errors as tor_eval; out->device_ms is the kernel time. */
int tor_eval_removal(tor_ctx *ctx, int n, const double *O, long ld, tor_result *out);

/* Verification aid: the recursive path's per-subtree partial sums.  Root r is
 * the include/exclude decision on modes 0..k-1 given by the bits of r (bit i =
 * mode i included); partial r sums the subsets Z with Z & (2^k - 1) == r.
 * The split depth is k = min(k_max, modes above the kernel's LDS and register
 * levels: n - 11 on the real path, n - 9 on the complex and double-double
 * paths, at least 0), not the context's own choice of k.  *k_out receives k;
 * partials receives 2^k (hi, lo, sum_abs) triples and must hold 3 * 2^k
 * doubles (0 <= k_max <= 30, else TOR_E_INVAL). */
int tor_eval_partials(tor_ctx *ctx, int n, const double *O, long ld, int k_max,
                      int *k_out, double *partials, tor_result *out);

/* Click probabilities of threshold detection for one Gaussian state (Sec. 1,
 * Eq. 1-2): for each pattern S (bit q of patterns[i] set = mode q clicked,
 * modes 0..M-1, M <= 64)
 *     p(S) = Tor(O_S) sqrt(det(I - O)),
 * O_S the principal submatrix of the M-mode O on rows and columns
 * {s, s + M : s in S}.  O is 2M x 2M complex128 row-major (interleaved re,
 * im), leading dimension ld >= 2M, device memory with TOR_INPUT_DEVICE; only
 * its lower triangle is read.  All patterns run as one batch (tor_eval_batch)
 * with the context's options (TOR_FACTOR_DD included), each O_S staged on the
 * device from O; sqrt(det(I - O)) is one FP64 Cholesky on the device.  probs receives count values (NaN
 * where a pattern failed); results (may be NULL) the per-pattern Tor(O_S)
 * records.  Errors: TOR_E_INVAL (bad sizes, a pattern with bits >= M or more
 * than max_n clicks), TOR_E_NOT_PD (I - O not positive definite), or the
 * first per-pattern error. */
int tor_click_probs(tor_ctx *ctx, int M, const double *O, long ld, int count,
                    const unsigned long long *patterns, double *probs, tor_result *results);

/* Click probabilities of every pattern of one Gaussian state at once, with
 * the work shared across patterns (Sec. 1, Eq. 1-2): every O_S draws its
 * terms from the same subset determinants of I - O, so one launch of the
 * recursive kernel over the whole M-mode state forms each of the 2^M terms
 * once, every prefix factor shared by all patterns, and stores it in device
 * memory; an exact double-double subset-sum transform over the subset lattice
 * then gives every Tor(O_S).  That is 2^M determinants and M passes over 2^M
 * sums, against 3^M determinants for the patterns one by one.  Pattern S is
 * indexed by its bitmask (bit q = mode q clicked).  probs (2^M doubles, may
 * be NULL) receives p(S) = Tor(O_S) sqrt(det(I - O)); tor_hi and tor_lo
 * (2^M doubles each, may be NULL) receive Tor(O_S) as a double-double; out
 * (may be NULL) the record of the whole state (Tor(O), its sum of |t|, the
 * device time of both steps).  tor_hi and tor_lo are both given or both NULL.
 * The outputs are host memory, or device memory with TOR_OUTPUT_DEVICE (out
 * stays a host record).  O is as for tor_click_probs.  The terms are those of the FP64 real quadrature path, and
 * each Tor(O_S) is their exact sum while its partial sums stay below 2^53
 * (for a Gaussian state every subset determinant of I - O is at most 1, so
 * every term is a double of magnitude at least 1, a multiple of 2^-52).  Device workspace: about 24 * 2^N bytes
 * beyond what tor_eval of the state needs, N = max(M, 11), plus 8 * 2^M bytes
 * for each output that goes to host memory (96 GiB at M = 32 with the
 * outputs on the device).
 * Errors: TOR_E_INVAL (M > TOR_CLICK_ALL_MAX_M or > max_n, a null O, no
 * output, only one of tor_hi and tor_lo, a context with TOR_FORCE_COMPLEX or TOR_FACTOR_DD, or an O without
 * the block structure of a Gaussian state), TOR_E_NOT_PD, TOR_E_NUMERIC (a
 * non-finite term; no re-run), TOR_E_NOMEM. */
#define TOR_CLICK_ALL_MAX_M 32
int tor_click_all(tor_ctx *ctx, int M, const double *O, long ld, double *probs, double *tor_hi, double *tor_lo,
                  tor_result *out);

/* Serving: enqueue one Torontonian request.  O is copied before return and
 * staged on the device when the request is admitted; a staging error
 * (TOR_E_INVAL), TOR_E_NOT_PD, or TOR_E_NOMEM when the device pool of the
 * serving loop cannot be allocated, is reported in the polled result's status.
 * *ticket identifies it for tor_poll.  TOR_E_BUSY when admission is refused;
 * TOR_E_NOMEM at once for a request larger than the whole pool. */
int tor_submit(tor_ctx *ctx, int n, const double *O, long ld, unsigned long long *ticket);

/* Serving: non-blocking.  TOR_OK and *out filled once the request is done
 * (the ticket is then released), TOR_PENDING while it runs, TOR_E_UNKNOWN for
 * a ticket this context does not hold. */
int tor_poll(tor_ctx *ctx, unsigned long long ticket, tor_result *out);

/* Serving: block until every submitted request has finished or timeout_ms
 * (< 0: no limit) passes (TOR_E_TIMEOUT). */
int tor_drain(tor_ctx *ctx, int timeout_ms);

/* Verification aid: the device's reciprocal square root and reciprocal for
 * count host doubles x.  out receives 4 * count doubles per input: rsqrt(x_i)
 * and 1/x_i as the kernels form them (hardware seed refined by one
 * third-order correction), then the two raw hardware seeds. */
int tor_debug_math(tor_ctx *ctx, int count, const double *x, double *out);

/* Measurement aid: the device's FP64 FMA throughput, to confirm the vector
 * peak the roofline is quoted against.  One kernel of 16 workgroups of 256
 * lanes per CU, each lane running 16 independent FMA chains of iters steps
 * (1 <= iters <= 2^20), timed with HIP events after one untimed launch.
 * *tflops receives 2 * 16 * iters * lanes / time; *ms (may be NULL) the
 * kernel time.  Uses the context's workspace. */
int tor_debug_fma_peak(tor_ctx *ctx, int iters, double *tflops, float *ms);

/* Test aid for the recovery described at tor_eval: in the next synchronous
 * evaluation on this context (tor_eval, tor_eval_batch, tor_eval_partials,
 * tor_click_probs), subtree root `root` of its first matrix reports a
 * numeric failure in its first `runs` launches (runs = 1: the re-run
 * recovers it; runs = 2: the result is TOR_E_NUMERIC; runs = 0 or root < 0
 * clears the request).  A root at or beyond that matrix's 2^k roots is
 * ignored.  The request is used up by that one evaluation.  Errors:
 * TOR_E_INVAL (null ctx, runs outside 0..2). */
int tor_debug_fail_root(tor_ctx *ctx, long long root, int runs);

/* Test aid: the subset-sum transform of tor_click_all on its own.  For the
 * 2^nbits host doubles t (1 <= nbits <= 26), g_hi and g_lo (host, 2^nbits
 * each) receive g[S] = sum over Z subset of S of t[Z] as double-doubles.
 * Errors: TOR_E_INVAL (null pointers, nbits out of range), TOR_E_NOMEM. */
int tor_debug_zeta(tor_ctx *ctx, int nbits, const double *t, double *g_hi, double *g_lo);

/* Serving policy.  Each chunked serving launch runs at most chunk_subsets
 * subsets (default 2^30, about 2.9 ms at n = 30 rates) taken from the
 * admitted requests with more than express_subsets subsets of work left:
 * oldest_share of it (default 0.5) goes to the oldest request, the rest to
 * the requests with the least remaining work, so a request larger than a
 * chunk is split over several launches (root ranges of its subtree roots)
 * while requests that arrive meanwhile join a later launch.  Chunked
 * launches run on all CUs but 16, one after another on a stream of their
 * own.  The requests with at most express_subsets subsets of work left
 * (default 2^24, n <= 24; 0 disables it) run whole in express launches on a
 * second stream: beside a chunked launch on the 16 CUs it leaves out, or on
 * the whole device when none runs, so they wait for no chunk (a chunk takes
 * them only while an express launch is busy).  max_queue bounds the
 * requests held (admitted or waiting); tor_submit beyond it returns
 * TOR_E_BUSY.  Applies from the scheduler's next round on.  Errors:
 * TOR_E_INVAL (chunk_subsets < 1024, express_subsets < 0, oldest_share
 * outside [0, 1], max_queue < 1). */
int tor_serve_config(tor_ctx *ctx, long long chunk_subsets, long long express_subsets,
                     double oldest_share, int max_queue);

/* Autotuner.  For every n in [n_min, n_max] and each selected path
 * (TOR_TUNE_REAL: Gaussian-state matrices, TOR_TUNE_COMPLEX: general ones,
 * TOR_TUNE_QUAD: the double-double factor)
 * time the recursive kernel over split depths k and persistent waves per CU
 * and keep the fastest pair for that size in the context; later evaluations
 * (single, batched and served) use it.  Timing does not depend on the matrix
 * values, so the tuner uses its own synthetic matrices.  Blocks for the
 * duration of the timing runs. */
#define TOR_TUNE_REAL 0x1u
#define TOR_TUNE_COMPLEX 0x2u
#define TOR_TUNE_QUAD 0x4u
int tor_autotune(tor_ctx *ctx, int n_min, int n_max, unsigned paths);

/* Write the context's tuning table as JSON (arch, CU count, entries). */
int tor_tune_save(tor_ctx *ctx, const char *path);

/* Load a table written by tor_tune_save; rejected (TOR_E_INVAL) when it was
 * made for another architecture or CU count. */
int tor_tune_load(tor_ctx *ctx, const char *path);

/* Static description of a code. */
const char *tor_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* TOR_H */
