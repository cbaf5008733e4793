/*
 * tor_oracle.c -- CPU oracle for the Torontonian.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load or call this library.  It shares no
 * code, header, table or helper with the GPU library; the product path never
 * links it.
 *
 * What it computes is the plain definition (Eq. 2 of the paper):
 *
 *     Tor(O) = sum over Z subset {0..n-1} of (-1)^(n-|Z|) / sqrt(det(I - O)_Z)
 *
 * where (I - O)_Z keeps rows and columns {i, i+n : i in Z} (mode i owns the
 * pair a_i, a_i^dagger in block order).  The empty subset contributes
 * (-1)^n, so n = 0 gives 1.
 *
 * Determinants.  Sec. 2 takes det A = prod |L_ii|^2 from the Cholesky factor
 * A = L L^H of a Hermitian positive definite A (Algorithm 1 defines L).  Here
 * every subset's matrix gets a fresh factorisation in its square-root-free
 * form, by Gaussian elimination on the lower triangle: eliminating column k
 * with the pivot p = A_kk replaces the trailing block by its Schur complement
 * A_ij - A_ik conj(A_jk) / p.  The pivots are the squared diagonal entries
 * |L_kk|^2 of the Cholesky factor, so det = prod p_k, and all of them are
 * positive exactly when A is positive definite (Sylvester's criterion);
 * a pivot that is not positive is reported as ORACLE_ENOTPD.  Only the lower
 * triangle of (I - O) is read: rows of the submatrix are taken in increasing
 * original index, so every element read lies in the lower triangle of I - O.
 *
 * Three precisions:
 *   ORACLE_F64  : FP64 elimination, determinant and term;
 *   ORACLE_QUAD : everything in __float128 (input converted exactly);
 *   ORACLE_LD   : everything in the x87 extended format (64-bit significand;
 *                 input converted exactly), the reference where __float128
 *                 is too slow (2^30 subsets) and FP64 too coarse.
 * In every mode the terms are summed in __float128, so summation adds no
 * error on top of the per-term rounding.  Beside the sum the oracle reports
 * sum |t| (the cancellation R = sum |t| / |Tor|) and sum t^2, whose square
 * root scales the spread of independent per-term rounding errors.
 *
 * Subsets are split over POSIX threads in interleaved chunks of 4096 masks
 * (masks with high modes included cost more, so contiguous ranges would
 * leave one thread with most of the work); the per-thread partial sums are
 * combined in thread order.  FP64 and extended terms are multiples of 2^-52
 * (2^-63) of magnitude >= 1 for the inputs here, so their __float128 sums are
 * exact and independent of this split.
 *
 * A restriction (fix_mask, fix_val) limits the sum to subsets Z with
 * (Z & fix_mask) == fix_val, i.e. one subtree of the include/exclude tree.
 */
#include <math.h>
#include <pthread.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define ORACLE_F64 0
#define ORACLE_QUAD 1
#define ORACLE_LD 2

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ENOTPD (-2)
#define ORACLE_ENOMEM (-3)

typedef __float128 q_t;
typedef long double ld_t;

/* ---- one determinant --------------------------------------------------------
 *
 * C is I - O as interleaved (re, im) pairs of type T, 2n x 2n, leading dim ldc
 * complex.  idx[0..m) are increasing row indices.  W is m*m complex scratch:
 * the submatrix's lower triangle is copied into it and eliminated in place.
 * Returns ORACLE_OK and det in *det, or ORACLE_ENOTPD.  The same elimination
 * is instantiated for each precision. */
#define DEFINE_DET(NAME, T)                                                      \
    static int NAME(const T *C, long ldc, const int *idx, int m, T *W, T *det)   \
    {                                                                            \
        for (int i = 0; i < m; i++)                                              \
            for (int j = 0; j <= i; j++) {                                       \
                const T *c = C + 2 * ((long)idx[i] * ldc + idx[j]);              \
                W[2 * ((long)i * m + j)] = c[0];                                 \
                W[2 * ((long)i * m + j) + 1] = c[1];                             \
            }                                                                    \
        T d = 1;                                                                 \
        for (int k = 0; k < m; k++) {                                            \
            const T p = W[2 * ((long)k * m + k)]; /* the diagonal is real */     \
            if (!(p > 0))                                                        \
                return ORACLE_ENOTPD;                                            \
            d *= p;                                                              \
            for (int i = k + 1; i < m; i++) {                                    \
                /* multiplier of row i: A_ik / p */                              \
                const T lr = W[2 * ((long)i * m + k)] / p;                       \
                const T li = W[2 * ((long)i * m + k) + 1] / p;                   \
                for (int j = k + 1; j <= i; j++) {                               \
                    /* A_ij -= (A_ik / p) conj(A_jk) */                          \
                    const T br = W[2 * ((long)j * m + k)];                       \
                    const T bi = W[2 * ((long)j * m + k) + 1];                   \
                    W[2 * ((long)i * m + j)] -= lr * br + li * bi;               \
                    W[2 * ((long)i * m + j) + 1] -= li * br - lr * bi;           \
                }                                                                \
            }                                                                    \
        }                                                                        \
        *det = d;                                                                \
        return ORACLE_OK;                                                        \
    }

DEFINE_DET(det_f64, double)
DEFINE_DET(det_ld, ld_t)
DEFINE_DET(det_quad, q_t)

/* rows {i, i+n : i in Z} in increasing order */
static int subset_rows(int n, uint64_t Z, int *idx)
{
    int m = 0;
    for (int i = 0; i < n; i++)
        if ((Z >> i) & 1u)
            idx[m++] = i;
    int d = m;
    for (int t = 0; t < d; t++)
        idx[m++] = idx[t] + n;
    return m;
}

/* I - O of one precision (full square copy; the lower triangle is what is
 * read) */
typedef struct {
    double *f64;
    ld_t *ld;
    q_t *q;
} cmat_t;

/* The signed term (-1)^(n-|Z|) / sqrt(det) of one subset, rounded to the
 * mode's precision and returned exactly as __float128; W is scratch of the
 * mode's type. */
static int subset_term(int n, int mode, const cmat_t *C, const int *idx, int m, void *W, q_t *t)
{
    const int N = 2 * n;
    const int neg = (n - m / 2) & 1;
    if (m == 0) {
        *t = neg ? -1 : 1;
        return ORACLE_OK;
    }
    if (mode == ORACLE_F64) {
        double det;
        if (det_f64(C->f64, N, idx, m, (double *)W, &det) != ORACLE_OK)
            return ORACLE_ENOTPD;
        const double td = 1.0 / sqrt(det);
        *t = (q_t)(neg ? -td : td);
    } else if (mode == ORACLE_LD) {
        ld_t det;
        if (det_ld(C->ld, N, idx, m, (ld_t *)W, &det) != ORACLE_OK)
            return ORACLE_ENOTPD;
        const ld_t tl = 1.0L / sqrtl(det);
        *t = (q_t)(neg ? -tl : tl);
    } else {
        q_t det;
        if (det_quad(C->q, N, idx, m, (q_t *)W, &det) != ORACLE_OK)
            return ORACLE_ENOTPD;
        const q_t tq = 1 / sqrtq(det);
        *t = neg ? -tq : tq;
    }
    return ORACLE_OK;
}

static size_t scalar_size(int mode)
{
    return mode == ORACLE_F64 ? sizeof(double) : mode == ORACLE_LD ? sizeof(ld_t) : sizeof(q_t);
}

/* ---- threaded sum ---------------------------------------------------------- */

#define CHUNK 4096

typedef struct {
    int n, mode;
    const cmat_t *C;
    uint64_t free_mask, fix_val;
    uint64_t total;       /* free-bit counters 0 .. total-1 */
    int tid, nthreads;    /* this thread takes chunks tid, tid + nthreads, ... */
    q_t sum, sum_abs, sum_sq;
    uint64_t count;
    int status;
} job_t;

/* scatter the bits of counter c onto the positions set in free_mask */
static uint64_t deposit(uint64_t c, uint64_t free_mask)
{
    uint64_t z = 0;
    for (int b = 0; free_mask; b++) {
        uint64_t low = free_mask & (~free_mask + 1);
        if ((c >> b) & 1u)
            z |= low;
        free_mask &= free_mask - 1;
    }
    return z;
}

static void *run_job(void *arg)
{
    job_t *jb = (job_t *)arg;
    int n = jb->n, N = 2 * n;
    int *idx = (int *)malloc(sizeof(int) * (N > 0 ? N : 1));
    void *W = malloc(2 * scalar_size(jb->mode) * (size_t)(N > 0 ? N * N : 1));
    if (!idx || !W) {
        jb->status = ORACLE_ENOMEM;
        free(idx);
        free(W);
        return NULL;
    }
    q_t sum = 0, sum_abs = 0, sum_sq = 0;
    for (uint64_t c0 = (uint64_t)jb->tid * CHUNK; c0 < jb->total && jb->status == ORACLE_OK;
         c0 += (uint64_t)jb->nthreads * CHUNK) {
        const uint64_t c1 = c0 + CHUNK < jb->total ? c0 + CHUNK : jb->total;
        for (uint64_t c = c0; c < c1; c++) {
            uint64_t Z = deposit(c, jb->free_mask) | jb->fix_val;
            int m = subset_rows(n, Z, idx);
            q_t t;
            if (subset_term(n, jb->mode, jb->C, idx, m, W, &t) != ORACLE_OK) {
                jb->status = ORACLE_ENOTPD;
                break;
            }
            sum += t;
            sum_abs += (t < 0 ? -t : t);
            sum_sq += t * t;
            jb->count++;
        }
    }
    jb->sum = sum;
    jb->sum_abs = sum_abs;
    jb->sum_sq = sum_sq;
    free(idx);
    free(W);
    return NULL;
}

/* Build C = I - O in the mode's precision; each input double is converted
 * exactly, and 1 - o on the diagonal is rounded once in that precision. */
static int make_c(int n, const double *O, long ld, int mode, cmat_t *C)
{
    const int N = 2 * n;
    const size_t cnt = 2 * (size_t)N * N;
    memset(C, 0, sizeof(*C));
    if (mode == ORACLE_F64)
        C->f64 = (double *)malloc(sizeof(double) * cnt);
    else if (mode == ORACLE_LD)
        C->ld = (ld_t *)malloc(sizeof(ld_t) * cnt);
    else
        C->q = (q_t *)malloc(sizeof(q_t) * cnt);
    if (!C->f64 && !C->ld && !C->q)
        return ORACLE_ENOMEM;
    for (int i = 0; i < N; i++)
        for (int j = 0; j < N; j++) {
            const double ore = O[2 * ((long)i * ld + j)];
            const double oim = O[2 * ((long)i * ld + j) + 1];
            const size_t at = 2 * ((size_t)i * N + j);
            if (C->f64) {
                C->f64[at] = i == j ? 1.0 - ore : -ore;
                C->f64[at + 1] = -oim;
            } else if (C->ld) {
                C->ld[at] = i == j ? 1.0L - (ld_t)ore : -(ld_t)ore;
                C->ld[at + 1] = -(ld_t)oim;
            } else {
                C->q[at] = i == j ? (q_t)1 - (q_t)ore : -(q_t)ore;
                C->q[at + 1] = -(q_t)oim;
            }
        }
    return ORACLE_OK;
}

static void free_c(cmat_t *C)
{
    free(C->f64);
    free(C->ld);
    free(C->q);
}

static int mode_ok(int mode) { return mode == ORACLE_F64 || mode == ORACLE_QUAD || mode == ORACLE_LD; }

/*
 * oracle_tor: sum over subsets Z with (Z & fix_mask) == fix_val.
 *   O       : complex128 interleaved, 2n x 2n, row-major, leading dim ld (complex elems)
 *   out[0], out[1] : the sum as a double-double (hi, lo)
 *   out[2]  : sum of |term|
 *   out[3]  : number of subsets summed
 *   out[4]  : sum of term^2
 * Returns ORACLE_OK, ORACLE_EINVAL, ORACLE_ENOTPD or ORACLE_ENOMEM.
 */
int oracle_tor(int n, const double *O, long ld, int mode, int nthreads,
               uint64_t fix_mask, uint64_t fix_val, double *out)
{
    if (n < 0 || n > 62 || !out || (n > 0 && (!O || ld < 2 * n)) || !mode_ok(mode))
        return ORACLE_EINVAL;
    uint64_t full = (1ull << n) - 1;
    if ((fix_mask & ~full) || (fix_val & ~fix_mask))
        return ORACLE_EINVAL;
    cmat_t C;
    memset(&C, 0, sizeof(C));
    if (n > 0 && make_c(n, O, ld, mode, &C) != ORACLE_OK)
        return ORACLE_ENOMEM;
    uint64_t free_mask = full & ~fix_mask;
    int nfree = __builtin_popcountll(free_mask);
    uint64_t total = 1ull << nfree;
    if (nthreads <= 0) {
        long p = sysconf(_SC_NPROCESSORS_ONLN);
        nthreads = p > 0 ? (int)p : 1;
    }
    const uint64_t nchunks = (total + CHUNK - 1) / CHUNK;
    if ((uint64_t)nthreads > nchunks)
        nthreads = (int)nchunks;
    job_t *jobs = (job_t *)calloc((size_t)nthreads, sizeof(job_t));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    int *started = (int *)calloc((size_t)nthreads, sizeof(int));
    if (!jobs || !th || !started) {
        free(jobs);
        free(th);
        free(started);
        free_c(&C);
        return ORACLE_ENOMEM;
    }
    for (int t = 0; t < nthreads; t++) {
        jobs[t].n = n;
        jobs[t].mode = mode;
        jobs[t].C = &C;
        jobs[t].free_mask = free_mask;
        jobs[t].fix_val = fix_val;
        jobs[t].total = total;
        jobs[t].tid = t;
        jobs[t].nthreads = nthreads;
    }
    int status = ORACLE_OK;
    if (nthreads == 1) {
        run_job(&jobs[0]);
    } else {
        for (int t = 0; t < nthreads; t++) {
            if (pthread_create(&th[t], NULL, run_job, &jobs[t]) == 0)
                started[t] = 1;
            else
                run_job(&jobs[t]);
        }
        for (int t = 0; t < nthreads; t++)
            if (started[t])
                pthread_join(th[t], NULL);
    }
    q_t sum = 0, sum_abs = 0, sum_sq = 0;
    uint64_t count = 0;
    for (int t = 0; t < nthreads; t++) {
        if (jobs[t].status != ORACLE_OK)
            status = jobs[t].status;
        sum += jobs[t].sum;
        sum_abs += jobs[t].sum_abs;
        sum_sq += jobs[t].sum_sq;
        count += jobs[t].count;
    }
    double hi = (double)sum;
    double lo = (double)(sum - (q_t)hi);
    out[0] = hi;
    out[1] = lo;
    out[2] = (double)sum_abs;
    out[3] = (double)count;
    out[4] = (double)sum_sq;
    free(jobs);
    free(th);
    free(started);
    free_c(&C);
    return status;
}

/*
 * oracle_det: det((I - O)_Z) for one subset Z (bitmask over modes), by the same
 * fresh elimination.  out[0] = det (rounded to double), out[1] = the signed term
 * (-1)^(n-|Z|)/sqrt(det) rounded to double.
 */
int oracle_det(int n, const double *O, long ld, uint64_t Z, int mode, double *out)
{
    if (n < 0 || n > 62 || !out || (n > 0 && (!O || ld < 2 * n)) || !mode_ok(mode))
        return ORACLE_EINVAL;
    uint64_t full = (1ull << n) - 1;
    if (Z & ~full)
        return ORACLE_EINVAL;
    int idx[124];
    int m = subset_rows(n, Z, idx);
    if (m == 0) {
        const int neg = n & 1;
        out[0] = 1.0;
        out[1] = neg ? -1.0 : 1.0;
        return ORACLE_OK;
    }
    cmat_t C;
    if (make_c(n, O, ld, mode, &C) != ORACLE_OK)
        return ORACLE_ENOMEM;
    void *W = malloc(2 * scalar_size(mode) * (size_t)m * m);
    if (!W) {
        free_c(&C);
        return ORACLE_ENOMEM;
    }
    int rc;
    if (mode == ORACLE_F64) {
        double det;
        rc = det_f64(C.f64, 2 * n, idx, m, (double *)W, &det);
        out[0] = det;
    } else if (mode == ORACLE_LD) {
        ld_t det;
        rc = det_ld(C.ld, 2 * n, idx, m, (ld_t *)W, &det);
        out[0] = (double)det;
    } else {
        q_t det;
        rc = det_quad(C.q, 2 * n, idx, m, (q_t *)W, &det);
        out[0] = (double)det;
    }
    if (rc == ORACLE_OK) {
        q_t t;
        rc = subset_term(n, mode, &C, idx, m, W, &t);
        out[1] = (double)t;
    }
    free(W);
    free_c(&C);
    return rc;
}
