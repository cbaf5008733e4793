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
 * pair a_i, a_i^dagger in block order).  Each determinant comes from a fresh
 * Cholesky decomposition of that submatrix (Algorithm 1 of the paper, row by
 * row: off-diagonal L_ij by forward substitution, then L_ii as the square root
 * of the remaining diagonal), and det = prod |L_ii|^2 (Sec. 2).  The empty
 * subset contributes (-1)^n, so n = 0 gives 1.
 *
 * Only the lower triangle of (I - O) is read, as Algorithm 1 needs.  Rows of
 * the submatrix are taken in increasing original index, so every element read
 * lies in the lower triangle of I - O.
 *
 * Two precisions:
 *   ORACLE_F64  : FP64 Cholesky, FP64 determinant and term, terms summed in
 *                 __float128 (so summation adds no error on top of the FP64
 *                 per-term rounding);
 *   ORACLE_QUAD : everything in __float128 (input converted exactly).
 *
 * Subsets are split over POSIX threads in contiguous ranges; the per-thread
 * partial sums are combined in thread order.
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

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ENOTPD (-2)
#define ORACLE_ENOMEM (-3)

typedef __float128 q_t;

/* ---- one determinant, FP64 ------------------------------------------------ */

/* C is I - O as interleaved (re, im) doubles, 2n x 2n, leading dim ldc complex.
 * idx[0..m) are increasing row indices.  L is m*m complex scratch (lower part).
 * Returns 0 and det in *det, or ORACLE_ENOTPD. */
static int det_f64(const double *C, long ldc, const int *idx, int m, double *L,
                   double *det)
{
    double d = 1.0;
    for (int i = 0; i < m; i++) {
        const double *crow = C + 2 * ((long)idx[i] * ldc);
        double *li = L + 2 * (long)i * m;
        for (int j = 0; j < i; j++) {
            const double *lj = L + 2 * (long)j * m;
            double sr = crow[2 * idx[j]], si = crow[2 * idx[j] + 1];
            for (int k = 0; k < j; k++) {
                /* s -= L_ik * conj(L_jk) */
                double ar = li[2 * k], ai = li[2 * k + 1];
                double br = lj[2 * k], bi = lj[2 * k + 1];
                sr -= ar * br + ai * bi;
                si -= ai * br - ar * bi;
            }
            double ljj = lj[2 * j]; /* real, positive */
            li[2 * j] = sr / ljj;
            li[2 * j + 1] = si / ljj;
        }
        double s = crow[2 * idx[i]];
        for (int k = 0; k < i; k++)
            s -= li[2 * k] * li[2 * k] + li[2 * k + 1] * li[2 * k + 1];
        if (!(s > 0.0))
            return ORACLE_ENOTPD;
        d *= s; /* |L_ii|^2 */
        li[2 * i] = sqrt(s);
        li[2 * i + 1] = 0.0;
    }
    *det = d;
    return ORACLE_OK;
}

/* ---- one determinant, __float128 ----------------------------------------- */

static int det_quad(const q_t *C, long ldc, const int *idx, int m, q_t *L, q_t *det)
{
    q_t d = 1;
    for (int i = 0; i < m; i++) {
        const q_t *crow = C + 2 * ((long)idx[i] * ldc);
        q_t *li = L + 2 * (long)i * m;
        for (int j = 0; j < i; j++) {
            const q_t *lj = L + 2 * (long)j * m;
            q_t sr = crow[2 * idx[j]], si = crow[2 * idx[j] + 1];
            for (int k = 0; k < j; k++) {
                q_t ar = li[2 * k], ai = li[2 * k + 1];
                q_t br = lj[2 * k], bi = lj[2 * k + 1];
                sr -= ar * br + ai * bi;
                si -= ai * br - ar * bi;
            }
            q_t ljj = lj[2 * j];
            li[2 * j] = sr / ljj;
            li[2 * j + 1] = si / ljj;
        }
        q_t s = crow[2 * idx[i]];
        for (int k = 0; k < i; k++)
            s -= li[2 * k] * li[2 * k] + li[2 * k + 1] * li[2 * k + 1];
        if (!(s > 0))
            return ORACLE_ENOTPD;
        d *= s;
        li[2 * i] = sqrtq(s);
        li[2 * i + 1] = 0;
    }
    *det = d;
    return ORACLE_OK;
}

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

/* ---- threaded sum ---------------------------------------------------------- */

typedef struct {
    int n, mode;
    const double *C64; /* I - O, FP64, ld = 2n */
    const q_t *Cq;     /* I - O, quad,  ld = 2n */
    uint64_t free_mask, fix_val;
    int nfree;
    uint64_t lo, hi; /* range of free-bit counters */
    q_t sum, sum_abs;
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
    double *L64 = NULL;
    q_t *Lq = NULL;
    if (jb->mode == ORACLE_F64)
        L64 = (double *)malloc(sizeof(double) * 2 * (size_t)(N > 0 ? N * N : 1));
    else
        Lq = (q_t *)malloc(sizeof(q_t) * 2 * (size_t)(N > 0 ? N * N : 1));
    if (!idx || (!L64 && !Lq)) {
        jb->status = ORACLE_ENOMEM;
        free(idx); free(L64); free(Lq);
        return NULL;
    }
    q_t sum = 0, sum_abs = 0;
    for (uint64_t c = jb->lo; c < jb->hi; c++) {
        uint64_t Z = deposit(c, jb->free_mask) | jb->fix_val;
        int m = subset_rows(n, Z, idx);
        int sign_neg = ((n - m / 2) & 1);
        q_t t;
        if (jb->mode == ORACLE_F64) {
            double det = 1.0;
            if (m > 0 && det_f64(jb->C64, N, idx, m, L64, &det) != ORACLE_OK) {
                jb->status = ORACLE_ENOTPD;
                break;
            }
            double td = 1.0 / sqrt(det);
            t = (q_t)(sign_neg ? -td : td);
        } else {
            q_t det = 1;
            if (m > 0 && det_quad(jb->Cq, N, idx, m, Lq, &det) != ORACLE_OK) {
                jb->status = ORACLE_ENOTPD;
                break;
            }
            q_t tq = 1 / sqrtq(det);
            t = sign_neg ? -tq : tq;
        }
        sum += t;
        sum_abs += (t < 0 ? -t : t);
        jb->count++;
    }
    jb->sum = sum;
    jb->sum_abs = sum_abs;
    free(idx); free(L64); free(Lq);
    return NULL;
}

/* Build C = I - O (full square copy, lower triangle is what is read). */
static void make_c(int n, const double *O, long ld, double *C64, q_t *Cq)
{
    int N = 2 * n;
    for (int i = 0; i < N; i++)
        for (int j = 0; j < N; j++) {
            double re = -O[2 * ((long)i * ld + j)];
            double im = -O[2 * ((long)i * ld + j) + 1];
            if (C64) {
                C64[2 * ((long)i * N + j)] = (i == j ? 1.0 - O[2 * ((long)i * ld + j)] : re);
                C64[2 * ((long)i * N + j) + 1] = im;
            }
            if (Cq) {
                /* exact conversion of the input, then 1 - o in quad */
                q_t ore = (q_t)O[2 * ((long)i * ld + j)];
                q_t oim = (q_t)O[2 * ((long)i * ld + j) + 1];
                Cq[2 * ((long)i * N + j)] = (i == j ? (q_t)1 - ore : -ore);
                Cq[2 * ((long)i * N + j) + 1] = -oim;
            }
        }
}

/*
 * oracle_tor: sum over subsets Z with (Z & fix_mask) == fix_val.
 *   O       : complex128 interleaved, 2n x 2n, row-major, leading dim ld (complex elems)
 *   out[0], out[1] : the sum as a double-double (hi, lo)
 *   out[2]  : sum of |term|
 *   out[3]  : number of subsets summed
 * Returns ORACLE_OK, ORACLE_EINVAL, ORACLE_ENOTPD or ORACLE_ENOMEM.
 */
int oracle_tor(int n, const double *O, long ld, int mode, int nthreads,
               uint64_t fix_mask, uint64_t fix_val, double *out)
{
    if (n < 0 || n > 62 || !out || (n > 0 && (!O || ld < 2 * n)))
        return ORACLE_EINVAL;
    if (mode != ORACLE_F64 && mode != ORACLE_QUAD)
        return ORACLE_EINVAL;
    uint64_t full = (n == 64) ? ~0ull : ((1ull << n) - 1);
    if ((fix_mask & ~full) || (fix_val & ~fix_mask))
        return ORACLE_EINVAL;
    int N = 2 * n;
    double *C64 = NULL;
    q_t *Cq = NULL;
    if (n > 0) {
        if (mode == ORACLE_F64)
            C64 = (double *)malloc(sizeof(double) * 2 * (size_t)N * N);
        else
            Cq = (q_t *)malloc(sizeof(q_t) * 2 * (size_t)N * N);
        if (!C64 && !Cq)
            return ORACLE_ENOMEM;
        make_c(n, O, ld, C64, Cq);
    }
    uint64_t free_mask = full & ~fix_mask;
    int nfree = __builtin_popcountll(free_mask);
    uint64_t total = 1ull << nfree;
    if (nthreads <= 0) {
        long p = sysconf(_SC_NPROCESSORS_ONLN);
        nthreads = p > 0 ? (int)p : 1;
    }
    if ((uint64_t)nthreads > total)
        nthreads = (int)total;
    job_t *jobs = (job_t *)calloc((size_t)nthreads, sizeof(job_t));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !th) {
        free(jobs); free(th); free(C64); free(Cq);
        return ORACLE_ENOMEM;
    }
    for (int t = 0; t < nthreads; t++) {
        jobs[t].n = n;
        jobs[t].mode = mode;
        jobs[t].C64 = C64;
        jobs[t].Cq = Cq;
        jobs[t].free_mask = free_mask;
        jobs[t].fix_val = fix_val;
        jobs[t].nfree = nfree;
        jobs[t].lo = total / nthreads * t + (t < (int)(total % nthreads) ? t : total % nthreads);
        jobs[t].hi = jobs[t].lo + total / nthreads + (t < (int)(total % nthreads) ? 1 : 0);
    }
    int status = ORACLE_OK;
    if (nthreads == 1) {
        run_job(&jobs[0]);
    } else {
        for (int t = 0; t < nthreads; t++)
            if (pthread_create(&th[t], NULL, run_job, &jobs[t]) != 0) {
                run_job(&jobs[t]);
                th[t] = 0;
            }
        for (int t = 0; t < nthreads; t++)
            if (th[t])
                pthread_join(th[t], NULL);
    }
    q_t sum = 0, sum_abs = 0;
    uint64_t count = 0;
    for (int t = 0; t < nthreads; t++) {
        if (jobs[t].status != ORACLE_OK)
            status = jobs[t].status;
        sum += jobs[t].sum;
        sum_abs += jobs[t].sum_abs;
        count += jobs[t].count;
    }
    double hi = (double)sum;
    double lo = (double)(sum - (q_t)hi);
    out[0] = hi;
    out[1] = lo;
    out[2] = (double)sum_abs;
    out[3] = (double)count;
    free(jobs); free(th); free(C64); free(Cq);
    return status;
}

/*
 * oracle_det: det((I - O)_Z) for one subset Z (bitmask over modes), by the same
 * fresh Cholesky.  out[0] = det (rounded to double), out[1] = the signed term
 * (-1)^(n-|Z|)/sqrt(det) rounded to double.
 */
int oracle_det(int n, const double *O, long ld, uint64_t Z, int mode, double *out)
{
    if (n < 0 || n > 62 || !out || (n > 0 && (!O || ld < 2 * n)))
        return ORACLE_EINVAL;
    uint64_t full = (1ull << n) - 1;
    if (Z & ~full)
        return ORACLE_EINVAL;
    int N = 2 * n;
    int idx[124];
    int m = subset_rows(n, Z, idx);
    int sign_neg = ((n - m / 2) & 1);
    int rc = ORACLE_OK;
    if (m == 0) {
        out[0] = 1.0;
        out[1] = sign_neg ? -1.0 : 1.0;
        return ORACLE_OK;
    }
    if (mode == ORACLE_F64) {
        double *C = (double *)malloc(sizeof(double) * 2 * (size_t)N * N);
        double *L = (double *)malloc(sizeof(double) * 2 * (size_t)m * m);
        if (!C || !L) { free(C); free(L); return ORACLE_ENOMEM; }
        make_c(n, O, ld, C, NULL);
        double det;
        rc = det_f64(C, N, idx, m, L, &det);
        if (rc == ORACLE_OK) {
            out[0] = det;
            double td = 1.0 / sqrt(det);
            out[1] = sign_neg ? -td : td;
        }
        free(C); free(L);
    } else {
        q_t *C = (q_t *)malloc(sizeof(q_t) * 2 * (size_t)N * N);
        q_t *L = (q_t *)malloc(sizeof(q_t) * 2 * (size_t)m * m);
        if (!C || !L) { free(C); free(L); return ORACLE_ENOMEM; }
        make_c(n, O, ld, NULL, C);
        q_t det;
        rc = det_quad(C, N, idx, m, L, &det);
        if (rc == ORACLE_OK) {
            out[0] = (double)det;
            q_t tq = 1 / sqrtq(det);
            out[1] = (double)(sign_neg ? -tq : tq);
        }
        free(C); free(L);
    }
    return rc;
}
