/* Driver for the host runtime built with AddressSanitizer and
 * UndefinedBehaviorSanitizer (host code only; the kernels are the usual ones).
 * It calls every entry point of the C ABI on seeded inputs written by the
 * test (raw complex128 matrices, row-major), the error paths included, and
 * prints one line per result so the test can compare them with the regular
 * build.  Any sanitizer report ends the process with a non-zero status.
 *
 * usage: runtime_sanitized DIR   (DIR holds mNN.bin, a matrix of NN modes,
 *        for NN in 5 8 10 12 14 16 20 and the 12-mode state s12.bin) */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "tor.h"

static const char *g_dir;

static double *load(const char *name, int n)
{
    char path[4096];
    snprintf(path, sizeof path, "%s/%s", g_dir, name);
    FILE *f = fopen(path, "rb");
    if (!f) {
        fprintf(stderr, "cannot open %s\n", path);
        exit(3);
    }
    const size_t cnt = (size_t)2 * (2 * n) * (2 * n);
    double *a = (double *)malloc(sizeof(double) * (cnt ? cnt : 1));
    if (cnt && fread(a, sizeof(double), cnt, f) != cnt) {
        fprintf(stderr, "short read %s\n", path);
        exit(3);
    }
    fclose(f);
    return a;
}

static int g_fail;
static void expect(int cond, const char *what)
{
    if (!cond) {
        fprintf(stderr, "check failed: %s\n", what);
        g_fail = 1;
    }
}

static void put(const char *tag, const tor_result *r)
{
    printf("%s %d %.17g %.17g %.17g %d %d\n", tag, r->status, r->tor, r->tor_lo, r->sum_abs, r->path, r->launches);
}

int main(int argc, char **argv)
{
    if (argc != 2) {
        fprintf(stderr, "usage: %s DIR\n", argv[0]);
        return 2;
    }
    g_dir = argv[1];
    tor_options opt;
    tor_default_options(&opt);
    opt.max_n = 34;
    tor_ctx *ctx = NULL;
    int rc = tor_create(&ctx, &opt);
    if (rc != TOR_OK) {
        fprintf(stderr, "tor_create: %s\n", tor_strerror(rc));
        return 4;
    }
    static const int sizes[] = {5, 8, 10, 12, 14, 16, 20};
    double *m[7];
    char name[64];
    for (int i = 0; i < 7; i++) {
        snprintf(name, sizeof name, "m%d.bin", sizes[i]);
        m[i] = load(name, sizes[i]);
    }
    tor_result r;

    /* single evaluations, the empty matrix included */
    rc = tor_eval(ctx, 0, NULL, 0, &r);
    expect(rc == TOR_OK && r.tor == 1.0, "n = 0");
    for (int i = 0; i < 7; i++) {
        rc = tor_eval(ctx, sizes[i], m[i], 2L * sizes[i], &r);
        expect(rc == TOR_OK, "tor_eval");
        snprintf(name, sizeof name, "eval%d", sizes[i]);
        put(name, &r);
    }

    /* one batch of all of them, in input order */
    {
        int ns[7];
        long lds[7];
        const double *ps[7];
        tor_result rs[7];
        for (int i = 0; i < 7; i++) {
            ns[i] = sizes[i];
            lds[i] = 2L * sizes[i];
            ps[i] = m[i];
        }
        rc = tor_eval_batch(ctx, 7, ns, ps, lds, rs);
        expect(rc == TOR_OK, "tor_eval_batch");
        for (int i = 0; i < 7; i++) {
            snprintf(name, sizeof name, "batch%d", sizes[i]);
            put(name, &rs[i]);
        }
    }

    /* partials of n = 16 at k = 4, summed */
    {
        int k = -1;
        double parts[3 * 16];
        rc = tor_eval_partials(ctx, 16, m[5], 32, 4, &k, parts, &r);
        expect(rc == TOR_OK && k == 4, "tor_eval_partials");
        double s = 0.0;
        for (int i = 0; i < 16; i++)
            s += parts[3 * i] + parts[3 * i + 1];
        printf("partials16 %d %.17g\n", k, s);
    }

    /* the allocation-free entry point, the comparison kernels */
    rc = tor_eval_static(ctx, 14, m[4], 28, &r);
    expect(rc == TOR_OK, "tor_eval_static");
    put("static14", &r);
    rc = tor_eval_plain(ctx, 8, m[1], 16, 0, 256, &r);
    expect(rc == TOR_OK, "tor_eval_plain");
    put("plain8", &r);
    rc = tor_eval_removal(ctx, 8, m[1], 16, &r);
    expect(rc == TOR_OK, "tor_eval_removal");
    put("removal8", &r);

    /* click probabilities: some patterns one by one, and all of them at once */
    {
        double *s12 = load("s12.bin", 12);
        unsigned long long pats[64];
        double probs[64];
        tor_result rs[64];
        for (int i = 0; i < 64; i++)
            pats[i] = (unsigned long long)i * 61u % 4096u;
        rc = tor_click_probs(ctx, 12, s12, 24, 64, pats, probs, rs);
        expect(rc == TOR_OK, "tor_click_probs");
        double *all = (double *)malloc(sizeof(double) * 4096);
        double *th = (double *)malloc(sizeof(double) * 4096);
        double *tl = (double *)malloc(sizeof(double) * 4096);
        rc = tor_click_all(ctx, 12, s12, 24, all, th, tl, &r);
        expect(rc == TOR_OK, "tor_click_all");
        double worst = 0.0, sum = 0.0;
        for (int i = 0; i < 64; i++)
            worst = fmax(worst, fabs(all[pats[i]] - probs[i]));
        for (int i = 0; i < 4096; i++)
            sum += all[i];
        printf("click %.3g %.17g\n", worst, sum);
        expect(worst <= 1e-14 && fabs(sum - 1.0) <= 1e-12, "click probabilities agree and sum to one");
        free(all);
        free(th);
        free(tl);
        free(s12);
    }

    /* recovery of a root forced to fail, then one that keeps failing */
    rc = tor_debug_fail_root(ctx, 3, 1);
    expect(rc == TOR_OK, "tor_debug_fail_root");
    rc = tor_eval(ctx, 20, m[6], 40, &r);
    expect(rc == TOR_OK && r.launches == 2, "recovered root");
    put("recovered20", &r);
    tor_debug_fail_root(ctx, 3, 2);
    rc = tor_eval(ctx, 20, m[6], 40, &r);
    expect(rc == TOR_E_NUMERIC, "persisting failure");

    /* serving: a few requests, a drain, then every ticket polled */
    {
        rc = tor_serve_config(ctx, 1 << 20, 1 << 12, 0.5, 64);
        expect(rc == TOR_OK, "tor_serve_config");
        unsigned long long t[7];
        for (int i = 0; i < 7; i++) {
            rc = tor_submit(ctx, sizes[i], m[i], 2L * sizes[i], &t[i]);
            expect(rc == TOR_OK, "tor_submit");
        }
        rc = tor_drain(ctx, 60000);
        expect(rc == TOR_OK, "tor_drain");
        for (int i = 0; i < 7; i++) {
            rc = tor_poll(ctx, t[i], &r);
            expect(rc == TOR_OK, "tor_poll");
            snprintf(name, sizeof name, "served%d", sizes[i]);
            put(name, &r);
        }
        expect(tor_poll(ctx, t[0], &r) == TOR_E_UNKNOWN, "released ticket");
    }

    /* the autotuner and its cache */
    {
        char path[4096];
        snprintf(path, sizeof path, "%s/tune.json", g_dir);
        expect(tor_autotune(ctx, 12, 13, TOR_TUNE_REAL) == TOR_OK, "tor_autotune");
        expect(tor_tune_save(ctx, path) == TOR_OK, "tor_tune_save");
        expect(tor_tune_load(ctx, path) == TOR_OK, "tor_tune_load");
    }

    /* error paths */
    expect(tor_eval(ctx, 5, NULL, 10, &r) == TOR_E_INVAL, "null matrix");
    expect(tor_eval(ctx, 35, m[0], 70, &r) == TOR_E_INVAL, "n > max_n");
    expect(tor_eval(ctx, 5, m[0], 9, &r) == TOR_E_INVAL, "ld < 2n");
    expect(tor_serve_config(ctx, 10, 0, 0.5, 1) == TOR_E_INVAL, "bad chunk");
    expect(tor_click_all(ctx, TOR_CLICK_ALL_MAX_M + 1, m[0], 2 * (TOR_CLICK_ALL_MAX_M + 1), NULL, NULL, NULL, &r) ==
               TOR_E_INVAL,
           "M too large");
    for (int c = -9; c <= 1; c++)
        expect(tor_strerror(c) != NULL && tor_strerror(c)[0] != 0, "tor_strerror");
    {
        double *bad = load("m5.bin", 5);
        bad[2 * (1 * 10 + 0)] = NAN;  /* element (1, 0): the lower triangle is read */
        expect(tor_eval(ctx, 5, bad, 10, &r) == TOR_E_INVAL, "NaN input");
        free(bad);
    }

    tor_destroy(ctx);
    for (int i = 0; i < 7; i++)
        free(m[i]);
    printf("done %d\n", g_fail);
    return g_fail ? 1 : 0;
}
