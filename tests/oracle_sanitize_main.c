/*
 * Driver for the sanitizer build of the CPU oracle (test infrastructure):
 * tests/test_oracle_sanitizers.py compiles this file together with
 * oracle/tor_oracle.c under AddressSanitizer and UndefinedBehaviorSanitizer
 * and compares what it prints with the oracle library loaded in Python.
 *
 *   oracle_sanitize_main FILE N
 *
 * FILE holds the 2N x 2N complex128 matrix O (row-major, interleaved re, im).
 * Printed, one per line, as %.17g: the full sum in FP64, extended and
 * __float128 modes (hi + lo, then sum |t|), a restricted FP64 sum over the
 * subtree with mode 0 included and mode 1 excluded (3 threads), and one
 * subset's determinant and term.  Exit status 0 on success.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_tor(int n, const double *O, long ld, int mode, int nthreads, uint64_t fix_mask, uint64_t fix_val,
               double *out);
int oracle_det(int n, const double *O, long ld, uint64_t Z, int mode, double *out);

int main(int argc, char **argv)
{
    if (argc != 3)
        return 2;
    const int n = atoi(argv[2]);
    const size_t cnt = 2 * (size_t)(2 * n) * (size_t)(2 * n);
    double *O = (double *)malloc(sizeof(double) * (cnt ? cnt : 1));
    FILE *f = fopen(argv[1], "rb");
    if (!O || !f || fread(O, sizeof(double), cnt, f) != cnt)
        return 3;
    fclose(f);
    double out[5];
    for (int mode = 0; mode < 3; mode++) {
        if (oracle_tor(n, O, 2 * n, mode, 2, 0, 0, out) != 0)
            return 4;
        printf("%.17g\n%.17g\n", out[0] + out[1], out[2]);
    }
    if (oracle_tor(n, O, 2 * n, 0, 3, 3, 1, out) != 0)
        return 5;
    printf("%.17g\n", out[0] + out[1]);
    if (oracle_det(n, O, 2 * n, ((uint64_t)1 << n) - 2, 0, out) != 0)
        return 6;
    printf("%.17g\n%.17g\n", out[0], out[1]);
    free(O);
    return 0;
}
