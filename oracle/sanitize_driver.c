/*
 * Test driver for a sanitizer build of the oracle (AddressSanitizer and
 * UndefinedBehaviorSanitizer, gcc): runs every exported oracle routine on
 * small inputs -- including the edge cases n = 1, n = 2, a zero matrix, range
 * requests, exact-eigenvalue shifts, split matrices and a bidiagonal -- so
 * that an out-of-bounds access, a leak or undefined arithmetic in the oracle
 * stops the run.  TEST INFRASTRUCTURE ONLY, like the oracle itself.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int or_eigvecs(int n, const double *d, const double *e, int il, int iu, const double *Win,
               int orth, int iters, uint64_t seed, double *W, double *Z, int ldz, int *status);
int or_eigvecs_split(int n, const double *d, const double *e, int il, int iu, int orth,
                     int iters, uint64_t seed, double *W, double *Z, int ldz, int *status,
                     int *blk);
int or_bidiag_svd(int n, const double *a, const double *b, int il, int iu, int orth, int iters,
                  uint64_t seed, double *S, double *U, int ldu, double *V, int ldv, int *status);
int or_orthogonalize(int n, int m, const double *V, int ldv, double *Q, int ldq, double *Y,
                     double *T, int variant, int *brk);

static uint64_t rng = 88172645463325252ULL;
static double urand(void)   /* xorshift64, U(-1, 1): inputs only */
{
    rng ^= rng << 13; rng ^= rng >> 7; rng ^= rng << 17;
    return (double)(rng >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

static int run(int n, const double *d, const double *e, int il, int iu, const double *Win,
               int orth, int iters)
{
    int m = iu - il + 1;
    double *W = malloc(sizeof(double) * m), *Z = malloc(sizeof(double) * (size_t)n * m);
    int *st = malloc(sizeof(int) * m);
    int rc = or_eigvecs(n, d, e, il, iu, Win, orth, iters, 0x12091910ULL, W, Z, n, st);
    free(W); free(Z); free(st);
    return rc < 0;
}

int main(void)
{
    int bad = 0;
    for (int n = 1; n <= 40; n += 13) {
        double *d = malloc(sizeof(double) * n), *e = malloc(sizeof(double) * (n > 1 ? n - 1 : 1));
        for (int i = 0; i < n; i++) d[i] = urand();
        for (int i = 0; i < n - 1; i++) e[i] = urand();
        for (int orth = 0; orth < 4; orth++)
            for (int iters = -1; iters <= 3; iters += 2) {
                bad |= run(n, d, e, 1, n, NULL, orth, iters);
                if (n > 2) bad |= run(n, d, e, 2, n - 1, NULL, orth, iters);
            }
        free(d); free(e);
    }
    {   /* glued Wilkinson blocks (clusters), zero matrix, exact shift */
        int g = 5, n = 21 * g;
        double *d = malloc(sizeof(double) * n), *e = malloc(sizeof(double) * n);
        for (int i = 0; i < n; i++) d[i] = fabs(10.0 - (double)(i % 21));
        for (int i = 0; i < n - 1; i++) e[i] = (i % 21 == 20) ? 1e-8 : 1.0;
        bad |= run(n, d, e, 1, n, NULL, 0, 3);
        bad |= run(n, d, e, 1, n, NULL, 3, -1);
        for (int i = 0; i < n - 1; i++) if (i % 21 == 20) e[i] = 0.0;
        double *W = malloc(sizeof(double) * n), *Z = malloc(sizeof(double) * n * n);
        int *st = malloc(sizeof(int) * n), *blk = malloc(sizeof(int) * n);
        bad |= or_eigvecs_split(n, d, e, 1, n, 0, 3, 7, W, Z, n, st, blk) < 0;
        bad |= or_eigvecs_split(n, d, e, 10, 40, 3, -1, 7, W, Z, n, st, blk) < 0;
        double zero[2] = {0.0, 0.0}, w0[1] = {0.0};
        bad |= run(1, zero, zero, 1, 1, NULL, 0, 3);
        bad |= run(1, zero, zero, 1, 1, w0, 0, 3);
        free(d); free(e); free(W); free(Z); free(st); free(blk);
    }
    {   /* bidiagonal through the Golub-Kahan tridiagonal */
        int n = 30;
        double a[30], b[29], S[30], U[900], V[900];
        int st[30];
        for (int i = 0; i < n; i++) a[i] = 2.0 + 0.5 * (urand() + 1.0);
        for (int i = 0; i < n - 1; i++) b[i] = urand();
        bad |= or_bidiag_svd(n, a, b, 1, n, 0, 3, 3, S, U, n, V, n, st) < 0;
        bad |= or_bidiag_svd(n, a, b, 5, 9, 0, -1, 3, S, U, n, V, n, st) < 0;
    }
    {   /* orthogonalization of given vectors, every variant, a dependent column */
        int n = 9, m = 5;
        double Vv[45], Q[45], Y[45], T[25];
        int brk[5];
        for (int i = 0; i < n * m; i++) Vv[i] = urand();
        for (int i = 0; i < n; i++) Vv[i + 2 * n] = Vv[i + n];
        for (int v = 0; v < 4; v++) bad |= or_orthogonalize(n, m, Vv, n, Q, n, Y, T, v, brk) != 0;
    }
    printf(bad ? "oracle sanitizer driver: FAILED\n" : "oracle sanitizer driver: ok\n");
    return bad;
}
