/*
 * Driver for the address/undefined-behaviour sanitizer check of the CPU oracle
 * (test infrastructure; built and run by tests/test_oracle_sanitized.py).  It
 * calls every oracle entry point on seeded random pencils of small and edge
 * sizes (n = 0, 1, 2, odd and even), subsets, leading dimensions larger than
 * n, a pencil with B not positive definite, and the forced QL failure; each
 * call's status is checked, and a residual check on the full solve guards
 * against a sanitizer run that silently computes nothing.  Any invalid memory
 * access, leak or undefined operation ends the process with a non-zero status.
 */
#include <complex.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

typedef double complex zc;

int oracle_potrf(int n, zc *B, int ldb);
void oracle_hegst(int n, const zc *A, int lda, const zc *L, int ldl, zc *C, int ldc);
void oracle_hetrd(int n, zc *C, int ldc, double *d, double *e, zc *U, int ldu, double *beta, zc *psi);
int oracle_steql(int n, double *d, double *e, double *Z, int ldz);
int oracle_zhegv(int n, const zc *A, int lda, const zc *B, int ldb, int il, int iu, double *W, zc *X, int ldx);
void oracle_set_ql_maxit(int maxit);

static unsigned long long rng = 88172645463325252ull;
static double urand(void) {   /* xorshift64, uniform in [-1, 1) */
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (double)(rng >> 11) / 4503599627370496.0 - 1.0;
}

/* lower triangles of A (Hermitian) and B (Hermitian positive definite), ld >= n */
static void pencil(int n, int ld, zc *A, zc *B) {
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < ld; ++i) {
            A[i + (size_t)j * ld] = i < n ? urand() + I * (i == j ? 0.0 : urand()) : 0.0;
            B[i + (size_t)j * ld] = i < n ? 0.1 * (urand() + I * (i == j ? 0.0 : urand())) : 0.0;
        }
    for (int j = 0; j < n; ++j) B[j + (size_t)j * ld] = 2.0 + n * 0.2;   /* diagonally dominant */
}

static int check_solve(int n, int ld, int il, int iu) {
    const int m = iu - il + 1;
    zc *A = calloc((size_t)ld * (n > 0 ? n : 1), sizeof(zc));
    zc *B = calloc((size_t)ld * (n > 0 ? n : 1), sizeof(zc));
    double *W = calloc(m > 0 ? m : 1, sizeof(double));
    zc *X = calloc((size_t)ld * (m > 0 ? m : 1), sizeof(zc));
    pencil(n, ld, A, B);
    int st = oracle_zhegv(n, A, ld, B, ld, il, iu, W, X, ld);
    int bad = st != 0;
    /* residual of the first returned pair: || A x - w B x ||_inf  (A, B Hermitian from lower) */
    if (!bad && n > 0) {
        double r = 0.0, s = 0.0;
        for (int i = 0; i < n; ++i) {
            zc ax = 0.0, bx = 0.0;
            for (int k = 0; k < n; ++k) {
                zc a = i >= k ? A[i + (size_t)k * ld] : conj(A[k + (size_t)i * ld]);
                zc b = i >= k ? B[i + (size_t)k * ld] : conj(B[k + (size_t)i * ld]);
                if (i == k) { a = creal(a); b = creal(b); }
                ax += a * X[k];
                bx += b * X[k];
            }
            r = fmax(r, cabs(ax - W[0] * bx));
            s = fmax(s, cabs(ax) + fabs(W[0]) * cabs(bx));
        }
        bad = !(r <= 1e-10 * (s + 1.0));
    }
    if (bad) fprintf(stderr, "solve n=%d ld=%d il=%d iu=%d: status %d\n", n, ld, il, iu, st);
    free(A); free(B); free(W); free(X);
    return bad;
}

int main(void) {
    int fails = 0;
    const int sizes[][4] = {{0, 1, 1, 1}, {1, 1, 1, 1}, {2, 2, 1, 2}, {5, 7, 2, 4}, {16, 16, 1, 16},
                            {33, 40, 5, 20}, {64, 64, 64, 64}, {97, 101, 1, 30}};
    for (unsigned c = 0; c < sizeof(sizes) / sizeof(sizes[0]); ++c) {
        const int n = sizes[c][0], ld = sizes[c][1];
        const int il = n > 0 ? sizes[c][2] : 1, iu = n > 0 ? sizes[c][3] : 0;
        if (n == 0) {   /* n = 0: nothing to do, status 0 */
            fails += oracle_zhegv(0, NULL, 1, NULL, 1, 1, 0, NULL, NULL, 1) != 0;
            continue;
        }
        fails += check_solve(n, ld, il, iu);
    }
    /* argument errors */
    {
        zc a[4] = {0}, b[4] = {0};
        double w[2];
        zc x[4];
        fails += oracle_zhegv(-1, a, 2, b, 2, 1, 1, w, x, 2) != -1;
        fails += oracle_zhegv(2, a, 1, b, 2, 1, 1, w, x, 2) != -3;
        fails += oracle_zhegv(2, a, 2, b, 2, 0, 1, w, x, 2) != -6;
        fails += oracle_zhegv(2, a, 2, b, 2, 2, 1, w, x, 2) != -7;
    }
    /* B not positive definite at order 3 of 5: status n + 3 */
    {
        const int n = 5;
        zc A[25], B[25];
        double W[5];
        zc X[25];
        pencil(n, n, A, B);
        B[2 + 2 * n] = -1.0;
        fails += oracle_zhegv(n, A, n, B, n, 1, n, W, X, n) != n + 3;
    }
    /* the stages on their own, and the forced QL failure */
    {
        const int n = 9;
        zc A[81], B[81], C[81], U[81], psi[9];
        double d[9], e[9], beta[9], Z[81];
        pencil(n, n, A, B);
        fails += oracle_potrf(n, B, n) != 0;
        oracle_hegst(n, A, n, B, n, C, n);
        oracle_hetrd(n, C, n, d, e, U, n, beta, psi);
        for (int i = 0; i < n * n; ++i) Z[i] = (i % (n + 1)) == 0 ? 1.0 : 0.0;
        fails += oracle_steql(n, d, e, Z, n) != 0;
        pencil(n, n, A, B);
        oracle_set_ql_maxit(0);
        double W[9];
        zc X[81];
        const int st = oracle_zhegv(n, A, n, B, n, 1, n, W, X, n);
        fails += !(st >= 1 && st <= n);
        oracle_set_ql_maxit(30);
    }
    if (fails) fprintf(stderr, "%d checks failed\n", fails);
    else printf("oracle sanitizer run: all checks passed\n");
    return fails ? 1 : 0;
}
