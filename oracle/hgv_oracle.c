/*
 * hgv_oracle.c -- plain, slow, obviously correct CPU reference for the
 * Hermitian-definite generalized eigenproblem  A x = lambda B x.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the HIP
 * library and includes nothing from it.
 *
 * Method (Algorithm 1 of the paper, with the one-stage form of Algorithm 2,
 * Sec. 4.1):
 *   1. B = L L^H                         (unblocked Cholesky, Alg. 1 step 1)
 *   2. A' = L^-1 A L^-H                  (explicit triangular solves, step 2)
 *   3. A' = Q T Q^H                      (unblocked Householder reduction to
 *                                         tridiagonal form, Alg. 2 step 1)
 *   4. T y' = lambda y'                  (implicit QL with shifts, rotations
 *                                         accumulated; Alg. 2 step 2)
 *   5. y = Q y',  x = L^-H y             (Alg. 2 step 3, Alg. 1 step 4)
 * Every eigenpair is computed; the il..iu subset (1-based, inclusive,
 * ascending) is selected at the end.  Arithmetic is IEEE double throughout,
 * no blocking, no BLAS.  OpenMP only splits loops whose iterations are
 * independent (columns of a solve, rows of a rotation sweep); the order of
 * every floating-point sum is fixed, so results do not depend on the thread
 * count.
 *
 * Storage: column-major, element (i,j) of an n x n matrix with leading
 * dimension ld at index i + j*ld.  Only the lower triangle of A and B is read
 * (the imaginary part of their diagonals is ignored).
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>

typedef double complex zc;

#define AT(M, i, j, ld) ((M)[(size_t)(i) + (size_t)(j) * (size_t)(ld)])

static int g_ql_maxit = 30; /* QL iterations allowed per eigenvalue */

/* Test hook: cap the QL iteration count (0 forces a convergence failure). */
void oracle_set_ql_maxit(int maxit) { g_ql_maxit = maxit; }

/* ------------------------------------------------------------------------ */
/* Step 1 (Alg. 1, step 1): B = L L^H, L lower with real positive diagonal. */
/* Column j of L:  L_jj = sqrt(B_jj - sum_k<j |L_jk|^2),
 *                 L_ij = (B_ij - sum_k<j L_ik conj(L_jk)) / L_jj,  i > j.
 * Overwrites the lower triangle of B with L and zeroes the strict upper one.
 * Returns 0, or k (1-based) when the leading minor of order k is not
 * positive definite (pivot <= 0 or NaN).                                     */
int oracle_potrf(int n, zc *B, int ldb)
{
    zc *col = (zc *)malloc(sizeof(zc) * (size_t)(n > 0 ? n : 1));
    int info = 0;
    for (int j = 0; j < n && !info; ++j) {
        for (int i = j; i < n; ++i) col[i] = AT(B, i, j, ldb);
        col[j] = creal(col[j]);
        /* subtract the contributions of the finished columns k < j */
        for (int k = 0; k < j; ++k) {
            zc c = conj(AT(B, j, k, ldb));
            if (c == 0) continue;
            for (int i = j; i < n; ++i) col[i] -= AT(B, i, k, ldb) * c;
        }
        double piv = creal(col[j]);
        if (!(piv > 0.0)) { info = j + 1; break; }
        double ljj = sqrt(piv);
        AT(B, j, j, ldb) = ljj;
        for (int i = j + 1; i < n; ++i) AT(B, i, j, ldb) = col[i] / ljj;
    }
    free(col);
    if (!info)
        for (int j = 1; j < n; ++j)
            for (int i = 0; i < j; ++i) AT(B, i, j, ldb) = 0;
    return info;
}

/* Solve L w = w in place (L lower, non-unit), column-oriented forward
 * substitution:  w_k /= L_kk,  w_i -= L_ik w_k for i > k.                    */
static void lower_solve(int n, const zc *L, int ldl, zc *w)
{
    for (int k = 0; k < n; ++k) {
        w[k] /= AT(L, k, k, ldl);
        zc wk = w[k];
        if (wk == 0) continue;
        for (int i = k + 1; i < n; ++i) w[i] -= AT(L, i, k, ldl) * wk;
    }
}

/* Solve L^H x = y in place (back substitution):
 * x_i = (y_i - sum_{k>i} conj(L_ki) x_k) / L_ii, i = n-1 .. 0.              */
static void lower_h_solve(int n, const zc *L, int ldl, zc *x)
{
    for (int i = n - 1; i >= 0; --i) {
        zc s = x[i];
        for (int k = i + 1; k < n; ++k) s -= conj(AT(L, k, i, ldl)) * x[k];
        x[i] = s / conj(AT(L, i, i, ldl));
    }
}

/* ------------------------------------------------------------------------ */
/* Step 2 (Alg. 1, step 2): C = L^-1 A L^-H from the lower triangle of A.
 * W = L^-1 A (full Hermitian A, column by column), then C = L^-1 W^H, which
 * equals (L^-1 A L^-H)^H = A'.  The result is made exactly Hermitian by
 * averaging with its conjugate transpose.  C is n x n, full storage.         */
void oracle_hegst(int n, const zc *A, int lda, const zc *L, int ldl,
                  zc *C, int ldc)
{
    zc *W = (zc *)malloc(sizeof(zc) * (size_t)n * (size_t)(n > 0 ? n : 1));
    /* full Hermitian A from its lower triangle */
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            zc v = (i > j) ? AT(A, i, j, lda)
                 : (i < j) ? conj(AT(A, j, i, lda)) : (zc)creal(AT(A, j, j, lda));
            W[(size_t)i + (size_t)j * n] = v;
        }
#pragma omp parallel for schedule(dynamic, 4)
    for (int j = 0; j < n; ++j) lower_solve(n, L, ldl, W + (size_t)j * n);
    /* C(:, j) = L^-1 (row j of W)^H */
#pragma omp parallel for schedule(dynamic, 4)
    for (int j = 0; j < n; ++j) {
        zc *c = &AT(C, 0, j, ldc);
        for (int i = 0; i < n; ++i) c[i] = conj(W[(size_t)j + (size_t)i * n]);
        lower_solve(n, L, ldl, c);
    }
    free(W);
    for (int j = 0; j < n; ++j) {
        AT(C, j, j, ldc) = creal(AT(C, j, j, ldc));
        for (int i = j + 1; i < n; ++i) {
            zc v = 0.5 * (AT(C, i, j, ldc) + conj(AT(C, j, i, ldc)));
            AT(C, i, j, ldc) = v;
            AT(C, j, i, ldc) = conj(v);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Step 3 (Alg. 2 step 1, one-stage form, Sec. 4.1): Householder reduction of
 * the full Hermitian C (overwritten) to real symmetric tridiagonal form.
 *
 * For k = 0 .. n-3, x = C[k+1:n, k], alpha = x_0, phi = alpha/|alpha|
 * (phi = 1 when alpha = 0), u = x + phi*||x|| e_1 and the Hermitian reflector
 * H_k = I - beta_k u u^H, beta_k = 2/(u^H u), maps x to -phi*||x|| e_1.  The
 * trailing block is updated two-sidedly, C22 <- H C22 H, through
 *   p = beta C22 u,  q = p - (u^H p / u^H u) u,  C22 <- C22 - u q^H - q u^H.
 * Reflectors with x[1:] = 0 are skipped (beta_k = 0).
 *
 * The complex tridiagonal T_c (subdiagonal e_k) is then scaled to the real
 * T_r = Psi^H T_c Psi with Psi = diag(psi), psi_0 = 1,
 * psi_{k+1} = psi_k e_k/|e_k|; T_r has subdiagonal |e_k| >= 0.
 *
 * Outputs: d[n], e[n-1] (real T_r); U (n x n, column k holds u_k in rows
 * k+1..n-1); beta[n]; psi[n].  So  A' = Q Psi T_r Psi^H Q^H  with
 * Q = H_0 H_1 ... H_{n-3}.                                                    */
void oracle_hetrd(int n, zc *C, int ldc, double *d, double *e,
                  zc *U, int ldu, double *beta, zc *psi)
{
    zc *p = (zc *)malloc(sizeof(zc) * (size_t)(n > 0 ? n : 1));
    zc *ec = (zc *)malloc(sizeof(zc) * (size_t)(n > 0 ? n : 1));
    for (int k = 0; k < n; ++k) beta[k] = 0.0;
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;          /* length of x */
        zc *x = &AT(C, k + 1, k, ldc);
        zc *u = &AT(U, k + 1, k, ldu);
        double tail = 0.0;                /* ||x[1:]||^2 */
        for (int i = 1; i < m; ++i) tail += creal(x[i]) * creal(x[i]) + cimag(x[i]) * cimag(x[i]);
        zc alpha = x[0];
        if (tail == 0.0) {                /* already reduced: H = I */
            for (int i = 0; i < m; ++i) u[i] = 0;
            ec[k] = alpha;
            continue;
        }
        double aabs = cabs(alpha);
        zc phi = (aabs == 0.0) ? 1.0 : alpha / aabs;
        double xnorm = sqrt(aabs * aabs + tail);
        for (int i = 0; i < m; ++i) u[i] = x[i];
        u[0] += phi * xnorm;
        double utu = 0.0;
        for (int i = 0; i < m; ++i) utu += creal(u[i]) * creal(u[i]) + cimag(u[i]) * cimag(u[i]);
        double bk = 2.0 / utu;
        beta[k] = bk;
        /* p = beta * C22 u  (C22 = C[k+1:, k+1:], full Hermitian storage;
         * row i of C22 read as the conjugate of its column i)               */
#pragma omp parallel for schedule(static)
        for (int i = 0; i < m; ++i) {
            const zc *ci = &AT(C, k + 1, k + 1 + i, ldc);
            zc s = 0;
            for (int j = 0; j < m; ++j) s += conj(ci[j]) * u[j];
            p[i] = bk * s;
        }
        zc uhp = 0;
        for (int i = 0; i < m; ++i) uhp += conj(u[i]) * p[i];
        double K = creal(uhp) / utu;      /* u^H p is real (C22 Hermitian) */
        for (int i = 0; i < m; ++i) p[i] -= K * u[i];   /* p now holds q */
        /* C22 <- C22 - u q^H - q u^H */
#pragma omp parallel for schedule(static)
        for (int j = 0; j < m; ++j) {
            zc cu = conj(u[j]), cq = conj(p[j]);
            zc *cj = &AT(C, k + 1, k + 1 + j, ldc);
            for (int i = 0; i < m; ++i) cj[i] -= u[i] * cq + p[i] * cu;
        }
        ec[k] = -phi * xnorm;
        x[0] = ec[k];
        for (int i = 1; i < m; ++i) x[i] = 0;
    }
    if (n >= 2) ec[n - 2] = AT(C, n - 1, n - 2, ldc);
    for (int k = 0; k < n; ++k) d[k] = creal(AT(C, k, k, ldc));
    if (n >= 1) psi[0] = 1.0;
    for (int k = 0; k + 1 < n; ++k) {
        double a = cabs(ec[k]);
        e[k] = a;
        psi[k + 1] = (a == 0.0) ? psi[k] : psi[k] * (ec[k] / a);
    }
    free(p);
    free(ec);
}

/* ------------------------------------------------------------------------ */
/* Step 4 (Alg. 2 step 2): implicit QL with shifts on the real symmetric
 * tridiagonal (d, e), accumulating rotations into Z (n x n real; must hold
 * the identity, or the basis to be rotated, on entry).
 *
 * The active block is rows l..m: e_l..e_{m-1} are non-negligible and e_m is
 * negligible (|e_k| <= eps (|d_k| + |d_{k+1}|)) or m = n-1.  One QL step with
 * shift sigma (the eigenvalue of [d_l e_l; e_l d_{l+1}] closest to d_l) is
 * carried out as an explicit chase of plane rotations G = [c -s; s c] acting
 * on coordinates (j, j+1), T <- G T G^T, Z <- Z G^T:
 *   - the first rotation (j = m-1) maps the vector (e_{m-1}, d_m - sigma),
 *     i.e. the last column of T - sigma I, to (0, r);
 *   - rotating (j, j+1) turns the coupling e_{j-1} into c e_{j-1} and leaves a
 *     bulge s e_{j-1} at position (j+1, j-1);
 *   - the next rotation, on (j-1, j), is chosen to annihilate that bulge:
 *     (c, s) proportional to (T[j+1, j], bulge).
 * The chase ends at j = l.  Each step's rotations are recorded and applied to
 * the rows of Z in parallel (rows are independent), in order.  Eigenvalues
 * are finally sorted ascending with Z's columns permuted alike.  Returns 0,
 * or l+1 when eigenvalue l needs more than the allowed number of steps.      */
static void rotate_2x2(double *a, double *b, double *dd, double c, double s)
{
    /* [a b; b dd] <- G [a b; b dd] G^T with G = [c -s; s c] */
    double a0 = *a, b0 = *b, d0 = *dd;
    *a = c * c * a0 - 2.0 * c * s * b0 + s * s * d0;
    *dd = s * s * a0 + 2.0 * c * s * b0 + c * c * d0;
    *b = c * s * (a0 - d0) + (c * c - s * s) * b0;
}

int oracle_steql(int n, double *d, double *e_in, double *Z, int ldz)
{
    if (n <= 0) return 0;
    double *e = (double *)calloc((size_t)n, sizeof(double));
    double *rc = (double *)malloc(sizeof(double) * 2 * (size_t)n);
    int *rj = (int *)malloc(sizeof(int) * (size_t)n);
    for (int i = 0; i + 1 < n; ++i) e[i] = e_in[i];
    int info = 0;
    for (int l = 0; l < n && !info; ++l) {
        int steps = 0;
        for (;;) {
            int m = l;
            while (m < n - 1 && fabs(e[m]) > DBL_EPSILON * (fabs(d[m]) + fabs(d[m + 1]))) ++m;
            if (m == l) break;                       /* d_l has converged */
            if (steps++ >= g_ql_maxit) { info = l + 1; break; }
            double delta = 0.5 * (d[l + 1] - d[l]);
            double root = hypot(delta, e[l]);
            double sigma = d[l] - e[l] * e[l] / (delta + (delta >= 0.0 ? root : -root));
            int nrot = 0;
            double bulge = 0.0;
            for (int j = m - 1; j >= l; --j) {
                double c, s, r;
                if (j == m - 1) {                    /* start from T - sigma I */
                    double x = d[m] - sigma, y = e[m - 1];
                    r = hypot(x, y);
                    if (r == 0.0) { c = 1.0; s = 0.0; } else { c = x / r; s = y / r; }
                } else {                             /* annihilate the bulge */
                    double x = e[j + 1], y = bulge;
                    r = hypot(x, y);
                    if (r == 0.0) { c = 1.0; s = 0.0; } else { c = x / r; s = y / r; }
                    e[j + 1] = r;                    /* T[j+2,j+1] after the rotation */
                }
                rotate_2x2(&d[j], &e[j], &d[j + 1], c, s);
                if (j > l) {                         /* coupling to row j-1 */
                    bulge = s * e[j - 1];
                    e[j - 1] = c * e[j - 1];
                }
                rj[nrot] = j;
                rc[2 * (size_t)nrot] = c;
                rc[2 * (size_t)nrot + 1] = s;
                ++nrot;
            }
            /* Z <- Z G^T for each rotation, in the order generated */
#pragma omp parallel for schedule(static)
            for (int row = 0; row < n; ++row) {
                double *zr = Z + row;
                for (int t = 0; t < nrot; ++t) {
                    size_t j = (size_t)rj[t];
                    double c = rc[2 * (size_t)t], s = rc[2 * (size_t)t + 1];
                    double zj = zr[j * ldz], zj1 = zr[(j + 1) * ldz];
                    zr[j * ldz] = c * zj - s * zj1;
                    zr[(j + 1) * ldz] = s * zj + c * zj1;
                }
            }
        }
    }
    free(rc);
    free(rj);
    free(e);
    if (info) return info;
    /* selection sort ascending, columns of Z permuted alike */
    for (int i = 0; i < n - 1; ++i) {
        int k = i;
        for (int j = i + 1; j < n; ++j)
            if (d[j] < d[k]) k = j;
        if (k != i) {
            double t = d[i]; d[i] = d[k]; d[k] = t;
            for (int row = 0; row < n; ++row) {
                double z = Z[row + (size_t)i * ldz];
                Z[row + (size_t)i * ldz] = Z[row + (size_t)k * ldz];
                Z[row + (size_t)k * ldz] = z;
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Whole solve (Alg. 1 with the one-stage Alg. 2).  A, B: lower triangles of
 * the pencil (not modified).  On success W[0..m) holds eigenvalues il..iu
 * ascending and X (n x m, ldx) the eigenvectors with X^H B X = I.
 * Returns 0; -k for bad argument k; n+k when B's leading minor of order k is
 * not positive definite; k in [1,n] when QL fails on eigenvalue k.           */
int oracle_zhegv(int n, const zc *A, int lda, const zc *B, int ldb,
                 int il, int iu, double *W, zc *X, int ldx)
{
    if (n < 0) return -1;
    if (lda < (n > 1 ? n : 1)) return -3;
    if (ldb < (n > 1 ? n : 1)) return -5;
    if (n == 0) return 0;
    if (il < 1 || il > n) return -6;
    if (iu < il || iu > n) return -7;
    if (ldx < n) return -10;
    const int m = iu - il + 1;
    size_t nn = (size_t)n * (size_t)n;
    zc *L = (zc *)malloc(sizeof(zc) * nn);
    zc *C = (zc *)malloc(sizeof(zc) * nn);
    zc *U = (zc *)calloc(nn, sizeof(zc));
    double *Z = (double *)calloc(nn, sizeof(double));
    double *d = (double *)malloc(sizeof(double) * n);
    double *e = (double *)calloc((size_t)n, sizeof(double));
    double *beta = (double *)malloc(sizeof(double) * n);
    zc *psi = (zc *)malloc(sizeof(zc) * n);
    int info = 0;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) L[i + (size_t)j * n] = (i >= j) ? AT(B, i, j, ldb) : 0;
    int pinfo = oracle_potrf(n, L, n);
    if (pinfo) { info = n + pinfo; goto done; }
    oracle_hegst(n, A, lda, L, n, C, n);
    oracle_hetrd(n, C, n, d, e, U, n, beta, psi);
    for (int i = 0; i < n; ++i) Z[i + (size_t)i * n] = 1.0;
    info = oracle_steql(n, d, e, Z, n);
    if (info) goto done;
    for (int j = 0; j < m; ++j) W[j] = d[il - 1 + j];
    /* back-transform each selected column: y = Q Psi z, x = L^-H y */
#pragma omp parallel for schedule(dynamic, 1)
    for (int j = 0; j < m; ++j) {
        zc *x = &AT(X, 0, j, ldx);
        const double *z = Z + (size_t)(il - 1 + j) * n;
        for (int i = 0; i < n; ++i) x[i] = psi[i] * z[i];
        for (int k = n - 3; k >= 0; --k) {       /* y <- H_k y, last first */
            if (beta[k] == 0.0) continue;
            const zc *u = &U[(size_t)(k + 1) + (size_t)k * n];
            zc *y = x + k + 1;
            zc s = 0;
            for (int i = 0; i < n - k - 1; ++i) s += conj(u[i]) * y[i];
            s *= beta[k];
            for (int i = 0; i < n - k - 1; ++i) y[i] -= u[i] * s;
        }
        lower_h_solve(n, L, n, x);
    }
done:
    free(L); free(C); free(U); free(Z); free(d); free(e); free(beta); free(psi);
    return info;
}
