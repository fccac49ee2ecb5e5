/*
 * oracle_hess.c -- plain, slow CPU reference for the Hessenberg reduction.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the test-suite loads it.  It shares no code,
 * header, table or constant with the HIP path.
 *
 * What it computes (paper Sec. 2, Eq. (3), the Hessenberg reduction): for a
 * dense real matrix A, an orthogonal Q1 and an upper Hessenberg H with
 * A = Q1 H Q1^T.  The paper defers the theory to Golub & Van Loan (cited at
 * the end of Sec. 2); this file follows that text's Householder reduction
 * (Sec. 7.4.3) in its own code: for each column k = 0 .. n-3 a Householder
 * reflector P_k = I - beta v v^T acting on rows and columns k+1 .. n-1 maps
 * A(k+1:n-1, k) to a multiple of e_1; it is applied from the left to
 * A(k+1:n-1, k:n-1) and from the right to A(0:n-1, k+1:n-1), and
 * accumulated into Q (Q <- Q P_k), so that Q1 e_1 = e_1.
 *
 * Readings where the paper is silent:
 *   - reflector sign: the new subdiagonal entry is -sign(x_1) ||x|| with
 *     sign(0) = +1 (the usual choice, free of cancellation); v_1 = 1;
 *   - a column whose tail is already zero gets the identity (beta = 0);
 *   - the entries below the subdiagonal are stored as exact zeros;
 *   - Q accumulates: Q <- Q_in Q1 (identity when Q_in is the identity).
 * Storage: column-major with a leading dimension.  Precision: binary64,
 * no BLAS or LAPACK.
 */
#include <math.h>
#include <stddef.h>
#include <stdlib.h>

#define AX(i, j) A[(size_t)(i) + (size_t)(j) * (size_t)lda]
#define QX(i, j) Q[(size_t)(i) + (size_t)(j) * (size_t)ldq]

/* Householder reflector of x (length m >= 1): v (v[0] = 1), beta and the
 * image alpha with (I - beta v v^T) x = alpha e_1.  Norm computed with a
 * scale factor so that squares cannot overflow. */
static void orh_house(int m, const double *x, double *v, double *beta, double *alpha)
{
    double scale = 0.0, ss = 0.0, nrm, d;
    int i;
    for (i = 0; i < m; ++i) scale = fmax(scale, fabs(x[i]));
    for (i = 1; i < m; ++i) {
        double t = (scale > 0.0) ? x[i] / scale : 0.0;
        ss += t * t;
    }
    v[0] = 1.0;
    if (ss == 0.0) {             /* tail already zero: identity */
        for (i = 1; i < m; ++i) v[i] = 0.0;
        *beta = 0.0;
        *alpha = x[0];
        return;
    }
    {
        double t0 = x[0] / scale;
        nrm = scale * sqrt(t0 * t0 + ss);
    }
    *alpha = (x[0] >= 0.0) ? -nrm : nrm;
    d = x[0] - *alpha;          /* no cancellation: x[0] and -alpha have the same sign */
    for (i = 1; i < m; ++i) v[i] = x[i] / d;
    /* beta = 2 / (v^T v), the reflector's definition */
    {
        double vv = 1.0;
        for (i = 1; i < m; ++i) vv += v[i] * v[i];
        *beta = 2.0 / vv;
    }
}

/* Reduce A (n x n, lda) to upper Hessenberg form in place; Q (ldq, may be
 * NULL) is multiplied from the right by every reflector.  Returns 0, or -1
 * when the workspace cannot be allocated. */
int oracle_hessenberg(int n, double *A, int lda, double *Q, int ldq)
{
    double *v, *w;
    int k, i, j;
    if (n <= 2) return 0;
    v = (double *)malloc(sizeof(double) * (size_t)n);
    w = (double *)malloc(sizeof(double) * (size_t)n);
    if (!v || !w) { free(v); free(w); return -1; }
    for (k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;           /* rows k+1 .. n-1 */
        double beta, alpha;
        for (i = 0; i < m; ++i) w[i] = AX(k + 1 + i, k);
        orh_house(m, w, v, &beta, &alpha);
        if (beta != 0.0) {
            /* left: A(k+1:, j) -= beta v (v^T A(k+1:, j)) for columns j >= k */
            for (j = k; j < n; ++j) {
                double s = 0.0;
                for (i = 0; i < m; ++i) s += v[i] * AX(k + 1 + i, j);
                s *= beta;
                for (i = 0; i < m; ++i) AX(k + 1 + i, j) -= s * v[i];
            }
            /* right: A(i, k+1:) -= beta (A(i, k+1:) v) v^T for all rows */
            for (i = 0; i < n; ++i) {
                double s = 0.0;
                for (j = 0; j < m; ++j) s += AX(i, k + 1 + j) * v[j];
                s *= beta;
                for (j = 0; j < m; ++j) AX(i, k + 1 + j) -= s * v[j];
            }
            if (Q) {
                for (i = 0; i < n; ++i) {
                    double s = 0.0;
                    for (j = 0; j < m; ++j) s += QX(i, k + 1 + j) * v[j];
                    s *= beta;
                    for (j = 0; j < m; ++j) QX(i, k + 1 + j) -= s * v[j];
                }
            }
        }
        AX(k + 1, k) = alpha;
        for (i = k + 2; i < n; ++i) AX(i, k) = 0.0;
    }
    free(v);
    free(w);
    return 0;
}
