/*
 * oracle_reorder.c -- plain, slow CPU reference for eigenvalue reordering.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the test-suite loads it.  It shares no code,
 * header, table or constant with the HIP path.
 *
 * What it computes (paper Sec. 2, Eq. (7)): for a standardised real Schur
 * form S and a selection of its eigenvalues, an orthogonal Q3 with
 * S = Q3 S' Q3^T where S' is again a standardised real Schur form whose
 * leading diagonal blocks carry exactly the selected eigenvalues; Q is
 * accumulated (Q <- Q Q3).  The paper names the tools (Sec. 3.2): sequences
 * of overlapping Givens rotations and 3x3 Householder reflectors.  This file
 * moves every selected block, in diagonal order, to the top of the part not
 * yet ordered by swapping it with its upper neighbour again and again
 * (Golub & Van Loan, Sec. 7.6.2); a swap of two adjacent diagonal blocks is
 *   - for two 1x1 blocks, a Givens rotation whose first column is the
 *     eigenvector of the lower eigenvalue;
 *   - otherwise direct swapping (Bai & Demmel): X solves the Sylvester
 *     equation T11 X - X T22 = T12, the columns of [-X; I] span the
 *     invariant subspace of T22's eigenvalues, and the orthogonal factor of
 *     their Householder QR (reflectors of order 3 or 4, then 2 or 3)
 *     exchanges the blocks; new 2x2 blocks are standardised.
 *
 * Readings where the paper is silent (the LAPACK conventions):
 *   - select[k] != 0 selects eigenvalue k; either entry of a 2x2 block
 *     selects the pair;
 *   - a swap is rejected when the part of the transformed block that must
 *     vanish is larger than 20 ulp max|T| (then the reordering stops and
 *     returns 1, S and Q holding the last accepted state);
 *   - a Sylvester pivot below max(ulp max|T|, tiny) is raised to it.
 * Storage: column-major with a leading dimension.  Precision: binary64,
 * no BLAS or LAPACK.
 */
#include <math.h>
#include <stddef.h>
#include <string.h>

#define SX(i, j) S[(size_t)(i) + (size_t)(j) * (size_t)lds]
#define QX(i, j) Q[(size_t)(i) + (size_t)(j) * (size_t)ldq]

static const double ORR_ULP = 2.220446049250313080847263336181640625e-16;   /* 2^-52 */
static const double ORR_TINY = 2.2250738585072014e-308;

/* the oracle's 2x2 standardisation (oracle_schur.c) */
void oracle_std2x2(double a, double b, double c, double d, double *out);

/* block size at row k of a standardised Schur form */
static int orr_bsize(int n, const double *S, int lds, int k)
{
    return (k + 1 < n && SX(k + 1, k) != 0.0) ? 2 : 1;
}

/* apply the orthogonal m x m matrix G (column-major, ld m) to rows and
 * columns j .. j+m-1: S <- G^T S G, Q <- Q G */
static void orr_apply(int n, double *S, int lds, double *Q, int ldq, int j, int m,
                      const double *G)
{
    double t[4];
    int r, c, a, b;
    for (c = j; c < n; ++c) {            /* rows j..j+m-1 from the left */
        for (a = 0; a < m; ++a) {
            double s = 0.0;
            for (b = 0; b < m; ++b) s += G[b + a * m] * SX(j + b, c);
            t[a] = s;
        }
        for (a = 0; a < m; ++a) SX(j + a, c) = t[a];
    }
    for (r = 0; r < j + m; ++r) {        /* columns j..j+m-1 from the right */
        for (a = 0; a < m; ++a) {
            double s = 0.0;
            for (b = 0; b < m; ++b) s += SX(r, j + b) * G[b + a * m];
            t[a] = s;
        }
        for (a = 0; a < m; ++a) SX(r, j + a) = t[a];
    }
    if (Q) {
        for (r = 0; r < n; ++r) {
            for (a = 0; a < m; ++a) {
                double s = 0.0;
                for (b = 0; b < m; ++b) s += QX(r, j + b) * G[b + a * m];
                t[a] = s;
            }
            for (a = 0; a < m; ++a) QX(r, j + a) = t[a];
        }
    }
}

/* standardise a 2x2 block at rows i-1, i (rotation on the full matrix) */
static void orr_std(int n, double *S, int lds, double *Q, int ldq, int i)
{
    double o[10], G[4];
    oracle_std2x2(SX(i - 1, i - 1), SX(i - 1, i), SX(i, i - 1), SX(i, i), o);
    G[0] = o[4]; G[1] = o[5]; G[2] = -o[5]; G[3] = o[4];   /* [[cs, -sn], [sn, cs]] */
    orr_apply(n, S, lds, Q, ldq, i - 1, 2, G);
    SX(i - 1, i - 1) = o[0]; SX(i - 1, i) = o[1]; SX(i, i - 1) = o[2]; SX(i, i) = o[3];
}

/* Householder reflector of x (length m): I - tau v v^T, v[0] = 1, maps x to
 * (beta, 0, ...); tau = 0 for a zero tail */
static void orr_house(int m, const double *x, double *v, double *tau)
{
    double tail = 0.0, nrm, beta;
    int i;
    for (i = 1; i < m; ++i) tail = hypot(tail, x[i]);
    v[0] = 1.0;
    if (tail == 0.0) {
        for (i = 1; i < m; ++i) v[i] = 0.0;
        *tau = 0.0;
        return;
    }
    nrm = hypot(x[0], tail);
    beta = (x[0] >= 0.0) ? -nrm : nrm;
    for (i = 1; i < m; ++i) v[i] = x[i] / (x[0] - beta);
    *tau = (beta - x[0]) / beta;
}

/* Solve T11 X - X T22 = T12 (n1 x n2, each <= 2) through its Kronecker
 * form, Gaussian elimination with complete pivoting. */
static void orr_sylvester(int n1, int n2, const double *T, int ldt, double smin, double *X)
{
    double K[16], rhs[4];
    int perm[4], N = n1 * n2, i, j, k, p, q;
    memset(K, 0, sizeof(K));
    /* unknown x(i, j) is number i + n1 j */
    for (j = 0; j < n2; ++j)
        for (i = 0; i < n1; ++i) {
            const int row = i + n1 * j;
            for (k = 0; k < n1; ++k) K[row + 4 * (k + n1 * j)] += T[i + k * ldt];          /* T11 */
            for (k = 0; k < n2; ++k) K[row + 4 * (i + n1 * k)] -= T[(n1 + k) + (n1 + j) * ldt]; /* X T22 */
            rhs[row] = T[i + (n1 + j) * ldt];
        }
    for (i = 0; i < N; ++i) perm[i] = i;
    for (k = 0; k < N; ++k) {
        int pr = k, pc = k;
        double best = -1.0;
        for (p = k; p < N; ++p)
            for (q = k; q < N; ++q)
                if (fabs(K[p + 4 * q]) > best) { best = fabs(K[p + 4 * q]); pr = p; pc = q; }
        if (pr != k) {
            for (q = 0; q < N; ++q) { double t = K[k + 4 * q]; K[k + 4 * q] = K[pr + 4 * q]; K[pr + 4 * q] = t; }
            { double t = rhs[k]; rhs[k] = rhs[pr]; rhs[pr] = t; }
        }
        if (pc != k) {
            for (p = 0; p < N; ++p) { double t = K[p + 4 * k]; K[p + 4 * k] = K[p + 4 * pc]; K[p + 4 * pc] = t; }
            { int t = perm[k]; perm[k] = perm[pc]; perm[pc] = t; }
        }
        if (fabs(K[k + 4 * k]) < smin) K[k + 4 * k] = (K[k + 4 * k] >= 0.0) ? smin : -smin;
        for (p = k + 1; p < N; ++p) {
            const double f = K[p + 4 * k] / K[k + 4 * k];
            for (q = k; q < N; ++q) K[p + 4 * q] -= f * K[k + 4 * q];
            rhs[p] -= f * rhs[k];
        }
    }
    {
        double sol[4];
        for (k = N - 1; k >= 0; --k) {
            double s = rhs[k];
            for (q = k + 1; q < N; ++q) s -= K[k + 4 * q] * sol[q];
            sol[k] = s / K[k + 4 * k];
        }
        for (k = 0; k < N; ++k) X[perm[k]] = sol[k];   /* X(i, j) at i + n1 j */
    }
}

/* Swap the adjacent blocks of orders n1 (rows j..j+n1-1) and n2 below it.
 * Returns 0, or 1 when the swap is rejected (S and Q unchanged). */
static int orr_swap(int n, double *S, int lds, double *Q, int ldq, int j, int n1, int n2)
{
    const int m = n1 + n2;
    double T[16], G[16], D[16], tmax = 0.0;
    int a, b, c;
    for (b = 0; b < m; ++b)
        for (a = 0; a < m; ++a) {
            T[a + 4 * b] = SX(j + a, j + b);
            tmax = fmax(tmax, fabs(T[a + 4 * b]));
        }
    if (n1 == 1 && n2 == 1) {
        /* first column: eigenvector of t22, (t12, t22 - t11) */
        const double t11 = T[0], t12 = T[4], t22 = T[5];
        const double x = t12, y = t22 - t11, r = hypot(x, y);
        if (r == 0.0) return 0;   /* equal eigenvalues, t12 = 0: nothing to do */
        G[0] = x / r; G[1] = y / r; G[2] = -y / r; G[3] = x / r;
        orr_apply(n, S, lds, Q, ldq, j, 2, G);
        SX(j, j) = t22; SX(j + 1, j + 1) = t11; SX(j + 1, j) = 0.0;
        return 0;
    } else {
        const double smin = fmax(ORR_ULP * tmax, ORR_TINY);
        double X[4], B[16], v[4], tau;
        int k, col;
        orr_sylvester(n1, n2, T, 4, smin, X);
        /* B = [-X; I] (m x n2), Householder QR; G = H_1 ... H_n2 */
        memset(B, 0, sizeof(B));
        for (b = 0; b < n2; ++b) {
            for (a = 0; a < n1; ++a) B[a + 4 * b] = -X[a + n1 * b];
            B[n1 + b + 4 * b] = 1.0;
        }
        memset(G, 0, sizeof(G));
        for (a = 0; a < m; ++a) G[a + m * a] = 1.0;
        for (k = 0; k < n2; ++k) {
            double x[4];
            const int len = m - k;
            for (a = 0; a < len; ++a) x[a] = B[k + a + 4 * k];
            orr_house(len, x, v, &tau);
            if (tau == 0.0) continue;
            for (col = k; col < n2; ++col) {       /* B <- H B */
                double s = 0.0;
                for (a = 0; a < len; ++a) s += v[a] * B[k + a + 4 * col];
                s *= tau;
                for (a = 0; a < len; ++a) B[k + a + 4 * col] -= s * v[a];
            }
            for (a = 0; a < m; ++a) {              /* G <- G H */
                double s = 0.0;
                for (c = 0; c < len; ++c) s += G[a + m * (k + c)] * v[c];
                s *= tau;
                for (c = 0; c < len; ++c) G[a + m * (k + c)] -= s * v[c];
            }
        }
        /* D = G^T T G; its lower-left n1 x n2 block must vanish */
        for (b = 0; b < m; ++b)
            for (a = 0; a < m; ++a) {
                double s = 0.0;
                int p, q;
                for (p = 0; p < m; ++p)
                    for (q = 0; q < m; ++q) s += G[p + m * a] * T[p + 4 * q] * G[q + m * b];
                D[a + 4 * b] = s;
            }
        {
            double low = 0.0;
            for (b = 0; b < n2; ++b)
                for (a = n2; a < m; ++a) low = fmax(low, fabs(D[a + 4 * b]));
            if (low > 20.0 * ORR_ULP * tmax) return 1;
        }
        orr_apply(n, S, lds, Q, ldq, j, m, G);
        for (b = 0; b < n2; ++b)   /* the part that vanishes: exact zeros */
            for (a = n2; a < m; ++a) SX(j + a, j + b) = 0.0;
        if (n2 == 2) orr_std(n, S, lds, Q, ldq, j + 1);
        if (n1 == 2) orr_std(n, S, lds, Q, ldq, j + n2 + 1);
        return 0;
    }
}

/* Reorder S (n x n, lds) so that the selected eigenvalues lead; Q (ldq) is
 * accumulated when given; wr/wi receive the eigenvalues of the result in
 * diagonal order and *m the number of selected ones.  Returns 0, or 1 when
 * a swap was rejected (the eigenvalues are then as S holds them). */
int oracle_reorder(int n, double *S, int lds, double *Q, int ldq, const int *select, double *wr,
                   double *wi, int *m)
{
    int k = 0, ks = 0, info = 0;
    while (k < n && !info) {
        const int s = orr_bsize(n, S, lds, k);
        const int sel = select[k] || (s == 2 && select[k + 1]);
        if (sel) {
            int pos = k;
            while (pos > ks) {
                const int s_up = (pos >= 2 && SX(pos - 1, pos - 2) != 0.0) ? 2 : 1;
                const int cur = orr_bsize(n, S, lds, pos);
                if (orr_swap(n, S, lds, Q, ldq, pos - s_up, s_up, cur)) { info = 1; break; }
                pos -= s_up;
            }
            /* a 2x2 block that split into two 1x1 blocks on the way still
             * occupies rows ks, ks+1 */
            if (!info) ks += s;
        }
        k += s;
    }
    if (m) *m = ks;
    for (k = 0; k < n;) {
        const int s = orr_bsize(n, S, lds, k);
        if (s == 1) {
            wr[k] = SX(k, k); wi[k] = 0.0;
        } else {
            const double w = sqrt(fabs(SX(k, k + 1))) * sqrt(fabs(SX(k + 1, k)));
            wr[k] = SX(k, k); wi[k] = w;
            wr[k + 1] = SX(k + 1, k + 1); wi[k + 1] = -w;
        }
        k += s;
    }
    return info;
}
