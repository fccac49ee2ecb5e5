/*
 * oracle_evec.c -- plain, slow CPU reference for the eigenvector step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the test-suite loads it.  It shares no code,
 * header, table or constant with the HIP path.
 *
 * What it computes (paper Sec. 2, Eqs. (5) and (6)): for every eigenvalue
 * lambda of a real Schur form S (standardised 1x1 and 2x2 diagonal blocks),
 * a vector y with (S - lambda I) y = 0, found by back substitution one
 * eigenvector at a time in complex arithmetic, and its backtransform
 * x = Q y when Q is given.  The computation is protected against overflow
 * (the paper's point about this step, Sec. 3.1): the running vector is
 * scaled down whenever a division or an update could exceed a threshold.
 *
 * Readings where the paper is silent (the LAPACK conventions):
 *   - a real eigenvalue at position p: y(p) = 1, y(r) = 0 for r > p;
 *   - a complex pair at rows p, p+1 (S(p,p) = S(p+1,p+1) = a, b = S(p,p+1),
 *     c = S(p+1,p), b c < 0, wi = sqrt|b| sqrt|c|) for lambda = a + i wi:
 *     (y(p), y(p+1)) = (1, i wi / b) when |b| >= |c|, else (-wi / c, i);
 *   - a diagonal pivot (or 2x2 pivot) smaller than
 *     smin = max(ulp |lambda|, tiny) is replaced by smin;
 *   - output as LAPACK's: column k holds a real eigenvector, columns k and
 *     k+1 the real and imaginary parts of the eigenvector of a + i wi;
 *   - every returned vector is scaled so that its largest |Re| + |Im| is 1
 *     (after the backtransform when Q is given).
 * Storage: column-major with a leading dimension.  Precision: binary64
 * (C99 complex double), no BLAS or LAPACK.
 */
#include <complex.h>
#include <math.h>
#include <stddef.h>
#include <stdlib.h>

#define SX(i, j) S[(size_t)(i) + (size_t)(j) * (size_t)lds]
#define QX(i, j) Q[(size_t)(i) + (size_t)(j) * (size_t)ldq]
#define XX(i, j) X[(size_t)(i) + (size_t)(j) * (size_t)ldx]

static const double ORE_ULP = 2.220446049250313080847263336181640625e-16;   /* 2^-52 */
static const double ORE_TINY = 2.2250738585072014e-308;                      /* 2^-1022 */
static const double ORE_BIG = 1.0e290;     /* scaling threshold, far below overflow */

static double ore_cabs1(double complex z) { return fabs(creal(z)) + fabs(cimag(z)); }

static double ore_vmax(const double complex *y, int m)
{
    double v = 0.0;
    int i;
    for (i = 0; i < m; ++i) v = fmax(v, ore_cabs1(y[i]));
    return v;
}

static void ore_scale(double complex *y, int m, double f)
{
    int i;
    for (i = 0; i < m; ++i) y[i] *= f;
}

/* a pivot no smaller than smin in modulus (same direction) */
static double complex ore_pivot(double complex d, double smin)
{
    if (ore_cabs1(d) < smin) return (cabs(d) > 0.0) ? d * (smin / cabs(d)) : smin;
    return d;
}

/* Eigenvector of lambda (block at rows p .. p+s-1) into y[0 .. p+s-1].
 * rn[r] = sum over l > r of |S(r, l)| (row bounds of the updates). */
static void ore_vector(int n, const double *S, int lds, int p, int s, double complex lam,
                       const double *rn, double complex *y)
{
    const double smin = fmax(ORE_ULP * ore_cabs1(lam), ORE_TINY);
    int r, l;
    (void)n;
    if (s == 1) {
        y[p] = 1.0;
    } else {
        const double b = SX(p, p + 1), c = SX(p + 1, p), wi = cimag(lam);
        if (fabs(b) >= fabs(c)) { y[p] = 1.0; y[p + 1] = I * (wi / b); }
        else { y[p] = -wi / c; y[p + 1] = I; }
    }
    r = p - 1;
    while (r >= 0) {
        /* a 2x2 diagonal block ends at row r when S(r, r-1) != 0 */
        const int two = (r >= 1 && SX(r, r - 1) != 0.0);
        const int top = two ? r - 1 : r;
        const int top_known = p + s;           /* y(top+k) known for rows > r */
        double complex f0 = 0.0, f1 = 0.0;
        const double ymax = ore_vmax(y + r + 1, top_known - r - 1);
        const double rb = two ? fmax(rn[top], rn[r]) : rn[r];
        /* the updates could exceed the threshold (rb ymax > BIG, tested
         * without forming the product): scale the vector first */
        if (rb > 0.0 && ymax > ORE_BIG / rb) ore_scale(y + r + 1, top_known - r - 1, (ORE_BIG / rb) / ymax);
        for (l = r + 1; l < top_known; ++l) {
            f1 -= SX(r, l) * y[l];
            if (two) f0 -= SX(top, l) * y[l];
        }
        if (!two) {
            const double complex d = ore_pivot(SX(r, r) - lam, smin);
            const double fm = ore_cabs1(f1);
            if (fm > ORE_BIG * ore_cabs1(d)) {   /* the quotient would be too large */
                const double g = ORE_BIG * ore_cabs1(d) / fm;
                ore_scale(y + r + 1, top_known - r - 1, g);
                f1 *= g;
            }
            y[r] = f1 / d;
        } else {
            /* [a11 a12; a21 a22] (y(top), y(r)) = (f0, f1), partial pivoting */
            double complex a11 = SX(top, top) - lam, a12 = SX(top, r);
            double complex a21 = SX(r, top), a22 = SX(r, r) - lam;
            double complex u1, u2, m, p22;
            int swap = ore_cabs1(a21) > ore_cabs1(a11);
            if (swap) {
                double complex t;
                t = a11; a11 = a21; a21 = t;
                t = a12; a12 = a22; a22 = t;
                t = f0; f0 = f1; f1 = t;
            }
            a11 = ore_pivot(a11, smin);
            m = a21 / a11;
            p22 = ore_pivot(a22 - m * a12, smin);
            f1 = f1 - m * f0;
            {
                const double fm = fmax(ore_cabs1(f0), ore_cabs1(f1));
                const double dm = fmin(ore_cabs1(a11), ore_cabs1(p22)) / (1.0 + ore_cabs1(a12));
                if (fm > ORE_BIG * dm) {
                    const double g = ORE_BIG * dm / fm;
                    ore_scale(y + r + 1, top_known - r - 1, g);
                    f0 *= g;
                    f1 *= g;
                }
            }
            u2 = f1 / p22;
            u1 = (f0 - a12 * u2) / a11;
            y[top] = u1;
            y[r] = u2;
        }
        r = top - 1;
    }
}

/* Eigenvectors of the real Schur form S (n x n, lds); X (ldx) receives them
 * in LAPACK's real layout; when Q (ldq) is given, X = Q Y.  Returns 0, or -1
 * when the workspace cannot be allocated. */
int oracle_eigenvectors(int n, const double *S, int lds, const double *Q, int ldq, double *X,
                        int ldx)
{
    double complex *y = (double complex *)malloc(sizeof(double complex) * (size_t)(n + 1));
    double complex *x = (double complex *)malloc(sizeof(double complex) * (size_t)(n + 1));
    double *rn = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    int k, r, l;
    if (!y || !x || !rn) { free(y); free(x); free(rn); return -1; }
    for (r = 0; r < n; ++r) {
        double t = 0.0;
        for (l = r + 1; l < n; ++l) t += fabs(SX(r, l));
        rn[r] = t;
    }
    k = 0;
    while (k < n) {
        const int s = (k + 1 < n && SX(k + 1, k) != 0.0) ? 2 : 1;
        double complex lam;
        int m = k + s;   /* entries 0 .. m-1 of y may be nonzero */
        double emax;
        if (s == 1) lam = SX(k, k);
        else lam = SX(k, k) + I * sqrt(fabs(SX(k, k + 1))) * sqrt(fabs(SX(k + 1, k)));
        for (r = 0; r < n; ++r) y[r] = 0.0;
        ore_vector(n, S, lds, k, s, lam, rn, y);
        if (Q) {   /* backtransform x = Q y */
            for (r = 0; r < n; ++r) {
                double complex t = 0.0;
                for (l = 0; l < m; ++l) t += QX(r, l) * y[l];
                x[r] = t;
            }
            m = n;
        } else {
            for (r = 0; r < n; ++r) x[r] = y[r];
        }
        emax = ore_vmax(x, m);
        if (emax > 0.0) ore_scale(x, m, 1.0 / emax);
        for (r = 0; r < n; ++r) {
            XX(r, k) = creal(x[r]);
            if (s == 2) XX(r, k + 1) = cimag(x[r]);
        }
        k += s;
    }
    free(y);
    free(x);
    free(rn);
    return 0;
}
