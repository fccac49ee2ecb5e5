/*
 * oracle_schur.c -- plain, slow CPU reference for the Schur-reduction step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header, table
 * or constant with the HIP path.
 *
 * What it computes (paper Sec. 2, Eq. (4), the Schur reduction): given an
 * upper Hessenberg H, an orthogonal Q2 and an upper quasi-triangular S with
 * 1x1 and 2x2 diagonal blocks such that H = Q2 S Q2^T; the eigenvalues are
 * read from the diagonal blocks.  The paper defers the theory to Golub & Van
 * Loan, "Matrix Computations" (cited at the end of Sec. 2); this file follows
 * the practical QR algorithm of that text (Sec. 7.5: the Francis double-shift
 * step, deflation on negligible subdiagonal entries, and the QR iteration on
 * the remaining unreduced block) in its own code:
 *
 *   - Francis double-shift step: the first column of (H - s1 I)(H - s2 I)
 *     has three nonzeros; a 3x3 Householder reflector built from it creates a
 *     bulge that further 3x3 reflectors chase to the bottom of the unreduced
 *     block; the last reflector is 2x2.
 *   - Deflation: |h(k,k-1)| <= ulp * (|h(k-1,k-1)| + |h(k,k)|) sets h(k,k-1)
 *     to exactly zero (readings: ties count as negligible; a zero sum falls
 *     back to the 1-norm of the leading active part).
 *   - Exceptional shifts after 10 and 20 non-deflating steps (Wilkinson &
 *     Reinsch style ad-hoc 2x2 with constants 0.75 and -0.4375).
 *   - 2x2 standardisation of converged blocks: complex pair -> equal
 *     diagonal entries and b*c < 0; real pair -> split into two 1x1 blocks.
 *
 * Storage: column-major with a leading dimension (ScaLAPACK/LAPACK
 * convention the paper keeps compatibility with, Sec. 4.2).  Q is
 * accumulated: Q <- Q_in * Q2 (Sec. 2, Eq. (6) uses the product Q1 Q2).
 * Precision: IEEE binary64 throughout; no BLAS or LAPACK.
 *
 * Readings where the paper is silent are listed beside each function.
 */
#include <math.h>
#include <stddef.h>
#include <string.h>

#define HX(i, j) H[(size_t)(i) + (size_t)(j) * (size_t)ldh]
#define QX(i, j) Q[(size_t)(i) + (size_t)(j) * (size_t)ldq]

static const double ORC_ULP = 2.220446049250313080847263336181640625e-16; /* 2^-52 */

/* Householder vector for a column (x, y, z) (z ignored when nr == 2):
 * find tau, v = (1, v2, v3) and beta with (I - tau v v^T) (x,y,z)^T = (beta,0,0)^T.
 * beta = -sign(x) * ||(x,y,z)||, sign(0) = +1.  A zero tail gives tau = 0. */
static void orc_house(int nr, double x, double y, double z,
                      double *tau, double *v2, double *v3, double *beta)
{
    double tail;
    if (nr == 2) z = 0.0;
    tail = fabs(y) + fabs(z);
    if (tail == 0.0) {
        *tau = 0.0; *v2 = 0.0; *v3 = 0.0; *beta = x;
        return;
    }
    {
        /* scale to avoid overflow in the squares */
        double s = fabs(x) + tail;
        double xs = x / s, ys = y / s, zs = z / s;
        double nrm = s * sqrt(xs * xs + ys * ys + zs * zs);
        double b = (x >= 0.0) ? -nrm : nrm;
        double d = x - b;
        *beta = b;
        *tau = (b - x) / b;
        *v2 = y / d;
        *v3 = z / d;
    }
}

/* Apply reflector rows r..r+nr-1 of H from the left, columns c0..c1. */
static void orc_left(double *H, int ldh, int r, int nr, int c0, int c1,
                     double tau, double v2, double v3)
{
    int c;
    for (c = c0; c <= c1; ++c) {
        double a1 = HX(r, c), a2 = HX(r + 1, c);
        double a3 = (nr == 3) ? HX(r + 2, c) : 0.0;
        double w = a1 + v2 * a2 + v3 * a3;
        HX(r, c) = a1 - tau * w;
        HX(r + 1, c) = a2 - tau * w * v2;
        if (nr == 3) HX(r + 2, c) = a3 - tau * w * v3;
    }
}

/* Apply reflector columns r..r+nr-1 of A from the right, rows r0..r1. */
static void orc_right(double *A, int lda, int r, int nr, int r0, int r1,
                      double tau, double v2, double v3)
{
    int i;
    for (i = r0; i <= r1; ++i) {
        double *p1 = &A[(size_t)i + (size_t)r * lda];
        double *p2 = &A[(size_t)i + (size_t)(r + 1) * lda];
        double *p3 = (nr == 3) ? &A[(size_t)i + (size_t)(r + 2) * lda] : NULL;
        double a1 = *p1, a2 = *p2, a3 = p3 ? *p3 : 0.0;
        double w = a1 + v2 * a2 + v3 * a3;
        *p1 = a1 - tau * w;
        *p2 = a2 - tau * w * v2;
        if (p3) *p3 = a3 - tau * w * v3;
    }
}

static void orc_rot2(double a, double b, double c, double d, double cs, double sn,
                     double *na, double *nb, double *nc, double *nd)
{
    /* B' = G^T B G with G = [[cs, -sn], [sn, cs]] */
    double t11 = a * cs + b * sn, t12 = -a * sn + b * cs;
    double t21 = c * cs + d * sn, t22 = -c * sn + d * cs;
    *na = cs * t11 + sn * t21;
    *nb = cs * t12 + sn * t22;
    *nc = -sn * t11 + cs * t21;
    *nd = -sn * t12 + cs * t22;
}

/*
 * Standardise one 2x2 block [[a, b], [c, d]] (paper Sec. 2: S has 1x1 and
 * 2x2 diagonal blocks and the eigenvalues are read from them).
 * Reading of the standard form: complex pair -> a' = d' and b'*c' < 0;
 * real pair -> c' = 0 (the block splits into two 1x1 blocks).
 * Derivation: with p = (a+d)/2, al = (a-d)/2, be = (b+c)/2, ga = (b-c)/2 the
 * block is p I + al diag(1,-1) + be [[0,1],[1,0]] + ga [[0,1],[-1,0]].  A plane
 * rotation G = [[cs,-sn],[sn,cs]] leaves p and ga unchanged and turns
 * (al, be) by twice its angle; the eigenvalues are p +- sqrt(al^2 + b c).
 * Outputs the rotation (cs, sn), the new block and the two eigenvalues
 * (wr1 + i wi1, wr2 + i wi2), wi1 >= 0 >= wi2.
 */
void oracle_std2x2(double a, double b, double c, double d,
                   double *out /* a', b', c', d', cs, sn, wr1, wi1, wr2, wi2 */)
{
    double cs = 1.0, sn = 0.0;
    double al = 0.5 * (a - d);
    double disc = al * al + b * c;
    double na = a, nb = b, nc = c, nd = d;
    int real_pair = (c == 0.0) || (disc >= 0.0);
    if (c != 0.0 && !real_pair) {
        /* complex pair: pick 2*theta with al*cos2t + be*sin2t = 0 */
        double be = 0.5 * (b + c);
        double rr = hypot(al, be);
        if (rr != 0.0) {
            double C = be / rr, S = -al / rr;
            if (C < 0.0) { C = -C; S = -S; }
            cs = sqrt(0.5 * (1.0 + C));
            sn = S / (2.0 * cs);
        }
        orc_rot2(a, b, c, d, cs, sn, &na, &nb, &nc, &nd);
        na = nd = 0.5 * (na + nd);
        if (nb * nc >= 0.0) { real_pair = 1; disc = 0.0; }
    }
    if (c != 0.0 && real_pair) {
        /* real pair: first column of G is an eigenvector for
         * l1 = p + sg*r, taken as (l1 - d, c) to avoid cancellation */
        double r = sqrt(disc > 0.0 ? disc : 0.0);
        double sg = (al >= 0.0) ? 1.0 : -1.0;
        double v1 = al + sg * r, v2 = c;
        double nv = hypot(v1, v2);
        cs = v1 / nv; sn = v2 / nv;
        orc_rot2(a, b, c, d, cs, sn, &na, &nb, &nc, &nd);
        nc = 0.0;
    }
    out[0] = na; out[1] = nb; out[2] = nc; out[3] = nd;
    out[4] = cs; out[5] = sn;
    if (nc == 0.0) {
        out[6] = na; out[7] = 0.0; out[8] = nd; out[9] = 0.0;
    } else {
        double wi = sqrt(fabs(nb)) * sqrt(fabs(nc));
        out[6] = na; out[7] = wi; out[8] = nd; out[9] = -wi;
    }
}

/* Standardise the isolated block at rows/cols (i-1, i) of the n x n matrix
 * and apply the rotation to the rest of H (rows i-1..i from column i-1 on,
 * columns i-1..i for rows 0..i) and to Q (all rows). */
static void orc_std_block(int n, double *H, int ldh, double *Q, int ldq, int i,
                          double *wr, double *wi)
{
    double o[10];
    int j;
    oracle_std2x2(HX(i - 1, i - 1), HX(i - 1, i), HX(i, i - 1), HX(i, i), o);
    {
        double cs = o[4], sn = o[5];
        if (!(cs == 1.0 && sn == 0.0)) {
            for (j = i + 1; j < n; ++j) {           /* rows i-1, i right of block */
                double x = HX(i - 1, j), y = HX(i, j);
                HX(i - 1, j) = cs * x + sn * y;
                HX(i, j) = -sn * x + cs * y;
            }
            for (j = 0; j < i - 1; ++j) {           /* cols i-1, i above block */
                double x = HX(j, i - 1), y = HX(j, i);
                HX(j, i - 1) = cs * x + sn * y;
                HX(j, i) = -sn * x + cs * y;
            }
            if (Q) {
                for (j = 0; j < n; ++j) {
                    double x = QX(j, i - 1), y = QX(j, i);
                    QX(j, i - 1) = cs * x + sn * y;
                    QX(j, i) = -sn * x + cs * y;
                }
            }
        }
        HX(i - 1, i - 1) = o[0]; HX(i - 1, i) = o[1];
        HX(i, i - 1) = o[2];     HX(i, i) = o[3];
    }
    wr[i - 1] = o[6]; wi[i - 1] = o[7];
    wr[i] = o[8];     wi[i] = o[9];
}

/*
 * One Francis double-shift step on the unreduced block l..i (0-based,
 * i - l >= 2) with shift sum s and product t, applied with the full-matrix
 * (Schur form) convention: left updates run to column n-1, right updates
 * start at row 0, and Q (if not NULL) accumulates the reflectors.
 */
void oracle_francis_step(int n, double *H, int ldh, double *Q, int ldq,
                         int l, int i, double s, double t)
{
    int r;
    double h00 = HX(l, l), h01 = HX(l, l + 1), h10 = HX(l + 1, l);
    double h11 = HX(l + 1, l + 1), h21 = HX(l + 2, l + 1);
    /* first column of (H - s1 I)(H - s2 I) = H^2 - s H + t I */
    double x = h00 * h00 + h01 * h10 - s * h00 + t;
    double y = h10 * (h00 + h11 - s);
    double z = h10 * h21;
    for (r = l; r <= i - 1; ++r) {
        int nr = (r <= i - 2) ? 3 : 2;
        double tau, v2, v3, beta;
        int rmax;
        if (r > l) {
            x = HX(r, r - 1);
            y = HX(r + 1, r - 1);
            z = (nr == 3) ? HX(r + 2, r - 1) : 0.0;
        }
        orc_house(nr, x, y, z, &tau, &v2, &v3, &beta);
        if (tau == 0.0) continue;
        if (r > l) {
            HX(r, r - 1) = beta;
            HX(r + 1, r - 1) = 0.0;
            if (nr == 3) HX(r + 2, r - 1) = 0.0;
        }
        orc_left(H, ldh, r, nr, r, n - 1, tau, v2, v3);
        rmax = (r + 3 < i) ? r + 3 : i;
        orc_right(H, ldh, r, nr, 0, rmax, tau, v2, v3);
        if (Q) orc_right(Q, ldq, r, nr, 0, n - 1, tau, v2, v3);
    }
}

/* 1-norm of the leading (i+1) x (i+1) part */
static double orc_norm1(const double *H, int ldh, int i)
{
    double best = 0.0;
    int j, k;
    for (j = 0; j <= i; ++j) {
        double s = 0.0;
        for (k = 0; k <= i && k <= j + 1; ++k) s += fabs(HX(k, j));
        if (s > best) best = s;
    }
    return best;
}

/*
 * Real Schur form of an upper Hessenberg matrix (paper Sec. 2, Eq. (4)).
 *   n        order (n >= 0)
 *   H        column-major, ldh >= max(1,n); entries below the first
 *            subdiagonal are ignored (set to zero on entry); overwritten by S
 *   Q        NULL, or column-major n x n (ldq >= max(1,n)); Q <- Q * Q2
 *   wr, wi   eigenvalues in diagonal order, conjugate pairs adjacent with
 *            the positive imaginary part first
 *   itmax    non-deflating steps allowed per block end (<= 0 -> 30)
 *   iters    optional: total Francis steps taken
 * Returns 0, or i+1 (1-based end of the unreduced block) when a block end
 * needed more than itmax steps; H = Q S Q^T still holds then.
 */
int oracle_schur(int n, double *H, int ldh, double *Q, int ldq,
                 double *wr, double *wi, int itmax, int *iters)
{
    int i, j, its, total = 0;
    if (itmax <= 0) itmax = 30;
    if (iters) *iters = 0;
    if (n <= 0) return 0;
    for (j = 0; j < n; ++j)
        for (i = j + 2; i < n; ++i) HX(i, j) = 0.0;

    i = n - 1;
    its = 0;
    while (i >= 0) {
        int l = 0, k;
        double s, t;
        /* deflation search, bottom-up */
        for (k = i; k >= 1; --k) {
            double sub = fabs(HX(k, k - 1));
            double tst = fabs(HX(k - 1, k - 1)) + fabs(HX(k, k));
            if (tst == 0.0) tst = orc_norm1(H, ldh, i);
            if (sub <= ORC_ULP * tst) {
                HX(k, k - 1) = 0.0;
                l = k;
                break;
            }
        }
        if (l == i) {
            wr[i] = HX(i, i); wi[i] = 0.0;
            i -= 1; its = 0;
            continue;
        }
        if (l == i - 1) {
            orc_std_block(n, H, ldh, Q, ldq, i, wr, wi);
            i -= 2; its = 0;
            continue;
        }
        its += 1;
        if (its > itmax) {
            if (iters) *iters = total;
            return i + 1;
        }
        if (its == 10 || its == 20) {
            /* exceptional shift (reading): the ad-hoc 2x2 [[e, w], [-0.4375 w, e]]
             * with e = h + 0.75 w, where w sums two subdiagonal magnitudes
             * taken from the bottom (step 10) or the top (step 20) of the block;
             * its eigenvalues are e +- i sqrt(0.4375) w */
            double w, e;
            if (its == 10) {
                w = fabs(HX(i, i - 1)) + fabs(HX(i - 1, i - 2));
                e = HX(i, i) + 0.75 * w;
            } else {
                w = fabs(HX(l + 1, l)) + fabs(HX(l + 2, l + 1));
                e = HX(l, l) + 0.75 * w;
            }
            s = 2.0 * e;
            t = e * e + 0.4375 * w * w;
        } else {
            double a = HX(i - 1, i - 1), b = HX(i - 1, i);
            double c = HX(i, i - 1), d = HX(i, i);
            s = a + d;
            t = a * d - b * c;
        }
        oracle_francis_step(n, H, ldh, Q, ldq, l, i, s, t);
        total += 1;
    }
    if (iters) *iters = total;
    return 0;
}
