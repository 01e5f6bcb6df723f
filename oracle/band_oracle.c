/*
 * Oracle: plain FP64 CPU reference for the band Cholesky factorization
 * A = L L^T and the band triangular solves that use the factor.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the GPU path and never calls it.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math (no fused multiply-add, no
 * reassociation), so every sum below is evaluated in the order written, each
 * operation rounded once, with IEEE sqrt and division.
 *
 * Storage: LAPACK lower band layout, column-major, A(i,j) for 0 <= i-j <= k
 * at ab[(i-j) + j*ldab], ldab >= k+1 (the paper keeps the standard LAPACK
 * band format, Sections 3 and 6; lower, ldab = k+1 as the interface fixes).  Rows
 * k+1..ldab-1 and the bottom-right triangle past row n-1 are never touched.
 *
 * Definition followed: the Cholesky factor of an SPD matrix is the unique
 * lower-triangular L with positive diagonal and L L^T = A, and
 * it has the lower bandwidth of A (Section 2).  The factor routine is the paper's
 * left-looking band algorithm (Algorithm 2, Section 3.2), row by row:
 *     L(i,j) = (A(i,j) - sum_{l=max(0,i-k)}^{j-1} L(i,l) L(j,l)) / L(j,j),  j < i
 *     L(i,i) = sqrt(A(i,i) - sum_{l=max(0,i-k)}^{i-1} L(i,l)^2)
 * Reading of Algorithm 2: its inner sum is printed with upper bound j, which
 * would use L(i,j) and L(j,j) before they exist; the sum runs to j-1.
 * Failure rule (the paper is silent; LAPACK pbtrf convention): the first row i
 * whose pivot A(i,i) - sum is not > 0 (zero, negative or NaN) stops the
 * factorization with info = i + 1.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Row-band copy: R[i*(k+1) + t] = A(i, i-k+t), t = 0..k (t = k is the
 * diagonal), so that each row's band is contiguous.  Entries left of column 0
 * are zero and are never summed. */
static double *to_rows(int64_t n, int64_t k, const double *ab, int64_t ldab)
{
    int64_t w = k + 1;
    double *r = (double *)calloc((size_t)(n > 0 ? n : 1) * (size_t)w, sizeof(double));
    for (int64_t j = 0; j < n; ++j) {
        int64_t dmax = (k < n - 1 - j) ? k : n - 1 - j;
        for (int64_t d = 0; d <= dmax; ++d)
            r[(j + d) * w + (k - d)] = ab[d + j * ldab];
    }
    return r;
}

static void from_rows(int64_t n, int64_t k, const double *r, double *ab, int64_t ldab)
{
    int64_t w = k + 1;
    for (int64_t j = 0; j < n; ++j) {
        int64_t dmax = (k < n - 1 - j) ? k : n - 1 - j;
        for (int64_t d = 0; d <= dmax; ++d)
            ab[d + j * ldab] = r[(j + d) * w + (k - d)];
    }
}

static int64_t check_args(int64_t n, int64_t k, const void *ab, int64_t ldab)
{
    if (n < 0) return -1;
    if (k < 0) return -2;
    if (ab == NULL && n > 0) return -3;
    if (ldab < k + 1) return -4;
    return 0;
}

/* Row-oriented factorization in the row-band copy; returns info. */
static int64_t factor_rows(int64_t n, int64_t k, double *r)
{
    int64_t w = k + 1;
    for (int64_t i = 0; i < n; ++i) {
        int64_t lo = i - k > 0 ? i - k : 0;
        double *ri = r + i * w;
        for (int64_t j = lo; j <= i; ++j) {
            const double *rj = r + j * w;
            double t = 0.0;
            for (int64_t l = lo; l < j; ++l)
                t += ri[l - i + k] * rj[l - j + k];
            if (j == i) {
                double d = ri[k] - t;
                if (!(d > 0.0))
                    return i + 1;
                ri[k] = sqrt(d);
            } else {
                ri[j - i + k] = (ri[j - i + k] - t) / rj[k];
            }
        }
    }
    return 0;
}

/* A = L L^T in place; returns 0, -arg for an illegal argument, or info > 0. */
int64_t oracle_pbtrf(int64_t n, int64_t k, double *ab, int64_t ldab)
{
    int64_t bad = check_args(n, k, ab, ldab);
    if (bad) return bad;
    if (n == 0) return 0;
    double *r = to_rows(n, k, ab, ldab);
    int64_t info = factor_rows(n, k, r);
    if (info == 0)
        from_rows(n, k, r, ab, ldab);
    free(r);
    return info;
}

/*
 * The same per-entry arithmetic in column order (Crout): for each column j
 * the pivot first, then the k entries below it, which are independent and
 * may run on several threads.  Every entry is formed by the identical sum, in
 * the identical order, so the result equals oracle_pbtrf bit for bit; it only
 * finishes large cases sooner on a many-core host.
 */
int64_t oracle_pbtrf_columns(int64_t n, int64_t k, double *ab, int64_t ldab)
{
    int64_t bad = check_args(n, k, ab, ldab);
    if (bad) return bad;
    if (n == 0) return 0;
    int64_t w = k + 1;
    double *r = to_rows(n, k, ab, ldab);
    int64_t info = 0;
    for (int64_t j = 0; j < n && info == 0; ++j) {
        int64_t lo = j - k > 0 ? j - k : 0;
        double *rj = r + j * w;
        double t = 0.0;
        for (int64_t l = lo; l < j; ++l)
            t += rj[l - j + k] * rj[l - j + k];
        double d = rj[k] - t;
        if (!(d > 0.0)) { info = j + 1; break; }
        rj[k] = sqrt(d);
        int64_t imax = (j + k < n - 1) ? j + k : n - 1;
        #pragma omp parallel for schedule(static) if (k >= 64)
        for (int64_t i = j + 1; i <= imax; ++i) {
            double *ri = r + i * w;
            int64_t li = i - k > 0 ? i - k : 0;
            double s = 0.0;
            for (int64_t l = li; l < j; ++l)
                s += ri[l - i + k] * rj[l - j + k];
            ri[j - i + k] = (ri[j - i + k] - s) / rj[k];
        }
    }
    if (info == 0)
        from_rows(n, k, r, ab, ldab);
    free(r);
    return info;
}

/*
 * Solve A X = B with the factor: forward L y = b, then back L^T x = y.
 *   y_i = (b_i - sum_{l=max(0,i-k)}^{i-1} L(i,l) y_l) / L(i,i),       i ascending
 *   x_i = (y_i - sum_{l=i+1}^{min(n-1,i+k)} L(l,i) x_l) / L(i,i),     i descending
 * Sums run in ascending l.  B is n x nrhs column-major with ldb >= max(1, n).
 */
int64_t oracle_pbtrs(int64_t n, int64_t k, int64_t nrhs, const double *ab, int64_t ldab,
                     double *b, int64_t ldb)
{
    if (n < 0) return -1;
    if (k < 0) return -2;
    if (nrhs < 0) return -3;
    if (ab == NULL && n > 0) return -4;
    if (ldab < k + 1) return -5;
    if (b == NULL && n > 0 && nrhs > 0) return -6;
    if (ldb < (n > 1 ? n : 1)) return -7;
    if (n == 0 || nrhs == 0) return 0;
    double *r = to_rows(n, k, ab, ldab);
    int64_t w = k + 1;
    for (int64_t c = 0; c < nrhs; ++c) {
        double *y = b + c * ldb;
        for (int64_t i = 0; i < n; ++i) {
            int64_t lo = i - k > 0 ? i - k : 0;
            const double *ri = r + i * w;
            double t = 0.0;
            for (int64_t l = lo; l < i; ++l)
                t += ri[l - i + k] * y[l];
            y[i] = (y[i] - t) / ri[k];
        }
        for (int64_t i = n - 1; i >= 0; --i) {
            int64_t hi = (i + k < n - 1) ? i + k : n - 1;
            const double *col = ab + i * ldab;      /* L(l, i) = col[l - i] */
            double t = 0.0;
            for (int64_t l = i + 1; l <= hi; ++l)
                t += col[l - i] * y[l];
            y[i] = (y[i] - t) / col[0];
        }
    }
    free(r);
    return 0;
}

/* y = A x for the symmetric band matrix (lower storage), one vector. */
void oracle_band_symv(int64_t n, int64_t k, const double *ab, int64_t ldab, const double *x, double *y)
{
    for (int64_t i = 0; i < n; ++i) y[i] = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        y[j] += ab[j * ldab] * x[j];
        int64_t dmax = (k < n - 1 - j) ? k : n - 1 - j;
        for (int64_t d = 1; d <= dmax; ++d) {
            y[j + d] += ab[d + j * ldab] * x[j];
            y[j] += ab[d + j * ldab] * x[j + d];
        }
    }
}

/* ||A||_inf = ||A||_1 of the symmetric band matrix: largest absolute row sum. */
double oracle_band_norm_inf(int64_t n, int64_t k, const double *ab, int64_t ldab)
{
    double *rs = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    for (int64_t j = 0; j < n; ++j) {
        rs[j] += fabs(ab[j * ldab]);
        int64_t dmax = (k < n - 1 - j) ? k : n - 1 - j;
        for (int64_t d = 1; d <= dmax; ++d) {
            rs[j] += fabs(ab[d + j * ldab]);
            rs[j + d] += fabs(ab[d + j * ldab]);
        }
    }
    double m = 0.0;
    for (int64_t j = 0; j < n; ++j) if (rs[j] > m) m = rs[j];
    free(rs);
    return m;
}

/*
 * Squared Frobenius norms over rows [row_lo, row_hi) of the band, counting
 * each off-diagonal entry twice (it stands for A(i,j) and A(j,i)):
 *   out[0] = sum (L L^T - A)(i,j)^2,   out[1] = sum A(i,j)^2,
 * with (L L^T)(i,j) = sum_{l=max(0,i-k)}^{j} L(i,l) L(j,l).
 * Summing out[] over a partition of the rows gives ||L L^T - A||_F^2 and
 * ||A||_F^2; a row sample gives a sampled backward error.
 */
void oracle_llt_residual_rows(int64_t n, int64_t k, const double *l, int64_t ldl, const double *a,
                              int64_t lda, int64_t row_lo, int64_t row_hi, double *out)
{
    double num = 0.0, den = 0.0;
    if (row_hi > n) row_hi = n;
    for (int64_t i = row_lo; i < row_hi; ++i) {
        int64_t lo = i - k > 0 ? i - k : 0;
        for (int64_t j = lo; j <= i; ++j) {
            double s = 0.0;
            for (int64_t m = lo; m <= j; ++m)
                s += l[(i - m) + m * ldl] * l[(j - m) + m * ldl];
            double aij = a[(i - j) + j * lda];
            double wgt = (i == j) ? 1.0 : 2.0;
            num += wgt * (s - aij) * (s - aij);
            den += wgt * aij * aij;
        }
    }
    out[0] = num;
    out[1] = den;
}

/*
 * Operation count of the factorization loop nest above, counting one
 * multiply and one add per inner term, one subtraction and one sqrt or
 * division per entry (a sqrt counts as one operation, Section 3.2).
 */
int64_t oracle_pbtrf_opcount(int64_t n, int64_t k)
{
    int64_t ops = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t lo = i - k > 0 ? i - k : 0;
        for (int64_t j = lo; j <= i; ++j)
            ops += 2 * (j - lo) + 2;
    }
    return ops;
}

/*
 * Gradient of loss = sum(w .* x), x = A^{-1} b, with respect to the stored
 * band of the symmetric A, given x and lambda = A^{-1} w (n x nrhs each,
 * column-major).  The full-matrix gradient is -lambda x^T summed over the
 * right-hand sides; a stored entry A(i, j), i > j, stands for both A(i, j)
 * and A(j, i), so its gradient is the sum of the two:
 *   g(i, j) = -sum_r (lambda(i,r) x(j,r) + lambda(j,r) x(i,r)),  i > j,
 *   g(i, i) = -sum_r lambda(i,r) x(i,r).
 * Written to gab in the band layout (ldg >= k+1).
 */
void oracle_band_outer_grad(int64_t n, int64_t k, int64_t nrhs, const double *lam, int64_t ldl, const double *x,
                            int64_t ldx, double *gab, int64_t ldg)
{
    for (int64_t j = 0; j < n; ++j) {
        int64_t dmax = (k < n - 1 - j) ? k : n - 1 - j;
        for (int64_t d = 0; d <= dmax; ++d) {
            int64_t i = j + d;
            double g = 0.0;
            for (int64_t r = 0; r < nrhs; ++r) {
                g -= lam[i + r * ldl] * x[j + r * ldx];
                if (d > 0) g -= lam[j + r * ldl] * x[i + r * ldx];
            }
            gab[d + j * ldg] = g;
        }
    }
}

/*
 * Reverse mode of the factorization: given the factor L of A (band, LAPACK
 * layout) and an upstream gradient Lbar = dloss/dL on the band (lower
 * triangle), the gradient Abar = dloss/dA with respect to the stored band
 * entries -- the entries A(i, j), i >= j, that the factorization reads.
 *
 * It runs the steps of Algorithm 2 (Section 3.2) backwards, in exactly the
 * reverse of their forward order (rows i descending, within a row j
 * descending), propagating the adjoint of each step into the adjoints of the
 * values that step read.  Forward, entry (i, j) computes
 *     t = sum_{l=lo}^{j-1} L(i,l) L(j,l),   lo = max(0, i-k),
 *     L(i,i) = sqrt(A(i,i) - t)          (j = i),
 *     L(i,j) = (A(i,j) - t) / L(j,j)     (j < i).
 * Backwards, with W holding the accumulated adjoint of every L entry (Lbar at
 * the start):
 *     j = i:  Abar(i,i) = W(i,i) / (2 L(i,i)),        tbar = -Abar(i,i)
 *     j < i:  Abar(i,j) = W(i,j) / L(j,j),            tbar = -Abar(i,j),
 *             W(j,j) -= W(i,j) L(i,j) / L(j,j)
 *     then for l = lo .. j-1:  W(i,l) += tbar L(j,l),  W(j,l) += tbar L(i,l)
 * (for j = i both updates land on W(i,l), the derivative of L(i,l)^2).  When
 * entry (i, j) is reached every later step that read L(i,j) has already been
 * reversed, so W(i,j) is complete.  W lives in a row-band copy like the
 * forward routine's.  Lbar and Abar are in the band layout with leading
 * dimensions ldlb, ldab >= k+1 (they may be the same array).  L must be the
 * factor of a positive definite A (no zero pivots).
 */
void oracle_pbtrf_backward(int64_t n, int64_t k, const double *l, int64_t ldl, const double *lbar,
                           int64_t ldlb, double *abar, int64_t ldab)
{
    if (n <= 0) return;
    int64_t w = k + 1;
    double *r = to_rows(n, k, l, ldl);        /* L(i, i-k+t) */
    double *g = to_rows(n, k, lbar, ldlb);    /* W, the adjoints */
    double *a = (double *)calloc((size_t)n * (size_t)w, sizeof(double));
    for (int64_t i = n - 1; i >= 0; --i) {
        int64_t lo = i - k > 0 ? i - k : 0;
        double *ri = r + i * w, *gi = g + i * w, *ai = a + i * w;
        for (int64_t j = i; j >= lo; --j) {
            double *rj = r + j * w, *gj = g + j * w;
            double tbar;
            if (j == i) {
                ai[k] = gi[k] / (2.0 * ri[k]);
                tbar = -ai[k];
            } else {
                double lij = ri[j - i + k], ljj = rj[k];
                ai[j - i + k] = gi[j - i + k] / ljj;
                tbar = -ai[j - i + k];
                gj[k] -= gi[j - i + k] * lij / ljj;
            }
            for (int64_t l = lo; l < j; ++l) {
                gi[l - i + k] += tbar * rj[l - j + k];
                gj[l - j + k] += tbar * ri[l - i + k];
            }
        }
    }
    from_rows(n, k, a, abar, ldab);
    free(r);
    free(g);
    free(a);
}

/*
 * FP32 band Cholesky: Algorithm 2 (row by row, inner bound l <= j-1) with
 * every operation in single precision (float products and sums, sqrtf,
 * float division), on a float band in the LAPACK lower layout.  Used by the
 * mixed-precision reference; returns info as oracle_pbtrf.
 */
int64_t oracle_spbtrf(int64_t n, int64_t k, float *ab, int64_t ldab)
{
    if (n < 0) return -1;
    if (k < 0) return -2;
    if (ab == NULL && n > 0) return -3;
    if (ldab < k + 1) return -4;
    for (int64_t i = 0; i < n; ++i) {
        int64_t lo = i - k > 0 ? i - k : 0;
        for (int64_t j = lo; j <= i; ++j) {
            float t = 0.0f;
            for (int64_t l = lo; l < j; ++l)
                t += ab[(i - l) + l * ldab] * ab[(j - l) + l * ldab];
            if (i == j) {
                float d = ab[j * ldab] - t;
                if (!(d > 0.0f)) return i + 1;
                ab[j * ldab] = sqrtf(d);
            } else {
                ab[(i - j) + j * ldab] = (ab[(i - j) + j * ldab] - t) / ab[j * ldab];
            }
        }
    }
    return 0;
}
