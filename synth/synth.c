/*
 * Seeded synthetic inputs for the band Cholesky factor + solve.
 *
 * This module is shared by the tests, the oracle checks and the benchmark.
 * It holds no step of the factorization or of the triangular solves: only
 * random draws and the construction of the test matrices and right-hand
 * sides (matrix products that build A from a chosen factor, and A*x0).
 *
 * Storage: LAPACK lower band layout, column-major, A(i,j) for 0 <= i-j <= k
 * at ab[(i-j) + j*ldab], ldab >= k+1.  Only rows 0..k of each band column are
 * written; padding rows and the unreferenced bottom-right triangle are left as
 * the caller filled them.
 *
 * Random numbers: SplitMix64 (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) used counter-style, so every
 * entry is a pure function of (seed, stream, index) and generation order or
 * thread count never changes a value:
 *     draw(key, idx) = mix64(key + (idx + 1) * GOLDEN)
 * Uniforms take the top 53 bits; normals use the Box-Muller transform.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t make_key(uint64_t seed, uint64_t stream)
{
    return mix64(mix64(seed + GOLDEN) ^ (stream * 0xD1B54A32D192ED03ULL));
}

static inline uint64_t draw(uint64_t key, uint64_t idx)
{
    return mix64(key + (idx + 1) * GOLDEN);
}

/* uniform on [0, 1) with 53 random bits */
static inline double u01(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

/* standard normal from two counter draws (Box-Muller, cosine branch) */
static inline double normal01(uint64_t key, uint64_t idx)
{
    double u1 = 1.0 - u01(draw(key, 2 * idx));      /* (0, 1] */
    double u2 = u01(draw(key, 2 * idx + 1));
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

enum { ST_OFFDIAG = 1, ST_DIAG = 2, ST_RHS = 3, ST_INT = 4, ST_X0 = 5 };

void synth_uniform(int64_t count, uint64_t seed, uint64_t stream, double lo, double hi, double *out)
{
    uint64_t key = make_key(seed, stream);
    for (int64_t i = 0; i < count; ++i)
        out[i] = lo + (hi - lo) * u01(draw(key, (uint64_t)i));
}

void synth_normal(int64_t count, uint64_t seed, uint64_t stream, double *out)
{
    uint64_t key = make_key(seed, stream);
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i)
        out[i] = normal01(key, (uint64_t)i);
}

/* Right-hand sides: n x nrhs column-major, ldb >= n, i.i.d. N(0,1). */
void synth_rhs(int64_t n, int64_t nrhs, uint64_t seed, double *b, int64_t ldb)
{
    uint64_t key = make_key(seed, ST_RHS);
    for (int64_t r = 0; r < nrhs; ++r)
        for (int64_t i = 0; i < n; ++i)
            b[i + r * ldb] = normal01(key, (uint64_t)(r * n + i));
}

/*
 * Diagonally dominant SPD band matrix (the paper's test matrices are random
 * and made positive definite through diagonal dominance).  Stored lower
 * off-diagonals i.i.d. uniform on [-1, 1); the upper part is their mirror;
 * the diagonal is 1 + the sum of |off-diagonals| over the full symmetric row,
 * so every eigenvalue is >= 1 (Gershgorin).
 */
void synth_band_diagdom(int64_t n, int64_t k, uint64_t seed, double *ab, int64_t ldab)
{
    uint64_t key = make_key(seed, ST_OFFDIAG);
    double *rs = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    for (int64_t j = 0; j < n; ++j) {
        int64_t dmax = (k < n - 1 - j) ? k : n - 1 - j;
        for (int64_t d = 1; d <= dmax; ++d) {
            double a = 2.0 * u01(draw(key, (uint64_t)(j * (k + 1) + d))) - 1.0;
            ab[d + j * ldab] = a;
            rs[j] += fabs(a);
            rs[j + d] += fabs(a);
        }
    }
    for (int64_t j = 0; j < n; ++j)
        ab[j * ldab] = 1.0 + rs[j];
    free(rs);
}

/*
 * Interior-point-like ill-conditioned SPD band matrix:
 *   L0 lower band k, off-diagonals N(0,1)/sqrt(k), diagonal 10^U[diag_exp_lo, 0];
 *   A = L0 L0^T (its band is exactly k wide);
 *   A += shift_rel * ||A||_inf * I.
 * The product is formed in a row-band copy of L0 (R0[i][t] = L0(i, i-k+t)),
 * one independent entry per (i, j), so the result does not depend on the
 * thread count.  ||A||_inf is the largest absolute row sum of the full
 * symmetric matrix.  Returns ||A||_inf before the shift.
 */
double synth_band_ipm(int64_t n, int64_t k, uint64_t seed, double diag_exp_lo, double shift_rel,
                      double *ab, int64_t ldab)
{
    uint64_t koff = make_key(seed, ST_OFFDIAG), kdia = make_key(seed, ST_DIAG);
    int64_t w = k + 1;
    double *r0 = (double *)calloc((size_t)(n > 0 ? n : 1) * (size_t)w, sizeof(double));
    double scale = k > 0 ? 1.0 / sqrt((double)k) : 1.0;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t t = 0; t < k; ++t) {
            int64_t l = i - k + t;
            if (l >= 0)
                r0[i * w + t] = scale * normal01(koff, (uint64_t)(i * w + t));
        }
        double e = diag_exp_lo * u01(draw(kdia, (uint64_t)i));   /* U[lo, 0] */
        r0[i * w + k] = pow(10.0, e);
    }
    /* A(i, j) = sum_{l = max(0, i-k)}^{j} L0(i,l) L0(j,l), for j in [i-k, i] */
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        int64_t jlo = i - k > 0 ? i - k : 0;
        const double *ri = r0 + i * w;
        for (int64_t j = jlo; j <= i; ++j) {
            const double *rj = r0 + j * w;
            double s = 0.0;
            for (int64_t l = jlo; l <= j; ++l)
                s += ri[l - i + k] * rj[l - j + k];
            ab[(i - j) + j * ldab] = s;
        }
    }
    free(r0);
    double *rs = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    for (int64_t j = 0; j < n; ++j) {
        int64_t dmax = (k < n - 1 - j) ? k : n - 1 - j;
        rs[j] += fabs(ab[j * ldab]);
        for (int64_t d = 1; d <= dmax; ++d) {
            double a = fabs(ab[d + j * ldab]);
            rs[j] += a;
            rs[j + d] += a;
        }
    }
    double norm = 0.0;
    for (int64_t j = 0; j < n; ++j)
        if (rs[j] > norm) norm = rs[j];
    free(rs);
    for (int64_t j = 0; j < n; ++j)
        ab[j * ldab] += shift_rel * norm;
    return norm;
}

/*
 * Integer-exact factor: L0 lower band k with off-diagonals drawn uniformly
 * from {-1, 0, 1} and diagonal 2^m, m drawn from {0..pow2_max} (pow2_max = 0
 * gives a unit diagonal).  Every product and partial sum that a Cholesky
 * factorization of L0 D L0^T forms is then a small dyadic rational, exact in
 * FP64, so any correct factorization returns L0 itself.
 */
void synth_int_factor(int64_t n, int64_t k, uint64_t seed, int pow2_max, double *l0, int64_t ldl)
{
    uint64_t key = make_key(seed, ST_INT);
    for (int64_t j = 0; j < n; ++j) {
        int64_t dmax = (k < n - 1 - j) ? k : n - 1 - j;
        int m = pow2_max > 0 ? (int)(draw(key, (uint64_t)(j * (k + 1))) % (uint64_t)(pow2_max + 1)) : 0;
        l0[j * ldl] = ldexp(1.0, m);
        for (int64_t d = 1; d <= dmax; ++d)
            l0[d + j * ldl] = (double)((int)(draw(key, (uint64_t)(j * (k + 1) + d)) % 3ULL) - 1);
    }
}

/*
 * A = L0 diag(dvec) L0^T on the band (dvec == NULL means the identity).
 * A(i,j) = sum_{l = max(0, i-k)}^{j} L0(i,l) d_l L0(j,l), i >= j.
 */
void synth_band_ldlt(int64_t n, int64_t k, const double *l0, int64_t ldl, const double *dvec,
                     double *ab, int64_t ldab)
{
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        int64_t jlo = i - k > 0 ? i - k : 0;
        for (int64_t j = jlo; j <= i; ++j) {
            double s = 0.0;
            for (int64_t l = jlo; l <= j; ++l) {
                double dl = dvec ? dvec[l] : 1.0;
                s += l0[(i - l) + l * ldl] * dl * l0[(j - l) + l * ldl];
            }
            ab[(i - j) + j * ldab] = s;
        }
    }
}

/*
 * Sparse integer-exact factor for large n and k: L0 lower band k, unit
 * diagonal, and each off-diagonal position (j + d, j), 1 <= d <= k, holds
 * +1 or -1 with probability `density` (else 0), drawn per position.  A =
 * L0 L0^T is then formed from each column's list of nonzeros, A(i, j) +=
 * L0(i, l) L0(j, l) for every pair of rows i >= j of column l, at O(n m^2)
 * cost for m nonzeros per column instead of O(n k^2).  Every value is a small
 * integer, so the order of the additions does not matter.  l0 and ab are
 * zeroed on rows 0..k first (ab's other rows are left alone).
 */
void synth_int_factor_sparse(int64_t n, int64_t k, uint64_t seed, double density, double *l0, int64_t ldl)
{
    uint64_t key = make_key(seed, ST_INT + 16);
    for (int64_t j = 0; j < n; ++j) {
        int64_t dmax = (k < n - 1 - j) ? k : n - 1 - j;
        l0[j * ldl] = 1.0;
        for (int64_t d = 1; d <= k; ++d) l0[d + j * ldl] = 0.0;
        for (int64_t d = 1; d <= dmax; ++d) {
            uint64_t x = draw(key, (uint64_t)(j * (k + 1) + d));
            if (u01(x) < density) l0[d + j * ldl] = (x & 1) ? 1.0 : -1.0;
        }
    }
}

void synth_band_llt_sparse(int64_t n, int64_t k, const double *l0, int64_t ldl, double *ab, int64_t ldab)
{
    /* column lists (rows ascending) and row lists (columns ascending) of the nonzeros */
    int64_t *cptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *rptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t l = 0; l < n; ++l) {
        int64_t dmax = (k < n - 1 - l) ? k : n - 1 - l;
        for (int64_t d = 0; d <= dmax; ++d)
            if (l0[d + l * ldl] != 0.0) { cptr[l + 1]++; rptr[l + d + 1]++; }
    }
    for (int64_t i = 0; i < n; ++i) { cptr[i + 1] += cptr[i]; rptr[i + 1] += rptr[i]; }
    int64_t nnz = cptr[n];
    int64_t *crow = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
    int64_t *rcol = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
    int64_t *rfill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) rfill[i] = rptr[i];
    for (int64_t l = 0; l < n; ++l) {
        int64_t dmax = (k < n - 1 - l) ? k : n - 1 - l, c = cptr[l];
        for (int64_t d = 0; d <= dmax; ++d)
            if (l0[d + l * ldl] != 0.0) { crow[c++] = l + d; rcol[rfill[l + d]++] = l; }
    }
    /* column j of A: A(i, j) = sum over l in row j's list of L0(j, l) L0(i, l), i >= j */
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t d = 0; d <= k; ++d) ab[d + j * ldab] = 0.0;
        for (int64_t p = rptr[j]; p < rptr[j + 1]; ++p) {
            int64_t l = rcol[p];
            double vj = l0[(j - l) + l * ldl];
            for (int64_t q = cptr[l]; q < cptr[l + 1]; ++q) {
                int64_t i = crow[q];
                if (i >= j) ab[(i - j) + j * ldab] += l0[(i - l) + l * ldl] * vj;
            }
        }
    }
    free(cptr); free(rptr); free(crow); free(rcol); free(rfill);
}

/* Integer right-hand-side solution x0 with entries uniform in {-8..8}. */
void synth_int_vector(int64_t count, uint64_t seed, double *x)
{
    uint64_t key = make_key(seed, ST_X0);
    for (int64_t i = 0; i < count; ++i)
        x[i] = (double)((int)(draw(key, (uint64_t)i) % 17ULL) - 8);
}

/* b = A x for the symmetric band A (lower storage), nrhs columns. */
void synth_band_symv(int64_t n, int64_t k, int64_t nrhs, const double *ab, int64_t ldab,
                     const double *x, int64_t ldx, double *b, int64_t ldb)
{
    for (int64_t r = 0; r < nrhs; ++r) {
        const double *xr = x + r * ldx;
        double *br = b + r * ldb;
        for (int64_t i = 0; i < n; ++i) br[i] = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            br[j] += ab[j * ldab] * xr[j];
            int64_t dmax = (k < n - 1 - j) ? k : n - 1 - j;
            for (int64_t d = 1; d <= dmax; ++d) {
                double a = ab[d + j * ldab];
                br[j + d] += a * xr[j];
                br[j] += a * xr[j + d];
            }
        }
    }
}

/* Sizes of the uneven batch: n_i uniform in [n_lo, n_hi], k_i uniform in [k_lo, k_hi]. */
void synth_batch_shapes(int64_t batch, uint64_t seed, int64_t n_lo, int64_t n_hi, int64_t k_lo,
                        int64_t k_hi, int64_t *nv, int64_t *kv)
{
    uint64_t key = make_key(seed, 6);
    for (int64_t b = 0; b < batch; ++b) {
        nv[b] = n_lo + (int64_t)(draw(key, (uint64_t)(2 * b)) % (uint64_t)(n_hi - n_lo + 1));
        kv[b] = k_lo + (int64_t)(draw(key, (uint64_t)(2 * b + 1)) % (uint64_t)(k_hi - k_lo + 1));
    }
}
