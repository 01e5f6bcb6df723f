"""Pins for the CPU oracle (no GPU).

Each test ties the oracle to something other than itself: brute force on the
dense matrix, closed forms, exact-arithmetic constructions, invariants, an
independent LAPACK implementation (scipy / numpy), and the paper's flop model.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
import synth

U = 2.0 ** -53  # unit roundoff of FP64


def band_to_dense(ab, k):
    n = ab.shape[1]
    a = np.zeros((n, n))
    for j in range(n):
        for d in range(0, min(k, n - 1 - j) + 1):
            a[j + d, j] = ab[d, j]
            a[j, j + d] = ab[d, j]
    return a


def lower_band(l_dense, k, ldab=None):
    n = l_dense.shape[0]
    ab = np.zeros((k + 1 if ldab is None else ldab, n), order="F")
    for j in range(n):
        for d in range(0, min(k, n - 1 - j) + 1):
            ab[d, j] = l_dense[j + d, j]
    return ab


def dense_cholesky_py(a):
    """Textbook Cholesky-Banachiewicz on the full matrix, pure Python floats.

    No band truncation: the sums run over every earlier column, so the terms
    outside the band are exact zeros."""
    n = len(a)
    L = [[0.0] * n for _ in range(n)]
    for i in range(n):
        for j in range(i + 1):
            t = 0.0
            for l in range(j):
                t += L[i][l] * L[j][l]
            if i == j:
                d = a[i][i] - t
                if not d > 0.0:
                    return L, i + 1
                L[i][i] = math.sqrt(d)
            else:
                L[i][j] = (a[i][j] - t) / L[j][j]
    return L, 0


# ---------------------------------------------------------------- P1 brute force

@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 13, 24, 40])
def test_dense_bruteforce_bitwise(n):
    for k in sorted({0, 1, 2, n // 3, n // 2, max(n - 2, 0), n - 1}):
        if k < 0:
            continue
        for seed, maker in ((n * 100 + k, "dd"), (n * 100 + k + 1, "ipm")):
            if maker == "dd":
                ab = synth.band_diagdom(n, k, seed)
            else:
                ab, _ = synth.band_ipm(n, k, seed, shift_rel=1e-6)
            a = band_to_dense(ab, k)
            Ld, info_d = dense_cholesky_py(a.tolist())
            l, info = oracle.factor(ab, k)
            assert info == info_d == 0
            ref = lower_band(np.array(Ld), k)
            assert np.array_equal(l, ref), (n, k, maker)


def test_dense_lapack_potrf():
    """numpy's dense LAPACK potrf (an independent implementation)."""
    for n, k in ((60, 7), (90, 30), (50, 49)):
        ab = synth.band_diagdom(n, k, 5 + n)
        l, info = oracle.factor(ab, k)
        assert info == 0
        ref = np.linalg.cholesky(band_to_dense(ab, k))
        assert np.max(np.abs(band_to_dense_lower(l, k) - ref)) <= 64 * U * np.max(np.abs(ref))
        # L has the lower bandwidth of A: LAPACK's dense factor is zero outside it
        mask = np.tril(np.ones((n, n)), -k - 1).astype(bool)
        assert np.max(np.abs(ref[mask]), initial=0.0) <= 64 * U * np.max(np.abs(ref))


def band_to_dense_lower(ab, k):
    n = ab.shape[1]
    a = np.zeros((n, n))
    for j in range(n):
        for d in range(0, min(k, n - 1 - j) + 1):
            a[j + d, j] = ab[d, j]
    return a


# ---------------------------------------------------------------- P2 closed form

def tridiag(n):
    ab = np.zeros((2, n), order="F")
    ab[0, :] = 2.0
    ab[1, :-1] = -1.0
    return ab


@pytest.mark.parametrize("n", [1, 2, 10, 50, 400])
def test_tridiag_closed_form(n):
    """T = tridiag(-1, 2, -1): with 1-based i, L_ii = sqrt((i+1)/i),
    L_{i+1,i} = -sqrt(i/(i+1)); T x = 1 has x_i = i (n + 1 - i) / 2."""
    ab = tridiag(n)
    l, info = oracle.factor(ab, 1)
    assert info == 0
    i = np.arange(1, n + 1, dtype=np.float64)
    diag = np.sqrt((i + 1) / i)
    sub = -np.sqrt(i[:-1] / (i[:-1] + 1))
    # the pivot recurrence d_i = 2 - 1/d_{i-1} carries at most ~i rounding steps
    tol = (8 + 2 * n) * U
    assert np.all(np.abs(l[0] - diag) <= tol * diag)
    assert np.all(np.abs(l[1, :-1] - sub) <= tol * np.abs(sub))
    x = oracle.solve(l, 1, np.ones(n))
    xe = i * (n + 1 - i) / 2.0
    assert np.max(np.abs(x - xe) / xe) <= (16 + 4 * n) * U * n


def test_tridiag_golden_fixture():
    """Stored closed-form values (40-digit decimal evaluation of the formulas)."""
    path = os.path.join(os.path.dirname(__file__), "golden", "tridiag_n8.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    l, info = oracle.factor(tridiag(8), 1)
    assert info == 0
    for kind, idx, val in rows:
        got = l[0, int(idx)] if kind == "diag" else l[1, int(idx)]
        assert abs(got - float(val)) <= 8 * U * abs(float(val)), (kind, idx)


def test_cond_estimate_tridiag():
    """Hager/Higham estimate vs the exact kappa_1 from the dense inverse."""
    for n in (10, 64, 200):
        ab = tridiag(n)
        l, _ = oracle.factor(ab, 1)
        a = band_to_dense(ab, 1)
        exact = np.linalg.norm(a, 1) * np.linalg.norm(np.linalg.inv(a), 1)
        est = oracle.cond1_estimate(ab, l, 1)
        assert est <= exact * (1 + 1e-10)
        assert est >= exact / 3.0


def test_cond_estimate_random():
    for n, k, seed in ((80, 5, 1), (120, 20, 2)):
        ab, _ = synth.band_ipm(n, k, seed, shift_rel=1e-6)
        l, info = oracle.factor(ab, k)
        assert info == 0
        a = band_to_dense(ab, k)
        exact = np.linalg.norm(a, 1) * np.linalg.norm(np.linalg.inv(a), 1)
        est = oracle.cond1_estimate(ab, l, k)
        assert exact / 10.0 <= est <= exact * (1 + 1e-8)


# ---------------------------------------------------------------- P3/P4 invariants

def test_padding_invariance_bitwise():
    """Zero diagonals added to the band (the paper's zero padding) leave L unchanged."""
    n, k = 300, 9
    ab = synth.band_diagdom(n, k, 11)
    l, _ = oracle.factor(ab, k)
    for p in (1, 5, 23):
        ab2 = np.zeros((k + 1 + p, n), order="F")
        ab2[: k + 1] = ab
        l2, info = oracle.factor(ab2, k + p)
        assert info == 0
        assert np.array_equal(l2[: k + 1], l)
        assert not np.any(l2[k + 1:])


def test_ldab_padding_rows_untouched():
    n, k, ldab = 200, 6, 11
    ab = synth.band_diagdom(n, k, 3, ldab=ldab, fill=np.nan)
    ab[k + 1:, :] = 123.25
    for j in range(n - k, n):                      # unreferenced bottom-right triangle
        ab[n - j: k + 1, j] = -7.5
    ref = synth.band_diagdom(n, k, 3)
    l, info = oracle.factor(ab, k)
    lr, _ = oracle.factor(ref, k)
    assert info == 0
    assert np.all(l[k + 1:] == 123.25)
    for j in range(n - k, n):
        assert np.all(l[n - j: k + 1, j] == -7.5)
        l[n - j: k + 1, j] = 0.0
    assert np.array_equal(l[: k + 1], lr)


def test_k0_is_sqrt():
    d = synth.uniform(500, 4, 9, 0.5, 3.0)
    ab = np.asfortranarray(d.reshape(1, -1))
    l, info = oracle.factor(ab, 0)
    assert info == 0 and np.array_equal(l[0], np.sqrt(d))
    b = synth.rhs(500, 2, 1)
    x = oracle.solve(l, 0, b)
    assert np.allclose(x, b / d[:, None], rtol=4 * U, atol=0)


def test_n0_and_args():
    ab = np.zeros((3, 0), order="F")
    assert oracle.pbtrf(ab, 2) == 0
    lib = oracle._load()
    assert lib.oracle_pbtrf(-1, 2, None, 3) == -1
    assert lib.oracle_pbtrf(5, -1, None, 3) == -2
    assert lib.oracle_pbtrf(5, 2, None, 3) == -3
    x = np.zeros((3, 5), order="F")
    assert lib.oracle_pbtrf(5, 2, x.ctypes.data_as(oracle._D), 2) == -4
    assert lib.oracle_pbtrs(5, 2, -1, None, 3, None, 5) == -3
    assert lib.oracle_pbtrs(5, 2, 1, x.ctypes.data_as(oracle._D), 3, x.ctypes.data_as(oracle._D), 4) == -7


# ---------------------------------------------------------------- P5 exact arithmetic

@pytest.mark.parametrize("n,k,p2", [(1000, 1, 0), (3000, 50, 0), (2000, 120, 2), (500, 499, 0)])
def test_integer_exact_factor_and_solve(n, k, p2):
    """A = L0 L0^T with integer/dyadic L0: every intermediate is exact, so the
    unique factor L0 and the integer solution x0 come back bit for bit."""
    l0 = synth.int_factor(n, k, 17 + k, pow2_max=p2)
    a = synth.band_ldlt(l0, k)
    l, info = oracle.factor(a, k)
    assert info == 0
    assert np.array_equal(l, l0)
    x0 = synth.int_vector(2 * n, 3).reshape(n, 2, order="F")
    b = synth.band_symv(a, k, x0)
    x = oracle.solve(l, k, b)
    assert np.array_equal(x, x0)
    assert oracle.llt_residual(l, a, k) == 0.0


# ---------------------------------------------------------------- P6 failure column

@pytest.mark.parametrize("m", [0, 1, 31, 32, 64, 257, 599])
@pytest.mark.parametrize("dval", [-1.0, 0.0])
def test_nonspd_info_exact(m, dval):
    """A = L0 D L0^T, D = I except D_m: the m-th pivot is exactly D_m, so the
    first leading minor that is not positive definite has order m + 1."""
    n, k = 600, 40
    l0 = synth.int_factor(n, k, 99)
    dvec = np.ones(n)
    dvec[m] = dval
    a = synth.band_ldlt(l0, k, dvec)
    _, info = oracle.factor(a, k)
    assert info == m + 1
    _, info_c = oracle.factor(a, k, columns=True)
    assert info_c == m + 1


def test_nan_info():
    n, k = 300, 12
    base = synth.band_diagdom(n, k, 21)
    for (i, j) in ((0, 0), (5, 5), (17, 9), (250, 240), (299, 287)):
        ab = base.copy(order="F")
        ab[i - j, j] = np.nan
        _, info = oracle.factor(ab, k)
        assert info == i + 1, (i, j)


def test_scipy_agrees_on_failure():
    """LAPACK pbtrf (through scipy) reports the same failing leading minor."""
    n, k = 200, 10
    l0 = synth.int_factor(n, k, 5)
    dvec = np.ones(n)
    dvec[77] = -1.0
    a = synth.band_ldlt(l0, k, dvec)
    with pytest.raises(np.linalg.LinAlgError, match="78"):
        scipy.linalg.cholesky_banded(a, lower=True)
    assert oracle.factor(a, k)[1] == 78


# ---------------------------------------------------------------- P8/P10 residuals, LAPACK

@pytest.mark.parametrize("n,k", [(2000, 50), (1500, 130), (600, 300)])
def test_residual_bounds_and_scipy(n, k):
    ab = synth.band_diagdom(n, k, n + k)
    l, info = oracle.factor(ab, k)
    assert info == 0
    eta = oracle.llt_residual(l, ab, k)
    assert eta <= 2 * (k + 1) * U
    ref = scipy.linalg.cholesky_banded(ab, lower=True)
    assert np.max(np.abs(ref - l)) <= 1e-13 * np.max(np.abs(ref))
    b = synth.rhs(n, 3, 2)
    x = oracle.solve(l, k, b)
    assert oracle.solve_residual(ab, k, x, b) <= 4 * (k + 1) * U
    xr = scipy.linalg.solveh_banded(ab, b, lower=True)
    assert np.max(np.abs(xr - x)) <= 1e-12 * np.max(np.abs(xr))


def test_ipm_recipe_conditioning():
    """The ill-conditioned recipe factors, with tiny backward error and a
    condition number near 1/shift."""
    n, k = 4000, 50
    ab, nrm = synth.band_ipm(n, k, 1000)
    l, info = oracle.factor(ab, k)
    assert info == 0
    assert oracle.llt_residual(l, ab, k) <= 4 * (k + 1) * U
    kap = oracle.cond1_estimate(ab, l, k)
    assert 1e5 < kap < 1e10
    b = synth.rhs(n, 1, 1000)
    x = oracle.solve(l, k, b)
    assert oracle.solve_residual(ab, k, x, b) <= 8 * (k + 1) * U
    xr = scipy.linalg.solveh_banded(ab, b, lower=True)
    assert np.max(np.abs(xr.ravel() - x.ravel())) <= 1e-14 * kap * np.max(np.abs(xr))


def test_residual_helpers_against_dense():
    n, k = 70, 6
    ab = synth.band_diagdom(n, k, 8)
    l, _ = oracle.factor(ab, k)
    rng = np.random.default_rng(0)
    lp = l + 1e-9 * rng.standard_normal(l.shape) * (l != 0)
    lp = np.asfortranarray(lp)
    a = band_to_dense(ab, k)
    ld = band_to_dense_lower(lp, k)
    ref = np.linalg.norm(ld @ ld.T - a) / np.linalg.norm(a)
    assert abs(oracle.llt_residual(lp, ab, k) - ref) <= 1e-6 * ref
    half = oracle.llt_residual(lp, ab, k, rows=[(0, 35), (35, 70)])
    assert abs(half - ref) <= 1e-6 * ref
    x = rng.standard_normal(n)
    bb = a @ x + 1e-7
    r = np.max(np.abs(bb - a @ x)) / (np.linalg.norm(a, np.inf) * np.max(np.abs(x)))
    assert abs(oracle.solve_residual(ab, k, x, bb) - r) <= 1e-6 * r
    assert np.allclose(oracle.symv(ab, k, x), a @ x, rtol=1e-13, atol=1e-13)
    assert oracle.norm_inf(ab, k) == pytest.approx(np.linalg.norm(a, np.inf), rel=1e-14)


# ---------------------------------------------------------------- P9 flop model

def eq1_corrected_py(N, k):
    """Eq. (1) of Section 3.2 with 1-based indices and the inner bound l <= j-1."""
    tot = 0
    for i in range(1, N + 1):
        r = max(1, i - k)
        for j in range(r, i + 1):
            tot += 2 * (j - r) + 2
    return tot


def eq1_printed_py(N, k):
    """Eq. (1) exactly as printed (inner bound l <= j)."""
    tot = 0
    for i in range(1, N + 1):
        r = max(1, i - k)
        for j in range(r, i + 1):
            tot += 2 * (j - r + 1) + 2
    return tot


def flops_closed(n, k):
    k = min(k, max(n - 1, 0))
    return (n - k) * (k + 1) * (k + 2) + k * (k + 1) * (k + 2) // 3


@pytest.mark.parametrize("n,k", [(1, 0), (7, 0), (7, 3), (30, 29), (50, 5), (200, 17)])
def test_flop_identity(n, k):
    assert oracle.opcount(n, k) == eq1_corrected_py(n, k) == flops_closed(n, k)
    # the printed bound would add 2 operations per (i, j) pair
    pairs = sum(min(i, k) + 1 for i in range(n))
    assert eq1_printed_py(n, k) == eq1_corrected_py(n, k) + 2 * pairs


def test_flop_model_vs_exact_at_paper_size():
    """The paper's closed approximation N(k^2 + 3k) is within 2% of the exact
    count for n = 1e5 across the benchmarked bandwidths."""
    n = 100000
    for k in (50, 100, 250, 500, 1000, 2000):
        exact = oracle.opcount(n, k)
        assert exact == flops_closed(n, k)
        assert 0.98 <= exact / (n * (k * k + 3 * k)) <= 1.01


# ---------------------------------------------------------------- P11 determinism

@pytest.mark.parametrize("n,k", [(3000, 80), (1200, 400)])
def test_column_variant_bitwise(n, k):
    ab = synth.band_diagdom(n, k, 77)
    l1, i1 = oracle.factor(ab, k)
    l2, i2 = oracle.factor(ab, k, columns=True)
    assert i1 == i2 == 0
    assert np.array_equal(l1, l2)
    ab2, _ = synth.band_ipm(n, k, 78)
    assert np.array_equal(oracle.factor(ab2, k)[0], oracle.factor(ab2, k, columns=True)[0])


def test_generator_is_order_free():
    """Counter-based draws: the same (seed, index) always gives the same value,
    regardless of how many threads built the matrix."""
    a1, n1 = synth.band_ipm(500, 30, 4)
    a2, n2 = synth.band_ipm(500, 30, 4)
    assert np.array_equal(a1, a2) and n1 == n2
    assert not np.array_equal(a1, synth.band_ipm(500, 30, 5)[0])
