"""GPU parity: the HIP factor and solves against the CPU oracle, through the C-ABI.

Bars (FP64): relative backward error ||L L^T - A||_F / ||A||_F <= 1e-12 and
solve residual ||b - A x||_inf / (||A||_inf ||x||_inf) <= 1e-12; the forward
error of x against the oracle's x within 1e-12 * kappa_1(A) (Hager/Higham
estimate); elementwise L against the oracle's L within a kappa-free bound for
the diagonally dominant matrices; bit-exact where the arithmetic is exact.
"""
import numpy as np
import pytest

import oracle
import synth
from helpers import ETA_TOL, U, col_rel_err, from_dev, gpu_factor, gpu_solve, rel_fro

pytestmark = pytest.mark.gpu


def check_against_oracle(ab, k, nrhs=1, seed=0, check_elementwise=True):
    l_gpu, info = gpu_factor(ab, k)
    assert info == 0
    l_or, info_or = oracle.factor(ab, k)
    assert info_or == 0
    eta = oracle.llt_residual(l_gpu, ab, k)
    assert eta <= ETA_TOL, eta
    # padding rows and the bottom-right triangle are never written
    n = ab.shape[1]
    kk = min(k, n - 1) if n else 0
    assert np.array_equal(l_gpu[kk + 1:], ab[kk + 1:])
    for j in range(max(n - kk, 0), n):
        assert np.array_equal(l_gpu[n - j: kk + 1, j], ab[n - j: kk + 1, j])
    if check_elementwise:
        # every column of L against the oracle's, relative to the column's norm
        assert col_rel_err(l_gpu[: kk + 1], l_or[: kk + 1]) <= 1e-13 * (kk + 1)
    b = synth.rhs(n, nrhs, seed)
    x_gpu = gpu_solve(l_gpu, k, b)
    assert oracle.solve_residual(ab, k, x_gpu, b) <= ETA_TOL
    x_or = oracle.solve(l_or, k, b)
    return l_gpu, x_gpu, l_or, x_or


def test_c0_diag_dominant_n2000_k50():
    """The small configuration: n = 2000, k = 50, diagonally dominant."""
    ab = synth.band_diagdom(2000, 50, 0)
    _, x_gpu, _, x_or = check_against_oracle(ab, 50, nrhs=1, seed=0)
    assert np.max(np.abs(x_gpu - x_or)) <= 1e-12 * np.max(np.abs(x_or)) * 10


@pytest.mark.parametrize("n,k", [
    (1, 0), (2, 1), (31, 3), (32, 31), (33, 32), (64, 5), (100, 33), (257, 64), (300, 299),
    (1000, 0), (1000, 1), (1000, 31), (1000, 32), (1000, 33), (777, 65), (1500, 96), (2049, 130),
    (3001, 200), (500, 257),
])
def test_ragged_shapes(n, k):
    """Several tiles with a ragged tail in n, in k, or both; k >= n-1 is dense."""
    ab = synth.band_diagdom(n, k, 1000 * n + k)
    check_against_oracle(ab, k, nrhs=2, seed=n + k)


@pytest.mark.parametrize("ldab_extra", [1, 7])
def test_ldab_padding_untouched(ldab_extra):
    n, k = 700, 40
    ab = synth.band_diagdom(n, k, 5, ldab=k + 1 + ldab_extra, fill=np.nan)
    for j in range(n - k, n):
        ab[n - j: k + 1, j] = np.nan                 # never referenced
    l_gpu, info = gpu_factor(ab, k)
    assert info == 0
    assert np.all(np.isnan(l_gpu[k + 1:]))
    ref = synth.band_diagdom(n, k, 5)
    l_or, _ = oracle.factor(ref, k)
    lg = l_gpu[: k + 1].copy()
    for j in range(n - k, n):
        assert np.all(np.isnan(lg[n - j:, j]))
        lg[n - j:, j] = 0.0
    assert rel_fro(lg, l_or) <= 1e-13 * (k + 1)


@pytest.mark.parametrize("n,k,p2", [(3000, 50, 0), (2000, 100, 2), (1000, 250, 0), (500, 499, 1)])
def test_integer_exact_bitwise(n, k, p2):
    l0 = synth.int_factor(n, k, 17 + k, pow2_max=p2)
    a = synth.band_ldlt(l0, k)
    l_gpu, info = gpu_factor(a, k)
    assert info == 0
    assert np.array_equal(l_gpu, l0)
    x0 = synth.int_vector(3 * n, 3).reshape(n, 3, order="F")
    b = synth.band_symv(a, k, x0)
    x = gpu_solve(l_gpu, k, b)
    assert np.array_equal(x, x0)


@pytest.mark.parametrize("m", [0, 1, 31, 32, 33, 64, 255, 599])
@pytest.mark.parametrize("dval", [-1.0, 0.0])
def test_nonspd_info_matches_oracle(m, dval):
    n, k = 600, 40
    l0 = synth.int_factor(n, k, 99)
    dvec = np.ones(n)
    dvec[m] = dval
    a = synth.band_ldlt(l0, k, dvec)
    _, info = gpu_factor(a, k)
    assert info == m + 1 == oracle.factor(a, k)[1]


@pytest.mark.parametrize("k", [180, 300, 500, 1300])
@pytest.mark.parametrize("m", [0, 33, 700, 2047])
def test_nonspd_info_with_helpers(k, m):
    """A failing pivot while helper workgroups are at work (K = 6, 10, 16 and
    41; from K = 12 on strips of four tiles wait at their shared barriers): the first
    failing column is reported as the oracle reports it, and every waiting
    workgroup leaves through the abort flag (the call returns within the
    test's time limit, far below the waits' own bound)."""
    import time
    n = 2048 if k < 1000 else 2900
    l0 = synth.int_factor(n, k, 77 + k)
    dvec = np.ones(n)
    dvec[m] = -1.0
    a = synth.band_ldlt(l0, k, dvec)
    t0 = time.time()
    _, info = gpu_factor(a, k)
    assert time.time() - t0 < 2.0
    assert info == m + 1 == oracle.factor(a, k)[1]


def test_nan_info_matches_oracle():
    n, k = 400, 45
    base = synth.band_diagdom(n, k, 21)
    for (i, j) in ((0, 0), (5, 5), (40, 9), (250, 240), (399, 360), (100, 55)):
        ab = base.copy(order="F")
        ab[i - j, j] = np.nan
        _, info = gpu_factor(ab, k)
        assert info == i + 1 == oracle.factor(ab, k)[1], (i, j)


def test_run_to_run_bitwise():
    ab, _ = synth.band_ipm(5000, 120, 7)
    l1, _ = gpu_factor(ab, 120)
    l2, _ = gpu_factor(ab, 120)
    assert np.array_equal(l1, l2)
    b = synth.rhs(5000, 2, 1)
    assert np.array_equal(gpu_solve(l1, 120, b), gpu_solve(l1, 120, b))


@pytest.mark.parametrize("k", [50, 100, 250])
def test_ipm_recipe_forward_error(k):
    """Ill-conditioned interior-point-like matrices (shift 1e-8 ||A||)."""
    n = 20000
    ab, _ = synth.band_ipm(n, k, 1000 + k)
    l_gpu, x_gpu, l_or, x_or = check_against_oracle(ab, k, nrhs=1, seed=k, check_elementwise=False)
    kap = oracle.cond1_estimate(ab, l_or, k)
    fwd = np.max(np.abs(x_gpu - x_or)) / np.max(np.abs(x_or))
    assert fwd <= 1e-12 * kap, (fwd, kap)


@pytest.fixture(params=["walk", "tiles"])
def schedule(request):
    import paper_2305_04635_amd as bc
    prev = bc.set_walk_limit(15 if request.param == "walk" else 0)
    yield request.param
    bc.set_walk_limit(prev)


@pytest.mark.parametrize("n,k", [(128, 70), (300, 299), (1000, 130), (777, 200), (2049, 33), (96, 95), (1, 0), (33, 1)])
def test_both_schedules(schedule, n, k):
    """The single-workgroup walk and the multi-workgroup tile schedule, each
    forced on bands of several tile widths (the walk's in-place trsm of
    K >= 3 tiles once raced: one wave read columns another wave had already
    overwritten)."""
    ab = synth.band_diagdom(n, k, 31 * n + k)
    check_against_oracle(ab, k, nrhs=1, seed=k)
    l0 = synth.int_factor(n, k, 5 + k, pow2_max=1)
    a = synth.band_ldlt(l0, k)
    l_gpu, info = gpu_factor(a, k)
    assert info == 0 and np.array_equal(l_gpu, l0)


@pytest.mark.parametrize("K", range(1, 11))
def test_tile_schedule_each_K(K):
    """The multi-workgroup schedule at every number of sub-diagonal tiles K = 1..10
    (which of the spine's extra terms and of the helper tasks exist changes
    with K up to 5), with k ragged in the last tile and n ragged, at a few tile
    rows past K and at many; the integer factor must come out bit for bit."""
    import paper_2305_04635_amd as bc
    prev = bc.set_walk_limit(0)
    try:
        k = 32 * K - 5
        for n in (32 * (K + 2) + 7, 32 * (3 * K + 6) - 3):
            ab = synth.band_diagdom(n, k, 7 * n + K)
            check_against_oracle(ab, k, nrhs=1, seed=K)
            l0 = synth.int_factor(n, k, 11 + K, pow2_max=1)
            l_gpu, info = gpu_factor(synth.band_ldlt(l0, k), k)
            assert info == 0 and np.array_equal(l_gpu, l0), (n, k)
    finally:
        bc.set_walk_limit(prev)


@pytest.mark.parametrize("K", [12, 13, 14, 15, 40, 41, 42, 43])
def test_tile_schedule_strips(K):
    """From K = 12 on the helpers take the tiles eight or more below the
    diagonal in strips of four (operands staged in LDS): every count of tiles
    left for the last strip (K - 7 rows: 1, 2, 3, 0 past whole strips), at
    the smallest K and at wide bands, n ragged, with few tile rows past K
    (strips running into the matrix's end) and with more; the integer factor
    must come out bit for bit."""
    import paper_2305_04635_amd as bc
    prev = bc.set_walk_limit(0)
    try:
        k = 32 * K - 5
        for n in (32 * (K + 2) + 7, 32 * (K + 14) - 3):
            ab = synth.band_diagdom(n, k, 13 * n + K)
            check_against_oracle(ab, k, nrhs=1, seed=K)
            l0 = synth.int_factor(n, k, 19 + K, pow2_max=1)
            l_gpu, info = gpu_factor(synth.band_ldlt(l0, k), k)
            assert info == 0 and np.array_equal(l_gpu, l0), (n, k)
    finally:
        bc.set_walk_limit(prev)


@pytest.mark.parametrize("K", range(1, 16))
def test_walk_each_K(K):
    """The single-workgroup walk at every tile-diagonal count it takes
    (1..15): its trailing updates keep eight blocks per wave in flight, in
    an order that changes with K; n ragged, a few tile rows past K and many;
    the integer factor must come out bit for bit."""
    import paper_2305_04635_amd as bc
    prev = bc.set_walk_limit(15)
    try:
        k = 32 * K - 5
        for n in (32 * (K + 2) + 7, 32 * (3 * K + 6) - 3):
            print("walk", n, k, flush=True)
            ab = synth.band_diagdom(n, k, 3 * n + K)
            check_against_oracle(ab, k, nrhs=1, seed=K)
            l0 = synth.int_factor(n, k, 13 + K, pow2_max=1)
            l_gpu, info = gpu_factor(synth.band_ldlt(l0, k), k)
            assert info == 0 and np.array_equal(l_gpu, l0), (n, k)
    finally:
        bc.set_walk_limit(prev)


@pytest.mark.parametrize("n,k,ldab", [(33, 32, 2900000), (130, 90, 1700000)])
def test_walk_huge_ldab(n, k, ldab):
    """A leading dimension so large that the tile columns one step touches
    span more than 2 GB: the walk takes its per-block path (no buffer
    resource; with K = 3 its panel and update work is split over the seven
    waves as on the buffer path), with the same result."""
    import paper_2305_04635_amd as bc
    prev = bc.set_walk_limit(15)
    try:
        print("walk huge ldab", n, k, ldab, flush=True)
        l0 = synth.int_factor(n, k, 99, pow2_max=1)
        a = synth.band_ldlt(l0, k, ldab=ldab)
        l_gpu, info = gpu_factor(a, k)
        assert info == 0 and np.array_equal(l_gpu[: k + 1], l0)
    finally:
        bc.set_walk_limit(prev)


@pytest.mark.parametrize("wg", [2, 3])
def test_tile_schedule_few_workgroups(wg, monkeypatch):
    """The multi-workgroup schedule with one or two helper workgroups: every
    task only waits for earlier tickets or for spine steps, so it completes
    (and correctly) whatever the number of workgroups."""
    import paper_2305_04635_amd as bc
    monkeypatch.setenv("BANDCHOL_MAX_WG", str(wg))
    prev = bc.set_walk_limit(0)
    try:
        for K in (3, 4, 5, 6, 9):
            n, k = 32 * (2 * K + 4) + 5, 32 * K - 3
            l0 = synth.int_factor(n, k, 23 + K, pow2_max=1)
            l_gpu, info = gpu_factor(synth.band_ldlt(l0, k), k)
            assert info == 0 and np.array_equal(l_gpu, l0), (wg, n, k)
    finally:
        bc.set_walk_limit(prev)


@pytest.mark.parametrize("n,k,nrhs", [(5000, 300, 20), (3000, 40, 9), (700, 699, 4), (4097, 250, 1)])
def test_solve_many_rhs_and_wide_bands(n, k, nrhs):
    """Solves with more right-hand sides than one launch takes and bands wide
    enough for the pre-accumulating helper workgroups."""
    ab = synth.band_diagdom(n, k, 3 * n + k)
    l_or, _ = oracle.factor(ab, k)
    b = synth.rhs(n, nrhs, 11)
    x = gpu_solve(l_or, k, b)
    assert oracle.solve_residual(ab, k, x, b) <= ETA_TOL
    x_or = oracle.solve(l_or, k, b)
    assert np.max(np.abs(x - x_or)) <= 1e-12 * np.max(np.abs(x_or))


def test_sync_factor_workspace_growth():
    """A synchronous factor whose launch has to grow the library's workspace
    (info once lived inside the workspace and was read back from the freed
    buffer after the growth)."""
    import paper_2305_04635_amd as bc
    bc.finalize()
    for n, k in ((300, 100), (5000, 120), (20000, 300)):
        ab = synth.band_diagdom(n, k, n + k)
        l_gpu, info = gpu_factor(ab, k)
        assert info == 0
        rows = [(0, min(n, 96)), (n - min(n, 96), n)]
        assert oracle.llt_residual(l_gpu, ab, k, rows=rows) <= ETA_TOL


@pytest.mark.parametrize("n,k", [(1000, 100), (3000, 300)])
def test_solve_nonfinite_rhs(n, k):
    """Results pass between workgroups by value, with a signalling-NaN pattern
    marking values not yet published; arithmetic never produces that pattern.
    A right-hand side holding NaN and that very bit pattern must still be
    solved (no wait on it), its solution is NaN like the oracle's, and the
    other right-hand side of the same launch is unaffected."""
    ab = synth.band_diagdom(n, k, 7 * n + k)
    l_or, _ = oracle.factor(ab, k)
    b = np.asfortranarray(synth.rhs(n, 2, 5))
    b[n // 2, 0] = np.nan
    b[3, 0] = np.frombuffer(np.uint64(0x7FF4DEADBEEF0001).tobytes(), dtype=np.float64)[0]
    x = gpu_solve(l_or, k, b)
    x_or = oracle.solve(l_or, k, b)
    assert np.array_equal(np.isnan(x[:, 0]), np.isnan(x_or[:, 0]))
    assert np.all(np.isfinite(x[:, 1]))
    assert np.max(np.abs(x[:, 1] - x_or[:, 1])) <= 1e-12 * np.max(np.abs(x_or[:, 1]))


@pytest.mark.parametrize("n,k", [(3000, 300), (5000, 50)])
def test_solve_reports_a_wait_that_gave_up(n, k, monkeypatch):
    """A solve whose bounded wait gives up must not report success.  The
    condition is forced from the host (a testing switch starts the solve with
    its abort flag raised, as a wait that timed out would leave it), so every
    kernel still exits normally: the synchronous solve and the mixed solve
    return BANDCHOL_EHANG; without the switch the same calls succeed."""
    import torch
    import paper_2305_04635_amd as bc
    ab = synth.band_diagdom(n, k, 3 * n + k)
    l_or, _ = oracle.factor(ab, k)
    b = synth.rhs(n, 2, 5)
    monkeypatch.setenv("BANDCHOL_TEST_SOLVE_ABORT", "1")
    with pytest.raises(bc.BandCholError, match=r"\(-1001\)"):
        gpu_solve(l_or, k, b)
    from helpers import to_dev
    d_ab, d_b = to_dev(ab), to_dev(b)
    x = torch.empty_like(d_b)
    with pytest.raises(bc.BandCholError, match=r"\(-1001\)"):
        bc.mixed_solve(d_ab, n, k, d_b, x, nrhs=2)
    monkeypatch.delenv("BANDCHOL_TEST_SOLVE_ABORT")
    x_gpu = gpu_solve(l_or, k, b)
    assert oracle.solve_residual(ab, k, x_gpu, b) <= ETA_TOL
    bc.mixed_solve(d_ab, n, k, d_b, x, nrhs=2)
    assert oracle.solve_residual(ab, k, from_dev(x, b.shape), b) <= ETA_TOL
