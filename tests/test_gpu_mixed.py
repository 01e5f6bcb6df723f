"""GPU parity of the FP32 factor and the mixed-precision solver against the
oracle's FP32 factor, the FP64 oracle and the pins of the mixed-precision
reference (integer-exact factors, exact non-SPD pivots, refinement to FP64
accuracy, the same fallback decisions)."""
import numpy as np
import pytest

import oracle
import synth
from helpers import from_dev, rel_fro, to_dev

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def gpu_factor_f32(a, k):
    import torch
    import paper_2305_04635_amd as bc
    n = a.shape[1]
    a32 = np.asfortranarray(a.astype(np.float32))
    d = torch.from_numpy(a32.ravel(order="F").copy()).cuda()
    info = torch.zeros(1, dtype=torch.int64, device="cuda")
    bc.factor_f32(d, n, k, info, ldab=a.shape[0])
    torch.cuda.synchronize()
    return d.cpu().numpy().reshape(a.shape, order="F"), int(info.item())


@pytest.mark.parametrize("n,k", [(3000, 50), (2000, 100), (1000, 155), (1337, 190), (1000, 250), (500, 499), (33, 32),
                                 (1, 0)])
def test_factor_f32_integer_exact(n, k):
    """Unit pivots only: the trsm multiplies by L(C,C)^{-T}, whose entries are
    then integers (below 2^15 for these seeds) and exact in FP32.  With pivots
    2^m the inverse needs more than 24 bits, and these +-1 factors are
    exponentially ill-conditioned, so FP32 rounding there is amplified until a
    pivot fails (the division-based oracle stays exact only because each of
    its quotients is); FP64 carries those cases exactly."""
    l0 = synth.int_factor(n, k, 17 + k, pow2_max=0)
    a = synth.band_ldlt(l0, k)
    l32, info = gpu_factor_f32(a, k)
    assert info == 0
    assert np.array_equal(l32.astype(np.float64), l0)


@pytest.mark.parametrize("n,k", [(2000, 100), (1500, 96), (777, 200), (3001, 33), (1300, 420), (2900, 1291)])
def test_factor_f32_matches_oracle(n, k):
    ab = synth.band_diagdom(n, k, 5 * n + k)
    l32, info = gpu_factor_f32(ab, k)
    assert info == 0
    assert oracle.llt_residual(l32.astype(np.float64), ab, k) <= 4 * (k + 1) * U32
    ref = np.asfortranarray(ab.astype(np.float32))
    assert oracle.spbtrf(ref, k) == 0
    assert rel_fro(l32.astype(np.float64), ref.astype(np.float64)) <= 1e-5


@pytest.mark.parametrize("m", [0, 31, 32, 250, 599])
def test_factor_f32_nonspd_info(m):
    n, k = 600, 100
    l0 = synth.int_factor(n, k, 99)
    dvec = np.ones(n)
    dvec[m] = -1.0
    a = synth.band_ldlt(l0, k, dvec)
    _, info = gpu_factor_f32(a, k)
    ref = np.asfortranarray(a.astype(np.float32))
    assert info == m + 1 == oracle.spbtrf(ref, k)


@pytest.mark.parametrize("n,k,nrhs,d", [(3000, 40, 3, 1), (3000, 40, 3, 2), (3000, 40, 3, 3), (3000, 40, 3, 5),
                                        (20000, 300, 8, 2), (4000, 120, 1, 4)])
def test_mixed_solve_matches_oracle(n, k, nrhs, d):
    import torch
    import paper_2305_04635_amd as bc
    ab, _ = synth.band_ipm(n, k, 70 + d, diag_exp_lo=-float(d), shift_rel=10.0 ** (-2 * d))
    b = np.asfortranarray(synth.rhs(n, nrhs, 9).reshape(n, nrhs))
    dab, db = to_dev(ab), to_dev(b)
    dx = torch.zeros_like(db)
    it, fb = bc.mixed_solve(dab, n, k, db, dx, nrhs=nrhs)
    x = from_dev(dx, (n, nrhs))
    assert np.array_equal(from_dev(dab, ab.shape), ab)          # A is read only
    x_or, it_or, fb_or = oracle.mixed_solve(ab, k, b)
    assert (fb is None) == (fb_or is None), (it, fb, it_or, fb_or)
    if fb is None:
        assert abs(it - it_or) <= 1, (it, it_or)
    l64, _ = oracle.factor(ab, k)
    x64 = oracle.solve(l64, k, b)
    kap = oracle.cond1_estimate(ab, l64, k)
    anrm = oracle.norm_inf(ab, k)
    for c in range(nrhs):
        r = b[:, c] - oracle.symv(ab, k, x[:, c])
        assert np.max(np.abs(r)) <= 1.01 * np.sqrt(n) * 2.0 ** -53 * anrm * np.max(np.abs(x[:, c]))
        assert np.max(np.abs(x[:, c] - x64[:, c])) / np.max(np.abs(x64[:, c])) <= 1e-12 * kap
