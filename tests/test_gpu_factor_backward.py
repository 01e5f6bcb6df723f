"""GPU parity of the reverse mode of the factorization (bandchol_factor_backward)
and of the differentiable factor (band_cholesky), through the C-ABI: against
the oracle's reverse sweep of Algorithm 2, the dense closed form at n = 500,
the log-det identity, and central finite differences of the oracle's loss.
Also the recompute option of the differentiable solves (the backward pass
factors A again instead of keeping L): same gradients as without it.

Bar: relative Frobenius error <= 1e-11 against the oracle on diagonally
dominant inputs (both sides are reverse sweeps of backward-stable factor
steps; their difference is rounding, of order (k+1) u times the condition of
the products with the tile inverses), 1e-10 against the dense closed form
(numpy inverses), 1e-6 (1 + |g|) against finite differences (h = 1e-6).
"""
import numpy as np
import pytest

import oracle
import synth
from helpers import dense_of, from_dev, to_dev

pytestmark = pytest.mark.gpu


def random_lbar(n, k, seed, ldab=None):
    ldab = k + 1 if ldab is None else ldab
    lb = np.zeros((ldab, n), order="F")
    lb[: k + 1] = synth.normal((k + 1) * n, seed, 3).reshape(k + 1, n, order="F")
    for j in range(max(n - k, 0), n):
        lb[n - j: k + 1, j] = 0.0
    return lb


def gpu_factor_backward(l, k, lbar, fill=np.nan):
    import torch
    import paper_2305_04635_amd as bc
    n = l.shape[1]
    d_l, d_lb = to_dev(l), to_dev(lbar)
    d_ab = to_dev(np.full(lbar.shape, fill, order="F"))
    status = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    bc.factor_backward(d_l, n, k, d_lb, d_ab, d_status=status, ldl=l.shape[0], ldlb=lbar.shape[0],
                       ldab=lbar.shape[0])
    torch.cuda.synchronize()
    assert status.item() == 0
    return from_dev(d_ab, lbar.shape)


def rel(x, ref):
    return float(np.linalg.norm(x - ref) / max(np.linalg.norm(ref), 1e-300))


@pytest.mark.parametrize("n,k", [
    (1, 0), (40, 0), (33, 1), (64, 5), (100, 31), (100, 32), (257, 64), (300, 299), (500, 499),
    (1000, 33), (777, 130), (2049, 200), (3001, 96), (4000, 400), (1500, 1000),
])
def test_factor_backward_matches_oracle(n, k):
    ab = synth.band_diagdom(n, k, 17 * n + k)
    l, info = oracle.factor(ab, k)
    assert info == 0
    lbar = random_lbar(n, k, 3 * n + k)
    ref = oracle.pbtrf_backward(l, k, lbar)
    got = gpu_factor_backward(l, k, lbar)
    kk = min(k, n - 1)
    # entries outside the matrix (bottom-right corner) are never written
    for j in range(max(n - kk, 0), n):
        assert np.all(np.isnan(got[n - j: kk + 1, j]))
        got[n - j: kk + 1, j] = 0.0
    assert rel(got[: kk + 1], ref[: kk + 1]) <= 1e-11, rel(got[: kk + 1], ref[: kk + 1])


def test_factor_backward_in_place_and_ldab():
    """abar may be the very array lbar; rows past k of a padded layout untouched."""
    import torch
    import paper_2305_04635_amd as bc
    n, k, pad = 1200, 70, 5
    ab = synth.band_diagdom(n, k, 8)
    l, _ = oracle.factor(ab, k)
    lbar = random_lbar(n, k, 9, ldab=k + 1 + pad)
    lbar[k + 1:] = np.nan
    ref = oracle.pbtrf_backward(l, k, lbar[: k + 1])
    lpad = np.full((k + 1 + pad, n), np.nan, order="F")
    lpad[: k + 1] = l
    d_l, d_g = to_dev(lpad), to_dev(lbar)
    bc.factor_backward(d_l, n, k, d_g, d_g, ldl=k + 1 + pad, ldlb=k + 1 + pad, ldab=k + 1 + pad)
    torch.cuda.synchronize()
    got = from_dev(d_g, lbar.shape)
    assert np.all(np.isnan(got[k + 1:]))
    assert rel(got[: k + 1], ref) <= 1e-11


def test_factor_backward_dense_closed_form_n500():
    n, k = 500, 60
    ab = synth.band_diagdom(n, k, 500)
    l, _ = oracle.factor(ab, k)
    lbar = random_lbar(n, k, 501)
    got = gpu_factor_backward(l, k, lbar, fill=0.0)
    L = np.zeros((n, n))
    Lb = np.zeros((n, n))
    for j in range(n):
        for d in range(min(k, n - 1 - j) + 1):
            L[j + d, j] = l[d, j]
            Lb[j + d, j] = lbar[d, j]
    P = L.T @ Lb
    Phi = np.tril(P) - 0.5 * np.diag(np.diag(P))
    Li = np.linalg.inv(L)
    S = Li.T @ Phi @ Li
    G = np.tril(S + S.T) - np.diag(np.diag(S))
    ref = np.zeros_like(got)
    for j in range(n):
        for d in range(min(k, n - 1 - j) + 1):
            ref[d, j] = G[j + d, j]
    assert rel(got, ref) <= 1e-10


def test_factor_backward_log_det():
    """Lbar = diag(1/L_ii): the gradient of log det(A) / 2, the band of A^{-1} / 2
    with off-diagonal entries counted for both triangles."""
    n, k = 600, 90
    ab = synth.band_diagdom(n, k, 600)
    l, _ = oracle.factor(ab, k)
    lbar = np.zeros((k + 1, n), order="F")
    lbar[0] = 1.0 / l[0]
    got = gpu_factor_backward(l, k, lbar, fill=0.0)
    ainv = np.linalg.inv(dense_of(ab, k))
    ref = np.zeros_like(got)
    for j in range(n):
        for d in range(min(k, n - 1 - j) + 1):
            ref[d, j] = ainv[j + d, j] * (0.5 if d == 0 else 1.0)
    assert rel(got, ref) <= 1e-10


@pytest.mark.parametrize("n,k", [(20000, 500), (4000, 1200), (100000, 64)])
def test_factor_backward_large(n, k):
    """Bands wide enough for many workgroups per step (K = 16 and 38, a grid
    barrier per tile column) and a long one; against the oracle's sweep."""
    print("factor backward n=%d k=%d" % (n, k), flush=True)
    ab = synth.band_diagdom(n, k, n + k)
    l, _ = oracle.factor(ab, k, columns=True)
    lbar = random_lbar(n, k, n + 2 * k)
    ref = oracle.pbtrf_backward(l, k, lbar)
    got = gpu_factor_backward(l, k, lbar, fill=0.0)
    assert rel(got, ref) <= 1e-11, rel(got, ref)


def test_band_cholesky_autograd_central_differences():
    import torch
    import paper_2305_04635_amd as bc
    n, k = 300, 24
    ab = synth.band_diagdom(n, k, 42)
    lbar = random_lbar(n, k, 43)
    abt = torch.from_numpy(ab.T.copy()).cuda().requires_grad_(True)
    w = torch.from_numpy(lbar.T.copy()).cuda()
    L = bc.band_cholesky(abt, k)
    (w * L).sum().backward()
    g = abt.grad.cpu().numpy().T

    def loss(a):
        ll, info = oracle.factor(a, k)
        assert info == 0
        return float(np.sum(lbar * ll))

    rng = np.random.default_rng(5)
    h = 1e-6
    for _ in range(50):
        j = int(rng.integers(0, n))
        d = int(rng.integers(0, min(k, n - 1 - j) + 1))
        ap, am = ab.copy(order="F"), ab.copy(order="F")
        ap[d, j] += h
        am[d, j] -= h
        fd = (loss(ap) - loss(am)) / (2 * h)
        assert abs(fd - g[d, j]) <= 1e-6 * (1 + abs(g[d, j])), (d, j, fd, g[d, j])
    # log det through the differentiable factor: gradient = band of A^{-1} (half on the diagonal)
    abt.grad = None
    L = bc.band_cholesky(abt, k)
    torch.log(L[:, 0]).sum().backward()
    ainv = np.linalg.inv(dense_of(ab, k))
    g = abt.grad.cpu().numpy().T
    ref = np.zeros_like(g)
    for j in range(n):
        for d in range(min(k, n - 1 - j) + 1):
            ref[d, j] = ainv[j + d, j] * (0.5 if d == 0 else 1.0)
    assert rel(g, ref) <= 1e-10


@pytest.mark.parametrize("nrhs", [1, 3])
def test_solve_recompute_matches_saved_factor(nrhs):
    import torch
    import paper_2305_04635_amd as bc
    n, k = 3000, 150
    ab = synth.band_diagdom(n, k, 77)
    b = np.ascontiguousarray(synth.rhs(n, nrhs, 78))
    w = torch.from_numpy(synth.normal(n * nrhs, 79, 0).reshape(n, nrhs)).cuda()
    grads = []
    for rec in (False, True):
        abt = torch.from_numpy(ab.T.copy()).cuda().requires_grad_(True)
        bt = torch.from_numpy(b).cuda().requires_grad_(True)
        x = bc.band_solve(abt, bt, k, recompute=rec)
        (w * x).sum().backward()
        grads.append((abt.grad.cpu().numpy(), bt.grad.cpu().numpy()))
    assert np.array_equal(grads[0][0], grads[1][0]) and np.array_equal(grads[0][1], grads[1][1])


def test_batch_recompute_matches_saved_factor():
    import torch
    import paper_2305_04635_amd as bc
    bsz, n, k, nrhs = 6, 2000, 120, 2
    abs_ = np.stack([synth.band_diagdom(n, k, 300 + i).T for i in range(bsz)])
    bs = np.stack([synth.rhs(n, nrhs, 400 + i) for i in range(bsz)])
    w = torch.from_numpy(synth.normal(bsz * n * nrhs, 81, 0).reshape(bsz, n, nrhs)).cuda()
    grads = []
    for rec in (False, True):
        abt = torch.from_numpy(abs_.copy()).cuda().requires_grad_(True)
        bt = torch.from_numpy(bs.copy()).cuda().requires_grad_(True)
        x = bc.band_solve_batch(abt, bt, k, recompute=rec)
        (w * x).sum().backward()
        grads.append((abt.grad.cpu().numpy(), bt.grad.cpu().numpy()))
    assert np.array_equal(grads[0][0], grads[1][0]) and np.array_equal(grads[0][1], grads[1][1])
