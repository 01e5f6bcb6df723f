"""GPU parity of the batched factor and solve (bandchol_batch_*): every system
of a batch of mixed orders and bandwidths against the CPU oracle, info per
system, several right-hand-side passes, and replays of a captured HIP graph."""
import numpy as np
import pytest

import oracle
import synth
from helpers import ETA_TOL, col_rel_err, from_dev, rel_fro, to_dev

pytestmark = pytest.mark.gpu

# (n, k): empty, scalar, ragged, dense (k >= n-1), every tile-diagonal count of
# the walk up to its limit, and bands too wide for it (k > 15 tiles = 480).
SHAPES = [(0, 5), (1, 0), (37, 3), (64, 5), (33, 32), (1000, 32), (2049, 33), (2000, 64), (777, 130),
          (500, 499), (3001, 256), (1200, 480), (1500, 600), (900, 1000), (4000, 1)]


def build(shapes, nrhs, seed):
    import torch
    abs_h, bs_h, abs_d, bs_d = [], [], [], []
    for idx, (n, k) in enumerate(shapes):
        if n == 0:
            ab = np.zeros((k + 1, 0), order="F")
            b = np.zeros((0, nrhs), order="F")
        else:
            ab = synth.band_diagdom(n, k, seed + 7 * idx)
            b = np.asfortranarray(synth.rhs(n, nrhs, seed + idx).reshape(n, nrhs))
        abs_h.append(ab)
        bs_h.append(b)
        abs_d.append(to_dev(ab) if n else torch.zeros(1, dtype=torch.float64, device="cuda"))
        bs_d.append(to_dev(b) if n else torch.zeros(1, dtype=torch.float64, device="cuda"))
    return abs_h, bs_h, abs_d, bs_d


def check_system(ab, b, l_gpu, x_gpu, k):
    n = ab.shape[1]
    if n == 0:
        return
    assert oracle.llt_residual(l_gpu, ab, k) <= ETA_TOL
    assert oracle.solve_residual(ab, k, x_gpu, b) <= ETA_TOL
    l_or, _ = oracle.factor(ab, k)
    kk = min(k, n - 1)
    assert col_rel_err(l_gpu[: kk + 1], l_or[: kk + 1]) <= 1e-13 * (kk + 1)
    x_or = oracle.solve(l_or, k, b)
    assert np.max(np.abs(x_gpu - x_or)) <= 1e-12 * np.max(np.abs(x_or))


@pytest.mark.parametrize("nrhs", [4, 11])
def test_batch_mixed_shapes(nrhs):
    import torch
    import paper_2305_04635_amd as bc
    abs_h, bs_h, abs_d, bs_d = build(SHAPES, nrhs, 100 + nrhs)
    ns = [n for n, _ in SHAPES]
    ks = [k for _, k in SHAPES]
    plan = bc.BatchPlan(ns, ks, abs_d, bs_d)
    info = torch.full((len(SHAPES),), -7, dtype=torch.int64, device="cuda")
    plan.factor(info)
    plan.solve(nrhs)
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [0] * len(SHAPES)
    for i, (n, k) in enumerate(SHAPES):
        if n == 0:
            continue
        l_gpu = from_dev(abs_d[i], abs_h[i].shape)
        x_gpu = from_dev(bs_d[i], bs_h[i].shape)
        check_system(abs_h[i], bs_h[i], l_gpu, x_gpu, k)
    plan.close()


def test_batch_info_per_system():
    """Non-positive-definite systems report their own first failing column;
    the others in the batch are factored normally."""
    import torch
    import paper_2305_04635_amd as bc
    shapes, mats, expect = [], [], []
    for j, (n, k, m) in enumerate([(600, 40, 31), (800, 100, None), (700, 250, 0), (300, 20, 299),
                                   (1000, 600, 517), (500, 64, None)]):
        l0 = synth.int_factor(n, k, 50 + j)
        dvec = np.ones(n)
        if m is not None:
            dvec[m] = -1.0
        a = synth.band_ldlt(l0, k, dvec)
        shapes.append((n, k))
        mats.append((a, l0))
        expect.append(0 if m is None else m + 1)
        assert oracle.factor(a, k)[1] == expect[-1]
    abs_d = [to_dev(a) for a, _ in mats]
    plan = bc.BatchPlan([n for n, _ in shapes], [k for _, k in shapes], abs_d)
    info = torch.zeros(len(shapes), dtype=torch.int64, device="cuda")
    plan.factor(info)
    torch.cuda.synchronize()
    assert info.cpu().tolist() == expect
    for i, (a, l0) in enumerate(mats):
        if expect[i] == 0:
            assert np.array_equal(from_dev(abs_d[i], a.shape), l0)   # integer-exact factor
    plan.close()


def test_batch_graph_replay():
    """Factor + solve of a batch captured in a HIP graph: every replay, with
    eager work in between, reproduces the eager result bit for bit."""
    import torch
    import paper_2305_04635_amd as bc
    shapes = [(1500, 40), (3000, 200), (777, 96), (2000, 600), (100, 99)]
    nrhs = 4
    abs_h, bs_h, abs_d, bs_d = build(shapes, nrhs, 900)
    ab0 = [t.clone() for t in abs_d]
    b0 = [t.clone() for t in bs_d]
    plan = bc.BatchPlan([n for n, _ in shapes], [k for _, k in shapes], abs_d, bs_d)
    info = torch.zeros(len(shapes), dtype=torch.int64, device="cuda")

    def restore_and_run():
        for t, t0 in zip(abs_d, ab0):
            t.copy_(t0)
        for t, t0 in zip(bs_d, b0):
            t.copy_(t0)
        plan.factor(info)
        plan.solve(nrhs)

    restore_and_run()
    torch.cuda.synchronize()
    ref_l = [t.clone() for t in abs_d]
    ref_x = [t.clone() for t in bs_d]
    for i, (n, k) in enumerate(shapes):
        check_system(abs_h[i], bs_h[i], from_dev(abs_d[i], abs_h[i].shape), from_dev(bs_d[i], bs_h[i].shape), k)

    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g):
            restore_and_run()
    torch.cuda.current_stream().wait_stream(side)
    scratch_ab = to_dev(synth.band_diagdom(5000, 300, 3))
    for rep in range(3):
        for t in abs_d + bs_d:
            t.fill_(np.nan)
        info.fill_(-5)
        g.replay()
        torch.cuda.synchronize()
        assert info.cpu().tolist() == [0] * len(shapes), rep
        for t, r in zip(abs_d + bs_d, ref_l + ref_x):
            assert torch.equal(t, r), rep
        bc.factor(scratch_ab.clone(), 5000, 300)   # unrelated eager work between replays
        torch.cuda.synchronize()
    plan.close()


def _pool():
    import os
    from concurrent.futures import ThreadPoolExecutor
    return ThreadPoolExecutor(max(1, min(16, os.cpu_count() or 1)))


@pytest.mark.parametrize("nrhs", [4])
def test_batch_more_systems_than_workgroups(nrhs):
    """600 systems of the batched workload's shapes (n ~ U{1000..20000}, k ~
    U{32..256}, diagonally dominant) -- more than the resident workgroups of
    the persistent walk, so that workgroups take a second and third system
    from the queue and reuse their LDS.  Every system's L (column by column)
    and x against the oracle's."""
    import torch
    import paper_2305_04635_amd as bc
    ns, ks = synth.batch_shapes(600, 77, 1000, 20000, 32, 256)
    shapes = list(zip(ns.tolist(), ks.tolist()))
    print("batch of", len(shapes), "systems", flush=True)
    with _pool() as ex:
        abs_h = list(ex.map(lambda t: synth.band_diagdom(t[1][0], t[1][1], 5000 + t[0]), enumerate(shapes)))
    bs_h = [np.asfortranarray(synth.rhs(n, nrhs, 6000 + i).reshape(n, nrhs)) for i, (n, k) in enumerate(shapes)]
    abs_d = [to_dev(a) for a in abs_h]
    bs_d = [to_dev(b) for b in bs_h]
    plan = bc.BatchPlan(ns.tolist(), ks.tolist(), abs_d, bs_d)
    info = torch.full((len(shapes),), -7, dtype=torch.int64, device="cuda")
    plan.factor(info)
    plan.solve(nrhs)
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [0] * len(shapes)

    def check(i):
        n, k = shapes[i]
        l_gpu = from_dev(abs_d[i], abs_h[i].shape)
        x_gpu = from_dev(bs_d[i], bs_h[i].shape)
        l_or, info_or = oracle.factor(abs_h[i], k)
        assert info_or == 0
        err_l = col_rel_err(l_gpu, l_or)
        x_or = oracle.solve(l_or, k, bs_h[i])
        err_x = float(np.max(np.abs(x_gpu - x_or)) / np.max(np.abs(x_or)))
        res = oracle.solve_residual(abs_h[i], k, x_gpu, bs_h[i])
        return err_l <= 1e-13 * (k + 1) and err_x <= 1e-12 and res <= ETA_TOL, (i, n, k, err_l, err_x, res)

    with _pool() as ex:
        results = list(ex.map(check, range(len(shapes))))
    bad = [r for ok, r in results if not ok]
    assert not bad, bad[:5]
    plan.close()


def test_batch_more_systems_integer_exact():
    """700 integer-exact systems (sparse unit L0 with entries in {-1, 0, 1},
    n ~ U{300..6000}, k ~ U{1..300}, right-hand sides A x0 with integer x0):
    the walk and its queue must return L0 and x0 bit for bit for every system,
    whichever workgroup takes it and whatever the system it took before."""
    import torch
    import paper_2305_04635_amd as bc
    ns, ks = synth.batch_shapes(700, 78, 300, 6000, 1, 300)
    shapes = list(zip(ns.tolist(), ks.tolist()))

    def make(i):
        n, k = shapes[i]
        l0 = synth.int_factor_sparse(n, k, 7000 + i, min(1.0, 24.0 / k))
        a = synth.band_llt_sparse(l0, k)
        x0 = synth.int_vector(2 * n, 8000 + i).reshape(n, 2, order="F")
        return l0, a, x0, synth.band_symv(a, k, x0)

    with _pool() as ex:
        mats = list(ex.map(make, range(len(shapes))))
    abs_d = [to_dev(m[1]) for m in mats]
    bs_d = [to_dev(m[3]) for m in mats]
    plan = bc.BatchPlan(ns.tolist(), ks.tolist(), abs_d, bs_d)
    info = torch.full((len(shapes),), -7, dtype=torch.int64, device="cuda")
    plan.factor(info)
    plan.solve(2)
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [0] * len(shapes)
    for i, (l0, a, x0, _) in enumerate(mats):
        assert np.array_equal(from_dev(abs_d[i], a.shape), l0), (i, shapes[i])
        assert np.array_equal(from_dev(bs_d[i], x0.shape), x0), (i, shapes[i])
    plan.close()
