"""GPU parity of the schedules a batch plan can take per (n, k) bucket: the
walk (many systems side by side in one persistent launch) or the
multi-workgroup schedule with any workgroup count, as set in the batch
schedule table or chosen by its measurement (bandchol_batch_tune).  Every
choice must give the oracle's factor (integer-exact systems bit for bit, the
others column by column) and the oracle's solution."""
import numpy as np
import pytest

import oracle
import synth
from helpers import ETA_TOL, col_rel_err, from_dev, to_dev

pytestmark = pytest.mark.gpu

# (n, k) per system; the buckets (floor(log2 n), ceil(k/32)) of the first three
# groups get forced schedules below
SHAPES = [(3000, 100), (3500, 110), (2500, 120),      # bucket (11, 4): forced choice A
          (9000, 250), (10000, 240),                 # bucket (13, 8): forced choice B
          (600, 40), (5000, 33), (1200, 300), (4097, 64), (33, 32), (1, 0)]


@pytest.fixture
def clean_tables():
    import paper_2305_04635_amd as bc
    bc.batch_tune_clear()
    yield bc
    bc.batch_tune_clear()


@pytest.mark.parametrize("wa,wb", [(2, 1), (3, 64), (64, 2), (1, 256)])
def test_forced_batch_schedules_match_oracle(clean_tables, wa, wb):
    import torch
    bc = clean_tables
    bc.batch_tune_set(3000, 100, wa)
    bc.batch_tune_set(9000, 250, wb)
    nrhs = 3
    mats, abs_d, bs_d = [], [], []
    for i, (n, k) in enumerate(SHAPES):
        ab = synth.band_diagdom(n, k, 40 + i)
        b = np.asfortranarray(synth.rhs(n, nrhs, 60 + i))
        mats.append((ab, b))
        abs_d.append(to_dev(ab))
        bs_d.append(to_dev(b))
    plan = bc.BatchPlan([n for n, _ in SHAPES], [k for _, k in SHAPES], abs_d, bs_d)
    info = torch.full((len(SHAPES),), -7, dtype=torch.int64, device="cuda")
    plan.factor(info)
    plan.solve(nrhs)
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [0] * len(SHAPES)
    for i, (n, k) in enumerate(SHAPES):
        ab, b = mats[i]
        l_gpu = from_dev(abs_d[i], ab.shape)
        x_gpu = from_dev(bs_d[i], b.shape)
        l_or, _ = oracle.factor(ab, k)
        kk = min(k, n - 1)
        assert col_rel_err(l_gpu[: kk + 1], l_or[: kk + 1]) <= 1e-13 * (kk + 1), (i, n, k)
        assert oracle.solve_residual(ab, k, x_gpu, b) <= ETA_TOL
        x_or = oracle.solve(l_or, k, b)
        assert np.max(np.abs(x_gpu - x_or)) <= 1e-12 * np.max(np.abs(x_or)), (i, n, k)
    plan.close()


@pytest.mark.parametrize("w", [1, 2, 5, 128])
def test_forced_batch_schedule_integer_exact(clean_tables, w):
    import torch
    bc = clean_tables
    shapes = [(1800, 210), (1900, 200), (2000, 195), (700, 50)]
    bc.batch_tune_set(2000, 200, w)            # the first three share bucket (10, 7)
    mats = []
    for i, (n, k) in enumerate(shapes):
        l0 = synth.int_factor(n, k, 90 + i)
        mats.append((l0, synth.band_ldlt(l0, k)))
    abs_d = [to_dev(a) for _, a in mats]
    plan = bc.BatchPlan([n for n, _ in shapes], [k for _, k in shapes], abs_d)
    info = torch.zeros(len(shapes), dtype=torch.int64, device="cuda")
    plan.factor(info)
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [0] * len(shapes)
    for i, (l0, a) in enumerate(mats):
        assert np.array_equal(from_dev(abs_d[i], a.shape), l0), (w, i)
    plan.close()


def test_batch_tune_settles_buckets_and_plans_stay_exact(clean_tables):
    """The measurement runs on device-generated bands, records a choice for the
    buckets it tried, and a plan made afterwards (whatever it chose) still
    returns the integer-exact factors."""
    import torch
    bc = clean_tables
    ns, ks = synth.batch_shapes(48, 5, 1000, 6000, 32, 256)
    ns, ks = ns.tolist(), ks.tolist()
    ms = bc.batch_tune(ns, ks, reps=2, max_buckets=3)
    assert ms > 0
    entries = bc.batch_tune_entries()
    assert 1 <= len(entries) <= 3
    for e in entries:
        assert e["wgs"] >= 1 and e["ms"] > 0
    mats = []
    for i, (n, k) in enumerate(zip(ns, ks)):
        l0 = synth.int_factor_sparse(n, k, 300 + i, min(1.0, 24.0 / k))
        mats.append((l0, synth.band_llt_sparse(l0, k)))
    abs_d = [to_dev(a) for _, a in mats]
    plan = bc.BatchPlan(ns, ks, abs_d)
    info = torch.zeros(len(ns), dtype=torch.int64, device="cuda")
    plan.factor(info)
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [0] * len(ns)
    for i, (l0, a) in enumerate(mats):
        assert np.array_equal(from_dev(abs_d[i], a.shape), l0), i
    plan.close()
