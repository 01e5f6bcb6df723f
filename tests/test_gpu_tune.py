"""GPU: the schedule table per (n, k) bucket.  The measurement records one of
its candidates, every schedule (the walk, the tile schedule with any number of
workgroups) yields the oracle's factor, and the schedules of the tile
schedule agree bit for bit: which workgroup takes a tile task does not change
the order of its sums."""
import numpy as np
import pytest

import oracle
import synth
from helpers import ETA_TOL, gpu_factor, rel_fro

pytestmark = pytest.mark.gpu

SPINE_COUNTS = {32, 64, 96, 128, 192, 256, 320, 384, 448, 512}


@pytest.fixture(autouse=True)
def empty_table():
    import paper_2305_04635_amd as bc
    bc.tune_clear()
    yield bc
    bc.tune_clear()


def candidates(bc, n, k):
    kk = min(k, n - 1)
    K = -(-kk // bc.tile())
    if K == 0:
        return {1}
    rule = 64 if K <= 11 else 256 if K <= 55 else 512
    return ({1} if K <= 15 else set()) | SPINE_COUNTS | {rule}


@pytest.mark.parametrize("n,k", [(3000, 200), (5000, 1000), (1000, 0), (1, 7), (2, 1), (700, 699)])
def test_tune_records_a_measured_schedule(empty_table, n, k):
    bc = empty_table
    print("tune", n, k, flush=True)
    wgs, ms = bc.tune_factor(n, k, reps=2)
    assert wgs in candidates(bc, n, k)
    assert ms > 0
    assert bc.schedule(n, k) == wgs
    entries = bc.tune_entries()
    assert len(entries) == 1
    assert entries[0]["wgs"] == wgs and entries[0]["n"] == n and entries[0]["k"] == min(k, n - 1)
    assert entries[0]["ms"] == pytest.approx(ms)
    # the factor now runs with the measured schedule
    ab = synth.band_diagdom(n, k, 77 + n)
    l_gpu, info = gpu_factor(ab, k)
    assert info == 0
    assert oracle.llt_residual(l_gpu, ab, k) <= ETA_TOL
    l_or, _ = oracle.factor(ab, k)
    kk = min(k, n - 1)
    assert rel_fro(l_gpu[: kk + 1], l_or[: kk + 1]) <= 1e-13 * (kk + 1)


def test_tune_second_measurement_replaces_the_bucket(empty_table):
    bc = empty_table
    bc.tune_set(2500, 300, 96)
    wgs, _ = bc.tune_factor(3000, 310, reps=1)      # same bucket: floor(log2 n) = 11, K = 10
    entries = bc.tune_entries()
    assert len(entries) == 1 and entries[0]["wgs"] == wgs and entries[0]["n"] == 3000


@pytest.mark.parametrize("K", [1, 2, 5, 9, 17])
def test_every_schedule_gives_the_exact_factor(empty_table, K):
    """Integer factor with unit and power-of-two pivots: every step is exact,
    so each schedule must return L itself."""
    bc = empty_table
    n, k = 32 * (2 * K + 5) + 11, 32 * K - 5
    l0 = synth.int_factor(n, k, 41 + K, pow2_max=1)
    ab = synth.band_ldlt(l0, k)
    for wgs in ([1] if K <= 15 else []) + [2, 3, 64, 96, 200, 512]:
        bc.tune_set(n, k, wgs)
        assert bc.schedule(n, k) == wgs
        print("schedule", n, k, wgs, flush=True)
        l_gpu, info = gpu_factor(ab, k)
        assert info == 0 and np.array_equal(l_gpu, l0), (K, wgs)


@pytest.mark.parametrize("n,k", [(4000, 130), (2500, 700)])
def test_tile_schedule_counts_agree_bitwise(empty_table, n, k):
    bc = empty_table
    ab = synth.band_diagdom(n, k, 5 * n + k)
    first = None
    for wgs in (2, 64, 160, 512):
        bc.tune_set(n, k, wgs)
        print("schedule", n, k, wgs, flush=True)
        l_gpu, info = gpu_factor(ab, k)
        assert info == 0
        if first is None:
            first = l_gpu
            assert oracle.llt_residual(l_gpu, ab, k) <= ETA_TOL
        else:
            assert np.array_equal(l_gpu, first), wgs


def test_batch_plan_takes_the_table_entry(empty_table):
    """A batch plan reads the table for its wide systems when it is created."""
    import torch
    bc = empty_table
    from helpers import from_dev, to_dev
    shapes = [(3000, 600), (1500, 40)]
    bc.tune_set(3000, 600, 96)
    abs_h = [synth.band_diagdom(n, k, 900 + n) for n, k in shapes]
    abs_d = [to_dev(a) for a in abs_h]
    plan = bc.BatchPlan([n for n, _ in shapes], [k for _, k in shapes], abs_d)
    info = torch.full((2,), -7, dtype=torch.int64, device="cuda")
    plan.factor(info)
    torch.cuda.synchronize()
    assert info.tolist() == [0, 0]
    for (n, k), a, d in zip(shapes, abs_h, abs_d):
        l_gpu = from_dev(d, a.shape)
        assert oracle.llt_residual(l_gpu, a, k) <= ETA_TOL


@pytest.mark.parametrize("k", [50, 700])
def test_spine_profile_accounts_for_the_step(k):
    """The spine's phase times (s_memtime) add up: wave 0's four phases cover
    its whole step, waves 1-3 are in step with it, and the implied shader
    clock is a plausible one; the pivot-chain probe is far below a step."""
    import paper_2305_04635_amd as bc
    n = 20000
    d = bc.spine_profile(n, k, reps=2)
    nb = (n + 31) // 32
    assert d["steps"] == nb - 1
    w0 = d["sweep"] + d["w0_wait"] + d["bc_w0"] + d["bc_wait"]
    ghz = w0 * d["steps"] / (d["factor_ms"] * 1e-3) / 1e9
    assert 0.5 < ghz < 3.5, ghz
    for w in (1, 2, 3):
        # the phase-A work and wait of waves 1-3 span wave 0's phase A
        assert abs(d["w%d_work" % w] + d["w%d_wait" % w] - (d["sweep"] + d["w0_wait"])) < 0.25 * w0
    ns = bc.pivot_chain_ns(1 << 16)
    assert 1.0 < ns < 1000.0 and 32 * ns * 1e-9 < d["factor_ms"] * 1e-3 / d["steps"]
