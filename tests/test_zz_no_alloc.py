"""The factor entry point that allocates nothing (bandchol_factor_noalloc),
through the C-ABI: its result equals bandchol_factor_async's bit for bit (same
kernels and schedule, working memory from the library's fixed device array) on
two calls in a row, the second smaller than the first, so that the second
starts from what the first left in the array; a band too large for the array
is rejected before anything is launched."""
import numpy as np
import pytest

import synth
from helpers import from_dev, to_dev

pytestmark = pytest.mark.gpu


def factor_both(ab, n, k):
    import torch
    import paper_2305_04635_amd as bc
    d_ref, d_new = to_dev(ab), to_dev(ab)
    info = torch.full((2,), -7, dtype=torch.int64, device="cuda")
    bc.factor_async(d_ref, n, k, info[0:1])
    bc.factor_noalloc(d_new, n, k, info[1:2])
    torch.cuda.synchronize()
    return from_dev(d_ref, ab.shape), from_dev(d_new, ab.shape), info.cpu().tolist()


@pytest.mark.parametrize("first,second", [((100000, 1000), (20000, 300)), ((30000, 2000), (3001, 200))])
def test_noalloc_matches_factor_async(first, second):
    for (n, k) in (first, second):
        print("noalloc factor n=%d k=%d" % (n, k), flush=True)
        ab = synth.band_diagdom(n, k, 11 * n + k)
        l_ref, l_new, info = factor_both(ab, n, k)
        assert info == [0, 0]
        assert np.array_equal(l_new, l_ref), (n, k)


def test_noalloc_integer_exact_and_info():
    import torch
    import paper_2305_04635_amd as bc
    n, k = 5000, 180
    l0 = synth.int_factor(n, k, 321)
    a = synth.band_ldlt(l0, k)
    l_ref, l_new, info = factor_both(a, n, k)
    assert info == [0, 0] and np.array_equal(l_new, l0) and np.array_equal(l_ref, l0)
    dvec = np.ones(n)
    dvec[777] = -1.0
    a = synth.band_ldlt(l0, k, dvec)
    _, _, info = factor_both(a, n, k)
    assert info == [778, 778]


def test_noalloc_rejects_too_large_band():
    import torch
    import paper_2305_04635_amd as bc
    n, k = 140000, 64
    d_ab = torch.zeros(n * (k + 1), dtype=torch.float64, device="cuda")
    info = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    with pytest.raises(bc.BandCholError, match=r"\(-1002\)"):
        bc.factor_noalloc(d_ab, n, k, info)
    torch.cuda.synchronize()
    assert info.item() == -7                # nothing was launched
    # n = 0 and a diagonal band need no working memory
    bc.factor_noalloc(d_ab, 0, k, info)
    torch.cuda.synchronize()
    assert info.item() == 0
