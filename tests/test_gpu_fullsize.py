"""GPU parity at the benchmark's size: n = 100000 and every bandwidth of the
sweep, k in {50, 100, 250, 500, 1000, 2000}, in the benchmark's launch
configuration (the library's default schedule and workgroup count, the
synchronous factor and the solve with one right-hand side).

Two inputs per k:

* an integer-exact band A = L0 L0^T with L0 unit lower triangular, entries in
  {-1, 0, 1} (dense for k <= 250; beyond, each off-diagonal position is
  nonzero with probability 64/k, so that A is cheap to form): the factor is
  unique (Section 2) and every value any correct factorization forms is an
  integer, so L must equal L0 and the solve of A x = A x0 must return x0,
  bit for bit;
* the benchmark's own interior-point-like matrix (same recipe and seed): the
  backward error of L over the whole band, the solve residual, the forward
  error of x against the oracle's x within 1e-12 kappa_1(A), and every
  column of L against the oracle's (relative to the column's norm, within the
  same kappa-scaled bound, since elementwise L is only bounded through kappa).

The oracle's factor runs in its column-order form (bitwise equal to the row
form, threaded); the backward error is summed over row blocks on a thread
pool.  Both are plain CPU C code from ``oracle/``.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import synth
from helpers import ETA_TOL, gpu_factor, gpu_solve

pytestmark = pytest.mark.gpu

N = 100000
KS = (50, 100, 250, 500, 1000, 2000)
SEED = 1000           # the benchmark's seed: matrix of bandwidth k has seed SEED + k


def threads():
    return max(1, min(16, os.cpu_count() or 1))


def llt_residual_threaded(l_band, a_band, k):
    """||L L^T - A||_F / ||A||_F over the whole band, rows split over threads
    (the oracle routine returns the two squared sums of a row range)."""
    n = a_band.shape[1]
    step = max(1, -(-n // (4 * threads())))
    ranges = [(lo, min(n, lo + step)) for lo in range(0, n, step)]
    out = np.zeros((len(ranges), 2))

    def part(i):
        lo, hi = ranges[i]
        o = np.zeros(2)
        oracle._load().oracle_llt_residual_rows(
            oracle._I64(n), oracle._I64(k), oracle._p(l_band), oracle._I64(l_band.shape[0]),
            oracle._p(a_band), oracle._I64(a_band.shape[0]), oracle._I64(lo), oracle._I64(hi),
            o.ctypes.data_as(oracle._D))
        out[i] = o

    with ThreadPoolExecutor(threads()) as ex:
        list(ex.map(part, range(len(ranges))))
    num, den = out.sum(axis=0)
    return float(np.sqrt(num / den))


def integer_case(k):
    if k <= 250:
        l0 = synth.int_factor(N, k, 4000 + k)
        a = synth.band_ldlt(l0, k)
    else:
        l0 = synth.int_factor_sparse(N, k, 4000 + k, 64.0 / k)
        a = synth.band_llt_sparse(l0, k)
    return l0, a


@pytest.mark.parametrize("k", KS)
def test_fullsize_integer_exact_bitwise(k):
    print("full-size integer-exact k =", k, flush=True)
    l0, a = integer_case(k)
    l_gpu, info = gpu_factor(a, k)
    assert info == 0
    mism = np.flatnonzero((l_gpu != l0).any(axis=0))
    assert mism.size == 0, "first differing column %d of %d" % (mism[0], mism.size)
    x0 = synth.int_vector(N, 17 + k)
    b = synth.band_symv(a, k, x0)
    x = gpu_solve(l_gpu, k, b)
    assert np.array_equal(x, x0), int(np.flatnonzero(x != x0)[0])


@pytest.mark.parametrize("k", KS)
def test_fullsize_ipm_against_oracle(k):
    print("full-size interior-point-like k =", k, flush=True)
    ab, _ = synth.band_ipm(N, k, SEED + k)
    l_gpu, info = gpu_factor(ab, k)
    assert info == 0
    eta = llt_residual_threaded(l_gpu, ab, k)
    assert eta <= ETA_TOL, eta
    b = synth.rhs(N, 1, SEED + k)
    x_gpu = gpu_solve(l_gpu, k, b)
    assert oracle.solve_residual(ab, k, x_gpu, b) <= ETA_TOL
    l_or, info_or = oracle.factor(ab, k, columns=True)
    assert info_or == 0
    x_or = oracle.solve(l_or, k, b)
    kap = oracle.cond1_estimate(ab, l_or, k)
    fwd = float(np.max(np.abs(x_gpu - x_or)) / np.max(np.abs(x_or)))
    assert fwd <= 1e-12 * kap, (fwd, kap)
    col = np.linalg.norm(l_gpu - l_or, axis=0) / np.linalg.norm(l_or, axis=0)
    assert float(col.max()) <= 1e-12 * kap, (float(col.max()), int(col.argmax()), kap)
    print("k=%d eta_F %.2e eta_x ok fwd %.2e kappa %.2e max column error %.2e" %
          (k, eta, fwd, kap, float(col.max())), flush=True)
