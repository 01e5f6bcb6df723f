"""Pins of the oracle's mixed-precision path: the FP32 band factor and the
FP64 iterative refinement built on it.

- FP32 factor: integer-exact matrices give L0 bit for bit (every intermediate
  is a small integer, exact in float); the backward error of a general SPD
  band sits at the FP32 level, (k+1) u32; non-SPD pivots report the exact
  column; planted mistakes (compiled variants) break one of these.
- Refinement: the tridiagonal closed form x_i = i (n+1-i) / 2; the stopping
  test holds at exit; the forward error against the FP64 oracle is at the
  FP64 level times the condition number; matrices beyond FP32's reach
  (cond > 1/u32) fall back to FP64.
"""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
import synth

U32 = 2.0 ** -24
U64 = 2.0 ** -53


def f32_backward_error(l32, ab, k):
    return oracle.llt_residual(l32.astype(np.float64), ab, k)


@pytest.mark.parametrize("n,k,p2", [(300, 20, 0), (200, 50, 2), (64, 63, 1), (1, 0, 0)])
def test_spbtrf_integer_exact(n, k, p2):
    l0 = synth.int_factor(n, k, 3 + k, pow2_max=p2)
    a = synth.band_ldlt(l0, k)
    a32 = np.asfortranarray(a.astype(np.float32))
    assert oracle.spbtrf(a32, k) == 0
    assert np.array_equal(a32.astype(np.float64), l0)


@pytest.mark.parametrize("n,k", [(500, 30), (400, 120), (90, 89)])
def test_spbtrf_backward_error_fp32_level(n, k):
    ab = synth.band_diagdom(n, k, n + k)
    a32 = np.asfortranarray(ab.astype(np.float32))
    assert oracle.spbtrf(a32, k) == 0
    eta = f32_backward_error(a32, ab, k)
    assert eta <= 4 * (k + 1) * U32, eta
    assert eta > 1e-12          # it really is single precision


@pytest.mark.parametrize("m", [0, 7, 150, 299])
def test_spbtrf_nonspd_info(m):
    n, k = 300, 25
    l0 = synth.int_factor(n, k, 11)
    dvec = np.ones(n)
    dvec[m] = -1.0
    a = synth.band_ldlt(l0, k, dvec)
    a32 = np.asfortranarray(a.astype(np.float32))
    assert oracle.spbtrf(a32, k) == m + 1


def test_mixed_tridiagonal_closed_form():
    n = 1000
    ab = np.zeros((2, n), order="F")
    ab[0, :] = 2.0
    ab[1, :-1] = -1.0
    b = np.ones((n, 1), order="F")
    x, it, fb = oracle.mixed_solve(ab, 1, b)
    i = np.arange(1, n + 1)
    exact = i * (n + 1 - i) / 2.0
    kappa = 4.0 * (n + 1) ** 2 / np.pi ** 2       # 2-norm condition of tridiag(-1, 2, -1), to leading order
    assert fb is None
    assert np.max(np.abs(x[:, 0] - exact)) / np.max(exact) <= 10 * kappa * U64


@pytest.mark.parametrize("d,expect_fallback", [(1, False), (2, False), (3, False), (5, True)])
def test_mixed_refinement(d, expect_fallback):
    n, k, nrhs = 3000, 40, 3
    ab, _ = synth.band_ipm(n, k, 70 + d, diag_exp_lo=-float(d), shift_rel=10.0 ** (-2 * d))
    b = synth.rhs(n, nrhs, 9)
    x, it, fb = oracle.mixed_solve(ab, k, b)
    assert (fb is not None) == expect_fallback, (it, fb)
    l64, _ = oracle.factor(ab, k)
    x64 = oracle.solve(l64, k, b)
    kap = oracle.cond1_estimate(ab, l64, k)
    for c in range(nrhs):
        r = b[:, c] - oracle.symv(ab, k, x[:, c])
        assert np.max(np.abs(r)) <= np.sqrt(n) * U64 * oracle.norm_inf(ab, k) * np.max(np.abs(x[:, c])) * 1.0001
        fwd = np.max(np.abs(x[:, c] - x64[:, c])) / np.max(np.abs(x64[:, c]))
        assert fwd <= 1e-12 * kap, (fwd, kap)
    if not expect_fallback:
        assert 1 <= it <= 10


SP_MUTATIONS = {
    "inner bound l <= j": [("for (int64_t l = lo; l < j; ++l)\n                t += ab[(i - l) + l * ldab] * ab[(j - l) + l * ldab];",
                            "for (int64_t l = lo; l <= j; ++l)\n                t += ab[(i - l) + l * ldab] * ab[(j - l) + l * ldab];")],
    "wrong sign": [("ab[(i - j) + j * ldab] = (ab[(i - j) + j * ldab] - t) / ab[j * ldab];",
                    "ab[(i - j) + j * ldab] = (ab[(i - j) + j * ldab] + t) / ab[j * ldab];")],
    "transposed operand": [("t += ab[(i - l) + l * ldab] * ab[(j - l) + l * ldab];",
                            "t += ab[(i - l) + l * ldab] * ab[(i - l) + l * ldab];")],
    "pivot accepts zero": [("if (!(d > 0.0f)) return i + 1;", "if (d < 0.0f) return i + 1;")],
}


@pytest.mark.parametrize("name", sorted(SP_MUTATIONS))
def test_spbtrf_pins_catch_planted_mistakes(name):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "band_oracle.c")).read()
    for old, new in SP_MUTATIONS[name]:
        assert old in src, old
        src = src.replace(old, new, 1)
    with tempfile.TemporaryDirectory() as tmp:
        c, so = os.path.join(tmp, "v.c"), os.path.join(tmp, "v.so")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-o", so,
                               c, "-lm"])
        lib = ctypes.CDLL(so)
        F = ctypes.POINTER(ctypes.c_float)
        lib.oracle_spbtrf.restype = ctypes.c_int64
        lib.oracle_spbtrf.argtypes = [ctypes.c_int64, ctypes.c_int64, F, ctypes.c_int64]

        def fac(a, k):
            a32 = np.asfortranarray(a.astype(np.float32))
            return a32, lib.oracle_spbtrf(a32.shape[1], k, a32.ctypes.data_as(F), a32.shape[0])

        ok = True
        l0 = synth.int_factor(120, 9, 4)
        a32, info = fac(synth.band_ldlt(l0, 9), 9)
        ok &= info == 0 and np.array_equal(a32.astype(np.float64), l0)
        ab = synth.band_diagdom(150, 12, 5)
        a32, info = fac(ab, 12)
        ok &= info == 0 and f32_backward_error(a32, ab, 12) <= 4 * 13 * U32
        dvec = np.ones(120)
        dvec[40] = 0.0
        _, info = fac(synth.band_ldlt(l0, 9, dvec), 9)
        ok &= info == 41
    assert not ok, name
