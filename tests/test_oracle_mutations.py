"""The oracle's pins catch plausible mistakes.

Each case compiles a copy of the oracle source with one planted mistake (on
the CPU, into a temporary directory) and checks that at least one pin fails on
it while the unmodified source passes them all.
"""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest
import scipy.linalg

import oracle
import synth

SRC = os.path.join(os.path.dirname(oracle.__file__), "band_oracle.c")
D = ctypes.POINTER(ctypes.c_double)
I = ctypes.c_int64

MUTATIONS = {
    "none": [],
    "inner bound l <= j (as printed)": [("for (int64_t l = lo; l < j; ++l)\n                t += ri[l - i + k] * rj[l - j + k];",
                                         "for (int64_t l = lo; l <= j; ++l)\n                t += ri[l - i + k] * rj[l - j + k];")],
    "dropped sum term": [("double d = ri[k] - t;", "double d = ri[k];")],
    "wrong sign": [("ri[j - i + k] = (ri[j - i + k] - t) / rj[k];", "ri[j - i + k] = (ri[j - i + k] + t) / rj[k];")],
    "transposed operand": [("t += ri[l - i + k] * rj[l - j + k];\n            if", "t += ri[l - i + k] * ri[l - j + k];\n            if")],
    "row lower bound off by one": [("int64_t lo = i - k > 0 ? i - k : 0;\n        double *ri = r + i * w;\n        for (int64_t j = lo;",
                                    "int64_t lo = i - k + 1 > 0 ? i - k + 1 : 0;\n        double *ri = r + i * w;\n        for (int64_t j = lo;")],
    "pivot test accepts zero": [("if (!(d > 0.0))\n                    return i + 1;", "if (d < 0.0)\n                    return i + 1;")],
    "back solve skips last band entry": [("int64_t hi = (i + k < n - 1) ? i + k : n - 1;", "int64_t hi = (i + k - 1 < n - 1) ? i + k - 1 : n - 1;")],
}


def build_variant(tmp, name, edits):
    src = open(SRC).read()
    for old, new in edits:
        assert old in src, (name, old)
        src = src.replace(old, new, 1)
    cpath = os.path.join(tmp, "v.c")
    open(cpath, "w").write(src)
    so = os.path.join(tmp, "v_%d.so" % abs(hash(name)))
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-o", so,
                           cpath, "-lm"])
    lib = ctypes.CDLL(so)
    lib.oracle_pbtrf.restype = I
    lib.oracle_pbtrf.argtypes = [I, I, D, I]
    lib.oracle_pbtrs.restype = I
    lib.oracle_pbtrs.argtypes = [I, I, I, D, I, D, I]
    return lib


def pins_pass(lib):
    """A compact run of the pins; False as soon as one fails."""
    def fac(ab, k):
        l = np.array(ab, order="F", copy=True)
        info = lib.oracle_pbtrf(l.shape[1], k, l.ctypes.data_as(D), l.shape[0])
        return l, info

    def sol(l, k, b):
        x = np.array(b, order="F", copy=True)
        lib.oracle_pbtrs(l.shape[1], k, 1, l.ctypes.data_as(D), l.shape[0], x.ctypes.data_as(D), l.shape[1])
        return x

    # integer-exact construction: factor and solve come back exactly
    n, k = 300, 7
    l0 = synth.int_factor(n, k, 3)
    a = synth.band_ldlt(l0, k)
    l, info = fac(a, k)
    if info != 0 or not np.array_equal(l, l0):
        return False
    x0 = synth.int_vector(n, 1)
    if not np.array_equal(sol(l, k, synth.band_symv(a, k, x0)), x0):
        return False
    # LAPACK cross-check on a random SPD band
    ab = synth.band_diagdom(400, 12, 9)
    l, info = fac(ab, 12)
    ref = scipy.linalg.cholesky_banded(ab, lower=True)
    if info != 0 or np.max(np.abs(l - ref)) > 1e-13 * np.max(np.abs(ref)):
        return False
    # exact failing column
    dvec = np.ones(n)
    dvec[40] = 0.0
    if fac(synth.band_ldlt(l0, k, dvec), k)[1] != 41:
        return False
    return True


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_pins_catch_mutation(name):
    with tempfile.TemporaryDirectory() as tmp:
        lib = build_variant(tmp, name, MUTATIONS[name])
        assert pins_pass(lib) == (name == "none")
