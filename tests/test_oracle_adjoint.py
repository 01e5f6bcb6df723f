"""Pins of the oracle's reverse mode of x = A^{-1} b (loss = sum(w .* x)).

The band gradient is checked against what does not depend on its formula:
central finite differences of the loss computed with the oracle's own factor
and solves (h = 1e-6, each stored entry perturbing A(i, j) and A(j, i)
together), and the dense gradient -lambda x^T formed with numpy.linalg.solve
on the embedded dense matrix.  Variants of the C routine with planted mistakes
(compiled on the CPU into a temporary directory) must fail the dense pin.
"""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
import synth
from helpers import dense_band_grad


def loss(ab, k, b, w):
    l, info = oracle.factor(ab, k)
    assert info == 0
    return float(np.sum(w * oracle.solve(l, k, b)))


@pytest.mark.parametrize("n,k,nrhs", [(300, 20, 2), (97, 96, 1), (200, 1, 3)])
def test_gradient_matches_central_differences(n, k, nrhs):
    ab = synth.band_diagdom(n, k, 11 + n)
    b = np.asfortranarray(synth.rhs(n, nrhs, 3).reshape(n, nrhs))
    w = np.asfortranarray(synth.normal(n * nrhs, 5, 0).reshape(n, nrhs, order="F"))
    l, _ = oracle.factor(ab, k)
    x = oracle.solve(l, k, b)
    db, g = oracle.solve_backward(l, k, x, w)
    assert np.allclose(db, oracle.solve(l, k, w), rtol=0, atol=0)
    rng = np.random.default_rng(7)
    h = 1e-6
    for _ in range(50):
        j = int(rng.integers(0, n))
        d = int(rng.integers(0, min(k, n - 1 - j) + 1))
        ap, am = ab.copy(order="F"), ab.copy(order="F")
        ap[d, j] += h
        am[d, j] -= h
        fd = (loss(ap, k, b, w) - loss(am, k, b, w)) / (2 * h)
        assert abs(fd - g[d, j]) <= 1e-6 * (1 + abs(g[d, j])), (d, j, fd, g[d, j])
    # db: central differences in b
    for _ in range(10):
        i, r = int(rng.integers(0, n)), int(rng.integers(0, nrhs))
        bp, bm = b.copy(order="F"), b.copy(order="F")
        bp[i, r] += h
        bm[i, r] -= h
        fd = (loss(ab, k, bp, w) - loss(ab, k, bm, w)) / (2 * h)
        assert abs(fd - db[i, r]) <= 1e-6 * (1 + abs(db[i, r]))


@pytest.mark.parametrize("n,k,nrhs", [(500, 30, 1), (500, 7, 4), (64, 63, 2)])
def test_gradient_matches_dense(n, k, nrhs):
    ab = synth.band_diagdom(n, k, 40 + k)
    b = np.asfortranarray(synth.rhs(n, nrhs, 8).reshape(n, nrhs))
    w = np.asfortranarray(synth.normal(n * nrhs, 9, 0).reshape(n, nrhs, order="F"))
    l, _ = oracle.factor(ab, k)
    x = oracle.solve(l, k, b)
    _, g = oracle.solve_backward(l, k, x, w)
    ref = dense_band_grad(ab, k, b, w)
    assert np.linalg.norm(g - ref) <= 1e-10 * np.linalg.norm(ref)


GRAD_MUTATIONS = {
    "wrong sign": [("g -= lam[i + r * ldl] * x[j + r * ldx];", "g += lam[i + r * ldl] * x[j + r * ldx];")],
    "symmetric term dropped": [("if (d > 0) g -= lam[j + r * ldl] * x[i + r * ldx];", "(void)0;")],
    "operands transposed": [("g -= lam[i + r * ldl] * x[j + r * ldx];", "g -= lam[j + r * ldl] * x[i + r * ldx];")],
    "diagonal counted twice": [("if (d > 0) g -= lam[j + r * ldl] * x[i + r * ldx];",
                                "g -= lam[j + r * ldl] * x[i + r * ldx];")],
    "last right-hand side skipped": [("for (int64_t r = 0; r < nrhs; ++r) {\n                g -=",
                                      "for (int64_t r = 0; r < nrhs - 1; ++r) {\n                g -=")],
}


@pytest.mark.parametrize("name", sorted(GRAD_MUTATIONS))
def test_dense_pin_catches_planted_mistakes(name):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "band_oracle.c")).read()
    for old, new in GRAD_MUTATIONS[name]:
        assert old in src, old
        src = src.replace(old, new, 1)
    n, k, nrhs = 120, 9, 2
    ab = synth.band_diagdom(n, k, 77)
    b = np.asfortranarray(synth.rhs(n, nrhs, 1).reshape(n, nrhs))
    w = np.asfortranarray(synth.normal(n * nrhs, 2, 0).reshape(n, nrhs, order="F"))
    l, _ = oracle.factor(ab, k)
    x = oracle.solve(l, k, b)
    lam = oracle.solve(l, k, w)
    ref = dense_band_grad(ab, k, b, w)
    with tempfile.TemporaryDirectory() as tmp:
        c = os.path.join(tmp, "v.c")
        so = os.path.join(tmp, "v.so")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-o", so,
                               c, "-lm"])
        lib = ctypes.CDLL(so)
        D, I = ctypes.POINTER(ctypes.c_double), ctypes.c_int64
        lib.oracle_band_outer_grad.argtypes = [I, I, I, D, I, D, I, D, I]
        g = np.zeros((k + 1, n), order="F")
        lam_f, x_f = np.asfortranarray(lam), np.asfortranarray(x)
        lib.oracle_band_outer_grad(n, k, nrhs, lam_f.ctypes.data_as(D), n, x_f.ctypes.data_as(D), n,
                                   g.ctypes.data_as(D), k + 1)
    assert np.linalg.norm(g - ref) > 1e-6 * np.linalg.norm(ref), name
