"""Pins of the oracle's reverse mode of the factorization (oracle_pbtrf_backward):
given L = chol(A) and an upstream gradient Lbar, the gradient Abar with respect
to the stored band entries of A.

Checked against what does not depend on the reverse sweep:

* central finite differences of loss(A) = sum(Lbar .* chol(A)) over the band,
  with chol the oracle's forward factor (h = 1e-6, each stored entry moved);
* the dense closed form: for a perturbation dA (symmetric), dL = L Phi(L^{-1} dA
  L^{-T}) with Phi the lower triangle and half the diagonal, so
  <Lbar, dL> = <S, dA> with S = L^{-T} Phi(L^T Lbar) L^{-1}; a stored entry
  A(i, j), i > j, moves A(i, j) and A(j, i), hence Abar(i, j) = S(i,j) + S(j,i)
  and Abar(i, i) = S(i, i) (numpy dense products and inverses);
* log det: Lbar = diag(1 / L_ii) makes the loss sum log L_ii = log det(A) / 2,
  whose gradient is A^{-1} / 2, so Abar(i, j) = (A^{-1})(i, j) for i > j and
  (A^{-1})(i, i) / 2 on the diagonal (A^{-1} from numpy.linalg.inv);
* k = 0: L_ii = sqrt(A_ii), Abar_ii = Lbar_ii / (2 sqrt(A_ii)).

Variants of the C routine with planted mistakes must fail one of them.
"""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
import synth
from helpers import dense_of


def band_to_dense_lower(lb, k):
    n = lb.shape[1]
    m = np.zeros((n, n))
    for j in range(n):
        for d in range(min(k, n - 1 - j) + 1):
            m[j + d, j] = lb[d, j]
    return m


def dense_to_band(m, k):
    n = m.shape[0]
    out = np.zeros((k + 1, n), order="F")
    for j in range(n):
        for d in range(min(k, n - 1 - j) + 1):
            out[d, j] = m[j + d, j]
    return out


def dense_adjoint(l_band, k, lbar_band):
    """Abar on the band from the closed form S = L^{-T} Phi(L^T Lbar) L^{-1}."""
    n = l_band.shape[1]
    L = band_to_dense_lower(l_band, k)
    Lb = band_to_dense_lower(lbar_band, k)
    P = L.T @ Lb
    Phi = np.tril(P) - 0.5 * np.diag(np.diag(P))
    Li = np.linalg.inv(L)
    S = Li.T @ Phi @ Li
    G = np.tril(S + S.T) - np.diag(np.diag(S))
    return dense_to_band(G, k)


def random_lbar(n, k, seed):
    lb = np.asfortranarray(synth.normal((k + 1) * n, seed, 3).reshape(k + 1, n, order="F"))
    for j in range(max(n - k, 0), n):
        lb[n - j:, j] = 0.0
    return lb


@pytest.mark.parametrize("n,k", [(120, 10), (64, 63), (200, 1), (150, 33)])
def test_matches_central_differences(n, k):
    ab = synth.band_diagdom(n, k, 3 * n + k)
    l, info = oracle.factor(ab, k)
    assert info == 0
    lbar = random_lbar(n, k, n + k)
    g = oracle.pbtrf_backward(l, k, lbar)

    def loss(a):
        ll, inf = oracle.factor(a, k)
        assert inf == 0
        return float(np.sum(lbar * ll))

    rng = np.random.default_rng(11)
    h = 1e-6
    for _ in range(40):
        j = int(rng.integers(0, n))
        d = int(rng.integers(0, min(k, n - 1 - j) + 1))
        ap, am = ab.copy(order="F"), ab.copy(order="F")
        ap[d, j] += h
        am[d, j] -= h
        fd = (loss(ap) - loss(am)) / (2 * h)
        assert abs(fd - g[d, j]) <= 1e-6 * (1 + abs(g[d, j])), (d, j, fd, g[d, j])


@pytest.mark.parametrize("n,k", [(300, 25), (200, 199), (257, 64), (500, 40)])
def test_matches_dense_closed_form(n, k):
    ab = synth.band_diagdom(n, k, 7 * n + k)
    l, _ = oracle.factor(ab, k)
    lbar = random_lbar(n, k, 5 * n + k)
    g = oracle.pbtrf_backward(l, k, lbar)
    ref = dense_adjoint(l, k, lbar)
    assert np.linalg.norm(g - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("n,k", [(300, 20), (128, 127)])
def test_log_det_gives_inverse(n, k):
    ab = synth.band_diagdom(n, k, 13 * n + k)
    l, _ = oracle.factor(ab, k)
    lbar = np.zeros((k + 1, n), order="F")
    lbar[0] = 1.0 / l[0]
    g = oracle.pbtrf_backward(l, k, lbar)
    ainv = np.linalg.inv(dense_of(ab, k))
    ref = dense_to_band(np.tril(ainv) - 0.5 * np.diag(np.diag(ainv)), k)
    assert np.linalg.norm(g - ref) <= 1e-12 * np.linalg.norm(ref)


def test_diagonal_band():
    n = 50
    ab = synth.band_diagdom(n, 0, 1)
    l, _ = oracle.factor(ab, 0)
    lbar = random_lbar(n, 0, 2)
    g = oracle.pbtrf_backward(l, 0, lbar)
    assert np.allclose(g[0], lbar[0] / (2 * np.sqrt(ab[0])), rtol=1e-15, atol=0)


def test_in_place_and_padding():
    """Abar may overwrite Lbar; rows past k of a padded Lbar are ignored."""
    n, k = 90, 12
    ab = synth.band_diagdom(n, k, 4)
    l, _ = oracle.factor(ab, k)
    lbar = random_lbar(n, k, 9)
    ref = oracle.pbtrf_backward(l, k, lbar)
    big = np.full((k + 4, n), 7.0, order="F")
    big[: k + 1] = lbar
    assert np.array_equal(oracle.pbtrf_backward(l, k, big), ref)


SRC = os.path.join(os.path.dirname(oracle.__file__), "band_oracle.c")
D = ctypes.POINTER(ctypes.c_double)
I = ctypes.c_int64

MUTATIONS = {
    "none": [],
    "diagonal without the factor 2": [("ai[k] = gi[k] / (2.0 * ri[k]);", "ai[k] = gi[k] / ri[k];")],
    "missing pivot adjoint": [("gj[k] -= gi[j - i + k] * lij / ljj;", "(void)lij;")],
    "one side of the product only": [("gj[l - j + k] += tbar * ri[l - i + k];", "(void)gj;")],
    "transposed operand": [("gi[l - i + k] += tbar * rj[l - j + k];", "gi[l - i + k] += tbar * ri[l - j + k];")],
    "forward order": [("for (int64_t j = i; j >= lo; --j) {", "for (int64_t j = lo; j <= i; ++j) {")],
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
    lib.oracle_pbtrf_backward.restype = None
    lib.oracle_pbtrf_backward.argtypes = [I, I, D, I, D, I, D, I]
    return lib


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_pins_catch_mutation(name):
    n, k = 160, 21
    ab = synth.band_diagdom(n, k, 77)
    l, _ = oracle.factor(ab, k)
    lbar = random_lbar(n, k, 78)
    ref = dense_adjoint(l, k, lbar)
    with tempfile.TemporaryDirectory() as tmp:
        lib = build_variant(tmp, name, MUTATIONS[name])
        out = np.zeros((k + 1, n), order="F")
        lib.oracle_pbtrf_backward(n, k, l.ctypes.data_as(D), k + 1, lbar.ctypes.data_as(D), k + 1,
                                  out.ctypes.data_as(D), k + 1)
    ok = np.linalg.norm(out - ref) <= 1e-12 * np.linalg.norm(ref)
    assert ok == (name == "none")
