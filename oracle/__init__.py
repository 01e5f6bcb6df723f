"""Oracle: plain FP64 CPU reference for the band Cholesky factor and solves.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import this package.  It shares no code
with the GPU path and never calls it.

The arithmetic lives in ``band_oracle.c`` (built with ``-ffp-contract=off
-fno-fast-math``): the paper's left-looking band algorithm (Algorithm 2,
Section 3.2) row by row, with the inner sum bound read as ``l <= j-1``; the
forward and back band solves; residual norms.  This module marshals numpy
arrays and adds the Hager/Higham 1-norm condition estimate, which only calls
the solves.

Band arrays are numpy arrays of shape ``(ldab, n)`` in Fortran order:
``ab[d, j] = A(j + d, j)`` (LAPACK lower band layout).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.c_int64


def build():
    """Compile ``band_oracle.c`` into ``liboracle.so`` (always recompiles)."""
    src = os.path.join(_HERE, "band_oracle.c")
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
                           "-shared", "-o", tmp, src, "-lm"])
    os.replace(tmp, _SO)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        I, D = _I64, _D
        sig = {
            "oracle_pbtrf": (ctypes.c_int64, [I, I, D, I]),
            "oracle_pbtrf_columns": (ctypes.c_int64, [I, I, D, I]),
            "oracle_pbtrs": (ctypes.c_int64, [I, I, I, D, I, D, I]),
            "oracle_pbtrf_opcount": (ctypes.c_int64, [I, I]),
            "oracle_band_norm_inf": (ctypes.c_double, [I, I, D, I]),
            "oracle_band_symv": (None, [I, I, D, I, D, D]),
            "oracle_llt_residual_rows": (None, [I, I, D, I, D, I, I, I, D]),
            "oracle_band_outer_grad": (None, [I, I, I, D, I, D, I, D, I]),
            "oracle_spbtrf": (ctypes.c_int64, [I, I, ctypes.POINTER(ctypes.c_float), I]),
            "oracle_pbtrf_backward": (None, [I, I, D, I, D, I, D, I]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.f_contiguous
    return a.ctypes.data_as(_D)


def pbtrf(ab, k, n=None, columns=False):
    """Factor the band array in place (A = L L^T); returns LAPACK-style info.

    ``columns=True`` runs the column-order variant, bitwise equal, threaded."""
    n = ab.shape[1] if n is None else n
    f = _load().oracle_pbtrf_columns if columns else _load().oracle_pbtrf
    return int(f(_I64(n), _I64(k), _p(ab), _I64(ab.shape[0])))


def pbtrs(ab, k, b):
    """Solve A X = B in place with the factor in ``ab``; b is (n,) or (n, nrhs), Fortran order."""
    n = ab.shape[1]
    b2 = b.reshape(n, -1, order="F") if b.ndim == 1 else b
    assert b2.flags.f_contiguous
    info = _load().oracle_pbtrs(_I64(n), _I64(k), _I64(b2.shape[1]), _p(ab), _I64(ab.shape[0]),
                                _p(b2), _I64(max(n, 1)))
    return int(info)


def factor(a_band, k, columns=False):
    """Return (L_band, info) without touching the input."""
    l = np.array(a_band, order="F", copy=True)
    return l, pbtrf(l, k, columns=columns)


def solve(l_band, k, b):
    x = np.array(b, order="F", copy=True, dtype=np.float64)
    info = pbtrs(l_band, k, x)
    assert info == 0, info
    return x


def symv(ab, k, x):
    """y = A x, symmetric band A (lower storage), x of shape (n,)."""
    n = ab.shape[1]
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(n, dtype=np.float64)
    _load().oracle_band_symv(_I64(n), _I64(k), _p(ab), _I64(ab.shape[0]), x.ctypes.data_as(_D),
                             y.ctypes.data_as(_D))
    return y


def norm_inf(ab, k):
    """||A||_inf (= ||A||_1) of the symmetric band matrix."""
    return float(_load().oracle_band_norm_inf(_I64(ab.shape[1]), _I64(k), _p(ab), _I64(ab.shape[0])))


def llt_residual(l_band, a_band, k, rows=None):
    """Backward error ||L L^T - A||_F / ||A||_F over the band.

    ``rows`` = iterable of (lo, hi) row ranges to sample; None = all rows."""
    n = a_band.shape[1]
    rows = [(0, n)] if rows is None else rows
    out = np.zeros(2)
    acc = np.zeros(2)
    for lo, hi in rows:
        _load().oracle_llt_residual_rows(_I64(n), _I64(k), _p(l_band), _I64(l_band.shape[0]), _p(a_band),
                                         _I64(a_band.shape[0]), _I64(lo), _I64(hi),
                                         out.ctypes.data_as(_D))
        acc += out
    return float(np.sqrt(acc[0] / acc[1])) if acc[1] > 0 else float(np.sqrt(acc[0]))


def solve_residual(a_band, k, x, b):
    """max over columns of ||b - A x||_inf / (||A||_inf ||x||_inf)."""
    n = a_band.shape[1]
    x2 = x.reshape(n, -1, order="F")
    b2 = b.reshape(n, -1, order="F")
    an = norm_inf(a_band, k)
    worst = 0.0
    for c in range(x2.shape[1]):
        r = b2[:, c] - symv(a_band, k, x2[:, c])
        den = an * np.max(np.abs(x2[:, c]))
        worst = max(worst, float(np.max(np.abs(r)) / den) if den > 0 else float(np.max(np.abs(r))))
    return worst


def opcount(n, k):
    """Operations executed by the factor's loop nest (sqrt = 1 operation)."""
    return int(_load().oracle_pbtrf_opcount(_I64(n), _I64(k)))


def band_outer_grad(lam, x, k, n):
    """Band gradient of sum(w .* x) from x and lambda = A^{-1} w (see band_oracle.c)."""
    lam = np.asfortranarray(np.asarray(lam, dtype=np.float64).reshape(n, -1))
    x = np.asfortranarray(np.asarray(x, dtype=np.float64).reshape(n, -1))
    g = np.zeros((k + 1, n), order="F")
    _load().oracle_band_outer_grad(n, k, x.shape[1], _p(lam), max(n, 1), _p(x), max(n, 1), _p(g), k + 1)
    return g


def solve_backward(l_band, k, x, w):
    """Reverse mode of x = A^{-1} b for loss = sum(w .* x) (A = L L^T given by its
    factor): returns (db, dA_band) with db = A^{-1} w (A is symmetric) and the
    band gradient of band_outer_grad."""
    n = l_band.shape[1]
    lam = solve(l_band, k, np.asarray(w, dtype=np.float64).reshape(n, -1))
    return lam, band_outer_grad(lam, x, k, n)


def pbtrf_backward(l_band, k, lbar_band):
    """Reverse mode of the factorization (see band_oracle.c): the gradient with
    respect to the stored band of A for an upstream gradient Lbar of the factor."""
    n = l_band.shape[1]
    lb = np.asfortranarray(lbar_band, dtype=np.float64)
    out = np.zeros((k + 1, n), order="F")
    _load().oracle_pbtrf_backward(n, k, _p(np.asfortranarray(l_band)), l_band.shape[0], _p(lb), lb.shape[0],
                                  _p(out), k + 1)
    return out


def spbtrf(ab32, k):
    """FP32 band Cholesky in place on a float32 (ldab, n) Fortran-order array; returns info."""
    assert ab32.dtype == np.float32 and ab32.flags.f_contiguous
    return int(_load().oracle_spbtrf(ab32.shape[1], k, ab32.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                     ab32.shape[0]))


def mixed_solve(ab, k, b, itmax=30, ratio=0.5):
    """Mixed-precision solve of A X = B: FP32 factor of fl32(A), then FP64
    iterative refinement (residual b - A x in FP64, correction solved with the
    FP32 factor widened to FP64), as in Buttari et al. (2007) and LAPACK dsposv.

    Stops when every column satisfies ||r||_inf <= sqrt(n) u64 ||A||_inf ||x||_inf.
    Falls back to the FP64 factor and solve when the FP32 factor fails, after
    itmax corrections, or when a correction is not at most `ratio` times the
    previous one.  Returns (x, iterations, fallback) with fallback one of
    None, "factor", "iterations", "stagnation"."""
    n = ab.shape[1]
    b = np.asfortranarray(np.asarray(b, dtype=np.float64).reshape(n, -1))
    eps = 2.0 ** -53
    anrm = norm_inf(ab, k)
    a32 = np.asfortranarray(ab.astype(np.float32))
    reason = None
    if spbtrf(a32, k) != 0:
        reason = "factor"
    it = 0
    if reason is None:
        l = np.asfortranarray(a32.astype(np.float64))
        x = solve(l, k, b)
        dprev = None
        while True:
            r = b - np.column_stack([symv(ab, k, x[:, c]) for c in range(x.shape[1])])
            rn = np.max(np.abs(r), axis=0)
            xn = np.max(np.abs(x), axis=0)
            if np.all(rn <= np.sqrt(n) * eps * anrm * xn):
                return x, it, None
            if it == itmax:
                reason = "iterations"
                break
            d = solve(l, k, r)
            dn = np.max(np.abs(d), axis=0)
            if dprev is not None and np.any(dn > ratio * dprev):
                reason = "stagnation"
                break
            x = x + d
            dprev = dn
            it += 1
    l64, info = factor(ab, k)
    assert info == 0, info
    return solve(l64, k, b), it, reason


def cond1_estimate(a_band, l_band, k, itmax=5):
    """kappa_1(A) = ||A||_1 * est(||A^{-1}||_1).

    The inverse-norm estimate is Hager's method (Hager 1984, "Condition
    estimates", SIAM J. Sci. Stat. Comput. 5) with Higham's refinements
    (Higham 1988, ACM TOMS 14, Algorithm 4.1 there): a few solves with A,
    which is symmetric, so A^{-T} solves are A^{-1} solves."""
    n = a_band.shape[1]
    if n == 0:
        return 0.0
    x = np.full(n, 1.0 / n)
    est = 0.0
    for it in range(itmax):
        y = solve(l_band, k, x)
        est_new = float(np.sum(np.abs(y)))
        if it > 0 and est_new <= est:
            break
        est = est_new
        z = solve(l_band, k, np.where(y >= 0, 1.0, -1.0))
        j = int(np.argmax(np.abs(z)))
        if np.abs(z[j]) <= z @ x:
            break
        x = np.zeros(n)
        x[j] = 1.0
    # Higham's alternative vector guards against the rare underestimate
    alt = np.array([(-1.0) ** i * (1.0 + i / max(n - 1, 1)) for i in range(n)])
    y = solve(l_band, k, alt)
    est = max(est, 2.0 * float(np.sum(np.abs(y))) / (3.0 * n))
    return norm_inf(a_band, k) * est
