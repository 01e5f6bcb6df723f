"""Seeded synthetic inputs for the band Cholesky factor + solve.

Shared by the tests, the oracle checks and the benchmark.  The arithmetic
lives in ``synth.c`` (SplitMix64 counter draws, Box-Muller normals, and the
matrix products that build each test matrix from a chosen factor); this module
only marshals numpy arrays.  It holds no step of the factorization or of the
solves.

Band arrays are numpy arrays of shape ``(ldab, n)`` in Fortran order, so that
``ab[d, j] = A(j + d, j)`` -- the LAPACK lower band layout, byte for byte.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsynth.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.c_int64
_U64 = ctypes.c_uint64


def build():
    """Compile ``synth.c`` into ``libsynth.so`` (always recompiles)."""
    src = os.path.join(_HERE, "synth.c")
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
    os.replace(tmp, _SO)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        I, U64, D, F = _I64, _U64, _D, ctypes.c_double
        P = ctypes.POINTER(ctypes.c_int64)
        sig = {
            "synth_uniform": (None, [I, U64, U64, F, F, D]),
            "synth_normal": (None, [I, U64, U64, D]),
            "synth_rhs": (None, [I, I, U64, D, I]),
            "synth_band_diagdom": (None, [I, I, U64, D, I]),
            "synth_band_ipm": (F, [I, I, U64, F, F, D, I]),
            "synth_int_factor": (None, [I, I, U64, ctypes.c_int, D, I]),
            "synth_band_ldlt": (None, [I, I, D, I, D, D, I]),
            "synth_int_vector": (None, [I, U64, D]),
            "synth_band_symv": (None, [I, I, I, D, I, D, I, D, I]),
            "synth_batch_shapes": (None, [I, U64, I, I, I, I, P, P]),
            "synth_int_factor_sparse": (None, [I, I, U64, F, D, I]),
            "synth_band_llt_sparse": (None, [I, I, D, I, D, I]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _p(a):
    assert a.dtype == np.float64 and (a.flags.f_contiguous or a.flags.c_contiguous)
    return a.ctypes.data_as(_D)


def empty_band(n, k, ldab=None, fill=0.0):
    """A band array of shape (ldab, n), Fortran order, filled with ``fill``."""
    ldab = k + 1 if ldab is None else ldab
    return np.full((ldab, n), fill, dtype=np.float64, order="F")


def band_diagdom(n, k, seed, ldab=None, fill=0.0):
    """Diagonally dominant SPD band: off-diagonals U[-1,1), diagonal 1 + |row|."""
    ab = empty_band(n, k, ldab, fill)
    _load().synth_band_diagdom(_I64(n), _I64(k), _U64(seed), _p(ab), _I64(ab.shape[0]))
    return ab


def band_ipm(n, k, seed, diag_exp_lo=-4.0, shift_rel=1e-8, ldab=None, fill=0.0):
    """A = L0 L0^T + shift_rel*||A||_inf*I, L0 diagonal 10^U[lo,0], off-diag N(0,1)/sqrt(k).

    Returns (ab, norm_inf_before_shift)."""
    ab = empty_band(n, k, ldab, fill)
    nrm = _load().synth_band_ipm(_I64(n), _I64(k), _U64(seed), ctypes.c_double(diag_exp_lo),
                                 ctypes.c_double(shift_rel), _p(ab), _I64(ab.shape[0]))
    return ab, nrm


def rhs(n, nrhs, seed):
    """n x nrhs right-hand sides, i.i.d. N(0,1), Fortran order."""
    b = np.zeros((max(n, 1), nrhs), dtype=np.float64, order="F")[:n]
    b = np.asfortranarray(b)
    if n and nrhs:
        _load().synth_rhs(_I64(n), _I64(nrhs), _U64(seed), _p(b), _I64(n))
    return b


def normal(count, seed, stream=7):
    out = np.empty(count, dtype=np.float64)
    if count:
        _load().synth_normal(_I64(count), _U64(seed), _U64(stream), _p(out))
    return out


def uniform(count, seed, stream, lo=0.0, hi=1.0):
    out = np.empty(count, dtype=np.float64)
    if count:
        _load().synth_uniform(_I64(count), _U64(seed), _U64(stream), ctypes.c_double(lo),
                              ctypes.c_double(hi), _p(out))
    return out


def int_factor(n, k, seed, pow2_max=0):
    """Integer/dyadic L0: off-diagonals in {-1,0,1}, diagonal 2^m, m in [0, pow2_max]."""
    l0 = empty_band(n, k)
    _load().synth_int_factor(_I64(n), _I64(k), _U64(seed), ctypes.c_int(pow2_max), _p(l0), _I64(k + 1))
    return l0


def band_ldlt(l0, k, dvec=None, ldab=None, fill=0.0):
    """A = L0 diag(dvec) L0^T on the band (dvec None = identity)."""
    n = l0.shape[1]
    ab = empty_band(n, k, ldab, fill)
    dkeep = None if dvec is None else np.ascontiguousarray(dvec, dtype=np.float64)
    dp = None if dkeep is None else _p(dkeep)
    _load().synth_band_ldlt(_I64(n), _I64(k), _p(l0), _I64(l0.shape[0]), dp, _p(ab), _I64(ab.shape[0]))
    return ab


def int_factor_sparse(n, k, seed, density):
    """Sparse integer L0: unit diagonal, each off-diagonal +-1 with probability ``density``, else 0."""
    l0 = empty_band(n, k)
    _load().synth_int_factor_sparse(_I64(n), _I64(k), _U64(seed), ctypes.c_double(density), _p(l0), _I64(k + 1))
    return l0


def band_llt_sparse(l0, k, ldab=None, fill=0.0):
    """A = L0 L0^T on the band, summed over each column's nonzeros (O(n m^2))."""
    n = l0.shape[1]
    ab = empty_band(n, k, ldab, fill)
    _load().synth_band_llt_sparse(_I64(n), _I64(k), _p(l0), _I64(l0.shape[0]), _p(ab), _I64(ab.shape[0]))
    return ab


def int_vector(count, seed):
    out = np.empty(count, dtype=np.float64)
    if count:
        _load().synth_int_vector(_I64(count), _U64(seed), _p(out))
    return out


def band_symv(ab, k, x):
    """b = A x for the symmetric band A (lower storage); x is n x nrhs (or n)."""
    n = ab.shape[1]
    x2 = np.asfortranarray(x.reshape(n, -1), dtype=np.float64)
    b = np.zeros_like(x2, order="F")
    if n:
        _load().synth_band_symv(_I64(n), _I64(k), _I64(x2.shape[1]), _p(ab), _I64(ab.shape[0]),
                                _p(x2), _I64(n), _p(b), _I64(n))
    return b.reshape(x.shape)


def batch_shapes(batch, seed, n_lo, n_hi, k_lo, k_hi):
    nv = np.empty(batch, dtype=np.int64)
    kv = np.empty(batch, dtype=np.int64)
    P = ctypes.POINTER(ctypes.c_int64)
    _load().synth_batch_shapes(_I64(batch), _U64(seed), _I64(n_lo), _I64(n_hi), _I64(k_lo), _I64(k_hi),
                               nv.ctypes.data_as(P), kv.ctypes.data_as(P))
    return nv, kv
