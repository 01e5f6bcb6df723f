"""Shared helpers for the GPU parity tests: host <-> device band transfers and
the tolerance rules, all in terms of the oracle's residual functions."""
import numpy as np

U = 2.0 ** -53

# Parity bar: relative backward error of the factor and of the solve.
ETA_TOL = 1e-12


def to_dev(a):
    """numpy Fortran-order array -> flat float64 GPU tensor with the same bytes."""
    import torch
    flat = np.asarray(a, dtype=np.float64).ravel(order="F")
    return torch.from_numpy(flat.copy()).to("cuda")


def from_dev(t, shape):
    return np.asarray(t.cpu().numpy()).reshape(shape, order="F")


def gpu_factor(ab, k):
    """Factor a numpy band array on the GPU; returns (L band as numpy, info)."""
    import paper_2305_04635_amd as bc
    ldab, n = ab.shape
    d = to_dev(ab)
    info = bc.factor(d, n, k, ldab)
    return from_dev(d, ab.shape), info


def gpu_solve(l_band, k, b):
    import paper_2305_04635_amd as bc
    ldab, n = l_band.shape
    b2 = np.asfortranarray(b.reshape(n, -1))
    dl = to_dev(l_band)
    db = to_dev(b2)
    bc.solve(dl, n, k, db, nrhs=b2.shape[1], ldab=ldab, ldb=max(n, 1))
    return from_dev(db, b2.shape).reshape(b.shape)


def rel_fro(x, ref):
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / den) if den > 0 else float(np.linalg.norm(x))


def col_rel_err(x, ref):
    """Largest column error of a band array, relative to that column's norm in ``ref``
    (an all-zero reference column counts its absolute error)."""
    num = np.linalg.norm(x - ref, axis=0)
    den = np.linalg.norm(ref, axis=0)
    return float(np.max(np.where(den > 0, num / np.where(den > 0, den, 1.0), num))) if x.size else 0.0


def dense_of(ab, k):
    """The symmetric dense matrix whose lower band is ab."""
    n = ab.shape[1]
    a = np.zeros((n, n))
    for j in range(n):
        for d in range(min(k, n - 1 - j) + 1):
            a[j + d, j] = ab[d, j]
            a[j, j + d] = ab[d, j]
    return a


def dense_band_grad(ab, k, b, w):
    """Gradient of sum(w .* A^{-1} b) with respect to the stored band, from dense
    numpy solves: -lambda x^T folded onto the band (i > j gets G_ij + G_ji)."""
    a = dense_of(ab, k)
    x = np.linalg.solve(a, b)
    lam = np.linalg.solve(a, w)
    g = -(lam @ x.T)
    n = ab.shape[1]
    out = np.zeros((k + 1, n), order="F")
    for j in range(n):
        for d in range(min(k, n - 1 - j) + 1):
            out[d, j] = g[j + d, j] + (g[j, j + d] if d else 0.0)
    return out
