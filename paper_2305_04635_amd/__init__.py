"""MI355X (gfx950) FP64 band Cholesky factor and band solves.

Thin ctypes binding over ``libbandchol.so`` (C-ABI in ``include/bandchol.h``).
Every function takes float64 GPU tensors and passes their device pointers and
the current torch stream; all arithmetic runs in the library's HIP kernels.
There is no fallback: if the library is missing or no GPU is present the calls
raise.

Band storage is LAPACK lower band, column-major: ``A(i, j)`` for
``0 <= i - j <= k`` at flat index ``(i - j) + j * ldab``.  A tensor of shape
``(n, ldab)`` (row ``j`` = band column ``j``) has exactly this memory layout.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbandchol.so")
_lib = None

_I64 = ctypes.c_int64
_VP = ctypes.c_void_p

# name -> (restype, argtypes); the exported C-ABI, as declared in include/bandchol.h
SIGNATURES = {
    "bandchol_factor": (_I64, [_I64, _I64, _VP, _I64]),
    "bandchol_solve": (_I64, [_I64, _I64, _I64, _VP, _I64, _VP, _I64]),
    "bandchol_factor_async": (_I64, [_I64, _I64, _VP, _I64, _VP, _VP]),
    "bandchol_solve_async": (_I64, [_I64, _I64, _I64, _VP, _I64, _VP, _I64, _VP]),
    "bandchol_factor_noalloc": (_I64, [_I64, _I64, _VP, _I64, _VP, _VP]),
    "bandchol_set_stream": (_I64, [_VP]),
    "bandchol_last_error": (ctypes.c_char_p, []),
    "bandchol_finalize": (None, []),
    "bandchol_tile": (_I64, []),
    "bandchol_set_walk_limit": (_I64, [_I64]),
    "bandchol_batch_create": (_I64, [_I64, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "bandchol_batch_factor": (_I64, [_VP, _VP, _VP]),
    "bandchol_batch_solve": (_I64, [_VP, _I64, _VP]),
    "bandchol_batch_destroy": (None, [_VP]),
    "bandchol_solve_backward": (_I64, [_I64, _I64, _I64, _VP, _I64, _VP, _I64, _VP, _I64, _VP, _I64, _VP]),
    "bandchol_factor_backward": (_I64, [_I64, _I64, _VP, _I64, _VP, _I64, _VP, _I64, _VP, _VP]),
    "bandchol_batch_set_adjoint": (_I64, [_VP, _VP, _VP, _VP]),
    "bandchol_batch_backward": (_I64, [_VP, _I64, _VP]),
    "bandchol_factor_f32": (_I64, [_I64, _I64, _VP, _I64, _VP, _VP]),
    "bandchol_mixed_solve": (_I64, [_I64, _I64, _I64, _VP, _I64, _VP, _I64, _VP, _I64, _VP, _VP]),
    "bandchol_schedule": (_I64, [_I64, _I64]),
    "bandchol_tune_set": (_I64, [_I64, _I64, _I64]),
    "bandchol_tune_entries": (_I64, [_I64, _VP, _VP, _VP, _VP]),
    "bandchol_tune_clear": (None, []),
    "bandchol_tune_factor": (_I64, [_I64, _I64, _I64, _VP, _VP]),
    "bandchol_pivot_chain_ns": (_I64, [_I64, _VP]),
    "bandchol_spine_profile": (_I64, [_I64, _I64, _I64, _VP, _I64]),
    "bandchol_batch_tune_set": (_I64, [_I64, _I64, _I64]),
    "bandchol_batch_tune_entries": (_I64, [_I64, _VP, _VP, _VP, _VP]),
    "bandchol_batch_tune_clear": (None, []),
    "bandchol_batch_tune": (_I64, [_I64, _VP, _VP, _I64, _I64, _VP]),
}

EHIP = -1000
EHANG = -1001
ETOOBIG = -1002


class BandCholError(RuntimeError):
    pass


def load(path=LIB_PATH):
    """Load the HIP library (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise BandCholError("libbandchol.so is not built (run paper_2305_04635_amd.build.build())")
        # torch first: its HIP runtime (same soname) then serves the library as
        # well.  Opened the other way round, the process holds two HIP/HSA
        # runtimes and the library's finds no device.
        import torch  # noqa: F401
        lib = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check_tensor(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError("%s must be a float64 GPU tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _raise(rc, what):
    msg = load().bandchol_last_error().decode(errors="replace")
    raise BandCholError("%s failed (%d): %s" % (what, rc, msg))


def tile():
    return int(load().bandchol_tile())


def set_walk_limit(kmax):
    """Largest sub-diagonal tile count factored by the single-workgroup walk; returns the previous value."""
    return int(load().bandchol_set_walk_limit(int(kmax)))


def schedule(n, k):
    """Workgroups the factor of an (n, k) band uses now (1 = the walk)."""
    rc = int(load().bandchol_schedule(int(n), int(k)))
    if rc < 0:
        _raise(rc, "bandchol_schedule")
    return rc


def tune_set(n, k, wgs):
    """Record the workgroup count for the (n, k) bucket (0 removes the entry)."""
    rc = int(load().bandchol_tune_set(int(n), int(k), int(wgs)))
    if rc != 0:
        _raise(rc, "bandchol_tune_set")


def tune_entries():
    """The schedule table: a list of dicts with keys n, k, wgs, ms."""
    lib = load()
    count = int(lib.bandchol_tune_entries(0, None, None, None, None))
    if count == 0:
        return []
    n, k, w = (ctypes.c_int64 * count)(), (ctypes.c_int64 * count)(), (ctypes.c_int64 * count)()
    ms = (ctypes.c_double * count)()
    got = int(lib.bandchol_tune_entries(count, n, k, w, ms))
    return [{"n": n[i], "k": k[i], "wgs": w[i], "ms": ms[i]} for i in range(min(got, count))]


def tune_clear():
    load().bandchol_tune_clear()


def tune_factor(n, k, reps=3):
    """Time the factor's schedules for an (n, k) band on the current device and
    stream, record the fastest for its bucket; returns (wgs, median ms)."""
    lib = load()
    lib.bandchol_set_stream(_stream())
    w, ms = ctypes.c_int64(0), ctypes.c_double(0.0)
    rc = int(lib.bandchol_tune_factor(int(n), int(k), int(reps), ctypes.byref(w), ctypes.byref(ms)))
    if rc != 0:
        _raise(rc, "bandchol_tune_factor")
    return int(w.value), float(ms.value)


def pivot_chain_ns(steps=1 << 20):
    """Measured latency (ns) of one step of the factor's pivot chain on the current device."""
    lib = load()
    lib.bandchol_set_stream(_stream())
    v = ctypes.c_double(0.0)
    rc = int(lib.bandchol_pivot_chain_ns(int(steps), ctypes.byref(v)))
    if rc != 0:
        _raise(rc, "bandchol_pivot_chain_ns")
    return float(v.value)


def batch_tune_set(n, k, wgs):
    """Record the schedule of the (n, k) bucket for batch plans (1 = walk, 0 removes it)."""
    rc = int(load().bandchol_batch_tune_set(int(n), int(k), int(wgs)))
    if rc != 0:
        _raise(rc, "bandchol_batch_tune_set")


def batch_tune_entries():
    """The batch schedule table: a list of dicts with keys n, k, wgs, ms."""
    lib = load()
    count = int(lib.bandchol_batch_tune_entries(0, None, None, None, None))
    if count == 0:
        return []
    n, k, w = (ctypes.c_int64 * count)(), (ctypes.c_int64 * count)(), (ctypes.c_int64 * count)()
    ms = (ctypes.c_double * count)()
    got = int(lib.bandchol_batch_tune_entries(count, n, k, w, ms))
    return [{"n": n[i], "k": k[i], "wgs": w[i], "ms": ms[i]} for i in range(min(got, count))]


def batch_tune_clear():
    load().bandchol_batch_tune_clear()


def batch_tune(ns, ks, reps=3, max_buckets=4):
    """Measure the batched factor of systems of these shapes and settle the schedule of
    its largest buckets in the batch table; returns the final median ms."""
    lib = load()
    lib.bandchol_set_stream(_stream())
    b = len(ns)
    I64 = ctypes.c_int64 * max(b, 1)
    ms = ctypes.c_double(0.0)
    rc = int(lib.bandchol_batch_tune(b, I64(*ns), I64(*ks), int(reps), int(max_buckets), ctypes.byref(ms)))
    if rc != 0:
        _raise(rc, "bandchol_batch_tune")
    return float(ms.value)


SPINE_PROFILE_KEYS = ("sweep", "w0_wait", "bc_w0", "bc_wait", "w1_work", "w1_wait", "w2_work", "w2_wait",
                      "w3_work", "w3_wait")


def spine_profile(n, k, reps=3):
    """Cycles per 32-column step of the diagonal chain's phases (see bandchol_spine_profile)."""
    lib = load()
    lib.bandchol_set_stream(_stream())
    out = (ctypes.c_double * 13)()
    rc = int(lib.bandchol_spine_profile(int(n), int(k), int(reps), out, 13))
    if rc != 0:
        _raise(rc, "bandchol_spine_profile")
    d = {key: out[i] for i, key in enumerate(SPINE_PROFILE_KEYS)}
    d.update(steps=int(out[10]), factor_ms=out[11], workgroups=int(out[12]))
    return d


def save_tuning(path):
    """Write both schedule tables (single matrices and batches) as JSON."""
    import json
    with open(path, "w") as f:
        json.dump({"single": tune_entries(), "batch": batch_tune_entries()}, f, indent=1)


def load_tuning(path):
    """Add the entries of JSON schedule tables written by save_tuning (a plain list is
    read as the single-matrix table)."""
    import json
    with open(path) as f:
        d = json.load(f)
    single, batch = (d, []) if isinstance(d, list) else (d.get("single", []), d.get("batch", []))
    for e in single:
        tune_set(e["n"], e["k"], e["wgs"])
    for e in batch:
        batch_tune_set(e["n"], e["k"], e["wgs"])


def factor(ab, n, k, ldab=None):
    """Factor the band in ``ab`` in place (A = L L^T); returns info (0 = success)."""
    ldab = k + 1 if ldab is None else ldab
    _check_tensor(ab, "ab")
    if ab.numel() < ldab * n:
        raise ValueError("ab holds fewer than ldab*n elements")
    lib = load()
    lib.bandchol_set_stream(_stream())
    rc = lib.bandchol_factor(n, k, ab.data_ptr(), ldab)
    if rc < 0:
        _raise(rc, "bandchol_factor")
    return int(rc)


def factor_async(ab, n, k, d_info, ldab=None):
    """Stream-ordered factor; writes info to the int64 GPU tensor d_info."""
    import torch
    ldab = k + 1 if ldab is None else ldab
    _check_tensor(ab, "ab")
    if d_info.dtype != torch.int64 or not d_info.is_cuda:
        raise TypeError("d_info must be an int64 GPU tensor")
    rc = load().bandchol_factor_async(n, k, ab.data_ptr(), ldab, d_info.data_ptr(), _stream())
    if rc != 0:
        _raise(rc, "bandchol_factor_async")


def factor_noalloc(ab, n, k, d_info, ldab=None):
    """As ``factor_async``, through the entry point that allocates no device memory."""
    import torch
    ldab = k + 1 if ldab is None else ldab
    _check_tensor(ab, "ab")
    if d_info.dtype != torch.int64 or not d_info.is_cuda:
        raise TypeError("d_info must be an int64 GPU tensor")
    rc = load().bandchol_factor_noalloc(n, k, ab.data_ptr(), ldab, d_info.data_ptr(), _stream())
    if rc != 0:
        _raise(rc, "bandchol_factor_noalloc")


def solve(ab, n, k, b, nrhs=None, ldab=None, ldb=None):
    """Solve A X = B in place in ``b`` (n x nrhs column-major) with the factor in ``ab``."""
    ldab = k + 1 if ldab is None else ldab
    _check_tensor(ab, "ab")
    _check_tensor(b, "b")
    nrhs = (b.numel() // max(n, 1)) if nrhs is None else nrhs
    ldb = max(n, 1) if ldb is None else ldb
    lib = load()
    lib.bandchol_set_stream(_stream())
    rc = lib.bandchol_solve(n, k, nrhs, ab.data_ptr(), ldab, b.data_ptr(), ldb)
    if rc != 0:
        _raise(rc, "bandchol_solve")


def solve_async(ab, n, k, b, nrhs=None, ldab=None, ldb=None):
    ldab = k + 1 if ldab is None else ldab
    _check_tensor(ab, "ab")
    _check_tensor(b, "b")
    nrhs = (b.numel() // max(n, 1)) if nrhs is None else nrhs
    ldb = max(n, 1) if ldb is None else ldb
    rc = load().bandchol_solve_async(n, k, nrhs, ab.data_ptr(), ldab, b.data_ptr(), ldb, _stream())
    if rc != 0:
        _raise(rc, "bandchol_solve_async")


FALLBACK_REASONS = {0: None, 1: "factor", 2: "iterations", 3: "stagnation"}


def factor_f32(ab32, n, k, d_info, ldab=None):
    """Stream-ordered FP32 factor of a float32 GPU band tensor; info to the int64 tensor d_info."""
    import torch
    ldab = k + 1 if ldab is None else ldab
    if not isinstance(ab32, torch.Tensor) or ab32.dtype != torch.float32 or not ab32.is_cuda:
        raise TypeError("ab32 must be a float32 GPU tensor")
    rc = load().bandchol_factor_f32(n, k, ab32.data_ptr(), ldab, d_info.data_ptr(), _stream())
    if rc != 0:
        _raise(rc, "bandchol_factor_f32")


def mixed_solve(ab, n, k, b, x, nrhs=None, ldab=None):
    """Mixed-precision solve (FP32 factor + FP64 refinement): x <- A^{-1} b.
    Returns (iterations, fallback reason or None)."""
    ldab = k + 1 if ldab is None else ldab
    for t, name in ((ab, "ab"), (b, "b"), (x, "x")):
        _check_tensor(t, name)
    nrhs = (b.numel() // max(n, 1)) if nrhs is None else nrhs
    it, fb = ctypes.c_int64(), ctypes.c_int64()
    lib = load()
    lib.bandchol_set_stream(_stream())
    ld = max(n, 1)
    rc = lib.bandchol_mixed_solve(n, k, nrhs, ab.data_ptr(), ldab, b.data_ptr(), ld, x.data_ptr(), ld,
                                  ctypes.byref(it), ctypes.byref(fb))
    if rc < 0:
        _raise(rc, "bandchol_mixed_solve")
    if rc > 0:
        raise BandCholError("matrix is not positive definite (info = %d)" % rc)
    return int(it.value), FALLBACK_REASONS[int(fb.value)]


def solve_backward(ab, n, k, x, g, gab, nrhs=None, ldab=None, ldgab=None):
    """Reverse mode of ``solve`` (stream-ordered): ``g`` (upstream gradient, n x nrhs
    column-major) becomes A^{-1} G; ``gab`` receives the band gradient of A."""
    ldab = k + 1 if ldab is None else ldab
    ldgab = k + 1 if ldgab is None else ldgab
    for t, name in ((ab, "ab"), (x, "x"), (g, "g"), (gab, "gab")):
        _check_tensor(t, name)
    nrhs = (x.numel() // max(n, 1)) if nrhs is None else nrhs
    ld = max(n, 1)
    rc = load().bandchol_solve_backward(n, k, nrhs, ab.data_ptr(), ldab, x.data_ptr(), ld, g.data_ptr(), ld,
                                        gab.data_ptr(), ldgab, _stream())
    if rc != 0:
        _raise(rc, "bandchol_solve_backward")


def factor_backward(l, n, k, lbar, abar, d_status=None, ldl=None, ldlb=None, ldab=None):
    """Reverse mode of ``factor`` (stream-ordered): ``abar`` receives the gradient with
    respect to the stored band of A for the upstream gradient ``lbar`` of the factor ``l``
    (all band tensors; ``abar`` may be ``lbar``).  ``d_status``: optional int64 GPU
    tensor, set to 0 or EHANG."""
    import torch
    ldl = k + 1 if ldl is None else ldl
    ldlb = k + 1 if ldlb is None else ldlb
    ldab = k + 1 if ldab is None else ldab
    for t, name in ((l, "l"), (lbar, "lbar"), (abar, "abar")):
        _check_tensor(t, name)
    if d_status is not None and (d_status.dtype != torch.int64 or not d_status.is_cuda):
        raise TypeError("d_status must be an int64 GPU tensor")
    rc = load().bandchol_factor_backward(n, k, l.data_ptr(), ldl, lbar.data_ptr(), ldlb, abar.data_ptr(), ldab,
                                         None if d_status is None else d_status.data_ptr(), _stream())
    if rc != 0:
        _raise(rc, "bandchol_factor_backward")


class BatchPlan:
    """Batch of independent band systems (``bandchol_batch_*``).

    ``abs``: list of float64 GPU tensors holding the bands (LAPACK lower layout,
    ldab = k+1 unless ``ldabs`` is given); ``bs``: optional list of float64 GPU
    tensors for the right-hand sides (n x nrhs column-major, ldb = n).  The
    tensors must stay alive as long as the plan.  ``factor`` and ``solve``
    only launch kernels on the current stream (they can be captured in a
    ``torch.cuda.CUDAGraph``).
    """

    def __init__(self, ns, ks, abs, bs=None, ldabs=None):
        batch = len(ns)
        if len(ks) != batch or len(abs) != batch or (bs is not None and len(bs) != batch):
            raise ValueError("ns, ks, abs and bs must have the same length")
        for t in abs:
            _check_tensor(t, "ab")
        if bs is not None:
            for t in bs:
                _check_tensor(t, "b")
        ldabs = [k + 1 for k in ks] if ldabs is None else list(ldabs)
        I64 = ctypes.c_int64 * max(batch, 1)
        PTR = ctypes.c_void_p * max(batch, 1)
        self._n = I64(*ns)
        self._k = I64(*ks)
        self._ldab = I64(*ldabs)
        self._ab = PTR(*[t.data_ptr() for t in abs])
        self._b = PTR(*[t.data_ptr() for t in bs]) if bs is not None else None
        self._ldb = I64(*[max(n, 1) for n in ns]) if bs is not None else None
        self._keep = (list(abs), list(bs) if bs is not None else None)
        self.batch = batch
        self._plan = ctypes.c_void_p()
        rc = load().bandchol_batch_create(batch, self._n, self._k, self._ab, self._ldab,
                                          self._b, self._ldb, ctypes.byref(self._plan))
        if rc != 0:
            _raise(rc, "bandchol_batch_create")

    def factor(self, d_info):
        """Factor every system in place; info per system into the int64 GPU tensor ``d_info``."""
        import torch
        if d_info.dtype != torch.int64 or not d_info.is_cuda or d_info.numel() < self.batch:
            raise TypeError("d_info must be an int64 GPU tensor with one entry per system")
        rc = load().bandchol_batch_factor(self._plan, d_info.data_ptr(), _stream())
        if rc != 0:
            _raise(rc, "bandchol_batch_factor")

    def solve(self, nrhs):
        """Overwrite every b with the solution (after ``factor``)."""
        rc = load().bandchol_batch_solve(self._plan, int(nrhs), _stream())
        if rc != 0:
            _raise(rc, "bandchol_batch_solve")

    def set_adjoint(self, gs, gabs, ldgabs=None):
        """Register per-system upstream gradients (overwritten by A^{-1} G) and band gradients."""
        if len(gs) != self.batch or len(gabs) != self.batch:
            raise ValueError("one g and one gab per system")
        for t in list(gs) + list(gabs):
            _check_tensor(t, "g/gab")
        PTR = ctypes.c_void_p * max(self.batch, 1)
        I64 = ctypes.c_int64 * max(self.batch, 1)
        self._g = PTR(*[t.data_ptr() for t in gs])
        self._gab = PTR(*[t.data_ptr() for t in gabs])
        self._ldgab = I64(*([k + 1 for k in self._k[:self.batch]] if ldgabs is None else ldgabs))
        self._keep_adj = (list(gs), list(gabs))
        rc = load().bandchol_batch_set_adjoint(self._plan, self._g, self._gab, self._ldgab)
        if rc != 0:
            _raise(rc, "bandchol_batch_set_adjoint")

    def backward(self, nrhs):
        """Reverse mode for every system (after ``factor``, ``solve`` and ``set_adjoint``)."""
        rc = load().bandchol_batch_backward(self._plan, int(nrhs), _stream())
        if rc != 0:
            _raise(rc, "bandchol_batch_backward")

    def close(self):
        if self._plan:
            load().bandchol_batch_destroy(self._plan)
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------- autograd

def _autograd_functions():
    import torch

    def refactor(ab, k):
        """A fresh factor of the band ``ab`` (the recompute path of the backward passes)."""
        l = ab.detach().contiguous().clone()
        info = factor(l, l.shape[0], k)
        if info != 0:
            raise BandCholError("matrix is not positive definite (info = %d)" % info)
        return l

    class BandSolve(torch.autograd.Function):
        """x = A^{-1} b with A given by its lower band ``ab`` of shape (n, k+1)
        (row j = band column j) and b of shape (n,) or (n, nrhs).  Backward:
        db = A^{-1} dx, dab = band gradient (see bandchol_solve_backward).
        recompute=True keeps no factor between the passes: backward factors
        A again (the band ``ab`` is held anyway), trading one factorization for
        a band-sized buffer per system."""

        @staticmethod
        def forward(ctx, ab, b, k, recompute=False):
            n = ab.shape[0]
            l = refactor(ab, k)
            xb = b.detach().t().contiguous() if b.dim() == 2 else b.detach().contiguous().clone()
            nrhs = b.shape[1] if b.dim() == 2 else 1
            solve_async(l, n, k, xb, nrhs=nrhs)
            ctx.k, ctx.nrhs, ctx.two_d, ctx.recompute = k, nrhs, b.dim() == 2, recompute
            ctx.save_for_backward(ab if recompute else l, xb)
            return xb.t() if b.dim() == 2 else xb

        @staticmethod
        def backward(ctx, gx):
            saved, xb = ctx.saved_tensors
            k = ctx.k
            l = refactor(saved, k) if ctx.recompute else saved
            n = l.shape[0]
            g = gx.t().contiguous() if ctx.two_d else gx.contiguous().clone()
            gab = torch.zeros_like(l)
            solve_backward(l, n, k, xb, g, gab, nrhs=ctx.nrhs)
            return gab, (g.t() if ctx.two_d else g), None, None

    class BandCholesky(torch.autograd.Function):
        """L = chol(A) on the band: ``ab`` of shape (n, k+1) (row j = band column j)
        -> the factor in the same layout.  Backward: the reverse mode of the
        factorization (bandchol_factor_backward), gradient on the stored band."""

        @staticmethod
        def forward(ctx, ab, k):
            l = refactor(ab, k)
            ctx.k = k
            ctx.save_for_backward(l)
            return l

        @staticmethod
        def backward(ctx, gl):
            (l,) = ctx.saved_tensors
            n, k = l.shape[0], ctx.k
            gab = gl.detach().contiguous().clone()
            # the band's bottom-right corner (past row n-1) holds no entry
            status = torch.zeros(1, dtype=torch.int64, device=l.device)
            factor_backward(l, n, k, gab, gab, d_status=status)
            if int(status.item()) != 0:
                raise BandCholError("bandchol_factor_backward: a device-side wait exceeded its bound")
            return gab, None

    class BandSolveBatch(torch.autograd.Function):
        """Batch of equal-shape systems: ab (B, n, k+1), b (B, n, nrhs) -> x (B, n, nrhs),
        through one BatchPlan (factor, solve and reverse mode batched)."""

        @staticmethod
        def forward(ctx, ab, b, k, recompute=False):
            bsz, n = ab.shape[0], ab.shape[1]
            nrhs = b.shape[2]
            l = ab.detach().contiguous().clone()
            xb = b.detach().transpose(1, 2).contiguous()
            plan = BatchPlan([n] * bsz, [k] * bsz, [l[i] for i in range(bsz)], [xb[i] for i in range(bsz)])
            info = torch.zeros(bsz, dtype=torch.int64, device=ab.device)
            plan.factor(info)
            plan.solve(nrhs)
            bad = torch.nonzero(info).flatten().tolist()
            if bad:
                plan.close()
                raise BandCholError("systems %s are not positive definite" % bad)
            ctx.nrhs, ctx.k, ctx.recompute = nrhs, k, recompute
            if recompute:
                # no factors kept: the plan (which names them) goes too
                torch.cuda.current_stream().synchronize()
                plan.close()
                ctx.plan = None
                ctx.save_for_backward(ab, xb)
            else:
                ctx.plan = plan
                ctx.save_for_backward(l, xb)
            return xb.transpose(1, 2)

        @staticmethod
        def backward(ctx, gx):
            saved, xb = ctx.saved_tensors
            plan = ctx.plan
            if ctx.recompute:
                bsz, n = saved.shape[0], saved.shape[1]
                l = saved.detach().contiguous().clone()
                plan = BatchPlan([n] * bsz, [ctx.k] * bsz, [l[i] for i in range(bsz)], [xb[i] for i in range(bsz)])
                info = torch.zeros(bsz, dtype=torch.int64, device=saved.device)
                plan.factor(info)
                if torch.count_nonzero(info).item():
                    plan.close()
                    raise BandCholError("refactorization failed")
            else:
                l = saved
            g = gx.transpose(1, 2).contiguous()
            gab = torch.zeros_like(l)
            plan.set_adjoint([g[i] for i in range(g.shape[0])], [gab[i] for i in range(gab.shape[0])])
            plan.backward(ctx.nrhs)
            torch.cuda.current_stream().synchronize()
            plan.close()
            return gab, g.transpose(1, 2), None, None

    return BandSolve, BandSolveBatch, BandCholesky


_FUNCS = None


def band_solve(ab, b, k, recompute=False):
    """Differentiable x = A^{-1} b (see BandSolve)."""
    global _FUNCS
    if _FUNCS is None:
        _FUNCS = _autograd_functions()
    return _FUNCS[0].apply(ab, b, k, recompute)


def band_solve_batch(ab, b, k, recompute=False):
    """Differentiable batched x = A^{-1} b (see BandSolveBatch)."""
    global _FUNCS
    if _FUNCS is None:
        _FUNCS = _autograd_functions()
    return _FUNCS[1].apply(ab, b, k, recompute)


def band_cholesky(ab, k):
    """Differentiable band Cholesky factor L of A (see BandCholesky)."""
    global _FUNCS
    if _FUNCS is None:
        _FUNCS = _autograd_functions()
    return _FUNCS[2].apply(ab, k)


def finalize():
    if _lib is not None:
        _lib.bandchol_finalize()
