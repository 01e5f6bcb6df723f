"""The C-ABI library: it loads, exports every symbol the header declares, and
rejects bad arguments before touching the GPU (no GPU needed)."""
import ctypes
import os
import re

import pytest

import paper_2305_04635_amd as bc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bandchol.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bandchol_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_header():
    lib = bc.load()
    names = declared_symbols()
    assert names, "no declarations found"
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(bc.SIGNATURES) == names


def test_tile_width():
    assert bc.tile() in (16, 32, 64)


def test_bad_arguments_rejected_on_host():
    lib = bc.load()
    assert lib.bandchol_factor(-1, 2, None, 3) == -1
    assert lib.bandchol_factor(5, -1, None, 3) == -2
    assert lib.bandchol_factor(5, 2, None, 3) == -3
    assert lib.bandchol_factor(5, 2, 8, 2) == -4
    assert lib.bandchol_factor_async(5, 2, 8, 3, None, None) == -5
    assert lib.bandchol_factor_noalloc(-1, 2, None, 3, None, None) == -1
    assert lib.bandchol_factor_noalloc(5, -1, None, 3, None, None) == -2
    assert lib.bandchol_factor_noalloc(5, 2, None, 3, None, None) == -3
    assert lib.bandchol_factor_noalloc(5, 2, 8, 2, None, None) == -4
    assert lib.bandchol_factor_noalloc(5, 2, 8, 3, None, None) == -5
    assert lib.bandchol_solve(-1, 2, 1, None, 3, None, 5) == -1
    assert lib.bandchol_solve(5, -2, 1, None, 3, None, 5) == -2
    assert lib.bandchol_solve(5, 2, -1, None, 3, None, 5) == -3
    assert lib.bandchol_solve(5, 2, 1, None, 3, None, 5) == -4
    assert lib.bandchol_solve(5, 2, 1, 8, 2, None, 5) == -5
    assert lib.bandchol_solve(5, 2, 1, 8, 3, None, 5) == -6
    assert lib.bandchol_solve(5, 2, 1, 8, 3, 8, 4) == -7


def test_nothing_to_do_is_success():
    lib = bc.load()
    assert lib.bandchol_solve(0, 3, 1, None, 4, None, 1) == 0
    assert lib.bandchol_solve(10, 3, 0, 8, 4, None, 10) == 0


def test_binding_rejects_cpu_tensors():
    torch = pytest.importorskip("torch")
    with pytest.raises(TypeError):
        bc.factor(torch.zeros(12, dtype=torch.float64), 4, 2)


def test_batch_bad_arguments_rejected_on_host():
    lib = bc.load()
    I64 = ctypes.c_int64 * 2
    P = ctypes.c_void_p * 2
    plan = ctypes.c_void_p()
    n, k, ldab = I64(10, 20), I64(3, 4), I64(4, 5)
    ab, b, ldb = P(8, 16), P(24, 32), I64(10, 20)
    ok = (n, k, ab, ldab, b, ldb)

    def create(batch=2, n=n, k=k, ab=ab, ldab=ldab, b=b, ldb=ldb, plan=ctypes.byref(plan)):
        return lib.bandchol_batch_create(batch, n, k, ab, ldab, b, ldb, plan)

    assert create(batch=-1) == -1
    assert create(plan=None) == -8
    assert create(n=I64(10, -1)) == -2
    assert create(k=I64(3, -4)) == -3
    assert create(ab=P(8, None)) == -4
    assert create(ldab=I64(4, 4)) == -5
    assert create(b=P(None, 32)) == -6
    assert create(ldb=I64(10, 19)) == -7
    assert ok and plan.value is None          # nothing was created
    assert lib.bandchol_batch_factor(None, 8, None) == -1
    assert lib.bandchol_batch_solve(None, -1, None) == -1
    assert lib.bandchol_batch_solve(None, 1, None) == -3
    lib.bandchol_batch_destroy(None)          # no-op


def test_f32_and_mixed_bad_arguments_rejected_on_host():
    lib = bc.load()
    assert lib.bandchol_factor_f32(-1, 2, None, 3, 8, None) == -1
    assert lib.bandchol_factor_f32(5, -1, None, 3, 8, None) == -2
    assert lib.bandchol_factor_f32(5, 2, None, 3, 8, None) == -3
    assert lib.bandchol_factor_f32(5, 2, 8, 2, 8, None) == -4
    assert lib.bandchol_factor_f32(5, 2, 8, 3, None, None) == -5
    m = lib.bandchol_mixed_solve
    assert m(-1, 2, 1, 8, 3, 8, 5, 8, 5, None, None) == -1
    assert m(5, -2, 1, 8, 3, 8, 5, 8, 5, None, None) == -2
    assert m(5, 2, -1, 8, 3, 8, 5, 8, 5, None, None) == -3
    assert m(5, 2, 1, None, 3, 8, 5, 8, 5, None, None) == -4
    assert m(5, 2, 1, 8, 2, 8, 5, 8, 5, None, None) == -5
    assert m(5, 2, 1, 8, 3, None, 5, 8, 5, None, None) == -6
    assert m(5, 2, 1, 8, 3, 8, 4, 8, 5, None, None) == -7
    assert m(5, 2, 1, 8, 3, 8, 5, None, 5, None, None) == -8
    assert m(5, 2, 1, 8, 3, 8, 5, 8, 4, None, None) == -9
    it, fb = ctypes.c_int64(7), ctypes.c_int64(7)
    assert m(0, 2, 1, None, 3, None, 1, None, 1, ctypes.byref(it), ctypes.byref(fb)) == 0
    assert it.value == 0 and fb.value == 0


def test_schedule_rule_and_table_on_host(tmp_path, monkeypatch):
    """The schedule per (n, k) bucket: the rule where the table has no entry,
    table entries per (floor(log2 n), K) bucket, the walk limit first, the
    argument checks, and a JSON round trip (host logic only)."""
    monkeypatch.delenv("BANDCHOL_MAX_WG", raising=False)
    lib = bc.load()
    bc.tune_clear()
    prev = bc.set_walk_limit(0)
    try:
        # rule: a quarter, one or two workgroups per CU (256 CUs) by K
        assert bc.schedule(100000, 0) == 1            # diagonal: the walk
        assert bc.schedule(100000, 50) == 64          # K = 2
        assert bc.schedule(100000, 352) == 64         # K = 11
        assert bc.schedule(100000, 353) == 256        # K = 12
        assert bc.schedule(100000, 500) == 256        # K = 16
        assert bc.schedule(100000, 768) == 256        # K = 24
        assert bc.schedule(100000, 1000) == 256       # K = 32
        assert bc.schedule(100000, 1500) == 256       # K = 47
        assert bc.schedule(100000, 1760) == 256       # K = 55
        assert bc.schedule(100000, 1761) == 512       # K = 56
        assert bc.schedule(100000, 2000) == 512       # K = 63
        assert bc.schedule(100000, 99999) == 512
        assert bc.schedule(40, 1000) == 64            # k clipped to n - 1: K = 2
        assert lib.bandchol_schedule(0, 5) == 0
        assert lib.bandchol_schedule(-1, 5) == -1
        assert lib.bandchol_schedule(5, -1) == -2
        # the walk limit comes first
        bc.set_walk_limit(3)
        assert bc.schedule(1000, 96) == 1 and bc.schedule(1000, 97) == 64
        bc.set_walk_limit(0)
        # one entry per (floor(log2 n), K) bucket
        bc.tune_set(100000, 1000, 384)
        assert bc.schedule(100000, 1000) == 384
        assert bc.schedule(70000, 993) == 384         # same bucket (16, 32)
        assert bc.schedule(140000, 1000) == 256       # bucket 17: the rule
        assert bc.schedule(100000, 1025) == 256       # K = 33: the rule
        bc.tune_set(90000, 999, 320)                  # replaces the entry of bucket (16, 32)
        assert bc.tune_entries() == [{"n": 90000, "k": 999, "wgs": 320, "ms": 0.0}]
        bc.tune_set(1000, 480, 1)                     # K = 15: the walk is allowed
        assert bc.schedule(1000, 470) == 1
        bc.tune_set(200, 300, 2)                      # k clipped: recorded as 199
        assert {"n": 200, "k": 199, "wgs": 2, "ms": 0.0} in bc.tune_entries()
        # the environment cap applies to the tile schedule only
        monkeypatch.setenv("BANDCHOL_MAX_WG", "100")
        assert bc.schedule(90000, 999) == 100 and bc.schedule(1000, 470) == 1
        monkeypatch.delenv("BANDCHOL_MAX_WG")
        # JSON round trip
        path = str(tmp_path / "tuning.json")
        saved = bc.tune_entries()
        bc.save_tuning(path)
        bc.tune_clear()
        assert bc.tune_entries() == [] and bc.schedule(90000, 999) == 256
        bc.load_tuning(path)
        assert sorted((e["n"], e["k"], e["wgs"]) for e in bc.tune_entries()) == \
            sorted((e["n"], e["k"], e["wgs"]) for e in saved)
        bc.tune_set(90000, 999, 0)                    # removes the bucket's entry
        assert bc.schedule(90000, 999) == 256 and len(bc.tune_entries()) == 2
        # argument checks
        assert lib.bandchol_tune_set(100000, 1000, 1) == -3     # K = 32: no walk
        assert lib.bandchol_tune_set(1000, 0, 64) == -3         # K = 0: walk only
        assert lib.bandchol_tune_set(1000, 100, 513) == -3      # above 2 x CUs
        assert lib.bandchol_tune_set(1000, 100, -1) == -3
        assert lib.bandchol_tune_set(0, 1, 64) == -1
        assert lib.bandchol_tune_set(10, -1, 64) == -2
        assert lib.bandchol_tune_entries(-1, None, None, None, None) == -1
        assert lib.bandchol_tune_entries(1, None, None, None, None) == -2
        assert lib.bandchol_tune_entries(0, None, None, None, None) == 2
        assert lib.bandchol_tune_factor(0, 1, 1, None, None) == -1
        assert lib.bandchol_tune_factor(10, -1, 1, None, None) == -2
        assert lib.bandchol_tune_factor(10, 1, 0, None, None) == -3
        assert lib.bandchol_tune_factor(10, 1, 1001, None, None) == -3
        with pytest.raises(bc.BandCholError):
            bc.tune_set(1000, 0, 64)
    finally:
        bc.tune_clear()
        bc.set_walk_limit(prev)


def test_batch_schedule_table_on_host(tmp_path):
    """The batch plans' schedule table: entries per bucket, JSON round trip
    together with the single-matrix table, argument checks (no GPU work)."""
    lib = bc.load()
    bc.batch_tune_clear()
    bc.tune_clear()
    try:
        bc.batch_tune_set(20000, 256, 64)             # bucket (14, 8): the tile schedule
        bc.batch_tune_set(17000, 250, 1)              # same bucket: replaced by the walk
        bc.batch_tune_set(3000, 100, 2)
        assert sorted((e["n"], e["k"], e["wgs"]) for e in bc.batch_tune_entries()) == \
            [(3000, 100, 2), (17000, 250, 1)]
        assert bc.tune_entries() == []                # the single-matrix table is apart
        bc.tune_set(100000, 1000, 384)
        path = str(tmp_path / "tuning.json")
        bc.save_tuning(path)
        bc.batch_tune_clear()
        bc.tune_clear()
        bc.load_tuning(path)
        assert len(bc.batch_tune_entries()) == 2 and len(bc.tune_entries()) == 1
        bc.batch_tune_set(3000, 100, 0)
        assert [e["k"] for e in bc.batch_tune_entries()] == [250]
        assert lib.bandchol_batch_tune_set(100000, 1000, 1) == -3   # K = 32: no walk
        assert lib.bandchol_batch_tune_set(1000, 0, 64) == -3       # K = 0: walk only
        assert lib.bandchol_batch_tune_set(0, 1, 1) == -1
        assert lib.bandchol_batch_tune_set(10, -1, 1) == -2
        assert lib.bandchol_batch_tune_entries(1, None, None, None, None) == -2
        I64 = ctypes.c_int64 * 2
        assert lib.bandchol_batch_tune(0, I64(10, 20), I64(1, 2), 1, 1, None) == -1
        assert lib.bandchol_batch_tune(2, None, I64(1, 2), 1, 1, None) == -2
        assert lib.bandchol_batch_tune(2, I64(10, 0), I64(1, 2), 1, 1, None) == -2
        assert lib.bandchol_batch_tune(2, I64(10, 20), I64(1, -2), 1, 1, None) == -3
        assert lib.bandchol_batch_tune(2, I64(10, 20), I64(1, 2), 0, 1, None) == -4
        assert lib.bandchol_batch_tune(2, I64(10, 20), I64(1, 2), 1, -1, None) == -5
    finally:
        bc.batch_tune_clear()
        bc.tune_clear()


def test_spine_profile_bad_arguments_on_host():
    lib = bc.load()
    out = (ctypes.c_double * 13)()
    assert lib.bandchol_spine_profile(1, 10, 1, out, 13) == -1
    assert lib.bandchol_spine_profile(100, 0, 1, out, 13) == -2
    assert lib.bandchol_spine_profile(100, 10, 0, out, 13) == -3
    assert lib.bandchol_spine_profile(100, 10, 1, None, 13) == -4
    assert lib.bandchol_spine_profile(100, 10, 1, out, 12) == -4
    assert lib.bandchol_pivot_chain_ns(0, None) == -1
    v = ctypes.c_double()
    assert lib.bandchol_pivot_chain_ns(10, None) == -2
