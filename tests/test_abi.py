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
