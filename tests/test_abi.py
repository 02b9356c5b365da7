"""The C-ABI library loads, exports every entry point include/tslb.h
declares, and rejects invalid arguments before touching a GPU (no compute
calls here: these tests run without one)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tslb.h")
LIB = os.path.join(ROOT, "paper_2401_17074_amd", "libtslb.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tslb_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__.build()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) == 30
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_the_header():
    from paper_2401_17074_amd import _binding
    assert sorted(_binding.SIGNATURES) == _declared()


def test_struct_layout_matches_header():
    from paper_2401_17074_amd import _binding
    # int[6], float[3], float[2], float, float, (pad to 8) uint64, int, float[3]
    assert ctypes.sizeof(_binding.tslb_bc) == 88
    assert _binding.tslb_bc.seed.offset == 56


@pytest.mark.parametrize("args,code", [
    ((8, 8, 8, 15, 0.8), -2),     # D3Q27, D3Q19 and D2Q9 only
    ((8, 8, 2, 9, 0.8), -1),      # D2Q9 needs nz = 1
    ((8, 8, 8, 27, 0.5), -1),     # tau must exceed 1/2
    ((0, 8, 8, 27, 0.8), -1),     # dims
    ((8, 8, 8, 27, float("nan")), -1),
    ((1024, 1024, 1024, 27, 0.8), -1),  # 2^30 nodes: beyond 32-bit field offsets
])
def test_create_rejects_invalid_arguments(lib, args, code):
    from paper_2401_17074_amd import _binding as C
    h = ctypes.c_void_p()
    rc = C.lib.tslb_create(*args, None, None, ctypes.byref(h))
    assert rc == code
    assert h.value is None
    assert C.tslb_last_error() != ""


def test_create_rejects_bad_boundaries(lib):
    from paper_2401_17074_amd import _binding as C
    h = ctypes.c_void_p()
    bc = C.make_bc(faces=(C.TSLB_PERIODIC, C.TSLB_WALL, 0, 0, 0, 0))
    assert C.lib.tslb_create(8, 8, 8, 27, 0.8, None, ctypes.byref(bc), ctypes.byref(h)) == -1
    assert "paired" in C.tslb_last_error()
    bc = C.make_bc(faces=(0, 0, C.TSLB_WALL, C.TSLB_WALL, 0, 0))
    assert C.lib.tslb_create(8, 2, 8, 27, 0.8, None, ctypes.byref(bc), ctypes.byref(h)) == -1
    bc = C.make_bc(storage=C.TSLB_FP16, scale=(3.0, 0.0, 0.0))
    assert C.lib.tslb_create(8, 8, 8, 27, 0.8, None, ctypes.byref(bc), ctypes.byref(h)) == -1
    assert "power of two" in C.tslb_last_error()
    assert C.lib.tslb_destroy(None) == 0


def test_noalloc_reduce_rejects_null_arguments(lib):
    from paper_2401_17074_amd import _binding as C
    assert C.lib.tslb_reduce_noalloc(None, None, None) == C.TSLB_E_INVALID
    assert "NULL" in C.tslb_last_error()


def test_stream_copy_rejects_bad_arguments(lib):
    """Argument checks come before any device access (the addresses below
    are never dereferenced)."""
    from paper_2401_17074_amd import _binding as C
    assert C.lib.tslb_stream_copy(None, None, 16, None) == C.TSLB_E_INVALID
    assert C.lib.tslb_stream_copy(0x10008, 0x20000, 16, None) == C.TSLB_E_INVALID
    assert "multiples of 16" in C.tslb_last_error()
    assert C.lib.tslb_stream_copy(0x10000, 0x10010, 64, None) == C.TSLB_E_INVALID
    assert "overlap" in C.tslb_last_error()
