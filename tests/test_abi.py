"""CPU checks of the C-ABI boundary: the library loads, exports every symbol
that include/sfpic.h declares, and rejects invalid input before touching a
GPU.  No compute call is made."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sfpic_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_2310_11393_amd import binding
    return binding.lib()


def test_library_exports_every_declared_symbol(L):
    from paper_2310_11393_amd import binding
    names = _declared("sfpic.h")
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert set(names) <= set(binding.EXPORTS)


def test_version_and_error_strings(L):
    assert b"gfx950" in L.sfpic_version()
    assert isinstance(L.sfpic_last_error(), bytes)


def test_invalid_grid_rejected_without_gpu(L):
    from paper_2310_11393_amd import binding as b
    g = b.sfpic_grid(3, 64, 64, 0.2, 0.2, 0.1)  # dims = 3
    h = C.c_void_p()
    rc = L.sfpic_create(C.byref(g), None, 0, None, 0, None, C.byref(h))
    assert rc == -1 and not h.value
    assert b"dims" in L.sfpic_last_error()
    g = b.sfpic_grid(2, 64, 64, 0.2, 0.2, 0.2)  # CFL violated
    rc = L.sfpic_create(C.byref(g), None, 0, None, 0, None, C.byref(h))
    assert rc == -1 and b"CFL" in L.sfpic_last_error()


def test_null_handles_rejected(L):
    assert L.sfpic_step(None, 1) == -1
    assert L.sfpic_sync(None) == -1
    L.sfpic_destroy(None)  # no-op
