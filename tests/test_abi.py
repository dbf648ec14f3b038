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
    return sorted(set(re.findall(r"\b(sfpic3?_\w+)\s*\(", text)))


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
    assert isinstance(L.sfpic_last_error(None), bytes)


def test_last_error_takes_a_handle(L):
    """The error call follows the boundary's per-handle form: a message for
    the last failure on a handle, NULL for the calling thread's last one."""
    text = open(os.path.join(ROOT, "include", "sfpic.h")).read()
    assert re.search(r"const char \*sfpic_last_error\(const void \*handle\);",
                     text)
    from paper_2310_11393_amd import binding as b
    g = b.sfpic_grid(3, 64, 64, 0.2, 0.2, 0.1)
    h = C.c_void_p()
    assert L.sfpic_create(C.byref(g), None, 0, None, 0, None,
                          C.byref(h)) == -1
    assert b"dims" in L.sfpic_last_error(None)
    # a handle that never failed (here: one that does not exist) has none
    assert L.sfpic_last_error(C.c_void_p(0x1000)) == b""


def test_invalid_grid_rejected_without_gpu(L):
    from paper_2310_11393_amd import binding as b
    g = b.sfpic_grid(3, 64, 64, 0.2, 0.2, 0.1)  # dims = 3
    h = C.c_void_p()
    rc = L.sfpic_create(C.byref(g), None, 0, None, 0, None, C.byref(h))
    assert rc == -1 and not h.value
    assert b"dims" in L.sfpic_last_error(None)
    g = b.sfpic_grid(2, 64, 64, 0.2, 0.2, 0.2)  # CFL violated
    rc = L.sfpic_create(C.byref(g), None, 0, None, 0, None, C.byref(h))
    assert rc == -1 and b"CFL" in L.sfpic_last_error(None)


def test_invalid_3d_input_rejected_without_gpu(L):
    from paper_2310_11393_amd import binding as b
    h = C.c_void_p()
    g = b.sfpic3_grid(16, 16, 16, 0.2, 0.2, 0.2, 0.2)  # CFL violated
    assert L.sfpic3_create(C.byref(g), None, 0, None, 0, None,
                           C.byref(h)) == -1
    assert b"CFL" in L.sfpic_last_error(None) and not h.value
    g = b.sfpic3_grid(16, 0, 16, 0.2, 0.2, 0.2, 0.05)
    assert L.sfpic3_create(C.byref(g), None, 0, None, 0, None,
                           C.byref(h)) == -1
    g = b.sfpic3_grid(16, 16, 16, 0.2, 0.2, 0.2, 0.05)
    assert L.sfpic3_create(C.byref(g), None, 0, None, 7, None,
                           C.byref(h)) == -1
    assert b"precision" in L.sfpic_last_error(None)
    g = b.sfpic3_grid(16, 16, 16, 0.2, 0.2, 0.2, 0.05)
    inc = b.sfpic_incident()
    inc.kind, inc.a0, inc.w0, inc.fwhm_t = 4, 1.0, 2.0, 5.0  # 2D-only beam
    assert L.sfpic3_create(C.byref(g), None, 0, C.byref(inc), 0, None,
                           C.byref(h)) == -1
    assert b"2D" in L.sfpic_last_error(None)
    x = (C.c_double * 1)(3.3)  # outside [0, 16 * 0.2)
    zero = (C.c_double * 1)(0.1)
    sp = b.sfpic3_species()
    sp.q, sp.m, sp.n_explicit, sp.weight = -1.0, 1.0, 1, 0.1
    sp.x, sp.y, sp.z = x, zero, zero
    sp.ux, sp.uy, sp.uz = zero, zero, zero
    assert L.sfpic3_create(C.byref(g), C.byref(sp), 1, None, 0, None,
                           C.byref(h)) == -1
    assert b"outside" in L.sfpic_last_error(None)
    assert L.sfpic3_step(None, 1) == -1
    L.sfpic3_destroy(None)


def test_null_handles_rejected(L):
    assert L.sfpic_step(None, 1) == -1
    assert L.sfpic_sync(None) == -1
    L.sfpic_destroy(None)  # no-op


STRUCTS = ["sfpic_grid", "sfpic_species", "sfpic_incident", "sfpic_runtime",
           "sfpic_diag", "sfpic_hist_spec", "sfpic_kernel_stats",
           "sfpic_sim_desc", "sfpic_result", "sfpic_batch_info",
           "sfpic_server_info", "sfpic3_grid", "sfpic3_species"]


def test_ctypes_layouts_match_the_header(tmp_path):
    """Size and every field offset of the binding's ctypes structures equal
    what a C compiler makes of include/sfpic.h."""
    import subprocess
    from paper_2310_11393_amd import binding as b
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sfpic.h"',
             'int main(void) {']
    for name in STRUCTS:
        cls = getattr(b, name)
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"),
                    str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True,
                         text=True).stdout.split("\n")
    got = dict(l.split() for l in out if l.strip())
    for name in STRUCTS:
        cls = getattr(b, name)
        assert int(got[name]) == C.sizeof(cls), name
        for f, _ in cls._fields_:
            assert int(got[f"{name}.{f}"]) == getattr(cls, f).offset, (name, f)


def test_footprint_is_computed_on_the_host(L):
    """sfpic_desc_footprint needs no GPU; it grows with the particle count
    by the bytes of two particle sets plus the sort and straggler arrays."""
    from paper_2310_11393_amd import binding as b
    from paper_2310_11393_amd import workloads as wl
    w = wl.sweep_member(3)
    d1 = b.SimDesc(w).footprint()
    w.species[0].ppc *= 2
    d2 = b.SimDesc(w).footprint()
    n = w.species[0].count() // 2
    per = 2 * 7 * 4 + 3 * 4  # FP32: two sets of 7 words, key/rank/straggler
    assert abs((d2 - d1) - n * per) <= 64 * 256
    assert d1 > 12 * (w.grid.nx + 6) * (w.grid.ny + 6) * 4


def test_batch_and_server_reject_bad_arguments(L):
    from paper_2310_11393_amd import binding as b
    from paper_2310_11393_amd import workloads as wl
    h = C.c_void_p()
    assert L.sfpic_batch_create(0, None, None, C.byref(h)) == -1
    d = b.SimDesc(wl.sweep_member(0), nsteps=-1)
    assert L.sfpic_batch_create(1, C.byref(d.desc), None, C.byref(h)) == -1
    assert b"nsteps" in L.sfpic_last_error(None)
    d = b.SimDesc(wl.sweep_member(0), hist=b.hist_spec(sp=3))
    assert L.sfpic_batch_create(1, C.byref(d.desc), None, C.byref(h)) == -1
    assert L.sfpic_server_create(0, 0, None, C.byref(h)) == -1
    assert L.sfpic_batch_run(None) == -1
    assert L.sfpic_server_submit(None, None, None) == -1
    L.sfpic_batch_destroy(None)
    L.sfpic_server_destroy(None)
