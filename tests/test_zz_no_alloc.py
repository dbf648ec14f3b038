"""The allocation-free histogram entry point (sfpic_histogram_noalloc)
against sfpic_histogram, called through the C ABI on the GPU: two calls in a
row, the second with a smaller histogram of a smaller simulation, each equal
to the allocating call's result (the bins are sums of the same weights,
accumulated by atomics in a run-dependent order: relative 1e-12)."""
import ctypes as C

import numpy as np
import pytest

from paper_2310_11393_amd import workloads as wl

from parity_util import make_gpu

pytestmark = pytest.mark.gpu


def _hist(L, b, h, n_e, n_t, emax, noalloc):
    spec = b.sfpic_hist_spec(0, n_e, emax, n_t, 0.0)
    out = np.full(n_e * n_t, -1.0)
    mom = np.zeros(5)
    fn = L.sfpic_histogram_noalloc if noalloc else L.sfpic_histogram
    rc = fn(h, C.byref(spec), out.ctypes.data_as(C.POINTER(C.c_double)),
            out.size, mom.ctypes.data_as(C.POINTER(C.c_double)))
    return rc, out, mom


def _check_equal(a, b):
    assert np.all(np.isfinite(a)) and a.sum() > 0
    assert np.allclose(a, b, rtol=1e-12, atol=1e-14 * b.max())


def test_noalloc_histogram_matches_the_allocating_call():
    from paper_2310_11393_amd import binding as b
    L = b.lib()
    big = wl.april_2d(nx=136, ny=72, plasma=(40, 100, 0, 72), ppc=8,
                      a0=20.0, s=10.0, steps=40, seed=11)
    small = wl.april_2d(nx=64, ny=40, plasma=(20, 44, 4, 36), ppc=2,
                        a0=15.0, s=10.0, steps=30, seed=12)
    gb = make_gpu(big)
    gs = make_gpu(small)
    gb.step(big.steps)
    gs.step(small.steps)
    # first call: a large histogram of the larger simulation
    rc1, h1, m1 = _hist(L, b, gb.h, 256, 180, 2.0, True)
    assert rc1 == 0, L.sfpic_last_error(gb.h)
    rc0, h0, m0 = _hist(L, b, gb.h, 256, 180, 2.0, False)
    assert rc0 == 0
    _check_equal(h1, h0)
    assert np.allclose(m1, m0, rtol=1e-12, atol=0)
    # second call: smaller histogram, smaller simulation; the bins the
    # first call left in the scratch must not leak into it
    rc1, h1, m1 = _hist(L, b, gs.h, 32, 18, 0.5, True)
    assert rc1 == 0, L.sfpic_last_error(gs.h)
    rc0, h0, m0 = _hist(L, b, gs.h, 32, 18, 0.5, False)
    assert rc0 == 0
    _check_equal(h1, h0)
    assert np.allclose(m1, m0, rtol=1e-12, atol=0)
    # above the fixed maximum: a clear error, nothing written
    n_e, n_t = 1024, 128
    rc, out, _ = _hist(L, b, gs.h, n_e, n_t, 1.0, True)
    assert rc == -2 and np.all(out == -1.0)
    assert b"SFPIC_HIST_NOALLOC_MAX_BINS" in L.sfpic_last_error(gs.h)
    gb.close()
    gs.close()
