"""The Sec. 3.1 plasma density profile as an input shape (CPU): the
super-Gaussian factor against its definition (half maximum at centre +-
FWHM/2, symmetric, zero at and below x_min), the per-column counts, and the
generated particles' placement."""
import math

import numpy as np
import pytest

from paper_2310_11393_amd import workloads as wl


def _sp(**kw):
    base = dict(q=-1.0, m=1.0, density=0.3, region=(4, 60, 2, 5), ppc=8,
                seed=9, profile=wl.PROFILE_SUPERGAUSS, profile_center=30.0,
                profile_fwhm=24.0, profile_order=12.0, profile_xmin=5.0)
    base.update(kw)
    return wl.Species(**base)


def test_profile_factor_definition():
    sp = _sp()
    assert wl.profile_factor(sp, 30.0) == 1.0
    for h in (18.0, 42.0):  # centre -+ FWHM / 2
        assert abs(wl.profile_factor(sp, h) - 0.5) < 1e-15
    for d in (3.0, 9.0, 11.5, 14.0):
        assert wl.profile_factor(sp, 30 - d) == wl.profile_factor(sp, 30 + d)
    assert wl.profile_factor(sp, 5.0) == 0.0  # at x_min: zero
    assert wl.profile_factor(sp, 4.9) == 0.0
    # order 12: flat top, steep sides
    assert wl.profile_factor(sp, 36.0) > 0.999
    assert wl.profile_factor(sp, 45.0) < 0.06


def test_column_counts_follow_the_profile():
    sp = _sp()
    dx = 0.5
    off = wl.profile_offsets(sp, 4, 60, dx)
    cnt = np.diff(off)
    for c, k in zip(range(4, 60), cnt):
        f = wl.profile_factor(sp, (c + 0.5) * dx)
        assert k == math.floor(sp.ppc * f + 0.5)
        assert abs(k / sp.ppc - f) <= 0.5 / sp.ppc
    assert sp.count(dx) == off[-1] * 3


def test_generated_particles_sit_in_their_columns():
    sp = _sp()
    g = wl.Grid(dims=2, nx=64, ny=8, dx=0.5, dy=0.5, dt=0.3)
    x, y, ux, uy, uz = wl.generate_particles(sp, g)
    off = wl.profile_offsets(sp, 4, 60, g.dx)
    assert len(x) == off[-1] * 3
    col = np.floor(x / g.dx).astype(int)
    row = np.floor(y / g.dy).astype(int)
    per_col = np.bincount(col - 4, minlength=56)
    assert np.array_equal(per_col, np.diff(off) * 3)
    assert row.min() == 2 and row.max() == 4
    # ids: rows outer, columns inner, a column's particles consecutive
    per_row = int(off[-1])
    assert np.all(row == 2 + np.arange(len(x)) // per_row)
    assert np.all(np.diff(col[:per_row]) >= 0)
    # a subrange generates the same particles
    xs, ys, *_ = wl.generate_particles(sp, g, first=37, count=50)
    assert np.array_equal(xs, x[37:87]) and np.array_equal(ys, y[37:87])


def test_paper3d_profile_workload():
    g, sp, inc = wl.paper3d_lp()
    off = wl.profile_offsets(sp, sp.region[0], sp.region[1], g.dx)
    cnt = np.diff(off)
    assert cnt.max() == sp.ppc and cnt[0] == 0
    # half-maximum point of the profile: x = 281.5 - 335.1 / 2 = 113.95
    c = int(113.95 / g.dx)
    assert abs(wl.profile_factor(sp, 113.95) - 0.5) < 1e-12
    assert cnt[c - 4 - sp.region[0]] <= 1 <= cnt[c + 4 - sp.region[0]]
