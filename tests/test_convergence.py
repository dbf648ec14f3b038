"""The convergence-analysis helpers (Sec. 3.1 norms and rate) against
closed forms: coarse and fine grids sample the same function at common
points; an error c h^2 g(x) gives rate 2 exactly; the dual-node mean is
exact for linear fields; the quiet start places the profile's counts."""
import math

import numpy as np

from paper_2310_11393_amd import convergence as cv
from paper_2310_11393_amd import workloads as wl

G = cv.GUARD


def _row(nx, h, f, dual=False):
    """A 1D array with guards holding f at the primal (or dual) nodes."""
    i = np.arange(nx + 2 * G) - G + (0.5 if dual else 0.0)
    return f(i * h)


def test_common_points_primal_and_dual():
    f = lambda x: 0.3 + 1.7 * x  # noqa: E731  linear: the dual mean is exact
    for ratio in (2, 4, 8):
        h = 0.4
        nc = 25
        fine_p = _row(nc * ratio, h / ratio, f)
        fine_d = _row(nc * ratio, h / ratio, f, dual=True)
        xp = np.arange(nc + 1) * h
        xd = (np.arange(nc) + 0.5) * h
        assert np.allclose(cv.common_values(fine_p, ratio, nc, False), f(xp),
                           rtol=0, atol=1e-12)
        assert np.allclose(cv.common_values(fine_d, ratio, nc, True), f(xd),
                           rtol=0, atol=1e-12)


def test_second_order_error_gives_rate_two():
    exact = np.sin
    g = np.cos
    L = 10.0
    norms = []
    for m in range(3):
        nc = 40 * 2 ** m
        h = L / nc
        coarse = _row(nc, h, lambda x: exact(x) + 0.7 * h * h * g(x))
        fine = _row(nc * 4, h / 4, exact)  # error-free reference
        norms.append(cv.l2_norm(coarse, fine, 4, nc, h))
    # ||0.7 h^2 cos||_{2,h} -> 0.7 h^2 ||cos||_{L2(0, L)}
    want = 0.7 * (L / 40) ** 2 * math.sqrt(L / 2 + math.sin(2 * L) / 4)
    assert abs(norms[0] - want) / want < 0.02
    for a, b in zip(norms, norms[1:]):
        assert abs(cv.rate(a, b) - 2.0) < 0.02


def test_quiet_start_follows_the_profile():
    grid = wl.Grid(1, 400, 1, 0.25, 0.25, 0.2)
    e = cv.quiet_profile_1d(grid, 0.1, 8, center=50.0, fwhm=40.0, order=12,
                            xmin=20.0)
    cells = np.floor(e["x"] / grid.dx).astype(int)
    counts = np.bincount(cells, minlength=grid.nx)
    for c in (0, 150, 200, 250, 399):
        f = wl.profile_factor(wl.Species(profile=1, profile_center=50.0,
                                         profile_fwhm=40.0, profile_order=12,
                                         profile_xmin=20.0),
                              (c + 0.5) * grid.dx)
        assert counts[c] == math.floor(8 * f + 0.5)
    # evenly spaced inside each cell
    full = np.nonzero(counts == 8)[0][0]
    xs = np.sort(e["x"][cells == full]) / grid.dx - full
    assert np.allclose(xs, (np.arange(8) + 0.5) / 8)
    assert e["weight"] == 0.1 / 8
