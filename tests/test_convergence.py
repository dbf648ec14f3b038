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


def test_cross_norm_counts_physical_nodes_only():
    nc, h = 30, 0.2
    a = np.full(nc + 2 * G, 5.0)
    b = a + 0.25
    b[:G] = b[G + nc + 1:] = 1e9  # guards never enter the norm
    assert math.isclose(cv.cross_norm(a, b, nc, h),
                        math.sqrt(h * (nc + 1) * 0.0625), rel_tol=1e-14)
    assert math.isclose(cv.cross_norm(a, b, nc, h, dual=True),
                        math.sqrt(h * nc * 0.0625), rel_tol=1e-14)


def test_energy_norm_is_the_mean_absolute_difference():
    assert cv.energy_norm([1.0, 2.0, 3.0], [1.0, 1.0, 1.0]) == 1.0
    assert cv.energy_norm([1.0, -2.0], [0.0, 0.0], scale=3.0) == 0.5
    for a, b in (([1.0], [1.0, 2.0]), ([], [])):
        try:
            cv.energy_norm(a, b)
        except ValueError:
            continue
        raise AssertionError("mismatched series accepted")


def test_study_cross_and_energy_norms_of_second_order_models():
    """Two models whose fields err by c_i h^2 cos(x) and whose energies err
    by d_i h^2: the cross-norm is |c_1 - c_2| h^2 ||cos||_{2,h} (rate 2) and
    the energy norms against the finest grid scale as h^2 - h_fine^2."""
    L = 12.0
    ts = (0.5, 1.0)

    def study(c, d):
        out = {}
        for m in range(4):
            nc = 24 * 2 ** m
            h = L / nc
            out[m] = {t: {"ey_total": _row(nc, h, lambda x: np.sin(x + t) +
                                           c * h * h * np.cos(x)),
                          "w_em": 1.0 + t + d * h * h, "nx": nc, "h": h}
                      for t in ts}
        return out

    s1, s2 = study(0.5, 2.0), study(-0.25, -1.0)
    cn = cv.study_cross_norms(s1, s2, "ey")
    for m in range(4):
        h = L / (24 * 2 ** m)
        x = np.arange(24 * 2 ** m + 1) * h
        want = 0.75 * h * h * math.sqrt(h * float(np.sum(np.cos(x) ** 2)))
        for t in ts:
            assert math.isclose(cn[m][t], want, rel_tol=1e-9)
    assert abs(cv.rate(cn[0][ts[0]], cn[1][ts[0]]) - 2.0) < 0.05
    hf = L / (24 * 8)
    en = cv.study_energy_norms(s1, "w_em", scale=2.0)
    for m, v in enumerate(en):
        h = L / (24 * 2 ** m)
        assert math.isclose(v, 2.0 * (h * h - hf * hf) / 2.0, rel_tol=1e-9)


def _plane(nx, ny, h, comp, f):
    """A 2D plane with guards holding f(x, y) at the component's nodes."""
    hx, hy = cv.STAGGER[comp]
    x = (np.arange(nx + 2 * G) - G + 0.5 * hx) * h
    y = (np.arange(ny + 2 * G) - G + 0.5 * hy) * h
    return f(x[None, :], y[:, None])


def test_2d_physical_nodes_and_frobenius_error():
    nx, ny, h = 20, 12, 0.3
    for comp, shape in (("ey", (12, 21)), ("ex", (13, 20)), ("ez", (13, 21)),
                        ("bz", (12, 20))):
        p = _plane(nx, ny, h, comp, lambda x, y: 1.0 + x * y)
        assert cv.physical(p, nx, ny, comp).shape == shape, comp
        q = p * 1.25
        q[:G] = 7e7  # guards never enter
        assert math.isclose(cv.frobenius_error(q, p, nx, ny, comp), 0.25,
                            rel_tol=1e-13)


def test_2d_intensity_and_axis_row_are_exact_for_linear_fields():
    nx, ny, h = 16, 10, 0.5
    fy = lambda x, y: 0.3 + 0.2 * x - 0.7 * y  # noqa: E731
    fx = lambda x, y: -1.1 + 0.4 * x + 0.9 * y  # noqa: E731
    ey = _plane(nx, ny, h, "ey", fy)
    ex = _plane(nx, ny, h, "ex", fx)
    xi = np.arange(1, nx) * h
    yj = np.arange(1, ny) * h
    X, Y = np.meshgrid(xi, yj)
    want = fy(X, Y) ** 2 + fx(X, Y) ** 2
    assert np.allclose(cv.intensity(ey, ex, nx, ny), want, rtol=0,
                       atol=1e-12)
    # scaling one model's fields by s gives |s^2 - 1| exactly
    assert math.isclose(cv.intensity_error(1.5 * ey, 1.5 * ex, ey, ex, nx,
                                           ny), 1.25, rel_tol=1e-13)
    x_all = (np.arange(nx + 2 * G) - G) * h
    ja = ny // 2
    assert np.allclose(cv.axis_row(ey, ja, "ey"), fy(x_all, ja * h),
                       rtol=0, atol=1e-12)
    xd = (np.arange(nx + 2 * G) - G + 0.5) * h
    assert np.allclose(cv.axis_row(ex, ja, "ex"), fx(xd, ja * h), rtol=0,
                       atol=1e-12)


def test_2d_axis_norms_of_a_second_order_model():
    L, t = 9.0, 1.0
    study = {}
    for m in range(3):
        n = 18 * 2 ** m
        h = L / n
        row = _row(n, h, lambda x: np.sin(x) + 0.4 * h * h * np.cos(x))
        study[m] = {t: {"ey_axis": row, "nx": n, "h": h}}
    norms = cv.study_axis_norms(study, "ey")[t]
    hf = L / 72
    for m, v in enumerate(norms):
        h = L / (18 * 2 ** m)
        x = np.arange(18 * 2 ** m + 1) * h
        want = 0.4 * (h * h - hf * hf) * math.sqrt(h * float(np.sum(
            np.cos(x) ** 2)))
        assert math.isclose(v, want, rel_tol=1e-9)
