"""Pins of the 2D oracle's energy-angle histogram and of its first-order Mur
faces and corners.

  * Histogram (the Sec. 4.2 energy-angle spectra): particles of known
    momentum land in the bins that their kinetic energy m (gamma - 1) and
    their angle from the propagation axis +x put them in (the polar angle,
    or in the x-z or x-y plane the angle of the projected momentum), with
    weight w dV
    (dV = dx dy in 2D, dx in 1D); the moments are the weighted means over
    particles above the energy cut; removed particles and energies beyond
    the last bin are handled as the definitions say.
  * Mur (reading of the paper's unstated boundary: first-order absorbing
    condition on tangential E at every outer array face).  For the
    continuous first-order condition (Engquist and Majda 1977; Mur 1981) a
    plane wave meeting a face at angle theta from its normal is reflected
    with amplitude R = (cos theta - 1) / (cos theta + 1).
      - Faces: a divergence-free packet sent at normal incidence onto the x
        faces, then onto the y faces (cells of aspect 1.6, so a coefficient
        of the wrong axis matters), in both polarizations, leaves at most
        the energy that one reflection with R over the packet's plane-wave
        spectrum would leave.
      - Corners: a packet sent along a diagonal straight into each of the
        four corners; at the corner node the field may differ from the
        free-space field (the same scheme in a box three times larger) by
        at most the two 45-degree reflections, |(1 + R)^2 - 1| = 0.314,
        plus a discretization margin.
  * Planted mistakes (a y-face Mur coefficient taken from the x axis, the
    corner nodes left out of the corner rule, a histogram angle measured
    from +y, the x-z view projecting on y) are compiled into copies of the
    oracle and must fail a pin.
"""
import math
import os
import shutil
import subprocess
import sys
import tempfile

import numpy as np
import pytest

from oracle import OracleSim
from paper_2310_11393_amd import workloads as wl

G = 3
HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


# ---------------------------------------------------------------------------
# Energy-angle histogram
# ---------------------------------------------------------------------------

def _angle(u, plane):
    """Angle from +x of the momentum (plane 0) or of its projection on the
    x-z (1) or x-y (2) plane, in degrees."""
    perp = {0: np.hypot(u[:, 1], u[:, 2]), 1: np.abs(u[:, 2]),
            2: np.abs(u[:, 1])}[plane]
    return np.degrees(np.arctan2(perp, u[:, 0]))


def _expected_histogram(u, w, dV, n_e, emax, n_t, ek_min, alive, plane=0):
    want = np.zeros((n_e, n_t))
    ek = np.sqrt(1.0 + (u ** 2).sum(1)) - 1.0
    th = _angle(u, plane)
    for e, t, a in zip(ek, th, alive):
        if not a:
            continue
        ie, it = math.floor(e / emax * n_e), min(math.floor(t / 180 * n_t),
                                                  n_t - 1)
        if 0 <= ie < n_e:
            want[ie, it] += w * dV
    sel = alive & (ek > ek_min)
    wt = np.full(sel.sum(), w * dV)
    mom = [wt.sum(), np.average(ek[sel], weights=wt),
           np.average(ek[sel] ** 2, weights=wt),
           np.average(th[sel], weights=wt), np.average(th[sel] ** 2,
                                                       weights=wt)]
    return want, np.array(mom)


@pytest.mark.parametrize("plane", [0, 1, 2])
@pytest.mark.parametrize("dims", [1, 2])
def test_energy_angle_histogram_of_known_particles(dims, plane):
    dx, dy = 0.3, 0.45
    grid = wl.Grid(dims, 10, 8 if dims == 2 else 1, dx, dy, 0.1)
    u = np.array([[1.0, 0.0, 0.0],     # E_k = sqrt(2) - 1, theta = 0
                  [0.0, 0.5, 0.0],     # theta = 90
                  [0.0, 0.0, -0.5],    # theta = 90 (the angle uses |u_perp|)
                  [-2.0, 0.0, 0.0],    # theta = 180: the last angle bin
                  [0.3, -0.4, 0.0],    # theta = atan2(0.4, 0.3)
                  [0.3, 0.0, 0.4],     # the same angle through u_z
                  [-0.6, 0.2, -0.1],   # backward
                  [0.02, 0.01, 0.0],   # below the moments' energy cut
                  [4.0, 1.0, 1.0],     # E_k beyond the last energy bin
                  [0.5, 0.5, 0.5]])    # removed before the histogram
    n = len(u)
    x = np.full(n, 4.2 * dx)
    y = np.full(n, 3.7 * dy) if dims == 2 else np.zeros(n)
    w = 0.25
    sim = OracleSim(grid, wl.Incident())
    sim.add_species(-1.0, 1.0, w, x, y, *u.T)
    alive = np.ones(n, dtype=bool)
    alive[-1] = False
    p = sim.particles()
    sim.set_particles(0, *p[:5], alive)
    n_e, emax, n_t, ek_min = 40, 2.0, 36, 1e-3
    h, mom = sim.energy_angle(n_e=n_e, emax=emax, n_theta=n_t, ek_min=ek_min,
                              plane=plane)
    dV = dx * dy if dims == 2 else dx
    want, want_mom = _expected_histogram(u, w, dV, n_e, emax, n_t, ek_min,
                                         alive, plane)
    assert np.array_equal(h, want)
    # angles that the planes must give: u = (0.3, -0.4, 0) is at
    # atan2(0.4, 0.3) = 53.13 degrees from +x in the polar and x-y views and
    # at 0 in the x-z view; u = (0.3, 0, 0.4) the other way round
    k53 = math.floor(math.degrees(math.atan2(0.4, 0.3)) / 180 * n_t)
    e_k = math.sqrt(1.25) - 1.0
    ie = math.floor(e_k / emax * n_e)
    both = h[ie, k53], h[ie, 0]
    w1 = w * dV
    # (0, 0.5, 0) and (0, 0, -0.5) have the same energy: 90 degrees in the
    # polar view, 0 in the view whose plane is across them
    if plane == 0:
        assert both == (2 * w1, 0.0)
    else:
        assert both == (w1, 2 * w1)
    assert h.sum() == pytest.approx(8 * w * dV, rel=1e-15)
    np.testing.assert_allclose(mom, want_mom, rtol=1e-14, atol=0)


# ---------------------------------------------------------------------------
# First-order Mur: faces and corners
# ---------------------------------------------------------------------------

LAMBDA, SIGMA = 2.4, 1.2   # packet carrier wavelength and Gaussian radius


def _write_packet(sim, pol, dx, dy, centre, direction, shift=(0, 0)):
    """Carrier packet cos(k d.(r - c)) exp(-|r - c|^2 / sigma^2) with B = 0:
    E_z itself (div E = 0 trivially), or the in-plane E = curl(A z) of that
    packet taken as a potential A on the B_z nodes, so that div_h E = 0
    exactly and no static field can stay behind.  shift: the box's first
    physical cell in the coordinates of `centre` (a larger reference box)."""
    d = np.asarray(direction, float)
    d = d / np.linalg.norm(d)

    def f(sx, sy):
        X = (np.arange(sim.NX) - G + 0.5 * sx + shift[0]) * dx
        Y = (np.arange(sim.NY) - G + 0.5 * sy + shift[1]) * dy
        X, Y = np.meshgrid(X, Y)
        s = (X - centre[0]) * d[0] + (Y - centre[1]) * d[1]
        r2 = (X - centre[0]) ** 2 + (Y - centre[1]) ** 2
        return np.cos(2 * math.pi / LAMBDA * s) * np.exp(-r2 / SIGMA ** 2)

    if pol == "ez":
        sim.field("ez")[...] = f(0, 0)
    else:
        a = f(1, 1)
        ex = np.zeros_like(a)
        ey = np.zeros_like(a)
        ex[1:, :] = (a[1:, :] - a[:-1, :]) / dy
        ey[:, 1:] = -(a[:, 1:] - a[:, :-1]) / dx
        sim.field("ex")[...] = ex
        sim.field("ey")[...] = ey


def _one_reflection_energy(direction):
    """Fraction of the packet's energy that one first-order Mur reflection
    leaves: sum over its plane-wave spectrum of R(theta)^2, theta the angle
    between the wave vector and the normal of the face it meets first (the
    packet starts at the centre of a square box)."""
    n, L = 256, 40.0
    h = L / n
    x = (np.arange(n) - n / 2) * h
    X, Y = np.meshgrid(x, x)
    d = np.asarray(direction, float)
    d = d / np.linalg.norm(d)
    f = np.cos(2 * math.pi / LAMBDA * (X * d[0] + Y * d[1])) * np.exp(
        -(X ** 2 + Y ** 2) / SIGMA ** 2)
    p = np.abs(np.fft.fft2(f)) ** 2
    k = np.fft.fftfreq(n, h)
    kx, ky = np.meshgrid(k, k)
    km = np.hypot(kx, ky)
    km[0, 0] = 1.0
    cx, cy = np.abs(kx) / km, np.abs(ky) / km
    c = np.maximum(cx, cy)   # the face met first is the one faced more
    r2 = ((c - 1.0) / (c + 1.0)) ** 2
    return float((p * r2).sum() / p.sum())


def _box(h=0.1, aspect=1.6, side=14.0):
    dx, dy = h, aspect * h
    nx, ny = int(round(side / dx)), int(round(side / dy))
    dt = 0.5 / math.sqrt(1.0 / dx ** 2 + 1.0 / dy ** 2)
    return wl.Grid(2, nx, ny, dx, dy, dt)


@pytest.mark.parametrize("pol", ["ez", "inplane"])
@pytest.mark.parametrize("direction", [(1, 0), (0, 1), (1, 1), (1, -1)])
def test_mur_absorbs_a_packet_at_faces_and_corners(pol, direction):
    g = _box()
    sim = OracleSim(g, wl.Incident())
    _write_packet(sim, pol, g.dx, g.dy, (g.nx * g.dx / 2, g.ny * g.dy / 2),
                  direction)
    w0 = sim.diagnostics()["w_em"]
    t_out = 0.5 * math.hypot(g.nx * g.dx, g.ny * g.dy) + 6 * SIGMA
    sim.step(int(t_out / g.dt))
    left = sim.diagnostics()["w_em"] / w0
    bound = _one_reflection_energy(direction)
    assert 1e-3 < bound < 2e-2
    assert left < bound, (left, bound)


def test_mur_corner_nodes_follow_the_outgoing_wave():
    """E_z at each array corner, for a packet aimed along the diagonal at
    it, against the free-space field of the same scheme (a box three times
    larger whose faces the packet never reaches in this time)."""
    dx, dy = 0.1, 0.16
    nx, ny = 74, 44             # array extents 80 dx = 50 dy: a square
    ox, oy = 80, 50             # the small box inside the large one
    dt = 0.5 / math.sqrt(1.0 / dx ** 2 + 1.0 / dy ** 2)
    centre = (nx / 2 * dx, ny / 2 * dy)
    r45 = (math.cos(math.pi / 4) - 1) / (math.cos(math.pi / 4) + 1)
    allowed = abs((1 + r45) ** 2 - 1) + 0.12
    for sx, sy in ((1, 1), (-1, 1), (1, -1), (-1, -1)):
        small = OracleSim(wl.Grid(2, nx, ny, dx, dy, dt), wl.Incident())
        big = OracleSim(wl.Grid(2, nx + 2 * ox, ny + 2 * oy, dx, dy, dt),
                        wl.Incident())
        _write_packet(small, "ez", dx, dy, centre, (sx, sy))
        _write_packet(big, "ez", dx, dy, centre, (sx, sy), shift=(-ox, -oy))
        i = small.NX - 1 if sx > 0 else 0
        j = small.NY - 1 if sy > 0 else 0
        es, eb = [], []
        for _ in range(int(1.3 * 4.0 * math.sqrt(2) / dt) + 40):
            small.step(1)
            big.step(1)
            es.append(small.field("ez")[j, i])
            eb.append(big.field("ez")[j + oy, i + ox])
        es, eb = np.array(es), np.array(eb)
        peak = np.abs(eb).max()
        assert peak > 0.2           # the packet does reach the corner
        dev = np.abs(es - eb).max() / peak
        assert dev < allowed, ((sx, sy), dev, allowed)


# ---------------------------------------------------------------------------
# Planted mistakes fail the pins above
# ---------------------------------------------------------------------------

MISTAKES = {
    # y-face Mur coefficient of E_x and E_z taken from the x axis
    "mur_y_face_coefficient": (
        [("AT(Ox, i, NY - 1), ky);", "AT(Ox, i, NY - 1), kx);"),
         ("AT(Oz, i, NY - 1), ky);", "AT(Oz, i, NY - 1), kx);"),
         ("AT(Ex, i, 1), AT(Ox, i, 0), ky);", "AT(Ex, i, 1), AT(Ox, i, 0), kx);"),
         ("AT(Ez, i, 1), AT(Oz, i, 0), ky);", "AT(Ez, i, 1), AT(Oz, i, 0), kx);")],
        "test_mur_absorbs_a_packet_at_faces_and_corners"),
    # the four E_z corner nodes never updated
    "mur_corner_rule": (
        [("for (int c = 0; c < 2; ++c) {\n    long j = jc[c];",
          "for (int c = 0; c < 0; ++c) {\n    long j = jc[c];")],
        "test_mur_corner_nodes_follow_the_outgoing_wave"),
    # histogram angle measured from +y instead of the propagation axis
    "histogram_angle_axis": (
        [("double th = atan2(perp, ux) * (180.0 / ORC_PI);",
          "double th = atan2(perp, uy) * (180.0 / ORC_PI);")],
        "test_energy_angle_histogram_of_known_particles"),
    # the x-z view projecting on the wrong transverse axis
    "histogram_plane_axis": (
        [("double perp = plane == 1   ? fabs(uz)",
          "double perp = plane == 1   ? fabs(uy)")],
        "test_energy_angle_histogram_of_known_particles"),
}


def _build_mutant(edits, where):
    src = os.path.join(ROOT, "oracle")
    text = open(os.path.join(src, "sfpic_oracle.c")).read()
    for old, new in edits:
        assert old in text, old
        text = text.replace(old, new)
    with open(os.path.join(where, "sfpic_oracle.c"), "w") as f:
        f.write(text)
    for name in ("sfpic_oracle.h", "sfpic_oracle3d.c"):
        shutil.copy(os.path.join(src, name), where)
    out = os.path.join(where, "liboracle_mutant.so")
    subprocess.check_call(
        ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", out,
         os.path.join(where, "sfpic_oracle.c"),
         os.path.join(where, "sfpic_oracle3d.c"), "-lm"])
    return out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("mistake", sorted(MISTAKES))
def test_planted_mistake_fails_a_pin(mistake):
    edits, test_name = MISTAKES[mistake]
    with tempfile.TemporaryDirectory() as tmp:
        lib = _build_mutant(edits, tmp)
        env = dict(os.environ, SFPIC_ORACLE_LIB=lib)
        r = subprocess.run(
            [sys.executable, "-m", "pytest", "-q", "-x", "-p",
             "no:cacheprovider", f"{os.path.abspath(__file__)}::{test_name}"],
            cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1, r.stdout[-2000:] + r.stderr[-2000:]
    assert "failed" in r.stdout
