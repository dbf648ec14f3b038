"""Pins of the 3D3V oracle against facts fixed by the mathematics.

Each test checks a property that a plausible mistake in one operator breaks:
  * Gauss's law from charge conservation (Esirkepov 2001): with E = 0 at the
    start, div_h E = rho - rho_0 at every interior node after any number of
    steps -- a wrong weight (1/2, 1/3), index, prefix direction or sign in the
    3D current, or a wrong curl_h B in Ampere, breaks it;
  * an oblique plane wave against the exact dispersion of the discrete Yee
    scheme, sin(w dt/2)/dt = |k~| with k~_a = 2 sin(k_a h_a/2)/h_a, in the
    part of the box the faces cannot reach yet -- every curl term, sign and
    staggering of Faraday and Ampere enters;
  * order-2 B-spline gather reproduces linear fields exactly on every
    component's staggering;
  * the 3D incident field is a vacuum Maxwell solution (finite differences in
    all three directions) and equals the pinned 2D slice at z = z_focus;
  * first-order Mur absorbs a pulse at normal incidence on each face;
  * a free particle streams on a straight line and is removed when it leaves.
"""
import math
from types import SimpleNamespace as NS

import numpy as np
import pytest

from oracle import oracle as O

G = O.GUARD
NOINC = NS(kind=0, a0=0.0)


def grid3(nx, ny, nz, h=(0.3, 0.25, 0.35), cfl=0.5):
    dt = cfl / math.sqrt(sum(1.0 / a ** 2 for a in h))
    return NS(nx=nx, ny=ny, nz=nz, dx=h[0], dy=h[1], dz=h[2], dt=dt)


def div_e(sim, g):
    ex, ey, ez = sim.field("ex"), sim.field("ey"), sim.field("ez")
    d = np.zeros_like(ex)
    d[1:, 1:, 1:] = ((ex[1:, 1:, 1:] - ex[1:, 1:, :-1]) / g.dx +
                     (ey[1:, 1:, 1:] - ey[1:, :-1, 1:]) / g.dy +
                     (ez[1:, 1:, 1:] - ez[:-1, 1:, 1:]) / g.dz)
    return d


def test_gauss_law_from_charge_conservation():
    g = grid3(14, 12, 11)
    rng = np.random.default_rng(7)
    n = 400
    x = rng.uniform(3, 11, n) * g.dx
    y = rng.uniform(3, 9, n) * g.dy
    z = rng.uniform(3, 8, n) * g.dz
    u = rng.normal(0, 1.5, (3, n))  # relativistic, several cells per step
    sim = O.OracleSim3(g, NOINC)
    sim.add_species(-1.0, 1.0, 0.05, x, y, z, *u)
    sim.add_species(2.0, 3.0, 0.02, x[::2], z[::2] * g.dy / g.dz,
                    y[::2] * g.dz / g.dy, *(0.5 * u[:, ::2]))
    rho0 = sim.rho()
    sim.step(12)
    assert sim.diagnostics()["n_alive"] < 600  # some left the box
    res = div_e(sim, g) - (sim.rho() - rho0)
    s = (slice(G + 4, -G - 4),) * 3
    scale = np.abs(sim.rho() - rho0)[s].max()
    assert scale > 1e-2
    assert np.abs(res[s]).max() < 1e-12 * max(1.0, scale)


@pytest.mark.parametrize("kvec", [(1.1, -0.7, 0.5), (0.3, 1.4, -1.2)])
def test_plane_wave_discrete_dispersion(kvec):
    g = grid3(26, 24, 22)
    h = np.array([g.dx, g.dy, g.dz])
    k = np.array(kvec)
    kt = 2.0 * np.sin(k * h / 2.0) / h
    # E0 perpendicular to k~, B0 = k~ x E0 / w~
    a = np.cross(kt, [0.3, -0.5, 0.8])
    e0 = a / np.linalg.norm(a)
    wt = np.linalg.norm(kt)
    b0 = np.cross(kt, e0) / wt
    w = 2.0 / g.dt * math.asin(g.dt * wt / 2.0)
    stag = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (0, 1, 1), (1, 0, 1), (1, 1, 0)]
    sim = O.OracleSim3(g, NOINC)
    nz, ny, nx = sim.shape
    idx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                      indexing="ij")

    def mode(c, t):
        pos = [(idx[2 - d] - G + 0.5 * stag[c][d]) * h[d] for d in range(3)]
        amp = e0[c] if c < 3 else b0[c - 3]
        return amp * np.cos(k[0] * pos[0] + k[1] * pos[1] + k[2] * pos[2]
                            - w * t)

    names = ["ex", "ey", "ez", "bx", "by", "bz"]
    for c in range(6):
        sim.field(names[c])[...] = mode(c, 0.0 if c < 3 else -0.5 * g.dt)
    nst = 6
    sim.step(nst)
    s = (slice(nst + 2, -nst - 2),) * 3
    for c in range(6):
        want = mode(c, nst * g.dt if c < 3 else (nst - 0.5) * g.dt)
        err = np.abs(sim.field(names[c])[s] - want[s]).max()
        assert err < 1e-12, (names[c], err)
    # the same run with the continuum frequency is visibly wrong: the pin
    # resolves the discrete dispersion
    w_cont = np.linalg.norm(k)
    assert abs(w_cont - w) * nst * g.dt > 1e-4


def test_gather_reproduces_linear_fields():
    g = grid3(9, 8, 7)
    sim = O.OracleSim3(g, NOINC)
    nz, ny, nx = sim.shape
    h = (g.dx, g.dy, g.dz)
    stag = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (0, 1, 1), (1, 0, 1), (1, 1, 0)]
    coef = np.random.default_rng(3).normal(size=(6, 4))
    kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                             indexing="ij")
    for c, name in enumerate(["ex", "ey", "ez", "bx", "by", "bz"]):
        px = (ii - G + 0.5 * stag[c][0]) * h[0]
        py = (jj - G + 0.5 * stag[c][1]) * h[1]
        pz = (kk - G + 0.5 * stag[c][2]) * h[2]
        sim.field(name)[...] = (coef[c, 0] + coef[c, 1] * px +
                                coef[c, 2] * py + coef[c, 3] * pz)
    rng = np.random.default_rng(4)
    for _ in range(20):
        p = rng.uniform(1, 6, 3) * np.array(h)
        E, B = sim.gather(*p)
        got = np.concatenate([E, B])
        want = coef[:, 0] + coef[:, 1:] @ p
        assert np.allclose(got, want, rtol=0, atol=1e-12)


@pytest.mark.parametrize("kind", [2, 3])
def test_incident_3d_is_a_vacuum_solution(kind):
    inc = NS(kind=kind, a0=4.0, w0=1.6, s=12.0, phi0=0.4, x_focus=0.3,
             y_focus=-0.2, z_focus=0.15, t_focus=0.5)
    h = 1e-4
    rng = np.random.default_rng(kind)
    for _ in range(6):
        x, y, z = rng.uniform(-2.5, 2.5, 3)
        t = rng.uniform(-2.0, 3.0)

        def F(dx=0.0, dy=0.0, dz=0.0, dtt=0.0):
            E, B = O.incident_eval3(inc, x + dx, y + dy, z + dz, t + dtt)
            return np.concatenate([E, B])

        d = [(F(dx=h) - F(dx=-h)) / (2 * h), (F(dy=h) - F(dy=-h)) / (2 * h),
             (F(dz=h) - F(dz=-h)) / (2 * h)]
        dt_ = (F(dtt=h) - F(dtt=-h)) / (2 * h)
        E = slice(0, 3)
        curl = lambda c: np.array([d[1][c + 2] - d[2][c + 1],  # noqa: E731
                                   d[2][c] - d[0][c + 2],
                                   d[0][c + 1] - d[1][c]])
        scale = np.abs(F()).max() + 1.0
        assert abs(d[0][0] + d[1][1] + d[2][2]) < 1e-6 * scale  # div E
        assert abs(d[0][3] + d[1][4] + d[2][5]) < 1e-6 * scale  # div B
        assert np.abs(curl(0) + dt_[3:]).max() < 1e-6 * scale   # Faraday
        assert np.abs(curl(3) - dt_[E]).max() < 1e-6 * scale    # Ampere
    # at z = z_focus the 3D field is the pinned 2D slice
    for _ in range(5):
        x, y = rng.uniform(-2, 2, 2)
        E3, B3 = O.incident_eval3(inc, x, y, inc.z_focus, 0.7)
        E2, B2 = O.incident_eval(inc, 2, x, y, 0.7)
        assert np.allclose(np.concatenate([E3, B3]), np.concatenate([E2, B2]),
                           rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_mur_absorbs_a_pulse_at_each_face(axis):
    # A carrier packet along `axis` with E the discrete curl of a potential
    # A_q e_q (so div_h E = 0 exactly: no static part can stay behind) and
    # B = 0: half of it runs to each face normal to `axis`.  With perfectly
    # conducting faces all of it would come back.
    h = 0.25
    n = [36, 36, 36]
    n[axis] = 56
    g = grid3(*n, h=(h, h, h), cfl=0.5)
    sim = O.OracleSim3(g, NOINC)
    shape = sim.shape  # (NZ, NY, NX): build axis d is array axis 2 - d
    p, q = (axis + 1) % 3, (axis + 2) % 3
    stag_b = [(0, 1, 1), (1, 0, 1), (1, 1, 0)]
    grids = np.meshgrid(*[np.arange(m) for m in shape], indexing="ij")
    arg = np.zeros(shape)
    sig = [5 * h] * 3
    sig[axis] = 3 * h
    carrier = None
    for d in range(3):
        L = shape[2 - d]
        pos = (grids[2 - d] - L / 2 + 0.5 * stag_b[q][d]) * h
        arg = arg + (pos / sig[d]) ** 2
        if d == axis:
            carrier = np.cos(2 * math.pi * pos / (6 * h))
    A = carrier * np.exp(-arg)

    def back_diff(a, d):
        out = np.zeros_like(a)
        ax = 2 - d
        hi = [slice(None)] * 3
        lo = [slice(None)] * 3
        hi[ax] = slice(1, None)
        lo[ax] = slice(0, -1)
        out[tuple(hi)] = (a[tuple(hi)] - a[tuple(lo)]) / h
        return out

    names_e = ["ex", "ey", "ez"]
    sim.field(names_e[p])[...] = -back_diff(A, axis)
    sim.field(names_e[axis])[...] = back_diff(A, p)
    w0 = sim.diagnostics()["w_em"]
    sim.step(int((n[axis] * h / 2 + 16 * sig[axis]) / g.dt))
    w1 = sim.diagnostics()["w_em"]
    assert w1 < 0.02 * w0, w1 / w0


def test_free_particle_streams_and_leaves():
    g = grid3(10, 9, 8)
    u = np.array([0.9, -0.4, 0.25])
    x0 = np.array([5.2 * g.dx, 4.1 * g.dy, 3.7 * g.dz])
    sim = O.OracleSim3(g, NOINC)
    sim.add_species(-1.0, 1.0, 1e-12, *[[v] for v in x0], *[[v] for v in u])
    gam = math.sqrt(1 + u @ u)
    nst = 5
    sim.step(nst)
    got = sim.particles()
    pos = np.array([got[0][0], got[1][0], got[2][0]])
    assert np.allclose(pos, x0 + nst * g.dt * u / gam, rtol=0, atol=1e-12)
    assert got[6][0]
    # it crosses x = nx dx after this many steps and is removed then
    t_out = (g.nx * g.dx - x0[0]) / (u[0] / gam)
    k_out = math.floor(t_out / g.dt) + 1
    sim.step(k_out - nst - 1)
    assert sim.particles()[6][0]
    sim.step(1)
    assert not sim.particles()[6][0]


@pytest.mark.parametrize("plane", [0, 1, 2])
def test_energy_angle_histogram_of_known_particles(plane):
    """Particles of known momentum land in the bins their kinetic energy
    m (gamma - 1) and angle from +x put them in, weighted by w dV: the polar
    angle (plane 0) or, in the x-z (1) or x-y (2) plane, the angle of the
    projected momentum."""
    g = grid3(8, 8, 8)
    u = np.array([[1.0, 0.0, 0.0],    # E_k = sqrt(2) - 1, theta = 0
                  [0.0, 0.5, 0.0],    # theta = 90
                  [-2.0, 0.0, 0.0],   # theta = 180 (last bin)
                  [0.3, 0.0, 0.4]])   # theta = atan2(0.4, 0.3)
    x = np.full(4, 4.2 * g.dx)
    sim = O.OracleSim3(g, NOINC)
    w = 0.25
    sim.add_species(-1.0, 1.0, w, x, x * g.dy / g.dx, x * g.dz / g.dx,
                    *u.T)
    n_e, emax, n_t = 40, 2.0, 36
    h, mom = sim.energy_angle(n_e=n_e, emax=emax, n_theta=n_t, ek_min=0.0,
                              plane=plane)
    dV = g.dx * g.dy * g.dz
    ek = np.sqrt(1.0 + (u ** 2).sum(1)) - 1.0
    perp = {0: np.hypot(u[:, 1], u[:, 2]), 1: np.abs(u[:, 2]),
            2: np.abs(u[:, 1])}[plane]
    th = np.degrees(np.arctan2(perp, u[:, 0]))
    want = np.zeros((n_e, n_t))
    for e, t in zip(ek, th):
        want[int(e / emax * n_e), min(int(t / 180 * n_t), n_t - 1)] += w * dV
    assert np.array_equal(h, want)
    assert math.isclose(mom[0], 4 * w * dV, rel_tol=1e-15)
    assert math.isclose(mom[1], ek.mean(), rel_tol=1e-14)
    assert math.isclose(mom[3], th.mean(), rel_tol=1e-14)


def test_total_field_energy_of_a_plane_pulse():
    """The 3D total-field energy of the plane pulse inside the box is its
    closed-form integral, a0^2 (1/2) sqrt(pi / alpha) (1 - exp(-1 / alpha))
    with alpha = 8 ln 2 / FWHM^2, times the cross-section ny dy nz dz, at
    step 0 and after steps (no particles: the scattered field stays zero)."""
    g = grid3(300, 3, 4, h=(0.2, 0.3, 0.25))
    inc = NS(kind=1, a0=0.9, fwhm_t=2 * math.pi, t0=-30.0)
    sim = O.OracleSim3(g, inc)
    alpha = 8.0 * math.log(2.0) / (2 * math.pi) ** 2
    want = 0.81 * 0.5 * math.sqrt(math.pi / alpha) * (
        1.0 - math.exp(-1.0 / alpha)) * (3 * 0.3) * (4 * 0.25)
    for steps in (0, 30):
        sim.step(steps)
        d = sim.diagnostics()
        assert d["w_em"] == 0.0
        assert abs(d["w_em_total"] - want) <= 1e-12 * want, \
            (steps, d["w_em_total"], want)
