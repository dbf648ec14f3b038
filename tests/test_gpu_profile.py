"""Device placement with the Sec. 3.1 density profile (GPU): the 2D
generator reproduces workloads.generate_particles bit for bit (FP64
positions; FP32 cells and offsets), and the 3D generator puts each
particle in the column and row the profile's column offsets assign.  A
short FP64 run with profile particles matches the oracle."""
import math

import numpy as np
import pytest

from paper_2310_11393_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _profiled(work_sp, center, fwhm, xmin, order=12.0):
    work_sp.profile = wl.PROFILE_SUPERGAUSS
    work_sp.profile_center = center
    work_sp.profile_fwhm = fwhm
    work_sp.profile_order = order
    work_sp.profile_xmin = xmin
    return work_sp


def test_2d_generator_with_profile_matches_inputs():
    from paper_2310_11393_amd.binding import Simulation
    g = wl.Grid(dims=2, nx=512, ny=96, dx=2 * math.pi / 32,
                dy=2 * math.pi / 32, dt=0.1)
    sp = wl.Species(q=-1.0, m=1.0, density=0.1, region=(16, 500, 8, 88),
                    ppc=12, temperature_ev=500.0, seed=21)
    _profiled(sp, center=60.0, fwhm=70.0, xmin=8.0)
    n = sp.count(g.dx)
    hx, hy, hux, huy, huz = wl.generate_particles(sp, g)
    assert len(hx) == n > 100000
    for prec in (wl.FP64, wl.FP32):
        print(f"[profile] 2D precision {prec}: {n} particles", flush=True)
        sim = Simulation(g, wl.Incident(), species=[sp], precision=prec)
        x, y, ux, uy, uz, ids = sim.particles()
        assert len(x) == n
        order = np.argsort(ids)
        assert np.array_equal(ids[order], np.arange(n, dtype=np.uint32))
        if prec == wl.FP64:
            assert np.array_equal(x[order], hx) and np.array_equal(y[order], hy)
            tol = 1e-14
        else:  # integer cell + float offset: cells exact, offsets to FP32
            assert np.array_equal(np.floor(x[order] / g.dx),
                                  np.floor(hx / g.dx))
            assert np.max(np.abs(x[order] - hx)) <= 1.2e-7 * g.dx
            tol = 1e-6
        for a, b in ((ux, hux), (uy, huy), (uz, huz)):
            assert np.allclose(a[order], b, rtol=tol, atol=1e-20)
        sim.close()


def test_3d_generator_with_profile_places_columns():
    from paper_2310_11393_amd.binding import Simulation3
    g = wl.grid3(96, 24, 20)
    sp = wl.Species3(q=-1.0, m=1.0, density=0.31, region=(10, 96, 2, 22, 3, 18),
                     ppc=6, seed=5)
    _profiled(sp, center=30.0, fwhm=30.0, xmin=5.0)
    off = wl.profile_offsets(sp, 10, 96, g.dx)
    per_row = int(off[-1])
    n = sp.count(g.dx)
    sim = Simulation3(g, wl.Incident(), species=[sp])
    x, y, z, ux, uy, uz, alive = sim.particles(0)
    assert len(x) == n == per_row * 20 * 15 and alive.all()
    i = np.arange(n)
    row = i // per_row
    col = 10 + np.searchsorted(off, i - row * per_row, side="right") - 1
    assert np.array_equal(np.floor(x / g.dx).astype(int), col)
    assert np.array_equal(np.floor(y / g.dy).astype(int), 2 + row % 20)
    assert np.array_equal(np.floor(z / g.dz).astype(int), 3 + row // 20)
    d = sim.diagnostics()
    q = -0.31 / sp.ppc * n * g.dx * g.dy * g.dz
    assert abs(d["charge"] - q) <= 1e-12 * abs(q)


def test_2d_profile_particles_parity():
    """A 30-step FP64 run from profile particles (explicit, the same arrays on
    both sides) matches the oracle to 1e-12."""
    from oracle import OracleSim
    from paper_2310_11393_amd.binding import Simulation
    g = wl.Grid(dims=2, nx=96, ny=40, dx=2 * math.pi / 32,
                dy=2 * math.pi / 32, dt=0.12)
    sp = wl.Species(q=-1.0, m=1.0, density=0.2, region=(8, 88, 6, 34), ppc=6,
                    temperature_ev=20.0, seed=4)
    _profiled(sp, center=9.0, fwhm=10.0, xmin=1.0)
    inc = wl.Incident(kind=wl.INC_PLANE_PULSE_1D, a0=1.5, fwhm_t=6.0, t0=-2.0)
    x, y, ux, uy, uz = wl.generate_particles(sp, g)
    e = dict(q=sp.q, m=sp.m, weight=sp.weight, x=x, y=y, ux=ux, uy=uy, uz=uz)
    o = OracleSim(g, inc)
    o.add_species(e["q"], e["m"], e["weight"], x, y, ux, uy, uz)
    s = Simulation(g, inc, explicit=[e], precision=wl.FP64)
    o.step(30)
    s.step(30)
    num = den = 0.0
    for c in ("ex", "ey", "ez", "bx", "by", "bz"):
        a, b = s.read_field(c), o.field(c)
        num += float(np.sum((a - b) ** 2))
        den += float(np.sum(b ** 2))
    assert den > 0 and (num / den) ** 0.5 <= 1e-12
