"""GPU parity of the HIP path against the FP64 oracle (needs an MI355X).

Element-wise comparisons on seeded inputs small enough for the oracle, and,
at the full 2048 x 1024 / 16.8M-particle workload, sampled outputs that the
oracle computes one by one plus properties that hold at any size.
Tolerance (FP64 path): relative L2 of the stacked scattered fields <= 1e-12
after 50 steps; particle positions and momenta to 1e-12 (absolute, cell-size
and unit-momentum scale), matched by particle id.
"""
import math
import sys

import numpy as np
import pytest

from paper_2310_11393_amd import workloads as wl

from parity_util import (explicit_species, field_rel_l2, make_gpu,
                         make_oracle, particle_errors)

pytestmark = pytest.mark.gpu

FP64_FIELD_TOL = 1e-12


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gauss_tol(g, d, grid, rel_eps):
    """Attainable Gauss-law residual.  In exact arithmetic the Esirkepov
    current keeps div_h E - (rho - rho_0) at zero for ever; in floating
    point every step adds the rounding of the Ampere update and of the
    deposited current, a few units of rel_eps * max|E| per node, which the
    discrete divergence divides by the cell size.  The bound therefore grows
    linearly with the number of steps taken (plus a relative part of the
    charge density)."""
    emax = max(np.max(np.abs(g.read_field(c))) for c in ("ex", "ey"))
    steps = max(1, int(d["step"]))
    return max(1e-12 * d["rho_max"],
               8 * steps * rel_eps * emax * (1 / grid.dx + 1 / grid.dy))


def _small_lp(kind=wl.INC_APRIL_LP, **kw):
    args = dict(nx=136, ny=72, plasma=(40, 100, 0, 72), ppc=4, kind=kind,
                w0_lambda=1.0, s=20.0, a0=10.0, temperature_ev=1.0, steps=50,
                seed=11)
    args.update(kw)
    return wl.april_2d(**args)


CASES = {
    "pulse1d_small": lambda: wl.plane_pulse_1d(nx=300, slab=(100, 230),
                                               ppc=16, a0=3.0, steps=50),
    "pulse1d_2048": lambda: wl.plane_pulse_1d(steps=50),
    "lp2d_small": lambda: _small_lp(),
    "rp2d_small": lambda: _small_lp(kind=wl.INC_APRIL_RP, w0_lambda=0.8,
                                    s=10.0, a0=30.0, temperature_ev=0.0),
    "lp2d_ragged": lambda: _small_lp(nx=101, ny=77, plasma=(30, 81, 3, 70),
                                     ppc=3, s=10.0),
    "gauss2d_small": lambda: wl.gauss_beam_2d(
        nx=160, ny=96, plasma=(50, 110, 20, 76), ppc=4, w0_lambda=2.0,
        cycles=3.0, a0=3.0, steps=50, cells_per_lambda=24),
}


@pytest.mark.parametrize("case", list(CASES))
def test_fp64_parity_50_steps(case):
    work = CASES[case]()
    _note(f"[parity] {case}: grid {work.grid.nx}x{work.grid.ny}, "
          f"{work.species[0].count()} particles, {work.steps} steps")
    sp = explicit_species(work)
    g = make_gpu(work, sp)
    o = make_oracle(work, sp)
    g.step(work.steps)
    o.step(work.steps)
    rel, den = field_rel_l2(g, o)
    assert den > 0, "no scattered field was generated"
    assert rel <= FP64_FIELD_TOL, rel
    jrel, _ = field_rel_l2(g, o, comps=("jx", "jy", "jz"))
    assert jrel <= FP64_FIELD_TOL, jrel
    dpos, du, umax = particle_errors(g, o)
    assert dpos <= 1e-12 and du <= 1e-12 * max(1.0, umax), (dpos, du)
    gd = g.diagnostics()
    od = o.diagnostics()
    assert gd["n_alive"] == od["n_alive"]
    assert abs(gd["w_kin"] - od["w_kin"]) <= 1e-11 * abs(od["w_kin"])
    assert abs(gd["w_em"] - od["w_em"]) <= 1e-11 * abs(od["w_em"])
    assert abs(gd["w_em_total"] - od["w_em_total"]) <= \
        1e-11 * abs(od["w_em_total"])
    assert gd["gauss_residual"] <= gauss_tol(g, gd, work.grid, 2.2e-16)
    assert gd["nonfinite"] == 0


@pytest.mark.parametrize("tile,sort_every", [((4, 4), 7), ((32, 4), 1),
                                              ((16, 8), 25)])
def test_fp64_parity_tiling(tile, sort_every):
    """Tile shape and sort cadence change only the summation order: tiny
    tiles sorted rarely push most particles through the straggler path."""
    work = _small_lp(a0=30.0, s=10.0)
    sp = explicit_species(work)
    g = make_gpu(work, sp, tile=tile, sort_every=sort_every)
    o = make_oracle(work, sp)
    g.step(work.steps)
    o.step(work.steps)
    rel, den = field_rel_l2(g, o)
    assert den > 0 and rel <= FP64_FIELD_TOL, rel
    dpos, du, umax = particle_errors(g, o)
    assert dpos <= 1e-12 and du <= 1e-12 * max(1.0, umax), (dpos, du)


FP32_FIELD_TOL = 1e-4


@pytest.mark.parametrize("case", ["pulse1d_small", "lp2d_small", "rp2d_small",
                                  "lp2d_ragged", "gauss2d_small"])
def test_fp32_form_against_fp64_oracle(case):
    """FP32 form (integer cell + float offset, float fields and momenta,
    FP64 incident-field phase and current accumulation) vs the FP64 oracle:
    relative L2 of the fields <= 1e-4 after 50 steps."""
    work = CASES[case]()
    sp = explicit_species(work)
    g = make_gpu(work, sp, precision=wl.FP32)
    o = make_oracle(work, sp)
    g.step(work.steps)
    o.step(work.steps)
    rel, den = field_rel_l2(g, o)
    _note(f"[fp32] {case}: field relative L2 {rel:.3e}")
    assert den > 0 and rel <= FP32_FIELD_TOL, rel
    dpos, du, umax = particle_errors(g, o)
    _note(f"[fp32] {case}: max |dx| {dpos:.2e}, max |du| {du:.2e} (|u| {umax:.2e})")
    # FP32 momentum rounding grows with |u| and moves the positions by the
    # same factor over the run: both bounds scale with max(1, |u|max)
    assert dpos <= 1e-5 * max(1.0, umax) and du <= 1e-4 * max(1.0, umax), \
        (dpos, du)
    gd = g.diagnostics()
    assert gd["nonfinite"] == 0
    # |dW| <= |F_inc + F_s| |dF_s|, so the field tolerance bounds the total
    # energy's relative error by twice itself
    od = o.diagnostics()
    assert abs(gd["w_em_total"] - od["w_em_total"]) <= \
        2 * FP32_FIELD_TOL * od["w_em_total"]
    assert gd["gauss_residual"] <= max(1e-5 * gd["rho_max"],
                                       gauss_tol(g, gd, work.grid, 1.2e-7))


def test_fp32_tiling_and_checkpoint():
    work = _small_lp(a0=30.0, s=10.0)
    sp = explicit_species(work)
    g = make_gpu(work, sp, precision=wl.FP32, tile=(4, 4), sort_every=7)
    o = make_oracle(work, sp)
    g.step(20)
    st = g.get_state()
    g.step(30)
    o.step(50)
    rel, _ = field_rel_l2(g, o)
    assert rel <= FP32_FIELD_TOL, rel
    a = g.read_field("ey")
    g.set_state(st)
    g.step(30)
    b = g.read_field("ey")
    assert np.max(np.abs(a - b)) <= 1e-5 * np.max(np.abs(a))


def test_fp64_two_species_parity():
    work = _small_lp(nx=80, ny=48, plasma=(20, 60, 4, 44), ppc=3)
    e = explicit_species(work)[0]
    ion = dict(q=1.0, m=1836.0, weight=e["weight"], x=e["x"][::-1].copy(),
               y=e["y"][::-1].copy(), ux=-e["ux"], uy=-e["uy"], uz=-e["uz"])
    g = make_gpu(work, [e, ion])
    o = make_oracle(work, [e, ion])
    g.step(40)
    o.step(40)
    rel, _ = field_rel_l2(g, o)
    assert rel <= FP64_FIELD_TOL
    for sp in (0, 1):
        dpos, du, umax = particle_errors(g, o, sp)
        assert dpos <= 1e-12 and du <= 1e-12 * max(1.0, umax)


def test_empty_and_vacuum_sims():
    """No species: the scattered field stays exactly zero (Sec. 2 split) and
    the total-field energy is the incident field's, as in the oracle."""
    work = _small_lp()
    g = make_gpu(work, [])
    g.step(20)
    for c in ("ex", "ey", "ez", "bx", "by", "bz", "jx", "jy", "jz"):
        assert not np.any(g.read_field(c))
    o = make_oracle(work, [])
    o.step(20)
    wt = o.diagnostics()["w_em_total"]
    assert wt > 0 and abs(g.diagnostics()["w_em_total"] - wt) <= 1e-12 * wt
    # zero-weight particles move but carry no current
    sp = explicit_species(work)
    sp[0]["weight"] = 0.0
    g = make_gpu(work, sp)
    g.step(20)
    for c in ("ex", "ey", "ez", "bx", "by", "bz", "jx", "jy", "jz"):
        assert not np.any(g.read_field(c))
    uy, ids = g.particles()[3], g.particles()[5]
    assert np.max(np.abs(uy - sp[0]["uy"][ids.astype(np.int64)])) > 1e-3


@pytest.mark.parametrize("dims", [1, 2])
def test_yee_eigenmode_parity(dims):
    """Vacuum field evolution from a written initial field equals the
    oracle's (exercises the Mur faces and corners)."""
    if dims == 1:
        grid = wl.Grid(1, 200, 1, 0.2, 0.2, 0.19)
    else:
        grid = wl.Grid(2, 90, 70, 0.2, 0.25, 0.12)
    work = wl.Workload("vac", grid, [], wl.Incident(), 60)
    g = make_gpu(work, [])
    o = make_oracle(work, [])
    rng = np.random.default_rng(4)
    for c in ("ex", "ey", "ez", "bx", "by", "bz"):
        a = rng.normal(size=(o.NY, o.NX))
        if dims == 1 and c == "bx":
            a[:] = 0.0
        o.field(c)[:, :] = a
        g.write_field(c, a)
    g.step(60)
    o.step(60)
    rel, _ = field_rel_l2(g, o)
    assert rel <= 1e-13


def test_checkpoint_roundtrip():
    work = _small_lp(ppc=2)
    g = make_gpu(work)
    g.step(10)
    st = g.get_state()
    g.step(15)
    a = {c: g.read_field(c) for c in ("ex", "ey", "bz")}
    pa = g.particles()
    g.set_state(st)
    assert g.diagnostics()["step"] == 10
    g.step(15)
    for c, v in a.items():
        b = g.read_field(c)
        assert np.max(np.abs(b - v)) <= 1e-12 * max(1.0, np.max(np.abs(v)))
    pb = g.particles()
    assert np.array_equal(np.sort(pa[5]), np.sort(pb[5]))


@pytest.mark.parametrize("plane", [0, 1, 2])
def test_histogram_parity(plane):
    """The energy-angle histogram (polar angle, or the angle in the x-z or
    x-y plane) against the oracle's after 50 steps."""
    work = _small_lp(a0=20.0)
    sp = explicit_species(work)
    g = make_gpu(work, sp)
    o = make_oracle(work, sp)
    g.step(50)
    o.step(50)
    hg, mg = g.histogram(n_e=64, emax=2.0, n_theta=36, plane=plane)
    ho, mo = o.energy_angle(n_e=64, emax=2.0, n_theta=36, plane=plane)
    assert abs(hg.sum() - ho.sum()) <= 1e-12 * ho.sum()
    big = ho > 0.01 * ho.sum()
    assert np.all(np.abs(hg[big] - ho[big]) <= 0.01 * ho[big])
    assert np.allclose(mg, mo, rtol=1e-9, atol=0)


RUN_CASES = {
    # the whole 5-cycle pulse crosses the slab
    "pulse1d_run": lambda: wl.plane_pulse_1d(nx=300, slab=(100, 230), ppc=16,
                                             a0=3.0, steps=500),
    # the beam focuses in the plasma and leaves it (it expels many electrons
    # through the y faces of this narrow box; thousands remain)
    "lp2d_run": lambda: _small_lp(nx=200, ny=96, plasma=(40, 120, 0, 96),
                                  ppc=3, a0=5.0, s=10.0, steps=300),
    "rp2d_run": lambda: _small_lp(nx=200, ny=128, plasma=(40, 120, 0, 128),
                                  ppc=6, kind=wl.INC_APRIL_RP,
                                  w0_lambda=0.8, a0=10.0, s=10.0,
                                  temperature_ev=0.0, steps=300),
}


@pytest.mark.parametrize("prec", [wl.FP64, wl.FP32])
@pytest.mark.parametrize("case", list(RUN_CASES))
def test_end_of_run_spectra(case, prec):
    """Electron energy-angle spectra and their moments at the end of a run
    (the pulse has crossed the plasma) against the oracle: <E_k>, <E_k^2>,
    <theta>, <theta^2> and the kinetic energy within 1%, and every bin
    holding at least 1% of the weight within 1% plus two macro-particles
    (a particle's weight is the histogram's quantum, and rounding can move a
    particle that sits on a bin edge into the neighbouring bin)."""
    work = RUN_CASES[case]()
    _note(f"[spectra] {case} prec {prec}: {work.steps} steps")
    sp = explicit_species(work)
    g = make_gpu(work, sp, precision=prec)
    o = make_oracle(work, sp)
    g.step(work.steps)
    o.step(work.steps)
    # energy range: four times the oracle's mean kinetic energy
    _, m0 = o.energy_angle(n_e=1, emax=1.0, n_theta=1, ek_min=0.0)
    emax = 4.0 * m0[1]
    hg, mg = g.histogram(n_e=64, emax=emax, n_theta=36, ek_min=0.0)
    ho, mo = o.energy_angle(n_e=64, emax=emax, n_theta=36, ek_min=0.0)
    gd, od = g.diagnostics(), o.diagnostics()
    _note(f"[spectra] {case}: W_kin gpu {gd['w_kin']:.6e} oracle "
          f"{od['w_kin']:.6e}; moments gpu {mg[1:]} oracle {mo[1:]}")
    assert od["w_kin"] > 0 and od["n_alive"] >= 300
    # one macro-particle's histogram weight: the histogram's quantum
    w1 = work.species[0].weight * (work.grid.dx * work.grid.dy
                                   if work.grid.dims == 2 else work.grid.dx)
    assert abs(hg.sum() - ho.sum()) <= 1e-6 * ho.sum() + 2 * w1
    big = ho > 0.01 * ho.sum()
    assert big.any()
    err = np.abs(hg[big] - ho[big])
    tol = 0.01 * ho[big] + 2 * w1
    w = int(np.argmax(err / tol))
    _note(f"[spectra] {case}: {int(big.sum())} bins >= 1% of the weight "
          f"({ho.sum() / w1:.0f} particles), worst bin {np.argwhere(big)[w]}: "
          f"oracle {ho[big][w] / w1:.1f} gpu {hg[big][w] / w1:.1f} particles")
    assert np.all(err <= tol)
    for k in range(1, 5):
        assert abs(mg[k] - mo[k]) <= 0.01 * abs(mo[k]), (k, mg[k], mo[k])
    assert abs(gd["w_kin"] - od["w_kin"]) <= 0.01 * od["w_kin"]
    assert abs(gd["w_em_total"] - od["w_em_total"]) <= 0.01 * od["w_em_total"]


def test_invalid_inputs_are_rejected():
    from paper_2310_11393_amd.binding import SfpicError
    work = _small_lp()
    sp = explicit_species(work)
    sp[0]["ux"] = sp[0]["ux"].copy()
    sp[0]["ux"][5] = np.nan
    with pytest.raises(SfpicError) as e:
        make_gpu(work, sp)
    assert e.value.code == -5
    sp = explicit_species(work)
    sp[0]["x"] = sp[0]["x"].copy()
    sp[0]["x"][0] = -1.0
    with pytest.raises(SfpicError) as e:
        make_gpu(work, sp)
    assert e.value.code == -1
    with pytest.raises(SfpicError) as e:
        make_gpu(work, explicit_species(work), item_particles=32)
    assert e.value.code == -1


@pytest.mark.parametrize("prec", [wl.FP64, wl.FP32])
@pytest.mark.parametrize("case", ["pulse1d_small", "lp2d_small", "rp2d_small",
                                  "lp2d_ragged"])
def test_incident_on_nodes_parity(case, prec):
    """Incident field sampled on the Yee nodes at t^n and gathered with the
    scattered field (sfpic_incident.on_nodes = 1) against the oracle in the
    same mode: FP64 <= 1e-12 relative L2 of the fields after 50 steps,
    particles <= 1e-12; FP32 form <= 1e-4."""
    work = CASES[case]()
    work.incident.on_nodes = 1
    sp = explicit_species(work)
    g = make_gpu(work, sp, precision=prec)
    o = make_oracle(work, sp)
    g.step(work.steps)
    o.step(work.steps)
    tol = FP64_FIELD_TOL if prec == wl.FP64 else FP32_FIELD_TOL
    rel, den = field_rel_l2(g, o)
    _note(f"[on_nodes] {case} prec {prec}: field relative L2 {rel:.3e}")
    assert den > 0 and rel <= tol, rel
    jrel, _ = field_rel_l2(g, o, comps=("jx", "jy", "jz"))
    assert jrel <= tol, jrel
    dpos, du, umax = particle_errors(g, o)
    ptol = 1e-12 if prec == wl.FP64 else 1e-5
    assert dpos <= ptol and du <= 10 * ptol * max(1.0, umax), (dpos, du)
    gd, od = g.diagnostics(), o.diagnostics()
    assert gd["n_alive"] == od["n_alive"]
    if prec == wl.FP64:
        assert abs(gd["w_kin"] - od["w_kin"]) <= 1e-11 * abs(od["w_kin"])
    # the two modes differ by the O(dx^2) sampling error, not by nothing
    work.incident.on_nodes = 0
    o0 = make_oracle(work, sp)
    o0.step(work.steps)
    d0, _ = field_rel_l2(g, o0)
    assert d0 > 10 * tol


@pytest.mark.parametrize("item,prec", [(64, wl.FP64), (200, wl.FP64),
                                       (100, wl.FP32)])
def test_parity_with_split_tiles(item, prec):
    """Tiles holding more than `item` particles are pushed by several
    workgroups (work items), each adding its own current window to the grid:
    only the summation order changes.  With 8 ppc every 16x16 tile holds
    2048 particles, so every tile is split (and the ragged last item of a
    tile is short)."""
    work = _small_lp(ppc=8, a0=30.0, s=10.0)
    sp = explicit_species(work)
    g = make_gpu(work, sp, precision=prec, item_particles=item)
    o = make_oracle(work, sp)
    g.step(work.steps)
    o.step(work.steps)
    tol = FP64_FIELD_TOL if prec == wl.FP64 else FP32_FIELD_TOL
    rel, den = field_rel_l2(g, o)
    _note(f"[items] item {item} prec {prec}: field relative L2 {rel:.3e}")
    assert den > 0 and rel <= tol, rel
    jrel, _ = field_rel_l2(g, o, comps=("jx", "jy", "jz"))
    assert jrel <= tol, jrel
    dpos, du, umax = particle_errors(g, o)
    ptol = 1e-12 if prec == wl.FP64 else 1e-5
    assert dpos <= ptol and du <= 10 * ptol * max(1.0, umax), (dpos, du)
    assert g.diagnostics()["n_alive"] == o.diagnostics()["n_alive"]


# ---------------------------------------------------------------------------
# Full-size 2048 x 1024, 16.8M particles (the benchmark workload)
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def full_lp():
    from paper_2310_11393_amd.binding import Simulation
    work = wl.lp_2048x1024()
    _note("[parity] full-size LP 2048x1024: creating 16.8M particles")
    sim = Simulation.from_workload(work)
    return work, sim


def test_full_size_device_generator_matches_inputs(full_lp):
    work, sim = full_lp
    x, y, ux, uy, uz, ids = sim.particles()
    sp = work.species[0]
    assert len(x) == sp.count() == 16777216
    rng = np.random.default_rng(7)
    pick = np.sort(rng.choice(len(x), 4096, replace=False))
    order = np.argsort(ids)
    hx, hy, hux, huy, huz = wl.generate_particles(sp, work.grid)
    sel = order[pick]
    assert np.array_equal(ids[sel], pick.astype(np.uint32))
    assert np.array_equal(x[sel], hx[pick]) and np.array_equal(y[sel], hy[pick])
    for a, b in ((ux, hux), (uy, huy), (uz, huz)):
        assert np.allclose(a[sel], b[pick], rtol=1e-14, atol=1e-20)


def test_full_size_first_step_window(full_lp):
    """After one step from rest fields, every particle moved in the incident
    field alone: sampled particles and the current in a window of cells are
    reproduced by the oracle from the particles near that window."""
    work, sim = full_lp
    sim.step(1)
    sp = work.species[0]
    x0, x1, y0, y1 = sp.region
    ncx = x1 - x0
    # window of cells at the plasma front, centred on the beam axis
    wx0, wx1, wy0, wy1 = x0, x0 + 24, 512 - 12, 512 + 12
    ids = []
    for cy in range(wy0 - 3, wy1 + 3):
        c0 = (cy - y0) * ncx + (wx0 - 3 - x0) if wx0 - 3 >= x0 else \
            (cy - y0) * ncx
        c1 = (cy - y0) * ncx + (wx1 + 3 - x0)
        ids.append(np.arange(c0 * sp.ppc, c1 * sp.ppc))
    ids = np.concatenate(ids)
    cols = wl.generate_particles(sp, work.grid)
    e = dict(q=sp.q, m=sp.m, weight=sp.weight,
             **{k: v[ids] for k, v in zip(("x", "y", "ux", "uy", "uz"), cols)})
    o = make_oracle(work, [e])
    o.step(1)
    G = 3
    # The current of one step is q w (dx/dt) times a shape difference taken
    # between x^n and x^{n+1}; both sides form those positions in their own
    # arithmetic (cell units here, physical units in the oracle), so each
    # particle's contribution carries an absolute error of a few ulp of the
    # position in cells.  At t = 0 the window current is thermal (J ~ 1e-5)
    # and that bound, not 1e-12 relative, is the attainable agreement.
    qw = abs(sp.q * sp.weight)
    atol_j = 16 * np.spacing(float(wx1 + 3)) * qw * work.grid.dx / work.grid.dt
    for c in ("jx", "jy", "jz", "ex", "ey"):
        gv = sim.read_field(c)[G + wy0 + 2:G + wy1 - 2, G + wx0 + 2:G + wx1 - 2]
        ov = o.field(c)[G + wy0 + 2:G + wy1 - 2, G + wx0 + 2:G + wx1 - 2]
        scale = max(np.max(np.abs(ov)), 1e-300)
        atol = atol_j * (work.grid.dt if c[0] == "e" else 1.0)
        assert np.max(np.abs(gv - ov)) <= 1e-12 * scale + atol, c
        assert np.max(np.abs(ov)) > 0, c
    gx, gy, gux, guy, guz, gid = sim.particles()
    pos = np.full(sp.count(), -1, dtype=np.int64)
    pos[gid.astype(np.int64)] = np.arange(len(gid))
    ox, oy, oux, ouy, ouz, alive = o.particles()
    k = pos[ids]
    assert (k >= 0).all()
    assert np.max(np.abs(gx[k] - ox)) <= 1e-12
    assert np.max(np.abs(gy[k] - oy)) <= 1e-12
    assert np.max(np.abs(guy[k] - ouy)) <= 1e-12 * max(1.0, np.max(np.abs(ouy)))


def test_full_size_fp32_rp_4096(full_lp):
    """The 4096^2 FP32-form workload (134M particles, RP beam): the device
    generator matches the inputs on sampled ids, a few steps keep Gauss's law
    at FP32 level, and nothing becomes non-finite."""
    from paper_2310_11393_amd.binding import Simulation
    work = wl.rp_4096_fp32()
    _note("[parity] full-size RP 4096^2 FP32: creating 134M particles")
    sim = Simulation.from_workload(work)
    sp = work.species[0]
    assert sim.particle_count() == sp.count() == 134217728
    sim.step(10)
    d = sim.diagnostics()
    _note(f"[parity] 4096^2 FP32 after 10 steps: {d}")
    assert d["nonfinite"] == 0 and d["rho_max"] > 0
    assert d["gauss_residual"] <= max(1e-5 * d["rho_max"],
                                      gauss_tol(sim, d, work.grid, 1.2e-7))
    sim.close()


def test_full_size_gauss_law_after_steps(full_lp):
    work, sim = full_lp
    sim.step(20)
    d = sim.diagnostics()
    assert d["nonfinite"] == 0
    assert d["rho_max"] > 0
    assert d["gauss_residual"] <= gauss_tol(sim, d, work.grid, 2.2e-16)
    assert d["n_alive"] <= 16777216
