"""GPU checks of the method's edge cases and of failure handling (needs an
MI355X):

  * the April ring u = 0 (r = a in the focal plane, Sec. 4.1), where the
    closed form is 0/0 and the device takes its Taylor series in u^2: the
    incident field on Yee nodes that sit on the ring, and 50-step parity with
    the oracle of a plasma that straddles the ring, LP and RP, FP64 (1e-12)
    and the FP32 form (1e-4, with its FP64 fallback near the ring);
  * the discrete continuity equation (the charge conservation of the
    deposition that Sec. 2 names) step by step on the device;
  * the Gauss-law reduction against a known injected divergence, including
    nodes in the last partial block, and a NaN that must show as +inf;
  * the default (adaptive) sort cadence of a single simulation: the longest
    interval for a cold plasma that makes no stragglers, the shortest for a
    hot one, whose run still matches the oracle;
  * a sweep member that goes non-finite fails alone with SFPIC_E_NUMERIC;
  * the per-handle error message of the C ABI.
"""
import ctypes as C
import math
import sys

import numpy as np
import pytest

from paper_2310_11393_amd import workloads as wl

from parity_util import (explicit_species, field_rel_l2, make_gpu,
                         make_oracle, particle_errors)

pytestmark = pytest.mark.gpu
G = 3
TWO_PI = 2.0 * math.pi


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# ---------------------------------------------------------------------------
# The April ring
# ---------------------------------------------------------------------------

RING_U2 = 0.0625   # both sides take the series when |u^2| < 1/16


def _ring_work(kind, nx=48, ny=96, ppc=8, cells_per_lambda=64, w0_lambda=0.3,
               a0=10.0, steps=50):
    """A tight beam (w0 = 0.3 lambda: a = 1.37 w0, so the ring lies where the
    field is still ~15% of its peak) focused inside a plasma that covers the
    whole focal plane of the box; the pulse peak crosses the focus at step
    25.  The ring points (x_f, y_f +- a) fall inside the box."""
    dx = TWO_PI / cells_per_lambda
    dt = 0.95 * dx / math.sqrt(2.0)
    grid = wl.Grid(2, nx, ny, dx, dx, dt)
    x_f, y_f = 0.5 * nx * dx, 0.5 * ny * dx
    inc = wl.Incident(kind=kind, a0=a0, w0=w0_lambda * TWO_PI, s=10.0,
                      x_focus=x_f, y_focus=y_f, t_focus=25 * dt)
    sp = wl.Species(q=-1.0, m=1.0, density=0.05, region=(8, nx - 8, 0, ny),
                    ppc=ppc, temperature_ev=1.0, seed=17)
    return wl.Workload("ring", grid, [sp], inc, steps)


def _ring_radius(inc):
    import oracle
    return oracle.oracle.ka_from_w0(inc.w0)


def _in_series_region(inc, x, y):
    a = _ring_radius(inc)
    X = (y - inc.y_focus) / a
    Z = (x - inc.x_focus) / a
    u2r, u2i = X * X + Z * Z - 1.0, 2.0 * Z
    return np.hypot(u2r, u2i) < RING_U2


def _ring_cluster(work, n_each=48, seed=5):
    """Extra cold electrons inside the series region around both ring points
    (a disc of radius 0.5 |u^2|-threshold in units of a)."""
    inc = work.incident
    a = _ring_radius(inc)
    rng = np.random.default_rng(seed)
    xs, ys = [], []
    for sgn in (1.0, -1.0):
        r = 0.5 * 0.5 * RING_U2 * a * np.sqrt(rng.uniform(0, 1, n_each))
        ph = rng.uniform(0, TWO_PI, n_each)
        xs.append(inc.x_focus + r * np.cos(ph))
        ys.append(inc.y_focus + sgn * a + r * np.sin(ph))
    x, y = np.concatenate(xs), np.concatenate(ys)
    z = np.zeros_like(x)
    return dict(q=-1.0, m=1.0, weight=work.species[0].weight, x=x, y=y,
                ux=z, uy=z.copy(), uz=z.copy())


@pytest.mark.parametrize("kind", [wl.INC_APRIL_LP, wl.INC_APRIL_RP])
def test_ring_incident_on_nodes(kind):
    """The total field of a vacuum sim is the incident field at each Yee
    node, evaluated on the device in FP64.  With the focus placed so that
    E_z nodes (and, half a cell away, the other staggerings) sit on the ring
    to rounding, the closed form would divide 0 by 0 there: the device must
    agree with the oracle's evaluation (its own series) at every node."""
    from oracle import oracle as O
    work = _ring_work(kind, nx=40, ny=80)
    inc = work.incident
    g = work.grid
    a = _ring_radius(inc)
    # node 56 of the primal y axis on the ring, x_f on primal node 20
    inc.x_focus = 20 * g.dx
    inc.y_focus = 56 * g.dy - a
    sim = make_gpu(work, [])
    stag = {"ex": (1, 0), "ey": (0, 1), "ez": (0, 0), "bx": (0, 1),
            "by": (1, 0), "bz": (1, 1)}
    for n in (20, 25):
        sim.set_step_index(n)
        worst, peak = 0.0, 0.0
        for ci, (c, (sx, sy)) in enumerate(stag.items()):
            got = sim.read_total_field(c)
            t = n * g.dt - (0.5 * g.dt if ci >= 3 else 0.0)
            X = (np.arange(got.shape[1]) - G + 0.5 * sx) * g.dx
            Y = (np.arange(got.shape[0]) - G + 0.5 * sy) * g.dy
            near = [(j, i) for j in range(got.shape[0])
                    for i in range(got.shape[1])
                    if abs(X[i] - inc.x_focus) < 3 * g.dx and
                    abs(abs(Y[j] - inc.y_focus) - a) < 3 * g.dy]
            assert near
            assert np.all(np.isfinite(got))
            for j, i in near:
                E, B = O.incident_eval(inc, 2, X[i], Y[j], t)
                want = (list(E) + list(B))[ci]
                worst = max(worst, abs(got[j, i] - want))
                peak = max(peak, abs(want))
            peak = max(peak, float(np.max(np.abs(got))))
        assert peak > 0.05 * inc.a0
        _note(f"[ring] kind {kind} step {n}: max |device - oracle| near the "
              f"ring {worst:.2e} (peak {peak:.2e})")
        assert worst <= 1e-12 * peak


@pytest.mark.parametrize("prec", [wl.FP64, wl.FP32])
@pytest.mark.parametrize("kind", [wl.INC_APRIL_LP, wl.INC_APRIL_RP])
def test_ring_parity_50_steps(kind, prec):
    """A plasma straddling the ring, plus a cluster of electrons inside the
    series region at each ring point: 50 steps against the oracle, FP64 to
    1e-12 and the FP32 form to 1e-4.  The oracle's own particle positions
    show how many particle-steps were taken inside the series region."""
    work = _ring_work(kind)
    sp = explicit_species(work)
    cl = _ring_cluster(work)
    for k in ("x", "y", "ux", "uy", "uz"):
        sp[0][k] = np.concatenate([sp[0][k], cl[k]])
    g = make_gpu(work, sp, precision=prec)
    o = make_oracle(work, sp)
    inside = 0
    for _ in range(work.steps):
        x, y, _ux, _uy, _uz, alive = o.particles()
        inside += int(np.count_nonzero(
            _in_series_region(work.incident, x[alive], y[alive])))
        o.step(1)
    g.step(work.steps)
    _note(f"[ring] kind {kind} prec {prec}: {inside} particle-steps in the "
          f"series region")
    assert inside >= 20 * work.steps
    rel, den = field_rel_l2(g, o)
    tol = 1e-12 if prec == wl.FP64 else 1e-4
    _note(f"[ring] kind {kind} prec {prec}: field relative L2 {rel:.3e}")
    assert den > 0 and rel <= tol, rel
    dpos, du, umax = particle_errors(g, o)
    if prec == wl.FP64:
        assert dpos <= 1e-12 and du <= 1e-12 * max(1.0, umax), (dpos, du)
    else:
        # FP32 momenta to 1e-4 of max(1, |u|max); a position is the time
        # integral of the velocity, so its error is bounded by that of the
        # momentum times the run's duration (the electrons near the ring of
        # this tight focus reach |u| ~ 9 and move several cells)
        t_run = work.steps * work.grid.dt
        assert du <= 1e-4 * max(1.0, umax), du
        assert dpos <= 1e-4 * max(1.0, umax) * t_run, (dpos, t_run)
    assert g.diagnostics()["n_alive"] == o.diagnostics()["n_alive"]


# ---------------------------------------------------------------------------
# Discrete continuity, step by step
# ---------------------------------------------------------------------------

def _continuity_bound(g, d, grid, eps):
    """Attainable per-step continuity residual.  In exact arithmetic the
    Esirkepov current makes [div_h E^{n+1} - div_h E^n] - [rho^{n+1} - rho^n]
    vanish at every node.  With the fields stored in the working precision
    each of the two divergences carries the rounding of its four E values,
    at most eps max|E| each, divided by the cell size; the charge-density
    part is relative to max|rho|."""
    emax = max(np.max(np.abs(g.read_field(c))) for c in ("ex", "ey"))
    return 1e-12 * d["rho_abs_max"] + 8 * eps * emax * (
        1.0 / grid.dx + 1.0 / grid.dy)


@pytest.mark.parametrize("prec", [wl.FP64, wl.FP32])
def test_continuity_residual_every_step(prec):
    """The per-step discrete continuity residual that the diagnostics report
    (difference of two consecutive Gauss defects) stays at rounding level on
    every one of 30 steps of an LP run whose pulse is inside the plasma; in
    FP64 it is below 1e-12 max|rho| (the charge-conservation bar) as well."""
    work = wl.april_2d(nx=136, ny=72, plasma=(40, 100, 0, 72), ppc=4,
                       a0=20.0, s=10.0, steps=30, seed=11)
    work.incident.t_focus -= 40 * work.grid.dt   # the pulse is in the plasma
    sp = explicit_species(work)
    g = make_gpu(work, sp, precision=prec)
    eps = 2.2e-16 if prec == wl.FP64 else 1.2e-7
    d0 = g.diagnostics()
    assert d0["continuity_steps"] == 0 and d0["continuity_residual"] == 0.0
    worst = 0.0
    for n in range(30):
        g.step(1)
        d = g.diagnostics()
        assert d["continuity_steps"] == 1
        assert d["rho_abs_max"] > 0.01
        bound = _continuity_bound(g, d, work.grid, eps)
        assert d["continuity_residual"] <= bound, (n, d, bound)
        worst = max(worst, d["continuity_residual"] / d["rho_abs_max"])
        if prec == wl.FP64:
            assert d["continuity_residual"] <= 1e-12 * d["rho_abs_max"], d
    _note(f"[continuity] prec {prec}: worst residual / max|rho| = {worst:.2e}")
    # a new step index resets the reference; several steps between calls
    g.set_step_index(d["step"])
    assert g.diagnostics()["continuity_steps"] == 0
    g.step(3)
    d = g.diagnostics()
    assert d["continuity_steps"] == 3
    assert d["continuity_residual"] <= 3 * _continuity_bound(
        g, d, work.grid, eps)


def test_continuity_residual_sees_a_written_field():
    """A field written between two diagnostics calls changes div_h E without
    any charge moving: the continuity residual is then exactly the change of
    the divergence, found at a node of the last, partial x-block of the
    reduction (the reference is not reset by a write)."""
    nx, ny = 300, 41
    grid = wl.Grid(2, nx, ny, 0.2, 0.25, 0.1)
    g = make_gpu(wl.Workload("vac", grid, [], wl.Incident(), 0), [])
    d = g.diagnostics()
    assert d["continuity_steps"] == 0 and d["continuity_residual"] == 0.0
    ex = np.zeros((ny + 2 * G, nx + 2 * G))
    ex[G + 17, G + nx - 5] = 4e-3
    g.write_field("ex", ex)
    d = g.diagnostics()
    assert d["continuity_steps"] == 0
    assert d["continuity_residual"] == pytest.approx(4e-3 / grid.dx,
                                                     rel=1e-15)
    d = g.diagnostics()            # nothing changed since
    assert d["continuity_residual"] == 0.0


# ---------------------------------------------------------------------------
# Gauss-law reduction against a known divergence
# ---------------------------------------------------------------------------

def test_gauss_residual_equals_injected_divergence_2d():
    """With no particles, div_h E of a written field is the whole residual.
    A bump at a node of the last, partial x-block of the reduction (and one
    in the last row) must be found exactly; a NaN must give +inf."""
    nx, ny = 300, 41            # 256-wide blocks: nodes 260..296 are partial
    grid = wl.Grid(2, nx, ny, 0.2, 0.25, 0.1)
    work = wl.Workload("vac", grid, [], wl.Incident(), 0)
    g = make_gpu(work, [])
    ex = np.zeros((ny + 2 * G, nx + 2 * G))
    # E_x at dual node (i + 1/2, j) feeds div at primal nodes i and i + 1
    i, j, v = nx - 5, ny - 4, 3e-3      # primal nodes nx - 5, nx - 4
    ex[G + j, G + i] = v
    g.write_field("ex", ex)
    d = g.diagnostics()
    assert d["gauss_residual"] == pytest.approx(v / grid.dx, rel=1e-15)
    assert d["rho_max"] == 0.0 and d["nonfinite"] == 0
    ey = np.zeros_like(ex)
    ey[G + 4, G + 150] = -7e-3      # the first row of the node range
    g.write_field("ey", ey)
    d = g.diagnostics()
    assert d["gauss_residual"] == pytest.approx(7e-3 / grid.dy, rel=1e-15)
    ex[G + 20, G + 100] = np.nan
    g.write_field("ex", ex)
    d = g.diagnostics()
    assert d["gauss_residual"] == math.inf
    assert d["nonfinite"] == 1


def test_gauss_residual_equals_injected_divergence_3d():
    """3D: a bump in the last group of eight z-planes and the last partial
    x-block of the reduction is found exactly; a NaN gives +inf."""
    from paper_2310_11393_amd.binding import Simulation3
    nx, ny, nz = 70, 13, 21        # 64-wide blocks; k groups of 8 planes
    grid = wl.Grid3(nx, ny, nz, 0.3, 0.25, 0.35,
                    0.4 / math.sqrt(1 / 0.09 + 1 / 0.0625 + 1 / 0.1225))
    sim = Simulation3(grid, wl.Incident())
    ez = np.zeros(sim.shape)
    k, j, i, v = nz - 4, ny - 5, nx - 4, 2.5e-3
    ez[G + k, G + j, G + i] = v     # E_z at (i, j, k + 1/2): nodes k, k + 1
    sim.write_field("ez", ez)
    d = sim.diagnostics()
    assert d["gauss_residual"] == pytest.approx(v / grid.dz, rel=1e-15)
    assert d["continuity_steps"] == 0 and d["continuity_residual"] == 0.0
    ez2 = ez.copy()
    ez2[G + k, G + j, G + i] = 0.0
    sim.write_field("ez", ez2)      # the change of div E between two calls
    d = sim.diagnostics()
    assert d["gauss_residual"] == 0.0
    assert d["continuity_residual"] == pytest.approx(v / grid.dz, rel=1e-15)
    ez[G + 8, G + 6, G + 10] = np.nan
    sim.write_field("ez", ez)
    d = sim.diagnostics()
    assert d["gauss_residual"] == math.inf
    sim.close()


# ---------------------------------------------------------------------------
# Adaptive sort cadence (single simulations, default runtime)
# ---------------------------------------------------------------------------
def _cadence_case(temperature_ev):
    return wl.april_2d(nx=136, ny=72, plasma=(40, 100, 0, 72), ppc=4,
                       a0=0.1, temperature_ev=temperature_ev, steps=34,
                       seed=23)


def _count_sorts(g, steps):
    g.profile(True)
    g.step(steps)
    g.sync()
    n = g.profile_read()["sort"][0]
    g.profile(False)
    return n


@pytest.mark.parametrize("prec", [wl.FP64, wl.FP32])
def test_adaptive_sort_cadence(prec):
    """With the default runtime a single simulation sorts 4 (FP32 form) or 8
    (FP64) to 16 steps after its last sort, once the push two steps earlier
    listed more than 2^-10 of the particles as stragglers.  A 1 eV plasma
    drifts far less than a cell in 34 steps: sorts at steps 16 and 32 only.
    A 2 MeV plasma (momenta of 2 m c per axis, up to ~0.65 cells per step)
    makes stragglers well within the shortest interval: a sort every
    4 / 8 steps, as a fixed cadence of that length gives.  The hot run, whose
    particles go through the straggler path between sorts, matches the
    oracle (fields and particles: FP64 1e-12, FP32 form 1e-4)."""
    steps = 34
    shortest = 4 if prec == wl.FP32 else 8
    cold, hot = _cadence_case(1.0), _cadence_case(2e6)
    g = make_gpu(cold, precision=prec)
    n_cold = _count_sorts(g, steps)
    g.close()
    g = make_gpu(hot, precision=prec, sort_every=shortest)
    n_fixed = _count_sorts(g, steps)
    g.close()
    g = make_gpu(hot, precision=prec)
    n_hot = _count_sorts(g, steps)
    _note(f"[cadence] prec {prec}: cold {n_cold} sorts, hot {n_hot}, fixed "
          f"every {shortest}: {n_fixed}")
    assert n_cold == steps // 16
    assert n_fixed == steps // shortest
    assert n_hot >= n_fixed - 1
    o = make_oracle(hot)
    o.step(steps)
    tol = 1e-12 if prec == wl.FP64 else 1e-4
    rel, den = field_rel_l2(g, o)
    dpos, du, umax = particle_errors(g, o)
    n_gpu = g.diagnostics()["n_alive"]
    g.close()
    _note(f"[cadence] prec {prec}: hot run fields {rel:.2e}, particles "
          f"{dpos:.2e} / {du:.2e} (|u| max {umax:.2f})")
    assert den > 0 and rel <= tol, rel
    if prec == wl.FP64:
        assert dpos <= 1e-12 and du <= 1e-12 * max(1.0, umax), (dpos, du)
    else:
        # momenta to 1e-4 of max(1, |u|max), positions to that times the
        # run's duration (the time integral of the velocity)
        t_run = steps * hot.grid.dt
        assert du <= 1e-4 * max(1.0, umax), du
        assert dpos <= 1e-4 * max(1.0, umax) * t_run, (dpos, t_run)
    assert n_gpu == o.diagnostics()["n_alive"]


# ---------------------------------------------------------------------------
# Failure isolation in sweeps
# ---------------------------------------------------------------------------

def _small_member(i, steps=40):
    return wl.april_2d(nx=96, ny=64, plasma=(30, 70, 0, 64), ppc=2, s=10.0,
                       a0=5.0 + 5 * i, steps=steps, seed=20 + i)


def test_batch_member_with_nan_fails_alone():
    """A NaN written into one member's field before the run: that member
    ends with SFPIC_E_NUMERIC, the others equal a batch without the fault
    (FP64, 1e-12: only the summation order of the deposit can differ)."""
    from paper_2310_11393_amd.binding import Batch
    works = [_small_member(i) for i in range(3)]
    clean = Batch(works, autotune=False)
    clean.run()
    bad = Batch(works, autotune=False)
    m1 = bad.member(1)
    ey = m1.read_field("ey")
    ey[G + 30, G + 50] = np.nan
    m1.write_field("ey", ey)
    bad.run()
    r1 = bad.result(1)
    assert r1["status"] == -5 and "non-finite" in r1["error"]
    for i in (0, 2):
        assert bad.result(i)["status"] == 0
        a, b = clean.member(i), bad.member(i)
        num = den = 0.0
        for c in ("ex", "ey", "ez", "bx", "by", "bz"):
            fa, fb = a.read_field(c), b.read_field(c)
            assert np.all(np.isfinite(fb))
            num += float(np.sum((fa - fb) ** 2))
            den += float(np.sum(fa ** 2))
        assert den > 0 and (num / den) ** 0.5 <= 1e-12
    bad.close()
    clean.close()


def test_server_request_that_overflows_fails_alone():
    """A request whose beam amplitude overflows the momenta (a0 = 1e200)
    fails with SFPIC_E_NUMERIC; the requests around it complete with the
    energies they have when run alone."""
    from paper_2310_11393_amd.binding import Server
    works = [_small_member(0), _small_member(1), _small_member(2)]
    works[1].incident.a0 = 1e200
    srv = Server(max_slots=4)
    tickets = [srv.submit(w) for w in works]
    for t in tickets:
        srv.wait(t, timeout_s=300)
    res = [srv.result(t) for t in tickets]
    assert res[1]["status"] == -5, res[1]
    from paper_2310_11393_amd.binding import Simulation
    alone = []
    for i in (0, 2):
        assert res[i]["status"] == 0
        s = Simulation.from_workload(works[i])   # the same device placement
        s.step(works[i].steps)
        alone.append(s.diagnostics())
        s.close()
    for r, d in zip((res[0], res[2]), alone):
        assert abs(r["diag"]["w_kin"] - d["w_kin"]) <= 1e-11 * d["w_kin"]
    st = srv.stats()
    assert st["failed"] == 1 and st["completed"] == 2
    srv.close()


# ---------------------------------------------------------------------------
# Per-handle error messages
# ---------------------------------------------------------------------------

def test_last_error_is_kept_per_handle():
    from paper_2310_11393_amd import binding as b
    L = b.lib()
    work = _small_member(0)
    s1 = make_gpu(work, explicit_species(work))
    s2 = make_gpu(work, explicit_species(work))
    out = np.zeros(4)
    rc = L.sfpic_read_field(s1.h, 99, out.ctypes.data_as(C.POINTER(
        C.c_double)), 4)
    assert rc == -1
    assert b"component" in L.sfpic_last_error(s1.h)
    assert L.sfpic_last_error(s2.h) == b""
    rc = L.sfpic_step(s2.h, -3)
    assert rc == -1 and b"nsteps" in L.sfpic_last_error(s2.h)
    assert b"component" in L.sfpic_last_error(s1.h)
    assert b"nsteps" in L.sfpic_last_error(None)
