"""Sweeps on the GPU: batches and the request server (needs an MI355X).

Members of a batch are advanced by the batched launches (one launch per
phase for all members, persistent push over a shared tile queue, a sort of
the members it is due for after every step, graph replay of 8 steps).  Each member must still equal its own oracle run
(FP64: relative L2 of the fields <= 1e-12 after its steps) and its own run
alone (FP32 form: <= 1e-4), whatever the other members, the tile chosen by
the autotuner, the cadence or the step count (not a multiple of the cadence).
"""
import sys
import time

import numpy as np
import pytest

from paper_2310_11393_amd import workloads as wl
from paper_2310_11393_amd.binding import (REQ_DONE, Batch, Server, SimDesc,
                                          hist_spec)

from parity_util import (explicit_species, field_rel_l2, make_gpu,
                         make_oracle, particle_errors)

pytestmark = pytest.mark.gpu

FP64_FIELD_TOL = 1e-12
FP32_FIELD_TOL = 1e-4


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _lp(**kw):
    args = dict(nx=136, ny=72, plasma=(40, 100, 0, 72), ppc=4,
                kind=wl.INC_APRIL_LP, w0_lambda=1.0, s=20.0, a0=10.0,
                temperature_ev=1.0, steps=50, seed=11)
    args.update(kw)
    return wl.april_2d(**args)


def _members(precision):
    """Uneven members: LP / RP, different grids, densities, a ragged grid
    and a 1D member (its own group)."""
    ms = [_lp(precision=precision),
          _lp(kind=wl.INC_APRIL_RP, w0_lambda=0.8, s=10.0, a0=30.0,
              temperature_ev=0.0, nx=96, ny=96, plasma=(30, 70, 20, 80),
              ppc=3, n=0.02, seed=12, precision=precision),
          _lp(nx=101, ny=77, plasma=(30, 81, 3, 70), ppc=3, s=10.0, seed=13,
              precision=precision),
          wl.plane_pulse_1d(nx=300, slab=(100, 230), ppc=16, a0=3.0,
                            steps=50)]
    ms[3].precision = precision
    return ms


STEPS = [50, 37, 44, 41]  # not all multiples of any cadence


@pytest.mark.parametrize("mode", ["graph", "fixed_eager", "split_items"])
def test_fp64_batch_members_match_oracle(mode):
    """Every member of an FP64 batch against its own oracle run: replayed
    graphs with the library's defaults, eager launches with a fixed tile and
    cadence, and work items of at most 64 particles (every tile shared by
    several workgroups of the persistent push)."""
    members = _members(wl.FP64)
    kw = ({} if mode == "graph" else
          dict(tile=(8, 4), sort_every=3, graph=False, autotune=False))
    if mode == "split_items":
        kw.update(tile=(16, 8), item_particles=64)
    _note(f"[batch] fp64 {mode}: {len(members)} members")
    b = Batch(members, nsteps=STEPS, **kw)
    b.run()
    st = b.stats()
    _note(f"[batch] groups {[(g['dims'], g['tile'], g['sort_every']) for g in st['groups']]}")
    assert len(st["groups"]) == 2
    if mode == "graph":
        # runs this short are not tuned (the trials would take too much of
        # them): library defaults and graph replays
        assert not any(g["tuned"] for g in st["groups"])
        assert st["graph_launches"] > 0
    for i, (work, n) in enumerate(zip(members, STEPS)):
        sp = explicit_species(work)
        o = make_oracle(work, sp)
        o.step(n)
        g = b.member(i)
        rel, den = field_rel_l2(g, o)
        assert den > 0 and rel <= FP64_FIELD_TOL, (i, rel)
        jrel, _ = field_rel_l2(g, o, comps=("jx", "jy", "jz"))
        assert jrel <= FP64_FIELD_TOL, (i, jrel)
        dpos, du, umax = particle_errors(g, o)
        assert dpos <= 1e-12 and du <= 1e-12 * max(1.0, umax), (i, dpos, du)
        r = b.result(i)
        od = o.diagnostics()
        assert r["status"] == 0 and r["steps"] == n
        assert r["diag"]["step"] == n
        assert r["diag"]["n_alive"] == od["n_alive"]
        assert abs(r["diag"]["w_kin"] - od["w_kin"]) <= 1e-11 * abs(od["w_kin"])
        assert abs(r["diag"]["w_em"] - od["w_em"]) <= 1e-11 * abs(od["w_em"])
        assert abs(r["diag"]["w_em_total"] - od["w_em_total"]) <= \
            1e-11 * abs(od["w_em_total"])
        # the member can be stepped on as an ordinary simulation afterwards
    b.close()


def _pulse_2d(precision):
    """A 2D member lit by the plane pulse (no April beam)."""
    dx = 2.0 * np.pi / 32
    grid = wl.Grid(2, 96, 40, dx, dx, 0.95 * dx / np.sqrt(2.0))
    fwhm = 3.0 * 2.0 * np.pi
    inc = wl.Incident(kind=wl.INC_PLANE_PULSE_1D, a0=3.0, fwhm_t=fwhm,
                      t0=fwhm - 30 * dx)
    sp = wl.Species(q=-1.0, m=1.0, density=0.02, region=(30, 80, 0, 40),
                    ppc=4, temperature_ev=1.0, seed=21)
    return wl.Workload("pulse_2d", grid, [sp], inc, 40, precision)


@pytest.mark.parametrize("prec", [wl.FP64, wl.FP32])
def test_batch_of_mixed_models(prec):
    """A 2D group in which one member has no April beam runs the push built
    for every model (an all-April group runs the LP / RP pushes, which the
    other tests cover); each member matches the oracle."""
    members = [_lp(precision=prec), _pulse_2d(prec),
               _lp(kind=wl.INC_APRIL_RP, w0_lambda=0.8, s=10.0, a0=30.0,
                   temperature_ev=0.0, nx=96, ny=96, plasma=(30, 70, 20, 80),
                   ppc=3, n=0.02, seed=12, precision=prec)]
    steps = [40, 33, 37]
    _note(f"[batch] mixed models, precision {prec}")
    b = Batch(members, nsteps=steps, tile=(8, 4), sort_every=3, graph=False,
              autotune=False)
    b.run()
    assert len(b.stats()["groups"]) == 1
    tol = FP64_FIELD_TOL if prec == wl.FP64 else FP32_FIELD_TOL
    for i, (work, n) in enumerate(zip(members, steps)):
        o = make_oracle(work, explicit_species(work))
        o.step(n)
        rel, den = field_rel_l2(b.member(i), o)
        _note(f"[batch] mixed member {i}: {rel:.2e}")
        assert den > 0 and rel <= tol, (i, rel)
        assert b.result(i)["status"] == 0
    b.close()


def _profiled_lp(precision):
    """An LP member whose plasma follows the Sec. 3.1 super-Gaussian profile
    along x."""
    w = _lp(precision=precision, ppc=6, seed=14)
    sp = w.species[0]
    sp.profile = wl.PROFILE_SUPERGAUSS
    sp.profile_center, sp.profile_fwhm = 70.0 * w.grid.dx, 30.0 * w.grid.dx
    sp.profile_order, sp.profile_xmin = 12.0, 40.0 * w.grid.dx
    return w


@pytest.mark.parametrize("prec", [wl.FP64, wl.FP32])
def test_batch_of_every_incident_source(prec):
    """A 2D batch whose members take the incident field every way a single
    simulation can: the April beam sampled on the Yee nodes, the paraxial
    Gaussian beam at the particles, and an April beam on a plasma with the
    Sec. 3.1 density profile; each member matches the oracle."""
    on_nodes = _lp(precision=prec, seed=15)
    on_nodes.incident.on_nodes = 1
    gauss = wl.gauss_beam_2d(nx=160, ny=96, plasma=(50, 110, 20, 76), ppc=4,
                             w0_lambda=2.0, cycles=3.0, a0=3.0, steps=40,
                             cells_per_lambda=24)
    gauss.precision = prec
    members = [on_nodes, gauss, _profiled_lp(prec)]
    steps = [40, 35, 38]
    _note(f"[batch] every source, precision {prec}")
    b = Batch(members, nsteps=steps, tile=(8, 4), sort_every=3, graph=True,
              autotune=False)
    b.run()
    assert len(b.stats()["groups"]) == 1
    tol = FP64_FIELD_TOL if prec == wl.FP64 else FP32_FIELD_TOL
    for i, (work, n) in enumerate(zip(members, steps)):
        sp = explicit_species(work)
        o = make_oracle(work, sp)
        o.step(n)
        rel, den = field_rel_l2(b.member(i), o)
        _note(f"[batch] source member {i}: {rel:.2e}")
        assert den > 0 and rel <= tol, (i, rel)
        r = b.result(i)
        assert r["status"] == 0 and r["steps"] == n
        assert r["diag"]["n_alive"] == o.diagnostics()["n_alive"]
    # the profiled member's pushes count the particles it placed, which the
    # profile makes fewer than its region times ppc
    w = members[2]
    sp = w.species[0]
    placed = sp.count(w.grid.dx)
    assert placed < (sp.region[1] - sp.region[0]) * \
        (sp.region[3] - sp.region[2]) * sp.ppc
    r = b.result(2)
    assert r["pushes"] == pytest.approx(
        steps[2] * 0.5 * (placed + r["diag"]["n_alive"]), rel=1e-12)
    b.close()


def test_fp32_batch_member_equals_its_run_alone():
    """Each FP32 member in the mix vs the same member run alone, and both vs
    the FP64 oracle."""
    members = _members(wl.FP32)
    b = Batch(members, nsteps=STEPS, hist=hist_spec(n_e=64, emax=0.05,
                                                    n_theta=36, ek_min=0.0))
    b.run()
    for i, (work, n) in enumerate(zip(members, STEPS)):
        alone = make_gpu(work, explicit_species(work), precision=wl.FP32)
        alone.step(n)
        g = b.member(i)
        num = den = 0.0
        for c in ("ex", "ey", "ez", "bx", "by", "bz"):
            a, m = alone.read_field(c), g.read_field(c)
            num += float(np.sum((a - m) ** 2))
            den += float(np.sum(a ** 2))
        rel = (num / den) ** 0.5
        _note(f"[batch] fp32 member {i}: mix vs alone {rel:.2e}")
        assert den > 0 and rel <= FP32_FIELD_TOL, (i, rel)
        o = make_oracle(work, explicit_species(work))
        o.step(n)
        orel, _ = field_rel_l2(g, o)
        assert orel <= FP32_FIELD_TOL, (i, orel)
        r = b.result(i)
        ad = alone.diagnostics()
        assert r["diag"]["n_alive"] == ad["n_alive"]
        assert abs(r["diag"]["w_kin"] - ad["w_kin"]) <= 1e-4 * ad["w_kin"]
        if work.grid.dims == 2:
            _, mom = alone.histogram(0, 64, 0.05, 36, 0.0)
            assert abs(r["moments"][0] - mom[0]) <= 1e-6 * mom[0]
            for k in range(1, 5):
                assert abs(r["moments"][k] - mom[k]) <= 1e-3 * abs(mom[k])
        alone.close()
    b.close()


def test_autotuned_fp32_batch():
    """Runs long enough are tuned on their own first steps: every tile
    candidate, then every sort cadence (2, 4, 8) is timed on real steps (two
    passes each for runs of 256 steps or more), members are re-tiled in
    between, the fastest candidates are the ones used, and the result still
    equals each member's run alone."""
    members = [_lp(precision=wl.FP32, seed=31),
               _lp(kind=wl.INC_APRIL_RP, w0_lambda=0.8, s=10.0, a0=30.0,
                   temperature_ev=0.0, nx=96, ny=96, plasma=(30, 70, 20, 80),
                   ppc=3, n=0.02, seed=32, precision=wl.FP32)]
    steps = [260, 251]
    b = Batch(members, nsteps=steps)
    b.run()
    st = b.stats()
    g = st["groups"][0]
    _note(f"[batch] tuned: tile {g['tile']} cadence {g['sort_every']} "
          f"trials {g['trials']}")
    assert g["tuned"] and len(g["trials"]) == 4 * 2 + 3 * 2
    tile_trials, cad_trials = g["trials"][:8], g["trials"][8:]
    assert all(t[1] == 4 for t in tile_trials)
    assert all(t[2] > 0 for t in g["trials"])
    mean = {}
    for tile, _c, ns in tile_trials:
        mean.setdefault(tile, []).append(ns)
    best_tile = min(mean, key=lambda k: sum(mean[k]) / len(mean[k]))
    assert g["tile"] == best_tile
    # the cadence pass runs with the chosen tile and tries every cadence
    assert all(t[0] == best_tile for t in cad_trials)
    assert sorted({t[1] for t in cad_trials}) == [2, 4, 8]
    cmean = {}
    for _tile, c, ns in cad_trials:
        cmean.setdefault(c, []).append(ns)
    best_c = min(cmean, key=lambda k: sum(cmean[k]) / len(cmean[k]))
    assert g["sort_every"] == best_c
    for i, (work, n) in enumerate(zip(members, steps)):
        alone = make_gpu(work, explicit_species(work), precision=wl.FP32)
        alone.step(n)
        m = b.member(i)
        num = den = 0.0
        for c in ("ex", "ey", "ez", "bx", "by", "bz"):
            a, x = alone.read_field(c), m.read_field(c)
            num += float(np.sum((a - x) ** 2))
            den += float(np.sum(a ** 2))
        rel = (num / den) ** 0.5
        _note(f"[batch] tuned member {i}: mix vs alone {rel:.2e}")
        assert den > 0 and rel <= FP32_FIELD_TOL, (i, rel)
        assert b.result(i)["steps"] == n
        alone.close()
    b.close()


def test_batch_graph_replays_equal_eager_launches():
    """Graph replays (with the eager sorts and reads between them) give the
    results of eager launches, member by member, to the FP64 tolerance."""
    members = _members(wl.FP64)[:3]
    steps = [29, 17, 23]
    ga = Batch(members, nsteps=steps, tile=(16, 8), sort_every=4, graph=True)
    ea = Batch(members, nsteps=steps, tile=(16, 8), sort_every=4, graph=False)
    ga.run()
    ea.run()
    assert ga.stats()["graph_launches"] >= 4
    assert ea.stats()["graph_launches"] == 0
    for i in range(len(members)):
        a, e = ga.member(i), ea.member(i)
        num = den = 0.0
        for c in ("ex", "ey", "ez", "bx", "by", "bz", "jx", "jy", "jz"):
            x, y = a.read_field(c), e.read_field(c)
            num += float(np.sum((x - y) ** 2))
            den += float(np.sum(y ** 2))
        assert den > 0 and (num / den) ** 0.5 <= FP64_FIELD_TOL, i
    ga.close()
    ea.close()


def test_server_results_equal_runs_alone():
    """Requests submitted while others run join at the next tick; each
    result equals the same simulation run alone (FP64 to 1e-11 on the
    energies, FP32 to 1e-4), also for a request with the incident field on
    the nodes and one with the Gaussian beam."""
    srv = Server(max_slots=8)
    hs = hist_spec(n_e=64, emax=0.05, n_theta=36, ek_min=0.0)
    reqs = []
    on_nodes = _lp(precision=wl.FP64, seed=16)
    on_nodes.incident.on_nodes = 1
    gauss = wl.gauss_beam_2d(nx=160, ny=96, plasma=(50, 110, 20, 76), ppc=4,
                             w0_lambda=2.0, cycles=3.0, a0=3.0, steps=30,
                             cells_per_lambda=24)
    gauss.precision = wl.FP32
    works = (_members(wl.FP64)[:3] + _members(wl.FP32)[:3] +
             [on_nodes, gauss])
    steps = [40, 23, 31, 40, 23, 31, 29, 30]
    # two at once, then the rest while those run
    for k, (w, n) in enumerate(zip(works, steps)):
        reqs.append((srv.submit(w, nsteps=n, hist=hs), w, n))
        if k == 1:
            time.sleep(0.2)
    for t, w, n in reqs:
        srv.wait(t, 300.0)
        assert srv.poll(t) == REQ_DONE
    st = srv.stats()
    _note(f"[server] {st}")
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["p99_s"] >= st["p50_s"] > 0.0
    for t, w, n in reqs:
        r = srv.result(t)
        assert r["status"] == 0 and r["steps"] == n
        alone = make_gpu(w, explicit_species(w))
        alone.step(n)
        ad = alone.diagnostics()
        tol = 1e-11 if w.precision == wl.FP64 else 1e-4
        assert r["diag"]["n_alive"] == ad["n_alive"]
        for key in ("w_kin", "w_em", "w_em_total"):
            assert abs(r["diag"][key] - ad[key]) <= tol * abs(ad[key]), key
        if w.grid.dims == 2:
            h, mom = alone.histogram(0, 64, 0.05, 36, 0.0)
            hs_ = srv.histogram(t)
            assert np.abs(hs_ - h).sum() <= 10 * tol * max(h.sum(), 1e-300)
        alone.close()
    srv.close()


def test_server_admits_by_device_footprint():
    """With a budget for two members, at most two are resident; the rest wait
    in FIFO order and all finish."""
    works = [_lp(precision=wl.FP32, seed=20 + k) for k in range(5)]
    fp = SimDesc(works[0]).footprint()
    srv = Server(budget_bytes=int(2.5 * fp), max_slots=16)
    tickets = [srv.submit(w, nsteps=12) for w in works]
    for t in tickets:
        srv.wait(t, 300.0)
    st = srv.stats()
    assert st["completed"] == 5
    assert st["max_running"] <= 2
    assert st["bytes_peak"] <= st["budget"]
    rs = [srv.result(t) for t in tickets]
    # FIFO: admission order follows submission order
    starts = [r["t_start"] for r in rs]
    assert starts == sorted(starts)
    for r in rs:
        assert r["device_bytes"] <= fp
    srv.close()
