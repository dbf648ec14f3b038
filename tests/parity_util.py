"""Helpers shared by the parity tests: run the same seeded input through the
HIP library and through the FP64 oracle, and compare."""
from __future__ import annotations

import numpy as np

from paper_2310_11393_amd import workloads as wl

FIELD_COMPS = ("ex", "ey", "ez", "bx", "by", "bz")


def explicit_species(work: wl.Workload, first=0, count=None):
    out = []
    for sp in work.species:
        x, y, ux, uy, uz = wl.generate_particles(sp, work.grid, first, count)
        out.append(dict(q=sp.q, m=sp.m, weight=sp.weight, x=x, y=y, ux=ux,
                        uy=uy, uz=uz))
    return out


def make_oracle(work: wl.Workload, species=None):
    from oracle import OracleSim
    sim = OracleSim(work.grid, work.incident)
    for e in (species if species is not None else explicit_species(work)):
        sim.add_species(e["q"], e["m"], e["weight"], e["x"], e["y"], e["ux"],
                        e["uy"], e["uz"])
    return sim


def make_gpu(work: wl.Workload, species=None, precision=None, **kw):
    from paper_2310_11393_amd.binding import Simulation
    return Simulation(work.grid, work.incident,
                      explicit=(species if species is not None
                                else explicit_species(work)),
                      precision=work.precision if precision is None
                      else precision, **kw)


def field_rel_l2(gsim, osim, comps=FIELD_COMPS):
    """Relative L2 of the stacked field components, GPU vs oracle."""
    num = den = 0.0
    for c in comps:
        g = gsim.read_field(c)
        o = osim.field(c)
        num += float(np.sum((g - o) ** 2))
        den += float(np.sum(o ** 2))
    return (num / den) ** 0.5 if den > 0 else num ** 0.5, den


def particle_errors(gsim, osim, sp=0):
    """Max abs position / momentum differences of particles matched by id;
    also the live-set agreement."""
    gx, gy, gux, guy, guz, gid = gsim.particles(sp)
    ox, oy, oux, ouy, ouz, alive = osim.particles(sp)
    live = np.nonzero(alive)[0]
    assert np.array_equal(np.sort(gid.astype(np.int64)), live), \
        "live particle sets differ"
    order = np.argsort(gid)
    idx = gid[order].astype(np.int64)
    dpos = max(np.max(np.abs(gx[order] - ox[idx]), initial=0.0),
               np.max(np.abs(gy[order] - oy[idx]), initial=0.0))
    du = max(np.max(np.abs(a[order] - b[idx]), initial=0.0)
             for a, b in ((gux, oux), (guy, ouy), (guz, ouz)))
    umax = max(np.max(np.abs(b[idx]), initial=0.0) for b in (oux, ouy, ouz))
    return dpos, du, umax
