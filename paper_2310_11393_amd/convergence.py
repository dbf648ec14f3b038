"""Convergence analysis of the scattered-field step (Sec. 3.1).

The paper measures how solutions at cell size h = 2 pi / (16 2^m) approach
the finest one, taken as exact:

  ||dE(., t_n)||_{2,h} = ( h sum_k |E^h(x_k, t_n) - E^exact(x_k, t_n)|^2 )^(1/2)

over the grid points the two resolutions share, and the numerical rate
p = log2( ||dE||_{2,h} / ||dE||_{2,h/2} ).

The paper also compares two ways of carrying the pulse: (i) the whole
field on the grid, the pulse launched by the solver, and (ii) the
scattered-field form, through a cross-norm between the two models' finest
solutions (same discrete norm) and through time averages of the energy
differences, (1/N) sum_n |W_h(t_n) - W_fine(t_n)| within a model and
(1/N) sum_n |W^(i)(t_n) - W^(ii)(t_n)| between them at the finest grid.
Model (i) here starts from the incident pulse sampled on the Yee nodes as
the initial condition (E at t = 0, B at -dt/2) of a run with no incident
field, in place of a laser launched from the boundary, so both models see
the same pulse and differ only in how it propagates to the plasma.

In the scattered-field form the incident field is the same closed form on
every grid, so differences of the total field at common primal nodes equal
differences of the scattered field; the studies record both.  The
refinement driver runs the 1D set-up of Sec. 3.1 (plane pulse, order-12
super-Gaussian plasma) through the library, from a quiet start (particles
evenly spaced in each cell) so that particle noise does not mask the grid
error.
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence

import numpy as np

from . import workloads as wl

GUARD = 3


def common_values(fine_row: np.ndarray, ratio: int, n_coarse: int,
                  dual: bool) -> np.ndarray:
    """Values of a 1D fine-grid array (with guards, cell size h / ratio) at
    the n_coarse + 1 primal (or n_coarse dual) nodes of the coarse grid.
    Primal coarse nodes are every ratio-th fine node; a dual coarse node
    (i + 1/2) h lies midway between fine dual nodes, so it takes their mean
    (second-order accurate; ratio even)."""
    if not dual:
        idx = GUARD + ratio * np.arange(n_coarse + 1)
        return fine_row[idx]
    if ratio % 2:
        raise ValueError("dual nodes coincide only for even ratios")
    # coarse dual node (i + 1/2) h = fine position (ratio i + ratio / 2) h_f,
    # between fine dual nodes ratio i + ratio/2 - 1 (+1/2) and + 0 (+1/2)
    j = ratio * np.arange(n_coarse) + ratio // 2
    return 0.5 * (fine_row[GUARD + j - 1] + fine_row[GUARD + j])


def l2_norm(coarse_row: np.ndarray, fine_row: np.ndarray, ratio: int,
            n_coarse: int, h: float, dual: bool = False) -> float:
    """||E^h - E^fine||_{2,h} over the coarse grid's physical nodes."""
    n = n_coarse if dual else n_coarse + 1
    a = coarse_row[GUARD:GUARD + n]
    b = common_values(fine_row, ratio, n_coarse, dual)
    return math.sqrt(h * float(np.sum((a - b) ** 2)))


def rate(e_h: float, e_h2: float) -> float:
    """Numerical convergence rate p = log2(e_h / e_h2)."""
    return math.log2(e_h / e_h2)


def cross_norm(row_a: np.ndarray, row_b: np.ndarray, n: int, h: float,
               dual: bool = False) -> float:
    """Cross-norm of Sec. 3.1: (h sum_k |a(x_k) - b(x_k)|^2)^(1/2) between
    two solutions on the same grid (n cells, guards included in the rows)
    over its physical primal (n + 1) or dual (n) nodes."""
    m = n if dual else n + 1
    d = row_a[GUARD:GUARD + m] - row_b[GUARD:GUARD + m]
    return math.sqrt(h * float(np.sum(d * d)))


def energy_norm(series_a: Sequence[float], series_b: Sequence[float],
                scale: float = 1.0) -> float:
    """Time-averaged energy difference of Sec. 3.1,
    (1/N) sum_{n=1..N} |W_a(t_n) - W_b(t_n)|, divided by scale (the paper
    quotes it relative to the peak total energy)."""
    a = np.asarray(series_a, dtype=np.float64)
    b = np.asarray(series_b, dtype=np.float64)
    if a.shape != b.shape or a.size == 0:
        raise ValueError("energy series must be non-empty and of one length")
    return float(np.mean(np.abs(a - b))) / scale


FIELDS = ("ex", "ey", "ez", "bx", "by", "bz")


def full_field_start(sim_ff, sim_sff) -> None:
    """Initial condition of model (i): the total field of sim_sff (a
    scattered-field run of the same grid at step 0, whose scattered field
    is zero, so this is the incident pulse on the Yee nodes: E at t = 0,
    B at t = -dt/2) written into the E and B of sim_ff, a run without an
    incident field."""
    for c in FIELDS:
        sim_ff.write_field(c, sim_sff.read_total_field(c))


def quiet_profile_1d(grid, density: float, ppc: int, center: float,
                     fwhm: float, order: float, xmin: float) -> dict:
    """Explicit cold electrons of the Sec. 3.1 profile: cell c holds
    floor(ppc f(x_c) + 1/2) particles (the library's own per-column rule),
    evenly spaced in the cell, each of weight density / ppc."""
    sp = wl.Species(q=-1.0, m=1.0, density=density, region=(0, grid.nx, 0, 1),
                    ppc=ppc, profile=wl.PROFILE_SUPERGAUSS,
                    profile_center=center, profile_fwhm=fwhm,
                    profile_order=order, profile_xmin=xmin)
    off = wl.profile_offsets(sp, 0, grid.nx, grid.dx)
    counts = np.diff(off)
    cells = np.repeat(np.arange(grid.nx), counts)
    j = np.arange(len(cells)) - np.repeat(off[:-1], counts)
    k = np.repeat(counts, counts)
    x = (cells + (j + 0.5) / k) * grid.dx
    z = np.zeros(len(x))
    return dict(q=-1.0, m=1.0, weight=density / ppc, x=x, y=z, ux=z, uy=z,
                uz=z)


def _model_sim(grid, inc, model: str, **kw):
    """A simulation of the given model: "sff", the scattered-field form
    with incident `inc`, or "ff", model (i) started from inc's pulse on the
    grid (the helper scattered-field run is released here)."""
    from .binding import Simulation
    sim = Simulation(grid, inc, **kw)
    if model == "sff":
        return sim
    try:
        ff = Simulation(grid, wl.Incident(kind=wl.INC_NONE), **kw)
        try:
            full_field_start(ff, sim)
        except BaseException:
            ff.close()
            raise
        return ff
    finally:
        sim.close()


def refinement_study_1d(ms: Sequence[int], length: float, a0: float,
                        fwhm_t: float, t0: float, density: float, ppc: int,
                        center: float, fwhm: float, order: float,
                        xmin: float, t_snap: Sequence[float],
                        cfl: float = 0.99, model: str = "sff"
                        ) -> Dict[int, Dict[float, dict]]:
    """Run the 1D set-up of Sec. 3.1 at cell sizes 2 pi / (16 2^m) for m in
    ms through the library (FP64) and return, per m and snapshot time: the
    stored E_x and E_y rows ("ex", "ey"), the total field rows ("ex_total",
    "ey_total"; guards included), the kinetic and total electromagnetic
    energies ("w_kin", "w_em") and the cell count and size.

    model "sff" is the scattered-field form (ii); "ff" is model (i), the
    pulse on the grid from t = 0 (full_field_start) with no incident field,
    which needs the pulse inside the box at t = 0 (t0 < 0 places its centre
    at x = -t0).  Snapshot times must be multiples of the coarsest time step
    so that every resolution reaches them exactly."""
    if model not in ("sff", "ff"):
        raise ValueError("model must be 'sff' or 'ff'")
    m0 = min(ms)
    dt0 = cfl * 2 * math.pi / (16 * 2 ** m0)
    out: Dict[int, Dict[float, dict]] = {}
    for m in ms:
        h = 2 * math.pi / (16 * 2 ** m)
        nx = int(round(length / h))
        grid = wl.Grid(1, nx, 1, h, h, cfl * h)
        inc = wl.Incident(kind=wl.INC_PLANE_PULSE_1D, a0=a0, fwhm_t=fwhm_t,
                          t0=t0)
        e = quiet_profile_1d(grid, density, ppc, center, fwhm, order, xmin)
        sim = _model_sim(grid, inc, model, explicit=[e])
        try:
            res = _snapshots_1d(sim, t_snap, dt0, m - m0, nx, h)
        finally:
            sim.close()
        out[m] = res
    return out


def _snapshots_1d(sim, t_snap, dt0, dm, nx, h):
    """Step sim to each snapshot time (2^dm steps per coarsest step dt0)
    and record its rows and energies there."""
    done = 0
    res = {}
    for t in t_snap:
        k0 = t / dt0
        if abs(k0 - round(k0)) > 1e-9:
            raise ValueError("snapshot times must be multiples of the "
                             "coarsest time step")
        target = int(round(k0)) * 2 ** dm
        sim.step(target - done)
        done = target
        d = sim.diagnostics()
        res[t] = {"ex": sim.read_field("ex")[0],
                  "ey": sim.read_field("ey")[0],
                  "ex_total": sim.read_total_field("ex")[0],
                  "ey_total": sim.read_total_field("ey")[0],
                  "w_kin": d["w_kin"], "w_em": d["w_em_total"],
                  "nx": nx, "h": h}
    return res


def study_norms(study: Dict[int, Dict[float, dict]], comp: str = "ey"
                ) -> Dict[float, List[float]]:
    """Norms of every resolution but the finest against the finest, per
    snapshot time, of a recorded row: "ey" / "ex" (stored field) or
    "ey_total" / "ex_total" (E_y, the transverse field, is primal; E_x, the
    longitudinal one, dual)."""
    ms = sorted(study)
    ref = ms[-1]
    out = {}
    for t in study[ref]:
        fine = study[ref][t]
        norms = []
        for m in ms[:-1]:
            c = study[m][t]
            ratio = 2 ** (ref - m)
            norms.append(l2_norm(c[comp], fine[comp], ratio, c["nx"], c["h"],
                                 dual=comp.startswith("ex")))
        out[t] = norms
    return out


def study_cross_norms(study_i: Dict[int, Dict[float, dict]],
                      study_ii: Dict[int, Dict[float, dict]],
                      comp: str = "ey") -> Dict[int, Dict[float, float]]:
    """Cross-norm between models (i) and (ii) of the total field comp
    ("ex" or "ey") per resolution m and snapshot time (the paper forms it
    at the finest grid; every grid is given here)."""
    out: Dict[int, Dict[float, float]] = {}
    for m in study_i:
        out[m] = {}
        for t, a in study_i[m].items():
            b = study_ii[m][t]
            out[m][t] = cross_norm(a[comp + "_total"], b[comp + "_total"],
                                   a["nx"], a["h"], dual=(comp == "ex"))
    return out


def study_energy_norms(study: Dict[int, Dict[float, dict]],
                       key: str = "w_em", scale: float = 1.0
                       ) -> List[float]:
    """Time-averaged difference of the energy `key` ("w_em" or "w_kin")
    from the finest grid over the snapshot times, for every resolution but
    the finest, divided by scale."""
    ms = sorted(study)
    ref = [study[ms[-1]][t][key] for t in study[ms[-1]]]
    return [energy_norm([study[m][t][key] for t in study[ms[-1]]], ref,
                        scale) for m in ms[:-1]]


# --- 2D (Sec. 3.2) ----------------------------------------------------------
#
# In 2D the paper compares the two models in vacuum through the relative L1
# error of the intensity I = E_par^2 + E_long^2 and the relative Frobenius
# error of each component, and convergence through the 1D norm above along
# the beam axis.  Build axes: propagation x, polarization y, so the paper's
# transverse E is E_y (primal in x, dual in y) and its longitudinal E is E_x
# (dual in x, primal in y).

# half-cell offsets (x, y) of the stored components on the Yee grid
STAGGER = dict(ex=(1, 0), ey=(0, 1), ez=(0, 0), bx=(0, 1), by=(1, 0),
               bz=(1, 1))


def physical(plane: np.ndarray, n_x: int, n_y: int, comp: str) -> np.ndarray:
    """The physical nodes of a 2D plane with guards: (n + 1) primal or n
    dual nodes along each axis."""
    hx, hy = STAGGER[comp]
    return plane[GUARD:GUARD + n_y + 1 - hy, GUARD:GUARD + n_x + 1 - hx]


def frobenius_error(plane_a: np.ndarray, plane_b: np.ndarray, n_x: int,
                    n_y: int, comp: str) -> float:
    """Relative Frobenius error of Sec. 3.2, ||a - b||_F / ||b||_F over the
    component's physical nodes (b is the reference model)."""
    a = physical(plane_a, n_x, n_y, comp)
    b = physical(plane_b, n_x, n_y, comp)
    return math.sqrt(float(np.sum((a - b) ** 2)) / float(np.sum(b * b)))


def intensity(ey: np.ndarray, ex: np.ndarray, n_x: int, n_y: int
              ) -> np.ndarray:
    """E_y^2 + E_x^2 at the interior primal nodes (i, j), 1 <= i < n_x,
    1 <= j < n_y: E_y (dual in y) and E_x (dual in x) each the mean of the
    two nodes that bracket (i, j) along their dual axis."""
    g = GUARD
    ey_p = 0.5 * (ey[g:g + n_y - 1, g + 1:g + n_x] +
                  ey[g + 1:g + n_y, g + 1:g + n_x])
    ex_p = 0.5 * (ex[g + 1:g + n_y, g:g + n_x - 1] +
                  ex[g + 1:g + n_y, g + 1:g + n_x])
    return ey_p * ey_p + ex_p * ex_p


def intensity_error(ey_a, ex_a, ey_b, ex_b, n_x: int, n_y: int) -> float:
    """Relative L1 error of the intensity, Sec. 3.2:
    sum |I_a - I_b| / sum I_b over the interior primal nodes."""
    ia = intensity(ey_a, ex_a, n_x, n_y)
    ib = intensity(ey_b, ex_b, n_x, n_y)
    return float(np.sum(np.abs(ia - ib))) / float(np.sum(ib))


def axis_row(plane: np.ndarray, j_axis: int, comp: str) -> np.ndarray:
    """The row of a 2D plane on the line y = j_axis h (the beam axis), guards
    included along x: a component dual in y takes the mean of the two rows
    that bracket the line."""
    g = GUARD
    if STAGGER[comp][1]:
        return 0.5 * (plane[g + j_axis - 1] + plane[g + j_axis])
    return plane[g + j_axis].copy()


def refinement_study_2d(ms: Sequence[int], lx: float, ly: float, a0: float,
                        w0: float, fwhm_t: float, x_center0: float,
                        x_focus: float, t_snap: Sequence[float],
                        density: float = 0.0, ppc: int = 0,
                        center: float = 0.0, fwhm: float = 1.0,
                        order: float = 12.0, xmin: float = 0.0,
                        seed: int = 7, cfl: float = 0.99, model: str = "sff",
                        keep_planes: bool = True
                        ) -> Dict[int, Dict[float, dict]]:
    """The 2D set-up of Sec. 3.2 through the library (FP64) at cell sizes
    2 pi / (16 2^m): the paraxial Gaussian beam focused on the box's axis at
    x_focus, its envelope centred at x_center0 at t = 0, optionally a cold
    plasma with the order-`order` super-Gaussian profile along x, uniform
    across y (density = 0: vacuum).  Per m and snapshot time: the total E_y
    and E_x planes ("ey_total", "ex_total", if keep_planes), their rows on
    the beam axis ("ey_axis", "ex_axis"), the energies ("w_kin", "w_em") and
    the cell counts and size.  model "sff" / "ff" as in the 1D study; the
    snapshot times must be multiples of the coarsest time step."""
    if model not in ("sff", "ff"):
        raise ValueError("model must be 'sff' or 'ff'")
    m0 = min(ms)
    dt0 = cfl * 2 * math.pi / (16 * 2 ** m0) / math.sqrt(2.0)
    out: Dict[int, Dict[float, dict]] = {}
    for m in ms:
        h = 2 * math.pi / (16 * 2 ** m)
        nx, ny = int(round(lx / h)), int(round(ly / h))
        if ny % 2:
            raise ValueError("the axis must be a node row: even ny needed")
        grid = wl.Grid(2, nx, ny, h, h, cfl * h / math.sqrt(2.0))
        inc = wl.Incident(kind=wl.INC_GAUSS_2D, a0=a0, w0=w0, fwhm_t=fwhm_t,
                          t0=x_focus - x_center0, x_focus=x_focus,
                          y_focus=0.5 * ny * h)
        species = []
        if density > 0.0:
            species = [wl.Species(q=-1.0, m=1.0, density=density,
                                  region=(0, nx, 0, ny), ppc=ppc, seed=seed,
                                  profile=wl.PROFILE_SUPERGAUSS,
                                  profile_center=center, profile_fwhm=fwhm,
                                  profile_order=order, profile_xmin=xmin)]
        sim = _model_sim(grid, inc, model, species=species)
        try:
            res = _snapshots_2d(sim, t_snap, dt0, m - m0, nx, ny, h,
                                keep_planes)
        finally:
            sim.close()
        out[m] = res
    return out


def _snapshots_2d(sim, t_snap, dt0, dm, nx, ny, h, keep_planes):
    """As _snapshots_1d for the 2D study: axis rows, energies and, if
    keep_planes, the total E_y and E_x planes."""
    done = 0
    res = {}
    for t in t_snap:
        k0 = t / dt0
        if abs(k0 - round(k0)) > 1e-9:
            raise ValueError("snapshot times must be multiples of the "
                             "coarsest time step")
        target = int(round(k0)) * 2 ** dm
        sim.step(target - done)
        done = target
        d = sim.diagnostics()
        ey = sim.read_total_field("ey")
        ex = sim.read_total_field("ex")
        row = {"ey_axis": axis_row(ey, ny // 2, "ey"),
               "ex_axis": axis_row(ex, ny // 2, "ex"),
               "w_kin": d["w_kin"], "w_em": d["w_em_total"],
               "nx": nx, "ny": ny, "h": h}
        if keep_planes:
            row.update(ey_total=ey, ex_total=ex)
        res[t] = row
    return res


def study_cross_errors_2d(study_i: Dict[int, Dict[float, dict]],
                          study_ii: Dict[int, Dict[float, dict]]
                          ) -> Dict[int, Dict[float, dict]]:
    """Per m and snapshot time, the Sec. 3.2 comparison of model (i) with
    model (ii) as the reference: relative intensity error "dI" and relative
    Frobenius errors "dEy", "dEx"."""
    out: Dict[int, Dict[float, dict]] = {}
    for m in study_i:
        out[m] = {}
        for t, a in study_i[m].items():
            b = study_ii[m][t]
            nx, ny = a["nx"], a["ny"]
            out[m][t] = {
                "dI": intensity_error(a["ey_total"], a["ex_total"],
                                      b["ey_total"], b["ex_total"], nx, ny),
                "dEy": frobenius_error(a["ey_total"], b["ey_total"], nx, ny,
                                       "ey"),
                "dEx": frobenius_error(a["ex_total"], b["ex_total"], nx, ny,
                                       "ex")}
    return out


def study_axis_norms(study: Dict[int, Dict[float, dict]], comp: str = "ey"
                     ) -> Dict[float, List[float]]:
    """Norms along the beam axis of every resolution but the finest against
    the finest (E_y primal in x, E_x dual), per snapshot time."""
    ms = sorted(study)
    ref = ms[-1]
    out = {}
    for t in study[ref]:
        fine = study[ref][t]
        norms = []
        for m in ms[:-1]:
            c = study[m][t]
            ratio = 2 ** (ref - m)
            norms.append(l2_norm(c[comp + "_axis"], fine[comp + "_axis"],
                                 ratio, c["nx"], c["h"],
                                 dual=(comp == "ex")))
        out[t] = norms
    return out
