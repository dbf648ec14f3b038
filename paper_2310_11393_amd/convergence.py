"""Convergence analysis of the scattered-field step (Sec. 3.1).

The paper measures how solutions at cell size h = 2 pi / (16 2^m) approach
the finest one, taken as exact:

  ||dE(., t_n)||_{2,h} = ( h sum_k |E^h(x_k, t_n) - E^exact(x_k, t_n)|^2 )^(1/2)

over the grid points the two resolutions share, and the numerical rate
p = log2( ||dE||_{2,h} / ||dE||_{2,h/2} ).

In the scattered-field form the incident field is the same closed form on
every grid, so differences of the total field equal differences of the
scattered field that the library stores; this module compares those.  The
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


def refinement_study_1d(ms: Sequence[int], length: float, a0: float,
                        fwhm_t: float, t0: float, density: float, ppc: int,
                        center: float, fwhm: float, order: float,
                        xmin: float, t_snap: Sequence[float],
                        cfl: float = 0.99) -> Dict[int, Dict[float, dict]]:
    """Run the 1D scattered-field set-up of Sec. 3.1 at cell sizes
    2 pi / (16 2^m) for m in ms through the library (FP64) and return, per
    m and snapshot time, the scattered E_x and E_y rows (guards included)
    and the cell count.  Snapshot times must be multiples of the coarsest
    time step so that every resolution reaches them exactly."""
    from .binding import Simulation
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
        sim = Simulation(grid, inc, explicit=[e])
        done = 0
        res = {}
        for t in t_snap:
            k0 = t / dt0
            if abs(k0 - round(k0)) > 1e-9:
                raise ValueError("snapshot times must be multiples of the "
                                 "coarsest time step")
            target = int(round(k0)) * 2 ** (m - m0)
            sim.step(target - done)
            done = target
            res[t] = {"ex": sim.read_field("ex")[0],
                      "ey": sim.read_field("ey")[0], "nx": nx, "h": h}
        sim.close()
        out[m] = res
    return out


def study_norms(study: Dict[int, Dict[float, dict]], comp: str = "ey"
                ) -> Dict[float, List[float]]:
    """Norms of every resolution but the finest against the finest, per
    snapshot time (component ey, the transverse field, is primal; ex, the
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
                                 dual=(comp == "ex")))
        out[t] = norms
    return out
