"""Seeded synthetic inputs shaped like the paper's workloads.

This module generates inputs only: grids, species placement and the incident
beam parameters of each workload.  It holds none of the method's arithmetic
(no field solver, interpolation, push or deposition) and is the one module
shared by the oracle harness and the HIP path.

Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11), keyed by (seed, species index) with the
counter (particle id low, particle id high, stream, 0).  Stream 0 gives the two
in-cell position uniforms, streams 1 and 2 the uniforms of a Box-Muller pair
each (thermal momenta).  The device generator in the library implements the
same published definition.

Units are the paper's normalized plasma units (Table 1): lengths in
lambda/(2 pi), times in 1/omega, densities in n_c, E in m_e c omega / e.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

TWO_PI = 2.0 * math.pi
ME_C2_EV = 510998.95  # electron rest energy in eV (unit conversion only)

PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85

INC_NONE, INC_PLANE_PULSE_1D, INC_APRIL_LP, INC_APRIL_RP = 0, 1, 2, 3
INC_GAUSS_2D = 4  # paraxial 2D Gaussian beam (Sec. 3.2)
FP64, FP32 = 0, 1


def philox4x32_10(ctr: np.ndarray, key: Tuple[int, int]) -> np.ndarray:
    """Philox4x32 with 10 rounds.  ctr: uint32 array (..., 4); key: 2 words."""
    c = [ctr[..., i].astype(np.uint64) for i in range(4)]
    k0 = np.uint64(key[0] & 0xFFFFFFFF)
    k1 = np.uint64(key[1] & 0xFFFFFFFF)
    mask = np.uint64(0xFFFFFFFF)
    m0 = np.uint64(PHILOX_M0)
    m1 = np.uint64(PHILOX_M1)
    for r in range(10):
        if r > 0:
            k0 = (k0 + np.uint64(PHILOX_W0)) & mask
            k1 = (k1 + np.uint64(PHILOX_W1)) & mask
        p0 = m0 * c[0]
        p1 = m1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & mask
        hi1, lo1 = p1 >> np.uint64(32), p1 & mask
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack([x.astype(np.uint32) for x in c], axis=-1)


def u01_pair(r: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Two uniforms in [0, 1) with 53 random bits each from 4 words."""
    scale = 1.0 / 9007199254740992.0  # 2^-53
    a = ((r[..., 0] >> np.uint32(5)).astype(np.float64) * 67108864.0 +
         (r[..., 1] >> np.uint32(6)).astype(np.float64)) * scale
    b = ((r[..., 2] >> np.uint32(5)).astype(np.float64) * 67108864.0 +
         (r[..., 3] >> np.uint32(6)).astype(np.float64)) * scale
    return a, b


def _counters(pid: np.ndarray, stream: int) -> np.ndarray:
    ctr = np.zeros(pid.shape + (4,), dtype=np.uint32)
    ctr[..., 0] = (pid & 0xFFFFFFFF).astype(np.uint32)
    ctr[..., 1] = (pid >> 32).astype(np.uint32)
    ctr[..., 2] = stream
    return ctr


@dataclasses.dataclass
class Grid:
    dims: int
    nx: int
    ny: int
    dx: float
    dy: float
    dt: float


@dataclasses.dataclass
class Species:
    q: float = -1.0
    m: float = 1.0
    density: float = 0.01          # n_c units
    region: Tuple[int, int, int, int] = (0, 0, 0, 1)  # cells [x0,x1) x [y0,y1)
    ppc: int = 1
    temperature_ev: float = 0.0    # 0: cold
    seed: int = 0
    species_index: int = 0
    # density profile along x (PROFILE_*): super-Gaussian parameters
    profile: int = 0
    profile_center: float = 0.0
    profile_fwhm: float = 0.0
    profile_order: float = 0.0
    profile_xmin: float = 0.0

    @property
    def weight(self) -> float:
        """Density carried by one macro-particle (n / ppc)."""
        return self.density / self.ppc

    def count(self, dx: float = 0.0) -> int:
        """Particles placed (dx, the cell size along x, is needed only with a
        density profile)."""
        x0, x1, y0, y1 = self.region
        if self.profile:
            return int(profile_offsets(self, x0, x1, dx)[-1]) * (y1 - y0)
        return (x1 - x0) * (y1 - y0) * self.ppc


@dataclasses.dataclass
class Incident:
    kind: int = INC_NONE
    a0: float = 0.0
    fwhm_t: float = 0.0
    t0: float = 0.0
    w0: float = 0.0
    s: float = 10.0
    phi0: float = 0.0
    x_focus: float = 0.0
    y_focus: float = 0.0
    t_focus: float = 0.0
    # 0: closed form at each particle; 1: sampled on the Yee nodes at t^n
    # and gathered with the scattered field
    on_nodes: int = 0
    z_focus: float = 0.0  # 3D runs: focus coordinate along z


@dataclasses.dataclass
class Workload:
    name: str
    grid: Grid
    species: List[Species]
    incident: Incident
    steps: int
    precision: int = FP64


PROFILE_UNIFORM, PROFILE_SUPERGAUSS = 0, 1


def profile_factor(sp, x: float) -> float:
    """Sec. 3.1 plasma profile along x relative to the peak density:
    2^{-|2 (x - centre) / FWHM|^order} beyond x_min, else 0."""
    if not x > sp.profile_xmin:
        return 0.0
    return math.pow(2.0, -math.pow(abs(2.0 * (x - sp.profile_center) /
                                       sp.profile_fwhm), sp.profile_order))


def profile_offsets(sp, x0: int, x1: int, dx: float) -> np.ndarray:
    """Column offsets: column c of [x0, x1) holds floor(ppc f(x_c) + 1/2)
    particles per cell, x_c its centre (the library computes the same table
    on the host)."""
    if sp.profile != PROFILE_SUPERGAUSS:
        raise ValueError("unknown density profile")
    counts = [math.floor(sp.ppc * profile_factor(sp, (c + 0.5) * dx) + 0.5)
              for c in range(x0, x1)]
    return np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)


def _profile_cells(sp, pid, x0, x1, nrows, dx):
    """(column, row) of particle ids under a density profile: rows outer,
    columns inner, a column's particles consecutive."""
    off = profile_offsets(sp, x0, x1, dx)
    per_row = int(off[-1])
    row = pid // per_row
    r = pid - row * per_row
    col = np.searchsorted(off, r, side="right") - 1
    return x0 + col, row


def generate_particles(sp: Species, grid: Grid, first: int = 0,
                       count: Optional[int] = None):
    """Positions and momenta of particles first .. first+count-1 of a species.

    Exactly ppc particles per cell of the region, each uniform in its cell;
    particle id = (cell row * cells per row + cell column) * ppc + k.
    Returns (x, y, ux, uy, uz) float64 arrays in physical units.
    """
    x0, x1, y0, y1 = sp.region
    ncx = x1 - x0
    total = sp.count(grid.dx)
    if count is None:
        count = total - first
    pid = np.arange(first, first + count, dtype=np.int64)
    if sp.profile:
        cx, row = _profile_cells(sp, pid, x0, x1, y1 - y0, grid.dx)
        cy = y0 + row
    else:
        cell = pid // sp.ppc
        cx = x0 + cell % ncx
        cy = y0 + cell // ncx
    key = (sp.seed, sp.species_index)
    ua, ub = u01_pair(philox4x32_10(_counters(pid, 0), key))
    x = (cx + ua) * grid.dx
    y = (cy + ub) * grid.dy if grid.dims == 2 else np.zeros(count)
    if sp.temperature_ev > 0.0:
        sigma = math.sqrt(sp.temperature_ev / (ME_C2_EV * sp.m))
        a1, b1 = u01_pair(philox4x32_10(_counters(pid, 1), key))
        a2, b2 = u01_pair(philox4x32_10(_counters(pid, 2), key))
        r1 = np.sqrt(-2.0 * np.log1p(-a1))
        r2 = np.sqrt(-2.0 * np.log1p(-a2))
        ux = sigma * r1 * np.cos(TWO_PI * b1)
        uy = sigma * r1 * np.sin(TWO_PI * b1)
        uz = sigma * r2 * np.cos(TWO_PI * b2)
    else:
        ux = np.zeros(count)
        uy = np.zeros(count)
        uz = np.zeros(count)
    return x, y, ux, uy, uz


# ---------------------------------------------------------------------------
# Workloads shaped like the paper's (Secs. 3.1, 3.2, 4): names say what they are
# ---------------------------------------------------------------------------

def plane_pulse_1d(nx=2048, steps=2000, slab=(768, 1280), n=0.01, ppc=64,
                   a0=1.0, cycles=5.0, seed=1, cfl=0.95,
                   cells_per_lambda=32) -> Workload:
    """1D3V slab hit by the exact plane-wave pulse (Sec. 3.1 model (ii))."""
    dx = TWO_PI / cells_per_lambda
    grid = Grid(1, nx, 1, dx, dx, cfl * dx)
    fwhm = cycles * TWO_PI
    x_front = slab[0] * dx
    inc = Incident(kind=INC_PLANE_PULSE_1D, a0=a0, fwhm_t=fwhm,
                   t0=fwhm - x_front)
    sp = Species(q=-1.0, m=1.0, density=n, region=(slab[0], slab[1], 0, 1),
                 ppc=ppc, seed=seed)
    return Workload(f"plane_pulse_1d_{nx}", grid, [sp], inc, steps)


def gauss_beam_2d(nx=1024, ny=512, plasma=(384, 640, 128, 384), n=0.31,
                  ppc=8, w0_lambda=16.0, cycles=1.0, a0=4.86, steps=400,
                  seed=6, cells_per_lambda=16, cfl=0.99) -> Workload:
    """2D3V plasma in the paraxial Gaussian beam of Sec. 3.2 (w0 = 16
    lambda, FWHM_T = 2 pi, E0 = 4.86 there), focused at the centre of the
    plasma block, the envelope's peak at the focus at t = 0."""
    dx = TWO_PI / cells_per_lambda
    grid = Grid(2, nx, ny, dx, dx, cfl * dx / math.sqrt(2.0))
    inc = Incident(kind=INC_GAUSS_2D, a0=a0, w0=w0_lambda * TWO_PI,
                   fwhm_t=cycles * TWO_PI, t0=0.0,
                   x_focus=0.5 * (plasma[0] + plasma[1]) * dx,
                   y_focus=0.5 * (plasma[2] + plasma[3]) * dx)
    sp = Species(q=-1.0, m=1.0, density=n, region=plasma, ppc=ppc, seed=seed)
    return Workload(f"gauss_beam_2d_{nx}x{ny}", grid, [sp], inc, steps)


def april_2d(nx=2048, ny=1024, plasma=(512, 1536, 0, 1024), n=0.05, ppc=16,
             kind=INC_APRIL_LP, w0_lambda=1.0, s=20.0, a0=10.0,
             temperature_ev=1.0, steps=1500, seed=2, cells_per_lambda=32,
             precision=FP64, cfl=0.95) -> Workload:
    """2D3V plasma block in a tightly focused April beam (Sec. 4 set-up,
    evaluated on the plane through the axis); focus at the box centre, focal
    time such that the pulse peak is 2 wavelengths before the plasma front at
    t = 0."""
    dx = TWO_PI / cells_per_lambda
    grid = Grid(2, nx, ny, dx, dx, cfl * dx / math.sqrt(2.0))
    x_f = 0.5 * nx * dx
    y_f = 0.5 * ny * dx
    x_front = plasma[0] * dx
    inc = Incident(kind=kind, a0=a0, w0=w0_lambda * TWO_PI, s=s,
                   x_focus=x_f, y_focus=y_f,
                   t_focus=(x_f - x_front) + 2.0 * TWO_PI)
    sp = Species(q=-1.0, m=1.0, density=n, region=plasma, ppc=ppc,
                 temperature_ev=temperature_ev, seed=seed)
    pol = "lp" if kind == INC_APRIL_LP else "rp"
    return Workload(f"april_{pol}_2d_{nx}x{ny}_ppc{ppc}", grid, [sp], inc,
                    steps, precision)


def lp_2048x1024() -> Workload:
    """2D3V FP64: 2048x1024 cells at lambda/32, 16.8M electrons (16 ppc, 1 eV)
    in the central 1024x1024 cells at 0.05 n_c, LP beam w0 = lambda, s = 20,
    a0 = 10, 1500 steps."""
    return april_2d()


def rp_4096_fp32() -> Workload:
    """2D3V FP32 form: 4096^2 cells at lambda/48, 134M cold electrons (32 ppc)
    in the central 2048^2 cells at 0.02 n_c, RP beam w0 = 0.8 lambda, s = 10,
    a0 = 30, 3000 steps."""
    return april_2d(nx=4096, ny=4096, plasma=(1024, 3072, 1024, 3072), n=0.02,
                    ppc=32, kind=INC_APRIL_RP, w0_lambda=0.8, s=10.0, a0=30.0,
                    temperature_ev=0.0, steps=3000, seed=3,
                    cells_per_lambda=48, precision=FP32)


def sweep_member(i: int, precision=FP32, steps=800) -> Workload:
    """Member i of the laser-focus / density sweep: grid side in
    {256, 512, 768, 1024}, central (side/2)^2 plasma, density log-uniform in
    [0.001, 0.1] n_c, w0 uniform in [0.6, 2] lambda, a0 uniform in [5, 50],
    LP or RP with probability 1/2, 8..32 ppc, s = 10, cold."""
    r = philox4x32_10(np.array([[i, 0, 0, 0], [i, 0, 1, 0]], dtype=np.uint32),
                      (4, 0xC0FFEE))
    u = np.concatenate(u01_pair(r))  # 4 uniforms
    side = 256 * (1 + int(u[0] * 4))
    dens = math.exp(math.log(0.001) + u[1] * (math.log(0.1) - math.log(0.001)))
    w0 = 0.6 + 1.4 * u[2]
    a0 = 5.0 + 45.0 * u[3]
    extra = u01_pair(philox4x32_10(np.array([[i, 0, 2, 0]], dtype=np.uint32),
                                   (4, 0xC0FFEE)))
    kind = INC_APRIL_LP if extra[0][0] < 0.5 else INC_APRIL_RP
    ppc = 8 + int(extra[1][0] * 25)
    q = side // 4
    wl = april_2d(nx=side, ny=side, plasma=(q, 3 * q, q, 3 * q), n=dens,
                  ppc=ppc, kind=kind, w0_lambda=w0, s=10.0, a0=a0,
                  temperature_ev=0.0, steps=steps, seed=(4 << 16) | i,
                  precision=precision)
    wl.name = f"sweep_{i}_{wl.name}"
    return wl


def big_sweep_member(i: int, precision=FP32, steps=800) -> Workload:
    """A large request of the served sweep: 2048^2 cells, 16 ppc in the
    central 1024^2 cells, beam and density drawn as for sweep_member."""
    wl = sweep_member(i, precision, steps)
    inc = wl.incident
    sp = wl.species[0]
    kind = inc.kind
    w0_lambda = inc.w0 / TWO_PI
    big = april_2d(nx=2048, ny=2048, plasma=(512, 1536, 512, 1536),
                   n=sp.density, ppc=16, kind=kind, w0_lambda=w0_lambda,
                   s=10.0, a0=inc.a0, temperature_ev=0.0, steps=steps,
                   seed=(5 << 16) | i, precision=precision)
    big.name = f"sweep_big_{i}_{big.name}"
    return big


def served_sweep(rate=20.0, window=60.0, seed=5, big_fraction=0.1,
                 precision=FP32, steps=800):
    """Poisson arrivals of sweep requests over `window` seconds: a list of
    (arrival time in s, workload).  A fraction `big_fraction` are 2048^2
    requests (big_sweep_member), the rest sweep_member draws."""
    out = []
    t = 0.0
    i = 0
    while True:
        r = philox4x32_10(np.array([[i, 0, 0, 0]], dtype=np.uint32),
                          (seed, 0xA221))
        u_gap, u_big = u01_pair(r)
        t += -math.log1p(-float(u_gap[0])) / rate
        if t >= window:
            break
        if float(u_big[0]) < big_fraction:
            out.append((t, big_sweep_member(i, precision, steps)))
        else:
            out.append((t, sweep_member(i, precision, steps)))
        i += 1
    return out


# ---------------------------------------------------------------------------
# 3D3V inputs (Sec. 4 runs the method in 3D): seeded grids and particles
# shared by the oracle and the library.
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Grid3:
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    dt: float


@dataclasses.dataclass
class Species3:
    """A species generated on the device in 3D: ppc per cell of region
    (x0, x1, y0, y1, z0, z1)."""
    q: float = -1.0
    m: float = 1.0
    density: float = 0.01
    region: Tuple[int, int, int, int, int, int] = (0, 1, 0, 1, 0, 1)
    ppc: int = 1
    temperature_ev: float = 0.0
    seed: int = 0
    profile: int = 0
    profile_center: float = 0.0
    profile_fwhm: float = 0.0
    profile_order: float = 0.0
    profile_xmin: float = 0.0

    def count(self, dx: float = 0.0) -> int:
        x0, x1, y0, y1, z0, z1 = self.region
        if self.profile:
            return int(profile_offsets(self, x0, x1, dx)[-1]) * \
                (y1 - y0) * (z1 - z0)
        return (x1 - x0) * (y1 - y0) * (z1 - z0) * self.ppc


def grid3(nx, ny, nz, h=2 * math.pi / 16, cfl=0.99):
    """Cubic cells of size h and dt = cfl h / sqrt(3) (Sec. 4 uses 0.99)."""
    return Grid3(nx, ny, nz, h, h, h, cfl * h / math.sqrt(3.0))


def plasma3d(seed, grid, region, ppc, u_sigma=0.0, q=-1.0, m=1.0,
             density=0.3):
    """Explicit particles: ppc per cell of region (x0, x1, y0, y1, z0, z1)
    at uniform random positions in the cell, momenta normal with width
    u_sigma (cold when 0); returns the dict the oracle and the binding take."""
    rng = np.random.default_rng(seed)
    x0, x1, y0, y1, z0, z1 = region
    cz, cy, cx = np.meshgrid(np.arange(z0, z1), np.arange(y0, y1),
                             np.arange(x0, x1), indexing="ij")
    cells = [np.repeat(c.ravel(), ppc) for c in (cx, cy, cz)]
    n = cells[0].size
    h = (grid.dx, grid.dy, grid.dz)
    pos = [(cells[d] + rng.uniform(0.0, 1.0, n)) * h[d] for d in range(3)]
    u = rng.normal(0.0, u_sigma, (3, n)) if u_sigma > 0 else np.zeros((3, n))
    return {"q": q, "m": m, "weight": density / ppc, "x": pos[0],
            "y": pos[1], "z": pos[2], "ux": u[0], "uy": u[1], "uz": u[2]}


def paper3d_lp(cells_per_lambda=16, ppc=2, a0=10.0):
    """Sec. 4 3D run: the box 2 pi [24, 24, 32] at Delta = 2 pi /
    cells_per_lambda (16: 512 x 384 x 384 cells; 32, the paper's finer
    resolution: 1024 x 768 x 768) with propagation along x; cold electrons with
    peak density n_e0 = 0.31 n_c in the Sec. 3.1 super-Gaussian profile along
    x (order 12, centre 281.5, FWHM 335.1, zero for x <= 20 pi: in this box
    its rising side, half maximum at x = 114), uniform across; ppc (unstated
    in the paper) at the peak, fewer where the profile is lower; tight April
    LP beam, w0 = 0.8 lambda, s = 20, focused on the axis at the profile's
    half-maximum point at t = 60 dt.  Returns (grid, species, incident) for
    binding.Simulation3."""
    c = int(cells_per_lambda)
    nx, ny, nz = 32 * c, 24 * c, 24 * c
    g = grid3(nx, ny, nz, h=2 * math.pi / c)
    xmin = 20 * math.pi
    x_half = 281.5 - 335.1 / 2
    sp = Species3(q=-1.0, m=1.0, density=0.31,
                  region=(int(xmin / g.dx), nx, 0, ny, 0, nz), ppc=ppc,
                  temperature_ev=0.0, seed=1, profile=PROFILE_SUPERGAUSS,
                  profile_center=281.5, profile_fwhm=335.1, profile_order=12.0,
                  profile_xmin=xmin)
    inc = Incident(kind=INC_APRIL_LP, a0=a0, w0=0.8 * 2 * math.pi, s=20.0,
                   x_focus=x_half, y_focus=ny / 2 * g.dy,
                   z_focus=nz / 2 * g.dz, t_focus=60 * g.dt)
    return g, sp, inc
