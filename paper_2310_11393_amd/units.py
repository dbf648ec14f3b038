"""Physical units for the April beams (Sec. 4.1).

The library works in normalized units: lengths in 1/k, times in 1/omega,
fields in m_e c omega / e, densities in n_c (Table 1).  This module converts
a beam given as the paper gives it -- wavelength, peak power, focal spot --
to the incident parameters of the library, and back to SI quantities.  The
peak power fixes the amplitude through the cycle-averaged Poynting flux
through the focal plane at the focal time (Sec. 4.1), which the library
integrates (sfpic_april_power).
"""
from __future__ import annotations

import copy
import math

from . import binding

# CODATA 2018
C_LIGHT = 299792458.0          # m/s
E_CHARGE = 1.602176634e-19     # C
M_E = 9.1093837015e-31         # kg
EPS0 = 8.8541878128e-12        # F/m


def omega(lambda_um: float) -> float:
    """Angular frequency (rad/s) of the wavelength in micrometres."""
    return 2.0 * math.pi * C_LIGHT / (lambda_um * 1e-6)


def field_unit(lambda_um: float) -> float:
    """m_e c omega / e in V/m: the field of normalized amplitude 1."""
    return M_E * C_LIGHT * omega(lambda_um) / E_CHARGE


def power_unit(lambda_um: float) -> float:
    """eps0 c (m_e c omega / e)^2 / k^2 in W: the unit of sfpic_april_power."""
    k = omega(lambda_um) / C_LIGHT
    return EPS0 * C_LIGHT * field_unit(lambda_um) ** 2 / (k * k)


def length_um(x: float, lambda_um: float) -> float:
    """Normalized length (1/k) in micrometres."""
    return x * lambda_um / (2.0 * math.pi)


def time_fs(t: float, lambda_um: float) -> float:
    """Normalized time (1/omega) in femtoseconds."""
    return t / omega(lambda_um) * 1e15


def a0_from_peak_power(incident, p_peak_w: float, lambda_um: float) -> float:
    """Amplitude a0 (library convention: the modulus of the on-axis field
    component at the focus at the focal time) of the April beam `incident`
    (kind, w0, s; its own a0 is ignored) that carries the peak power
    p_peak_w watts at the wavelength lambda_um."""
    unit = copy.copy(incident)
    unit.a0 = 1.0
    p1 = binding.april_power(unit)
    return math.sqrt(p_peak_w / (power_unit(lambda_um) * p1))


def peak_intensity_w_cm2(a0: float, lambda_um: float) -> float:
    """Cycle-averaged intensity eps0 c |E|^2 / 2 at a field modulus of a0
    (normalized), in W/cm^2."""
    e = a0 * field_unit(lambda_um)
    return 0.5 * EPS0 * C_LIGHT * e * e * 1e-4


def focal_intensity(incident, x: float, y: float) -> float:
    """|E|^2 of the beam in the focal plane at the focal time, at (x, y)
    from the axis (paper axes, normalized)."""
    e, _ = binding.april_field(incident, x, y, 0.0, 0.0)
    return float(sum(abs(c) ** 2 for c in e))


def focal_fwhm(incident) -> tuple:
    """Full widths at half maximum of |E|^2 in the focal plane along the
    polarization axis x and across it (y), normalized lengths."""
    i0 = focal_intensity(incident, 0.0, 0.0)

    def half(axis):
        lo, hi = 0.0, 1.0
        while focal_intensity(incident, *(hi, 0.0)[::axis]) > 0.5 * i0:
            hi *= 2.0
        for _ in range(60):
            mid = 0.5 * (lo + hi)
            if focal_intensity(incident, *(mid, 0.0)[::axis]) > 0.5 * i0:
                lo = mid
            else:
                hi = mid
        return 2.0 * 0.5 * (lo + hi)
    return half(1), half(-1)


def w0_for_focal_fwhm(incident, fwhm: float) -> float:
    """Waist parameter w0 (normalized) for which the mean of the two focal
    FWHM of |E|^2 equals `fwhm` (normalized), by bisection on w0."""
    beam = copy.copy(incident)

    def mean_fwhm(w0):
        beam.w0 = w0
        fx, fy = focal_fwhm(beam)
        return 0.5 * (fx + fy)
    lo, hi = 0.05 * fwhm, 5.0 * fwhm
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if mean_fwhm(mid) < fwhm:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)
