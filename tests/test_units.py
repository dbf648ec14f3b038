"""Physical-unit front end of the April beams (Sec. 4.1): the library's
peak-power integral (sfpic_april_power) against an independent quadrature
of the oracle's fields, limits it must reach, and the paper's printed
example.  Host code only: no GPU is used."""
import math

import numpy as np
import pytest

import oracle
from paper_2310_11393_amd import units
from paper_2310_11393_amd import workloads as wl

TWO_PI = 2.0 * math.pi


def _oracle_power(kind, w0, s, half=8.0, per_w0=24):
    """(1/2) int Re{E_x cB_y* - E_y cB_x*} dx dy over the focal plane at the
    focal time, a0 = 1, from the oracle's complex April fields (trapezoid on
    a square of half-side `half` w0, `per_w0` nodes per w0)."""
    inc = wl.Incident(kind=kind, a0=1.0, w0=w0, s=s)
    norm = oracle.incident_norm(inc)
    ka = oracle.ka_from_w0(w0)
    h = w0 / per_w0
    n = int(round(half * per_w0))
    xs = np.arange(-n, n + 1) * h
    wts = np.ones(len(xs))
    wts[0] = wts[-1] = 0.5
    tot = 0.0
    for j, y in enumerate(xs):
        for i, x in enumerate(xs):
            e, b = oracle.april_complex(kind, x / ka, y / ka, 0.0, 0.0, ka, s)
            f = (e[0] * np.conj(b[1]) - e[1] * np.conj(b[0])).real
            tot += wts[i] * wts[j] * f
    return 0.5 * tot * h * h * norm * norm


@pytest.mark.parametrize("kind,w0,s", [(wl.INC_APRIL_LP, TWO_PI, 10.0),
                                       (wl.INC_APRIL_RP, 0.8 * TWO_PI, 20.0)])
def test_library_power_matches_oracle_quadrature(kind, w0, s):
    from paper_2310_11393_amd import binding
    p = binding.april_power(wl.Incident(kind=kind, a0=1.0, w0=w0, s=s))
    q = _oracle_power(kind, w0, s, half=8.0, per_w0=24)
    assert p > 0 and abs(p - q) <= 1e-10 * q, (p, q)
    # the power scales with a0^2
    p3 = binding.april_power(wl.Incident(kind=kind, a0=3.0, w0=w0, s=s))
    assert abs(p3 - 9.0 * p) <= 1e-12 * p3


def test_power_reaches_the_gaussian_beam_limit():
    """Weak focusing and a long pulse: the beam is a paraxial Gaussian of
    waist w0, whose power is pi w0^2 / 2 times the peak cycle-averaged
    intensity a0^2 / 2.  A 2-cycle pulse (s = 10) carries less: each
    frequency of the isodiffracting pulse has its own waist."""
    ka = 200.0
    w0 = math.sqrt(2.0 * (math.sqrt(1.0 + ka * ka) - 1.0))
    gauss = math.pi * w0 * w0 / 4.0
    long_pulse = _oracle_power(wl.INC_APRIL_LP, w0, 640.0, half=4.0,
                               per_w0=12)
    short_pulse = _oracle_power(wl.INC_APRIL_LP, w0, 10.0, half=4.0,
                                per_w0=12)
    assert 0.99 < long_pulse / gauss < 1.02
    assert short_pulse / gauss < 0.9


def test_unit_conversions():
    """m_e c omega / e at 0.8 um is 4.01e12 V/m, and a0 = 1 of linear
    polarization is I lambda^2 = 1.37e18 W/cm^2 um^2."""
    assert abs(units.field_unit(0.8) / 4.013e12 - 1) < 1e-3
    for lam in (0.8, 1.8):
        i = units.peak_intensity_w_cm2(1.0, lam) * lam * lam
        assert abs(i / 1.37e18 - 1) < 5e-3
    assert abs(units.time_fs(units.omega(0.8) * 1e-15, 0.8) - 1.0) < 1e-12
    assert abs(units.length_um(TWO_PI, 1.8) - 1.8) < 1e-12


def test_paper_peak_intensity_example():
    """Sec. 4.2: an LP pulse of 2e11 W peak power at 1.8 um, 2 cycles (s =
    10), focused to a 2 um FWHM spot, reaches 4.8e18 W/cm^2 at the focus in
    vacuum.  Readings: the FWHM is that of |E|^2 in the focal plane, mean of
    the two transverse axes; the intensity is eps0 c |E|^2 / 2 at the peak.
    They give 4.43e18 (8% below the printed value)."""
    lam = 1.8
    inc = wl.Incident(kind=wl.INC_APRIL_LP, a0=1.0, w0=TWO_PI, s=10.0)
    inc.w0 = units.w0_for_focal_fwhm(inc, 2.0 * TWO_PI / lam)
    fx, fy = units.focal_fwhm(inc)
    assert abs(units.length_um(0.5 * (fx + fy), lam) - 2.0) < 1e-6
    a0 = units.a0_from_peak_power(inc, 2e11, lam)
    i = units.peak_intensity_w_cm2(a0, lam)
    assert abs(i / 4.8e18 - 1) < 0.10, i
