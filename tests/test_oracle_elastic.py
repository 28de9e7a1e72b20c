"""Pins for the oracle's elastodynamics (not GPU).

* The first-derivative operator is exact on polynomials of degree <= 4 in
  the bulk, <= 2 one cell in from a face and <= 1 on a face cell.
* The paper's racetrack demonstration (Table 1 parameters for NiO) prints
  a shear pulse travelling at about 4 km/s with a strain of about 0.14 %
  for a 0.3 GPa shear traction; a bar driven by one period of that traction
  through the oracle reproduces both numbers.
* With no damping, no coupling and no drive the elastic energy
  1/2 sigma:eps + 1/2 rho v^2 of an interior pulse is conserved.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import elastic as el
from oracle.system import Problem
from paper_2411_18194_amd import inputs


def test_derivative_polynomial_exactness():
    n, h = 12, 0.7
    x = np.arange(n) * h
    for deg in range(5):
        f = x ** deg
        df = deg * x ** (deg - 1) if deg else 0 * x
        d = el.deriv(f, 0, h)
        bulk = slice(2, n - 2)
        assert np.allclose(d[bulk], df[bulk], rtol=1e-12, atol=1e-9)
        if deg <= 2:
            assert np.allclose(d[[1, n - 2]], df[[1, n - 2]], rtol=1e-12, atol=1e-9)
        if deg <= 1:
            assert np.allclose(d[[0, n - 1]], df[[0, n - 1]], rtol=1e-12, atol=1e-9)
    # a single cell has no derivative
    assert el.deriv(np.ones((1, 3)), 0, 1.0).max() == 0.0


with open(os.path.join(os.path.dirname(__file__), "golden", "paper_printed.json")) as _fh:
    NIO = json.load(_fh)["nio_racetrack"]


def _nio_bar(nx, dx):
    p = inputs.base_params((nx, 1, 1), (dx, dx, dx))
    # the paper's NiO table: rho, C11, C12, C44; magnetisation switched off
    p.update(Ms=[0.0], elastic=dict(rho=NIO["rho_kg_m3"], C11=NIO["C11_Pa"], C12=NIO["C12_Pa"],
                                    C44=NIO["C44_Pa"], eta=0.0,
                                    trac_amp=NIO["traction_amplitude_Pa"],
                                    trac_freq=NIO["traction_frequency_Hz"]))
    return p


def test_printed_racetrack_numbers():
    nx, dx = 400, 3e-9
    p = _nio_bar(nx, dx)
    P = Problem(p)
    m = np.zeros((1, 3, 1, 1, nx))
    m[0, 2] = 1.0
    y = P.initial_state(m)
    # one period of the 8 GHz drive, then switch it off and let it travel
    dt = 1e-13
    nper = int(round(NIO["traction_periods"] / NIO["traction_frequency_Hz"] / dt))
    y, t = P.run_fixed(y, 0.0, dt, nper)
    P.p = dict(p)
    P.p["elastic"] = dict(p["elastic"], trac_amp=0.0)
    P.stepper.invalidate()
    t1 = t
    y, t = P.run_fixed(y, t, dt, 600)
    uz = y[1][2, 0, 0, :]
    eps_xz = el.strain(y[1], p["cell"])[4, 0, 0, :]
    # pulse front position: the leading edge where |u_z| rises above 1 %
    x = (np.arange(nx) + 0.5) * dx
    front = x[np.nonzero(np.abs(uz) > 0.01 * np.abs(uz).max())[0].max()]
    speed = front / t
    c_shear = math.sqrt(NIO["C44_Pa"] / NIO["rho_kg_m3"])
    # "about 4 km/s": the printed speed to its one significant digit
    assert c_shear == pytest.approx(NIO["pulse_speed_m_s_about"], rel=0.05)
    assert speed == pytest.approx(c_shear, rel=0.06)
    assert speed == pytest.approx(NIO["pulse_speed_m_s_about"], rel=0.1)
    # strain amplitude in the travelling pulse: sigma/(2 C44) ~ 0.136 %
    amp = NIO["traction_amplitude_Pa"] / (2 * NIO["C44_Pa"])
    assert np.abs(eps_xz).max() == pytest.approx(amp, rel=0.06)
    # "approximately 0.14 %"
    assert abs(np.abs(eps_xz).max() * 100 - NIO["strain_amplitude_percent_about"]) < 0.01


def test_energy_conservation_free_pulse():
    nx, dx = 200, 2e-9
    p = _nio_bar(nx, dx)
    p["elastic"] = dict(p["elastic"], trac_amp=0.0)
    P = Problem(p)
    m = np.zeros((1, 3, 1, 1, nx))
    m[0, 2] = 1.0
    y = P.initial_state(m)
    x = np.arange(nx) * dx
    y[1][2, 0, 0, :] = 1e-11 * np.exp(-((x - 200e-9) / 20e-9) ** 2)
    y[1][0, 0, 0, :] = 5e-12 * np.exp(-((x - 200e-9) / 25e-9) ** 2)
    E0 = P.energies(y[0], y[1], y[2])["elastic"]
    y, t = P.run_fixed(y, 0.0, 2e-14, 500)
    E1 = P.energies(y[0], y[1], y[2])["elastic"]
    assert E1 == pytest.approx(E0, rel=1e-5)


def test_printed_rayleigh_damping_ratio():
    """A free-free standing shear wave of 24 nm wavelength decays with the
    damping ratio beta*omega/2 of stiffness-proportional (Kelvin-Voigt)
    damping, and the printed coefficient gives the printed ~5 %."""
    dx = 1e-9
    lam = NIO["rayleigh_shear_wavelength_m"]
    nx = int(round(2 * lam / dx))                  # two wavelengths, free ends
    p = _nio_bar(nx, dx)
    beta = NIO["rayleigh_stiffness_coefficient_s"]
    p["elastic"] = dict(p["elastic"], trac_amp=0.0, rayleigh=beta)
    P = Problem(p)
    m = np.zeros((1, 3, 1, 1, nx))
    m[0, 2] = 1.0
    y = P.initial_state(m)
    k = 2 * math.pi / lam
    phi = np.cos(k * (np.arange(nx) + 0.5) * dx)
    y[1][2, 0, 0, :] = 1e-12 * phi
    dt = 2e-14
    amp, ts = [], []
    t = 0.0
    for _ in range(120):
        y, t = P.run_fixed(y, t, dt, 5)
        amp.append(float(y[1][2, 0, 0, :] @ phi / (phi @ phi)))
        ts.append(t)
    amp, ts = np.array(amp), np.array(ts)
    # local extrema of the modal amplitude: their spacing is half a damped
    # period, the log of their magnitudes falls at rate zeta*omega
    ext = [i for i in range(1, len(amp) - 1)
           if (amp[i] - amp[i - 1]) * (amp[i + 1] - amp[i]) < 0]
    te, ae = ts[ext], np.log(np.abs(amp[ext]))
    omega = math.pi / np.mean(np.diff(te))
    slope = np.polyfit(te, ae, 1)[0]
    zeta = -slope / omega
    c = math.sqrt(NIO["C44_Pa"] / NIO["rho_kg_m3"])
    assert omega == pytest.approx(k * c, rel=0.03)
    assert zeta == pytest.approx(beta * k * c / 2, rel=0.08)
    assert zeta == pytest.approx(NIO["rayleigh_damping_ratio_about"], abs=0.008)
    # without the viscous stress the same wave does not decay
    p["elastic"] = dict(p["elastic"], rayleigh=0.0)
    P0 = Problem(p)
    y0 = P0.initial_state(m)
    y0[1][2, 0, 0, :] = 1e-12 * phi
    y0, _ = P0.run_fixed(y0, 0.0, dt, 600)
    E = P0.energies(y0[0], y0[1], y0[2])["elastic"]
    assert E > 0.98 * P0.energies(m, 1e-12 * np.stack([0 * phi, 0 * phi, phi])[:, None, None, :],
                                  np.zeros((3, 1, 1, nx)))["elastic"]
