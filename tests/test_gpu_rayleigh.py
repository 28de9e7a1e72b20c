"""GPU parity of the elastic strain-rate (Rayleigh) damping.

The viscous stress beta C : eps(v) joins the elastic stress before the
traction rows and the divergence.  Checks: fixed FP64 steps of the
magnetoelastic crop with random displacement and velocity (max |dm| <=
1e-12, u and v within 1e-12 of their largest value), and 600 steps of the
free-free 24 nm standing shear wave of the NiO bar, whose modal amplitude
and elastic energy match the oracle's run (FP64, relative 1e-10).
"""
import json
import math
import os

import numpy as np
import pytest

from oracle.system import Problem
from paper_2411_18194_amd import inputs, mmp

pytestmark = pytest.mark.gpu

with open(os.path.join(os.path.dirname(__file__), "golden", "paper_printed.json")) as fh:
    NIO = json.load(fh)["nio_racetrack"]


def test_fixed_steps_crop_fp64():
    p, m = inputs.config_c4_crop()
    p = dict(p)
    p["elastic"] = dict(p["elastic"], rayleigh=NIO["rayleigh_stiffness_coefficient_s"])
    nx, ny, nz = p["n"]
    r = inputs.rng(15)
    u = 1e-12 * r.standard_normal((3, nz, ny, nx))
    v = 1e-3 * r.standard_normal((3, nz, ny, nx))
    g = mmp.Grid(p, mmp.FP64)
    g.set_state(m, u, v)
    g.run_fixed(1e-14, 4)
    mg, ug, vg, _, _ = g.get_state()
    g.close()
    P = Problem(p)
    y, _ = P.run_fixed([m, u, v], 0.0, 1e-14, 4)
    assert np.abs(mg - y[0]).max() < 1e-12
    assert np.abs(ug - y[1]).max() <= 1e-12 * np.abs(y[1]).max()
    assert np.abs(vg - y[2]).max() <= 1e-12 * np.abs(y[2]).max()


def test_standing_shear_wave_decay():
    dx, lam = 1e-9, NIO["rayleigh_shear_wavelength_m"]
    nx = int(round(2 * lam / dx))
    p = inputs.base_params((nx, 1, 1), (dx, dx, dx))
    p.update(Ms=[0.0], elastic=dict(rho=NIO["rho_kg_m3"], C11=NIO["C11_Pa"],
                                    C12=NIO["C12_Pa"], C44=NIO["C44_Pa"], eta=0.0,
                                    trac_amp=0.0, trac_freq=0.0,
                                    rayleigh=NIO["rayleigh_stiffness_coefficient_s"]))
    m = np.zeros((1, 3, 1, 1, nx))
    m[0, 2] = 1.0
    phi = np.cos(2 * math.pi / lam * (np.arange(nx) + 0.5) * dx)
    u = np.zeros((3, 1, 1, nx))
    u[2, 0, 0] = 1e-12 * phi
    v = np.zeros_like(u)
    g = mmp.Grid(p, mmp.FP64)
    g.set_state(m, u, v)
    g.run_fixed(2e-14, 600)
    _, ug, vg, _, _ = g.get_state()
    _, e = g.eval_heff(mmp.T_ALL, want_b=False)
    g.close()
    P = Problem(p)
    y, _ = P.run_fixed([m, u, v], 0.0, 2e-14, 600)
    a_gpu = ug[2, 0, 0] @ phi / (phi @ phi)
    a_ref = y[1][2, 0, 0] @ phi / (phi @ phi)
    assert a_gpu == pytest.approx(a_ref, rel=1e-10)
    assert np.abs(ug - y[1]).max() <= 1e-10 * np.abs(y[1]).max()
    Eref = P.energies(y[0], y[1], y[2])["elastic"]
    assert e["elastic"] == pytest.approx(Eref, rel=1e-10)
    # two damped periods take away most of the wave's energy
    E0 = P.energies(m, u, v)["elastic"]
    assert Eref < 0.5 * E0
