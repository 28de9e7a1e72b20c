"""Pins for the oracle's periodic boundaries (not GPU).

* Exchange, DMI and the Zhang-Li derivative of spirals whose period divides
  the periodic length match their discrete closed forms at every cell,
  boundary cells included (with Neumann ghosts they do not); so does the
  whole Zhang-Li torque of a helix (both of its terms, any alpha and xi).
* The periodic demag field by FFT equals the plain double sum over cell
  pairs and images (tiny grids, odd and even lengths, so the half-period
  offset is covered).
* Trace identity: for uniform M along x, y and z in turn, the three
  demagnetising factors of every cell sum to 1 (the cell lies inside the
  symmetric image box the kernel sums over), whatever the repetitions.
* Thin film periodic in x and y: N_zz -> 1 and N_xx, N_yy -> 0 as the
  repetitions grow, monotonically; the field of a uniform state is uniform.
* Cyclic translation along a periodic axis translates the field.
"""
import math

import numpy as np
import pytest

from oracle import fields as fl
from oracle import torque as tq
from oracle.constants import MU0
from oracle.demag import Demag, direct_sum_periodic
from oracle.system import Problem
from paper_2411_18194_amd import inputs

PX = (True, False, False)


def _spiral(n, d, period_cells, plane=(0, 1)):
    k = 2 * math.pi / (period_cells * d[0])
    x = np.arange(n[0]) * d[0]
    m = np.zeros((3, n[2], n[1], n[0]))
    m[plane[0]] = np.cos(k * x)
    m[plane[1]] = np.sin(k * x)
    return k, x, m


def test_exchange_spiral_periodic_all_cells():
    n, d = (24, 3, 2), (1e-9, 1.5e-9, 2e-9)
    k, x, m = _spiral(n, d, 8)
    A, Ms = 1.3e-11, 8e5
    ref = -(2 * A / Ms) * (2 - 2 * math.cos(k * d[0])) / d[0] ** 2 * m
    B = fl.exchange_field(m, Ms, A, d, periodic=PX)
    assert np.abs(B - ref).max() < 1e-12 * np.abs(ref).max()
    # Neumann ghosts break it at the x faces
    Bn = fl.exchange_field(m, Ms, A, d)
    assert np.abs(Bn - ref).max() > 1e-3 * np.abs(ref).max()
    # same for the inter-sublattice term
    Bp = fl.afm_nn_field(m, Ms, -5e-12, d, periodic=PX)
    refp = -(-5e-12 / Ms) * (2 - 2 * math.cos(k * d[0])) / d[0] ** 2 * m
    assert np.abs(Bp - refp).max() < 1e-12 * np.abs(refp).max()


def test_dmi_cycloid_periodic_all_cells():
    n, d = (30, 4, 1), (2e-9, 2e-9, 2e-9)
    k, x, m = _spiral(n, d, 10, plane=(0, 2))
    D, Ms, A = 3e-3, 1.1e6, 1.5e-11
    B = fl.dmi_field(m, Ms, A, D, d, periodic=(True, True, False))
    ref = (2 * D / Ms) * math.sin(k * d[0]) / d[0] * np.stack(
        [np.cos(k * x), 0 * x, np.sin(k * x)])[:, None, None, :]
    assert np.abs(B - np.broadcast_to(ref, B.shape)).max() < 1e-12 * np.abs(ref).max()


def test_zhang_li_derivative_periodic():
    n, d = (16, 2, 1), (1e-9, 1e-9, 1e-9)
    k, x, m = _spiral(n, d, 4)
    u = (3.0, 0.0, 0.0)
    dm = tq.directional_derivative(m, u, d, periodic=PX)
    s = math.sin(k * d[0]) / d[0]
    ref = 3.0 * s * np.stack([-np.sin(k * x), np.cos(k * x), 0 * x])[:, None, None, :]
    assert np.abs(dm - np.broadcast_to(ref, dm.shape)).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("alpha,xi", [(0.02, 0.1), (0.3, 0.05), (0.1, 0.1)])
def test_zhang_li_torque_helix_closed_form(alpha, xi):
    """Periodic in-plane helix phi = k x, drift u along x: with a = (u.grad) m,
    m x a = u s z and m x (m x a) = -a (s = sin(k dx)/dx), so the torque is
    [(1 + xi alpha) a - (xi - alpha) u s z] / (1 + alpha^2) at every cell;
    for xi = alpha it is the pure advection a."""
    n, d = (24, 2, 1), (1.5e-9, 1e-9, 1e-9)
    k, x, m = _spiral(n, d, 8)
    ux = -40.0
    tau = tq.zhang_li_torque(m, (ux, 0.0, 0.0), alpha, xi, d, periodic=PX)
    s = math.sin(k * d[0]) / d[0]
    a = ux * s * np.stack([-np.sin(k * x), np.cos(k * x), 0 * x])
    zhat = np.stack([0 * x, 0 * x, 1 + 0 * x])
    ref = ((1 + xi * alpha) * a - (xi - alpha) * ux * s * zhat) / (1 + alpha * alpha)
    ref = np.broadcast_to(ref[:, None, None, :], tau.shape)
    assert np.abs(tau - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("n,pbc", [((4, 3, 2), (2, 0, 0)), ((3, 4, 1), (1, 2, 0))])
def test_fft_equals_direct_sum(n, pbc):
    d = (2e-9, 3e-9, 1.5e-9)
    M = inputs.rng(50).standard_normal((3, n[2], n[1], n[0])) * 8e5
    B1 = Demag(n, d, pbc=pbc).field(M)
    B2 = direct_sum_periodic(M, d, pbc)
    assert np.abs(B1 - B2).max() <= 1e-13 * np.abs(B2).max()


def _factors(n, d, pbc):
    D = Demag(n, d, pbc=pbc)
    out = np.zeros((3,) + (n[2], n[1], n[0]))
    for c in range(3):
        M = np.zeros((3, n[2], n[1], n[0]))
        M[c] = 1.0
        out[c] = -D.field(M)[c] / MU0
    return out


@pytest.mark.parametrize("n,pbc", [((6, 4, 2), (3, 0, 0)), ((5, 6, 3), (0, 2, 0)),
                                   ((4, 4, 2), (2, 1, 0))])
def test_trace_identity(n, pbc):
    f = _factors(n, (2e-9, 2.5e-9, 1e-9), pbc)
    assert np.abs(f.sum(axis=0) - 1.0).max() < 1e-12


def test_thin_film_limit():
    n, d = (8, 8, 1), (2e-9, 2e-9, 2e-9)
    prev = None
    for R in (1, 4, 16):
        f = _factors(n, d, (R, R, 0))
        # a uniform state of a periodic film feels a uniform field
        assert np.ptp(f[2]) < 1e-12 and np.ptp(f[0]) < 1e-12
        nzz, nxx = f[2].mean(), f[0].mean()
        if prev is not None:
            assert nzz > prev[0] and nxx < prev[1]
        prev = (nzz, nxx)
    assert prev[0] > 0.995 and prev[1] < 0.0025


def test_cyclic_translation():
    n, d = (6, 5, 2), (2e-9, 2e-9, 3e-9)
    D = Demag(n, d, pbc=(2, 0, 0))
    M = inputs.rng(51).standard_normal((3, n[2], n[1], n[0]))
    B = D.field(M)
    Bs = D.field(np.roll(M, 2, axis=3))
    assert np.abs(Bs - np.roll(B, 2, axis=3)).max() < 1e-12 * np.abs(B).max()
    # along the open y axis a translation is not a symmetry
    By = D.field(np.roll(M, 1, axis=2))
    assert np.abs(By - np.roll(B, 1, axis=2)).max() > 1e-3 * np.abs(B).max()


def test_problem_rejects_unsupported():
    p = inputs.base_params((4, 4, 2), (1e-9,) * 3)
    p.update(pbc=(0, 0, 1))
    with pytest.raises(ValueError):
        Problem(p)
