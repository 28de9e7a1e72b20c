"""Pins for the oracle's demagnetising tensor (not GPU).

What fixes the tensor independently of the oracle's own formulas:
* a cube's self-term is 1/3 per axis by symmetry, and tr N(0) = 1 for any
  cuboid (Gauss: the trace of the cell-averaged kernel is the volume average
  of the delta term);
* away from the origin the point kernel is traceless, so tr N(R) = 0;
* the parity of each component (diagonal even, xy odd in X and Y, ...);
* the point-dipole limit -(V/4pi)(3 R_i R_j - delta_ij R^2)/R^5;
* high-precision (50-digit) evaluation of Newell's formula shows the FP64
  rounding error where the near regime is used;
* the pair-sum identity: the self-term of a whole prism of cells equals the
  average over its cell pairs of the cell-cell tensor.  A prism long enough
  to contain offsets in all three regimes pins all of them at once.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import tensor as T


CELLS = [(2e-9, 2e-9, 2e-9), (7.8125e-9, 7.8125e-9, 3e-9), (1e-9, 2e-9, 3.5e-9)]


def test_cube_self_term():
    N = T.newell_tensor(0.0, 0.0, 0.0, (2e-9,) * 3).ravel()
    assert np.allclose(N[:3], 1.0 / 3.0, rtol=0, atol=2e-15)
    assert np.all(np.abs(N[3:]) < 1e-15)


@pytest.mark.parametrize("d", CELLS)
def test_trace_one_at_origin(d):
    N = T.tensor_at(0.0, 0.0, 0.0, d).ravel()
    assert abs(N[:3].sum() - 1.0) < 1e-14


def test_thin_cell_self_term_limits():
    # a flat cell is mostly Nzz, a long needle along x has Nxx -> 0
    n1 = T.newell_tensor(0, 0, 0, (100e-9, 100e-9, 1e-9)).ravel()
    n2 = T.newell_tensor(0, 0, 0, (1000e-9, 1000e-9, 1e-9)).ravel()
    assert 0.95 < n1[2] < n2[2] and n2[2] > 0.99 and n2[0] < 0.005
    N = T.newell_tensor(0, 0, 0, (100e-9, 1e-9, 1e-9)).ravel()
    assert N[0] < 0.01 and abs(N[1] - 0.5) < 0.01


@pytest.mark.parametrize("d", CELLS)
def test_traceless_away_from_origin(d):
    m = max(d)
    rng = np.random.default_rng(0)
    # offsets on the integer lattice in all three regimes
    pts = [(1, 0, 0), (1, 1, 0), (2, 1, 1), (3, 2, 0), (5, 1, 1), (12, 7, 2),
           (30, 20, 3), (45, 3, 1), (60, 40, 2)]
    for p in pts:
        R = np.array(p) * np.array(d)
        N = T.tensor_at(*R, d).ravel()
        scale = (d[0] * d[1] * d[2]) / (4 * math.pi) / np.linalg.norm(R) ** 3
        assert abs(N[:3].sum()) < 1e-9 * scale + 1e-15, p


@pytest.mark.parametrize("d", CELLS)
def test_parity(d):
    R = np.array([2, 1, 1]) * np.array(d)
    for X, Y, Z in [(2, 1, 1), (5, 3, 2), (50, 7, 1)]:
        base = T.tensor_at(X * d[0], Y * d[1], Z * d[2], d).ravel()
        for sx in (1, -1):
            for sy in (1, -1):
                for sz in (1, -1):
                    v = T.tensor_at(sx * X * d[0], sy * Y * d[1], sz * Z * d[2], d).ravel()
                    for c, (px, py, pz) in T.PARITY.items():
                        s = (px if sx < 0 else 1) * (py if sy < 0 else 1) * (pz if sz < 0 else 1)
                        assert v[c] == pytest.approx(s * base[c], rel=1e-13, abs=2e-15)


@pytest.mark.parametrize("d", CELLS)
def test_point_dipole_limit(d):
    V = d[0] * d[1] * d[2]
    for rcells in (200.0, 1000.0):
        u = np.array([0.6, 0.48, 0.64])
        R = rcells * max(d) * u
        N = T.tensor_at(*R, d).ravel()
        r = np.linalg.norm(R)
        dip = -(V / (4 * math.pi)) * np.array([
            3 * R[0] * R[0] - r * r, 3 * R[1] * R[1] - r * r, 3 * R[2] * R[2] - r * r,
            3 * R[0] * R[1], 3 * R[0] * R[2], 3 * R[1] * R[2]]) / r ** 5
        rel = np.abs(N - dip).max() / np.abs(dip).max()
        assert rel < 2.0 / rcells ** 2


def _mp_f(x, y, z):
    x, y, z = abs(x), abs(y), abs(z)
    R = mp.sqrt(x * x + y * y + z * z)
    out = (2 * x * x - y * y - z * z) * R / 6
    if y * (z * z - x * x) != 0:
        out += y / 2 * (z * z - x * x) * mp.asinh(y / mp.sqrt(x * x + z * z))
    if z * (y * y - x * x) != 0:
        out += z / 2 * (y * y - x * x) * mp.asinh(z / mp.sqrt(x * x + y * y))
    if x * y * z != 0:
        out -= x * y * z * mp.atan(y * z / (x * R))
    return out


def _mp_g(x, y, z):
    s = mp.sign(x) * mp.sign(y)
    x, y, z = abs(x), abs(y), abs(z)
    R = mp.sqrt(x * x + y * y + z * z)
    out = -x * y * R / 3
    if x * y * z != 0:
        out += x * y * z * mp.asinh(z / mp.sqrt(x * x + y * y))
    if y * (3 * z * z - y * y) != 0:
        out += y / 6 * (3 * z * z - y * y) * mp.asinh(x / mp.sqrt(y * y + z * z))
    if x * (3 * z * z - x * x) != 0:
        out += x / 6 * (3 * z * z - x * x) * mp.asinh(y / mp.sqrt(x * x + z * z))
    if z != 0:
        out -= z ** 3 / 6 * mp.atan(x * y / (z * R))
    if z * y != 0:
        out -= z * y * y / 2 * mp.atan(x * z / (y * R))
    if z * x != 0:
        out -= z * x * x / 2 * mp.atan(y * z / (x * R))
    return s * out


def _mp_second_diff(fun, X, Y, Z, dx, dy, dz):
    w = {-1: -1, 0: 2, 1: -1}
    acc = mp.mpf(0)
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            for c in (-1, 0, 1):
                acc += w[a] * w[b] * w[c] * fun(X + a * dx, Y + b * dy, Z + c * dz)
    return acc / (4 * mp.pi * dx * dy * dz)


@pytest.mark.parametrize("d", CELLS[:2])
def test_near_regime_fp64_rounding(d):
    """FP64 Newell within a few 1e-15 of 50-digit arithmetic where it is used."""
    mp.mp.dps = 50
    dx, dy, dz = (mp.mpf(v) for v in d)
    for (X, Y, Z) in [(0, 0, 0), (1, 0, 0), (1, 1, 0), (2, 1, 1), (2, 2, 0)]:
        Xm, Ym, Zm = X * dx, Y * dy, Z * dz
        ref = [
            _mp_second_diff(_mp_f, Xm, Ym, Zm, dx, dy, dz),
            _mp_second_diff(_mp_f, Ym, Xm, Zm, dy, dx, dz),
            _mp_second_diff(_mp_f, Zm, Ym, Xm, dz, dy, dx),
            _mp_second_diff(_mp_g, Xm, Ym, Zm, dx, dy, dz),
            _mp_second_diff(_mp_g, Xm, Zm, Ym, dx, dz, dy),
            _mp_second_diff(_mp_g, Ym, Zm, Xm, dy, dz, dx),
        ]
        got = T.newell_tensor(X * d[0], Y * d[1], Z * d[2], d).ravel()
        for c in range(6):
            assert abs(got[c] - float(ref[c])) < 5e-15, (X, Y, Z, c)
        # the exact values also carry the invariants
        if (X, Y, Z) == (0, 0, 0):
            assert abs(float(ref[0] + ref[1] + ref[2]) - 1) < 1e-40
        else:
            assert abs(float(ref[0] + ref[1] + ref[2])) < 1e-40


@pytest.mark.parametrize("d", CELLS[:2])
def test_regimes_agree_at_cutoffs(d):
    m = max(d)
    for R in [(3.0 * m, 0, 0), (2.2 * m, 2.0 * m, 0.5 * m), (4 * m, 1 * m, 0)]:
        a = T.newell_tensor(*R, d).ravel()
        b = T.quad_tensor(*R, d).ravel()
        assert np.abs(a - b).max() < 2e-14
    for R in [(40.0 * m, 0, 0), (30 * m, 26.5 * m, 3 * m)]:
        b = T.quad_tensor(*R, d).ravel()
        c = T.moment_tensor(*R, d).ravel()
        assert np.abs(b - c).max() < 1e-10 * np.abs(b).max()


def test_quadrature_converged():
    """Doubling the Gauss points changes nothing at FP64 level."""
    for d in CELLS:
        m = max(d)
        for R in [(3.0 * m, 0.1 * m, 0), (5 * m, 3 * m, 1 * m)]:
            a = T.quad_tensor(*R, d).ravel()
            b = T.quad_tensor(*R, d, n=24).ravel()
            assert np.abs(a - b).max() < 1e-16


@pytest.mark.parametrize("shape,d", [((64, 2, 1), (2e-9, 2e-9, 2e-9)),
                                     ((12, 10, 3), (2e-9, 2e-9, 2e-9)),
                                     ((56, 4, 1), (7.8125e-9, 7.8125e-9, 3e-9))])
def test_pair_sum_identity(shape, d):
    """sum_{i,j in prism} N(r_i - r_j)/ncell = Newell self-term of the prism."""
    nx, ny, nz = shape
    N6 = T.demag_tensor(shape, d)
    tot = np.zeros(3)
    for Z in range(nz):
        for Y in range(ny):
            for X in range(nx):
                mult = ((nx - X) * (2 if X else 1) * (ny - Y) * (2 if Y else 1)
                        * (nz - Z) * (2 if Z else 1))
                tot += mult * N6[:3, Z, Y, X]
    tot /= nx * ny * nz
    big = T.newell_tensor(0, 0, 0, (nx * d[0], ny * d[1], nz * d[2])).ravel()[:3]
    assert np.abs(tot - big).max() < 1e-12
    assert abs(tot.sum() - 1.0) < 1e-12
