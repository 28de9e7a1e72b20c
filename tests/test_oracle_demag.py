"""Pins for the oracle's FFT demagnetising field (not GPU).

* The zero-padded FFT convolution equals the plain double sum
  B_i = -mu0 sum_j N(r_i - r_j) M_j on tiny grids whose sizes give every
  small pad length.
* A uniformly magnetised prism has energy 1/2 mu0 Ms^2 V N_prism with
  N_prism the analytic self-term of the whole prism.
* The operator is self-adjoint: sum M . B(M') = sum M' . B(M).
* A wide thin film magnetised out of plane has B_z -> -mu0 Ms inside.
"""
import itertools
import math

import numpy as np
import pytest

from oracle.constants import MU0
from oracle import demag as dm
from oracle import tensor as T


@pytest.mark.parametrize("n", [(1, 1, 1), (2, 1, 1), (3, 2, 1), (4, 3, 2),
                               (5, 1, 3), (2, 5, 4), (7, 3, 1), (3, 3, 3)])
def test_fft_equals_direct_sum(n):
    d = (2e-9, 3e-9, 2.5e-9)
    rng = np.random.default_rng(sum(n))
    M = rng.standard_normal((3,) + n[::-1]) * 8e5
    D = dm.Demag(n, d)
    B1 = D.field(M)
    B2 = dm.direct_sum(M, D.N6)
    assert np.abs(B1 - B2).max() < 1e-13 * np.abs(B2).max()


@pytest.mark.parametrize("n,d", [((8, 6, 2), (2e-9,) * 3),
                                 ((16, 4, 1), (7.8125e-9, 7.8125e-9, 3e-9))])
def test_uniform_prism_energy(n, d):
    Ms = 8e5
    D = dm.Demag(n, d)
    nx, ny, nz = n
    V = d[0] * d[1] * d[2]
    big = T.newell_tensor(0, 0, 0, (nx * d[0], ny * d[1], nz * d[2])).ravel()
    for axis in range(3):
        M = np.zeros((3,) + n[::-1])
        M[axis] = Ms
        B = D.field(M)
        E = -0.5 * np.sum(M * B) * V
        Eref = 0.5 * MU0 * Ms ** 2 * (nx * ny * nz * V) * big[axis]
        assert E == pytest.approx(Eref, rel=1e-12)


def test_self_adjoint():
    n, d = (6, 5, 3), (2e-9, 2.5e-9, 3e-9)
    rng = np.random.default_rng(7)
    M1 = rng.standard_normal((3,) + n[::-1])
    M2 = rng.standard_normal((3,) + n[::-1])
    D = dm.Demag(n, d)
    a = np.sum(M1 * D.field(M2))
    b = np.sum(M2 * D.field(M1))
    assert a == pytest.approx(b, rel=1e-12)


def test_thin_film_limit():
    n, d = (64, 64, 1), (5e-9, 5e-9, 1e-9)
    Ms = 1e6
    M = np.zeros((3,) + n[::-1])
    M[2] = Ms
    B = dm.Demag(n, d).field(M)
    centre = B[2, 0, 32, 32]
    assert -MU0 * Ms < centre < -0.99 * MU0 * Ms
