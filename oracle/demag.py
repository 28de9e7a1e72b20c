"""Demagnetising field by zero-padded FFT convolution (FP64).

Methods, "Magnetostatic field": B_d(r_i) = -mu0 sum_j N(r_i - r_j) M_j, with
M = sum_s Ms^(s) m^(s) for a multi-sublattice magnet (the cell's spins are
summed before the field is evaluated) and the same B_d acting on every
sublattice.  Open boundaries: the convolution is linear, made cyclic by
zero-padding each axis to P = 2n (P = 1 when n = 1), which is >= 2n - 1 so
no wrapped term overlaps.  The tensor is placed with wrap (offset k at index
k, offset -k at index P - k) and both factors are transformed with
scipy.fft.rfftn; the product is transformed back and cropped to [0, n).

``direct_sum`` is the same convolution written as the plain double sum; the
tests use it on tiny grids to pin the FFT path.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from .constants import MU0
from .tensor import PARITY, COMPONENTS, demag_tensor


def pad_len(n: int) -> int:
    return 1 if n == 1 else 2 * n


def _sym_index(c):
    """Map (i, j) -> component index in (xx, yy, zz, xy, xz, yz)."""
    table = {}
    for k, (i, j) in enumerate(COMPONENTS):
        table[(i, j)] = k
        table[(j, i)] = k
    return table[c]


def wrapped_kernel(N6, n, P):
    """Place the octant table on the padded grid, shape (6, Pz, Py, Px)."""
    nx, ny, nz = n
    Px, Py, Pz = P
    K = np.zeros((6, Pz, Py, Px))
    for c in range(6):
        sx, sy, sz = PARITY[c]
        for zs in (1, -1):
            for ys in (1, -1):
                for xs in (1, -1):
                    s = 1.0
                    if xs < 0:
                        s *= sx
                    if ys < 0:
                        s *= sy
                    if zs < 0:
                        s *= sz
                    zi = np.arange(nz) if zs > 0 else (Pz - np.arange(1, nz)) % Pz
                    yi = np.arange(ny) if ys > 0 else (Py - np.arange(1, ny)) % Py
                    xi = np.arange(nx) if xs > 0 else (Px - np.arange(1, nx)) % Px
                    zsrc = np.arange(nz) if zs > 0 else np.arange(1, nz)
                    ysrc = np.arange(ny) if ys > 0 else np.arange(1, ny)
                    xsrc = np.arange(nx) if xs > 0 else np.arange(1, nx)
                    if len(zi) == 0 or len(yi) == 0 or len(xi) == 0:
                        continue
                    K[c][np.ix_(zi, yi, xi)] = s * N6[c][np.ix_(zsrc, ysrc, xsrc)]
    return K


class Demag:
    """Precomputed tensor spectrum for one grid; call ``field(M)``."""

    def __init__(self, n, d, N6=None, workers=None):
        self.n = tuple(n)
        self.d = tuple(d)
        self.P = tuple(pad_len(v) for v in self.n)
        self.N6 = demag_tensor(self.n, self.d) if N6 is None else N6
        self.workers = workers
        Px, Py, Pz = self.P
        K = wrapped_kernel(self.N6, self.n, self.P)
        self.Kf = sfft.rfftn(K, axes=(1, 2, 3), workers=workers)

    def field(self, M):
        """B_d (T) from M (A/m), both shape (3, nz, ny, nx)."""
        nx, ny, nz = self.n
        Px, Py, Pz = self.P
        Mp = np.zeros((3, Pz, Py, Px))
        Mp[:, :nz, :ny, :nx] = M
        Mf = sfft.rfftn(Mp, axes=(1, 2, 3), workers=self.workers)
        Bf = np.zeros_like(Mf)
        for i in range(3):
            for j in range(3):
                Bf[i] += self.Kf[_sym_index((i, j))] * Mf[j]
        B = sfft.irfftn(Bf, s=(Pz, Py, Px), axes=(1, 2, 3), workers=self.workers)
        return -MU0 * B[:, :nz, :ny, :nx]


def direct_sum(M, N6):
    """B_d = -mu0 sum_j N(r_i - r_j) M_j by explicit loops (tiny grids)."""
    _, nz, ny, nx = M.shape
    B = np.zeros_like(M, dtype=np.float64)
    for zi in range(nz):
        for yi in range(ny):
            for xi in range(nx):
                acc = np.zeros(3)
                for zj in range(nz):
                    for yj in range(ny):
                        for xj in range(nx):
                            X, Y, Z = xi - xj, yi - yj, zi - zj
                            nn = np.empty(6)
                            for c in range(6):
                                sx, sy, sz = PARITY[c]
                                s = (sx if X < 0 else 1) * (sy if Y < 0 else 1) \
                                    * (sz if Z < 0 else 1)
                                nn[c] = s * N6[c, abs(Z), abs(Y), abs(X)]
                            Nm = np.array([[nn[0], nn[3], nn[4]],
                                           [nn[3], nn[1], nn[5]],
                                           [nn[4], nn[5], nn[2]]])
                            acc += Nm @ M[:, zj, yj, xj]
                B[:, zi, yi, xi] = -MU0 * acc
    return B
