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

Periodic boundaries ("DMI and boundary conditions": periodic boundaries
also change the magnetostatic field; the paper gives no formula, so this is
a reading, listed with the others): along an axis with R >= 1 image
repetitions the convolution is cyclic with period n (no padding), and the
kernel at the offset X (the nearest image, -n/2 < X <= n/2) is the sum of
N(X + k n d) over k = -R..R.  At X = n/2 (n even) the offsets +n/2 and
-n/2 are the same cyclic index; it holds their mean, which keeps every
component's parity (zero for a component odd along that axis) and the
spectrum real.  ``direct_sum_periodic`` writes this out as a double sum.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from .constants import MU0
from .tensor import PARITY, COMPONENTS, demag_tensor, tensor_at


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


def _axis_terms(i, n, P, R):
    """(offset in cells, weight) pairs that make up kernel index i of one axis."""
    if R == 0:
        if P == 1:
            return [(0, 1.0)]
        if i < n:
            return [(i, 1.0)]
        if i > P - n:
            return [(i - P, 1.0)]
        return []
    if 2 * i == n:
        return [(s * (n // 2) + k * n, 0.5) for s in (1, -1) for k in range(-R, R + 1)]
    X = i if 2 * i < n else i - n
    return [(X + k * n, 1.0) for k in range(-R, R + 1)]


def periodic_kernel(n, d, P, pbc):
    """The tensor on the cyclic grid of shape P = (Px, Py, Pz), shape
    (6, Pz, Py, Px), with image sums on the periodic axes."""
    idx, off, wt = [], [], []
    terms = [[_axis_terms(i, n[a], P[a], pbc[a]) for i in range(P[a])] for a in range(3)]
    for iz in range(P[2]):
        for iy in range(P[1]):
            for ix in range(P[0]):
                for oz, wz in terms[2][iz]:
                    for oy, wy in terms[1][iy]:
                        for ox, wx in terms[0][ix]:
                            idx.append((iz, iy, ix))
                            off.append((ox * d[0], oy * d[1], oz * d[2]))
                            wt.append(wx * wy * wz)
    K = np.zeros((6, P[2], P[1], P[0]))
    if not idx:
        return K
    idx = np.array(idx)
    off = np.array(off)
    vals = tensor_at(off[:, 0], off[:, 1], off[:, 2], d) * np.array(wt)[None]
    for c in range(6):
        np.add.at(K[c], (idx[:, 0], idx[:, 1], idx[:, 2]), vals[c])
    return K


class Demag:
    """Precomputed tensor spectrum for one grid; call ``field(M)``."""

    def __init__(self, n, d, N6=None, workers=None, pbc=(0, 0, 0)):
        self.n = tuple(n)
        self.d = tuple(d)
        self.pbc = tuple(pbc)
        self.P = tuple(v if r > 0 else pad_len(v) for v, r in zip(self.n, self.pbc))
        self.workers = workers
        if any(self.pbc):
            self.N6 = None
            K = periodic_kernel(self.n, self.d, self.P, self.pbc)
        else:
            self.N6 = demag_tensor(self.n, self.d) if N6 is None else N6
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


def direct_sum_periodic(M, d, pbc):
    """The periodic convolution as a plain double sum over cell pairs and
    images (tiny grids): per axis the nearest-image offset of i - j, image
    sums over k = -R..R, the mean of +-n/2 at the half-period offset."""
    _, nz, ny, nx = M.shape
    n = (nx, ny, nz)
    B = np.zeros_like(M, dtype=np.float64)

    def terms(a, delta):
        R, L = pbc[a], n[a]
        if R == 0:
            return [(delta, 1.0)]
        X = delta % L
        if 2 * X == L:
            return [(X + k * L, 0.5) for k in range(-R, R + 1)] + \
                   [(X - L + k * L, 0.5) for k in range(-R, R + 1)]
        if 2 * X > L:
            X -= L
        return [(X + k * L, 1.0) for k in range(-R, R + 1)]

    for zi in range(nz):
        for yi in range(ny):
            for xi in range(nx):
                acc = np.zeros(3)
                for zj in range(nz):
                    for yj in range(ny):
                        for xj in range(nx):
                            Nm = np.zeros((3, 3))
                            for oz, wz in terms(2, zi - zj):
                                for oy, wy in terms(1, yi - yj):
                                    for ox, wx in terms(0, xi - xj):
                                        v = tensor_at([ox * d[0]], [oy * d[1]], [oz * d[2]], d)[:, 0]
                                        w = wx * wy * wz
                                        Nm += w * np.array([[v[0], v[3], v[4]],
                                                            [v[3], v[1], v[5]],
                                                            [v[4], v[5], v[2]]])
                            acc += Nm @ M[:, zj, yj, xj]
                B[:, zi, yi, xi] = -MU0 * acc
    return B
