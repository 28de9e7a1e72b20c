"""Stray field of the magnet in a layer of cells above it (FP64).

Test infrastructure: only tests/, the package's smoke check and the
benchmark's CPU baseline use this module.

The paper images a film by the out-of-plane stray field at a height above
its surface ("Stray field imaging of the non-collinear antiferromagnet
Mn3Sn"), with the magnetostatic field of "Magnetostatic field"
(B = -mu0 sum_j N(r - r_j) M_j, M = sum_s Ms^(s) m^(s)).  Reading: the field
is averaged over a layer of cells of the grid's own size whose centres lie
`height` above the top surface, so the cell-pair tensor N of the demag
kernel applies at the vertical offsets Z = z_t - z dz, z_t = (nz - 1/2) dz +
height (layer 0 centred at z = 0); a height of dz/2 + k dz puts the layer
on the grid's own lattice, k layers above the top one.  Per source layer
the in-plane sum is a 2-D linear convolution, done by zero-padded FFTs.

Pins (tests/test_oracle_stray.py): the FFT path equals the plain double
sum; at height dz/2 + k dz it equals the demag field of the grid extended
by empty layers; far above one magnetised cell it is the point-dipole field.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from .constants import MU0
from .tensor import tensor_at


def target_z(nz, dz, height):
    return (nz - 0.5) * dz + height


def _offsets(n, P):
    """Signed cell offset of each index of a zero-padded axis (None: unused)."""
    out = []
    for i in range(P):
        if i < n:
            out.append(i)
        elif i > P - n:
            out.append(i - P)
        else:
            out.append(None)
    return out


def stray_field(M, d, height):
    """B (3, ny, nx) in tesla from M (3, nz, ny, nx) in A/m."""
    _, nz, ny, nx = M.shape
    dx, dy, dz = d
    Px = 1 if nx == 1 else 2 * nx
    Py = 1 if ny == 1 else 2 * ny
    ox, oy = _offsets(nx, Px), _offsets(ny, Py)
    zt = target_z(nz, dz, height)
    Bf = np.zeros((3, Py, Px // 2 + 1), dtype=np.complex128)
    comp = {(0, 0): 0, (1, 1): 1, (2, 2): 2, (0, 1): 3, (1, 0): 3, (0, 2): 4, (2, 0): 4,
            (1, 2): 5, (2, 1): 5}
    for z in range(nz):
        iy, ix = np.meshgrid(np.arange(Py), np.arange(Px), indexing="ij")
        valid = np.array([[ox[a] is not None and oy[b] is not None for a in range(Px)]
                          for b in range(Py)])
        X = np.array([[ox[a] if ox[a] is not None else 0 for a in range(Px)]
                      for b in range(Py)], dtype=np.float64) * dx
        Y = np.array([[oy[b] if oy[b] is not None else 0 for a in range(Px)]
                      for b in range(Py)], dtype=np.float64) * dy
        Z = np.full_like(X, zt - z * dz)
        K = tensor_at(X.ravel(), Y.ravel(), Z.ravel(), d).reshape(6, Py, Px) * valid[None]
        Kf = sfft.rfft2(K, axes=(1, 2))
        Mp = np.zeros((3, Py, Px))
        Mp[:, :ny, :nx] = M[:, z]
        Mf = sfft.rfft2(Mp, axes=(1, 2))
        for i in range(3):
            for j in range(3):
                Bf[i] += Kf[comp[(i, j)]] * Mf[j]
    B = sfft.irfft2(Bf, s=(Py, Px), axes=(1, 2))
    return -MU0 * B[:, :ny, :nx]


def stray_direct(M, d, height):
    """The same field by the plain double sum (tiny grids)."""
    _, nz, ny, nx = M.shape
    dx, dy, dz = d
    zt = target_z(nz, dz, height)
    B = np.zeros((3, ny, nx))
    for yt in range(ny):
        for xt in range(nx):
            acc = np.zeros(3)
            for z in range(nz):
                for y in range(ny):
                    for x in range(nx):
                        v = tensor_at([(xt - x) * dx], [(yt - y) * dy], [zt - z * dz], d)[:, 0]
                        N = np.array([[v[0], v[3], v[4]], [v[3], v[1], v[5]],
                                      [v[4], v[5], v[2]]])
                        acc += N @ M[:, z, y, x]
            B[:, yt, xt] = -MU0 * acc
    return B
