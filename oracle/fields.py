"""Local and short-range effective-field terms (FP64), per sublattice.

Arrays are (3, nz, ny, nx) per sublattice, x fastest; fields in tesla.

Exchange (Eq. 3, Methods "Exchange field"), for sublattice s with partner s':
  B = (2 A11/Ms) lap m^(s) + (A12/Ms) lap m^(s') + (4 A0/(Ms a^2)) m^(s')
with the 6-neighbour Laplacian sum_axes (m_+ + m_- - 2 m)/d^2.  Missing
neighbours are ghost cells: a copy of the boundary cell (Neumann, Eq. 5 with
no DMI and no inter-sublattice term), except in a layer with interfacial DMI.

Interfacial DMI (Eq. 4 with D_ijk of C_inf_v symmetry), energy density
D [m_z div m - (m.grad) m_z]; field (2D/Ms)(dx mz, dy mz, -dx mx - dy my) by
central differences.  Its natural boundary condition (Eq. 5 for one
sublattice): 2A dn m = -D (z x n) x m, i.e. at both x faces
dx m = -(D/2A)(mz, 0, -mx) and at both y faces dy m = -(D/2A)(0, mz, -my);
ghost = m + d*dm on a + face and m - d*dm on a - face.  The same ghosts feed
the exchange and DMI stencils.  z faces stay plain Neumann (no z
derivatives in this DMI).

Periodic boundaries ("DMI and boundary conditions": open, Neumann or
periodic): on a periodic axis the ghost of a boundary cell is the cell at
the opposite end, for the exchange, inter-sublattice and DMI stencils alike,
and no DMI boundary condition applies on that axis's faces.

Grain boundaries (demonstrations of polycrystalline magnets: the
ferromagnetic and inhomogeneous antiferromagnetic exchange constants are
reduced at grain boundaries): a link between cells of different grains
carries scale * A in the exchange and A12 stencils; DMI is not scaled.

Homogeneous DMI of a two-sublattice magnet: energy density d.(m1 x m2)
(the pair counted once; summing both orders would cancel it), fields
-(m2 x d)/Ms1 and -(d x m1)/Ms2.  It is reported with the DMI term.

Uniaxial anisotropy: (2 Ku1/Ms)(u.m) u + (4 Ku2/Ms)(u.m)^3 u.
Cubic anisotropy: -(2 Kc1/Ms) sum_k a_k (a_l^2 + a_n^2) c_k with
a_k = m.c_k in the frame (c1, c2, c1 x c2).
Zeeman: B_ext.
Magnetoelastic (Eq. 9): -(2/Ms)(B1 eps_ii m_i + B2 sum_{j != i} eps_ij m_j).

Pins (tests/test_oracle_fields.py): spin-spiral and cycloid closed forms,
uniform-state zeros, the 1-D edge-canting boundary-value problem, energy
gradient = field, per-cell closed forms of the local terms.
"""
from __future__ import annotations

import numpy as np


def ghost_pad(m, periodic=(False, False, False)):
    """One ghost cell on every side: a copy of the boundary cell, or on a
    periodic axis the cell at the opposite end."""
    g = np.pad(m, ((0, 0), (1, 1), (1, 1), (1, 1)), mode="edge")
    px, py, pz = periodic
    if px:
        g[:, :, :, 0] = g[:, :, :, -2]
        g[:, :, :, -1] = g[:, :, :, 1]
    if py:
        g[:, :, 0, :] = g[:, :, -2, :]
        g[:, :, -1, :] = g[:, :, 1, :]
    if pz:
        g[:, 0, :, :] = g[:, -2, :, :]
        g[:, -1, :, :] = g[:, 1, :, :]
    return g


def ghosted(m, d, D=None, A=None, dmi_layer=None, periodic=(False, False, False)):
    """Return m with one ghost cell on every side, shape (3, nz+2, ny+2, nx+2).

    ``D``/``A`` give the interfacial DMI boundary condition in the layer
    ``dmi_layer`` (or every layer when ``dmi_layer`` is None and D != 0) on
    the faces of the axes that are not periodic.
    """
    dx, dy, dz = d
    g = ghost_pad(m, periodic)
    if D is None or D == 0.0 or A is None or A == 0.0:
        return g
    k = -D / (2.0 * A)
    layers = range(m.shape[1]) if dmi_layer is None else [dmi_layer]
    for iz in layers:
        zg = iz + 1
        # x faces: dx m = k (mz, 0, -mx)
        for xb, xg, sgn in (() if periodic[0] else
                            ((0, 0, -1.0), (m.shape[3] - 1, m.shape[3] + 1, 1.0))):
            mb = m[:, iz, :, xb]
            dm = np.stack([k * mb[2], np.zeros_like(mb[0]), -k * mb[0]])
            g[:, zg, 1:-1, xg] = mb + sgn * dx * dm
        # y faces: dy m = k (0, mz, -my)
        for yb, yg, sgn in (() if periodic[1] else
                            ((0, 0, -1.0), (m.shape[2] - 1, m.shape[2] + 1, 1.0))):
            mb = m[:, iz, yb, :]
            dm = np.stack([np.zeros_like(mb[0]), k * mb[2], -k * mb[1]])
            g[:, zg, yg, 1:-1] = mb + sgn * dy * dm
    return g


def laplacian(g, d):
    """6-neighbour Laplacian of a ghosted array (interior cells)."""
    dx, dy, dz = d
    c = g[:, 1:-1, 1:-1, 1:-1]
    out = (g[:, 1:-1, 1:-1, 2:] + g[:, 1:-1, 1:-1, :-2] - 2.0 * c) / (dx * dx)
    out = out + (g[:, 1:-1, 2:, 1:-1] + g[:, 1:-1, :-2, 1:-1] - 2.0 * c) / (dy * dy)
    out = out + (g[:, 2:, 1:-1, 1:-1] + g[:, :-2, 1:-1, 1:-1] - 2.0 * c) / (dz * dz)
    return out


def link_weights(grain, scale, periodic=(False, False, False)):
    """Exchange weight of each cell's six links (x-, x+, y-, y+, z-, z+):
    ``scale`` between cells of different grains, 1 inside a grain and
    towards a ghost (the paper reduces the exchange constants at grain
    boundaries).  grain: (nz, ny, nx) ids."""
    g = ghost_pad(np.asarray(grain, dtype=np.int64)[None], periodic)[0]
    c = g[1:-1, 1:-1, 1:-1]
    nb = (g[1:-1, 1:-1, :-2], g[1:-1, 1:-1, 2:], g[1:-1, :-2, 1:-1], g[1:-1, 2:, 1:-1],
          g[:-2, 1:-1, 1:-1], g[2:, 1:-1, 1:-1])
    return [np.where(n == c, 1.0, scale) for n in nb]


def laplacian_weighted(g, d, w):
    """Laplacian of a ghosted array with per-link weights w (link_weights)."""
    dx, dy, dz = d
    c = g[:, 1:-1, 1:-1, 1:-1]
    out = (w[0] * (g[:, 1:-1, 1:-1, :-2] - c) + w[1] * (g[:, 1:-1, 1:-1, 2:] - c)) / (dx * dx)
    out = out + (w[2] * (g[:, 1:-1, :-2, 1:-1] - c) + w[3] * (g[:, 1:-1, 2:, 1:-1] - c)) / (dy * dy)
    out = out + (w[4] * (g[:, :-2, 1:-1, 1:-1] - c) + w[5] * (g[:, 2:, 1:-1, 1:-1] - c)) / (dz * dz)
    return out


def central_dx(g, d):
    return (g[:, 1:-1, 1:-1, 2:] - g[:, 1:-1, 1:-1, :-2]) / (2.0 * d[0])


def central_dy(g, d):
    return (g[:, 1:-1, 2:, 1:-1] - g[:, 1:-1, :-2, 1:-1]) / (2.0 * d[1])


def dmi_layer_mask(shape_zyx, dmi_layer):
    nz, ny, nx = shape_zyx
    mask = np.zeros((nz, ny, nx))
    if dmi_layer is None:
        mask[:] = 1.0
    else:
        mask[dmi_layer] = 1.0
    return mask


def exchange_field(m, Ms, A, d, D=0.0, dmi_layer=None, periodic=(False, False, False),
                   links=None):
    """(2A/Ms) lap m with Neumann (or DMI, or periodic) ghosts; ``links``
    (link_weights) scales the exchange at grain boundaries."""
    if Ms == 0.0:
        return np.zeros_like(m)
    g = ghosted(m, d, D, A, dmi_layer, periodic)
    lap = laplacian(g, d) if links is None else laplacian_weighted(g, d, links)
    return (2.0 * A / Ms) * lap


def afm_nn_field(mp, Ms, A12, d, periodic=(False, False, False), links=None):
    """(A12/Ms) lap m' with plain Neumann (or periodic) ghosts (second term of
    Eq. 3), scaled at grain boundaries by ``links``."""
    if Ms == 0.0:
        return np.zeros_like(mp)
    g = ghosted(mp, d, periodic=periodic)
    lap = laplacian(g, d) if links is None else laplacian_weighted(g, d, links)
    return (A12 / Ms) * lap


def afm_cell_field(mp, Ms, A0, a):
    """(4 A0/(Ms a^2)) m' (third term of Eq. 3)."""
    if Ms == 0.0:
        return np.zeros_like(mp)
    return (4.0 * A0 / (Ms * a * a)) * mp


def dmi_field(m, Ms, A, D, d, dmi_layer=None, periodic=(False, False, False)):
    """Interfacial DMI field with the natural-BC (or periodic) ghosts."""
    if Ms == 0.0 or D == 0.0:
        return np.zeros_like(m)
    g = ghosted(m, d, D, A, dmi_layer, periodic)
    ddx = central_dx(g, d)
    ddy = central_dy(g, d)
    B = np.stack([ddx[2], ddy[2], -ddx[0] - ddy[1]])
    mask = dmi_layer_mask(m.shape[1:], dmi_layer)
    return (2.0 * D / Ms) * B * mask[None]


def homogeneous_dmi_field(m, mp, Ms, dvec, first):
    """Homogeneous DMI between the two sublattices of a cell ("DMI and
    boundary conditions"): energy density d . (m^(1) x m^(2)), the pair
    counted once.  B^(1) = -(m^(2) x d)/Ms1, B^(2) = -(d x m^(1))/Ms2;
    ``first`` selects the sublattice m belongs to, mp is the other one."""
    if Ms == 0.0 or not np.any(dvec):
        return np.zeros_like(m)
    d = np.asarray(dvec, dtype=np.float64)[:, None, None, None]
    c = np.cross(mp, d, axis=0)          # m' x d
    return (-c if first else c) / Ms


def uniaxial_field(m, Ms, Ku1, Ku2, u):
    """u: 3-vector or per-cell array (3, nz, ny, nx)."""
    if Ms == 0.0:
        return np.zeros_like(m)
    u = np.asarray(u, dtype=np.float64)
    if u.ndim == 1:
        u = u[:, None, None, None]
    um = np.sum(u * m, axis=0)
    return (2.0 * Ku1 / Ms) * um * u + (4.0 * Ku2 / Ms) * um ** 3 * u


def cubic_frame(c1, c2):
    c1 = np.asarray(c1, dtype=np.float64)
    c2 = np.asarray(c2, dtype=np.float64)
    return c1, c2, np.cross(c1, c2)


def cubic_field(m, Ms, Kc1, c1, c2):
    if Ms == 0.0:
        return np.zeros_like(m)
    cs = cubic_frame(c1, c2)
    a = [np.tensordot(c, m, axes=(0, 0)) for c in cs]
    B = np.zeros_like(m)
    for k in range(3):
        others = [a[l] ** 2 for l in range(3) if l != k]
        B += (a[k] * (others[0] + others[1]))[None] * cs[k][:, None, None, None]
    return -(2.0 * Kc1 / Ms) * B


def zeeman_field(m, B_ext):
    return np.broadcast_to(np.asarray(B_ext, dtype=np.float64)[:, None, None, None],
                           m.shape).copy()


def magnetoelastic_field(m, Ms, B1, B2, eps):
    """Eq. 9; eps = (xx, yy, zz, xy, xz, yz) strain, shape (6, nz, ny, nx)."""
    if Ms == 0.0:
        return np.zeros_like(m)
    exx, eyy, ezz, exy, exz, eyz = eps
    mx, my, mz = m
    B = np.stack([
        B1 * exx * mx + B2 * (exy * my + exz * mz),
        B1 * eyy * my + B2 * (exy * mx + eyz * mz),
        B1 * ezz * mz + B2 * (exz * mx + eyz * my),
    ])
    return -(2.0 / Ms) * B
