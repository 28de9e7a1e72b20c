"""General DMI tensor (Eq. 4) and the Neumann boundary condition of Eq. 6.

Test infrastructure: only tests/, the package's smoke check and the
benchmark's CPU baseline use this module.

DMI tensor.  D_ijk = -D_ikj has 9 independent components; they are given
as three DMI vectors W_i (i = x, y, z spatial direction) with
D_ijk = sum_a eps_ajk W_ia, i.e. W_ix = D_i,yz, W_iy = D_i,zx, W_iz = D_i,xy.
Energy density (Eq. 4) sum_{s,s'} sum_ijk D^(s,s')_ijk m^(s)_j d_i m^(s')_k
with D^(s,s) the tensor of sublattice s and D^(1,2) = D^(2,1) the
inter-sublattice one.  The variational derivative gives the fields
  B^(s) = -(2/Ms^(s)) sum_i [ d_i m^(s) x W^(s)_i + d_i m^(s') x W^(12)_i ],
derivatives by central differences over ghost cells.  The interfacial
(C_inf_v) tensor is W_x = (0, D, 0), W_y = (-D, 0, 0), W_z = 0.

Boundary condition (Eq. 6, the paper's default Neumann condition): on a
face with outward normal n, for each sublattice s (partner s'),
  2 A11^(s) d_n m^(s) = A12 (d_n m^(s') x m^(s)) x m^(s) + D^(s).(n (x) m^(s)),
where the contraction (D.(n (x) m))_l = D_ilj n_i m_j = (m x (n.W))_l is the
one the variational principle yields for the energy above (it reproduces
Eq. 5 for the interfacial tensor).  With (g x m) x m = -(I - m m^T) g the two
sublattices' normal derivatives solve the 6x6 linear system
  2 A11^(1) g1 + A12 Q1 g2 = m1 x w1,   2 A11^(2) g2 + A12 Q2 g1 = m2 x w2,
Q = I - m m^T, per boundary cell (one sublattice: g = m x w / (2 A11)); the
ghost cell beyond the face is m + d_a g.  These ghosts feed every stencil:
exchange, the inter-sublattice exchange and the DMI.  Faces of periodic
axes wrap instead.  The inter-sublattice DMI does not enter Eq. 6, and the
condition is not applied on a sublattice with A11 = 0 (its ghosts copy the
boundary cell).

Pins (tests/test_oracle_dmi.py): the energy gradient equals the field in
the bulk; the interfacial tensor reproduces the interfacial-DMI field and
its Eq. 5 ghosts cell by cell; the ghosts satisfy Eq. 6 (residual ~1e-16);
a spin spiral gives the closed-form bulk-DMI field; for a uniform state
the boundary ghosts with A12 and no DMI reduce to copies of the cell.
"""
from __future__ import annotations

import numpy as np

from .fields import ghost_pad

EPS = np.zeros((3, 3, 3))
EPS[0, 1, 2] = EPS[1, 2, 0] = EPS[2, 0, 1] = 1.0
EPS[0, 2, 1] = EPS[2, 1, 0] = EPS[1, 0, 2] = -1.0


def tensor_from_vectors(W):
    """D_ijk from the DMI vectors W (3x3, row i = direction i)."""
    W = np.asarray(W, dtype=np.float64)
    return np.einsum("ajk,ia->ijk", EPS, W)


# (numpy axis of a (3, nz, ny, nx) array, cell size index) per spatial axis
_AX = {0: 3, 1: 2, 2: 1}


def eq6_ghosts(m, d, A11, A12, W, periodic=(False, False, False)):
    """Ghosted copies (nsub, 3, nz+2, ny+2, nx+2) with the ghosts of Eq. 6.

    m: (nsub, 3, nz, ny, nx); A11: per sublattice; W: (nsub, 3, 3) DMI
    vectors of each sublattice's own tensor.
    """
    nsub = m.shape[0]
    g = np.stack([ghost_pad(m[s], periodic) for s in range(nsub)])
    W = np.asarray(W, dtype=np.float64)
    for a in range(3):
        if periodic[a]:
            continue
        ax = _AX[a]
        n_a = m.shape[ax + 1]
        for side in (-1, 1):
            face = 0 if side < 0 else n_a - 1
            gidx = 0 if side < 0 else n_a + 1
            mb = np.take(m, face, axis=ax + 1)              # (nsub, 3, ...)
            shp = mb.shape[2:]
            mf = mb.reshape(nsub, 3, -1)                    # (nsub, 3, P)
            P = mf.shape[2]
            rhs = np.zeros((P, 3 * nsub))
            mat = np.zeros((P, 3 * nsub, 3 * nsub))
            active = [A11[s] != 0.0 for s in range(nsub)]
            for s in range(nsub):
                w = side * W[s][a]
                if active[s]:
                    rhs[:, 3 * s:3 * s + 3] = np.cross(mf[s].T, w)
                    mat[:, 3 * s:3 * s + 3, 3 * s:3 * s + 3] = 2.0 * A11[s] * np.eye(3)
                else:
                    mat[:, 3 * s:3 * s + 3, 3 * s:3 * s + 3] = np.eye(3)
            if nsub == 2 and A12 != 0.0:
                for s in range(2):
                    if not active[s]:
                        continue
                    o = 1 - s
                    ms = mf[s].T                                # (P, 3)
                    Q = np.eye(3)[None] - ms[:, :, None] * ms[:, None, :]
                    mat[:, 3 * s:3 * s + 3, 3 * o:3 * o + 3] = A12 * Q
            sol = np.linalg.solve(mat, rhs[:, :, None])[:, :, 0]   # (P, 3 nsub)
            for s in range(nsub):
                gs = sol[:, 3 * s:3 * s + 3].T.reshape((3,) + shp)
                ghost = mb[s] + d[a] * gs
                idx = [slice(None)] * 4
                idx[ax] = gidx
                for b in range(3):
                    if b == a:
                        continue
                    idx[_AX[b]] = slice(1, -1)
                g[s][tuple(idx)] = ghost
    return g


def central(gs, d, a):
    """Central difference along spatial axis a of a ghosted (3, ...) array."""
    ax = _AX[a]
    hi = [slice(1, -1)] * 4
    lo = [slice(1, -1)] * 4
    hi[0] = lo[0] = slice(None)
    hi[ax] = slice(2, None)
    lo[ax] = slice(None, -2)
    return (gs[tuple(hi)] - gs[tuple(lo)]) / (2.0 * d[a])


def tensor_field(gs, go, Ms, W_own, W_inter, d):
    """-(2/Ms) sum_i [d_i m x W_own_i + d_i m' x W_inter_i] (ghosted inputs)."""
    out = np.zeros_like(gs[:, 1:-1, 1:-1, 1:-1])
    if Ms == 0.0:
        return out
    for i in range(3):
        wi = np.asarray(W_own[i], dtype=np.float64)
        if np.any(wi):
            out -= np.cross(central(gs, d, i), wi[:, None, None, None], axis=0)
        if go is not None:
            wo = np.asarray(W_inter[i], dtype=np.float64)
            if np.any(wo):
                out -= np.cross(central(go, d, i), wo[:, None, None, None], axis=0)
    return (2.0 / Ms) * out
