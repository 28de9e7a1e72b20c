"""Elastodynamics and magnetoelastic force (FP64).

Methods, "Elasticity" (Eq. 7) and "Magnetoelasticity" (Eq. 8):
  rho d2u/dt2 = f_el + sum_s f_mel^(s) - eta v,  integrated as du/dt = v,
  dv/dt = (...)/rho.  (The velocity-proportional body force with constant
  eta is the damping model of the racetrack workload.)
  strain  eps_ij = (d_i u_j + d_j u_i)/2 from the numeric gradient of u;
  stress  sigma_ii = C11 eps_ii + C12 (eps_jj + eps_kk), sigma_ij = 2 C44 eps_ij
          (cubic stiffness), plus the viscous (strain-rate) stress of the
          paper's "Elasticity" section, read as stiffness-proportional
          Rayleigh damping: beta C : eps(v), with the stiffness coefficient
          beta of the NiO table (0.1 ps);
  f_el    = div sigma by the same derivative operator.
The first derivative is 4th-order central (-f2 + 8 f1 - 8 f-1 + f-2)/(12 d)
in the bulk, 2nd-order central one cell in from a face and 1st-order
one-sided on the face cell (the paper: lower-order schemes close to and at
the boundaries).  Axes with a single cell have zero derivative.

Traction sigma.n = t: on every face of an axis with more than one cell the
face cell's stress row along that axis is replaced by the prescribed
traction (zero = traction-free) before the divergence; the drive is a shear
traction sigma_xz = sigma_zx = amp sin(2 pi f t) on the x = 0 face, applied
after the traction-free rows so it wins on its own component.

Magnetoelastic force (Eq. 8), per sublattice with its own B1, B2:
  f_i = 2 B1 m_i d_i m_i + B2 sum_{j != i} (m_i d_j m_j + m_j d_j m_i).

Pins (tests/test_oracle_elastic.py): the operator is exact on polynomials
of degree <= 4 in the bulk (<= 2 one cell in, <= 1 on the face); the shear
wave speed sqrt(C44/rho) and the static strain of a shear traction
reproduce the paper's printed ~4 km/s and ~0.14 % for the NiO parameters;
energy balance with eta = 0; the printed Rayleigh coefficient gives the
printed ~5 % damping ratio of 24 nm shear waves.
tests/test_oracle_magnetoelastic.py: the force equals the divergence of the
magnetoelastic stress de/deps of the cubic magnetoelastic energy (symbolic,
sympy) on polynomial magnetisations, B1 and B2 parts separately.
tests/test_oracle_balance.py: the coupled system's energy balance closes at
the solver's order, and the discrete boundary power tends to the traction
power and the magnetostrictive stress's boundary work at first order.
"""
from __future__ import annotations

import math

import numpy as np


def deriv(f, axis, h):
    """First derivative of f along ``axis`` (numpy axis index)."""
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[axis]
    out = np.zeros_like(f)
    if n == 1:
        return out
    fm = np.moveaxis(f, axis, 0)
    om = np.moveaxis(out, axis, 0)
    om[0] = (fm[1] - fm[0]) / h
    om[n - 1] = (fm[n - 1] - fm[n - 2]) / h
    if n >= 3:
        om[1] = (fm[2] - fm[0]) / (2.0 * h)
        om[n - 2] = (fm[n - 1] - fm[n - 3]) / (2.0 * h)
    if n >= 5:
        om[2:n - 2] = (-fm[4:] + 8.0 * fm[3:n - 1] - 8.0 * fm[1:n - 3]
                       + fm[0:n - 4]) / (12.0 * h)
    return out


# spatial axis k (0 = x, 1 = y, 2 = z) -> numpy axis of a (nz, ny, nx) array
AX = {0: 2, 1: 1, 2: 0}
VOIGT = {(0, 0): 0, (1, 1): 1, (2, 2): 2, (0, 1): 3, (1, 0): 3,
         (0, 2): 4, (2, 0): 4, (1, 2): 5, (2, 1): 5}


def strain(u, d):
    """(xx, yy, zz, xy, xz, yz), shape (6, nz, ny, nx)."""
    g = [[deriv(u[j], AX[i], d[i]) for j in range(3)] for i in range(3)]
    return np.stack([
        g[0][0], g[1][1], g[2][2],
        0.5 * (g[0][1] + g[1][0]),
        0.5 * (g[0][2] + g[2][0]),
        0.5 * (g[1][2] + g[2][1]),
    ])


def stress(eps, C11, C12, C44):
    exx, eyy, ezz, exy, exz, eyz = eps
    return np.stack([
        C11 * exx + C12 * (eyy + ezz),
        C11 * eyy + C12 * (exx + ezz),
        C11 * ezz + C12 * (exx + eyy),
        2.0 * C44 * exy,
        2.0 * C44 * exz,
        2.0 * C44 * eyz,
    ])


def apply_traction(sig, n, t, el):
    """Boundary rows of the stress (in place on a copy)."""
    sig = sig.copy()
    nx, ny, nz = n
    sizes = (nx, ny, nz)
    for k in range(3):
        if sizes[k] < 2:
            continue
        for face in (0, sizes[k] - 1):
            idx = [slice(None)] * 3
            idx[AX[k]] = face
            for j in range(3):
                sig[(VOIGT[(k, j)],) + tuple(idx)] = 0.0
    if el is not None and el.get("trac_amp", 0.0) != 0.0 and nx >= 2:
        val = el["trac_amp"] * math.sin(2.0 * math.pi * el["trac_freq"] * t)
        sig[VOIGT[(0, 2)], :, :, 0] = val
    return sig


def elastic_force(u, d, n, t, el, v=None):
    eps = strain(u, d)
    sig = stress(eps, el["C11"], el["C12"], el["C44"])
    beta = el.get("rayleigh", 0.0)
    if beta != 0.0 and v is not None:
        sig = sig + beta * stress(strain(v, d), el["C11"], el["C12"], el["C44"])
    sig = apply_traction(sig, n, t, el)
    f = np.zeros_like(u)
    for i in range(3):
        for j in range(3):
            f[i] += deriv(sig[VOIGT[(i, j)]], AX[j], d[j])
    return f


def magnetoelastic_force(m, B1, B2, d):
    dm = [[deriv(m[i], AX[j], d[j]) for j in range(3)] for i in range(3)]
    f = np.zeros_like(m)
    for i in range(3):
        f[i] += 2.0 * B1 * m[i] * dm[i][i]
        for j in range(3):
            if j != i:
                f[i] += B2 * (m[i] * dm[j][j] + m[j] * dm[i][j])
    return f


def elastic_energy_density(u, v, d, el):
    eps = strain(u, d)
    sig = stress(eps, el["C11"], el["C12"], el["C44"])
    w = np.array([1.0, 1.0, 1.0, 2.0, 2.0, 2.0])  # sigma:eps counts ij and ji
    return 0.5 * np.tensordot(w, sig * eps, axes=(0, 0)) + 0.5 * el["rho"] * np.sum(v * v, axis=0)
