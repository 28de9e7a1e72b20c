"""Torques (FP64): LLG (Eq. 2) and Zhang-Li spin-transfer torque.

LLG: tau = -gamma/(1+alpha^2) [m x B + alpha m x (m x B)].

Zhang-Li (Methods, "Micromagnetism": implemented as in mumax3, whose text is
not reproduced in the paper):
  tau_ZL = -1/(1+alpha^2) [(1 + xi alpha) m x (m x (u.grad) m)
                           + (xi - alpha) m x (u.grad) m]
with the drift velocity u = P mu_B j / (e Ms) (g = 2).  The torque's
structure is pinned (a uniform state feels no torque; a periodic helix
gives the closed form of both terms, tests/test_oracle_pbc.py), but the
drift-velocity prefactor is a reading taken here: it is "parity
unpinned" beyond GPU/oracle agreement.  (u.grad) m uses central differences with clamped neighbours
(the boundary cell stands in for the missing one) over 2*d.
"""
from __future__ import annotations

import numpy as np

from .constants import MU_B, QE
from .fields import ghost_pad


def cross(a, b):
    return np.stack([
        a[1] * b[2] - a[2] * b[1],
        a[2] * b[0] - a[0] * b[2],
        a[0] * b[1] - a[1] * b[0],
    ])


def llg_torque(m, B, gamma, alpha):
    mxB = cross(m, B)
    return -gamma / (1.0 + alpha * alpha) * (mxB + alpha * cross(m, mxB))


def drift_velocity(P, j, Ms):
    if Ms == 0.0:
        return np.zeros(3)
    return P * MU_B * np.asarray(j, dtype=np.float64) / (QE * Ms)


def directional_derivative(m, u, d, periodic=(False, False, False)):
    """(u.grad) m with clamped (or, on periodic axes, wrapped) neighbours and
    2d central differences."""
    g = ghost_pad(m, periodic)
    out = np.zeros_like(m)
    if u[0] != 0.0:
        out += u[0] * (g[:, 1:-1, 1:-1, 2:] - g[:, 1:-1, 1:-1, :-2]) / (2.0 * d[0])
    if u[1] != 0.0:
        out += u[1] * (g[:, 1:-1, 2:, 1:-1] - g[:, 1:-1, :-2, 1:-1]) / (2.0 * d[1])
    if u[2] != 0.0:
        out += u[2] * (g[:, 2:, 1:-1, 1:-1] - g[:, :-2, 1:-1, 1:-1]) / (2.0 * d[2])
    return out


def zhang_li_torque(m, u, alpha, xi, d, periodic=(False, False, False)):
    if not np.any(u):
        return np.zeros_like(m)
    dm = directional_derivative(m, u, d, periodic)
    mxdm = cross(m, dm)
    return -1.0 / (1.0 + alpha * alpha) * (
        (1.0 + xi * alpha) * cross(m, mxdm) + (xi - alpha) * mxdm)
