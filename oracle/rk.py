"""Dormand-Prince 5(4) embedded Runge-Kutta pair (Table 2), FP64.

Tableau of Dormand & Prince (1980): 7 stages, first-same-as-last, the
5th-order solution is propagated and the 4th-order one only enters the
error estimate e = b - b*.  Every stage input and the accepted result are
renormalised per cell and sublattice (m only; u and v are not).

Step control (the paper names the methods but no controller; these
constants are this build's reading, "parity unpinned" beyond GPU/oracle
agreement):
  err   = dt * max over cells and sublattices of |sum_j e_j k_j|_2
  accept when err <= tol
  dt'   = dt * clip(0.8 (tol/err)^(1/5), 0.1, 2.0)   (factor 2 if err == 0)
  a step is clipped so it lands on the next output time; the controller
  continues from the clipped dt.  A rejected step keeps k1 (y unchanged).

Pins (tests/test_oracle_rk.py): the tableau's order conditions, 5th-order
convergence of a smooth ODE, the analytic damped single-spin trajectory.
"""
from __future__ import annotations

from fractions import Fraction as F

import numpy as np

C = [F(0), F(1, 5), F(3, 10), F(4, 5), F(8, 9), F(1), F(1)]
A = [
    [],
    [F(1, 5)],
    [F(3, 40), F(9, 40)],
    [F(44, 45), F(-56, 15), F(32, 9)],
    [F(19372, 6561), F(-25360, 2187), F(64448, 6561), F(-212, 729)],
    [F(9017, 3168), F(-355, 33), F(46732, 5247), F(49, 176), F(-5103, 18656)],
    [F(35, 384), F(0), F(500, 1113), F(125, 192), F(-2187, 6784), F(11, 84)],
]
B5 = [F(35, 384), F(0), F(500, 1113), F(125, 192), F(-2187, 6784), F(11, 84), F(0)]
B4 = [F(5179, 57600), F(0), F(7571, 16695), F(393, 640), F(-92097, 339200),
      F(187, 2100), F(1, 40)]
E = [b - bs for b, bs in zip(B5, B4)]

SAFETY = 0.8
FAC_MIN = 0.1
FAC_MAX = 2.0


def new_dt(dt, err, tol):
    if err == 0.0:
        return dt * FAC_MAX
    fac = SAFETY * (tol / err) ** 0.2
    return dt * min(FAC_MAX, max(FAC_MIN, fac))


class Stepper:
    """Generic DP45 over a state of several arrays.

    ``rhs(t, state) -> derivs`` (same structure as state);
    ``normalise(state) -> state`` projects the magnetisation arrays;
    ``err_parts(vec) -> max norm`` takes sum_j e_j k_j for each array.
    """

    def __init__(self, rhs, normalise, err_norm):
        self.rhs = rhs
        self.normalise = normalise
        self.err_norm = err_norm
        self.k1 = None

    def invalidate(self):
        self.k1 = None

    def step(self, t, y, dt):
        """One DP45 attempt; returns (y_new, k7, err)."""
        if self.k1 is None:
            self.k1 = self.rhs(t, y)
        k = [self.k1]
        ys = None
        for s in range(1, 7):
            ys = []
            for idx in range(len(y)):
                acc = y[idx].copy()
                for j in range(s):
                    a = float(A[s][j])
                    if a != 0.0:
                        acc = acc + (a * dt) * k[j][idx]
                ys.append(acc)
            ys = self.normalise(ys)
            k.append(self.rhs(t + float(C[s]) * dt, ys))
        errv = []
        for idx in range(len(y)):
            acc = np.zeros_like(y[idx])
            for j in range(7):
                e = float(E[j])
                if e != 0.0:
                    acc = acc + e * k[j][idx]
            errv.append(acc)
        err = dt * self.err_norm(errv)
        return ys, k[6], err

    def accept(self, k7):
        self.k1 = k7
