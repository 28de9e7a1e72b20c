"""Embedded Runge-Kutta pairs of the paper's solver table (Table 2), FP64.

Test infrastructure: only tests/, the package's smoke check and the
benchmark's CPU baseline use this module.

The table lists five pairs with their convergence order p (the solution
that is propagated) and the order q of the embedded solution that only
enters the error estimate:

  Heun (RK12)               p = 2, q = 1   Heun's method with Euler embedded
  Bogacki-Shampine (RK23)   p = 3, q = 2   Bogacki & Shampine (1989), FSAL
  Cash-Karp                 p = 5, q = 4   Cash & Karp (1990)
  Fehlberg (RKF45)          p = 5, q = 4   Fehlberg (1969), 5th order propagated
  Dormand-Prince (RK45)     p = 5, q = 4   Dormand & Prince (1980), FSAL

The coefficients are those of the cited papers, exact as fractions.  A
step evaluates k_i = f(t + c_i h, normalise(y + h sum_{j<i} a_ij k_j)),
propagates y' = normalise(y + h sum_i b_i k_i) and estimates the error from
e = b - b*.  Every stage input and the accepted result are renormalised
per cell and sublattice (m only; u and v are not).  For a
first-same-as-last pair the last stage is evaluated at y' itself and its
slope is the next step's k_1; otherwise k_1 = f(y') is evaluated at the
start of the next step.  A rejected step keeps k_1 (y is unchanged).

Step control (the paper names the methods and the error-estimate order but
no controller; these constants are a reading taken here, "parity unpinned"
beyond GPU/oracle agreement):
  err   = h * max over cells and sublattices of |sum_j e_j k_j|_2
  accept when err <= tol
  h'    = h * clip(0.8 (tol/err)^(1/(q+1)), 0.1, 2.0)   (factor 2 if err == 0)
  a step is clipped so it lands on the next output time; the controller
  continues from the clipped step.

Pins (tests/test_oracle_rk.py): every pair's weights meet Butcher's order
conditions exactly up to the printed orders p and q and miss one of the
next order; row sums c_i; the measured convergence order of each pair on a
smooth ODE; the local order of each error estimate; the analytic damped
single-spin trajectory under every pair with adaptive steps.
"""
from __future__ import annotations

from dataclasses import dataclass
from fractions import Fraction as F

import numpy as np


@dataclass(frozen=True)
class Tableau:
    name: str
    c: tuple
    a: tuple          # a[i] = (a_i0 .. a_i,i-1)
    b: tuple          # propagated weights (order p)
    bs: tuple         # embedded weights (order q)
    p: int
    q: int
    fsal: bool

    @property
    def stages(self):
        return len(self.c)

    @property
    def e(self):
        return tuple(x - y for x, y in zip(self.b, self.bs))


HEUN = Tableau(
    "heun", (F(0), F(1)),
    ((), (F(1),)),
    (F(1, 2), F(1, 2)), (F(1), F(0)), 2, 1, False)

BS23 = Tableau(
    "bs23", (F(0), F(1, 2), F(3, 4), F(1)),
    ((), (F(1, 2),), (F(0), F(3, 4)), (F(2, 9), F(1, 3), F(4, 9))),
    (F(2, 9), F(1, 3), F(4, 9), F(0)),
    (F(7, 24), F(1, 4), F(1, 3), F(1, 8)), 3, 2, True)

CASH_KARP = Tableau(
    "cashkarp", (F(0), F(1, 5), F(3, 10), F(3, 5), F(1), F(7, 8)),
    ((), (F(1, 5),), (F(3, 40), F(9, 40)), (F(3, 10), F(-9, 10), F(6, 5)),
     (F(-11, 54), F(5, 2), F(-70, 27), F(35, 27)),
     (F(1631, 55296), F(175, 512), F(575, 13824), F(44275, 110592), F(253, 4096))),
    (F(37, 378), F(0), F(250, 621), F(125, 594), F(0), F(512, 1771)),
    (F(2825, 27648), F(0), F(18575, 48384), F(13525, 55296), F(277, 14336), F(1, 4)),
    5, 4, False)

FEHLBERG = Tableau(
    "rkf45", (F(0), F(1, 4), F(3, 8), F(12, 13), F(1), F(1, 2)),
    ((), (F(1, 4),), (F(3, 32), F(9, 32)),
     (F(1932, 2197), F(-7200, 2197), F(7296, 2197)),
     (F(439, 216), F(-8), F(3680, 513), F(-845, 4104)),
     (F(-8, 27), F(2), F(-3544, 2565), F(1859, 4104), F(-11, 40))),
    (F(16, 135), F(0), F(6656, 12825), F(28561, 56430), F(-9, 50), F(2, 55)),
    (F(25, 216), F(0), F(1408, 2565), F(2197, 4104), F(-1, 5), F(0)),
    5, 4, False)

DORMAND_PRINCE = Tableau(
    "dp45", (F(0), F(1, 5), F(3, 10), F(4, 5), F(8, 9), F(1), F(1)),
    ((), (F(1, 5),), (F(3, 40), F(9, 40)), (F(44, 45), F(-56, 15), F(32, 9)),
     (F(19372, 6561), F(-25360, 2187), F(64448, 6561), F(-212, 729)),
     (F(9017, 3168), F(-355, 33), F(46732, 5247), F(49, 176), F(-5103, 18656)),
     (F(35, 384), F(0), F(500, 1113), F(125, 192), F(-2187, 6784), F(11, 84))),
    (F(35, 384), F(0), F(500, 1113), F(125, 192), F(-2187, 6784), F(11, 84), F(0)),
    (F(5179, 57600), F(0), F(7571, 16695), F(393, 640), F(-92097, 339200),
     F(187, 2100), F(1, 40)),
    5, 4, True)

TABLEAUS = {t.name: t for t in (HEUN, BS23, CASH_KARP, FEHLBERG, DORMAND_PRINCE)}

# Dormand-Prince views kept for the tests that pin that pair on its own
C = list(DORMAND_PRINCE.c)
A = [list(r) for r in DORMAND_PRINCE.a]
B5 = list(DORMAND_PRINCE.b)
B4 = list(DORMAND_PRINCE.bs)
E = list(DORMAND_PRINCE.e)

SAFETY = 0.8
FAC_MIN = 0.1
FAC_MAX = 2.0


def new_dt(dt, err, tol, q=4, safety=SAFETY, fac_min=FAC_MIN, fac_max=FAC_MAX, dt_max=None):
    """Next step size: dt * clip(safety (tol/err)^(1/(q+1)), fac_min, fac_max)
    (fac_max when err == 0), then at most dt_max."""
    if err == 0.0:
        out = dt * fac_max
    else:
        fac = safety * (tol / err) ** (1.0 / (q + 1))
        out = dt * min(fac_max, max(fac_min, fac))
    return out if not dt_max else min(out, dt_max)


class Stepper:
    """One embedded pair over a state of several arrays.

    ``rhs(t, state) -> derivs`` (same structure as state);
    ``normalise(state) -> state`` projects the magnetisation arrays;
    ``err_norm(vecs) -> max norm`` takes sum_j e_j k_j for each array.
    """

    def __init__(self, rhs, normalise, err_norm, tableau=DORMAND_PRINCE):
        self.rhs = rhs
        self.normalise = normalise
        self.err_norm = err_norm
        self.tab = tableau
        self.k1 = None

    def invalidate(self):
        self.k1 = None

    def _combine(self, y, k, w, dt):
        out = []
        for idx in range(len(y)):
            acc = y[idx].copy()
            for j, wj in enumerate(w):
                if wj != 0:
                    acc = acc + (float(wj) * dt) * k[j][idx]
            out.append(acc)
        return self.normalise(out)

    def step(self, t, y, dt):
        """One attempt; returns (y_new, k1 of the next step or None, err)."""
        tab = self.tab
        if self.k1 is None:
            self.k1 = self.rhs(t, y)
        k = [self.k1]
        for i in range(1, tab.stages):
            yi = self._combine(y, k, tab.a[i], dt)
            k.append(self.rhs(t + float(tab.c[i]) * dt, yi))
        if tab.fsal:
            ynew, knext = yi, k[-1]
        else:
            ynew, knext = self._combine(y, k, tab.b, dt), None
        errv = []
        for idx in range(len(y)):
            acc = np.zeros_like(y[idx])
            for j, ej in enumerate(tab.e):
                if ej != 0:
                    acc = acc + float(ej) * k[j][idx]
            errv.append(acc)
        err = dt * self.err_norm(errv)
        return ynew, knext, err

    def accept(self, knext):
        self.k1 = knext
