"""Pins for the oracle's magnetoelastic force (Eq. 8, "Magnetoelasticity").

Eq. 8 and Eq. 9 are the two derivatives of one cubic magnetoelastic energy
density, e(eps, m) = B1 sum_i eps_ii m_i^2 + B2 sum_{i != j} eps_ij m_i m_j
(the textbook cubic magnetostriction energy): the field is -(1/Ms) de/dm
(pinned by the energy gradient in test_oracle_fields.py) and the body force
is the divergence of the magnetoelastic stress sigma_ij = de/deps_ij, since
-delta/delta u of the energy integral is div(de/deps).  Here the stress is
obtained by symbolic differentiation of that energy (sympy), its divergence
symbolically, with m a polynomial field; the oracle's numeric force must
match it wherever its derivative operator is exact:

* m of degree 2: every bulk cell (the 4th-order central difference is exact
  on the quadratic m, and m_i d_j m_k is then exactly the product rule);
* m of degree 1: every cell, faces included (the one-sided and 2nd-order
  boundary differences are exact on linear fields).

The B1 and B2 parts are checked separately, on a non-cubic cell, and a
force with the B2 index swapped (m_j d_i m_j for m_j d_j m_i, the misreading
a plain retyping of Eq. 8 would not catch) fails the same comparison.
"""
import numpy as np
import pytest
import sympy as sp

from oracle import elastic as el

X = sp.symbols("x y z")


def _symbolic_force(mexpr, B1, B2):
    """f_i = sum_j d_j (de/deps_ij) for the polynomial field mexpr."""
    eps = sp.Matrix(3, 3, lambda i, j: sp.Symbol(f"e{i}{j}"))
    ms = sp.symbols("m0 m1 m2")
    e = sum(B1 * eps[i, i] * ms[i] ** 2 for i in range(3))
    e += sum(B2 * eps[i, j] * ms[i] * ms[j] for i in range(3) for j in range(3) if i != j)
    sub = dict(zip(ms, mexpr))
    sig = [[sp.diff(e, eps[i, j]).subs(sub) for j in range(3)] for i in range(3)]
    return [sp.expand(sum(sp.diff(sig[i][j], X[j]) for j in range(3))) for i in range(3)]


def _poly_field(rng, degree):
    mons = [sp.Integer(1)]
    for dgr in range(1, degree + 1):
        mons += [X[0] ** a * X[1] ** b * X[2] ** (dgr - a - b)
                 for a in range(dgr + 1) for b in range(dgr + 1 - a)]
    return [sum(sp.Rational(int(rng.integers(-9, 10)), 7) * mo for mo in mons)
            for _ in range(3)]


def _grid_values(exprs, n, d):
    nx, ny, nz = n
    zz, yy, xx = np.meshgrid(np.arange(nz) * d[2], np.arange(ny) * d[1], np.arange(nx) * d[0],
                             indexing="ij")
    out = []
    for ex in exprs:
        f = sp.lambdify(X, ex, "numpy")
        out.append(np.broadcast_to(np.asarray(f(xx, yy, zz), dtype=np.float64), xx.shape))
    return np.stack(out)


# cells of order 1 so the polynomial values stay O(1) (the operator is
# linear in 1/d, so the units do not matter for exactness)
N = (9, 8, 7)
D = (0.9, 1.3, 1.1)
BULK = (slice(None), slice(2, N[2] - 2), slice(2, N[1] - 2), slice(2, N[0] - 2))


def _check(m_of, degree, B1, B2, region, force=el.magnetoelastic_force, seed=7):
    rng = np.random.default_rng(seed)
    mexpr = _poly_field(rng, degree)
    m = _grid_values(mexpr, N, D)
    ref = _grid_values(_symbolic_force(mexpr, B1, B2), N, D)
    got = force(m, B1, B2, D)
    scale = np.abs(ref[region]).max()
    assert scale > 0
    return np.abs(got[region] - ref[region]).max() / scale


@pytest.mark.parametrize("B1,B2", [(1.7, 0.0), (0.0, -2.3), (1.7, -2.3)])
def test_force_is_divergence_of_magnetoelastic_stress_bulk(B1, B2):
    assert _check(None, 2, B1, B2, BULK) < 1e-13


@pytest.mark.parametrize("B1,B2", [(1.7, 0.0), (0.0, -2.3)])
def test_force_linear_field_every_cell(B1, B2):
    assert _check(None, 1, B1, B2, (slice(None),) * 4) < 1e-13


def _swapped_b2(m, B1, B2, d):
    """Eq. 8 with the B2 term misread as m_j d_i m_j (a planted mistake)."""
    dm = [[el.deriv(m[i], el.AX[j], d[j]) for j in range(3)] for i in range(3)]
    f = np.zeros_like(m)
    for i in range(3):
        f[i] += 2.0 * B1 * m[i] * dm[i][i]
        for j in range(3):
            if j != i:
                f[i] += B2 * (m[i] * dm[j][j] + m[j] * dm[j][i])
    return f


def _sign_flipped_b1(m, B1, B2, d):
    return el.magnetoelastic_force(m, -B1, B2, d)


@pytest.mark.parametrize("bad", [_swapped_b2, _sign_flipped_b1])
def test_planted_mistakes_fail_the_pin(bad):
    err = _check(None, 2, 1.7, -2.3, BULK, force=bad)
    assert err > 1e-2
