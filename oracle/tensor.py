"""Cell-averaged demagnetising tensor N(R) for cuboid cells (FP64).

Follows the Methods section ("Magnetostatic field"): the interaction between
two cells is the analytic Newell-Williams-Dunlop result below a cutoff
radius and an asymptotic (multipole) result beyond it.  The paper gives no
cutoff radius; it is read here as three regimes of r = |R| / max(d):

* r <  R_NEAR (3):  Newell's closed form - the 27-point second difference of
  the functions f (diagonal) and g (off-diagonal), in plain FP64.
* R_NEAR <= r < R_FAR (40):  the same cell-pair average evaluated by
  Gauss-Legendre quadrature.  Two cells of widths d_k at offset R see the
  point-dipole kernel averaged over s = R + t, where each t_k has the
  triangle density (1 - |t_k|/d_k)/d_k on [-d_k, d_k]; each half [-d, 0],
  [0, d] takes an n-point rule with the linear density folded into the
  weights.  This keeps FP64 accuracy where Newell's formula cancels.
* r >= R_FAR:  the 4th-moment asymptotic expansion
  N_ij = -(V/4pi)[1 + sum_k d_k^2/12 d_k^2-derivative + sum_k d_k^4/360 ...
  + sum_{k<l} d_k^2 d_l^2/144 ...] d_i d_j (1/R)
  (moments <t^2> = d^2/6, <t^4> = d^4/15 of the triangle density).

Components are ordered (xx, yy, zz, xy, xz, yz); B_d = -mu0 N M.

Pins (tests/test_oracle_tensor.py): cube self-term 1/3 and trace 1 for any
cuboid, zero trace away from the origin, parity symmetries, point-dipole
limit, 50-digit mpmath Newell values, regime agreement at the cutoffs and
the prism pair-sum identity.
"""
from __future__ import annotations

import functools
import math

import numpy as np

R_NEAR = 3.0
R_FAR = 40.0

COMPONENTS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


# ------------------------------------------------------------ Newell ----

def newell_f(x, y, z):
    """Newell's f for the diagonal term (even in every argument)."""
    x, y, z = (np.abs(np.asarray(a, dtype=np.float64)) for a in (x, y, z))
    x2, y2, z2 = x * x, y * y, z * z
    R = np.sqrt(x2 + y2 + z2)
    out = (2.0 * x2 - y2 - z2) * R / 6.0
    with np.errstate(divide="ignore", invalid="ignore"):
        p = 0.5 * y * (z2 - x2)
        t = np.where(p != 0.0, p * np.arcsinh(y / np.sqrt(x2 + z2)), 0.0)
        out = out + t
        p = 0.5 * z * (y2 - x2)
        t = np.where(p != 0.0, p * np.arcsinh(z / np.sqrt(x2 + y2)), 0.0)
        out = out + t
        p = x * y * z
        t = np.where(p != 0.0, p * np.arctan(y * z / (x * R)), 0.0)
        out = out - t
    return out


def newell_g(x, y, z):
    """Newell's g for the off-diagonal term (odd in x and in y)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    sgn = np.sign(x) * np.sign(y)
    x, y, z = np.abs(x), np.abs(y), np.abs(z)
    x2, y2, z2 = x * x, y * y, z * z
    R = np.sqrt(x2 + y2 + z2)
    out = -x * y * R / 3.0
    with np.errstate(divide="ignore", invalid="ignore"):
        terms_asinh = (
            (x * y * z, z / np.sqrt(x2 + y2)),
            (y * (3.0 * z2 - y2) / 6.0, x / np.sqrt(y2 + z2)),
            (x * (3.0 * z2 - x2) / 6.0, y / np.sqrt(x2 + z2)),
        )
        for p, a in terms_asinh:
            out = out + np.where(p != 0.0, p * np.arcsinh(a), 0.0)
        terms_atan = (
            (z2 * z / 6.0, x * y / (z * R)),
            (0.5 * z * y2, x * z / (y * R)),
            (0.5 * z * x2, y * z / (x * R)),
        )
        for p, a in terms_atan:
            out = out - np.where(p != 0.0, p * np.arctan(a), 0.0)
    return sgn * out


_W = {-1: -1.0, 0: 2.0, 1: -1.0}


def _second_difference(fun, X, Y, Z, dx, dy, dz):
    acc = 0.0
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            for c in (-1, 0, 1):
                acc = acc + _W[a] * _W[b] * _W[c] * fun(
                    X + a * dx, Y + b * dy, Z + c * dz)
    return acc / (4.0 * math.pi * dx * dy * dz)


def newell_tensor(X, Y, Z, d):
    """Newell's analytic N at offsets (X, Y, Z) in metres; shape (6, ...)."""
    dx, dy, dz = d
    X, Y, Z = (np.asarray(a, dtype=np.float64) for a in (X, Y, Z))
    nxx = _second_difference(newell_f, X, Y, Z, dx, dy, dz)
    nyy = _second_difference(newell_f, Y, X, Z, dy, dx, dz)
    nzz = _second_difference(newell_f, Z, Y, X, dz, dy, dx)
    nxy = _second_difference(newell_g, X, Y, Z, dx, dy, dz)
    nxz = _second_difference(newell_g, X, Z, Y, dx, dz, dy)
    nyz = _second_difference(newell_g, Y, Z, X, dy, dz, dx)
    return np.stack(np.broadcast_arrays(nxx, nyy, nzz, nxy, nxz, nyz))


# -------------------------------------------------------- quadrature ----

def quad_points(aspect: float) -> int:
    """Gauss-Legendre points per half-axis: 8 for near-cubic cells, else 12."""
    return 8 if aspect <= 1.25 else 12


@functools.lru_cache(maxsize=8)
def triangle_rule(n: int):
    """Nodes/weights on [-1, 1] for the density (1 - |t|) (unit width).

    Each half is an n-point Gauss-Legendre rule on [0, 1] (or [-1, 0]) with
    the linear density multiplied into the weights; weights sum to 1.
    """
    x, w = np.polynomial.legendre.leggauss(n)
    t = 0.5 * (x + 1.0)              # nodes on [0, 1]
    wt = 0.5 * w * (1.0 - t)         # weights for density (1 - t) on [0, 1]
    nodes = np.concatenate([-t[::-1], t])
    weights = np.concatenate([wt[::-1], wt])
    return nodes, weights


def dipole_kernel(sx, sy, sz):
    """d_i d_j (1/|s|) = (3 s_i s_j - delta_ij s^2)/s^5, shape (6, ...)."""
    s2 = sx * sx + sy * sy + sz * sz
    inv5 = 1.0 / (s2 * s2 * np.sqrt(s2))
    return np.stack([
        (3.0 * sx * sx - s2) * inv5,
        (3.0 * sy * sy - s2) * inv5,
        (3.0 * sz * sz - s2) * inv5,
        3.0 * sx * sy * inv5,
        3.0 * sx * sz * inv5,
        3.0 * sy * sz * inv5,
    ])


def quad_tensor(X, Y, Z, d, n=None, chunk=64):
    """Cell-pair quadrature of N at offsets (X, Y, Z) (1-D arrays, metres)."""
    dx, dy, dz = d
    if n is None:
        n = quad_points(max(d) / min(d))
    t, w = triangle_rule(n)
    tx, ty, tz = t * dx, t * dy, t * dz
    W = (w[:, None, None] * w[None, :, None] * w[None, None, :]).ravel()
    TX = np.broadcast_to(tx[:, None, None], (2 * n,) * 3).ravel()
    TY = np.broadcast_to(ty[None, :, None], (2 * n,) * 3).ravel()
    TZ = np.broadcast_to(tz[None, None, :], (2 * n,) * 3).ravel()
    X, Y, Z = (np.atleast_1d(np.asarray(a, dtype=np.float64)) for a in (X, Y, Z))
    out = np.empty((6, X.size))
    pref = -(dx * dy * dz) / (4.0 * math.pi)
    for s in range(0, X.size, chunk):
        e = min(X.size, s + chunk)
        k = dipole_kernel(X[s:e, None] + TX[None, :],
                          Y[s:e, None] + TY[None, :],
                          Z[s:e, None] + TZ[None, :])
        out[:, s:e] = pref * (k @ W)
    return out


# --------------------------------------------------- moment expansion ----

@functools.lru_cache(maxsize=1)
def _derivative_table():
    """Exact d^a_x d^b_y d^c_z (1/r) for a+b+c in {2, 4, 6} (sympy)."""
    import sympy as sp

    x, y, z = sp.symbols("x y z", real=True)
    r = sp.sqrt(x * x + y * y + z * z)
    base = 1 / r
    table = {}
    for order in (2, 4, 6):
        for a in range(order + 1):
            for b in range(order + 1 - a):
                c = order - a - b
                expr = base
                if a:
                    expr = sp.diff(expr, x, a)
                if b:
                    expr = sp.diff(expr, y, b)
                if c:
                    expr = sp.diff(expr, z, c)
                expr = sp.factor(expr)
                table[(a, b, c)] = sp.lambdify((x, y, z), expr, "numpy")
    return table


def moment_tensor(X, Y, Z, d):
    """4th-moment asymptotic N at offsets (X, Y, Z) (metres), shape (6, ...)."""
    D = _derivative_table()
    dx, dy, dz = d
    dd = (dx, dy, dz)
    X, Y, Z = (np.asarray(a, dtype=np.float64) for a in (X, Y, Z))
    pref = -(dx * dy * dz) / (4.0 * math.pi)
    comps = []
    for (i, j) in COMPONENTS:
        base = [0, 0, 0]
        base[i] += 1
        base[j] += 1

        def term(extra):
            idx = tuple(base[k] + extra[k] for k in range(3))
            return D[idx](X, Y, Z)

        acc = term((0, 0, 0))
        for k in range(3):
            e2 = [0, 0, 0]
            e2[k] = 2
            e4 = [0, 0, 0]
            e4[k] = 4
            acc = acc + dd[k] ** 2 / 12.0 * term(e2)
            acc = acc + dd[k] ** 4 / 360.0 * term(e4)
        for k in range(3):
            for l in range(k + 1, 3):
                e = [0, 0, 0]
                e[k] = 2
                e[l] = 2
                acc = acc + dd[k] ** 2 * dd[l] ** 2 / 144.0 * term(e)
        comps.append(pref * acc)
    return np.stack(np.broadcast_arrays(*comps))


# ----------------------------------------------------------- assembly ----

def tensor_at(X, Y, Z, d):
    """N at arbitrary offsets (1-D arrays, metres), regime by r = |R|/max d."""
    X, Y, Z = (np.atleast_1d(np.asarray(a, dtype=np.float64)) for a in (X, Y, Z))
    r = np.sqrt(X * X + Y * Y + Z * Z) / max(d)
    out = np.empty((6, X.size))
    near = r < R_NEAR
    far = r >= R_FAR
    mid = ~(near | far)
    if near.any():
        out[:, near] = newell_tensor(X[near], Y[near], Z[near], d)
    if mid.any():
        out[:, mid] = quad_tensor(X[mid], Y[mid], Z[mid], d)
    if far.any():
        out[:, far] = moment_tensor(X[far], Y[far], Z[far], d)
    return out


def demag_tensor(n, d):
    """N on all non-negative offsets 0 <= X < nx, 0 <= Y < ny, 0 <= Z < nz.

    Returns shape (6, nz, ny, nx); index [c, Z, Y, X] is offset
    (X dx, Y dy, Z dz).  Other octants follow from the parity of each
    component (diagonal even; xy odd in X, Y; xz odd in X, Z; yz odd in Y, Z).
    """
    nx, ny, nz = n
    dx, dy, dz = d
    Zi, Yi, Xi = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                             indexing="ij")
    vals = tensor_at((Xi * dx).ravel(), (Yi * dy).ravel(), (Zi * dz).ravel(), d)
    return vals.reshape(6, nz, ny, nx)


PARITY = {  # sign of component under X -> -X, Y -> -Y, Z -> -Z
    0: (1, 1, 1), 1: (1, 1, 1), 2: (1, 1, 1),
    3: (-1, -1, 1), 4: (-1, 1, -1), 5: (1, -1, -1),
}


def full_tensor_value(N6, X, Y, Z):
    """N(X, Y, Z) for signed integer offsets from the octant table."""
    out = np.empty(6)
    for c in range(6):
        sx, sy, sz = PARITY[c]
        s = 1.0
        if X < 0:
            s *= sx
        if Y < 0:
            s *= sy
        if Z < 0:
            s *= sz
        out[c] = s * N6[c, abs(Z), abs(Y), abs(X)]
    return out
