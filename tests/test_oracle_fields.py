"""Pins for the oracle's short-range field terms (not GPU).

* Exchange: a spin spiral (cos kx, sin kx, 0) is an eigenvector of the
  discrete Laplacian, so in the interior B = -(2A/Ms)(2 - 2 cos k d)/d^2 m.
* Interfacial DMI: a cycloid (cos kx, 0, sin kx) gives in the interior
  B = (2D/Ms)(sin kd/d)(cos kx, 0, sin kx).
* Uniform states feel no exchange, no inter-sublattice Laplacian term.
* Field = -(1/(Ms V)) dE/dm (finite differences of the FP64 energy).  For
  the local terms (anisotropy, Zeeman, magnetoelastic) the oracle's energy
  densities are written independently of its fields; for the bilinear
  terms (exchange, A12, A0, DMI) the oracle's energy is -1/2 M.B of the
  same operator, which only shows the operator is symmetric, so those
  fields are also checked against energies written here from scratch: a
  sum over nearest-neighbour links of A |m_j - m_i|^2 (exchange),
  A12 (m1_j - m1_i).(m2_j - m2_i) (inhomogeneous inter-sublattice), the
  homogeneous -4 A0/a^2 m1.m2 per cell and the interfacial DMI density
  D [m_z div m - (m.grad) m_z] with central differences (interior).
  Magnitudes are pinned again by the spiral and cycloid closed forms.
* The edge canting along x of a relaxed wide strip with exchange +
  interfacial DMI + perpendicular anisotropy converges to the 1-D problem
  A theta'' = K sin(theta) cos(theta), theta' = -D/(2A) at both ends
  (natural boundary condition of the DMI energy), solved by scipy.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_bvp

from oracle import fields as fl
from oracle.system import Problem, TERMS
from paper_2411_18194_amd import inputs


def test_exchange_spin_spiral():
    n, d = (40, 3, 1), (1e-9, 1e-9, 1e-9)
    k = 2 * math.pi / 17e-9
    x = np.arange(n[0]) * d[0]
    m = np.zeros((3, 1, 3, 40))
    m[0] = np.cos(k * x)
    m[1] = np.sin(k * x)
    A, Ms = 1.3e-11, 8e5
    B = fl.exchange_field(m, Ms, A, d)
    ref = -(2 * A / Ms) * (2 - 2 * math.cos(k * d[0])) / d[0] ** 2 * m
    inner = (slice(None), slice(None), slice(None), slice(1, -1))
    assert np.abs(B[inner] - ref[inner]).max() < 1e-12 * np.abs(ref).max()


def test_dmi_cycloid():
    n, d = (40, 4, 1), (2e-9, 2e-9, 2e-9)
    k = 2 * math.pi / 23e-9
    x = np.arange(n[0]) * d[0]
    m = np.zeros((3, 1, 4, 40))
    m[0] = np.cos(k * x)
    m[2] = np.sin(k * x)
    D, Ms, A = 3e-3, 1.1e6, 1.5e-11
    B = fl.dmi_field(m, Ms, A, D, d)
    ref = (2 * D / Ms) * math.sin(k * d[0]) / d[0] * np.stack(
        [np.cos(k * x), 0 * x, np.sin(k * x)])[:, None, None, :]
    inner = (slice(None), slice(None), slice(1, -1), slice(1, -1))
    assert np.abs(B[inner] - np.broadcast_to(ref, B.shape)[inner]).max() < 1e-12 * np.abs(ref).max()


def test_uniform_no_exchange():
    m = np.zeros((3, 2, 5, 6))
    m[0] = 0.6
    m[2] = 0.8
    assert np.abs(fl.exchange_field(m, 8e5, 1e-11, (1e-9,) * 3)).max() == 0.0
    assert np.abs(fl.afm_nn_field(m, 8e5, -5e-12, (1e-9,) * 3)).max() == 0.0


def _energy_gradient_check(p, m, terms, interior_only=False, u=None):
    P = Problem(p)
    V = P.V
    B = P.eval_heff(m, terms, u=u)
    rng = np.random.default_rng(3)
    nsub, _, nz, ny, nx = m.shape
    for _ in range(6):
        s = rng.integers(nsub)
        c = rng.integers(3)
        if interior_only:
            z = rng.integers(nz)
            y = rng.integers(1, ny - 1)
            x = rng.integers(1, nx - 1)
        else:
            z, y, x = rng.integers(nz), rng.integers(ny), rng.integers(nx)
        h = 1e-6

        def E(delta):
            mm = m.copy()
            mm[s, c, z, y, x] += delta
            en = P.energies(mm, u=u)
            return sum(en[t] for t in terms)
        g = (E(h) - E(-h)) / (2 * h)
        expect = -g / (p["Ms"][s] * V)
        assert B[s, c, z, y, x] == pytest.approx(expect, rel=2e-6, abs=1e-9 * np.abs(B).max())


def test_energy_gradient_local_terms():
    p = inputs.base_params((5, 4, 2), (2e-9, 3e-9, 1e-9), nsub=2)
    p.update(Ms=[8e5, 5e5], Ku1=[5e5, 3e5], Ku2=[1e5, 0.0],
             anis_u=[(0.6, 0, 0.8), (0, 1, 0)], Kc1=[2e4, -3e4],
             cub_c1=[(1, 0, 0), (0.6, 0.8, 0)], cub_c2=[(0, 1, 0), (-0.8, 0.6, 0)],
             B_ext=(0.01, -0.02, 0.05), A0=-2e-11, latcon=0.35e-9)
    m = inputs.random_unit(inputs.rng(1), 2, p["n"])
    for terms in (("anis_u",), ("anis_c",), ("zeeman",), ("afm_cell",)):
        _energy_gradient_check(p, m, terms)


def test_energy_gradient_exchange_afm():
    p = inputs.base_params((6, 5, 3), (2e-9, 3e-9, 1.5e-9), nsub=2)
    p.update(Ms=[8e5, 5e5], A11=[1e-11, 2e-11], A12=-5e-12)
    m = inputs.random_unit(inputs.rng(2), 2, p["n"])
    _energy_gradient_check(p, m, ("exch",))
    _energy_gradient_check(p, m, ("afm_nn",))


def test_energy_gradient_dmi_bulk():
    p = inputs.base_params((8, 7, 2), (2e-9, 2e-9, 2e-9))
    p.update(Ms=[1.1e6], A11=[1.5e-11], Dint=[3e-3], dmi_layer=0)
    m = inputs.random_unit(inputs.rng(3), 1, p["n"])
    _energy_gradient_check(p, m, ("dmi",), interior_only=True)
    _energy_gradient_check(p, m, ("exch",), interior_only=True)


def _link_energy_checks(p, m, field_terms, energy, interior_only=False):
    """Field of the named terms against -(1/(Ms V)) dE/dm of `energy`."""
    P = Problem(p)
    B = P.eval_heff(m, field_terms)
    rng = np.random.default_rng(11)
    nsub, _, nz, ny, nx = m.shape
    for _ in range(8):
        s, c = rng.integers(nsub), rng.integers(3)
        z = rng.integers(nz)
        y = rng.integers(1, ny - 1) if interior_only else rng.integers(ny)
        x = rng.integers(1, nx - 1) if interior_only else rng.integers(nx)
        h = 1e-6
        mp, mm_ = m.copy(), m.copy()
        mp[s, c, z, y, x] += h
        mm_[s, c, z, y, x] -= h
        g = (energy(mp) - energy(mm_)) / (2 * h)
        expect = -g / (p["Ms"][s] * P.V)
        assert B[s, c, z, y, x] == pytest.approx(expect, rel=2e-6, abs=1e-9 * np.abs(B).max())


def _links(f, axis):
    """Differences f_j - f_i over the nearest-neighbour links along a spatial
    axis (0 = x) of a (3, nz, ny, nx) field."""
    return np.diff(f, axis=3 - axis)


def test_energy_gradient_against_link_energies():
    d = (2e-9, 3e-9, 1.5e-9)
    p = inputs.base_params((6, 5, 3), d, nsub=2)
    p.update(Ms=[8e5, 5e5], A11=[1e-11, 2e-11], A12=-5e-12, A0=-2e-11, latcon=0.35e-9)
    m = inputs.random_unit(inputs.rng(12), 2, p["n"])
    V = d[0] * d[1] * d[2]

    def e_exch(mm):
        return sum(p["A11"][s] * V / d[a] ** 2 * np.sum(_links(mm[s], a) ** 2)
                   for s in range(2) for a in range(3))

    def e_a12(mm):
        return sum(p["A12"] * V / d[a] ** 2 * np.sum(_links(mm[0], a) * _links(mm[1], a))
                   for a in range(3))

    def e_a0(mm):
        return -4.0 * p["A0"] / p["latcon"] ** 2 * V * np.sum(mm[0] * mm[1])

    _link_energy_checks(p, m, ("exch",), e_exch)
    _link_energy_checks(p, m, ("afm_nn",), e_a12)
    _link_energy_checks(p, m, ("afm_cell",), e_a0)


def test_dmi_field_against_its_energy_density():
    d = (2e-9, 2.5e-9, 2e-9)
    p = inputs.base_params((9, 8, 1), d)
    D = 3e-3
    p.update(Ms=[1.1e6], Dint=[D], dmi_layer=0)
    m = inputs.random_unit(inputs.rng(13), 1, p["n"])
    V = d[0] * d[1] * d[2]

    def cdiff(f, axis):
        # central difference on the cells that have both neighbours
        g = np.moveaxis(f, 2 - axis, 0)
        return np.moveaxis((g[2:] - g[:-2]) / (2 * d[axis]), 0, 2 - axis)

    def energy(mm):
        mx, my, mz = mm[0, 0], mm[0, 1], mm[0, 2]        # (nz, ny, nx)
        e = 0.0
        # x part on cells with both x neighbours, y part likewise
        e += np.sum(mz[:, :, 1:-1] * cdiff(mx, 0) - mx[:, :, 1:-1] * cdiff(mz, 0))
        e += np.sum(mz[:, 1:-1, :] * cdiff(my, 1) - my[:, 1:-1, :] * cdiff(mz, 1))
        return D * V * e

    # the field two cells in from every edge sees only interior energy terms
    P = Problem(p)
    B = P.eval_heff(m, ("dmi",))
    for (y, x, c) in [(3, 4, 0), (4, 2, 1), (5, 6, 2), (2, 3, 2), (4, 5, 0)]:
        h = 1e-6
        mp, mm_ = m.copy(), m.copy()
        mp[0, c, 0, y, x] += h
        mm_[0, c, 0, y, x] -= h
        expect = -(energy(mp) - energy(mm_)) / (2 * h) / (p["Ms"][0] * V)
        assert B[0, c, 0, y, x] == pytest.approx(expect, rel=2e-6, abs=1e-9 * np.abs(B).max())


def test_magnetoelastic_energy_gradient():
    p = inputs.base_params((6, 5, 1), (2e-9, 2e-9, 2e-9), nsub=2)
    p.update(Ms=[4e5, 3e5], B1=[-6e6, 2e6], B2=[-3e6, 5e6],
             elastic=dict(rho=6800.0, C11=3.2e11, C12=1.3e11, C44=1.1e11,
                          eta=0.0, trac_amp=0.0, trac_freq=0.0))
    m = inputs.random_unit(inputs.rng(4), 2, p["n"])
    u = inputs.rng(5).standard_normal((3, 1, 5, 6)) * 1e-11
    _energy_gradient_check(p, m, ("mel",), u=u)


def _relax_strip(nx, ny, dx, A, D, K, Ms):
    p = inputs.base_params((nx, ny, 1), (dx, dx, dx))
    p.update(Ms=[Ms], A11=[A], Dint=[D], Ku1=[K], anis_u=[(0, 0, 1)],
             alpha=[1.0])
    m = np.zeros((1, 3, 1, ny, nx))
    m[0, 2] = 1.0
    P = Problem(p)
    y, t, info, _ = P.run([m], 0.0, 0.3e-9, tol=1e-7, dt0=1e-14)
    mm = y[0][0, :, 0, ny // 2, :]
    return np.arctan2(mm[0], mm[2])


def test_dmi_edge_canting_bvp():
    """Middle row of a wide strip vs the 1-D natural-BC problem along x.

    The strip is 40 nm long and 60 nm wide (15 exchange lengths), so the
    y-edge canting has decayed to ~1e-4 rad at the middle row.
    """
    A, D, K, Ms = 1.5e-11, 3e-3, 1e6, 1.1e6
    L = 40e-9
    # lengths in nm for the solver
    kk = K / A * 1e-18
    slope = -D / (2 * A) * 1e-9

    def f(x, y):
        return np.vstack([y[1], kk * np.sin(y[0]) * np.cos(y[0])])

    def bc(ya, yb):
        return np.array([ya[1] - slope, yb[1] - slope])

    xs = np.linspace(0, L * 1e9, 401)
    sol = solve_bvp(f, bc, xs, np.zeros((2, xs.size)), tol=1e-10, max_nodes=100000)
    assert sol.success
    # the continuum edge angle obeys sin(theta0) = D / (2 sqrt(A K))
    assert math.sin(sol.sol(0.0)[0]) == pytest.approx(D / (2 * math.sqrt(A * K)), rel=1e-3)
    errs = []
    for nx in (20, 40):
        dx = L / nx
        th = _relax_strip(nx, int(round(60e-9 / dx)), dx, A, D, K, Ms)
        xc = (np.arange(nx) + 0.5) * dx
        ref = sol.sol(xc * 1e9)[0]
        errs.append(np.abs(th - ref).max())
    # converges (first order: the ghost carries the face derivative from the
    # cell centre) to the continuum profile
    assert errs[1] < 0.005 * abs(sol.sol(0.0)[0])
    assert errs[0] / errs[1] > 1.7


def test_homogeneous_dmi():
    """d.(m1 x m2): the energy gradient is the field, and the closed forms
    for m1 = x, m2 = y, d = D z: energy D V per cell, B1 = -D/Ms1 x,
    B2 = -D/Ms2 y."""
    p = inputs.base_params((4, 3, 2), (2e-9, 2e-9, 1e-9), nsub=2)
    p.update(Ms=[4e5, 3e5], dmi_homo=(2e5, -1e5, 3e5))
    m = inputs.random_unit(inputs.rng(6), 2, p["n"])
    _energy_gradient_check(p, m, ("dmi",))
    D = 7e5
    p.update(dmi_homo=(0.0, 0.0, D))
    m = np.zeros((2, 3, 2, 3, 4))
    m[0, 0] = 1.0
    m[1, 1] = 1.0
    P = Problem(p)
    B = P.eval_heff(m, ("dmi",))
    assert np.allclose(B[0, 0], -D / 4e5, rtol=1e-15) and np.allclose(B[0, 1:], 0)
    assert np.allclose(B[1, 1], -D / 3e5, rtol=1e-15) and np.allclose(B[1, [0, 2]], 0)
    assert P.energies(m)["dmi"] == pytest.approx(D * P.V * 24, rel=1e-14)


def _three(n=(5, 4, 2), d=(2e-9, 3e-9, 1.5e-9)):
    p = inputs.base_params(n, d, nsub=3)
    p.update(Ms=[4e5, 3e5, 3.5e5], A11=[1e-11, 8e-12, 9e-12], A12=-4e-12, A0=-2e-11,
             latcon=0.4e-9)
    return p


def test_three_sublattices_energy_gradient():
    """Eq. 3 with every pair of three sublattices coupled: the energy
    gradient is the field for both inter-sublattice terms."""
    p = _three()
    m = inputs.random_unit(inputs.rng(8), 3, p["n"])
    _energy_gradient_check(p, m, ("afm_nn",))
    _energy_gradient_check(p, m, ("afm_cell",))


def test_three_sublattices_reduce_to_two():
    """With m3 = m2 the first sublattice feels twice the coupling of a
    two-sublattice magnet with the same A12 and A0."""
    p3 = _three()
    m = inputs.random_unit(inputs.rng(9), 3, p3["n"])
    m[2] = m[1]
    p2 = dict(p3, nsub=2, Ms=p3["Ms"][:2], A11=p3["A11"][:2])
    for k in ("alpha", "Ku1", "Ku2", "anis_u", "Kc1", "cub_c1", "cub_c2", "Dint", "B1", "B2",
              "zl_P", "zl_xi"):
        p2[k] = p3[k][:2]
    b3 = Problem(p3).eval_heff(m, ("afm_nn", "afm_cell"))
    b2 = Problem(p2).eval_heff(m[:2], ("afm_nn", "afm_cell"))
    assert np.allclose(b3[0], 2 * b2[0], rtol=1e-13, atol=0)


def test_three_sublattice_triangular_state_torque_free():
    """The 120 degree state of three equal sublattices (sum m = 0): the
    homogeneous exchange field of each is antiparallel to its own m, so the
    exchange leaves no torque (the non-collinear ground state)."""
    p = _three((3, 3, 1))
    p.update(Ms=[4e5] * 3, A11=[1e-11] * 3, alpha=[0.01] * 3)
    m = np.zeros((3, 3, 1, 3, 3))
    for s in range(3):
        ang = 2 * math.pi * s / 3
        m[s, 0] = math.cos(ang)
        m[s, 1] = math.sin(ang)
    P = Problem(p)
    B = P.eval_heff(m, ("afm_cell",))
    for s in range(3):
        assert np.allclose(np.cross(m[s], B[s], axis=0), 0, atol=1e-9 * np.abs(B).max())
    assert np.abs(P.torque(m)).max() < 1e-9 * P.p["gamma"] * np.abs(B).max()


def _grains(n, seed):
    ids, _ = inputs.voronoi_grains(inputs.rng(seed), n, (2e-9, 2e-9, 2e-9), 5)
    return ids


def test_grain_boundary_exchange_gradient():
    """Scaled links at grain boundaries: the field is still the energy
    gradient (every cell, boundaries and periodic wrap included)."""
    n = (7, 6, 2)
    p = inputs.base_params(n, (2e-9, 2e-9, 2e-9), nsub=2)
    p.update(Ms=[4e5, 3e5], A11=[1e-11, 8e-12], A12=-5e-12, grain=_grains(n, 10),
             grain_axes=np.tile([0.0, 0.0, 1.0], (5, 1)), grain_exchange_scale=0.25,
             pbc=(1, 0, 0))
    m = inputs.random_unit(inputs.rng(11), 2, n)
    _energy_gradient_check(p, m, ("exch",))
    _energy_gradient_check(p, m, ("afm_nn",))


def test_grain_boundary_exchange_limits():
    """Scale 1 is the plain exchange; scale 0 decouples the grains: a state
    uniform inside each grain then has no exchange field."""
    n = (8, 7, 1)
    ids = _grains(n, 12)
    base = inputs.base_params(n, (2e-9, 2e-9, 2e-9))
    base.update(Ms=[8e5], A11=[1.3e-11], grain=ids, grain_axes=np.tile([0.0, 0.0, 1.0], (5, 1)))
    m = inputs.random_unit(inputs.rng(13), 1, n)
    b1 = Problem(dict(base, grain_exchange_scale=1.0)).eval_heff(m, ("exch",))
    b0 = Problem(dict(base)).eval_heff(m, ("exch",))
    assert np.array_equal(b1, b0)
    dirs = inputs.random_unit(inputs.rng(14), 1, (5, 1, 1))[0, :, 0, 0, :]
    mg = dirs[:, ids][None]
    bz = Problem(dict(base, grain_exchange_scale=0.0)).eval_heff(mg, ("exch",))
    assert np.abs(bz).max() < 1e-12 * np.abs(b0).max()
    assert np.abs(Problem(dict(base)).eval_heff(mg, ("exch",))).max() > 0


def test_grain_boundary_exchange_link_energy():
    """Brute force over links: for unit vectors the exchange energy is
    V sum_links w A |m_i - m_j|^2 / d^2, w = scale across a grain boundary
    (periodic wrap along x included)."""
    n = (6, 5, 3)
    d = (2e-9, 2.5e-9, 1.5e-9)
    ids = _grains(n, 15)
    scale, A = 0.3, 1.2e-11
    p = inputs.base_params(n, d)
    p.update(Ms=[7e5], A11=[A], grain=ids, grain_axes=np.tile([0.0, 0.0, 1.0], (5, 1)),
             grain_exchange_scale=scale, pbc=(1, 0, 0))
    m = inputs.random_unit(inputs.rng(16), 1, n)
    P = Problem(p)
    nx, ny, nz = n
    E = 0.0
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                for (ddx, ddy, ddz), h in (((1, 0, 0), d[0]), ((0, 1, 0), d[1]),
                                           ((0, 0, 1), d[2])):
                    X, Y, Z = x + ddx, y + ddy, z + ddz
                    if X == nx:
                        X = 0
                    if Y == ny or Z == nz:
                        continue
                    w = 1.0 if ids[z, y, x] == ids[Z, Y, X] else scale
                    dm = m[0, :, z, y, x] - m[0, :, Z, Y, X]
                    E += w * A * float(dm @ dm) / h ** 2
    E *= P.V
    assert P.energies(m)["exch"] == pytest.approx(E, rel=1e-12)


def test_grain_boundary_exchange_with_dmi_tensors():
    """Grain-boundary scaling over the Eq. 6 ghosts (interfacial DMI tensors
    of a two-sublattice magnet): the bulk field is the energy gradient, and
    the DMI field is not scaled."""
    n = (8, 6, 1)
    D = 1.5e-3
    Wi = [[0.0, D, 0.0], [-D, 0.0, 0.0], [0.0, 0.0, 0.0]]
    p = inputs.base_params(n, (2e-9, 2e-9, 2e-9), nsub=2)
    p.update(Ms=[4e5, 4e5], A11=[1e-11, 1e-11], A0=-2e-11, A12=-4e-12, latcon=0.35e-9,
             bc="eq6", dmi_W=[Wi, Wi], grain=_grains(n, 17),
             grain_axes=np.tile([0.0, 0.0, 1.0], (5, 1)), grain_exchange_scale=0.25)
    m = inputs.random_unit(inputs.rng(18), 2, n)
    for t in ("exch", "afm_nn", "dmi"):
        _energy_gradient_check(p, m, (t,), interior_only=True)
    b1 = Problem(p).eval_heff(m, ("dmi",))
    b0 = Problem(dict(p, grain_exchange_scale=1.0)).eval_heff(m, ("dmi",))
    assert np.array_equal(b1, b0)
    e1 = Problem(p).eval_heff(m, ("exch",))
    e0 = Problem(dict(p, grain_exchange_scale=1.0)).eval_heff(m, ("exch",))
    assert not np.allclose(e1, e0)
