"""Pins for the oracle's time integration and torques (not GPU).

* Every pair of the solver table meets Butcher's order conditions (all
  rooted trees, exact in fractions) up to exactly its printed convergence
  order (b) and error-estimate order (b*), with row sums c_i; first-same-
  as-last pairs end on b.
* Each pair converges at its printed order on a smooth ODE, and its error
  estimate scales as h^(q+1).
* A single spin in a static field B z follows the closed-form damped
  precession phi = phi0 + g' B t, tan(theta/2) = tan(theta0/2) exp(-a g' B t),
  g' = gamma/(1+a^2); the precession frequency is gamma B/(2 pi (1+a^2)).
  A one-cell cube with demag on gives the same (its self-field is parallel
  to m).
* Two sublattices coupled by homogeneous exchange with uniaxial anisotropy
  resonate at omega = gamma sqrt(B_A (2 B_E + B_A)) (Kittel-Keffer AFMR),
  B_E = 4|A0|/(Ms a^2), B_A = 2K/Ms.
* |m| = 1 after every step; energy does not increase with damping, no
  current and no time dependence.
* Zhang-Li: a uniform state feels no spin-transfer torque.
"""
import json
import math
import os
from fractions import Fraction as F

import numpy as np
import pytest

from oracle import rk
from oracle import torque as tq
from oracle.system import Problem
from paper_2411_18194_amd import inputs


# ------------------------------------------------ Butcher order conditions --
# Rooted trees in canonical form (a tree is the sorted tuple of its
# subtrees); every tree of order n + 1 arises by attaching a leaf to some
# node of a tree of order n.

def _canon(t):
    return tuple(sorted(_canon(c) for c in t))


def _grow(t):
    out = {_canon(t + ((),))}
    for i, c in enumerate(t):
        for g in _grow(c):
            out.add(_canon(t[:i] + (g,) + t[i + 1:]))
    return out


def _trees(n):
    level = {()}
    for _ in range(n - 1):
        level = set().union(*(_grow(t) for t in level))
    return sorted(level)


def _order(t):
    return 1 + sum(_order(c) for c in t)


def _gamma(t):
    g = _order(t)
    for c in t:
        g *= _gamma(c)
    return g


def _phi(tab, t):
    """Elementary weights Phi_i(t) of every stage i."""
    s = tab.stages
    out = [F(1)] * s
    for c in t:
        pc = _phi(tab, c)
        for i in range(s):
            out[i] *= sum((tab.a[i][j] * pc[j] for j in range(i)), F(0))
    return out


def _meets(tab, w, t):
    return sum(wi * x for wi, x in zip(w, _phi(tab, t))) == F(1, _gamma(t))


def test_rooted_tree_counts():
    # 1, 1, 2, 4, 9, 20 rooted trees of orders 1..6
    assert [len(_trees(n)) for n in range(1, 7)] == [1, 1, 2, 4, 9, 20]


def _printed():
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_printed.json")) as fh:
        return json.load(fh)["rk_solvers"]


SOLVERS = {"heun": "Heun", "bs23": "Bogacki-Shampine", "cashkarp": "Cash-Karp",
           "rkf45": "Fehlberg", "dp45": "Dormand-Prince"}


@pytest.mark.parametrize("name", sorted(SOLVERS))
def test_order_conditions(name):
    """b has exactly the printed convergence order and b* the printed
    error-estimate order: every condition up to that order holds exactly,
    and one of the next order fails."""
    tab = rk.TABLEAUS[name]
    p, q = _printed()[SOLVERS[name]]
    assert (tab.p, tab.q) == (p, q)
    s = tab.stages
    assert len(tab.a) == s and len(tab.b) == s and len(tab.bs) == s
    for i in range(s):
        assert len(tab.a[i]) == i and sum(tab.a[i], F(0)) == tab.c[i]
    for w, order in ((tab.b, p), (tab.bs, q)):
        for n in range(1, order + 1):
            for t in _trees(n):
                assert _meets(tab, w, t), (name, order, t)
        assert not all(_meets(tab, w, t) for t in _trees(order + 1)), (name, order)
    if tab.fsal:
        # the last stage is evaluated at the propagated solution
        assert tab.c[-1] == 1 and tab.b[-1] == 0 and tuple(tab.a[-1]) == tuple(tab.b[:-1])


def _ode(t, y):
    return [np.array([y[0][0] * math.cos(t) - y[0][1], y[0][0] + 0.3 * y[0][1]])]


def _integrate(tab, n, t_end=2.0):
    st = rk.Stepper(_ode, lambda y: y, lambda e: 0.0, tab)
    y = [np.array([1.0, 0.5])]
    h = t_end / n
    for i in range(n):
        y, kn, _ = st.step(i * h, y, h)
        st.accept(kn)
    return y[0]


@pytest.mark.parametrize("name", sorted(SOLVERS))
def test_convergence_order(name):
    """Halving the step divides the global error by ~2^p."""
    tab = rk.TABLEAUS[name]
    ref = _integrate(rk.DORMAND_PRINCE, 4096)
    n = {2: 128, 3: 64, 5: 16}[tab.p]
    e1 = np.abs(_integrate(tab, n) - ref).max()
    e2 = np.abs(_integrate(tab, 2 * n) - ref).max()
    assert 0.75 * 2 ** tab.p < e1 / e2 < 1.3 * 2 ** tab.p, (name, e1 / e2)


@pytest.mark.parametrize("name", sorted(SOLVERS))
def test_error_estimate_order(name):
    """The one-step estimate |h sum e_j k_j| scales as h^(q+1)."""
    tab = rk.TABLEAUS[name]

    def est(h):
        st = rk.Stepper(_ode, lambda y: y, lambda e: float(np.abs(e[0]).max()), tab)
        return st.step(0.3, [np.array([1.0, 0.5])], h)[2]
    r = est(0.02) / est(0.01)
    assert 0.75 * 2 ** (tab.q + 1) < r < 1.3 * 2 ** (tab.q + 1), (name, r)


def _single_spin(alpha, B, th0, t_end, demag=False, solver="dp45", tol=1e-9):
    p = inputs.base_params((1, 1, 1), (3e-9,) * 3)
    p.update(Ms=[8e5], alpha=[alpha], B_ext=(0.0, 0.0, B), demag=demag, solver=solver)
    m = np.array([math.sin(th0), 0.0, math.cos(th0)]).reshape(1, 3, 1, 1, 1)
    P = Problem(p)
    y, t, info, s = P.run([m], 0.0, t_end, tol=tol, dt0=1e-14,
                          sample_every=t_end / 20, sample=lambda y: y[0].ravel().copy())
    assert t == t_end and len(s) == 21
    return p, s


@pytest.mark.parametrize("alpha,demag,solver,tol", [
    (0.0, False, "dp45", 1e-9), (0.1, False, "dp45", 1e-9), (0.02, True, "dp45", 1e-9),
    (0.1, False, "heun", 1e-7), (0.1, False, "bs23", 1e-8), (0.1, False, "cashkarp", 1e-8),
    (0.1, False, "rkf45", 1e-8)])
def test_single_spin_closed_form(alpha, demag, solver, tol):
    """Adaptive runs under every pair of the solver table."""
    B, th0 = 0.1, 1.0
    p, s = _single_spin(alpha, B, th0, 200e-12, demag, solver, tol)
    gp = p["gamma"] / (1 + alpha ** 2)
    for t, m in s:
        th = 2 * math.atan(math.tan(th0 / 2) * math.exp(-alpha * gp * B * t))
        ph = gp * B * t
        ref = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
        assert np.abs(m - ref).max() < 2e-6
        assert abs(np.linalg.norm(m) - 1) < 1e-14


def test_afmr_frequency():
    Ms, A0, a, K = 4e5, -1e-13, 0.35e-9, 6e4
    p = inputs.base_params((1, 1, 1), (1e-9,) * 3, nsub=2)
    p.update(Ms=[Ms, Ms], A0=A0, latcon=a, Ku1=[K, K], alpha=[0.0, 0.0])
    BE = 4 * abs(A0) / (Ms * a * a)
    BA = 2 * K / Ms
    w = p["gamma"] * math.sqrt(BA * (2 * BE + BA))
    T = 2 * math.pi / w
    eps = 0.01
    m = np.zeros((2, 3, 1, 1, 1))
    m[0, :, 0, 0, 0] = [math.sin(eps), 0, math.cos(eps)]
    m[1, :, 0, 0, 0] = [math.sin(eps), 0, -math.cos(eps)]
    P = Problem(p)
    n = 200
    y, t, info, s = P.run([m], 0.0, 4 * T, tol=1e-10, dt0=1e-15,
                          sample_every=4 * T / n, sample=lambda y: y[0][0, 0].ravel()[0])
    ts = np.array([a for a, _ in s])
    mx = np.array([b for _, b in s])
    # least-squares fit of a cos(wt) + b sin(wt) + c over a fine grid of w
    ws = np.linspace(0.9 * w, 1.1 * w, 2001)
    res = []
    for wi in ws:
        X = np.stack([np.cos(wi * ts), np.sin(wi * ts), np.ones_like(ts)], axis=1)
        coef, r, *_ = np.linalg.lstsq(X, mx, rcond=None)
        res.append(np.sum((X @ coef - mx) ** 2))
    wfit = ws[int(np.argmin(res))]
    assert wfit == pytest.approx(w, rel=2e-3)


def test_energy_decreases_and_norm():
    p, m0 = inputs.config_c1()
    p = dict(p)
    p["alpha"] = [0.5]
    P = Problem(p)
    y = [m0.copy()]
    E_prev = sum(P.energies(y[0]).values())
    t = 0.0
    for _ in range(8):
        y, t, info, _ = P.run(y, t, t + 2e-12, tol=1e-6, dt0=1e-14)
        E = sum(P.energies(y[0]).values())
        assert E <= E_prev + 1e-12 * abs(E_prev)
        E_prev = E
        assert np.abs(np.linalg.norm(y[0], axis=1) - 1).max() < 1e-14


def test_zhang_li_uniform_zero():
    m = np.zeros((3, 1, 4, 5))
    m[0] = 0.6
    m[1] = 0.8
    u = tq.drift_velocity(0.5, (1e12, 0, 0), 4e5)
    assert np.abs(tq.zhang_li_torque(m, u, 0.01, 0.1, (1e-9,) * 3)).max() == 0.0
    assert u[0] == pytest.approx(0.5 * 9.2740100783e-24 * 1e12 / (1.602176634e-19 * 4e5))


def test_output_times_merge_with_the_end():
    """Sampling every 1e-11 s up to 5e-11 s: 5 * 1e-11 is not 5e-11 in
    floating point, yet the run ends at t_end with one sample per output time
    (the last one at t_end) instead of a spurious ~1e-26 s landing step."""
    p = inputs.base_params((1, 1, 1), (2e-9,) * 3)
    p.update(Ms=[8e5], A11=[0.0], alpha=[0.1], B_ext=(0.0, 0.0, 0.1), demag=False)
    P = Problem(p)
    m = np.zeros((1, 3, 1, 1, 1))
    m[0, 0] = 1.0
    every, t_end = 1e-11, 0.05e-9
    assert 5 * every != t_end
    y, t, info, samples = P.run(P.initial_state(m), 0.0, t_end, sample_every=every,
                                sample=lambda y: y[0].copy())
    assert t == t_end
    ts = [s[0] for s in samples]
    assert len(ts) == 6 and ts[-1] == t_end
    assert np.allclose(ts, np.arange(6) * every, rtol=1e-12, atol=0)


def test_step_size_rule_parameters():
    """The step-size rule with explicit safety, clamps and dt_max: an error
    equal to tol scales the step by the safety factor alone; a tiny error
    (or zero) hits fac_max, a huge one fac_min; dt_max caps the result."""
    dt, tol = 1e-13, 1e-5
    kw = dict(safety=0.9, fac_min=0.2, fac_max=5.0)
    assert rk.new_dt(dt, tol, tol, 4, **kw) == pytest.approx(0.9 * dt, rel=1e-15)
    assert rk.new_dt(dt, tol * 2 ** 5, tol, 4, **kw) == pytest.approx(0.45 * dt, rel=1e-14)
    assert rk.new_dt(dt, 1e-30, tol, 4, **kw) == 5.0 * dt
    assert rk.new_dt(dt, 0.0, tol, 4, **kw) == 5.0 * dt
    assert rk.new_dt(dt, 1.0, tol, 4, **kw) == 0.2 * dt
    assert rk.new_dt(dt, 0.0, tol, 4, dt_max=3e-13, **kw) == 3e-13
    assert rk.new_dt(dt, tol, tol, 4) == pytest.approx(0.8 * dt, rel=1e-15)


def test_dt_max_bounds_every_step():
    """An adaptive run with dt_max takes no step longer than dt_max: the
    times it lands on are spaced by at most dt_max, and it needs at least
    T/dt_max steps."""
    p, m0 = inputs.config_c1()
    T, dmax = 20e-12, 2.5e-13
    q = dict(p, dt_max=dmax)
    P = Problem(q)
    times = []
    P.stepper.step = _record(P.stepper.step, times)
    _, t, info, _ = P.run([m0.copy()], 0.0, T, tol=1e-5, dt0=1e-12)
    assert t == T and info["steps"] >= math.ceil(T / dmax)
    assert max(times) <= dmax
    free = Problem(p).run([m0.copy()], 0.0, T, tol=1e-5, dt0=1e-12)[2]
    assert free["steps"] < info["steps"]


def _record(step, out):
    def wrapped(t, y, h):
        out.append(h)
        return step(t, y, h)
    return wrapped


@pytest.mark.parametrize("bad", [dict(fac_min=1.0), dict(fac_min=1.5), dict(safety=1.2),
                                 dict(fac_max=0.5)])
def test_step_control_that_cannot_shrink_is_rejected(bad):
    """With fac_min >= 1 a rejected attempt would retry the same step
    forever; such settings are refused before the first step."""
    p, m0 = inputs.config_c1()
    P = Problem(dict(p, **bad))
    with pytest.raises(ValueError):
        P.run([m0.copy()], 0.0, 1e-12, tol=1e-5, dt0=1e-13)
