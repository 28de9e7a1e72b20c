"""FP64 energy bookkeeping of the coupled magnetisation-displacement system
("Elasticity" Eq. 7, "Magnetoelasticity" Eq. 8-9, LLG Eq. 1-2) in the oracle.

The total energy of a magnetoelastic racetrack (exchange, inter-sublattice
exchange, cubic anisotropy, magnetoelastic, elastic strain and kinetic)
changes only through

  * the power the boundaries put in, P_b = V sum [sigma:eps(v) + v.f] over
    the elastic stress with its traction rows and the magnetoelastic stress
    sigma_mel = de_mel/deps with its force f_mel (Eq. 8): the discrete form
    of the work of the applied traction and of the magnetostrictive stress
    on the faces;
  * the viscous body force, P_eta = eta sum |v|^2 V;
  * Gilbert damping, P_alpha = sum_s Ms gamma alpha/(1+alpha^2) |m x B_eff|^2 V
    (the LLG dissipation, from the torque's closed form, not from the
    oracle's torque routine).

Test 1 integrates these powers alongside the state with the same
Dormand-Prince stages (an augmented ODE), so E(t) - E(0) - (W_b - W_eta -
W_alpha) is the time-integration error alone: it must fall at (at least) the
pair's fifth order as dt is halved.  That holds only if the field is the
magnetisation gradient of the energy for every term (magnetoelastic field
Eq. 9 included), the torque dissipates at the LLG rate and the viscous term
has the right sign.

Test 2 pins the boundary power itself: on smooth states of a bar that meet
the boundary conditions, the elastic part of P_b tends to the power of the
applied shear traction and the magnetoelastic part to the work of the
magnetostrictive stress on the two faces, both at first order in the cell
size (the paper's lower-order boundary differences); a magnetoelastic force
with the B2 index misread does not converge.
"""
import math

import numpy as np
import pytest

from oracle import elastic as el
from oracle.rk import DORMAND_PRINCE, Stepper
from oracle.system import Problem, TERMS
from paper_2411_18194_amd import inputs

W6 = np.array([1.0, 1.0, 1.0, 2.0, 2.0, 2.0])   # sigma:eps counts ij and ji


def _mel_stress(m, B1, B2):
    """de/deps of e = B1 sum eps_ii m_i^2 + B2 sum_{i != j} eps_ij m_i m_j,
    Voigt order (xx, yy, zz, xy, xz, yz)."""
    return np.stack([B1 * m[0] ** 2, B1 * m[1] ** 2, B1 * m[2] ** 2,
                     B2 * m[0] * m[1], B2 * m[0] * m[2], B2 * m[1] * m[2]])


def _powers(P, t, m, u, v):
    p, V, d, e = P.p, P.V, P.d, P.p["elastic"]
    B = P.eval_heff(m, TERMS, u)
    p_alpha = 0.0
    for s in range(P.nsub):
        a = p["alpha"][s]
        c = np.cross(m[s], B[s], axis=0)
        p_alpha += p["Ms"][s] * p["gamma"] * a / (1.0 + a * a) * np.sum(c * c)
    ev = el.strain(v, d)
    sig = el.stress(el.strain(u, d), e["C11"], e["C12"], e["C44"])
    p_b = np.sum(np.tensordot(W6, sig * ev, axes=(0, 0)))
    p_b += np.sum(v * el.elastic_force(u, d, P.n, t, e, v))
    for s in range(P.nsub):
        B1, B2 = p["B1"][s], p["B2"][s]
        p_b += np.sum(np.tensordot(W6, _mel_stress(m[s], B1, B2) * ev, axes=(0, 0)))
        p_b += np.sum(v * el.magnetoelastic_force(m[s], B1, B2, d))
    return np.array([V * p_b, V * e["eta"] * np.sum(v * v), V * p_alpha])


def _racetrack():
    # the x = 0 end of the magnetoelastic racetrack (drive face included),
    # with damping raised so that both losses are a visible share of the
    # energy change within a picosecond, and a 50 GHz drive
    p, m0 = inputs.config_c4()
    pc = dict(p)
    pc["n"] = (40, 3, 1)
    pc["alpha"] = [0.05, 0.05]
    pc["elastic"] = dict(p["elastic"], eta=1e15, trac_freq=50e9)
    return pc, np.ascontiguousarray(m0[:, :, :, :3, :40])


def _balance(dt, T=1e-12):
    p, m0 = _racetrack()
    P = Problem(p)

    def rhs(t, y):
        return P.rhs(t, y[:3]) + [_powers(P, t, *y[:3])]

    st = Stepper(rhs, P.normalise, P.err_norm, DORMAND_PRINCE)
    y = P.initial_state(m0) + [np.zeros(3)]
    E0 = sum(P.energies(*y[:3]).values())
    n = int(round(T / dt))
    t = 0.0
    for i in range(n):
        y, knext, _ = st.step(t, y, dt)
        st.accept(knext)
        t = (i + 1) * dt
    dE = sum(P.energies(*y[:3]).values()) - E0
    w_b, w_eta, w_alpha = y[3]
    return dE, w_b, w_eta, w_alpha


def test_energy_balance_closes_at_the_scheme_order():
    res = []
    for dt in (1e-14, 5e-15, 2.5e-15):
        dE, w_b, w_eta, w_alpha = _balance(dt)
        res.append(dE - (w_b - w_eta - w_alpha))
    # every channel carries a material share of the change
    assert w_b > 0 and w_eta > 0.01 * abs(dE) and w_alpha > 0.1 * abs(dE)
    # fifth-order pair: the residual shrinks ~32x per halving (>= 20 asked)
    assert abs(res[0]) / abs(res[1]) > 20
    assert abs(res[1]) / abs(res[2]) > 20
    scale = abs(w_b) + abs(w_eta) + abs(w_alpha)
    assert abs(res[2]) < 1e-6 * scale


# ------------------------------------------------ boundary power (static) --

L = 80e-9
ELAS = dict(rho=6800.0, C11=3.2e11, C12=1.3e11, C44=1.1e11, eta=0.0, trac_amp=2.2e8,
            trac_freq=2e9)
B1 = B2 = -6.3e6
T_EVAL = 0.1e-9


def _bar_powers(nx, mel_force=el.magnetoelastic_force):
    """Discrete and continuum boundary powers on a smooth bar state whose
    strain meets the boundary conditions (shear traction at x = 0, free
    elsewhere).  Nodes at x = 0 .. L."""
    dx = L / (nx - 1)
    d = (dx, 2e-9, 2e-9)
    A = d[1] * d[2]
    V = dx * A
    x = np.arange(nx) * dx
    val = ELAS["trac_amp"] * math.sin(2 * math.pi * ELAS["trac_freq"] * T_EVAL)
    u = np.zeros((3, 1, 1, nx))
    v = np.zeros((3, 1, 1, nx))
    # du_x/dx = du_y/dx = 0 at both ends, C44 du_z/dx = val at 0 and 0 at L
    u[0, 0, 0] = 1e-11 * np.cos(math.pi * x / L)
    u[1, 0, 0] = 2e-11 * np.cos(2 * math.pi * x / L)
    u[2, 0, 0] = val / ELAS["C44"] * (x - x * x / (2 * L)) + 3e-11 * np.cos(3 * math.pi * x / L)
    v[0, 0, 0] = 3.0 * np.sin(0.6 * math.pi * x / L + 0.5)
    v[1, 0, 0] = np.cos(1.2 * math.pi * x / L)
    v[2, 0, 0] = 2.0 * np.cos(math.pi * x / L + 0.4)
    th = 0.6 + 0.5 * np.sin(1.6 * math.pi * x / L)
    ph = 0.3 + 0.4 * np.cos(math.pi * x / L)
    m = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])[:, None, None, :]
    ev = el.strain(v, d)
    sig = el.stress(el.strain(u, d), ELAS["C11"], ELAS["C12"], ELAS["C44"])
    f = el.elastic_force(u, d, (nx, 1, 1), T_EVAL, ELAS)
    pd_el = V * (np.sum(np.tensordot(W6, sig * ev, axes=(0, 0))) + np.sum(v * f))
    # traction vector on the x = 0 face (outward normal -x): t_z = -val
    pc_el = -val * v[2, 0, 0, 0] * A
    smel = _mel_stress(m, B1, B2)
    fm = mel_force(m, B1, B2, d)
    pd_mel = V * (np.sum(np.tensordot(W6, smel * ev, axes=(0, 0))) + np.sum(v * fm))
    pc_mel = 0.0
    for i in range(3):
        s_ix = smel[el.VOIGT[(i, 0)]][0, 0]
        pc_mel += (v[i, 0, 0, -1] * s_ix[-1] - v[i, 0, 0, 0] * s_ix[0]) * A
    return (pd_el - pc_el) / abs(pc_el), (pd_mel - pc_mel) / abs(pc_mel)


def test_boundary_power_tends_to_traction_and_magnetostrictive_work():
    errs = [_bar_powers(40 * s + 1) for s in (1, 2, 4, 8)]
    el_err = [abs(a) for a, _ in errs]
    mel_err = [abs(b) for _, b in errs]
    for seq in (el_err, mel_err):
        for a, b in zip(seq, seq[1:]):
            assert 1.7 < a / b < 2.3        # first order in the cell size
    assert el_err[-1] < 0.06 and mel_err[-1] < 0.005


def _swapped_b2(m, B1_, B2_, d):
    dm = [[el.deriv(m[i], el.AX[j], d[j]) for j in range(3)] for i in range(3)]
    f = np.zeros_like(m)
    for i in range(3):
        f[i] += 2.0 * B1_ * m[i] * dm[i][i]
        for j in range(3):
            if j != i:
                f[i] += B2_ * (m[i] * dm[j][j] + m[j] * dm[j][i])
    return f


def test_misread_force_breaks_the_magnetostrictive_work():
    errs = [abs(_bar_powers(40 * s + 1, _swapped_b2)[1]) for s in (1, 4)]
    assert errs[1] > 0.5 * errs[0] and errs[1] > 0.05
