"""GPU parity: the HIP library against the FP64 oracle, element by element.

Norm (stated for every check): max over cells and components of
|B_gpu - B_ref| divided by max |B_ref|, per term and for the sum.  Bars:
FP64 GPU <= 1e-12, FP32 GPU <= 2e-6 (the FP32 run sees the state rounded
to FP32, and so does the oracle).  Energies: |dE| <= tol * sum_t |E_t|.
"""
import math

import numpy as np
import pytest

from oracle import tensor as OT
from oracle.system import Problem, TERMS
from paper_2411_18194_amd import inputs, mmp

pytestmark = pytest.mark.gpu

TOL = {mmp.FP64: 1e-12, mmp.FP32: 2e-6}
ETOL = {mmp.FP64: 1e-12, mmp.FP32: 2e-6}


def relerr(a, b):
    s = np.abs(b).max()
    return np.abs(a - b).max() / (s if s > 0 else 1.0)


def _ragged3d():
    p = inputs.base_params((37, 23, 5), (2e-9, 3e-9, 2.5e-9))
    p.update(Ms=[8e5], A11=[1.3e-11], alpha=[0.1], Ku1=[2e5], Ku2=[5e4],
             anis_u=[(0.6, 0.0, 0.8)], Dint=[2e-3], dmi_layer=1,
             B_ext=(0.01, -0.02, 0.03), demag=True)
    return p, inputs.smoothed_random_unit(inputs.rng(11), 1, p["n"], sigma=2.0)


def _ragged2d():
    p = inputs.base_params((21, 13, 1), (3e-9, 2e-9, 1e-9))
    p.update(Ms=[6e5], A11=[1e-11], alpha=[0.05], Kc1=[3e4], cub_c1=[(0.6, 0.8, 0.0)],
             cub_c2=[(-0.8, 0.6, 0.0)], B_ext=(0.0, 0.02, 0.0), demag=True,
             Dint=[1e-3], dmi_layer=None)
    return p, inputs.random_unit(inputs.rng(12), 1, p["n"])


def _afm_demag():
    p = inputs.base_params((12, 10, 3), (1.5e-9, 1.5e-9, 1.5e-9), nsub=2)
    p.update(Ms=[4e5, 3e5], A11=[1e-11, 8e-12], alpha=[0.01, 0.02], A0=-2.5e-11,
             A12=-5e-12, latcon=0.35e-9, Ku1=[6e4, 5e4], demag=True,
             B_ext=(0.0, 0.0, 0.1), zl_P=[0.5, 0.4], zl_xi=[0.1, 0.2], j=(3e11, -1e11, 5e10))
    return p, inputs.random_unit(inputs.rng(13), 2, p["n"])


def _afm_dmih():
    # homogeneous inter-sublattice DMI with demag and a current
    p, m = _afm_demag()
    p.update(dmi_homo=(1.5e5, -0.8e5, 2.2e5))
    return p, m


def _c4_crop_u():
    p, m = inputs.config_c4_crop()
    nx, ny, nz = p["n"]
    g = inputs.rng(14)
    u = 1e-12 * g.standard_normal((3, nz, ny, nx))
    v = 1e-3 * g.standard_normal((3, nz, ny, nx))
    return p, m, u, v


def _tiny(n):
    p = inputs.base_params(n, (2e-9, 2e-9, 2e-9))
    p.update(Ms=[1e6], A11=[1e-11], alpha=[0.1], demag=True, B_ext=(0.0, 0.0, 0.01))
    return p, inputs.random_unit(inputs.rng(sum(n)), 1, n)


def _pow2_3d():
    p = inputs.base_params((32, 32, 16), (2e-9, 2e-9, 2e-9))
    p.update(Ms=[1.1e6], A11=[1.5e-11], alpha=[0.1], Ku1=[5e5], anis_u=[(0, 0, 1)],
             Dint=[3e-3], dmi_layer=0, B_ext=(0.0, 0.0, 0.05), demag=True)
    return p, inputs.smoothed_random_unit(inputs.rng(21), 1, p["n"])


def _pow2_2d():
    p = inputs.base_params((256, 64, 1), (3e-9, 3e-9, 2e-9))
    p.update(Ms=[8e5], A11=[1.3e-11], alpha=[0.02], B_ext=(-0.02, 0.004, 0.0), demag=True)
    return p, inputs.smoothed_random_unit(inputs.rng(22), 1, p["n"])


def _pow2_afm():
    p = inputs.base_params((16, 8, 4), (1e-9, 1e-9, 1e-9), nsub=2)
    p.update(Ms=[4e5, 3.5e5], A11=[1e-11, 1e-11], alpha=[0.01, 0.01], A0=-2.5e-11,
             A12=-5e-12, latcon=0.35e-9, Ku1=[6e4, 6e4], demag=True)
    return p, inputs.random_unit(inputs.rng(23), 2, p["n"])


CASES = {
    "c1": lambda: inputs.config_c1(),
    "c2crop": lambda: inputs.config_c2_crop(),
    "c3crop": lambda: inputs.config_c3_crop(),
    "ragged3d": _ragged3d,
    "ragged2d": _ragged2d,
    "afm_demag": _afm_demag,
    "afm_dmih": _afm_dmih,
    "tiny111": lambda: _tiny((1, 1, 1)),
    "tiny213": lambda: _tiny((2, 1, 3)),
    "tiny171": lambda: _tiny((1, 7, 1)),
    "tiny2x2": lambda: _tiny((2, 2, 2)),
    "pow2_3d": _pow2_3d,
    "pow2_2d": _pow2_2d,
    "pow2_afm": _pow2_afm,
}

_oracles = {}


def oracle_for(name, p):
    if name not in _oracles:
        _oracles[name] = Problem(p)
    return _oracles[name]


def fp32_round(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


@pytest.mark.parametrize("name", list(CASES))
def test_demag_tensor_parity(name):
    p, m = CASES[name]()
    if not p["demag"]:
        pytest.skip("no demag")
    g = mmp.Grid(p, mmp.FP64)
    n6 = g.demag_tensor()
    ref = OT.demag_tensor(p["n"], p["cell"])
    # near/mid regimes: absolute (N_self ~ 1/3); far: relative to the entry
    assert np.abs(n6 - ref).max() < 2e-14
    g.close()


@pytest.mark.parametrize("prec", [mmp.FP64, mmp.FP32])
@pytest.mark.parametrize("name", list(CASES))
def test_eval_heff_per_term(name, prec):
    p, m = CASES[name]()
    if prec == mmp.FP32:
        m = fp32_round(m)
    P = oracle_for(name, p)
    g = mmp.Grid(p, prec)
    g.set_state(m)
    worst = {}
    for term in TERMS:
        bit = mmp.TERM_BITS[term]
        b, _ = g.eval_heff(bit)
        ref = P.eval_heff(m, (term,))
        if np.abs(ref).max() == 0:
            assert np.abs(b).max() == 0, term
            continue
        worst[term] = relerr(b, ref)
    b, e = g.eval_heff(mmp.T_ALL)
    ref = P.eval_heff(m)
    worst["total"] = relerr(b, ref)
    bad = {k: v for k, v in worst.items() if not v <= TOL[prec]}
    assert not bad, (name, prec, worst)
    # energies of every term
    Eref = P.energies(m)
    scale = sum(abs(v) for v in Eref.values())
    for k in mmp.ENERGY_NAMES:
        assert abs(e[k] - Eref[k]) <= ETOL[prec] * scale, (k, e[k], Eref[k])
    g.close()


@pytest.mark.parametrize("prec", [mmp.FP64, mmp.FP32])
@pytest.mark.parametrize("name", ["c3crop", "afm_demag", "c2crop", "afm_dmih"])
def test_torque_parity(name, prec):
    p, m = CASES[name]()
    if prec == mmp.FP32:
        m = fp32_round(m)
    P = oracle_for(name, p)
    g = mmp.Grid(p, prec)
    g.set_state(m)
    b, _ = g.eval_heff(mmp.T_ALL | mmp.T_ZL | mmp.OUT_TORQUE)
    ref = P.torque(m)
    assert relerr(b, ref) <= TOL[prec]
    g.close()


@pytest.mark.parametrize("prec", [mmp.FP64, mmp.FP32])
def test_magnetoelastic_parity(prec):
    p, m, u, v = _c4_crop_u()
    if prec == mmp.FP32:
        m, u, v = fp32_round(m), fp32_round(u), fp32_round(v)
    P = Problem(p)
    g = mmp.Grid(p, prec)
    g.set_state(m, u, v)
    for term in ("mel", "anis_c", "afm_cell", "exch"):
        b, _ = g.eval_heff(mmp.TERM_BITS[term])
        ref = P.eval_heff(m, (term,), u=u)
        assert relerr(b, ref) <= TOL[prec], term
    _, e = g.eval_heff(mmp.T_ALL)
    Eref = P.energies(m, u, v)
    scale = sum(abs(x) for x in Eref.values())
    for k in mmp.ENERGY_NAMES:
        assert abs(e[k] - Eref[k]) <= ETOL[prec] * scale, (k, e[k], Eref[k])
    g.close()


@pytest.mark.parametrize("name", ["c2crop", "ragged3d", "afm_demag", "c3crop", "afm_dmih"])
def test_fixed_steps_fp64(name):
    p, m = CASES[name]()
    P = Problem(p)
    # stable steps: the 2000 T inter-sublattice field needs dt ~ 1e-15
    dt = 1e-15 if p["nsub"] == 2 else 5e-14
    g = mmp.Grid(p, mmp.FP64)
    g.set_state(m)
    g.run_fixed(dt, 3)
    mg, _, _, t, _ = g.get_state()
    y, t_ref = P.run_fixed(P.initial_state(m), 0.0, dt, 3)
    assert abs(t - t_ref) < 1e-25
    assert np.abs(mg - y[0]).max() < 1e-12
    g.close()


def test_fixed_steps_elastic_fp64():
    p, m, u, v = _c4_crop_u()
    P = Problem(p)
    g = mmp.Grid(p, mmp.FP64)
    g.set_state(m, u, v)
    dt = 1e-14
    g.run_fixed(dt, 4)
    mg, ug, vg, t, _ = g.get_state()
    y, _ = P.run_fixed([m, u, v], 0.0, dt, 4)
    assert np.abs(mg - y[0]).max() < 1e-12
    assert relerr(ug, y[1]) < 1e-12
    assert relerr(vg, y[2]) < 1e-12
    g.close()


def test_adaptive_run_c1_samples():
    """Adaptive DP45 with device-side control reproduces the oracle's run."""
    p, m0 = inputs.config_c1()
    P = Problem(p)
    g = mmp.Grid(p, mmp.FP64, tol=1e-5, dt0=1e-14)
    g.set_state(m0)
    info, ts, ms = g.run(20e-12, sample_every=5e-12, max_samples=8)
    y, t, oinfo, samples = P.run([m0.copy()], 0.0, 20e-12, tol=1e-5, dt0=1e-14,
                                 sample_every=5e-12,
                                 sample=lambda y: y[0].mean(axis=(2, 3, 4)))
    assert info.steps == oinfo["steps"] and info.rejects == oinfo["rejects"]
    assert len(ts) == len(samples) - 1
    for (tr, mr), tg, mgv in zip(samples[1:], ts, ms):
        assert tg == tr
        assert np.abs(mgv - mr).max() < 1e-11
    mg = g.get_state()[0]
    assert np.abs(mg - y[0]).max() < 1e-10
    g.close()
