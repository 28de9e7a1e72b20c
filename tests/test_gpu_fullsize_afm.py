"""Full-size parity of the two-sublattice workloads against the FP64 oracle.

* the polycrystalline antiferromagnet, 1024x256x1 (40 Voronoi grains with
  random easy axes, Zhang-Li current, no demag): every cell's per-term
  fields, the torque with the Zhang-Li term and the energies; three fixed
  FP64 steps;
* the magnetoelastic racetrack, 2048x64x1 (cubic anisotropy, B1 = B2,
  elastodynamics with the shear traction at x = 0): the same, with a seeded
  displacement and velocity, and four fixed FP64 steps of the coupled
  state.
Fields, torque, energies: FP64 <= 1e-12, FP32 <= 2e-6; steps: max |dm| and
relative u, v <= 1e-12.
"""
import numpy as np
import pytest

from oracle.system import Problem, TERMS
from paper_2411_18194_amd import inputs, mmp

pytestmark = pytest.mark.gpu

TOL = {mmp.FP64: 1e-12, mmp.FP32: 2e-6}


def relerr(a, b):
    s = np.abs(b).max()
    return np.abs(a - b).max() / (s if s > 0 else 1.0)


def fp32_round(a):
    return np.asarray(a, np.float32).astype(np.float64)


def _c4_uv(p):
    nx, ny, nz = p["n"]
    g = inputs.rng(41)
    return 1e-12 * g.standard_normal((3, nz, ny, nx)), 1e-3 * g.standard_normal((3, nz, ny, nx))


_cache = {}


def _case(name):
    if name not in _cache:
        if name == "c3":
            p, m = inputs.config_c3()
            u = v = None
        else:
            p, m = inputs.config_c4()
            u, v = _c4_uv(p)
        _cache[name] = (p, m, u, v, Problem(p))
    return _cache[name]


@pytest.mark.parametrize("prec", [mmp.FP64, mmp.FP32])
@pytest.mark.parametrize("name", ["c3", "c4"])
def test_fields_fullsize(name, prec):
    p, m, u, v, P = _case(name)
    if prec == mmp.FP32:
        m = fp32_round(m)
        if u is not None:
            u, v = fp32_round(u), fp32_round(v)
    g = mmp.Grid(p, prec)
    g.set_state(m, u, v)
    worst = {}
    for term in TERMS:
        b, _ = g.eval_heff(mmp.TERM_BITS[term])
        ref = P.eval_heff(m, (term,), u=u)
        if np.abs(ref).max() == 0:
            assert np.abs(b).max() == 0, term
            continue
        worst[term] = relerr(b, ref)
    t, e = g.eval_heff(mmp.T_ALL | mmp.T_ZL | mmp.OUT_TORQUE)
    worst["torque"] = relerr(t, P.torque(m, u=u))
    g.close()
    bad = {k: x for k, x in worst.items() if not x <= TOL[prec]}
    assert not bad, (name, prec, worst)
    Eref = P.energies(m, u, v)
    scale = sum(abs(x) for x in Eref.values())
    for k in mmp.ENERGY_NAMES:
        assert abs(e[k] - Eref[k]) <= TOL[prec] * scale, (k, e[k], Eref[k])


@pytest.mark.parametrize("name", ["c3", "c4"])
def test_fixed_steps_fullsize_fp64(name):
    p, m, u, v, P = _case(name)
    g = mmp.Grid(p, mmp.FP64)
    if u is None:
        dt, nsteps = 1e-15, 3
        g.set_state(m)
        y0 = P.initial_state(m)
    else:
        dt, nsteps = inputs.C4_FIXED_DT, 4
        g.set_state(m, u, v)
        y0 = [m, u, v]
    g.run_fixed(dt, nsteps)
    mg, ug, vg, _, _ = g.get_state()
    g.close()
    y, _ = P.run_fixed(y0, 0.0, dt, nsteps)
    assert np.abs(mg - y[0]).max() < 1e-12
    if u is not None:
        assert relerr(ug, y[1]) < 1e-12
        assert relerr(vg, y[2]) < 1e-12
