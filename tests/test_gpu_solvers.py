"""GPU parity of every embedded Runge-Kutta pair of the solver table.

The device runs each pair as a fixed sequence of stage kernels (the last
one evaluates the slope at y_{n+1}, which is the next step's k_1), with the
step controller on the device; the oracle steps the same pair the plain
way.  Bars as for the Dormand-Prince checks: fixed steps max |dm| <= 1e-12
in FP64 and <= 2e-6 in FP32 (state rounded to FP32 on both sides); adaptive
runs take the same accepted and rejected steps as the oracle, samples of
<m> within 1e-11 and the final state within 1e-10 (FP64).
"""
import numpy as np
import pytest

from oracle.system import Problem
from paper_2411_18194_amd import inputs, mmp

pytestmark = pytest.mark.gpu

SOLVERS = ["heun", "bs23", "cashkarp", "rkf45", "dp45"]


def _with(p, solver):
    q = dict(p)
    q["solver"] = solver
    return q


def _afm_demag():
    p = inputs.base_params((12, 10, 3), (1.5e-9, 1.5e-9, 1.5e-9), nsub=2)
    p.update(Ms=[4e5, 3e5], A11=[1e-11, 8e-12], alpha=[0.01, 0.02], A0=-2.5e-11,
             A12=-5e-12, latcon=0.35e-9, Ku1=[6e4, 5e4], demag=True,
             B_ext=(0.0, 0.0, 0.1), zl_P=[0.5, 0.4], zl_xi=[0.1, 0.2], j=(3e11, -1e11, 5e10))
    return p, inputs.random_unit(inputs.rng(13), 2, p["n"])


@pytest.mark.parametrize("solver", SOLVERS)
@pytest.mark.parametrize("name", ["c2crop", "afm_demag"])
def test_fixed_steps_fp64(solver, name):
    p, m = {"c2crop": inputs.config_c2_crop, "afm_demag": _afm_demag}[name]()
    p = _with(p, solver)
    dt = 1e-15 if p["nsub"] == 2 else 5e-14
    g = mmp.Grid(p, mmp.FP64)
    g.set_state(m)
    g.run_fixed(dt, 3)
    mg, _, _, t, _ = g.get_state()
    g.close()
    P = Problem(p)
    y, t_ref = P.run_fixed(P.initial_state(m), 0.0, dt, 3)
    assert abs(t - t_ref) < 1e-25
    assert np.abs(mg - y[0]).max() < 1e-12, solver


@pytest.mark.parametrize("solver", SOLVERS)
def test_fixed_steps_fp32(solver):
    p, m = inputs.config_c2_crop()
    p = _with(p, solver)
    m = np.asarray(m, np.float32).astype(np.float64)
    dt = inputs.c2_fixed_dt()
    g = mmp.Grid(p, mmp.FP32)
    g.set_state(m)
    g.run_fixed(dt, 3)
    mg = g.get_state()[0]
    g.close()
    P = Problem(p)
    y, _ = P.run_fixed(P.initial_state(m), 0.0, dt, 3)
    assert np.abs(mg - y[0]).max() < 2e-6, solver


@pytest.mark.parametrize("solver", SOLVERS)
def test_fixed_steps_elastic_fp64(solver):
    p, m = inputs.config_c4_crop()
    p = _with(p, solver)
    nx, ny, nz = p["n"]
    r = inputs.rng(14)
    u = 1e-12 * r.standard_normal((3, nz, ny, nx))
    v = 1e-3 * r.standard_normal((3, nz, ny, nx))
    g = mmp.Grid(p, mmp.FP64)
    g.set_state(m, u, v)
    g.run_fixed(1e-14, 3)
    mg, ug, vg, _, _ = g.get_state()
    g.close()
    P = Problem(p)
    y, _ = P.run_fixed([m, u, v], 0.0, 1e-14, 3)
    assert np.abs(mg - y[0]).max() < 1e-12
    assert np.abs(ug - y[1]).max() <= 1e-12 * np.abs(y[1]).max()
    assert np.abs(vg - y[2]).max() <= 1e-12 * np.abs(y[2]).max()


@pytest.mark.parametrize("solver", SOLVERS)
def test_adaptive_run_c1(solver):
    """Device-side control with the pair's own exponent 1/(q+1)."""
    p, m0 = inputs.config_c1()
    p = _with(p, solver)
    g = mmp.Grid(p, mmp.FP64, tol=1e-5, dt0=1e-14)
    g.set_state(m0)
    info, ts, ms = g.run(10e-12, sample_every=2.5e-12, max_samples=8)
    mg = g.get_state()[0]
    g.close()
    P = Problem(p)
    y, t, oinfo, samples = P.run([m0.copy()], 0.0, 10e-12, tol=1e-5, dt0=1e-14,
                                 sample_every=2.5e-12,
                                 sample=lambda y: y[0].mean(axis=(2, 3, 4)))
    assert (info.steps, info.rejects) == (oinfo["steps"], oinfo["rejects"]), solver
    assert len(ts) == len(samples) - 1
    for (tr, mr), tg, mgv in zip(samples[1:], ts, ms):
        assert tg == tr
        assert np.abs(mgv - mr).max() < 1e-11
    assert np.abs(mg - y[0]).max() < 1e-10


@pytest.mark.parametrize("solver", ["heun", "bs23", "rkf45"])
def test_graph_replay_and_solver_switch(solver):
    """Captured attempts of a shorter pair replay like direct launches, and
    switching the pair on a grid equals a fresh grid with that pair."""
    p, m = inputs.config_c2_crop()
    dt = inputs.c2_fixed_dt()
    a = mmp.Grid(p, mmp.FP32)           # starts with Dormand-Prince
    a.set_params(_with(p, solver), mmp.FP32)
    b = mmp.Grid(_with(p, solver), mmp.FP32)
    b.set_graphs(False)
    for g in (a, b):
        g.set_state(m)
    for n in (8, 3, 17):
        a.run_fixed(dt, n, sync=False)
        b.run_fixed(dt, n, sync=False)
        a.eval_heff(mmp.T_ALL)
        sa, sb = a.get_state(), b.get_state()
        assert np.array_equal(sa[0], sb[0]) and sa[3] == sb[3]
    a.close()
    b.close()


def test_server_request_with_another_pair():
    """A request that names another pair runs on its own stream (batches
    step the Dormand-Prince pair) and equals the run alone."""
    p = inputs.base_params((24, 16, 1), (1.5e-9,) * 3, nsub=2)
    p.update(Ms=[4e5, 4e5], A11=[1e-11, 1e-11], alpha=[0.05, 0.05], A0=-2.5e-11,
             A12=-5e-12, latcon=0.35e-9, Ku1=[6e4, 6e4], solver="bs23")
    mm = inputs.smoothed_random_unit(inputs.rng(77), 1, p["n"], sigma=1.5)
    m = np.concatenate([mm, -mm])
    srv = mmp.Server(hbm_budget=8 << 30, max_active=2, precision=mmp.FP32, batch=True)
    out = srv.wait(srv.submit(p, m, 3e-12))
    srv.close()
    assert out.status == 0
    g = mmp.Grid(p, mmp.FP32)
    g.set_state(m)
    info, _, _ = g.run(3e-12)
    ref = g.get_state()[0].reshape(2, 3, -1).mean(axis=2)
    g.close()
    assert (out.steps, out.rejects) == (info.steps, info.rejects)
    got = np.array([[out.m_avg[s][c] for c in range(3)] for s in range(2)])
    assert np.allclose(got, ref, rtol=0, atol=1e-12)


def test_unknown_solver_rejected():
    p, _ = inputs.config_c1()
    g = mmp.Grid(p, mmp.FP32)
    P, keep = mmp.make_params(p, mmp.FP32)
    P.solver = 5
    with pytest.raises(mmp.MMPError) as e:
        mmp._check(g.lib.mmp_set_params(g.h, mmp.C.byref(P)))
    assert e.value.code == -1
    g.close()


@pytest.mark.parametrize("ctl", [dict(safety=0.9, fac_min=0.2, fac_max=5.0),
                                 dict(dt_max=2.5e-13, safety=0.7)])
def test_step_control_parameters(ctl):
    """Device-side control with the caller's safety, clamps and dt_max: the
    oracle's accept/reject sequence and trajectory (FP64)."""
    p, m0 = inputs.config_c1()
    p = dict(p, **ctl)
    g = mmp.Grid(p, mmp.FP64, tol=1e-6, dt0=1e-11)
    g.set_state(m0)
    info, _, _ = g.run(10e-12)
    mg = g.get_state()[0]
    g.close()
    y, _, oinfo, _ = Problem(p).run([m0.copy()], 0.0, 10e-12, tol=1e-6, dt0=1e-11)
    assert oinfo["rejects"] > 0 or "dt_max" in ctl
    assert (info.steps, info.rejects) == (oinfo["steps"], oinfo["rejects"])
    assert np.abs(mg - y[0]).max() < 1e-10


def test_step_control_rejections():
    p, _ = inputs.config_c1()
    for bad in (dict(safety=1.5), dict(fac_min=2.0), dict(fac_max=0.5), dict(dt_max=-1.0)):
        with pytest.raises(mmp.MMPError):
            mmp.Grid(dict(p, **bad), mmp.FP32).close()
