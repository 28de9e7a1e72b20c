"""Failure handling, step-control limits, state races and checkpoint/resume
of the HIP library (through the C ABI).

Every failure here is forced from the host: a NaN in the uploaded state, a
tolerance no step can meet, a request above the HBM budget, an injected
failure of the server's batch set-up.  No kernel is made to fault; every
kernel exits normally and the library reports the condition as a status.

* a non-finite state stops an adaptive run with MMP_E_NONFINITE;
* a tolerance of 1e-30 drives the step below dt_min: MMP_E_DT_UNDERFLOW;
* step control that could not shrink a rejected step (fac_min >= 1) is
  refused by mmp_set_params; an adaptive mmp_step that is rejected 1000
  times in a row (fac_min just below 1) returns MMP_E_STATE;
* mmp_set_state right after work enqueued without synchronisation keeps
  the new state (the call waits for that work);
* checkpoint/resume: get_state at a sample time, a new grid with the saved
  step size, set_state, and the rest of the run give bitwise the state of
  the uninterrupted run (adaptive FP64 and fixed FP32 steps);
* the server rejects a request above its whole budget (MMP_E_TOO_LARGE),
  admits a second request only after the first has freed the budget, and
  after a failed batch set-up finishes the batch's requests with the error
  and serves later requests normally.
"""
import ctypes as C

import numpy as np
import pytest

from paper_2411_18194_amd import inputs, mmp

pytestmark = pytest.mark.gpu


def _film(n=(24, 16, 2)):
    p = inputs.base_params(n, (2e-9, 2e-9, 2e-9))
    p.update(Ms=[8e5], A11=[1.3e-11], alpha=[0.1], Ku1=[3e5], B_ext=(0.0, 0.0, 0.05),
             demag=True)
    return p, inputs.smoothed_random_unit(inputs.rng(41), 1, n)


def _afm(n=(32, 24, 1), seed=42):
    p = inputs.base_params(n, (1.5e-9,) * 3, nsub=2)
    p.update(Ms=[4e5, 4e5], A11=[1e-11, 1e-11], A0=-2.5e-11, A12=-5e-12, alpha=[0.05, 0.05],
             Ku1=[6e4, 6e4], latcon=0.35e-9)
    m = inputs.smoothed_random_unit(inputs.rng(seed), 1, n)
    return p, np.concatenate([m, -m])


def test_nonfinite_state_is_reported():
    p, m = _film()
    m = m.copy()
    m[0, 1, 1, 3, 5] = np.nan
    g = mmp.Grid(p, mmp.FP32)
    g.set_state(m)
    with pytest.raises(mmp.MMPError) as ei:
        g.run(2e-12)
    assert ei.value.code == -4
    g.close()


def test_unreachable_tolerance_underflows():
    p, m = _film()
    g = mmp.Grid(p, mmp.FP64, tol=1e-30)
    g.set_state(m)
    with pytest.raises(mmp.MMPError) as ei:
        g.run(1e-12)
    assert ei.value.code == -5
    with pytest.raises(mmp.MMPError) as ei:
        g.step()
    assert ei.value.code == -5
    g.close()


def test_step_control_that_cannot_shrink_is_refused():
    p, m = _film()
    for bad in (dict(fac_min=1.0), dict(fac_min=1.5), dict(safety=1.5)):
        with pytest.raises(mmp.MMPError) as ei:
            mmp.Grid(dict(p, **bad), mmp.FP32)
        assert ei.value.code == -1
    # fac_min just below 1 with an unreachable tolerance: 1000 rejected
    # attempts shrink the step only to ~0.37x, far above dt_min
    g = mmp.Grid(dict(p, fac_min=0.999), mmp.FP32, tol=1e-30)
    g.set_state(m)
    with pytest.raises(mmp.MMPError) as ei:
        g.step()
    assert ei.value.code == -7
    g.close()


def test_set_state_waits_for_enqueued_steps():
    p, m = _film((64, 48, 4))
    g = mmp.Grid(p, mmp.FP32)
    g.set_state(m)
    m2 = inputs.random_unit(inputs.rng(43), 1, p["n"])
    m2 = np.asarray(m2, np.float32).astype(np.float64)
    for _ in range(3):
        g.run_fixed(inputs.c2_fixed_dt(), 40, sync=False)   # returns with work queued
        g.set_state(m2, t=1e-9)
        got, _, _, t, _ = g.get_state()
        assert t == 1e-9
        assert np.array_equal(got, m2)
    g.close()


def _sampled_run(g, T, every):
    info, ts, ms = g.run(T, sample_every=every, max_samples=8)
    return info, ts, ms


@pytest.mark.parametrize("prec", [mmp.FP64, mmp.FP32])
def test_checkpoint_resume_adaptive_is_bitwise(prec):
    p, m = _film()
    T = 20e-12
    # uninterrupted, landing on T/2 (a sample time) on the way
    a = mmp.Grid(p, prec)
    a.set_state(m)
    ia, _, _ = _sampled_run(a, T, T / 2)
    ma, _, _, ta, _ = a.get_state()
    # first half, checkpoint (state, time, the controller's next step)
    b = mmp.Grid(p, prec)
    b.set_state(m)
    ib, _, _ = _sampled_run(b, T / 2, T / 2)
    mh, _, _, th, dth = b.get_state()
    b.close()
    assert th == T / 2
    # resume in a new grid: the saved step size as the first step
    c = mmp.Grid(p, prec, dt0=dth)
    c.set_state(mh, t=th)
    ic, _, _ = _sampled_run(c, T, T / 2)
    mc, _, _, tc, _ = c.get_state()
    assert tc == ta
    assert ib.steps + ic.steps == ia.steps and ib.rejects + ic.rejects == ia.rejects
    assert np.array_equal(mc, ma)
    a.close()
    c.close()


def test_checkpoint_resume_fixed_steps_is_bitwise():
    p, m = _film()
    dt = 5e-14
    a = mmp.Grid(p, mmp.FP32)
    a.set_state(m)
    a.run_fixed(dt, 40)
    ma, _, _, ta, _ = a.get_state()
    b = mmp.Grid(p, mmp.FP32)
    b.set_state(m)
    b.run_fixed(dt, 20)
    mh, _, _, th, _ = b.get_state()
    b.close()
    c = mmp.Grid(p, mmp.FP32)
    c.set_state(mh, t=th)
    c.run_fixed(dt, 20)
    mc, _, _, tc, _ = c.get_state()
    assert np.array_equal(mc, ma) and tc == ta
    a.close()
    c.close()


def _req_bytes(p):
    nx, ny, nz = p["n"]
    N = nx * ny * nz
    return (4 + 7) * p["nsub"] * 3 * N * 4 + (1 << 20)


def test_server_budget_admission_and_rejection():
    p, m = _afm()
    one = _req_bytes(p)
    # a budget for one such request at a time (and not two)
    srv = mmp.Server(hbm_budget=int(1.5 * one), max_active=8, precision=mmp.FP32, batch=False)
    big, mb = _afm((200, 200, 1))
    with pytest.raises(mmp.MMPError) as ei:
        srv.submit(big, mb, 1e-12)
    assert ei.value.code == -6
    t1 = srv.submit(p, m, 5e-12)
    t2 = srv.submit(p, m, 5e-12)
    r1, r2 = srv.wait(t1), srv.wait(t2)
    assert r1.status == 0 and r2.status == 0
    assert r2.t_admit >= r1.t_done       # admitted only once the first freed its memory
    # a result is handed out once
    with pytest.raises(mmp.MMPError) as ei:
        srv.poll(t1)
    assert ei.value.code == -8
    srv.close()


def test_server_recovers_from_a_failed_batch():
    lib = mmp.load()
    inject = lib.mmp_test_fail_batch_rebuilds
    inject.argtypes = [C.c_int]
    inject.restype = None
    srv = mmp.Server(hbm_budget=8 << 30, max_active=8, precision=mmp.FP32, batch=True)
    try:
        # one injected failure per batch the three requests can form (they
        # may be placed together or one by one)
        inject(3)
        reqs = [_afm(seed=50 + i) for i in range(3)]
        tk = [srv.submit(p, m, 2e-12) for p, m in reqs]
        res = [srv.wait(t, timeout=120.0) for t in tk]
        assert all(r.status == -2 for r in res)
        inject(0)
        # later requests run on a fresh batch, as they would alone
        tk = [srv.submit(p, m, 2e-12) for p, m in reqs]
        res = [srv.wait(t, timeout=120.0) for t in tk]
        assert all(r.status == 0 for r in res)
        for (p, m), r in zip(reqs, res):
            g = mmp.Grid(p, mmp.FP32)
            g.set_state(m)
            info, _, _ = g.run(2e-12)
            mm = g.get_state()[0]
            g.close()
            assert info.steps == r.steps
            avg = mm.mean(axis=(2, 3, 4))
            assert np.array_equal(avg[:, :], np.array(r.m_avg)[:2, :]) or \
                np.abs(avg - np.array(r.m_avg)[:2, :]).max() < 1e-12
    finally:
        inject(0)
        srv.close()
