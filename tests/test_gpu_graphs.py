"""HIP-graph replay of the step loops against direct launches.

Every kernel of an attempt reads the step controller and the stage buffer
table from device memory, so replaying one captured graph must reproduce
the directly launched sequence bit for bit.  Each check replays the graphs
several times with direct work (an effective-field evaluation, host reads)
in between and compares every replay with the direct result.
"""
import numpy as np
import pytest

from paper_2411_18194_amd import inputs, mmp

pytestmark = pytest.mark.gpu


def _pair(p, m, prec, u=None, v=None):
    out = []
    for on in (True, False):
        g = mmp.Grid(p, prec)
        g.set_graphs(on)
        g.set_state(m, u, v)
        out.append(g)
    return out


def _same(a, b):
    sa, sb = a.get_state(), b.get_state()
    for x, y in zip(sa[:3], sb[:3]):
        assert np.array_equal(x, y)
    assert sa[3] == sb[3] and sa[4] == sb[4]


@pytest.mark.parametrize("prec", [mmp.FP32, mmp.FP64])
@pytest.mark.parametrize("name", ["c2crop", "c3crop", "c4crop"])
def test_fixed_steps_graph_replay(name, prec):
    build = {"c2crop": inputs.config_c2_crop, "c3crop": inputs.config_c3_crop,
             "c4crop": inputs.config_c4_crop}[name]
    p, m = build()
    dt = {"c2crop": inputs.c2_fixed_dt(), "c3crop": 2e-15, "c4crop": inputs.C4_FIXED_DT}[name]
    a, b = _pair(p, m, prec)
    for r, n in enumerate((8, 3, 17, 24)):
        a.run_fixed(dt, n, sync=False)
        b.run_fixed(dt, n, sync=False)
        # direct work on the graph grid's stream between replays
        a.eval_heff(mmp.T_ALL)
        _same(a, b)
    a.close()
    b.close()


@pytest.mark.parametrize("prec", [mmp.FP32, mmp.FP64])
def test_adaptive_run_graph_replay(prec):
    p, m = inputs.config_c1()
    a, b = _pair(p, m, prec)
    for t_end in (0.05e-9, 0.12e-9, 0.2e-9):
        ia, ta, ma = a.run(t_end, sample_every=0.01e-9, max_samples=64)
        ib, tb, mb = b.run(t_end, sample_every=0.01e-9, max_samples=64)
        assert (ia.steps, ia.rejects) == (ib.steps, ib.rejects)
        assert np.array_equal(ta, tb) and np.array_equal(ma, mb)
        _same(a, b)
        a.eval_heff(mmp.T_ALL)
    a.close()
    b.close()


def test_server_matches_direct_run():
    """Requests served concurrently (batched, graph replay) give the result of
    the same relaxation run alone on a grid: bitwise for the two-sublattice
    requests (the batch runs the grid's own kernels); for the ferromagnets
    with demag the batched passes are separately compiled instances of the
    same LDS transforms, so FP32 results agree to the trajectory bar (1e-4)."""
    reqs = [r for r in inputs.request_stream(seed=5, count=40) if
            r["params"]["n"][0] * r["params"]["n"][1] * r["params"]["n"][2] <= 40000][:4]
    assert len(reqs) >= 2
    for r in reqs:
        r["t_relax"] = 0.02e-9
    srv = mmp.Server(hbm_budget=8 << 30, max_active=4, precision=mmp.FP32)
    tickets = [srv.submit(r["params"], inputs.request_state(r), r["t_relax"]) for r in reqs]
    res = [srv.wait(t) for t in tickets]
    srv.close()
    for r, out in zip(reqs, res):
        assert out.status == 0
        ns = r["params"]["nsub"]
        g = mmp.Grid(r["params"], mmp.FP32, tol=r["tol"])
        if r["params"]["demag"]:
            # the server's batched demag runs every pass through the LDS kernels
            g.set_plan(lds_axes=7)
        g.set_state(inputs.request_state(r))
        info, _, _ = g.run(r["t_relax"])
        m = g.get_state()[0].reshape(ns, 3, -1).mean(axis=2)
        g.close()
        got = np.array([[out.m_avg[s][c] for c in range(3)] for s in range(ns)])
        if r["params"]["demag"]:
            assert np.abs(got - m).max() <= 1e-4
        else:
            assert out.steps == info.steps and out.rejects == info.rejects
            assert np.allclose(got, m, rtol=0, atol=1e-12)


def _small_afm(n, seed):
    p = inputs.base_params(n, (1.5e-9,) * 3, nsub=2)
    p.update(Ms=[4e5, 4e5], A11=[1e-11, 1e-11], alpha=[0.05, 0.05], A0=-2.5e-11,
             A12=-5e-12, latcon=0.35e-9, Ku1=[6e4, 6e4], demag=False)
    m = inputs.smoothed_random_unit(inputs.rng(seed), 1, n, sigma=1.5)
    return p, np.concatenate([m, -m])


@pytest.mark.parametrize("batch", [True, False])
def test_batched_afm_requests_match_alone(batch):
    """Requests without demag of different sizes step together in one batch
    (one launch per stage for all of them), join at different times and
    leave when done; each result equals the same relaxation run alone."""
    cases = [_small_afm(n, 40 + i) for i, n in
             enumerate(((48, 20, 1), (17, 33, 3), (64, 64, 1), (5, 7, 2), (40, 24, 2)))]
    t_relax = [4e-12, 7e-12, 3e-12, 9e-12, 5e-12]
    srv = mmp.Server(hbm_budget=8 << 30, max_active=3, precision=mmp.FP32, batch=batch)
    tickets = [srv.submit(p, m, t) for (p, m), t in zip(cases, t_relax)]
    res = [srv.wait(t) for t in tickets]
    srv.close()
    for (p, m), t, out in zip(cases, t_relax, res):
        assert out.status == 0
        g = mmp.Grid(p, mmp.FP32)
        g.set_state(m)
        info, _, _ = g.run(t)
        ref = g.get_state()[0].reshape(2, 3, -1).mean(axis=2)
        _, e = g.eval_heff(mmp.T_ALL, want_b=False)
        g.close()
        assert (out.steps, out.rejects) == (info.steps, info.rejects)
        got = np.array([[out.m_avg[s][c] for c in range(3)] for s in range(2)])
        assert np.allclose(got, ref, rtol=0, atol=1e-12)
        etot = sum(e.values())
        assert abs(out.energy - etot) <= 1e-9 * abs(etot)


def _small_fm(n, seed, d=2e-9):
    p = inputs.base_params(n, (d, d, d))
    p.update(Ms=[1.0e6], A11=[1.4e-11], Ku1=[4e5], Dint=[2.5e-3], dmi_layer=0, alpha=[0.1],
             B_ext=(0.0, 0.0, 0.05), demag=True)
    return p, inputs.smoothed_random_unit(inputs.rng(seed), 1, n, sigma=1.5)


def _serve(cases, t_relax, prec, max_active):
    srv = mmp.Server(hbm_budget=8 << 30, max_active=max_active, precision=prec, batch=True)
    tickets = [srv.submit(p, m, t) for (p, m), t in zip(cases, t_relax)]
    res = [srv.wait(t) for t in tickets]
    srv.close()
    return res


@pytest.mark.parametrize("prec", [mmp.FP32, mmp.FP64])
def test_batched_demag_requests_match_alone(prec):
    """Ferromagnets with demag of different sizes and pads (2-D and 3-D,
    power-of-two and 7-smooth) step together: each demag pass of a stage is
    one launch for all of them.  Each result is bitwise the one the same
    request gets served alone (a batch of one), and agrees with the same
    relaxation run alone on a grid with the LDS kernels: FP64 with identical
    steps and rejects and <m> to 1e-12, energy to 1e-12 of its size; FP32
    within the trajectory bar (1e-4; the batched transforms are a separate
    compilation of the same arithmetic, so FP32 roundings may differ)."""
    cases = [_small_fm(n, 60 + i) for i, n in
             enumerate(((48, 20, 1), (17, 33, 3), (64, 64, 1), (5, 7, 2), (40, 24, 4),
                        (30, 45, 1)))]
    t_relax = [4e-12, 7e-12, 3e-12, 9e-12, 5e-12, 6e-12]
    mixed = _serve(cases, t_relax, prec, 4)
    for (p, m), t, out in zip(cases, t_relax, mixed):
        assert out.status == 0
        alone = _serve([(p, m)], [t], prec, 4)[0]
        assert (out.steps, out.rejects) == (alone.steps, alone.rejects), p["n"]
        assert np.array_equal(np.array(out.m_avg), np.array(alone.m_avg)), p["n"]
        assert out.energy == alone.energy
        g = mmp.Grid(p, prec)
        g.set_plan(lds_axes=7)
        g.set_state(m)
        info, _, _ = g.run(t)
        ref = g.get_state()[0].reshape(1, 3, -1).mean(axis=2)
        _, e = g.eval_heff(mmp.T_ALL, want_b=False)
        g.close()
        got = np.array([[out.m_avg[0][c] for c in range(3)]])
        etot = sum(e.values())
        scale = sum(abs(v) for v in e.values())
        if prec == mmp.FP64:
            assert (out.steps, out.rejects) == (info.steps, info.rejects), p["n"]
            assert np.abs(got - ref).max() <= 1e-12, p["n"]
            assert abs(out.energy - etot) <= 1e-12 * scale
        else:
            assert np.abs(got - ref).max() <= 1e-4, p["n"]
            assert abs(out.energy - etot) <= 1e-4 * scale


@pytest.mark.parametrize("prec", [mmp.FP32, mmp.FP64])
def test_lds_kernels_on_power_of_two_pads(prec):
    """The LDS kernels forced onto power-of-two pads compute the same field
    as the register kernels (field bars), and the plan reports them."""
    p, m = _small_fm((64, 32, 8), 70)
    a = mmp.Grid(p, prec)
    assert a.plan()["kinds"] == 7
    b = mmp.Grid(p, prec)
    pl = b.set_plan(lds_axes=7)
    assert pl["kinds"] == 0 and pl["lds_axes"] == 7
    for g in (a, b):
        g.set_state(m)
    ba, _ = a.eval_heff(mmp.T_DEMAG)
    bb, _ = b.eval_heff(mmp.T_DEMAG)
    tol = 1e-12 if prec == mmp.FP64 else 2e-6
    assert np.abs(ba - bb).max() <= tol * np.abs(ba).max()
    a.close()
    b.close()
