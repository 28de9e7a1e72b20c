"""Adaptive runs, served requests and serving-size demag pads against the
FP64 oracle.

References come from tests/golden/make_adaptive.py (FP64 oracle only):

* the 64x16x1 film's protocol (200 ps of alpha = 1 relaxation without field,
  then 1 ns with the field and <m> every 5 ps, Dormand-Prince, tol 1e-5):
  in FP64 the device takes exactly the oracle's accepted and rejected steps
  in both phases and every sample agrees to 1e-9; in FP32 (with the FP64
  error norm and time) every sample and the final state agree to 1e-4;
* the 128x64 two-sublattice crop (grains, Zhang-Li current) run adaptively
  for 0.1 ns: FP64 with the oracle's step sequence and samples to 1e-9, FP32
  with every cell within 1e-4 (Euclidean per cell and sublattice);
* a seeded subsample of the request stream (four ferromagnets with demag,
  two two-sublattice magnets, relaxed for 20 ps each) served by the
  library's server with continuous batching: in FP64 each result has the
  oracle's step counts and <m> to 1e-9 and energy to 1e-9 of sum |E_term|;
  in FP32 <m> within 1e-4 and energy within 1e-4 of sum |E_term|.

The serving-size pads: the server's ferromagnets take the smallest 7-smooth
pads, whose transforms run through the LDS Stockham kernels (radix 3, 5, 7
stages); fields of such grids match the oracle to the field bars (FP64
1e-12, FP32 2e-6 of max |B|, per term and total).
"""
import json
import os

import numpy as np
import pytest

from oracle.system import Problem, TERMS
from paper_2411_18194_amd import inputs, mmp

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _meta(name):
    path = os.path.join(GOLD, "adaptive.json")
    if not os.path.exists(path):
        pytest.skip("tests/golden/adaptive.json not generated")
    meta = json.load(open(path))
    if name not in meta:
        pytest.skip(f"{name} not in tests/golden/adaptive.json")
    return meta[name]


def _c1_phases(prec):
    meta = _meta("c1protocol")
    gold = np.load(os.path.join(GOLD, "adaptive_c1protocol.npz"))
    p, m0 = inputs.config_c1()
    relax = dict(p, alpha=[1.0], B_ext=(0.0, 0.0, 0.0))
    g = mmp.Grid(relax, prec, tol=1e-5, dt0=1e-14)
    g.set_state(m0)
    ir, _, _ = g.run(meta["relax"]["t_end"])
    m_rel = g.get_state()[0]
    g.close()
    g = mmp.Grid(p, prec, tol=1e-5, dt0=1e-14)
    g.set_state(m_rel, t=0.0)
    n = meta["run"]["nsamples"]
    info, ts, ms = g.run(meta["run"]["t_end"], sample_every=meta["run"]["sample_every"],
                         max_samples=n)
    m_end = g.get_state()[0]
    g.close()
    return meta, gold, ir, m_rel, info, ts, ms, m_end


def test_c1_protocol_fp64():
    meta, gold, ir, m_rel, info, ts, ms, m_end = _c1_phases(mmp.FP64)
    assert (ir.steps, ir.rejects) == (meta["relax"]["steps"], meta["relax"]["rejects"])
    assert np.abs(m_rel - gold["m_relaxed"]).max() < 1e-9
    assert (info.steps, info.rejects) == (meta["run"]["steps"], meta["run"]["rejects"])
    # the oracle also samples t = 0
    assert len(ts) == meta["run"]["nsamples"] - 1
    assert np.array_equal(ts, gold["t"][1:])
    assert np.abs(ms - gold["m_avg"][1:]).max() < 1e-9
    assert np.abs(m_end - gold["m_end"]).max() < 1e-9


def test_c1_protocol_fp32():
    meta, gold, ir, m_rel, info, ts, ms, m_end = _c1_phases(mmp.FP32)
    assert np.linalg.norm(m_rel - gold["m_relaxed"], axis=1).max() < 1e-4
    assert len(ts) == meta["run"]["nsamples"] - 1
    assert np.allclose(ts, gold["t"][1:], rtol=1e-12, atol=0)
    assert np.abs(ms - gold["m_avg"][1:]).max() < 1e-4
    assert np.linalg.norm(m_end - gold["m_end"], axis=1).max() < 1e-4


@pytest.mark.parametrize("prec", [mmp.FP64, mmp.FP32])
def test_c3crop_adaptive(prec):
    meta = _meta("c3crop_adaptive")
    gold = np.load(os.path.join(GOLD, "adaptive_c3crop.npz"))
    p, m0 = inputs.config_c3_crop()
    g = mmp.Grid(p, prec, tol=1e-5, dt0=1e-14)
    g.set_state(m0)
    nsamp = len(gold["t"]) - 1
    info, ts, ms = g.run(meta["t_end"], sample_every=meta["sample_every"], max_samples=nsamp)
    m_end = g.get_state()[0]
    g.close()
    assert len(ts) == nsamp
    dm = np.linalg.norm(m_end - gold["m_end"].astype(np.float64), axis=1).max()
    davg = np.abs(ms - gold["m_avg"][1:]).max()
    if prec == mmp.FP64:
        assert (info.steps, info.rejects) == (meta["steps"], meta["rejects"])
        assert davg < 1e-9
        assert dm < 1e-6          # the stored state is rounded to float32
    else:
        assert dm < 1e-4, (dm, davg, info.steps, meta["steps"])
        assert davg < 1e-4


def _served_requests():
    meta = _meta("served")
    reqs = inputs.request_stream(seed=5, count=300)
    out = []
    for ref in meta["requests"]:
        r = reqs[ref["index"]]
        assert list(r["params"]["n"]) == ref["n"]
        out.append((r, inputs.request_state(r), ref))
    return meta, out


@pytest.mark.parametrize("prec", [mmp.FP64, mmp.FP32])
def test_served_results_against_oracle(prec):
    meta, items = _served_requests()
    srv = mmp.Server(hbm_budget=8 << 30, max_active=8, precision=prec, batch=True)
    tickets = [srv.submit(r["params"], m, meta["t_relax"], tol=r["tol"]) for r, m, _ in items]
    res = [srv.wait(t, timeout=300.0) for t in tickets]
    srv.close()
    for (r, _, ref), x in zip(items, res):
        assert x.status == 0
        ns = ref["nsub"]
        avg = np.array(x.m_avg)[:ns]
        dav = np.abs(avg - np.array(ref["m_avg"])).max()
        de = abs(x.energy - ref["energy"]) / ref["energy_abs_sum"]
        if prec == mmp.FP64:
            assert (x.steps, x.rejects) == (ref["steps"], ref["rejects"]), ref["index"]
            assert dav < 1e-9 and de < 1e-9, (ref["index"], dav, de)
        else:
            assert dav < 1e-4 and de < 1e-4, (ref["index"], dav, de)


def _serving_pad_case(n, seed):
    d = 2.5e-9
    p = inputs.base_params(n, (d, d, d))
    p.update(Ms=[1.1e6 * 0.9], A11=[1.5e-11 * 1.1], Ku1=[5e5 * 0.8], Dint=[3e-3 * 1.2],
             dmi_layer=0, alpha=[0.1], B_ext=(0.0, 0.0, 0.05), demag=True)
    return p, inputs.smoothed_random_unit(inputs.rng(seed), 1, n)


@pytest.mark.parametrize("prec", [mmp.FP64, mmp.FP32])
@pytest.mark.parametrize("n,pads", [((301, 134, 2), (630, 270, 4)),
                                    ((386, 332, 3), (784, 672, 6))])
def test_serving_size_pads(n, pads, prec):
    p, m = _serving_pad_case(n, sum(n))
    if prec == mmp.FP32:
        m = np.asarray(m, np.float32).astype(np.float64)
    g = mmp.Grid(p, prec)
    pl = g.plan()
    assert tuple(pl["pad"]) == pads
    assert pl["kinds"] & 3 == 0          # x and y through the LDS Stockham kernels
    g.set_state(m)
    P = Problem(p)
    tol = 1e-12 if prec == mmp.FP64 else 2e-6
    Bd = P.demag_field(m)
    for term in ("demag", "exch", "dmi"):
        b, _ = g.eval_heff(mmp.TERM_BITS[term])
        ref = P.eval_heff(m, (term,)) if term != "demag" else Bd[None]
        err = np.abs(b - ref).max() / np.abs(ref).max()
        assert err <= tol, (term, err)
    b, _ = g.eval_heff(mmp.T_ALL)
    ref = P.eval_heff(m, TERMS)
    assert np.abs(b - ref).max() / np.abs(ref).max() <= tol
    g.close()
