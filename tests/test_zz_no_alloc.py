"""The allocation-free stray-field entry point against the allocating one.

mmp_stray_field_noalloc keeps its tensor table in the library's fixed
per-device array and writes into a caller-owned device buffer; its output
must equal mmp_stray_field's (same kernels: FP64 <= 1e-12, FP32 <= 2e-6 of
max |B|, the stray-field parity bar) on two calls in a row, the second on a
smaller grid, so that the second call reuses the array the first one
filled.  Both are also checked against the FP64 oracle, and a grid whose
table does not fit the array is rejected before any work.
"""
import ctypes as C

import numpy as np
import pytest
import torch

from oracle.stray import stray_field
from paper_2411_18194_amd import inputs, mmp

pytestmark = pytest.mark.gpu

TOL = {mmp.FP64: 1e-12, mmp.FP32: 2e-6}


def _case(n, cell, nsub, seed):
    p = inputs.base_params(n, cell, nsub=nsub)
    if nsub == 1:
        p.update(Ms=[8e5], A11=[1.3e-11], alpha=[0.1])
    else:
        p.update(Ms=[4e5, 3e5], A11=[1e-11, 1e-11], alpha=[0.01, 0.01], A0=-2e-11,
                 latcon=0.35e-9)
    return p, inputs.random_unit(inputs.rng(seed), nsub, n)


def _noalloc(g, h):
    nx, ny, _ = g.n
    out = torch.full((3, ny, nx), float("nan"), dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    g.stray_field_noalloc(h, out.data_ptr())
    g.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("prec", [mmp.FP64, mmp.FP32])
def test_noalloc_matches_allocating_call(prec):
    torch.cuda.set_device(0)
    cases = [_case((40, 36, 3), (2e-9, 2.5e-9, 1.5e-9), 1, 301),   # larger first
             _case((17, 9, 2), (1.5e-9, 1.5e-9, 1.5e-9), 2, 302)]  # then smaller
    for (p, m), h in zip(cases, (0.9e-9, 2e-9)):
        if prec == mmp.FP32:
            m = np.asarray(m, np.float32).astype(np.float64)
        g = mmp.Grid(p, prec)
        g.set_state(m)
        b_alloc = g.stray_field(h)
        b_free = _noalloc(g, h)
        scale = np.abs(b_alloc).max()
        assert np.isfinite(b_free).all()
        assert np.abs(b_free - b_alloc).max() <= TOL[prec] * scale, (p["n"], prec)
        M = sum(p["Ms"][s] * m[s] for s in range(p["nsub"]))
        ref = stray_field(M, p["cell"], h)
        assert np.abs(b_free - ref).max() <= TOL[prec] * np.abs(ref).max(), (p["n"], prec)
        g.close()


def test_noalloc_rejects_oversized_and_bad_arguments():
    torch.cuda.set_device(0)
    # 6 * 1 * (2*300-1) * (2*300-1) = 2.15e6 doubles > the fixed 2^21
    p, m = _case((300, 300, 1), (2e-9, 2e-9, 2e-9), 1, 303)
    g = mmp.Grid(p, mmp.FP32)
    g.set_state(m)
    out = torch.zeros((3, 300, 300), dtype=torch.float64, device="cuda:0")
    with pytest.raises(mmp.MMPError) as ei:
        g.stray_field_noalloc(2e-9, out.data_ptr())
    assert ei.value.code == -6
    # a height inside the magnet, and a host buffer, are argument errors
    p, m = _case((8, 8, 1), (2e-9, 2e-9, 2e-9), 1, 304)
    g2 = mmp.Grid(p, mmp.FP32)
    g2.set_state(m)
    out = torch.zeros((3, 8, 8), dtype=torch.float64, device="cuda:0")
    with pytest.raises(mmp.MMPError) as ei:
        g2.stray_field_noalloc(0.4e-9, out.data_ptr())
    assert ei.value.code == -1
    host = np.zeros((3, 8, 8))
    with pytest.raises(mmp.MMPError) as ei:
        g2.stray_field_noalloc(2e-9, host.ctypes.data)
    assert ei.value.code == -1
    g.close()
    g2.close()
