"""Host-side checks of the C ABI (no GPU needed, no compute calls).

* libmmp.so loads and exports every function include/mmp.h declares;
* the ctypes structures have the size and field offsets the C compiler
  gives the header's structs;
* argument validation errors come back as codes with a message.
"""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2411_18194_amd import mmp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mmp.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mmp_[a-z_]+)\s*\(", src)))


def test_library_exports_header():
    lib = mmp.load()
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing
    assert set(names) == set(mmp.EXPORTS)


def test_struct_layout_matches_header(tmp_path):
    prog = tmp_path / "sz.c"
    prog.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "mmp.h"\n'
        'int main(){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n",'
        "sizeof(mmp_params), sizeof(mmp_request), sizeof(mmp_result),"
        "sizeof(mmp_run_opts), sizeof(mmp_run_info), sizeof(mmp_step_info),"
        "sizeof(mmp_server_opts), offsetof(mmp_params, grain),"
        "offsetof(mmp_params, rho), offsetof(mmp_request, m0), sizeof(mmp_plan),"
        "offsetof(mmp_plan, z_lanes), offsetof(mmp_plan, field_ms),"
        "offsetof(mmp_params, solver), offsetof(mmp_params, grain_exch_reduction));"
        "return 0;}\n")
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)],
                   check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = [C.sizeof(mmp.Params), C.sizeof(mmp.Request), C.sizeof(mmp.Result),
            C.sizeof(mmp.RunOpts), C.sizeof(mmp.RunInfo), C.sizeof(mmp.StepInfo),
            C.sizeof(mmp.ServerOpts), mmp.Params.grain.offset, mmp.Params.rho.offset,
            mmp.Request.m0.offset, C.sizeof(mmp.Plan), mmp.Plan.z_lanes.offset,
            mmp.Plan.field_ms.offset, mmp.Params.solver.offset,
            mmp.Params.grain_exch_reduction.offset]
    assert got == want


def test_argument_errors_without_device():
    lib = mmp.load()
    h = C.c_void_p()
    cs = np.array([1e-9, 1e-9, 1e-9])
    rc = lib.mmp_grid_create(0, 4, 4, cs.ctypes.data_as(C.POINTER(C.c_double)), C.byref(h))
    assert rc == -1 and b"sizes" in lib.mmp_last_error()
    bad = np.array([1e-9, -1.0, 1e-9])
    rc = lib.mmp_grid_create(4, 4, 4, bad.ctypes.data_as(C.POINTER(C.c_double)), C.byref(h))
    assert rc == -1
    assert lib.mmp_set_params(None, None) == -1
    assert lib.mmp_eval_heff(None, 0, None, None) == -1
    res = mmp.Result()
    assert lib.mmp_poll(None, 1, C.byref(res)) == -1
    assert lib.mmp_grid_destroy(None) == 0
    pl = mmp.Plan(struct_size=C.sizeof(mmp.Plan))
    assert lib.mmp_get_plan(None, C.byref(pl)) == -1
    assert lib.mmp_set_plan(None, C.byref(pl)) == -1
    assert lib.mmp_autotune(None, None) == -1
