"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The library's sources are compiled as for the product (gfx950 device code
included, unchanged) with the host pass instrumented
(-Xarch_host -fsanitize=address,undefined), linked with
tests/sanitize/abi_driver.cpp, and run with no GPU present (nothing is
launched): argument validation of every entry point and a server's whole life
(worker and builder threads, admission, requests failing their set-up for
want of a device, results handed out once, shutdown with requests queued).
A sanitizer finding aborts the driver; the test wants exit status 0.  Leak
checking is off (the HIP runtime's own allocations at exit).
"""
import os
import shutil
import subprocess
import concurrent.futures as cf

import pytest

pytestmark = pytest.mark.slow

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2411_18194_amd", "csrc")
SOURCES = ["abi.hip", "grid.hip", "field.hip", "demag.hip", "demag4.hip", "tensor.hip",
           "elastic.hip", "server.hip", "stray.hip"]


def _hipcc():
    for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    pytest.skip("hipcc not available")


def test_host_code_under_asan_ubsan(tmp_path):
    hipcc = _hipcc()
    flags = ["--offload-arch=gfx950", "-O3", "-Xarch_host", "-g", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fno-omit-frame-pointer",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Wno-unused-command-line-argument",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC]

    def compile_one(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        r = subprocess.run([hipcc, *flags, "-c", os.path.join(CSRC, src), "-o", obj],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    drv = str(tmp_path / "abi_driver.o")
    r = subprocess.run(["g++", "-O1", "-g", "-fsanitize=address,undefined",
                        "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-c",
                        os.path.join(ROOT, "tests", "sanitize", "abi_driver.cpp"), "-o", drv],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    exe = str(tmp_path / "abi_driver")
    # the link pulls in the host sanitizer runtimes; no device code is
    # instrumented (-fno-gpu-sanitize)
    link = ["-fsanitize=address,undefined", "-fno-gpu-sanitize"]
    r = subprocess.run([hipcc, "--offload-arch=gfx950", *link, "-o", exe, drv, *objs, "-lpthread"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "0 failures" in r.stdout
