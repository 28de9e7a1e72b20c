"""Benchmark: cell-field-evals/s of the micromagnetic hot path on one MI355X.

Workload: 512x512x16 ferromagnetic film of 2 nm cubes (demag, exchange,
interfacial DMI on the bottom layer, uniaxial anisotropy, Zeeman), fixed
Dormand-Prince 5(4) steps of 0.1 ns/1667.  One step = 6 new effective-field
evaluations (the 7-stage pair is first-same-as-last) over every cell; the
value is cells * 6 * steps / seconds for the FP32 path, with the FP64 path
timed the same way beside it.  The state is resident in HBM before the timed
region; nothing is copied to or from the host inside it.

The timed region runs the steps as a caller does (attempts captured once
and replayed as HIP graphs, no instrumentation).  The same number of steps
is then run again with a HIP event pair around every launch on the grid's
stream (direct launches: the events sit between them); that profiled region
gives each kernel's average duration, and its step time is reported too.

Also reported: the dominant kernel's algorithmic bytes per launch over its
average HIP-event duration in the profiled region (roofline vs 8 TB/s), the
HBM traffic the rocprofv3 counters measured for that kernel (when the
committed counter summary matches the current kernel source), the rate of a
plain device copy moving the same number of bytes (the stream rate reachable
at that working set; frac_of_copy), and the FP64 CPU oracle timed on a
bounded sample of the same workload.

Before the warm-up the demag plan is autotuned (candidate pads and launch
shapes timed on the device, the fastest installed), as a caller would do
once per shape; --no-autotune keeps the default plan.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-fp64]
       [--no-cpu-baseline] [--no-prof] [--no-autotune]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("cell-field-evals/s 512x512x16 FP32 vs FP64; batched solves/s with p50/p99 "
          "latency")
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = tuple("paper_2411_18194_amd/csrc/" + f for f in (
    "demag.hip", "demag4.hip", "fft4.h", "fft_engine.h", "field.hip", "field.h", "common.h"))
COUNTERS = os.path.join(ROOT, "profiles", "counters_c2_fp32.json")


def smooth_pad(n):
    if n == 1:
        return 1
    p = 2 * n - 1
    while True:
        if p % 2 == 0:
            q = p
            for f in (2, 3, 5, 7):
                while q % f == 0:
                    q //= f
            if q == 1:
                return p
        p += 1


def algorithmic_bytes(n, rb, nsub=1, pads=None):
    """Bytes each kernel class must move per launch (operands read once)."""
    nx, ny, nz = n
    N = nx * ny * nz
    cb = 2 * rb
    Px, Py, Pz = pads or (smooth_pad(nx), smooth_pad(ny), smooth_pad(nz))
    Hx, Hy, Hz = Px // 2 + 1, Py // 2 + 1, Pz // 2 + 1
    s1 = cb * 3 * nz * Hx * ny
    out = {"fftx_fwd": rb * nsub * 3 * N + s1, "fftx_inv": s1 + rb * 3 * N}
    if nz > 1:
        s2 = cb * 3 * nz * Hx * Py
        out["ffty_fwd"] = s1 + s2
        out["fftz_mul"] = 2 * s2 + rb * 6 * Hz * Hx * Hy
        out["ffty_inv"] = s2 + s1
    else:
        out["ffty_mul2d"] = 2 * s1 + rb * 4 * Hx * Hy
    # field kernel, fixed-step stages s = 2..7.  s < 7 reads the stage input,
    # B_d, y_n and k_1..k_{s-1} and writes k_s and the next stage input; s = 7
    # reads its input and B_d and writes k_7 and the next step's stage-2 input.
    v = rb * 3 * nsub * N
    bd = rb * 3 * N
    per_stage = [(s + 3) * v + bd for s in range(2, 7)] + [3 * v + bd]
    out["field"] = sum(per_stage) / len(per_stage)
    return out


def src_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def run_gpu(precision, steps, warmup, prof=True, tune=True):
    import torch

    from paper_2411_18194_amd import inputs, mmp

    p, m0 = inputs.config_c2()
    g = mmp.Grid(p, precision)
    stream = torch.cuda.current_stream()
    g.set_stream(stream.cuda_stream)
    g.set_state(m0)
    t_tune = time.perf_counter()
    plan = g.autotune() if tune else g.plan()
    t_tune = time.perf_counter() - t_tune
    dt = inputs.c2_fixed_dt()
    g.run_fixed(dt, warmup)
    torch.cuda.synchronize()
    # timed region: the steps as a caller runs them (captured attempts
    # replayed as HIP graphs, no instrumentation)
    t0 = time.perf_counter()
    g.run_fixed(dt, steps, sync=False)
    g.synchronize()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # profiled region: the same number of steps again with a HIP event pair
    # around every launch on the grid's stream (direct launches, since the
    # events sit between them); per-kernel durations for the roofline
    kern, prof_ms = None, None
    if prof:
        g.prof_reset()
        g.prof_enable(True)
        t2 = time.perf_counter()
        g.run_fixed(dt, steps, sync=False)
        g.synchronize()
        torch.cuda.synchronize()
        prof_ms = 1e3 * (time.perf_counter() - t2) / steps
        g.prof_enable(False)
        kern = g.prof_read()
    m = g.get_state()[0]
    finite = bool(np.isfinite(m).all())
    norm_err = float(np.abs(np.linalg.norm(m, axis=1) - 1).max())
    g.close()
    N = p["n"][0] * p["n"][1] * p["n"][2]
    sec = t1 - t0
    return dict(value=N * 6 * steps / sec, ms_per_step=1e3 * sec / steps, kernels=kern,
                finite=finite, norm_err=norm_err, n=p["n"], plan=plan,
                tune_s=t_tune if tune else None, prof_ms_per_step=prof_ms)


def roofline(res, rb):
    ab = algorithmic_bytes(res["n"], rb, pads=tuple(res["plan"]["pad"]))
    kern = res["kernels"]
    tot = {k: v[0] for k, v in kern.items() if v[1] > 0}
    dom = max((k for k in tot if k in ab), key=lambda k: tot[k])
    ms, cnt = kern[dom]
    avg_s = ms / cnt / 1e3
    ach = ab[dom] / avg_s / 1e9
    traffic = None
    if os.path.exists(COUNTERS):
        with open(COUNTERS) as fh:
            c = json.load(fh)
        if c.get("source_hash") == src_hash() and dom in c.get("kernels", {}):
            traffic = c["kernels"][dom]["bytes_per_launch"]
    share = {k: round(v / sum(tot.values()), 4) for k, v in tot.items()}
    return {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
            "algorithmic_bytes_per_launch": ab[dom], "avg_launch_ms": round(avg_s * 1e3, 4),
            "time_share": share}


def copy_rate(nbytes, reps=10):
    """GB/s of a plain device copy moving nbytes in total (half read, half
    written): the stream rate reachable at the dominant kernel's working set."""
    import torch
    n = max(1, nbytes // 8)
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    del src, dst
    return 2 * n * 4 / sec / 1e9


def cpu_baseline():
    """FP64 oracle on a 256x256x16 block of the same film (1/4 of the cells)."""
    from oracle.system import Problem
    from paper_2411_18194_amd import inputs

    cores = len(os.sched_getaffinity(0))
    n = (256, 256, 16)
    p = inputs.base_params(n, (2e-9,) * 3)
    full, _ = inputs.config_c2(n=(8, 8, 16))
    for k in ("Ms", "A11", "alpha", "Ku1", "anis_u", "Dint", "dmi_layer", "B_ext", "demag"):
        p[k] = full[k]
    m = inputs.smoothed_random_unit(inputs.rng(2), 1, n)
    P = Problem(p, demag_workers=cores)
    dt = inputs.c2_fixed_dt()
    y = P.initial_state(m)
    y, _ = P.run_fixed(y, 0.0, dt, 1)          # warm-up (also fills the FSAL stage)
    t0 = time.perf_counter()
    nsteps = 6   # ~10 s of host work
    y, _ = P.run_fixed(y, 0.0, dt, nsteps)
    sec = time.perf_counter() - t0
    N = n[0] * n[1] * n[2]
    return {"value": N * 6 * nsteps / sec, "unit": "cell-field-evals/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{n[0]}x{n[1]}x{n[2]} block of the 512x512x16 film (same material, "
                      f"own open-boundary demag), {nsteps} fixed DP45 steps = {6 * nsteps} "
                      f"field evaluations, FP64 numpy/scipy (FFT on {cores} threads, "
                      f"element-wise work on 1)", "seconds": round(sec, 2)}


def _percentiles(lat):
    lat = np.sort(np.asarray(lat))
    return (float(np.percentile(lat, 50)), float(np.percentile(lat, 99)))


def _serve_pass(reqs, states, precision, rate_scale, max_active, batch=True):
    """Open-loop replay of the request stream through the server.

    Request i is submitted at t_arrive[i] * rate_scale after the start (a
    scale above 1 slows the arrivals down).  Latency = t_done - t_submit on
    the server's clock."""
    from paper_2411_18194_amd import mmp

    srv = mmp.Server(hbm_budget=64 << 30, max_active=max_active, precision=precision,
                     batch=batch)
    t0 = srv.clock()
    tickets = []
    for r, m in zip(reqs, states):
        while srv.clock() - t0 < r["t_arrive"] * rate_scale:
            time.sleep(2e-4)
        tickets.append(srv.submit(r["params"], m, r["t_relax"], tol=r["tol"]))
    res = [srv.wait(t, timeout=900.0) for t in tickets]
    srv.close()
    bad = [x.status for x in res if x.status != 0]
    if bad:
        raise RuntimeError(f"serving: {len(bad)} requests failed: {bad[:5]}")
    lat = [x.t_done - x.t_submit for x in res]
    span = max(x.t_done for x in res) - min(x.t_submit for x in res)
    p50, p99 = _percentiles(lat)
    cells = sum(r["params"]["n"][0] * r["params"]["n"][1] * r["params"]["n"][2] for r in reqs)
    steps = sum(x.steps + x.rejects for x in res)
    return {"solves_per_s": len(res) / span, "p50_s": p50, "p99_s": p99, "makespan_s": span,
            "requests": len(res), "attempts": int(steps), "cells": int(cells)}


def _sequential_fp64(reqs, states):
    """Each request alone, one after another, FP64, direct launches (no
    graphs, no server); latencies by FIFO replay of the measured service
    times against the stream's arrival times."""
    from paper_2411_18194_amd import mmp

    service = []
    for r, m in zip(reqs, states):
        t0 = time.perf_counter()
        g = mmp.Grid(r["params"], mmp.FP64, tol=r["tol"])
        g.set_graphs(False)
        g.set_state(m)
        g.run(r["t_relax"])
        g.get_state()
        g.eval_heff(0, want_b=False)
        g.close()
        service.append(time.perf_counter() - t0)
    t_free, lat = 0.0, []
    for r, sv in zip(reqs, service):
        start = max(t_free, r["t_arrive"])
        t_free = start + sv
        lat.append(t_free - r["t_arrive"])
    p50, p99 = _percentiles(lat)
    return {"solves_per_s": len(reqs) / sum(service), "p50_s": p50, "p99_s": p99,
            "requests": len(reqs), "service_s": [round(x, 3) for x in service]}


def _progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_serve(count, max_active=8, baseline=0):
    """Relaxation requests (a seeded prefix of the 4000-request stream at
    200/s: 70 % FM with demag, 30 % two-sublattice AFM, 0.5 ns each) served
    by the library's server in FP32; then the same requests re-timed with
    arrivals slowed to 0.8 x the measured capacity."""
    from paper_2411_18194_amd import inputs, mmp

    reqs = inputs.request_stream(seed=5, count=count)
    states = [inputs.request_state(r) for r in reqs]
    full = _serve_pass(reqs, states, mmp.FP32, 1.0, max_active)
    _progress("serving: offered stream done")
    # arrivals at 0.8 x capacity: scale the stream's mean rate (200/s) down
    scale = 200.0 / (0.8 * full["solves_per_s"])
    sus = _serve_pass(reqs, states, mmp.FP32, scale, max_active)
    _progress("serving: 0.8 x capacity done")
    base = None
    if baseline > 0:
        base = _sequential_fp64(reqs[:baseline], states[:baseline])
        _progress("serving: sequential FP64 baseline done")
        # the same subsample through the server, for a like-for-like ratio
        sub = _serve_pass(reqs[:baseline], states[:baseline], mmp.FP32, 1.0, max_active)
        base["served_fp32_same_requests"] = {k: round(v, 4) if isinstance(v, float) else v
                                             for k, v in sub.items()}
        base["note"] = (f"sequential plain FP64 timed on the first {baseline} requests only "
                        "(a seeded subsample; the full list would take minutes)")
    return {"workload": f"first {count} requests of the seeded c5 stream (Poisson 200/s, "
                        "nx, ny log-uniform 32..512, nz log-uniform 1..8, 70 % FM with "
                        "demag / 30 % AFM, 0.5 ns DP45 relaxation each, tol 1e-5)",
            "precision": "f32", "max_active": max_active,
            "offered": {k: round(v, 4) if isinstance(v, float) else v for k, v in full.items()},
            "at_0.8_capacity": {k: round(v, 4) if isinstance(v, float) else v
                                for k, v in sus.items()},
            "arrival_rate_0.8_capacity_per_s": round(200.0 / scale, 3),
            "sequential_fp64": base}


# rocprofv3 kernel names -> kernel classes of the library's event profiler
KERNEL_CLASSES = (("k4_fftx_fwd", "fftx_fwd"), ("k_fftx_fwd", "fftx_fwd"),
                  ("k4_fftx_inv", "fftx_inv"), ("k_fftx_inv", "fftx_inv"),
                  ("k4_fftz_mul", "fftz_mul"), ("k_fftz_mul", "fftz_mul"),
                  ("k4_ffty_mul2d", "ffty_mul2d"), ("k_ffty_mul2d", "ffty_mul2d"),
                  ("k_field", "field"))


def _kernel_class(name):
    base = name.split("(")[0].replace("void ", "").replace("mmp::", "")
    for pre, cls in KERNEL_CLASSES:
        if base.startswith(pre + "<") or base == pre:
            return cls
    if base.startswith(("k4_ffty<", "k_ffty<")):
        targs = [a.strip() for a in base.split("<", 1)[1].rstrip(">").split(",")]
        # <T, L1, L2, INV, FULL> / <T, INV, P2>
        inv = targs[3] if base.startswith("k4_ffty<") else targs[1]
        return "ffty_inv" if inv == "true" else "ffty_fwd"
    return None


def counters_from(root, last):
    """profiles/counters_c2_fp32.json from rocprofv3 --pmc CSVs.

    root holds four runs: fetch/ and write/ (FETCH_SIZE, WRITE_SIZE of a
    short bench.py run) and cfetch/ and cwrite/ (the same counters for
    bench.py --copy-calib, a 1 GiB device copy).  Per kernel class the last
    `last` dispatches (the timed steps, after the autotuner's candidate
    launches) are averaged; KiB per dispatch are scaled by what the counter
    reads per byte of the copy."""
    import csv
    import glob

    def read(sub, ctr):
        out = {}
        for f in glob.glob(os.path.join(root, sub, "**", "*counter_collection.csv"),
                           recursive=True):
            with open(f) as fh:
                for r in csv.DictReader(fh):
                    if r["Counter_Name"] == ctr:
                        out.setdefault(r["Kernel_Name"], []).append(
                            (int(r["Dispatch_Id"]), float(r["Counter_Value"])))
        return out

    copy_bytes = 1 << 30
    cf = max(v for vals in read("cfetch", "FETCH_SIZE").values() for _, v in vals)
    cw = max(v for vals in read("cwrite", "WRITE_SIZE").values() for _, v in vals)
    f_scale, w_scale = copy_bytes / (cf * 1024.0), copy_bytes / (cw * 1024.0)
    res = {}
    for ctr, sub, scale, key in (("FETCH_SIZE", "fetch", f_scale, "read"),
                                 ("WRITE_SIZE", "write", w_scale, "write")):
        per = {}
        for name, vals in read(sub, ctr).items():
            cls = _kernel_class(name)
            if cls:
                per.setdefault(cls, []).extend(vals)
        for cls, vals in per.items():
            vals.sort()
            tail = [v for _, v in vals[-last:]]
            res.setdefault(cls, {})[key + "_bytes_per_launch"] = \
                sum(tail) / len(tail) * 1024.0 * scale
    for cls, d in res.items():
        d["bytes_per_launch"] = d.get("read_bytes_per_launch", 0.0) + \
            d.get("write_bytes_per_launch", 0.0)
    out = {"source_hash": src_hash(), "fetch_scale": f_scale, "write_scale": w_scale,
           "note": "rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE per dispatch (KiB), scaled by the "
                   "counter's reading for a 1 GiB device-to-device copy; mean of the last "
                   f"{last} dispatches of each kernel class (the timed steps)",
           "kernels": res}
    with open(COUNTERS, "w") as fh:
        json.dump(out, fh, indent=1)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-prof", action="store_true")
    ap.add_argument("--serve", type=int, default=8,
                    help="requests in the serving measurement (0 = skip)")
    ap.add_argument("--serve-baseline", type=int, default=3,
                    help="requests of that list also run one at a time in FP64")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default demag plan instead of timing candidates first")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a 1 GiB device-to-device copy (counter calibration)")
    ap.add_argument("--counters-from", metavar="DIR",
                    help="write the HBM-traffic summary from rocprofv3 --pmc runs in DIR "
                         "(fetch/, write/, cfetch/, cwrite/) and exit")
    ap.add_argument("--counters-last", type=int, default=12)
    args = ap.parse_args()
    if args.counters_from:
        print(json.dumps(counters_from(args.counters_from, args.counters_last), indent=1))
        return
    if args.copy_calib:
        import torch
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        a.fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": a.numel() * 4, "copies": 3}))
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the method has no multi-GPU path here "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    from paper_2411_18194_amd import mmp
    tune = not args.no_autotune
    r32 = run_gpu(mmp.FP32, args.steps, args.warmup, prof=not args.no_prof, tune=tune)
    _progress("FP32 film done")
    out = {
        "metric": METRIC, "value": round(r32["value"], 1), "unit": "cell-field-evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(r32["ms_per_step"], 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "512x512x16 film, 2 nm cells, demag + exchange + interfacial "
                               "DMI (bottom layer) + uniaxial + Zeeman, fixed-step DP45 "
                               "(0.1 ns / 1667)",
                   "cells": 512 * 512 * 16, "field_evals_per_step": 6,
                   "demag_pad": r32["plan"]["pad"]},
        "state_finite": r32["finite"], "max_norm_error": r32["norm_err"],
        "plan": {k: v for k, v in r32["plan"].items() if k != "demag_ms"},
        "autotune_s": None if r32["tune_s"] is None else round(r32["tune_s"], 3),
    }
    if not args.no_prof:
        out["roofline"] = roofline(r32, 4)
        out["roofline"]["profiled_ms_per_step"] = round(r32["prof_ms_per_step"], 4)
        cr = copy_rate(out["roofline"]["algorithmic_bytes_per_launch"])
        out["roofline"]["copy_same_bytes_GBps"] = round(cr, 1)
        out["roofline"]["frac_of_copy"] = round(out["roofline"]["achieved"] / cr, 4)
    if not args.no_fp64:
        r64 = run_gpu(mmp.FP64, max(3, args.steps // 3), args.warmup, prof=False, tune=tune)
        _progress("FP64 film done")
        out["fp64"] = {"value": round(r64["value"], 1), "unit": "cell-field-evals/s",
                       "ms_per_step": round(r64["ms_per_step"], 4),
                       "fp32_speedup": round(r32["value"] / r64["value"], 3),
                       "plan": {k: v for k, v in r64["plan"].items() if k != "demag_ms"}}
    if args.serve > 0:
        out["serving"] = run_serve(args.serve, baseline=min(args.serve_baseline, args.serve))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
        _progress("CPU baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
