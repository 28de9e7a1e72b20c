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

Serving: a prefix of the seeded request stream through the library's
server (FP32, continuous batching), time-boxed, then at 0.8x the measured
capacity, beside plain sequential FP64 on a subsample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-fp64]
       [--no-cpu-baseline] [--no-prof] [--no-autotune] [--no-accuracy] [--serve N]
       [--serve-seconds S] [--serve-active A] [--serve-baseline K]
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


def run_gpu(precision, steps, warmup, prof=True, tune=True, plan_fields=None):
    import torch

    from paper_2411_18194_amd import inputs, mmp

    p, m0 = inputs.config_c2()
    g = mmp.Grid(p, precision)
    stream = torch.cuda.current_stream()
    g.set_stream(stream.cuda_stream)
    g.set_state(m0)
    t_tune = time.perf_counter()
    if plan_fields:
        plan = g.set_plan(**plan_fields)
    else:
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


def gpu_first_torque():
    """dm/dt of every term at the film's initial state, FP32 and FP64 grids
    (the FP32 grid holds the state rounded to float32)."""
    from paper_2411_18194_amd import inputs, mmp

    p, m0 = inputs.config_c2()
    out = {}
    for prec, name in ((mmp.FP32, "f32"), (mmp.FP64, "f64")):
        g = mmp.Grid(p, prec)
        g.set_state(m0)
        out[name] = g.eval_heff(mmp.T_ALL | mmp.T_ZL | mmp.OUT_TORQUE)[0].astype(np.float64)
        g.close()
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(gpu_torque=None):
    """FP64 oracle on the full 512x512x16 film: three single-stage
    evaluations (field + torque of every cell, then one Runge-Kutta stage
    combination), FFTs on every host core, then one on a single core.  The
    first two evaluations are of the initial state in FP64 and rounded to
    float32: the GPU's first-stage torques of the same states are checked
    against them (max |d tau| / max |tau|)."""
    import numpy
    import scipy

    from oracle.system import Problem
    from paper_2411_18194_amd import inputs

    cores = len(os.sched_getaffinity(0))
    p, m64 = inputs.config_c2()
    m32 = m64.astype(np.float32).astype(np.float64)
    N = p["n"][0] * p["n"][1] * p["n"][2]
    t_setup = time.perf_counter()
    P = Problem(p, demag_workers=cores)
    t_setup = time.perf_counter() - t_setup
    dt = inputs.c2_fixed_dt()

    def stage(m):
        t0 = time.perf_counter()
        k = P.rhs(0.0, [m])
        y2 = P.stepper._combine([m], [k], [0.2], dt)
        return time.perf_counter() - t0, k[0], y2

    secs, acc = [], {}
    for name, m in (("f64", m64), ("f32", m32), ("f64", m64)):
        sec, tau, _ = stage(m)
        secs.append(sec)
        if gpu_torque is not None and name not in acc:
            ref = tau
            acc[name] = float(np.abs(gpu_torque[name] - ref).max() / np.abs(ref).max())
        _progress(f"cpu baseline: evaluation {len(secs)} took {sec:.1f} s")
    P.demag.workers = 1
    sec1, _, _ = stage(m64)
    _progress(f"cpu baseline: single-core evaluation took {sec1:.1f} s")
    med = float(np.median(secs))
    out = {"value": N / med, "unit": "cell-field-evals/s", "cores": cores, "kind": "oracle",
           "sample": "the full 512x512x16 film, 3 single-stage evaluations (field + torque of "
                     "every cell + one DP45 stage combination), median; FP64 numpy/scipy "
                     f"(FFT on {cores} threads, element-wise work on 1)",
           "seconds": [round(x, 2) for x in secs], "setup_s": round(t_setup, 1),
           "value_1core": N / sec1, "seconds_1core": round(sec1, 2),
           "cpu_model": _cpu_model(), "numpy": numpy.__version__, "scipy": scipy.__version__}
    if acc:
        out["gpu_first_stage_torque_rel_err"] = acc
    return out


def accuracy_c2crop():
    """The 64x64x4 crop of the film (its own open-boundary system) run for
    0.1 ns of fixed DP45 steps in FP32 and FP64, against the FP64 oracle's
    stored run of the same steps (tests/golden/traj_c2crop.*): max over cells
    of |m_gpu - m_ref| and |E_gpu - E_ref| / sum |E_ref,term| at the end."""
    from paper_2411_18194_amd import inputs, mmp

    path = os.path.join(ROOT, "tests", "golden", "traj_c2crop")
    if not os.path.exists(path + ".npz"):
        return None
    gold = np.load(path + ".npz")
    with open(path + ".json") as fh:
        meta = json.load(fh)
    p, m0 = inputs.config_c2_crop()
    out = {"workload": f"64x64x4 crop of the film, {meta['steps']} fixed DP45 steps of "
                       f"{meta['dt']:.4g} s (0.1 ns), vs the FP64 oracle"}
    for prec, name in ((mmp.FP32, "f32"), (mmp.FP64, "f64")):
        g = mmp.Grid(p, prec)
        g.set_state(m0)
        g.run_fixed(meta["dt"], meta["steps"])
        m = g.get_state()[0]
        _, e = g.eval_heff(mmp.T_ALL, want_b=False)
        g.close()
        r = {"max_dm": float(np.linalg.norm(m - gold["m"].astype(np.float64), axis=1).max())}
        if "energy" in gold:
            ref = dict(zip([str(x) for x in gold["energy_names"]], gold["energy"]))
            scale = sum(abs(v) for v in ref.values())
            r["rel_energy_err"] = abs(sum(e.values()) - sum(ref.values())) / scale
        out[name] = r
    return out


def _percentiles(lat):
    if len(lat) == 0:
        return (None, None)
    lat = np.sort(np.asarray(lat))
    return (float(np.percentile(lat, 50)), float(np.percentile(lat, 99)))


def _stats(prefix, vals):
    p50, p99 = _percentiles(vals)
    return {prefix + "_p50_s": None if p50 is None else round(p50, 4),
            prefix + "_p99_s": None if p99 is None else round(p99, 4)}


def _serve_pass(reqs, states, precision, arrivals, box_s, max_active, batch=True):
    """Open-loop replay through the library's server: request i is submitted
    at arrivals[i] seconds after the start; results are collected until all
    are done or box_s seconds have passed (the rest are counted as
    unfinished).  Latency = t_done - t_submit, queue wait = t_admit -
    t_submit, service = t_done - t_admit, on the server's clock."""
    from paper_2411_18194_amd import mmp

    srv = mmp.Server(hbm_budget=64 << 30, max_active=max_active, precision=precision,
                     batch=batch)
    t0 = srv.clock()
    tickets, res = [], {}
    i = 0
    while True:
        now = srv.clock() - t0
        while i < len(reqs) and arrivals[i] <= now:
            tickets.append(srv.submit(reqs[i]["params"], states[i], reqs[i]["t_relax"],
                                      tol=reqs[i]["tol"]))
            i += 1
        for k, t in enumerate(tickets):
            if k not in res:
                r = srv.poll(t)
                if r is not None:
                    res[k] = r
        if len(res) == len(reqs) or now > box_s:
            break
        time.sleep(2e-3)
    end = srv.clock() - t0
    srv.close()
    done = [res[k] for k in sorted(res)]
    bad = [x.status for x in done if x.status != 0]
    if bad:
        raise RuntimeError(f"serving: {len(bad)} requests failed: {bad[:5]}")
    lat = [x.t_done - x.t_submit for x in done]
    span = (max(x.t_done for x in done) - t0) if done else end
    out = {"submitted": i, "completed": len(done), "unfinished": len(reqs) - len(done),
           "time_box_s": box_s, "elapsed_s": round(end, 3),
           "solves_per_s": round(len(done) / (span if len(done) == len(reqs) else end), 4),
           "attempts": int(sum(x.steps + x.rejects for x in done)),
           "cells_done": int(sum(reqs[k]["params"]["n"][0] * reqs[k]["params"]["n"][1] *
                                 reqs[k]["params"]["n"][2] for k in res))}
    out.update(_stats("latency", lat))
    out.update(_stats("queue", [x.t_admit - x.t_submit for x in done]))
    out.update(_stats("service", [x.t_done - x.t_admit for x in done]))
    if len(done) < len(reqs):
        out["note"] = ("percentiles over the completed requests only; the unfinished ones "
                       "had waited at least time_box_s - t_arrive when the box closed")
    return out


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
    out = {"solves_per_s": round(len(reqs) / sum(service), 4), "requests": len(reqs),
           "service_s": [round(x, 3) for x in service]}
    out.update(_stats("latency", lat))
    return out


def _progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_serve(count, box_s, max_active=16, baseline=0, baseline_short=0, short_frac=0.1):
    """A prefix of the seeded 4000-request stream (Poisson 200/s: 70 % FM
    with demag, 30 % two-sublattice AFM, 0.5 ns of relaxation each) served by
    the library's server in FP32 with continuous batching, arrivals at their
    stream times, in a time box; then the same requests with arrivals at 0.8
    times the capacity the first pass measured; then the first `baseline`
    requests run one at a time in plain FP64 and, for a like-for-like ratio,
    served in FP32."""
    from paper_2411_18194_amd import inputs, mmp

    reqs = inputs.request_stream(seed=5, count=count)
    states = [inputs.request_state(r) for r in reqs]
    _progress(f"serving: {count} request states generated")
    arr = np.array([r["t_arrive"] for r in reqs])
    full = _serve_pass(reqs, states, mmp.FP32, arr, box_s, max_active)
    _progress(f"serving: offered stream done ({full['completed']}/{count} in "
              f"{full['elapsed_s']} s)")
    cap = max(full["solves_per_s"], 1e-3)
    rate = 0.8 * cap
    # the stream's inter-arrival pattern, stretched to the lower mean rate
    sus = _serve_pass(reqs, states, mmp.FP32, arr * (200.0 / rate), box_s, max_active)
    _progress("serving: 0.8 x capacity done")
    base = None
    if baseline > 0:
        base = _sequential_fp64(reqs[:baseline], states[:baseline])
        _progress("serving: sequential FP64 baseline done")
        sub = _serve_pass(reqs[:baseline], states[:baseline], mmp.FP32, arr[:baseline],
                          1e9, max_active)
        base["served_fp32_same_requests"] = sub
        base["served_fp32_speedup"] = round(sub["solves_per_s"] / base["solves_per_s"], 3)
        base["note"] = (f"sequential plain FP64 timed on the first {baseline} requests of the "
                        "prefix (a seeded subsample)")
    short = None
    if baseline_short > 0:
        # the first requests of the prefix with their relaxation shortened,
        # so that a larger subsample of both fits the run's time budget
        sreqs = [dict(r, t_relax=r["t_relax"] * short_frac) for r in reqs[:baseline_short]]
        sstates = states[:baseline_short]
        short = _sequential_fp64(sreqs, sstates)
        _progress("serving: sequential FP64 baseline (shortened relaxations) done")
        sub = _serve_pass(sreqs, sstates, mmp.FP32, arr[:baseline_short], 1e9, max_active)
        short["served_fp32_same_requests"] = sub
        short["served_fp32_speedup"] = round(sub["solves_per_s"] / short["solves_per_s"], 3)
        short["note"] = (f"the first {baseline_short} requests of the prefix with t_relax x "
                         f"{short_frac} ({short_frac * 0.5:g} ns): sequential plain FP64 vs "
                         "served FP32")
    return {"workload": f"first {count} requests of the seeded 4000-request stream (Poisson "
                        "200/s, nx, ny log-uniform 32..512, nz log-uniform 1..8, cubic cells "
                        "1-5 nm, 70 % FM with demag / 30 % two-sublattice AFM, 0.5 ns DP45 "
                        "relaxation each, tol 1e-5)",
            "precision": "f32", "max_active": max_active, "offered": full,
            "at_0.8_capacity": dict(sus, arrival_rate_per_s=round(rate, 4)),
            "sequential_fp64": base, "sequential_fp64_shortened": short}


# rocprofv3 kernel names -> kernel classes of the library's event profiler
KERNEL_CLASSES = (("k4_fftx_fwd", "fftx_fwd"), ("k_fftx_fwd", "fftx_fwd"),
                  ("k4_fftx_inv", "fftx_inv"), ("k_fftx_inv", "fftx_inv"),
                  ("k4_fftz_mul", "fftz_mul"), ("k4_fftz_mul_w", "fftz_mul"),
                  ("k4_fftz_mul_kl", "fftz_mul"), ("k_fftz_mul", "fftz_mul"),
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
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the accuracy check against the stored oracle run")
    ap.add_argument("--serve", type=int, default=200,
                    help="requests of the stream in the serving measurement (0 = skip)")
    ap.add_argument("--serve-seconds", type=float, default=45.0,
                    help="time box of each serving pass")
    ap.add_argument("--serve-active", type=int, default=16,
                    help="requests on the device at once")
    ap.add_argument("--serve-baseline-short", type=int, default=20,
                    help="first requests of that list, relaxations cut to a tenth, also run "
                         "one at a time in FP64 and served in FP32")
    ap.add_argument("--serve-baseline", type=int, default=3,
                    help="first requests of that list also run one at a time in FP64")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default demag plan instead of timing candidates first")
    ap.add_argument("--plan", metavar="JSON",
                    help="FP32 demag/field plan fields to install instead of autotuning "
                         "(so that profiler runs time and count the same launches)")
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
    r32 = run_gpu(mmp.FP32, args.steps, args.warmup, prof=not args.no_prof, tune=tune,
                  plan_fields=json.loads(args.plan) if args.plan else None)
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
        out["serving"] = run_serve(args.serve, args.serve_seconds, args.serve_active,
                                   baseline=min(args.serve_baseline, args.serve),
                                   baseline_short=min(args.serve_baseline_short, args.serve))
    acc = None if args.no_accuracy else accuracy_c2crop()
    if acc is not None:
        out["accuracy"] = acc
        _progress("accuracy check done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(gpu_first_torque())
        _progress("CPU baseline done")
        if "gpu_first_stage_torque_rel_err" in out["cpu_baseline"]:
            out.setdefault("accuracy", {})["fullsize_first_stage_torque_rel_err"] = \
                out["cpu_baseline"].pop("gpu_first_stage_torque_rel_err")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
