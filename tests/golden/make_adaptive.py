"""Write the oracle's adaptive-run references used by the GPU tests.

Runs only the FP64 CPU oracle (oracle/) on seeded inputs from
paper_2411_18194_amd.inputs, with the Dormand-Prince pair and the step
control of the oracle (tol 1e-5, dt0 1e-14):

* c1protocol: the 64x16x1 film's protocol - 200 ps of relaxation with
  alpha = 1 and no field from the random initial state, then t reset to 0,
  alpha = 0.02 and the field on, 1 ns with <m> every 5 ps (201 samples);
  stores both phases' step/reject counts, the samples and the final states;
* c3crop_adaptive: the 128x64 two-sublattice crop (grains, Zhang-Li
  current) for 0.1 ns adaptively, <m> every 10 ps, final state as float32;
* served: a seeded subsample of the request stream (the first requests of
  its first 300 with at most 64*64*2 cells: four ferromagnets with demag and
  two two-sublattice magnets), each relaxed alone for 20 ps; stores <m> per
  sublattice, the total energy, steps and rejects.

Usage:  python tests/golden/make_adaptive.py [c1protocol c3crop_adaptive served]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.system import Problem  # noqa: E402
from paper_2411_18194_amd import inputs  # noqa: E402

TOL, DT0 = 1e-5, 1e-14
C1_RELAX, C1_RUN, C1_EVERY = 200e-12, 1e-9, 5e-12
C3_T, C3_EVERY = 0.1e-9, 10e-12
SERVED_T = 20e-12
SERVED_MAX_CELLS = 64 * 64 * 2
SERVED_FM, SERVED_AFM = 4, 2


def _avg(y):
    return y[0].mean(axis=(2, 3, 4))


def c1_relax_params(p):
    return dict(p, alpha=[1.0], B_ext=(0.0, 0.0, 0.0))


def c1protocol():
    p, m0 = inputs.config_c1()
    P = Problem(c1_relax_params(p))
    y, t, info_r, _ = P.run([m0.copy()], 0.0, C1_RELAX, tol=TOL, dt0=DT0)
    m_relaxed = y[0]
    P = Problem(p)
    y, t, info, samples = P.run([m_relaxed.copy()], 0.0, C1_RUN, tol=TOL, dt0=DT0,
                                sample_every=C1_EVERY, sample=_avg)
    np.savez_compressed(os.path.join(HERE, "adaptive_c1protocol.npz"),
                        m_relaxed=m_relaxed, m_end=y[0],
                        t=np.array([s[0] for s in samples]),
                        m_avg=np.array([s[1] for s in samples]))
    return {"relax": {"t_end": C1_RELAX, "steps": info_r["steps"], "rejects": info_r["rejects"],
                      "alpha": 1.0, "B_ext": [0.0, 0.0, 0.0]},
            "run": {"t_end": C1_RUN, "steps": info["steps"], "rejects": info["rejects"],
                    "sample_every": C1_EVERY, "nsamples": len(samples)}}


def c3crop_adaptive():
    p, m0 = inputs.config_c3_crop()
    P = Problem(p)
    y, t, info, samples = P.run([m0.copy()], 0.0, C3_T, tol=TOL, dt0=DT0,
                                sample_every=C3_EVERY, sample=_avg)
    np.savez_compressed(os.path.join(HERE, "adaptive_c3crop.npz"), m_end=y[0].astype(np.float32),
                        t=np.array([s[0] for s in samples]),
                        m_avg=np.array([s[1] for s in samples]))
    return {"t_end": C3_T, "steps": info["steps"], "rejects": info["rejects"],
            "sample_every": C3_EVERY}


def served_subsample():
    """Indices into request_stream(seed=5, count=300) of the subsample."""
    reqs = inputs.request_stream(seed=5, count=300)
    fm, afm = [], []
    for i, r in enumerate(reqs):
        nx, ny, nz = r["params"]["n"]
        if nx * ny * nz > SERVED_MAX_CELLS:
            continue
        (fm if r["params"]["nsub"] == 1 else afm).append(i)
    return reqs, fm[:SERVED_FM] + afm[:SERVED_AFM]


def served():
    reqs, idx = served_subsample()
    out = []
    for i in idx:
        r = reqs[i]
        P = Problem(r["params"])
        m0 = inputs.request_state(r)
        y, t, info, _ = P.run([m0], 0.0, SERVED_T, tol=r["tol"], dt0=DT0)
        E = P.energies(y[0])
        out.append({"index": i, "n": list(r["params"]["n"]), "nsub": r["params"]["nsub"],
                    "m_avg": _avg(y).tolist(), "energy": float(sum(E.values())),
                    "energy_abs_sum": float(sum(abs(v) for v in E.values())),
                    "steps": info["steps"], "rejects": info["rejects"]})
        print(f"served {i}: {r['params']['n']} nsub {r['params']['nsub']} steps {info['steps']}",
              flush=True)
    return {"t_relax": SERVED_T, "stream": "request_stream(seed=5, count=300)",
            "selection": f"first {SERVED_FM} ferromagnets and first {SERVED_AFM} two-sublattice "
                         f"requests with at most {SERVED_MAX_CELLS} cells",
            "requests": out}


JOBS = {"c1protocol": c1protocol, "c3crop_adaptive": c3crop_adaptive, "served": served}


if __name__ == "__main__":
    path = os.path.join(HERE, "adaptive.json")
    meta = json.load(open(path)) if os.path.exists(path) else {}
    for name in sys.argv[1:] or list(JOBS):
        t0 = time.perf_counter()
        meta[name] = JOBS[name]()
        meta[name]["written_by"] = "python tests/golden/make_adaptive.py " + name
        meta[name]["oracle"] = "FP64 oracle.system.Problem.run (DP45, tol 1e-5, dt0 1e-14)"
        print(f"{name}: {time.perf_counter() - t0:.0f} s", flush=True)
        with open(path, "w") as fh:
            json.dump(meta, fh, indent=1)
