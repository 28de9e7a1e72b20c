"""Write the oracle's 0.1 ns fixed-step trajectories used by the GPU tests.

Runs only the FP64 CPU oracle (oracle/) on the seeded crop systems from
paper_2411_18194_amd.inputs and stores, per system, the state after every
`every` steps' worth of time (<m> per sublattice) and the full final state
rounded to float32 (enough for a 1e-4 comparison), with the per-term
energies of the final FP64 state.  Usage:

    python tests/golden/make_trajectories.py [c2crop c3crop c4crop]

Takes minutes per system on a few cores (oracle FFTs use all of them).
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

# name -> (config builder, dt, steps, sample every n steps)
SYSTEMS = {
    "c2crop": (inputs.config_c2_crop, inputs.c2_fixed_dt(), 1667, 167),
    "c3crop": (inputs.config_c3_crop, 5e-15, 20000, 2000),
    "c4crop": (inputs.config_c4_crop, inputs.C4_FIXED_DT, 10000, 1000),
}


def run(name):
    build, dt, steps, every = SYSTEMS[name]
    p, m = build()
    P = Problem(p)
    y = P.initial_state(m)
    t = 0.0
    samples = []
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        k = min(every, steps - done)
        y, t = P.run_fixed(y, t, dt, k)
        done += k
        samples.append([t] + [float(v) for v in y[0].mean(axis=(2, 3, 4)).ravel()])
        print(f"{name}: {done}/{steps} steps, {time.perf_counter() - t0:.0f} s", flush=True)
    out = {"m": y[0].astype(np.float32), "samples": np.array(samples)}
    # energies of the final FP64 state, per term (joules), for the relative
    # energy error of a run against this one
    E = P.energies(*y) if len(y) > 1 else P.energies(y[0])
    out["energy_names"] = np.array(list(E.keys()))
    out["energy"] = np.array([E[k] for k in E])
    if len(y) > 1:
        out["u"] = y[1].astype(np.float32)
        out["v"] = y[2].astype(np.float32)
    np.savez_compressed(os.path.join(HERE, f"traj_{name}.npz"), **out)
    meta = {"system": name, "dt": dt, "steps": steps, "sample_every": every,
            "t_end": t, "n": list(p["n"]), "nsub": p["nsub"],
            "written_by": "python tests/golden/make_trajectories.py " + name,
            "oracle": "FP64 oracle.system.Problem.run_fixed (DP45, no step control)"}
    with open(os.path.join(HERE, f"traj_{name}.json"), "w") as fh:
        json.dump(meta, fh, indent=1)


if __name__ == "__main__":
    for name in sys.argv[1:] or list(SYSTEMS):
        run(name)
