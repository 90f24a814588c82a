"""Autotuner of the kernel dispatch thresholds (spaqr_tuning).

The thresholds choose which kernel factors each block -- register-panel or
LDS-panel QR, whole fronts or pivot block plus trailing tiles, vector-ALU or
matrix-core trailing update, register, cooperative or single-workgroup CPQR,
fused or general scaling, dense or reflector interface operators -- never
what is computed.  For one workload the tuner times the numeric
factorization plus the FGMRES solve (the benchmark's step, values resident
on the device, the analysis made once) under candidate settings, by
coordinate descent from the library defaults: every knob in turn takes each
of its candidate values with the others fixed, the fastest is kept, and the
sweep repeats until no knob changes.  Each candidate is timed as the median
of `reps` steps after one warm-up step; the step's result must still reach
the solve tolerance.

The table it writes (tuning.json beside this file, one entry per workload)
holds the chosen settings and the measured times; load_table() reads it and
apply(workload) sets the entry for a workload.

    python -m paper_2010_06807_amd.autotune c4 [--reps 3]
"""

from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tuning.json")

# candidate values of every knob, the library default first
CANDIDATES = {
    "trail_mfma": [1, 0],
    "split_rows": [1024, 512, 2048],
    "split_cols": [1024, 512, 2048],
    "qr_reg_max_rows": [1024, 512, 256],
    "cpqr_coop": [1, 0],
    "cpqr_dd": [2, 1, 0],
    "cpqr_team": [2, 1, 0],
    "scale_small": [64, 32],
    "iface_dense": [64, 32],
}


def load_table(path=TABLE):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def apply(workload, path=TABLE):
    """Set the tuned thresholds of `workload` if the table has them; returns
    the settings applied (None: defaults kept)."""
    import paper_2010_06807_amd as P
    e = load_table(path).get(workload)
    if not e:
        return None
    P.set_tuning(**e["tuning"])
    return e["tuning"]


def tune(workload, reps=3, seeds=1, eps=1e-2, tol=1e-10, log=print):
    import numpy as np
    import torch
    import paper_2010_06807_amd as P
    sys.path.insert(0, os.path.dirname(HERE))
    from problems import config_problem, make_rhs
    dev = torch.device("cuda:0")
    probs = [config_problem(workload, seed=i) for i in range(seeds)]
    A, dims, L = probs[0]["A"], probs[0]["dims"], probs[0]["levels"]
    N = A.shape[0]
    sym = P.analyze(A, P.order_grid(dims, L))
    dAs = [P.DeviceCSR(q["A"], dev) for q in probs]
    bs = [torch.from_numpy(make_rhs(N, 1, seed=i)).to(dev) for i in range(seeds)]

    def step(i):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fac = P.factor_device(probs[i % seeds]["A"], sym, dAs[i % seeds], eps=eps, precision=32)
        x, info = fac.solve(bs[i % seeds], tol=tol)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if not info[0]["converged"]:
            raise RuntimeError("a tuned step missed the solve tolerance")
        return dt

    def measure(setting):
        P.set_tuning()
        P.set_tuning(**setting)
        step(0)
        return statistics.median(step(i) for i in range(reps))

    best = {k: v[0] for k, v in CANDIDATES.items()}
    best_t = measure(best)
    default_t = best_t
    log(f"[autotune] {workload}: defaults {1e3 * best_t:.2f} ms")
    trials = [{"tuning": dict(best), "ms": 1e3 * best_t}]
    changed = True
    while changed:
        changed = False
        for knob, values in CANDIDATES.items():
            for v in values:
                if v == best[knob]:
                    continue
                cand = dict(best, **{knob: v})
                t = measure(cand)
                trials.append({"tuning": cand, "ms": 1e3 * t})
                log(f"[autotune] {knob}={v}: {1e3 * t:.2f} ms")
                if t < 0.98 * best_t:
                    best, best_t, changed = cand, t, True
    P.set_tuning()
    props = torch.cuda.get_device_properties(0)
    return {"workload": workload, "n": N, "device": props.name, "reps": reps,
            "tuning": best, "ms_step": 1e3 * best_t, "ms_step_defaults": 1e3 * default_t,
            "trials": trials}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("workloads", nargs="+")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--seeds", type=int, default=1)
    ap.add_argument("--out", default=TABLE)
    a = ap.parse_args()
    table = load_table(a.out)
    for w in a.workloads:
        table[w] = tune(w, reps=a.reps, seeds=a.seeds, log=lambda s: print(s, file=sys.stderr, flush=True))
        with open(a.out, "w") as f:
            json.dump(table, f, indent=1)
    print(json.dumps({w: {k: table[w][k] for k in ("tuning", "ms_step", "ms_step_defaults")} for w in a.workloads}))


if __name__ == "__main__":
    main()
