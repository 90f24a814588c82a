#!/usr/bin/env python3
"""Write the oracle's expected values for the full-size workloads.

Every number in the files this script writes comes from the FP64 oracle
(oracle/) run on the seeded inputs of problems/; nothing is read from the GPU
engine.  One JSON file per (workload, seed, eps):

  tests/golden/<workload>_s<seed>_eps<eps>.json

holding
  * the cluster sizes after every stage (ranks of the sparsified interfaces,
    Alg. 2 with the ratio rule of Section 4), zlib + base64 int32 arrays;
  * the (|p|, m, r) shape of every CPQR and the algorithmic CPQR flops
    4|p|mr - 2r^2(|p| + m) + 4/3 r^3 + m r summed over them;
  * for b = make_rhs(N, 1, seed): M^{-1} b (the preconditioner apply of
    Section 2.8) and the FGMRES solution x of Section 4 to 1e-10, each as its
    2-norm plus 512 entries at seeded indices, the iteration count and the
    true relative residual;
  * an estimate of ||A^{-1}||_2 (oracle/conditioning.py), which turns the two
    residual bounds into a bound on ||x_engine - x_oracle||.

With --unscaled the oracle runs the sparsification without scaling of
Section 2.5 (scale=False) and the file is <workload>_s<seed>_eps<eps>_unscaled.json.

Usage (from the repository root; one process per case, single-threaded BLAS):
  python tests/golden/make_goldens.py c2 --seeds 0 1 2 --eps 1e-2 1e-4 1e-6
  python tests/golden/make_goldens.py c4 --seeds 0 1 2
  python tests/golden/make_goldens.py c3 --seeds 0
  python tests/golden/make_goldens.py c2 --seeds 0 --eps 1e-2 --unscaled
"""

from __future__ import annotations

import argparse
import base64
import json
import os
import sys
import time
import zlib

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

NSAMPLE = 512


def pack(a, dtype):
    return base64.b64encode(zlib.compress(np.ascontiguousarray(a, dtype=dtype).tobytes(), 9)).decode()


def unpack(s, dtype):
    return np.frombuffer(zlib.decompress(base64.b64decode(s)), dtype=dtype)


def golden_path(workload, seed, eps, scale=True):
    return os.path.join(HERE, f"{workload}_s{seed}_eps{eps:g}{'' if scale else '_unscaled'}.json")


def load(workload, seed, eps, scale=True):
    """The stored record of one case, with its arrays decoded (None if absent)."""
    p = golden_path(workload, seed, eps, scale)
    if not os.path.exists(p):
        return None
    with open(p) as f:
        g = json.load(f)
    g["stage_sizes"] = {int(k): unpack(v, np.int32) for k, v in g["stage_sizes"].items()}
    g["cpqr_shapes"] = unpack(g["cpqr_shapes"], np.int32).reshape(-1, 3)
    g["sample_idx"] = unpack(g["sample_idx"], np.int64)
    g["apply_sample"] = np.array(g["apply_sample"])
    g["x_sample"] = np.array(g["x_sample"])
    return g


def cpqr_flops(shapes):
    """Algorithmic flops of the partial CPQRs: Householder QR of the first r
    pivot columns of a |p| x m matrix with the trailing update, plus one norm
    update per column and step."""
    tot = 0.0
    for P, m, r in shapes:
        P, m, r = float(P), float(m), float(r)
        tot += 4 * P * m * r - 2 * r * r * (P + m) + 4.0 / 3.0 * r ** 3 + m * r
    return tot


def make_case(workload, seed, eps, tol=1e-10, scale=True):
    from threadpoolctl import threadpool_limits
    from problems import config_problem, make_rhs
    from oracle.ordering import order_grid
    from oracle import spaqr as osq, gmres as ogm
    from oracle.conditioning import inv_norm2_estimate

    prob = config_problem(workload, seed=seed)
    A, dims, L = prob["A"], prob["dims"], prob["levels"]
    N = A.shape[0]
    b = make_rhs(N, 1, seed=seed)[:, 0]
    t0 = time.perf_counter()
    with threadpool_limits(limits=1):
        F = osq.factor(A, order_grid(dims, L), eps, scale=scale)
        t1 = time.perf_counter()
        y = osq.apply(F, b)
        x, it, rel = ogm.fgmres(lambda v: A @ v, lambda v: osq.apply(F, v), b, tol)
        t2 = time.perf_counter()
    inv = inv_norm2_estimate(A)
    shapes = []
    for k in range(L, 0, -1):
        rec = F.stages[k]
        for p in sorted(rec.get("cpqr_shapes", {})):
            shapes.append(rec["cpqr_shapes"][p])
    shapes = np.array(shapes, dtype=np.int64).reshape(-1, 3)
    rng = np.random.default_rng([seed, 7])
    idx = np.sort(rng.choice(N, size=min(NSAMPLE, N), replace=False)).astype(np.int64)
    out = {
        "workload": workload, "seed": seed, "eps": eps, "scale": bool(scale), "tol": tol, "n": N, "levels": L,
        "dims": list(dims),
        "stage_sizes": {str(k): pack(F.stages[k]["sizes_post"], np.int32) for k in range(L, 0, -1)},
        "sparsified_stages": [k for k in range(L, 0, -1) if F.stages[k]["sparsified"]],
        "interfaces_scaled": sum(1 for op in F.ops if op[0] == "scale"),
        "cpqr_shapes": pack(shapes, np.int32),
        "cpqr_flops": cpqr_flops(shapes),
        "factor_bytes_fp64": osq.factor_bytes(F, 8),
        "rhs_seed": seed,
        "b_norm": float(np.linalg.norm(b)),
        "sample_idx": pack(idx, np.int64),
        "apply_norm": float(np.linalg.norm(y)),
        "apply_sample": [float(v) for v in y[idx]],
        "gmres_iterations": int(it), "gmres_relres": float(rel),
        "x_norm": float(np.linalg.norm(x)),
        "x_sample": [float(v) for v in x[idx]],
        "inv_norm2_est": inv,
        "oracle_seconds": {"factor": t1 - t0, "apply_and_gmres": t2 - t1},
    }
    with open(golden_path(workload, seed, eps, scale), "w") as f:
        json.dump(out, f, indent=0)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("workload", choices=["c1", "c2", "c3", "c4"])
    ap.add_argument("--seeds", type=int, nargs="+", default=[0])
    ap.add_argument("--eps", type=float, nargs="+", default=None)
    ap.add_argument("--unscaled", action="store_true", help="the sparsification without scaling (Section 2.5)")
    a = ap.parse_args()
    from problems import config_problem
    eps_list = a.eps if a.eps else [e for e in config_problem(a.workload)["eps"] if e > 0]
    for s in a.seeds:
        for e in eps_list:
            t = time.perf_counter()
            g = make_case(a.workload, s, e, scale=not a.unscaled)
            print(f"{a.workload} seed {s} eps {e:g}: {time.perf_counter() - t:.1f} s, "
                  f"{g['gmres_iterations']} its, relres {g['gmres_relres']:.2e}", flush=True)


if __name__ == "__main__":
    main()
