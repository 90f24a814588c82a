#!/usr/bin/env python3
"""spaQR on one MI355X: unknowns/s for one pass of the whole hot path.

A step factors one problem of the 1024 x 1024 advection-dominated workload
(N = 1,048,576, beta = (500, -300), 5% of the off-diagonal entries scaled by
U[0.5, 1.5] per seed, eps = 1e-2, 14 levels; the steps cycle through seeds
0..2) with FP32 blocks and factors -- every front, scaling and
sparsification of a level in one launch per phase -- and solves A x = b with
FP64 FGMRES to ||Ax - b|| / ||b|| <= 1e-10.  A's CSR and b are resident in HBM
when the timed region starts; the factorization reads the values from
device memory.  The ordering and symbolic analysis depend only on the
pattern, which the seeds share: they are made once, timed on their own and
reported separately, and an end-to-end figure includes them.

Printed as one JSON line: the throughput (value = N x steps / seconds of
factor + solve), per-step latency percentiles, the plain FP64 GPU path on
the same steps, the cross-request batched 256 x 256 workload (16 requests
per step) as a second figure, the roofline of the dominant kernel (HIP
events around its launches during the timed region) with the achieved HBM
rate of the apply and scaling phases, a replayed serving trace, and the
oracle timed on the host on a bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "unknowns/s factor+GMRES to 1e-10, batched FP32 vs plain FP64; p50/p99 latency"

WORKLOAD_TEXT = {
    "c1": "2D convection-diffusion, 5-point upwind,",
    "c2": "2D variable-coefficient convection-diffusion, 5-point upwind,",
    "c3": "3D convection-diffusion, 7-point upwind,",
    "c4": "2D advection-dominated, 5-point upwind with perturbed entries,",
}

# Published MI355X peaks used for the roofline fractions (dense matrix-core
# FP32 and the FP32 vector rate are the same published figure).
PEAK = {
    "hbm": (8000.0, "GB/s"),
    "alu32": (157.3, "TFLOP/s"),
    "alu64": (78.6, "TFLOP/s"),
    "mfma32": (157.3, "TFLOP/s"),
}
# bound of each kernel: HBM-bound data movement / apply, or vector-ALU
# arithmetic (the factorization kernels run on the VALU, not on MFMA; the
# CPQR's work is counted from the ranks read back after each stage)
KERNEL_BOUND = {
    "front_qr": "alu", "front_trail": "mfma", "front_wy_blocks": "mfma", "scale_qr": "alu", "scale_blocks": "alu",
    "sparsify": "alu", "sparsify_unscaled": "alu64",
    "apply_front_fwd": "hbm", "apply_front_bwd": "hbm", "apply_iface_fwd": "hbm", "apply_iface_bwd": "hbm",
}


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=6)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c4", help="c1..c4 (default c4, the largest single problem)")
    ap.add_argument("--seeds", type=int, default=3, help="the steps cycle through seeds 0..seeds-1")
    ap.add_argument("--eps", type=float, default=1e-2)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--fp64-steps", type=int, default=3, help="steps of the plain FP64 path (0: skip)")
    ap.add_argument("--unscaled-steps", type=int, default=3,
                    help="steps of the sparsification without scaling, Section 2.5 (0: skip)")
    ap.add_argument("--graph-points", type=int, default=65536,
                    help="points of the unstructured leg (algebraic MND of a Delaunay mesh; 0: skip)")
    ap.add_argument("--graph-steps", type=int, default=3)
    ap.add_argument("--unscaled-workload", default="c2",
                    help="workload of that leg (default c2: on c4 its FGMRES does not reach 1e-10 in 1000 steps)")
    ap.add_argument("--batch-workload", default="c2",
                    help="workload of the cross-request batched figure ('' to skip)")
    ap.add_argument("--batch", type=int, default=16, help="requests per step of the batched figure")
    ap.add_argument("--batch-steps", type=int, default=6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-side", type=int, default=256,
                    help="grid side of the bounded sample the oracle runs for cpu_baseline")
    ap.add_argument("--kernel", default=None, help="kernel group for the roofline (default: the slowest)")
    ap.add_argument("--tuning", default=None,
                    help="dispatch thresholds for the run, e.g. 'trail_mfma=0,split_rows=512' (spaqr_tuning); "
                         "'table' applies the autotuned entry of the workload")
    ap.add_argument("--serving-requests", type=int, default=16,
                    help="requests of the serving trace replayed after the single-problem steps (0: skip)")
    ap.add_argument("--serving-load", type=float, default=0.7,
                    help="arrival rate of the serving trace as a fraction of the plain FP64 path's capacity")
    ap.add_argument("--serving-only", action="store_true",
                    help="run only the serving trace and print its record")
    ap.add_argument("--serving-calibration", type=float, default=None,
                    help="makespan (s) of the FP64 calibration pass of the same trace, measured before: "
                         "skips that pass")
    ap.add_argument("--serving-leg", choices=("both", "batched", "sequential"), default="both",
                    help="which replays of the serving trace to run")
    ap.add_argument("--rocprof-summary", metavar="DIR", default=None,
                    help="print a markdown summary of a rocprofv3 --kernel-trace --stats --output-format csv "
                         "directory of this script's run and exit (--fp32-steps: FP32 steps in that run)")
    ap.add_argument("--fp32-steps", type=int, default=None)
    ap.add_argument("--copy-calibration", metavar="BYTES", type=int, default=None,
                    help="only run a plain device-to-device copy of BYTES bytes three times (the reference "
                         "kernel for scaling the HBM counters) and exit")
    ap.add_argument("--pmc-summary", metavar="DIR", default=None,
                    help="from rocprofv3 --pmc runs in DIR/fetch and DIR/write (this script's run, counters "
                         "FETCH_SIZE and WRITE_SIZE) and DIR/cal_fetch and DIR/cal_write (--copy-calibration "
                         "runs), write the measured HBM traffic per launch of the --kernel group on "
                         "--workload under profiles/ and exit")
    return ap.parse_args()


# HBM traffic of a kernel group measured with rocprofv3 counters (see
# pmc_summary), one file per group and workload; reported only while
# kernels.hip is the source it was measured on
def traffic_file(group, workload):
    return os.path.join("profiles", f"{group}_{workload}_traffic.json")


KERNEL_SOURCE = os.path.join("paper_2010_06807_amd", "csrc", "kernels.hip")
CAL_BYTES = 1 << 30


def source_sha256():
    """SHA-256 over the device kernel sources (every .hip file beside
    KERNEL_SOURCE, names and contents, in name order)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for path in sorted(glob.glob(os.path.join(ROOT, os.path.dirname(KERNEL_SOURCE), "*.hip"))):
        h.update(os.path.basename(path).encode())
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def copy_calibration(nbytes):
    """A plain copy of nbytes (read nbytes, write nbytes), three times."""
    import torch
    a = torch.ones(nbytes, dtype=torch.uint8, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copied {nbytes} bytes three times")


def pmc_counters(d, counter, match):
    """Per-dispatch values (KiB) of one counter for the kernels whose name
    contains one of `match`, from a rocprofv3 --pmc CSV directory."""
    import csv
    import glob
    vals = {}
    for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(path)):
            if r.get("Counter_Name") != counter or not any(m in r.get("Kernel_Name", "") for m in match):
                continue
            key = (path, r.get("Dispatch_Id"))
            vals[key] = vals.get(key, 0.0) + float(r["Counter_Value"])
    return list(vals.values())


def pmc_summary(d, group="sparsify", workload="c4"):
    """Traffic per launch of one kernel group: FETCH_SIZE and WRITE_SIZE per
    dispatch, each scaled by the factor that makes the same counter read the
    known bytes of the calibration copy."""
    import statistics
    cal = CAL_BYTES / 1024.0
    cf = pmc_counters(os.path.join(d, "cal_fetch"), "FETCH_SIZE", ("copy", "Copy", "elementwise"))
    cw = pmc_counters(os.path.join(d, "cal_write"), "WRITE_SIZE", ("copy", "Copy", "elementwise"))
    if not cf or not cw or max(cf) <= 0 or max(cw) <= 0:
        raise SystemExit("pmc-summary: no calibration copy dispatch found")
    # the copies of the calibration buffer are the run's largest dispatches
    big_f = [v for v in cf if v >= 0.5 * max(cf)]
    big_w = [v for v in cw if v >= 0.5 * max(cw)]
    kf, kw = cal / statistics.median(big_f), cal / statistics.median(big_w)
    pats = GROUP_KERNELS[group]
    f = pmc_counters(os.path.join(d, "fetch"), "FETCH_SIZE", pats)
    w = pmc_counters(os.path.join(d, "write"), "WRITE_SIZE", pats)
    if not f or not w:
        raise SystemExit(f"pmc-summary: no {group} dispatch found")
    out = {"kernel": group, "workload": workload, "kernels": list(pats), "dispatches": [len(f), len(w)],
           "fetch_KiB_per_launch_raw": sum(f) / len(f), "write_KiB_per_launch_raw": sum(w) / len(w),
           "calibration_bytes": CAL_BYTES, "scale_fetch": kf, "scale_write": kw,
           "traffic_bytes_per_launch": 1024.0 * (kf * sum(f) / len(f) + kw * sum(w) / len(w)),
           "kernels_hip_sha256": source_sha256()}
    with open(os.path.join(ROOT, traffic_file(group, workload)), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def measured_traffic(group, workload):
    """Bytes per launch of a kernel group from the counter runs, or None when
    there are none or the kernels changed since."""
    try:
        with open(os.path.join(ROOT, traffic_file(group, workload))) as fh:
            t = json.load(fh)
        return t["traffic_bytes_per_launch"] if t.get("kernels_hip_sha256") == source_sha256() else None
    except (OSError, ValueError, KeyError):
        return None


def log(msg):
    """Progress on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def pct(v, q):
    v = sorted(v)
    if not v:
        return None
    i = min(len(v) - 1, max(0, int(math.ceil(q / 100.0 * len(v))) - 1))
    return v[i]


# kernel symbols behind each profiler group (FP32 instantiations)
GROUP_KERNELS = {
    "front_qr": ("k_qr_reg<float", "k_qr<float"),
    "trailing updates (fronts and scaling)": ("k_trail<float", "k_trail_mfma<float", "k_wy_tblock<float"),
    "block copies and zero fills": ("k_copy<float", "k_copy_t<float", "k_zero", "k_fill<float"),
    "descriptor uploads and readbacks": ("__amd_rocclr_copyBuffer", "k_gather_ints"),
    "interface operators (forming)": ("k_iface_form<float",),
    "scale_blocks": ("k_scale<float", "k_scale_small<float", "k_scale_right<float"),
    "sparsify": ("k_cpqr_dd", "k_cpqr_team", "k_cpqr_reg<float", "k_cpqr_coop<float", "k_sparsify_small<float", "k_sparsify<float"),
    "sparsify_unscaled": ("k_sparsify_unscaled<float",),
    "apply_front_fwd": ("k_ap_front_fwd_reg<float", "k_ap_front_fwd_wy<float"),
    "apply_front_bwd": ("k_ap_front_bwd_reg<float",),
    "apply_iface": ("k_ap_iface_dense<float", "k_ap_iface_dense_lat<float", "k_ap_iface_dense_big<float",
                    "k_ap_iface_fwd<float", "k_ap_iface_bwd<float"),
}


def rocprof_summary(d, fp32_steps):
    """Markdown summary of a rocprofv3 CSV directory: the kernel table and,
    per profiler group, the total kernel time per FP32 step."""
    import csv
    import glob
    stats = list(csv.DictReader(open(glob.glob(os.path.join(d, "*_kernel_stats.csv"))[0])))
    tot = sum(float(r["TotalDurationNs"]) for r in stats)
    out = ["| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:30]:
        name = r["Name"].replace("spaqr::(anonymous namespace)::", "").replace("void ", "")
        name = name.split("(spaqr::")[0].split("(double")[0].split("(long")[0]
        out.append(f"| `{name[:70]}` | {int(r['Calls'])} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {100 * float(r['TotalDurationNs']) / tot:.1f} |")
    out.append("")
    out.append(f"Per FP32 step ({fp32_steps} FP32 steps in the run):")
    out.append("")
    out.append("| group | kernels | ms per step |")
    out.append("|---|---|---|")
    for g, pats in GROUP_KERNELS.items():
        ms = sum(float(r["TotalDurationNs"]) for r in stats if any(p in r["Name"] for p in pats)) / 1e6
        n = sum(int(r["Calls"]) for r in stats if any(p in r["Name"] for p in pats))
        out.append(f"| {g} | {n} launches | {ms / fp32_steps:.3f} |")
    return "\n".join(out)


def serving(nreq, tol, load=1.0, seed=0, calibration=None, leg="both"):
    """The serving workload: the first nreq requests of the seeded trace
    (2D sides 64..512 or 3D sides 16..48, |beta| 1..200, 1..32 right-hand
    sides, eps 1e-2).  A calibration pass runs the plain FP64 path over the
    requests back to back (or `calibration` gives its makespan from an
    earlier run of the same trace); the arrival times are then scaled so that
    path would be busy a fraction `load` of the time (1.0: exactly
    saturated), and the trace is replayed through the batched FP32 server
    and through the sequential FP64 path on the same timestamps (`leg`
    selects one of the two).  Throughput counts unknowns x right-hand sides
    per second of makespan; latency runs from a request's arrival to its
    last solution."""
    import numpy as np
    import paper_2010_06807_amd as P
    from paper_2010_06807_amd.server import serve_trace, serve_sequential
    from problems.trace import serving_trace, build_request
    reqs = serving_trace(nreq, seed=seed)
    jobs = []
    for i, r in enumerate(reqs):
        q = build_request(r)
        jobs.append(dict(arrival=r["arrival"], A=q["A"], ordering=P.order_grid(q["dims"], q["levels"]), b=q["b"],
                         eps=r["eps"]))
        if (i + 1) % 32 == 0:
            log(f"serving: {i + 1} requests built")
    if calibration is None:
        log(f"serving: {len(jobs)} requests built; calibration pass (FP64, back to back)")
        _, cal = serve_sequential(jobs, tol=tol, precision=64, time_scale=0.0, log=log)
        calibration = cal["makespan_s"]
    log(f"serving: calibration {calibration:.1f} s")
    service = calibration / len(jobs)
    mean_gap = float(np.mean(np.diff([0.0] + [r["arrival"] for r in reqs])))
    scale = service / load / mean_gap
    out = {"requests": len(jobs), "unknowns_x_rhs": int(sum(j["A"].shape[0] * j["b"].shape[1] for j in jobs)),
           "arrival_rate_per_s": 1.0 / (mean_gap * scale), "load_fp64": load, "calibration_s": calibration,
           "unit": "unknowns*rhs/s"}
    worst = 0.0
    if leg in ("both", "batched"):
        res_b, batched = serve_trace(jobs, mem_budget=64 << 30, tol=tol, precision=32, time_scale=scale, log=log)
        log(f"serving: batched FP32 makespan {batched['makespan_s']:.1f} s")
        out["batched_fp32"] = {k: batched[k] for k in ("throughput", "p50_ms", "p99_ms", "makespan_s")}
        worst = max(worst, max(max(r["relres"]) for r in res_b))
    if leg in ("both", "sequential"):
        res_s, plain = serve_sequential(jobs, tol=tol, precision=64, time_scale=scale, log=log)
        log(f"serving: sequential FP64 makespan {plain['makespan_s']:.1f} s")
        out["plain_fp64"] = {k: plain[k] for k in ("throughput", "p50_ms", "p99_ms", "makespan_s")}
        worst = max(worst, max(max(r["relres"]) for r in res_s))
    out["max_relres"] = worst
    return out


def cpu_info():
    """CPU model (from /proc/cpuinfo) and the cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return model, avail


def cpu_baseline(workload, side, eps, tol):
    """The oracle, as it stands, on one host core, on a bounded sample of the
    workload: the same recipe (coefficients, flow, perturbation, eps) on a
    side x side grid, ordering + factor + FGMRES once."""
    from threadpoolctl import threadpool_limits
    import numpy as np
    from problems import make_rhs
    from problems.grids import convdiff, perturb_offdiagonals, default_levels
    from oracle.ordering import order_grid
    from oracle import spaqr as osq, gmres as ogm
    dims = (side, side)
    if workload == "c4":
        A = perturb_offdiagonals(convdiff(dims, (500.0, -300.0)), 0.05, 0.5, 1.5, np.random.default_rng(0))
        what = "1024^2 recipe (beta = (500, -300), 5% perturbed entries, seed 0)"
    elif workload == "c3":
        dims = (side, side, side)
        A = convdiff(dims, (20.0, 20.0, 20.0))
        what = "64^3 recipe (beta = (20, 20, 20))"
    else:
        from problems import config_problem
        prob = config_problem(workload, seed=0)
        A, dims = prob["A"], prob["dims"]
        what = f"{workload} workload, full size"
    N = A.shape[0]
    L = default_levels(N)
    b = make_rhs(N, 1, seed=0)[:, 0]
    model, avail = cpu_info()
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        o = order_grid(dims, L)
        F = osq.factor(A, o, eps)
        x, it, rel = ogm.fgmres(lambda v: A @ v, lambda v: osq.apply(F, v), b, tol)
        dt = time.perf_counter() - t0
    return {"value": N / dt, "unit": "unknowns/s", "cores": 1, "kind": "oracle",
            "sample": f"{what} on a {'x'.join(str(d) for d in dims)} grid (N={N}, {L} levels, eps={eps}): "
                      f"ordering + factor + FGMRES once on one core, {dt:.1f} s, {it} iterations, "
                      f"relres {rel:.1e}",
            "cpu_model": model, "host_cores_available": avail}


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.pmc_summary:
        pmc_summary(args.pmc_summary, args.kernel or "sparsify", args.workload)
        return
    if args.rocprof_summary:
        print(rocprof_summary(args.rocprof_summary, args.fp32_steps or 1))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported by this build "
              "(the nested-dissection tree would shard over GPUs, see the design notes)", file=sys.stderr)
        sys.exit(2)
    if args.serving_only:
        print(json.dumps(serving(args.serving_requests, args.tol, args.serving_load,
                                 calibration=args.serving_calibration, leg=args.serving_leg)), flush=True)
        return
    import numpy as np
    import torch
    import paper_2010_06807_amd as P
    from problems import config_problem, make_rhs

    tuning = None
    if args.tuning == "table":
        from paper_2010_06807_amd import autotune
        tuning = autotune.apply(args.workload)
    elif args.tuning:
        tuning = {k: int(v) for k, v in (kv.split("=") for kv in args.tuning.split(","))}
        P.set_tuning(**tuning)
    S = max(1, args.seeds)
    probs = [config_problem(args.workload, seed=i) for i in range(S)]
    prob = probs[0]
    A, dims, L = prob["A"], prob["dims"], prob["levels"]
    N = A.shape[0]
    for q in probs[1:]:
        assert np.array_equal(q["A"].indptr, A.indptr) and np.array_equal(q["A"].indices, A.indices)
    dev = torch.device("cuda:0")
    # ordering + symbolic analysis of the shared pattern, timed on their own
    t_an = []
    for _ in range(3):
        t0 = time.perf_counter()
        ordg = P.order_grid(dims, L)
        sym = P.analyze(A, ordg)
        t_an.append(time.perf_counter() - t0)
    t_analysis = min(t_an)
    dAs = [P.DeviceCSR(q["A"], dev) for q in probs]
    bs = [torch.from_numpy(make_rhs(N, 1, seed=i)).to(dev) for i in range(S)]
    torch.cuda.synchronize()

    def step(i, precision):
        """One problem: numeric factorization (values from HBM) + FGMRES."""
        t0 = time.perf_counter()
        fac = P.factor_device(probs[i % S]["A"], sym, dAs[i % S], eps=args.eps, precision=precision)
        t1 = time.perf_counter()
        x, info = fac.solve(bs[i % S], tol=args.tol)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return fac, x, info[0], t1 - t0, t2 - t1

    def run(precision, steps, warmup):
        for i in range(warmup):
            step(i, precision)
        torch.cuda.synchronize()
        lat, fac_t, sol_t, its, res = [], [], [], [], []
        t0 = time.perf_counter()
        for i in range(steps):
            s0 = time.perf_counter()
            fac, x, info, tf, ts = step(i, precision)
            lat.append(time.perf_counter() - s0)
            fac_t.append(tf)
            sol_t.append(ts)
            its.append(info["iterations"])
            res.append(info["relres"])
        dt = time.perf_counter() - t0
        return dict(dt=dt, lat=lat, fac_t=fac_t, sol_t=sol_t, its=its, res=res, fac=fac, x=x)

    log(f"{prob['name']}: N={N}, {L} levels, seeds 0..{S - 1}; analysis {1e3 * t_analysis:.1f} ms; survey step")
    # which kernel group dominates: one untimed step with every launch timed
    step(0, 32)
    P.profile_enable(True)
    step(0, 32)
    torch.cuda.synchronize()
    survey = {n: P.profile_query(n) for n in KERNEL_BOUND}
    P.profile_enable(False)
    kern = args.kernel or max(survey, key=lambda n: survey[n]["total_ms"])

    # timed region: FP32 factors + FP64 FGMRES, only the roofline kernel timed
    log(f"timed FP32 steps (roofline kernel: {kern})")
    P.profile_enable(True, only=kern)
    r32 = run(32, args.steps, args.warmup)
    prof = P.profile_query(kern)
    P.profile_enable(False)
    log(f"FP32: {1e3 * r32['dt'] / args.steps:.2f} ms/step")
    # true residuals of the timed steps' last solution, recomputed on the host
    i_last = args.steps - 1
    bb = bs[i_last % S].cpu().numpy()[:, 0]
    res_host = float(np.linalg.norm(probs[i_last % S]["A"] @ r32["x"].cpu().numpy()[:, 0] - bb) / np.linalg.norm(bb))
    st = r32["fac"].stats()
    value = N * args.steps / r32["dt"]
    ms_step = 1e3 * r32["dt"] / args.steps

    plain64 = None
    if args.fp64_steps > 0:
        r64 = run(64, args.fp64_steps, 1)
        log(f"FP64 plain: {1e3 * r64['dt'] / args.fp64_steps:.2f} ms/step")
        plain64 = {"value": N * args.fp64_steps / r64["dt"], "ms_per_step": 1e3 * r64["dt"] / args.fp64_steps,
                   "latency_ms": {"p50": 1e3 * pct(r64["lat"], 50), "p99": 1e3 * pct(r64["lat"], 99)},
                   "gmres_iterations": max(r64["its"]), "relres": max(r64["res"]),
                   "ms_factor": 1e3 * float(np.mean(r64["fac_t"])), "ms_solve": 1e3 * float(np.mean(r64["sol_t"]))}

    def rate(bound, q):
        """(achieved, peak, unit) of one profiler record under its bound."""
        if bound == "hbm":
            peak, unit = PEAK["hbm"]
            return (q["bytes"] / (q["total_ms"] * 1e-3) / 1e9 if q["total_ms"] > 0 else 0.0), peak, unit
        peak, unit = PEAK[{"mfma": "mfma32", "alu64": "alu64"}.get(bound, "alu32")]
        return (q["flops"] / (q["total_ms"] * 1e-3) / 1e12 if q["total_ms"] > 0 else 0.0), peak, unit

    unscaled = None
    if args.unscaled_steps > 0:
        # the sparsification without scaling (Section 2.5) on its own workload
        uprobs = [config_problem(args.unscaled_workload, seed=i) for i in range(S)]
        uN = uprobs[0]["A"].shape[0]
        usym = P.analyze(uprobs[0]["A"], P.order_grid(uprobs[0]["dims"], uprobs[0]["levels"]))
        udA = [P.DeviceCSR(q["A"], dev) for q in uprobs]
        ub = [torch.from_numpy(make_rhs(uN, 1, seed=i)).to(dev) for i in range(S)]

        def ustep(i):
            t0 = time.perf_counter()
            fac = P.factor_device(uprobs[i % S]["A"], usym, udA[i % S], eps=args.eps, precision=32, scale=False)
            t1 = time.perf_counter()
            x, info = fac.solve(ub[i % S], tol=args.tol)
            torch.cuda.synchronize()
            return info[0], t1 - t0, time.perf_counter() - t1

        ustep(0)
        torch.cuda.synchronize()
        log("FP32 factors without scaling")
        P.profile_enable(True, only="sparsify_unscaled")
        uf, us, uit, ures = [], [], [], []
        t0 = time.perf_counter()
        for i in range(args.unscaled_steps):
            info, tf, ts = ustep(i)
            uf.append(tf)
            us.append(ts)
            uit.append(info["iterations"])
            ures.append(info["relres"])
        dtu = time.perf_counter() - t0
        qu = P.profile_query("sparsify_unscaled")
        P.profile_enable(False)
        ach, pk, un = rate("alu64", qu)
        log(f"without scaling: {1e3 * dtu / args.unscaled_steps:.2f} ms/step")
        unscaled = {"workload": f"{uprobs[0]['name']} (N={uN}), eps={args.eps}, FP32 factors without scaling "
                                f"+ FP64 FGMRES to {args.tol}, seeds 0..{S - 1} in turn",
                    "value": uN * args.unscaled_steps / dtu, "unit": "unknowns/s",
                    "ms_per_step": 1e3 * dtu / args.unscaled_steps,
                    "ms_factor": 1e3 * float(np.mean(uf)), "ms_solve": 1e3 * float(np.mean(us)),
                    "gmres_iterations": max(uit), "relres": max(ures),
                    "sparsify_kernel": {"kernel": "k_sparsify_unscaled", "bound": "alu64", "achieved": ach,
                                        "peak": pk, "unit": un, "frac": ach / pk,
                                        "ms_per_step": qu["total_ms"] / args.unscaled_steps,
                                        "launches_per_step": qu["launches"] / args.unscaled_steps,
                                        "avg_launch_us": 1e3 * qu["total_ms"] / max(1, qu["launches"]),
                                        "flops_per_step": qu["flops"] / args.unscaled_steps}}

    graph = None
    if args.graph_points > 0 and args.graph_steps > 0:
        # a matrix without a grid: convection-diffusion on a Delaunay mesh,
        # ordered by the algebraic MND (ordering and analysis timed apart)
        from problems.unstructured import delaunay_convdiff
        log(f"unstructured leg: Delaunay mesh of {args.graph_points} points")
        gA = [delaunay_convdiff(args.graph_points, seed=i) for i in range(min(S, 1))]
        gN = gA[0].shape[0]
        t0 = time.perf_counter()
        gord = P.order_graph(gA[0])
        t1 = time.perf_counter()
        gsym = P.analyze(gA[0], gord)
        t2 = time.perf_counter()
        gdA = P.DeviceCSR(gA[0], dev)
        gb = torch.from_numpy(make_rhs(gN, 1, seed=0)).to(dev)

        def gstep():
            s0 = time.perf_counter()
            fac = P.factor_device(gA[0], gsym, gdA, eps=args.eps, precision=32)
            s1 = time.perf_counter()
            x, info = fac.solve(gb, tol=args.tol)
            torch.cuda.synchronize()
            return info[0], s1 - s0, time.perf_counter() - s1

        gstep()
        torch.cuda.synchronize()
        gf, gs, git, gres = [], [], [], []
        t3 = time.perf_counter()
        for _ in range(args.graph_steps):
            info, tf, ts = gstep()
            gf.append(tf)
            gs.append(ts)
            git.append(info["iterations"])
            gres.append(info["relres"])
        dtg = time.perf_counter() - t3
        log(f"unstructured: {1e3 * dtg / args.graph_steps:.2f} ms/step")
        graph = {"workload": f"convection-diffusion on the Delaunay mesh of {args.graph_points} uniform random "
                             f"points (seed 0), eps={args.eps}, algebraic MND ({gord.levels} levels), FP32 factors + "
                             f"FP64 FGMRES to {args.tol}",
                 "value": gN * args.graph_steps / dtg, "unit": "unknowns/s",
                 "ms_per_step": 1e3 * dtg / args.graph_steps,
                 "ms_factor": 1e3 * float(np.mean(gf)), "ms_solve": 1e3 * float(np.mean(gs)),
                 "gmres_iterations": max(git), "relres": max(gres),
                 "ms_ordering": 1e3 * (t1 - t0), "ms_analysis": 1e3 * (t2 - t1), "nnz": int(gA[0].nnz)}

    bound = KERNEL_BOUND[kern]
    achieved, peak, unit = rate(bound, prof)
    nsteps = args.steps + args.warmup
    roof = {"bound": bound, "kernel": kern, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "traffic": measured_traffic(kern, args.workload),
            "launches": prof["launches"], "avg_launch_us": 1e3 * prof["total_ms"] / max(1, prof["launches"]),
            "ms_per_step": prof["total_ms"] / nsteps,
            "work_per_step": (prof["bytes"] if bound == "hbm" else prof["flops"]) / nsteps,
            "work_per_launch": (prof["bytes"] if bound == "hbm" else prof["flops"]) / max(1, prof["launches"]),
            "survey_ms": {n: round(v["total_ms"], 3) for n, v in survey.items() if v["launches"]},
            # every group of the survey step: time, work and the rate against its bound's peak
            "survey": {n: dict(zip(("achieved", "peak", "unit"), rate(KERNEL_BOUND[n], v)), ms=v["total_ms"],
                               launches=v["launches"], bound=KERNEL_BOUND[n])
                       for n, v in survey.items() if v["launches"]}}
    # achieved HBM rate of the apply and scaling phases in the survey step
    # (algorithmic bytes of the launches / their event time)
    phases = {}
    for name, groups in (("apply", ("apply_front_fwd", "apply_front_bwd", "apply_iface_fwd", "apply_iface_bwd")),
                         ("scale_blocks", ("scale_blocks",))):
        by = sum(survey[g]["bytes"] for g in groups)
        ms = sum(survey[g]["total_ms"] for g in groups)
        if ms > 0:
            phases[name] = {"GB_per_s": by / (ms * 1e-3) / 1e9, "frac_hbm": by / (ms * 1e-3) / 1e9 / PEAK["hbm"][0],
                            "ms_per_step": ms, "bytes_per_step": by}
    roof["phases_hbm"] = phases

    out = {
        "metric": METRIC, "value": value, "unit": "unknowns/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{prob['name']}: {WORKLOAD_TEXT.get(prob['name'], 'convection-diffusion')} "
                               f"{'x'.join(str(d) for d in dims)} (N={N}), eps={args.eps}, "
                               f"{L} ND levels, FP32 factors + FP64 FGMRES to {args.tol}, 1 RHS, one problem per "
                               f"step (seeds 0..{S - 1} in turn), analysis of the shared pattern made once",
                   "eps": args.eps, "levels": L, "n": N, "tuning": tuning},
        "latency_ms": {"p50": 1e3 * pct(r32["lat"], 50), "p99": 1e3 * pct(r32["lat"], 99)},
        "phase_ms": {"factor": 1e3 * float(np.mean(r32["fac_t"])), "solve": 1e3 * float(np.mean(r32["sol_t"])),
                     "order_and_analysis": 1e3 * t_analysis},
        "end_to_end": {"value": N / (r32["dt"] / args.steps + t_analysis),
                       "note": "ordering + symbolic analysis included in every step"},
        "gmres_iterations": max(r32["its"]), "relres": max(max(r32["res"]), res_host),
        "fp64_plain": plain64,
        "unscaled": unscaled,
        "unstructured": graph,
        "factor": {"ms_factor": st["ms_factor"], "factor_bytes": st["factor_bytes"],
                   "top_separator": st["top_separator"], "flops_sparsify": st["flops_sparsify"]},
        "roofline": roof,
    }
    if args.batch_workload:
        out["batched_requests"] = batched_figure(args.batch_workload, args.batch, args.batch_steps, args.eps,
                                                 args.tol)
    if args.serving_requests > 0:
        out["serving"] = serving(args.serving_requests, args.tol, args.serving_load)
    if not args.no_cpu_baseline:
        log("oracle on the host (cpu_baseline)")
        out["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_side, args.eps, args.tol)
    print(json.dumps(out), flush=True)


def batched_figure(workload, B, steps, eps, tol, warmup=2):
    """Cross-request batching: steps of B requests of `workload` (seeds
    0..B-1) factored together stage by stage and solved with one FGMRES,
    batches back to back as a server runs them (the host analyses of batch
    i + 1 overlap batch i's solve, inside the timed region)."""
    import torch
    import paper_2010_06807_amd as P
    from problems import config_problem, make_rhs
    from concurrent.futures import ThreadPoolExecutor
    probs = [config_problem(workload, seed=i) for i in range(B)]
    dims, L = probs[0]["dims"], probs[0]["levels"]
    N = probs[0]["A"].shape[0]
    dev = torch.device("cuda:0")
    dAs = [P.DeviceCSR(p["A"], dev) for p in probs]
    bs = [torch.from_numpy(make_rhs(N, 1, seed=i)).to(dev) for i in range(B)]
    torch.cuda.synchronize()
    pool = ThreadPoolExecutor(max_workers=min(B, 16))

    def host_prep(i):
        return P.analyze(probs[i]["A"], P.order_grid(dims, L))

    def step(prep, next_prep):
        syms = [f.result() for f in prep]
        facs = P.factor_batch([p["A"] for p in probs], syms, dAs, eps=eps, precision=32)
        nxt = [pool.submit(host_prep, i) for i in range(B)] if next_prep else None
        xs, infos = P.solve_batch(facs, bs, tol=tol)
        return xs, infos, nxt

    log(f"batched {workload}: {B} requests per step")
    for _ in range(warmup):
        step([pool.submit(host_prep, i) for i in range(B)], False)
    torch.cuda.synchronize()
    lat, its = [], 0
    t0 = time.perf_counter()
    start = time.perf_counter()
    prep = [pool.submit(host_prep, i) for i in range(B)]
    for i in range(steps):
        last = i + 1 == steps
        xs, infos, nxt = step(prep, not last)
        torch.cuda.synchronize()
        now = time.perf_counter()
        lat.append(now - start)
        its = max(its, max(inf[0]["iterations"] for inf in infos))
        start, prep = now, nxt
    dt = time.perf_counter() - t0
    pool.shutdown()
    log(f"batched {workload}: {1e3 * dt / steps:.2f} ms/step")
    return {"workload": f"{workload}, {'x'.join(str(d) for d in dims)} (N={N}), {B} requests per step batched "
                        f"(seeds 0..{B - 1}), FP32 factors + FP64 FGMRES, host analyses inside the timed region",
            "value": B * N * steps / dt, "unit": "unknowns/s", "ms_per_step": 1e3 * dt / steps,
            "latency_ms": {"p50": 1e3 * pct(lat, 50), "p99": 1e3 * pct(lat, 99)}, "gmres_iterations": its}


if __name__ == "__main__":
    main()
