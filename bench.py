#!/usr/bin/env python3
"""spaQR on one MI355X: unknowns/s for one pass of the whole hot path.

A step serves a batch of B requests of the 256 x 256 variable-coefficient
convection-diffusion workload (N = 65,536 each, eps = 1e-2, 10 levels; the
requests differ in their seeded coefficient field and flow direction): per
request grid ordering + symbolic analysis (host, in parallel threads), then
the numeric factorizations of all B advanced together stage by stage (FP32
blocks and factors, one launch per phase for the whole batch), then FGMRES in
FP64 to ||Ax - b|| / ||b|| <= 1e-10 for all B together (one launch per apply
phase for the whole batch).  Batches run back to back as a server runs them:
the host analyses of batch i + 1 proceed while batch i solves on the GPU
(every analysis of the timed batches is inside the timed region).  A's CSR and b
are resident in HBM when the timed region starts; the factorization reads
the values from device memory and the host sees only the pattern.

Printed as one JSON line: batched throughput (value), the same path one
request at a time, the plain FP64 GPU path one request at a time, per-step
latency percentiles, the roofline of the dominant kernel (HIP events around
its launches during the timed region), a replayed serving trace and the
oracle timed on one host core on the same workload.
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

# Published MI355X peaks used for the roofline fractions.
PEAK = {
    "hbm": (8000.0, "GB/s"),
    "alu32": (157.3, "TFLOP/s"),
    "alu64": (78.6, "TFLOP/s"),
}
# bound of each kernel: HBM-bound data movement / apply, or vector-ALU
# arithmetic (the factorization kernels run on the VALU, not on MFMA; the
# CPQR's work is counted from the ranks read back after each stage)
KERNEL_BOUND = {
    "front_qr": "alu", "front_trail": "alu", "scale_qr": "alu", "scale_blocks": "alu", "sparsify": "alu",
    "apply_front_fwd": "hbm", "apply_front_bwd": "hbm", "apply_iface_fwd": "hbm", "apply_iface_bwd": "hbm",
}


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--eps", type=float, default=1e-2)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--batch", type=int, default=16, help="requests per step (cross-request batching)")
    ap.add_argument("--single-steps", type=int, default=5, help="steps of the one-request-at-a-time FP32 path")
    ap.add_argument("--fp64-steps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel", default=None, help="kernel for the roofline (default: the slowest)")
    ap.add_argument("--serving-requests", type=int, default=16,
                    help="requests of the serving trace replayed after the single-problem steps (0: skip)")
    ap.add_argument("--serving-load", type=float, default=1.0,
                    help="arrival rate of the serving trace as a fraction of the plain FP64 path's capacity")
    ap.add_argument("--rocprof-summary", metavar="DIR", default=None,
                    help="print a markdown summary of a rocprofv3 --kernel-trace --stats --output-format csv "
                         "directory of this script's run and exit")
    ap.add_argument("--copy-calibration", metavar="BYTES", type=int, default=None,
                    help="only run a plain device-to-device copy of BYTES bytes three times (the reference "
                         "kernel for scaling the HBM counters) and exit")
    ap.add_argument("--pmc-summary", metavar="DIR", default=None,
                    help="from rocprofv3 --pmc runs in DIR/fetch and DIR/write (this script's run, counters "
                         "FETCH_SIZE and WRITE_SIZE) and DIR/cal_fetch and DIR/cal_write (--copy-calibration "
                         "runs), write the measured HBM traffic per launch of the roofline kernel to "
                         f"{TRAFFIC_FILE} and exit")
    return ap.parse_args()


# HBM traffic of the roofline kernel measured with rocprofv3 counters (see
# pmc_summary); reported only while kernels.hip is the source it was measured on
TRAFFIC_FILE = os.path.join("profiles", "sparsify_c2_256x256_traffic.json")
KERNEL_SOURCE = os.path.join("paper_2010_06807_amd", "csrc", "kernels.hip")
CAL_BYTES = 1 << 30


def source_sha256():
    import hashlib
    with open(os.path.join(ROOT, KERNEL_SOURCE), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


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


def pmc_summary(d):
    """Traffic per launch of the sparsification kernels: FETCH_SIZE and
    WRITE_SIZE per dispatch, each scaled by the factor that makes the same
    counter read the known bytes of the calibration copy."""
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
    pats = GROUP_KERNELS["sparsify"]
    f = pmc_counters(os.path.join(d, "fetch"), "FETCH_SIZE", pats)
    w = pmc_counters(os.path.join(d, "write"), "WRITE_SIZE", pats)
    if not f or not w:
        raise SystemExit("pmc-summary: no sparsification dispatch found")
    out = {"kernel": "sparsify", "kernels": list(pats), "dispatches": [len(f), len(w)],
           "fetch_KiB_per_launch_raw": sum(f) / len(f), "write_KiB_per_launch_raw": sum(w) / len(w),
           "calibration_bytes": CAL_BYTES, "scale_fetch": kf, "scale_write": kw,
           "traffic_bytes_per_launch": 1024.0 * (kf * sum(f) / len(f) + kw * sum(w) / len(w)),
           "kernels_hip_sha256": source_sha256()}
    with open(os.path.join(ROOT, TRAFFIC_FILE), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def measured_traffic():
    """Bytes per launch of the roofline kernel from the counter runs, or None
    when there are none or the kernels changed since."""
    try:
        with open(os.path.join(ROOT, TRAFFIC_FILE)) as fh:
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
    "trailing updates (fronts and scaling)": ("k_trail<float",),
    "block copies and zero fills": ("k_copy<float", "k_copy_t<float", "k_zero", "k_fill<float"),
    "descriptor uploads and readbacks": ("__amd_rocclr_copyBuffer", "k_gather_ints"),
    "interface operators (forming)": ("k_iface_form<float",),
    "scale_blocks": ("k_scale<float", "k_scale_small<float", "k_scale_right<float"),
    "sparsify": ("k_cpqr_reg<float", "k_cpqr_coop<float", "k_sparsify_small<float", "k_sparsify<float"),
    "apply_front_fwd": ("k_ap_front_fwd_reg<float", "k_ap_front_fwd_wy<float"),
    "apply_front_bwd": ("k_ap_front_bwd_reg<float",),
    "apply_iface": ("k_ap_iface_dense<float", "k_ap_iface_fwd<float", "k_ap_iface_bwd<float"),
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


def serving(nreq, tol, load=1.0, seed=0):
    """The serving workload: the first nreq requests of the seeded trace
    (2D sides 64..512 or 3D sides 16..48, |beta| 1..200, 1..32 right-hand
    sides, eps 1e-2).  A calibration pass runs the plain FP64 path over the
    requests back to back; the arrival times are then scaled so that path
    would be busy a fraction `load` of the time (1.0: exactly saturated), and
    the trace is replayed through the
    batched FP32 server and through the sequential FP64 path on the same
    timestamps.  Throughput counts unknowns x right-hand sides per second of
    makespan; latency runs from a request's arrival to its last solution."""
    import numpy as np
    import paper_2010_06807_amd as P
    from paper_2010_06807_amd.server import serve_trace, serve_sequential
    from problems.trace import serving_trace, build_request
    reqs = serving_trace(nreq, seed=seed)
    jobs = []
    for r in reqs:
        q = build_request(r)
        jobs.append(dict(arrival=r["arrival"], A=q["A"], ordering=P.order_grid(q["dims"], q["levels"]), b=q["b"],
                         eps=r["eps"]))
    log(f"serving: {len(jobs)} requests built; calibration pass (FP64, back to back)")
    _, cal = serve_sequential(jobs, tol=tol, precision=64, time_scale=0.0, log=log)
    log(f"serving: calibration {cal['makespan_s']:.1f} s")
    service = cal["makespan_s"] / len(jobs)
    mean_gap = float(np.mean(np.diff([0.0] + [r["arrival"] for r in reqs])))
    scale = service / load / mean_gap
    res_b, batched = serve_trace(jobs, mem_budget=64 << 30, tol=tol, precision=32, time_scale=scale, log=log)
    log(f"serving: batched FP32 makespan {batched['makespan_s']:.1f} s")
    res_s, plain = serve_sequential(jobs, tol=tol, precision=64, time_scale=scale, log=log)
    log(f"serving: sequential FP64 makespan {plain['makespan_s']:.1f} s")
    worst = max(max(r["relres"]) for r in res_b + res_s)
    return {"requests": len(jobs), "unknowns_x_rhs": int(sum(j["A"].shape[0] * j["b"].shape[1] for j in jobs)),
            "arrival_rate_per_s": 1.0 / (mean_gap * scale), "load_fp64": load,
            "batched_fp32": {k: batched[k] for k in ("throughput", "p50_ms", "p99_ms", "makespan_s")},
            "plain_fp64": {k: plain[k] for k in ("throughput", "p50_ms", "p99_ms", "makespan_s")},
            "max_relres": worst, "unit": "unknowns*rhs/s"}


def cpu_baseline(prob, eps, tol):
    """The oracle, as it stands, on one host core: factor + FGMRES on the same
    workload (one full problem)."""
    from threadpoolctl import threadpool_limits
    import numpy as np
    from problems import make_rhs
    from oracle.ordering import order_grid
    from oracle import spaqr as osq, gmres as ogm
    A, dims, L = prob["A"], prob["dims"], prob["levels"]
    N = A.shape[0]
    b = make_rhs(N, 1, seed=0)[:, 0]
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        o = order_grid(dims, L)
        F = osq.factor(A, o, eps)
        x, it, rel = ogm.fgmres(lambda v: A @ v, lambda v: osq.apply(F, v), b, tol)
        dt = time.perf_counter() - t0
    return {"value": N / dt, "unit": "unknowns/s", "cores": 1, "kind": "oracle",
            "sample": f"{prob['name']} full problem (N={N}), ordering+factor+FGMRES once, "
                      f"{dt:.1f} s, {it} iterations, relres {rel:.1e}"}


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.pmc_summary:
        pmc_summary(args.pmc_summary)
        return
    if args.rocprof_summary:
        # FP32 steps of a run: 2 survey steps, the warmup and the timed steps
        print(rocprof_summary(args.rocprof_summary, 2 + args.warmup + args.steps))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported by this build "
              "(the nested-dissection tree would shard over GPUs, see the design notes)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_2010_06807_amd as P
    from problems import config_problem, make_rhs

    from concurrent.futures import ThreadPoolExecutor

    B = max(1, args.batch)
    probs = [config_problem(args.workload, seed=i) for i in range(B)]
    prob = probs[0]
    A, dims, L = prob["A"], prob["dims"], prob["levels"]
    N = A.shape[0]
    dev = torch.device("cuda:0")
    dAs = [P.DeviceCSR(p["A"], dev) for p in probs]
    bs = [torch.from_numpy(make_rhs(N, 1, seed=i)).to(dev) for i in range(B)]
    torch.cuda.synchronize()
    # one analysis per host core (16 per GPU), so that a batch's analyses
    # fit in the previous batch's solve
    pool = ThreadPoolExecutor(max_workers=min(B, 16))

    phases = {"host_order_analyze": [], "factor": [], "solve": []}

    def host_prep(i):
        t0 = time.perf_counter()
        o = P.order_grid(dims, L)
        t1 = time.perf_counter()
        sym = P.analyze(probs[i]["A"], o)
        return sym, t1 - t0, time.perf_counter() - t1

    def prep_batch():
        """Ordering + analysis of every request of a batch, in the host threads."""
        return [pool.submit(host_prep, i) for i in range(B)]

    def step_batch(precision, record=False, prep=None, next_prep=False):
        """One batch of B requests: ordering + analysis per request (threads),
        batched factorization, batched FGMRES.  prep: the batch's analyses
        already under way (started while the previous batch was on the GPU);
        next_prep: start the next batch's analyses before this one's solve
        (returned as the fourth value, with their start time)."""
        t0 = time.perf_counter()
        futs = prep if prep is not None else prep_batch()
        syms = [f.result()[0] for f in futs]
        t1 = time.perf_counter()
        facs = P.factor_batch([p["A"] for p in probs], syms, dAs, eps=args.eps, precision=precision)
        t2 = time.perf_counter()
        # the next batch's analyses overlap this batch's solve (the FGMRES
        # loop leaves the host cores idle, the factorization's planning does
        # not); started earlier they would add a step to every latency
        nxt = (prep_batch(), time.perf_counter()) if next_prep else None
        xs, infos = P.solve_batch(facs, bs, tol=args.tol)
        t3 = time.perf_counter()
        if record:
            phases["host_order_analyze"].append(t1 - t0)
            phases["factor"].append(t2 - t1)
            phases["solve"].append(t3 - t2)
        if next_prep:
            return facs, xs, [inf[0] for inf in infos], nxt
        return facs, xs, [inf[0] for inf in infos]

    def run_pipelined(precision, steps, warmup):
        """Batches back to back, as a server runs them: the host analyses of
        batch i + 1 run while batch i solves on the GPU.  Every
        analysis of the timed batches happens inside the timed region; a
        batch's latency runs from the start of its analyses to its solution."""
        for _ in range(warmup):
            step_batch(precision)
        torch.cuda.synchronize()
        lat, infos = [], []
        t0 = time.perf_counter()
        start = time.perf_counter()
        prep = prep_batch()
        for i in range(steps):
            last = i + 1 == steps
            out = step_batch(precision, record=True, prep=prep, next_prep=not last)
            facs, xs, inf = out[:3]
            torch.cuda.synchronize()
            now = time.perf_counter()
            lat.append(now - start)
            infos.append(inf)
            if not last:
                prep, start = out[3]
        dt = time.perf_counter() - t0
        return dt, lat, infos, facs, xs

    def step_one(precision, i=0):
        """One request alone: ordering, analysis, factorization, FGMRES."""
        ordg = P.order_grid(dims, L)
        sym = P.analyze(probs[i]["A"], ordg)
        fac = P.factor_device(probs[i]["A"], sym, dAs[i], eps=args.eps, precision=precision)
        x, info = fac.solve(bs[i], tol=args.tol)
        return [fac], [x], [info[0]]

    def run(fn, precision, steps, warmup, record=False):
        for _ in range(warmup):
            fn(precision)
        torch.cuda.synchronize()
        lat, infos = [], []
        t0 = time.perf_counter()
        for _ in range(steps):
            s0 = time.perf_counter()
            facs, xs, inf = fn(precision, record=True) if record else fn(precision)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - s0)
            infos.append(inf)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return dt, lat, infos, facs, xs

    log(f"{prob['name']}: N={N}, {L} levels, batch {B}; survey step")
    # which kernel dominates: one untimed step with every launch timed
    step_batch(32)
    P.profile_enable(True)
    step_batch(32)
    torch.cuda.synchronize()
    names = list(KERNEL_BOUND)
    survey = {n: P.profile_query(n) for n in names}
    P.profile_enable(False)
    kern = args.kernel or max(survey, key=lambda n: survey[n]["total_ms"])

    # timed region: batches of B requests, FP32 factors + FP64 GMRES, only the
    # roofline kernel timed
    log(f"timed FP32 batched steps (roofline kernel: {kern})")
    P.profile_enable(True, only=kern)
    dt, lat, infos, facs, xs = run_pipelined(32, args.steps, args.warmup)
    log(f"FP32 batch of {B}: {1e3 * dt / args.steps:.2f} ms/step")
    prof = P.profile_query(kern)
    P.profile_enable(False)
    res = 0.0
    for p, b, x in zip(probs, bs, xs):
        bb = b.cpu().numpy()[:, 0]
        res = max(res, float(np.linalg.norm(p["A"] @ x.cpu().numpy()[:, 0] - bb) / np.linalg.norm(bb)))
    st = facs[0].stats()
    value = B * N * args.steps / dt

    def single(precision, steps, what):
        """The path one request at a time (None when steps == 0)."""
        if steps <= 0:
            return None
        dt1, lat1, infos1, _, _ = run(step_one, precision, steps, 1)
        log(f"{what}: {1e3 * dt1 / steps:.2f} ms/step")
        return {"value": N * steps / dt1, "ms_per_step": 1e3 * dt1 / steps,
                "latency_ms": {"p50": 1e3 * pct(lat1, 50), "p99": 1e3 * pct(lat1, 99)},
                "gmres_iterations": infos1[-1][0]["iterations"]}

    one32 = single(32, args.single_steps, "FP32 one request")
    plain64 = single(64, args.fp64_steps, "FP64 plain")

    bound = KERNEL_BOUND[kern]
    if bound == "hbm":
        peak, unit = PEAK["hbm"]
        achieved = prof["bytes"] / (prof["total_ms"] * 1e-3) / 1e9 if prof["total_ms"] > 0 else 0.0
    else:
        peak, unit = PEAK["alu32"]
        achieved = prof["flops"] / (prof["total_ms"] * 1e-3) / 1e12 if prof["total_ms"] > 0 else 0.0
    roof = {"bound": bound, "kernel": kern, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "traffic": measured_traffic() if kern == "sparsify" else None,
            "launches": prof["launches"], "avg_launch_us": 1e3 * prof["total_ms"] / max(1, prof["launches"]),
            "ms_per_step": prof["total_ms"] / (args.steps + args.warmup),
            "work_per_step": (prof["bytes"] if bound == "hbm" else prof["flops"]) / (args.steps + args.warmup),
            "survey_ms": {n: round(v["total_ms"], 3) for n, v in survey.items() if v["launches"]}}

    out = {
        "metric": METRIC, "value": value, "unit": "unknowns/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{prob['name']}: {WORKLOAD_TEXT.get(prob['name'], 'convection-diffusion')} "
                               f"{'x'.join(str(d) for d in dims)} (N={N}), eps={args.eps}, "
                               f"{L} ND levels, FP32 factors + FP64 FGMRES to {args.tol}, 1 RHS per request, "
                               f"{B} requests per step batched (seeds 0..{B - 1})",
                   "eps": args.eps, "levels": L, "n": N, "batch": B},
        "latency_ms": {"p50": 1e3 * pct(lat, 50), "p99": 1e3 * pct(lat, 99)},
        "gmres_iterations": max(i["iterations"] for i in infos[-1]), "relres": res,
        "phase_ms": {k: round(1e3 * sum(v) / max(1, len(v)), 3) for k, v in phases.items()},
        "fp32_one_request": one32,
        "fp64_plain": plain64,
        "factor": {"ms_symbolic_host": st["ms_symbolic"], "ms_factor": st["ms_factor"],
                   "factor_bytes": st["factor_bytes"], "top_separator": st["top_separator"]},
        "roofline": roof,
    }
    if args.serving_requests > 0:
        out["serving"] = serving(args.serving_requests, args.tol, args.serving_load)
    if not args.no_cpu_baseline:
        log("oracle on the host (cpu_baseline)")
        out["cpu_baseline"] = cpu_baseline(prob, args.eps, args.tol)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
