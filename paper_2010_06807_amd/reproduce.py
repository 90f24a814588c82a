"""Reproduction runs of the paper's own advection-diffusion experiments.

The problems of Section 4 (centered differences, problems/paper_ad.py) are
factored on the GPU in FP64 (the paper's precision) with the same
tolerances and solved by FGMRES to ||Ax - b|| / ||b|| <= 1e-12 (the paper's
stopping rule), and the GMRES iteration counts and factorization times are
printed beside the counts the paper reports:

  ad2_q    2D, a = 1, b = 1, q in {1, 25, 1000}, eps = 1e-2, n = 128..1024
           (Fig. ad_figure)
  ad2_eps  2D, a = 1, b = e^{x+y}, q = 1000, eps in {1e-1, 1e-2, 1e-4},
           n = 128..1024 (Fig. ad_eps)
  ad3      3D, a = b = q = 1, eps in {1e-1, 1e-2}, n = 64, 80, 96
           (Fig. 3d_ad)
  hc       2D high contrast rho in {1, 10, 100}, b = q = 1, eps = 1e-2,
           n = 128..512 (Section 4.1.1's problem with scaling only)
  hc_abl   the comparison of Section 4.1.1 (Fig. hc_ad_comparison): the
           high-contrast problem with rho in {1, 10, 100} at eps in
           {1e-3, 1e-5}, n = 127..1023, with and without scaling

The partition differs from the paper's (its code is not public: this
library's geometric nested dissection with two-layer separators), so the
counts are a trend comparison, not parity.  Right-hand sides are U[-1, 1]
from seed 0.

    python -m paper_2010_06807_amd.reproduce [ad2_q ad2_eps ad3 hc hc_abl] [--max-n 1024] [--json out.json]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))

# GMRES counts printed in the paper (Section 4.2), keyed by (series, n)
PAPER = {
    ("q=1", 128): 9, ("q=1", 256): 11, ("q=1", 512): 14, ("q=1", 1024): 17, ("q=1", 2048): 23,
    ("q=25", 128): 8, ("q=25", 256): 9, ("q=25", 512): 11, ("q=25", 1024): 13, ("q=25", 2048): 16,
    ("q=1000", 128): 8, ("q=1000", 256): 9, ("q=1000", 512): 9, ("q=1000", 1024): 11, ("q=1000", 2048): 13,
    ("eps=1e-1", 128): 14, ("eps=1e-1", 256): 16, ("eps=1e-1", 512): 23, ("eps=1e-1", 1024): 33,
    ("eps=1e-1", 2048): 44,
    ("eps=1e-2", 128): 7, ("eps=1e-2", 256): 9, ("eps=1e-2", 512): 9, ("eps=1e-2", 1024): 10, ("eps=1e-2", 2048): 11,
    ("eps=1e-4", 128): 4, ("eps=1e-4", 256): 4, ("eps=1e-4", 512): 4, ("eps=1e-4", 1024): 4, ("eps=1e-4", 2048): 4,
    ("3d eps=1e-1", 64): 68, ("3d eps=1e-1", 80): 87, ("3d eps=1e-1", 96): 102,
    ("3d eps=1e-2", 64): 12, ("3d eps=1e-2", 80): 14, ("3d eps=1e-2", 96): 14,
}


# GMRES counts of Fig. hc_ad_comparison, keyed by (rho, eps, scaled) then n;
# None where the paper marks no convergence
PAPER_HC = {
    (1, 1e-3, True): (5, 6, 7, 7), (1, 1e-3, False): (17, 40, 81, 159),
    (10, 1e-3, True): (5, 7, 8, 10), (10, 1e-3, False): (22, 90, 174, None),
    (100, 1e-3, True): (6, 9, 13, 21), (100, 1e-3, False): (22, 121, None, None),
    (1, 1e-5, True): (3, 3, 3, 3), (1, 1e-5, False): (8, 13, 23, 46),
    (10, 1e-5, True): (3, 3, 4, 4), (10, 1e-5, False): (11, 27, 63, 123),
    (100, 1e-5, True): (3, 4, 5, 5), (100, 1e-5, False): (13, 57, 259, None),
}
HC_N = (127, 255, 511, 1023)


def run(series, max_n=1024, tol=1e-12, log=print, only_n=None, only_eps=None):
    import gc
    import numpy as np
    import torch
    import paper_2010_06807_amd as P
    sys.path.insert(0, os.path.dirname(HERE))
    from problems import make_rhs
    from problems.paper_ad import paper_problem
    from problems.grids import default_levels
    out = []
    cases = []
    ns2 = [n for n in (128, 256, 512, 1024, 2048) if n <= max_n]
    if "ad2_q" in series:
        cases += [("ad2", f"q={q:g}", n, dict(q=q, b="one"), 1e-2) for q in (1.0, 25.0, 1000.0) for n in ns2]
    if "ad2_eps" in series:
        cases += [("ad2", f"eps={e:.0e}".replace("e-0", "e-"), n, dict(q=1000.0, b="exp"), e)
                  for e in (1e-1, 1e-2, 1e-4) for n in ns2]
    if "ad3" in series:
        cases += [("ad3", f"3d eps={e:.0e}".replace("e-0", "e-"), n, dict(), e) for e in (1e-1, 1e-2) for n in (64, 80, 96)
                  if n ** 3 <= max_n ** 2]
    if "hc" in series:
        cases += [("hc", f"rho={r:g}", n, dict(rho=r), 1e-2) for r in (1.0, 10.0, 100.0) for n in ns2 if n <= 512]
    cases = [c + (True,) for c in cases]
    if only_n:
        cases = [c for c in cases if c[2] in only_n]
    if only_eps:
        cases = [c for c in cases if any(abs(c[4] - e) <= 1e-3 * e for e in only_eps)]
    if "hc_abl" in series:
        cases += [("hc", f"rho={r} eps={e:.0e} {'scaled' if sc else 'unscaled'}".replace("e-0", "e-"), n,
                   dict(rho=float(r)), e, sc)
                  for e in (1e-3, 1e-5) for r in (1, 10, 100) for sc in (True, False) for n in HC_N if n <= max_n]
    for kind, label, n, kw, eps, scale in cases:
        prob = paper_problem(kind, n, **kw)
        A, dims = prob["A"], prob["dims"]
        N = A.shape[0]
        L = default_levels(N)
        o = P.order_grid(dims, L)
        L = o.levels
        b = torch.from_numpy(make_rhs(N, 1, seed=0)).to("cuda:0")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fac = P.factor(A, o, eps=eps, precision=64, scale=scale)
        torch.cuda.synchronize()
        tf = time.perf_counter() - t0
        x, info = fac.solve(b, tol=tol)
        res = float(np.linalg.norm(A @ x.cpu().numpy()[:, 0] - b.cpu().numpy()[:, 0]) /
                    np.linalg.norm(b.cpu().numpy()[:, 0]))
        st = fac.stats()
        if "scaled" in label:
            r = int(kw["rho"])
            pit = PAPER_HC[(r, eps, scale)][HC_N.index(n)]
        else:
            pit = PAPER.get((label, n))
        rec = dict(series=label, kind=kind, n=n, N=N, levels=L, eps=eps, scale=scale,
                   iterations=info[0]["iterations"], converged=info[0]["converged"], relres=res, factor_s=tf,
                   solve_s=info[0]["seconds"], top_separator=st["top_separator"], factor_bytes=st["factor_bytes"],
                   paper_iterations=pit)
        out.append(rec)
        log(json.dumps(rec))
        del fac, x
        gc.collect()
        print(f"[reproduce] device memory free after the case: {torch.cuda.mem_get_info()[0] / 2**30:.1f} GiB",
              file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("series", nargs="*", default=["ad2_q", "ad2_eps", "ad3", "hc", "hc_abl"])
    ap.add_argument("--max-n", type=int, default=1024)
    ap.add_argument("--json", default=None)
    ap.add_argument("--n", type=int, nargs="*", default=None,
                    help="run only the cases of these sizes")
    ap.add_argument("--eps", type=float, nargs="*", default=None, help="run only the cases of these tolerances")
    a = ap.parse_args()
    res = run(a.series, a.max_n, log=lambda s: print(s, file=sys.stderr, flush=True), only_n=a.n, only_eps=a.eps)
    if a.json:
        with open(a.json, "w") as f:
            json.dump(res, f, indent=1)
    print("| series | n | N | eps | GMRES (this build) | GMRES (paper) | factor s | relres |")
    print("|---|---|---|---|---|---|---|---|")
    for r in res:
        its = r["iterations"] if r["converged"] else f"{r['iterations']} (not converged)"
        print(f"| {r['series']} | {r['n']} | {r['N']} | {r['eps']:g} | {its} | "
              f"{r['paper_iterations'] if r['paper_iterations'] is not None else '-'} | {r['factor_s']:.3f} | "
              f"{r['relres']:.1e} |")


if __name__ == "__main__":
    main()
