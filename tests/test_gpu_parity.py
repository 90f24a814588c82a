"""GPU parity: the HIP engine against the FP64 oracle, through the C ABI.

Bars (the tolerances the method's hot path is held to):
  * eps = 0 (exact nested-dissection QR): ||A x - b|| / ||b|| <= 1e-12 for
    the FP64 engine, and M^{-1} b equal to the oracle's element by element;
  * eps > 0: FP64 per-interface ranks equal to the oracle's on every case
    here, so M^{-1} b is checked element by element on every case (max
    difference <= 1e-11 of the largest entry), GMRES iteration counts within
    max(1, ceil(0.1 * oracle)) and both solves at <= 1e-10;
  * FP32 factors with FP64 GMRES: ranks within +-1, iteration counts within
    the same window in both directions, residual <= 1e-10, and the FP32
    M^{-1} b within 1e-3 (relative 2-norm) of the oracle's: FP32 unit
    roundoff 6e-8 times the apply's error growth, which the FP64 comparison
    bounds below 1e3 on these grids.
"""

import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2010_06807_amd as P
from problems import convdiff, config_problem, make_rhs
from oracle.ordering import order_grid as oracle_order
from oracle import spaqr as oracle_spaqr, gmres as oracle_gmres

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _dev(b):
    return torch.from_numpy(np.asfortranarray(b).T.copy()).to(DEV).T


def _oracle(A, dims, L, eps):
    return oracle_spaqr.factor(A, oracle_order(dims, L), eps)


def _oracle_its(A, F, b, tol=1e-10):
    x, it, rel = oracle_gmres.fgmres(lambda v: A @ v, lambda v: oracle_spaqr.apply(F, v), b, tol)
    return it, rel


def _ranks_agree(fac, F, L, slack):
    worst = 0
    for k in range(L, 0, -1):
        rec = F.stages[k]
        if not rec["sparsified"]:
            continue
        sizes = fac.stage_sizes(k)
        for p, r in rec["ranks"].items():
            worst = max(worst, abs(int(sizes[p]) - int(r)))
    assert worst <= slack, worst
    return worst


CASES = [
    # dims, L, beta, eps
    ((32, 32), 5, (10.0, 10.0), 0.0),
    ((32, 32), 5, (10.0, 10.0), 1e-3),
    ((24, 40), 5, (-30.0, 15.0), 1e-2),
    ((8, 8, 8), 4, (20.0, -5.0, 3.0), 1e-2),
    ((12, 12, 12), 6, (5.0, 5.0, 5.0), 1e-3),
    ((64, 64), 7, (50.0, -20.0), 1e-4),
    # exact factorizations whose fronts span the apply kernels' row classes
    # (up to 64, 65-128, 129-192, 193-256 and more than 256 pivots, with and
    # without ancestor columns): the apply alone must invert A
    ((11, 11, 11), 3, (5.0, 5.0, 5.0), 0.0),
    ((14, 14, 14), 4, (2.0, -3.0, 1.0), 0.0),
    ((13, 13), 1, (4.0, 1.0), 0.0),
]


@pytest.mark.parametrize("dims,L,beta,eps", CASES)
def test_fp64_apply_matches_oracle(dims, L, beta, eps):
    print(f"case fp64 dims={dims} L={L} eps={eps}", flush=True)
    A = convdiff(dims, beta)
    N = A.shape[0]
    F = _oracle(A, dims, L, eps)
    fac = P.factor(A, P.order_grid(dims, L), eps=eps, precision=64)
    _ranks_agree(fac, F, L, 0)
    b = make_rhs(N, 3, seed=5)
    xo = oracle_spaqr.apply(F, b)
    xg = fac.apply(_dev(b)).cpu().numpy()
    err = np.abs(xg - xo).max() / np.abs(xo).max()
    print(f"fp64 apply max rel diff {err:.2e}", flush=True)
    assert err <= 1e-11, err
    if eps == 0.0:
        res = np.linalg.norm(A @ xg - b, axis=0) / np.linalg.norm(b, axis=0)
        assert res.max() <= 1e-12, res


@pytest.mark.parametrize("dims,L,beta,eps", CASES)
def test_fp64_solve_matches_oracle(dims, L, beta, eps):
    print(f"case solve fp64 dims={dims} L={L} eps={eps}", flush=True)
    A = convdiff(dims, beta)
    N = A.shape[0]
    F = _oracle(A, dims, L, eps)
    b = make_rhs(N, 1, seed=11)
    it_o, rel_o = _oracle_its(A, F, b[:, 0])
    fac = P.factor(A, P.order_grid(dims, L), eps=eps, precision=64)
    x, info = fac.solve(_dev(b), tol=1e-10)
    x = x.cpu().numpy()
    res = np.linalg.norm(A @ x - b) / np.linalg.norm(b)
    assert rel_o <= 1e-10 and res <= 1e-10 and info[0]["converged"]
    assert abs(info[0]["iterations"] - it_o) <= max(1, math.ceil(0.1 * it_o)), (info, it_o)
    if eps == 0.0:
        assert info[0]["iterations"] == 1 and res <= 1e-12


@pytest.mark.parametrize("dims,L,beta,eps", CASES[1:])
def test_fp32_factor_fp64_gmres(dims, L, beta, eps):
    print(f"case fp32 dims={dims} L={L} eps={eps}", flush=True)
    A = convdiff(dims, beta)
    N = A.shape[0]
    F = _oracle(A, dims, L, eps)
    fac = P.factor(A, P.order_grid(dims, L), eps=eps, precision=32)
    _ranks_agree(fac, F, L, 1 if eps >= 1e-4 else 10 ** 6)
    # every scaled interface of every sparsified stage is counted once
    assert fac.stats()["interfaces_sparsified"] == sum(1 for op in F.ops if op[0] == "scale")
    b = make_rhs(N, 1, seed=3)
    yo = oracle_spaqr.apply(F, b)
    yg = fac.apply(_dev(b)).cpu().numpy()
    dy = np.linalg.norm(yg - yo) / np.linalg.norm(yo)
    print(f"fp32 apply rel diff {dy:.2e}", flush=True)
    assert dy <= 1e-3, dy
    it_o, _ = _oracle_its(A, F, b[:, 0])
    x, info = fac.solve(_dev(b), tol=1e-10)
    res = np.linalg.norm(A @ x.cpu().numpy() - b) / np.linalg.norm(b)
    assert res <= 1e-10 and info[0]["converged"]
    assert abs(info[0]["iterations"] - it_o) <= max(1, math.ceil(0.1 * it_o)), (info, it_o)


def test_multi_rhs_ragged():
    """nrhs spanning several RHS blocks with a ragged tail, and ld > n."""
    dims, L = (32, 32), 5
    A = convdiff(dims, (10.0, 10.0))
    N = A.shape[0]
    F = _oracle(A, dims, L, 1e-3)
    fac = P.factor(A, P.order_grid(dims, L), eps=1e-3, precision=64)
    b = make_rhs(N, 11, seed=2)
    xo = oracle_spaqr.apply(F, b)
    big = torch.zeros((N + 7, 11), dtype=torch.float64).T.contiguous().T  # column-major, ld = N + 7
    big = torch.zeros((11, N + 7), dtype=torch.float64, device=DEV).T
    big[:N] = torch.from_numpy(b).to(DEV)
    out = torch.zeros_like(big)
    fac.apply(big, out=out)
    xg = out[:N].cpu().numpy()
    assert np.abs(xg - xo).max() <= 1e-11 * np.abs(xo).max()
    x, info = fac.solve(_dev(b), tol=1e-10)
    res = np.linalg.norm(A @ x.cpu().numpy() - b, axis=0) / np.linalg.norm(b, axis=0)
    assert res.max() <= 1e-10 and all(i["converged"] for i in info)


def test_host_pointers_and_degenerate_grids():
    """Host buffers through the ABI; a one-level grid (a single leaf, no
    separators) and a grid whose root separator has no neighbours."""
    for dims, L in [((6, 6), 1), ((9, 9), 2), ((4, 4, 4), 1)]:
        A = convdiff(dims, (3.0,) * len(dims))
        N = A.shape[0]
        fac = P.factor(A, P.order_grid(dims, L), eps=1e-2, precision=64)
        b = make_rhs(N, 2, seed=1)
        x = fac.apply(b)
        res = np.linalg.norm(A @ x - b, axis=0) / np.linalg.norm(b, axis=0)
        assert res.max() <= 1e-12
        xs, info = fac.solve(b, tol=1e-10)
        assert all(i["iterations"] == 1 for i in info)


def test_device_resident_input_matches_host_input():
    """spaqr_factor_device (values read from HBM, column scaling on the GPU)
    against spaqr_factor (host values): same ranks, same M^{-1} b."""
    dims, L = (48, 48), 6
    A = convdiff(dims, (35.0, -12.0))
    N = A.shape[0]
    o = P.order_grid(dims, L)
    sym = P.analyze(A, o)
    dA = P.DeviceCSR(A, DEV)
    for prec in (64, 32):
        f_host = P.factor(A, o, eps=1e-2, precision=prec)
        f_dev = P.factor_device(A, sym, dA, eps=1e-2, precision=prec)
        for k in range(L, 0, -1):
            assert np.array_equal(f_host.stage_sizes(k), f_dev.stage_sizes(k))
        b = make_rhs(N, 2, seed=8)
        xh = f_host.apply(_dev(b)).cpu().numpy()
        xd = f_dev.apply(_dev(b)).cpu().numpy()
        tol = 1e-12 if prec == 64 else 1e-4
        assert np.abs(xh - xd).max() <= tol * np.abs(xh).max()


def test_kernel_profiler_counts_launches():
    dims, L = (32, 32), 5
    A = convdiff(dims, (10.0, 10.0))
    P.profile_enable(True)
    fac = P.factor(A, P.order_grid(dims, L), eps=1e-3, precision=32)
    fac.apply(_dev(make_rhs(A.shape[0], 1, seed=0)))
    q = P.profile_query("front_qr")
    a = P.profile_query("apply_front_fwd")
    P.profile_enable(False)
    assert q["launches"] >= L and q["total_ms"] > 0 and q["flops"] > 0
    assert a["launches"] >= L and a["bytes"] > 0
    P.profile_enable(True, only="sparsify")
    P.factor(A, P.order_grid(dims, L), eps=1e-3, precision=32)
    assert P.profile_query("front_qr")["launches"] == 0
    assert P.profile_query("sparsify")["launches"] > 0
    # a prefix filter: the host phases only
    P.profile_enable(True, only="host_*")
    P.factor(A, P.order_grid(dims, L), eps=1e-3, precision=32)
    assert P.profile_query("host_plan_fronts")["launches"] >= L
    assert P.profile_query("host_wait_gpu")["total_ms"] > 0
    assert P.profile_query("sparsify")["launches"] == 0
    P.profile_enable(False)


# dispatch thresholds that send the blocks of a small 3D grid through every
# kernel the large workloads use: the LDS-panel QR (fronts over 256 rows), the
# matrix-core trailing update (64-reflector blocks), the general scaling
# kernels (blocks over 16), the cooperative CPQR for every interface, the
# reflector apply of interfaces over 16 unknowns; the FP32 single-workgroup
# and team CPQRs with downdated norms by default, the exact-norm register and
# cooperative ones with those off; and with the cooperative
# CPQR and the matrix cores off, the single-workgroup LDS and generic CPQR
# kernels and the vector-ALU trailing-update slices
FORCED = [
    # (thresholds, kernels an FP64 factorization + apply must launch, the same for FP32)
    (dict(), ("k_qr_reg", "k_cpqr_coop", "k_scale_small", "k_ap_iface_dense", "k_wy_tblock", "k_trail_mfma"),
     ("k_qr_reg", "k_cpqr_dd", "k_cpqr_team", "k_wy_tblock", "k_trail_mfma")),
    (dict(qr_reg_max_rows=256, split_rows=256, split_cols=256, cpqr_reg=0, scale_small=16, iface_dense=16,
          cpqr_team=0),
     ("k_qr", "k_wy_tblock", "k_trail_mfma", "k_scale_right", "k_cpqr_coop", "k_ap_iface_fwd", "k_ap_iface_bwd",
      "k_ap_front_bwd_reg"),
     ("k_qr", "k_wy_tblock", "k_trail_mfma", "k_cpqr_dd", "k_cpqr_coop")),
    (dict(cpqr_dd=0, cpqr_team=0), ("k_qr_reg", "k_cpqr_coop"), ("k_qr_reg", "k_cpqr_reg", "k_cpqr_coop")),
    (dict(cpqr_reg=0, cpqr_coop=0, scale_small=0, iface_dense=0, trail_mfma=0, cpqr_dd=0, cpqr_team=0),
     ("k_sparsify", "k_trail", "k_scale_right", "k_ap_iface_fwd", "k_ap_iface_bwd"),
     ("k_sparsify_small", "k_trail", "k_scale_right")),
]


def test_3d_every_kernel_path_against_oracle():
    """20^3 grid (interfaces up to ~280 unknowns with ~4000 columns, fronts
    up to ~540 rows and ~1500 trailing columns): the FP64 engine under the
    default dispatch and under thresholds that force the other kernel of every
    phase, each checked against the oracle -- ranks equal on every interface
    and M^{-1} b element by element -- with launch counts showing the kernels
    ran.  FP32 under the same dispatch variants: ranks within +-1 and M^{-1} b
    within 1e-3; both precisions converge within the iteration window."""
    dims = (20, 20, 20)
    A = convdiff(dims, (5.0, 5.0, 5.0))
    N = A.shape[0]
    L = P.order_grid(dims).levels
    F = _oracle(A, dims, L, 1e-2)
    assert max(max(r for r in F.stages[k]["ranks"].values()) for k in F.stages
               if F.stages[k]["sparsified"]) > 64
    b = make_rhs(N, 2, seed=3)
    yo = oracle_spaqr.apply(F, b)
    it_o, _ = _oracle_its(A, F, b[:, 0])
    families = ("k_qr_reg", "k_qr", "k_trail", "k_wy_tblock", "k_trail_mfma", "k_scale_small", "k_scale",
                "k_scale_right", "k_cpqr_reg", "k_cpqr_dd", "k_cpqr_team",
                "k_cpqr_coop", "k_sparsify_small", "k_sparsify", "k_iface_form", "k_ap_front_fwd_reg",
                "k_ap_front_fwd_wy", "k_ap_front_bwd_reg", "k_ap_iface_dense", "k_ap_iface_fwd", "k_ap_iface_bwd")
    try:
        for tune, kernels64, kernels32 in FORCED:
            for prec in (64, 32):
                kernels = kernels64 if prec == 64 else kernels32
                print(f"case 3d 20^3 precision={prec} tuning={tune}", flush=True)
                P.set_tuning()
                P.set_tuning(**tune)
                P.kernel_launches(None)
                fac = P.factor(A, P.order_grid(dims, L), eps=1e-2, precision=prec)
                yg = fac.apply(_dev(b)).cpu().numpy()
                counts = {k: P.kernel_launches(k) for k in families}
                print(f"launches {counts}", flush=True)
                assert all(counts[k] > 0 for k in kernels), counts
                if prec == 64:
                    _ranks_agree(fac, F, L, 0)
                    err = np.abs(yg - yo).max() / np.abs(yo).max()
                    print(f"fp64 apply max rel diff {err:.2e}", flush=True)
                    assert err <= 1e-10, err
                else:
                    _ranks_agree(fac, F, L, 1)
                    err = np.linalg.norm(yg - yo) / np.linalg.norm(yo)
                    print(f"fp32 apply rel diff {err:.2e}", flush=True)
                    assert err <= 1e-3, err
                x, info = fac.solve(_dev(b[:, :1]), tol=1e-10)
                assert np.linalg.norm(A @ x.cpu().numpy()[:, 0] - b[:, 0]) / np.linalg.norm(b[:, 0]) <= 1e-10
                assert abs(info[0]["iterations"] - it_o) <= max(1, math.ceil(0.1 * it_o))
    finally:
        P.set_tuning()


def test_stage_statistics_against_oracle():
    """Per-stage statistics (Section 4.3 quantities): every sparsified
    interface's (|p|, m_p, r_p) equals the oracle's CPQR shape, the counted
    CPQR work equals the method's formula on the oracle's shapes, the
    per-stage sums add up to the totals, the phase times are measured, and
    the solve's residual history ends at the true residual."""
    sys_path_golden()
    from make_goldens import cpqr_flops
    dims, L = (48, 40), 6
    A = convdiff(dims, (-30.0, 15.0))
    N = A.shape[0]
    F = _oracle(A, dims, L, 1e-2)
    fac = P.factor(A, P.order_grid(dims, L), eps=1e-2, precision=64)
    st = fac.stats()
    tot_if = tot_fs = tot_ff = tot_bytes = 0.0
    shapes = []
    ms = 0.0
    for k in range(L, 0, -1):
        g = fac.stage_stats(k)
        assert g["stage"] == k
        tot_ff += g["flops_front"]
        tot_fs += g["flops_sparsify"]
        tot_bytes += g["factor_bytes"]
        ms += g["ms_front"] + g["ms_scale"] + g["ms_sparsify"] + g["ms_merge"]
        rec = F.stages[k]
        assert g["sparsified"] == int(rec["sparsified"])
        assert g["fronts"] == len(rec["fronts"])
        ifs = fac.stage_interfaces(k)
        assert ifs.shape[0] == g["interfaces"]
        tot_if += g["interfaces"]
        if rec["sparsified"]:
            want = {p: v for p, v in rec["cpqr_shapes"].items() if v[0] > 0}
            got = {int(c): (int(p), int(m), int(r)) for c, p, m, r in ifs}
            assert got == want
            sizes = fac.stage_sizes(k)
            assert all(sizes[c] == r for c, _, _, r in ifs)
            assert g["iface_unknowns_out"] == int(ifs[:, 3].sum()) and g["nbr_cols"] == int(ifs[:, 2].sum())
            assert g["iface_size_q1"] <= g["iface_size_median"] <= g["iface_size_q3"] <= g["iface_size_max"]
            shapes.extend(want.values())
    assert tot_if == st["interfaces_sparsified"]
    assert abs(tot_ff - st["flops_front"]) <= 1e-9 * st["flops_front"]
    assert abs(tot_fs - st["flops_sparsify"]) <= 1e-9 * max(1.0, st["flops_sparsify"])
    assert abs(st["flops_sparsify"] - cpqr_flops(np.array(shapes))) <= 1e-9 * st["flops_sparsify"]
    assert tot_bytes <= st["factor_bytes"] and ms > 0 and sum(st["ms_phase"]) > 0
    assert st["top_separator"] == fac.stage_stats(2)["top_separator"] > 0
    assert st["ms_symbolic"] > 0
    b = make_rhs(N, 1, seed=2)
    x, info = fac.solve(_dev(b), tol=1e-10)
    h = fac.solve_history()
    assert len(h) == info[0]["iterations"] + 1
    assert h[-1] == pytest.approx(info[0]["relres"], rel=1e-12) and h[-2] <= 1e-10 and h[0] < 1.0


def sys_path_golden():
    import os
    import sys
    d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    if d not in sys.path:
        sys.path.insert(0, d)


def test_apply_graph_replays_match_eager():
    """From its second apply of a width on, a factorization replays its two
    sweeps from a captured HIP graph: every replay, with other eager work
    and synchronizations between them (a different width, a solve), equals
    the first, eager apply bit for bit."""
    dims, L = (40, 40), 6
    A = convdiff(dims, (20.0, -10.0))
    N = A.shape[0]
    for prec in (32, 64):
        fac = P.factor(A, P.order_grid(dims, L), eps=1e-2, precision=prec)
        b = _dev(make_rhs(N, 2, seed=6))
        b1 = _dev(make_rhs(N, 1, seed=7))
        y0 = fac.apply(b).clone()
        for rep in range(4):
            y = fac.apply(b)
            z = fac.apply(b1)            # another width: eager, then its own graph
            torch.cuda.synchronize()
            assert torch.equal(y, y0), (prec, rep)
            if rep == 1:
                fac.solve(b1, tol=1e-10)  # FGMRES applies in between
            if rep >= 1:
                assert torch.equal(z, z_prev), (prec, rep)
            z_prev = z.clone()
