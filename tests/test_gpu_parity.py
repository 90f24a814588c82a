"""GPU parity: the HIP engine against the FP64 oracle, through the C ABI.

Bars (the tolerances the method's hot path is held to):
  * eps = 0 (exact nested-dissection QR): ||A x - b|| / ||b|| <= 1e-12 for
    the FP64 engine, and M^{-1} b equal to the oracle's element by element;
  * eps > 0: per-interface ranks within +-1 (identical ranks are then checked
    element by element on M^{-1} b), GMRES iteration counts within
    max(1, ceil(0.1 * oracle)) and both solves at <= 1e-10;
  * FP32 factors with FP64 GMRES: same rank and iteration bars, residual
    <= 1e-10; the FP32 apply's distance to the oracle's is reported and bounded
    by a multiple of FP32 unit roundoff times the preconditioner's growth.
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
    worst = _ranks_agree(fac, F, L, 1)
    b = make_rhs(N, 3, seed=5)
    xo = oracle_spaqr.apply(F, b)
    xg = fac.apply(_dev(b)).cpu().numpy()
    if worst == 0:
        err = np.abs(xg - xo).max() / np.abs(xo).max()
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
    it_o, _ = _oracle_its(A, F, b[:, 0])
    x, info = fac.solve(_dev(b), tol=1e-10)
    res = np.linalg.norm(A @ x.cpu().numpy() - b) / np.linalg.norm(b)
    assert res <= 1e-10 and info[0]["converged"]
    assert info[0]["iterations"] <= it_o + max(1, math.ceil(0.1 * it_o)), (info, it_o)


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


def test_c2_fp32_against_oracle():
    """The 256^2 variable-coefficient workload at eps = 1e-2."""
    prob = config_problem("c2", seed=0)
    A, dims, L = prob["A"], prob["dims"], prob["levels"]
    N = A.shape[0]
    F = _oracle(A, dims, L, 1e-2)
    b = make_rhs(N, 1, seed=0)
    it_o, _ = _oracle_its(A, F, b[:, 0])
    for prec in (64, 32):
        print(f"case c2 precision={prec}", flush=True)
        fac = P.factor(A, P.order_grid(dims, L), eps=1e-2, precision=prec)
        _ranks_agree(fac, F, L, 1)
        x, info = fac.solve(_dev(b), tol=1e-10)
        res = np.linalg.norm(A @ x.cpu().numpy() - b) / np.linalg.norm(b)
        assert res <= 1e-10
        assert abs(info[0]["iterations"] - it_o) <= max(1, math.ceil(0.1 * it_o)), (prec, info, it_o)


def test_c2_fp32_tight_tolerance_against_oracle():
    """The 256^2 workload at eps = 1e-4: some interfaces of 33-64 unknowns
    reach 2049-2560 columns, so the register CPQR keeps a column per thread
    in global memory (and a few wider ones take the cooperative kernel)."""
    prob = config_problem("c2", seed=0)
    A, dims, L = prob["A"], prob["dims"], prob["levels"]
    N = A.shape[0]
    F = _oracle(A, dims, L, 1e-4)
    b = make_rhs(N, 1, seed=0)
    it_o, _ = _oracle_its(A, F, b[:, 0])
    print("case c2 eps=1e-4 precision=32", flush=True)
    fac = P.factor(A, P.order_grid(dims, L), eps=1e-4, precision=32)
    _ranks_agree(fac, F, L, 1)
    x, info = fac.solve(_dev(b), tol=1e-10)
    res = np.linalg.norm(A @ x.cpu().numpy() - b) / np.linalg.norm(b)
    assert res <= 1e-10
    assert info[0]["iterations"] <= it_o + max(1, math.ceil(0.1 * it_o)), (info, it_o)


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


def test_3d_wide_interfaces_against_oracle():
    """20^3 grid: the coarse interfaces have more than 64 unknowns and
    thousands of columns, so the sparsification runs in the cooperative
    multi-workgroup CPQR.  FP64 ranks within +-1 of the oracle, iteration
    counts within the 10% bar, both solves at 1e-10."""
    print("case 3d 20^3 fp64 eps=1e-2", flush=True)
    dims = (20, 20, 20)
    A = convdiff(dims, (5.0, 5.0, 5.0))
    N = A.shape[0]
    L = P.order_grid(dims).levels
    F = _oracle(A, dims, L, 1e-2)
    assert max(max(r for r in F.stages[k]["ranks"].values()) for k in F.stages
               if F.stages[k]["sparsified"]) > 64
    fac = P.factor(A, P.order_grid(dims, L), eps=1e-2, precision=64)
    _ranks_agree(fac, F, L, 1)
    b = make_rhs(N, 1, seed=3)[:, 0]
    x, info = fac.solve(b, tol=1e-10)
    it_o, rel_o = _oracle_its(A, F, b)
    assert np.linalg.norm(A @ x - b) / np.linalg.norm(b) <= 1e-10
    assert abs(info[0]["iterations"] - it_o) <= max(1, math.ceil(0.1 * it_o))
    fac32 = P.factor(A, P.order_grid(dims, L), eps=1e-2, precision=32)
    x32, info32 = fac32.solve(b, tol=1e-10)
    assert np.linalg.norm(A @ x32 - b) / np.linalg.norm(b) <= 1e-10
