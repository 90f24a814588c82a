"""GPU parity on matrices without a grid, ordered by the algebraic MND
(spaqr_order_graph, readings G1-G6 of oracle/ordering.py): the HIP engine
against the oracle factoring with the oracle's own graph ordering (the two
orderings are bit-exact, tests/test_abi_host.py).

Bars, as for the grid workloads: FP64 ranks equal to the oracle's on every
interface, M^{-1} b element by element within 1e-10 of the largest entry,
GMRES iterations within max(1, ceil(0.1 * oracle)), both solves at <= 1e-10;
FP32 factors: ranks within +-1, residual <= 1e-10 and the same iteration
window.
"""

import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2010_06807_amd as P
from problems import convdiff, make_rhs
from problems.unstructured import delaunay_convdiff, permuted
from oracle.ordering import order_graph as oracle_order_graph
from oracle import spaqr as oracle_spaqr, gmres as oracle_gmres

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

MATS = {
    "delaunay3000": lambda: delaunay_convdiff(3000, seed=3),
    "delaunay12000": lambda: delaunay_convdiff(12000, beta=(40.0, -25.0), seed=6),
    "perm48": lambda: permuted(convdiff((48, 48), (5.0, -3.0)), seed=5)[0],
    "grid3d": lambda: convdiff((12, 11, 10), (2.0, 1.0, 1.0)),
}
CASES = [("delaunay3000", 1e-2), ("delaunay3000", 1e-4), ("delaunay12000", 1e-2), ("perm48", 1e-3),
         ("grid3d", 1e-2)]


def _dev(b):
    return torch.from_numpy(np.asfortranarray(b).T.copy()).to(DEV).T


@pytest.mark.parametrize("name,eps", CASES)
def test_graph_ordering_parity(name, eps):
    print(f"case graph {name} eps={eps}", flush=True)
    A = MATS[name]()
    N = A.shape[0]
    ob = oracle_order_graph(A)
    F = oracle_spaqr.factor(A, ob, eps)
    assert any(rec["sparsified"] for rec in F.stages.values())
    o = P.order_graph(A)
    sym = P.analyze(A, o)
    b = make_rhs(N, 2, seed=7)
    xo1, it_o, rel_o = oracle_gmres.fgmres(lambda v: A @ v, lambda v: oracle_spaqr.apply(F, v), b[:, 0], 1e-10)
    for prec in (64, 32):
        fac = P.Factorization(A, symbolic=sym, eps=eps, precision=prec)
        worst = 0
        for k in range(ob.L, 0, -1):
            rec = F.stages[k]
            if not rec["sparsified"]:
                continue
            sizes = fac.stage_sizes(k)
            for p, r in rec["ranks"].items():
                worst = max(worst, abs(int(sizes[p]) - int(r)))
        x, info = fac.solve(_dev(b[:, :1]), tol=1e-10)
        res = np.linalg.norm(A @ x.cpu().numpy()[:, 0] - b[:, 0]) / np.linalg.norm(b[:, 0])
        print(f"precision {prec}: rank diff {worst}, iterations {info[0]['iterations']} (oracle {it_o}), "
              f"relres {res:.1e}", flush=True)
        assert res <= 1e-10 and info[0]["converged"]
        assert abs(info[0]["iterations"] - it_o) <= max(1, math.ceil(0.1 * it_o))
        if prec == 64:
            assert worst == 0
            yo = oracle_spaqr.apply(F, b)
            yg = fac.apply(_dev(b)).cpu().numpy()
            err = np.abs(yg - yo).max() / np.abs(yo).max()
            print(f"fp64 apply max rel diff {err:.2e}", flush=True)
            assert err <= 1e-10
        else:
            assert worst <= 1
