"""Server bookkeeping that needs no GPU: submission copies and validates the
request, and a request whose estimated memory exceeds the budget is refused
at submission; the estimate (the symbolic analysis's bound on device memory)
covers the factors the oracle stores for the same problem."""

import numpy as np
import pytest

import paper_2010_06807_amd as P
from paper_2010_06807_amd import _abi
from paper_2010_06807_amd.server import Server
from problems import convdiff, make_rhs


def test_oversized_request_is_refused():
    A = convdiff((32, 32), (1.0, 1.0))
    o = P.order_grid((32, 32), 5)
    srv = Server(mem_budget=1 << 16)
    with pytest.raises(_abi.SpaqrError) as e:
        srv.submit(A, o, make_rhs(A.shape[0], 1, seed=0))
    assert e.value.status == -2  # SPAQR_ENOMEM


def test_bad_submission_arguments():
    A = convdiff((16, 16), (1.0, 1.0))
    o = P.order_grid((32, 32), 5)  # ordering of another size
    srv = Server(mem_budget=1 << 30)
    with pytest.raises(_abi.SpaqrError):
        srv.submit(A, o, make_rhs(A.shape[0], 1, seed=0))


def test_unknown_ticket_is_pending():
    srv = Server(mem_budget=1 << 30)
    srv._keep[12345] = (4, 1)
    assert srv.poll(12345) is None


def test_budget_one_byte_below_the_estimate_is_refused():
    A = convdiff((40, 40), (10.0, 5.0))
    o = P.order_grid((40, 40), 5)
    est = P.analyze(A, o).estimate_bytes(precision=32, nrhs=2)
    with pytest.raises(_abi.SpaqrError) as e:
        Server(mem_budget=est - 1).submit(A, o, make_rhs(A.shape[0], 2, seed=0))
    assert e.value.status == -2
    srv = Server(mem_budget=est)
    srv.submit(A, o, make_rhs(A.shape[0], 2, seed=0))
    assert srv.status() == (1, 0, 0)


@pytest.mark.parametrize("dims,beta,eps", [((32, 32), (10.0, 10.0), 0.0), ((32, 32), (10.0, 10.0), 1e-3),
                                           ((8, 8, 8), (20.0, -5.0, 3.0), 1e-2),
                                           ((12, 12, 12), (5.0, 5.0, 5.0), 0.0),
                                           ((64, 64), (50.0, -20.0), 1e-4)])
def test_estimate_covers_the_oracle_factor_bytes(dims, beta, eps):
    from oracle.ordering import order_grid as oracle_order
    from oracle import spaqr as osq
    from problems.grids import default_levels
    A = convdiff(dims, beta)
    L = default_levels(A.shape[0])
    F = osq.factor(A, oracle_order(dims, L), eps)
    sym = P.analyze(A, P.order_grid(dims, L))
    for prec, item in ((32, 4), (64, 8)):
        assert osq.factor_bytes(F, item) <= sym.estimate_bytes(precision=prec), (dims, prec)


def test_estimate_covers_the_full_size_goldens():
    """The 256^2, 1024^2 and 64^3 workloads: the bound of the analysis against
    the factor bytes the oracle stored (FP64) in the golden files."""
    import glob
    import json
    import os
    from problems import config_problem
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    seen = {}
    for path in sorted(glob.glob(os.path.join(here, "c*_s0_eps0.01.json"))):
        g = json.load(open(path))
        if g["workload"] in seen:
            continue
        prob = config_problem(g["workload"], seed=0)
        sym = P.analyze(prob["A"], P.order_grid(prob["dims"], prob["levels"]))
        seen[g["workload"]] = True
        assert g["factor_bytes_fp64"] <= sym.estimate_bytes(precision=64), g["workload"]
        assert g["factor_bytes_fp64"] // 2 <= sym.estimate_bytes(precision=32), g["workload"]
    assert "c2" in seen
