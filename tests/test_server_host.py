"""Server bookkeeping that needs no GPU: submission copies and validates the
request, and a request whose estimated memory exceeds the budget is refused
at submission."""

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
