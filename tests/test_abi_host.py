"""Host-side checks of the C ABI library (no GPU work).

The library loads, exports every function include/spaqr.h declares, and its
host logic -- grid ordering and symbolic analysis -- is bit-exact against the
oracle's independent implementation (clusters, permutation, merge parents,
block patterns before and after each stage's fronts, front row/column sets,
front and interface colourings).
"""

import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2010_06807_amd as P
from paper_2010_06807_amd import _abi
from problems import convdiff, config_problem
from oracle.ordering import order_grid as oracle_order
from oracle import spaqr as oracle_spaqr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    txt = open(os.path.join(ROOT, "include", "spaqr.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(spaqr_[a-z_]+)\s*\(", txt)))


def test_exports_every_declared_symbol():
    lib = C.CDLL(_abi.LIB_PATH)
    names = _declared_functions()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding declares the same set
    assert set(names) == set(_abi.SIGNATURES), set(names) ^ set(_abi.SIGNATURES)


@pytest.mark.parametrize("dims,L", [((32, 32), 5), ((256, 256), 10), ((64, 64, 64), 12), ((17, 23), 5),
                                     ((9, 7, 8), 3), ((1024, 1024), 14), ((5, 5), 1)])
def test_ordering_bit_exact(dims, L):
    o = P.order_grid(dims, L)
    ob = oracle_order(dims, L)
    assert o.levels == L and o.n == ob.N
    assert np.array_equal(o.perm(), ob.perm)
    for k in range(L, 0, -1):
        for a, b in zip(o.clusters(k), ob.stage_clusters(k)):
            assert np.array_equal(a, b)
        if k > 1:
            assert np.array_equal(o.merge_parents(k), ob.merge_parents(k))


def test_default_levels():
    assert P.order_grid((256, 256)).levels == 10
    assert P.order_grid((32, 32)).levels == 4
    assert P.order_grid((64, 64, 64)).levels == 12


def test_default_levels_capped_by_the_grid():
    """ceil(log2(N/64)) = 8 for 21^3, but a box of the 8th level would need a
    split of a box narrower than 4: the default stops at 7, and asking for 8
    explicitly is an error."""
    assert P.order_grid((21, 21, 21)).levels == 7
    assert P.order_grid((44, 44, 44)).levels == 10
    with pytest.raises(_abi.SpaqrError):
        P.order_grid((21, 21, 21), 8)
    # the capped default is a valid ordering: the oracle builds the same one
    o = P.order_grid((21, 21, 21))
    ob = oracle_order((21, 21, 21), 7)
    assert np.array_equal(o.perm(), ob.perm)


@pytest.mark.parametrize("dims,L,eps", [((32, 32), 5, 1e-3), ((24, 24), 5, 1e-2), ((8, 8, 8), 4, 1e-2),
                                        ((16, 16, 16), 6, 1e-2), ((64, 64), 7, 1e-2), ((20, 13), 4, 1e-2)])
def test_symbolic_bit_exact(dims, L, eps):
    A = convdiff(dims, (10.0, -4.0, 7.0)[:len(dims)])
    o = P.order_grid(dims, L)
    sym = P.analyze(A, o)
    F = oracle_spaqr.factor(A, oracle_order(dims, L), eps)
    for k in range(L, 0, -1):
        rec = F.stages[k]
        assert sym.pattern(k) == [tuple(x) for x in rec["pattern_in"]]
        assert sym.pattern(k, post=True) == [tuple(x) for x in rec["pattern_post"]]
        want = {s: (list(a), list(b), c) for s, (a, b, c) in rec["fronts"].items()}
        assert sym.fronts(k) == want
        assert sym.iface_colours(k) == (rec["iface_colour"] if rec["sparsified"] else {})


def test_invalid_inputs_rejected():
    with pytest.raises(P.SpaqrError) as e:
        P.order_grid((8, 8), 6)
    assert e.value.status == _abi.EINVAL
    with pytest.raises(P.SpaqrError):
        P.order_grid((0, 8), 2)
    A = convdiff((8, 8), (1.0, 1.0))
    o = P.order_grid((8, 8), 3)
    B = A.copy()
    B.indices = B.indices.copy()
    B.indices[3], B.indices[4] = B.indices[4], B.indices[3]   # unsorted columns
    with pytest.raises(P.SpaqrError):
        P.analyze(B, o)
    o2 = P.order_grid((8, 9), 3)
    with pytest.raises(P.SpaqrError):
        P.analyze(A, o2)            # size mismatch
    lib = _abi.load()
    assert lib.spaqr_status_string(-3).decode().startswith("exactly singular")


# ---------------------------------------------------------------- graph MND
from problems.unstructured import delaunay_convdiff, permuted  # noqa: E402
from oracle.ordering import order_graph as oracle_order_graph  # noqa: E402

GRAPH_MATS = {
    "delaunay3000": lambda: delaunay_convdiff(3000, seed=3),
    "delaunay20000": lambda: delaunay_convdiff(20000, seed=4),
    "perm48": lambda: permuted(convdiff((48, 48), (5.0, -3.0)), seed=5)[0],
    "grid3d": lambda: convdiff((10, 9, 8), (2.0, 1.0, 1.0)),
}


@pytest.mark.parametrize("name,L", [("delaunay3000", 0), ("delaunay3000", 4), ("delaunay20000", 0),
                                    ("perm48", 0), ("grid3d", 0)])
def test_graph_ordering_bit_exact(name, L):
    A = GRAPH_MATS[name]()
    o = P.order_graph(A, L)
    ob = oracle_order_graph(A, L)
    assert o.levels == ob.L and o.n == ob.N
    assert np.array_equal(o.perm(), ob.perm)
    for k in range(ob.L, 0, -1):
        for a, b in zip(o.clusters(k), ob.stage_clusters(k)):
            assert np.array_equal(a, b)
        if k > 1:
            assert np.array_equal(o.merge_parents(k), ob.merge_parents(k))


@pytest.mark.parametrize("name,eps", [("delaunay3000", 1e-2), ("perm48", 1e-3)])
def test_graph_symbolic_bit_exact(name, eps):
    A = GRAPH_MATS[name]()
    o = P.order_graph(A)
    ob = oracle_order_graph(A)
    sym = P.analyze(A, o)
    F = oracle_spaqr.factor(A, ob, eps)
    for k in range(ob.L, 0, -1):
        rec = F.stages[k]
        assert sym.pattern(k) == [tuple(x) for x in rec["pattern_in"]]
        assert sym.pattern(k, post=True) == [tuple(x) for x in rec["pattern_post"]]
        want = {s: (list(a), list(b), c) for s, (a, b, c) in rec["fronts"].items()}
        assert sym.fronts(k) == want
        assert sym.iface_colours(k) == (rec["iface_colour"] if rec["sparsified"] else {})


def test_graph_ordering_rejects_bad_input():
    import scipy.sparse as sp
    with pytest.raises(P.SpaqrError):
        P.order_graph(convdiff((6, 6), (1.0, 1.0)), 5)   # too many levels for 36 unknowns
    B = sp.csr_matrix((np.ones(2), np.array([0, 1]), np.array([0, 1, 2, 2])), shape=(3, 3))
    with pytest.raises(P.SpaqrError):
        P.order_graph(B, 3)
