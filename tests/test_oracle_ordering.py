"""Pins for the oracle's geometric modified nested dissection (Section 2.3)."""

import os

import numpy as np
import pytest
import scipy.sparse as sp

from problems import convdiff
from oracle.ordering import order_grid, GridOrderingError

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _ata_pattern(dims):
    A = convdiff(dims, (1.0,) * len(dims))
    P = (abs(A) > 0).astype(np.float64)
    return (P.T @ P).tocsr()


def _descendants(o, node):
    """Mask of points whose node is `node` or one of its descendants."""
    nd = o.node
    lv = o.level
    lvl = node.bit_length()
    return (lv >= lvl) & ((nd >> np.maximum(0, lv - lvl)) == node)


@pytest.mark.parametrize("dims,L", [((16, 16), 4), ((12, 16), 4), ((8, 8, 8), 4), ((9, 7, 8), 3),
                                     ((16, 16), 5)])
def test_separators_cut_ata(dims, L):
    """No entry of A^T A couples the low and high child of any node (ND on the
    graph of A^T A, Section 2.1 / 2.3): brute force over all nodes."""
    o = order_grid(dims, L)
    G = _ata_pattern(dims)
    for node in range(1, 1 << (L - 1)):
        lo = _descendants(o, 2 * node)
        hi = _descendants(o, 2 * node + 1)
        if lo.sum() == 0 or hi.sum() == 0:
            continue
        assert G[np.ix_(np.nonzero(lo)[0], np.nonzero(hi)[0])].nnz == 0


@pytest.mark.parametrize("dims,L", [((16, 16), 4), ((8, 8, 8), 4), ((20, 14), 4)])
def test_unrelated_clusters_decoupled(dims, L):
    """Clusters whose nodes are not ancestor-related have a zero A^T A block."""
    o = order_grid(dims, L)
    G = _ata_pattern(dims)
    st, en, nd, lv = o.stage_clusters(L)
    p = o.perm
    Gp = G[p][:, p].tocsr()
    cl = np.zeros(o.N, dtype=np.int64)
    for c in range(st.size):
        cl[st[c]:en[c]] = c
    coo = Gp.tocoo()
    ci, cj = cl[coo.row], cl[coo.col]
    a, b = nd[ci], nd[cj]
    related = (a == b) | o.is_ancestor(a, b) | o.is_ancestor(b, a)
    assert np.all(related)


@pytest.mark.parametrize("dims,L", [((32, 32), 5), ((16, 16, 16), 6), ((17, 23), 5)])
def test_partitions_nest(dims, L):
    o = order_grid(dims, L)
    assert np.array_equal(np.sort(o.perm), np.arange(o.N))
    for k in range(L, 0, -1):
        st, en, nd, lv = o.stage_clusters(k)
        # cover exactly the points of level <= k, contiguously
        assert np.all(en > st)
        assert np.all(st[1:] == en[:-1])
        assert en[-1] == o.N
        assert (en - st).sum() == int((o.level <= k).sum())
        # every point in a cluster belongs to the cluster's node
        lab = np.repeat(nd, en - st)
        assert np.array_equal(lab, o.node[o.perm[st[0]:]])
        if k > 1:
            par = o.merge_parents(k)
            st2, en2, nd2, _ = o.stage_clusters(k - 1)
            for c in range(st.size):
                if lv[c] < k:
                    P = par[c]
                    assert st2[P] <= st[c] and en[c] <= en2[P] and nd2[P] == nd[c]
                else:
                    assert par[c] == -1
    # a separator of level l is a single cluster at stages l and l+1
    for k in range(2, L + 1):
        st, en, nd, lv = o.stage_clusters(k)
        sel = lv == k - 1
        assert len(np.unique(nd[sel])) == int(sel.sum())


def test_root_interfaces_32x32_golden():
    """Hand-derived interface sizes of the root separator (fixture)."""
    o = order_grid((32, 32), 5)
    want = {}
    with open(os.path.join(GOLDEN, "mnd_32x32.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            t = [int(x) for x in line.split()]
            want[t[0]] = t[1:]
    for k, sizes in want.items():
        st, en, nd, lv = o.stage_clusters(k)
        got = sorted((en - st)[nd == 1].tolist())
        assert got == sizes, (k, got, sizes)


def test_too_many_levels_rejected():
    with pytest.raises(GridOrderingError):
        order_grid((8, 8), 6)


def test_leaf_sizes_c4_shape():
    """1024^2 with 14 levels: leaves of 6..7 x 14..15 points (84..105)."""
    o = order_grid((1024, 1024), 14)
    st, en, nd, lv = o.stage_clusters(14)
    leaf = (en - st)[lv == 14]
    assert leaf.min() == 84 and leaf.max() == 105 and leaf.size == 8192
