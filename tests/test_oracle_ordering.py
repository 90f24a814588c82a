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


# ----------------------------------------------------------------------------
# algebraic MND (readings G1-G6 in oracle/ordering.py)
from problems.unstructured import delaunay_convdiff, permuted  # noqa: E402
from oracle.ordering import order_graph  # noqa: E402

GRAPH_CASES = {
    "delaunay1500": lambda: delaunay_convdiff(1500, seed=1),
    "perm24": lambda: permuted(convdiff((24, 24), (5.0, 5.0)), seed=2)[0],
    "grid3d": lambda: convdiff((8, 8, 8), (3.0, 2.0, 1.0)),
}


def _dense_ata(A):
    P = (A.toarray() != 0).astype(np.int64)
    return (P.T @ P) != 0


@pytest.mark.parametrize("name", sorted(GRAPH_CASES))
def test_graph_separators_cut_ata(name):
    """No entry of A^T A (a dense product of the pattern) couples the two
    children's subtrees of any node."""
    A = GRAPH_CASES[name]()
    o = order_graph(A)
    G = _dense_ata(A)
    assert o.L >= 3
    for node in range(1, 1 << (o.L - 1)):
        lo = np.nonzero(_descendants(o, 2 * node))[0]
        hi = np.nonzero(_descendants(o, 2 * node + 1))[0]
        assert lo.size and hi.size
        assert not G[np.ix_(lo, hi)].any()


@pytest.mark.parametrize("name", sorted(GRAPH_CASES))
def test_graph_split_rule_against_csgraph(name):
    """G2/G3 recomputed from scipy's unweighted shortest paths on each node's
    induced subgraph: the two far vertices, the key classes d_r - d_u, the
    chosen separator pair, its thinning on the dense adjacency, and both
    children."""
    from scipy.sparse.csgraph import shortest_path
    A = GRAPH_CASES[name]()
    o = order_graph(A)
    G = sp.csr_matrix(_dense_ata(A).astype(np.float64))
    G.setdiag(0)
    G.eliminate_zeros()
    for X, (root, far, t) in o.splits.items():
        if X.bit_length() >= o.L:
            continue
        V = np.nonzero(_descendants(o, X))[0]
        S = G[V][:, V]
        D = shortest_path(S, unweighted=True, directed=False)

        def depth_of(i):
            d = D[i]
            return int(d[np.isfinite(d)].max())

        r = 0  # index into V of min(V)
        for _ in range(4):
            u = int(np.nonzero(D[r] == depth_of(r))[0].min())
            if depth_of(u) > depth_of(r):
                r = u
            else:
                break
        u = int(np.nonzero(D[r] == depth_of(r))[0].min())
        assert V[r] == root and V[u] == far
        comp = np.isfinite(D[r])
        key = (D[r] - D[u])[comp].astype(np.int64)
        kmin, kmax = int(key.min()), int(key.max())
        n_other = int((~comp).sum())
        best = min((abs(int((key < q).sum()) - int((key > q + 1).sum()) - n_other),
                    int(((key == q) | (key == q + 1)).sum()), q) for q in range(kmin + 1, kmax - 1))
        assert best[2] == t
        # thinning on the dense adjacency of the induced subgraph
        Sd = S.toarray() != 0
        idx = np.nonzero(comp)[0]
        low = np.zeros(V.size, dtype=bool)
        high = ~comp.copy()
        low[idx[key < t]] = True
        high[idx[key > t + 1]] = True
        band = np.zeros(V.size, dtype=bool)
        band[idx[(key == t) | (key == t + 1)]] = True
        to_low = band & ~(Sd[:, high].any(axis=1))
        low |= to_low
        band &= ~to_low
        to_high = band & ~(Sd[:, low].any(axis=1))
        band &= ~to_high
        assert np.array_equal(np.sort(V[band]), np.nonzero(o.node == X)[0])
        assert np.array_equal(np.sort(V[low]), np.nonzero(_descendants(o, 2 * X))[0])


@pytest.mark.parametrize("name", sorted(GRAPH_CASES))
def test_graph_interfaces_brute_force(name):
    """G4: desc_C(q) is the deepest tree node that is an ancestor-or-self of
    the node of every neighbour of q inside C's subtree (C if none), found by
    trying every node id."""
    A = GRAPH_CASES[name]()
    o = order_graph(A)
    G = _dense_ata(A)
    np.fill_diagonal(G, False)
    L = o.L
    ids = np.arange(1, 1 << L)
    for q in np.nonzero(o.level < L)[0]:
        B = int(o.node[q])
        for side in (0, 1):
            C = 2 * B + side
            nb = o.node[np.nonzero(G[q])[0]]
            inside = [int(x) for x in nb if (int(x) >> max(0, int(x).bit_length() - C.bit_length())) == C
                      and int(x).bit_length() >= C.bit_length()]
            best = C
            for D in ids:
                D = int(D)
                if D.bit_length() <= best.bit_length():
                    continue
                if all((x >> max(0, x.bit_length() - D.bit_length())) == D and x.bit_length() >= D.bit_length()
                       for x in inside) and inside:
                    best = D
            assert o.keys[L, side, q] == best, (q, side)


@pytest.mark.parametrize("name", sorted(GRAPH_CASES))
def test_graph_partitions_nest(name):
    A = GRAPH_CASES[name]()
    o = order_graph(A)
    assert np.array_equal(np.sort(o.perm), np.arange(o.N))
    for k in range(o.L, 0, -1):
        st, en, nd, lv = o.stage_clusters(k)
        assert np.all(en > st) and np.all(st[1:] == en[:-1]) and en[-1] == o.N
        assert (en - st).sum() == int((o.level <= k).sum())
        assert np.array_equal(np.repeat(nd, en - st), o.node[o.perm[st[0]:]])
        if k > 1:
            par = o.merge_parents(k)
            st2, en2, _, _ = o.stage_clusters(k - 1)
            for c in range(st.size):
                if lv[c] < k:
                    assert st2[par[c]] <= st[c] and en[c] <= en2[par[c]]


@pytest.mark.parametrize("name", ["delaunay1500", "perm24"])
def test_graph_ordering_exact_at_eps0(name):
    """The ordering is a valid nested dissection for the method: at eps = 0
    spaQR with it solves A exactly (against a dense solve) and every update
    skipped by reading R4 is zero."""
    from oracle import spaqr
    from problems import make_rhs
    A = GRAPH_CASES[name]()
    o = order_graph(A)
    F = spaqr.factor(A, o, 0.0, check_skipped=True)
    b = make_rhs(A.shape[0], 1, seed=4)[:, 0]
    x = spaqr.apply(F, b)
    xd = np.linalg.solve(A.toarray(), b)
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)
    assert F.max_skipped_update <= 1e-13


def test_graph_default_levels():
    A = delaunay_convdiff(5000, seed=0)
    o = order_graph(A)
    assert o.L == 7  # ceil(log2(5000 / 64))
    with pytest.raises(GridOrderingError):
        order_graph(convdiff((6, 6), (1.0, 1.0)), 5)


def test_graph_split_keys_by_hand():
    """G3 on key class sizes worked out by hand: balance first, then the
    smaller separator pair, then the lower key."""
    from oracle.ordering import _split_keys
    # keys 0..4 of sizes 2, 1, 1, 3, 1: t = 1 splits 2 | 2 | 4, t = 2 splits 3 | 4 | 1
    assert _split_keys([2, 1, 1, 3, 1], 0) == 1
    # keys -3..3: t = -1 and t = 0 both leave imbalance 3 with separators of 7: the lower key
    assert _split_keys([1, 2, 3, 4, 3, 2, 1], 0) == 2
    # keys 0..5 of sizes 2, 1, 3, 1, 1, 2: imbalances 2, 0, 4
    assert _split_keys([2, 1, 3, 1, 1, 2], 0) == 2
    # vertices outside the root's component count on the high side
    assert _split_keys([3, 1, 1, 1, 1, 1], 0) == 1
    assert _split_keys([3, 1, 1, 1, 1, 1], 3) == 2  # imbalances 3, 1, 1: the lower key
