"""Modified nested dissection (MND) -- oracle: geometric on a regular grid,
and algebraic (the graph of A^T A) for matrices without a grid (readings
G1-G6 further down).

Follows the paper's ordering and clustering (Section 2.3): nested dissection
on the graph of A^T A defines separators (column partition); modified ND
(Fig. "mnd", Fig. "mnd_multilvl") splits every separator into interfaces and
gives each separator a cluster hierarchy; rows are ordered like columns
(diagonally dominant matrices, Section 2.3).  For the advection-diffusion
grids the paper uses geometric partitioning on A^T A (Section 4).

Readings (the paper defers the construction to another work):
  * A separator must cut the graph of A^T A, which couples grid points up to
    distance 2 apart; separators are therefore two grid layers thick.
  * Split of a box [lo, hi): axis = longest extent (ties -> lowest axis index),
    width w >= 4 required, m = lo + floor((w - 2) / 2), separator = layers
    {m, m+1}, low child [lo, m), high child [m+2, hi).
  * Node ids are heap numbers (root 1, children 2k and 2k+1); level(k) is the
    bit length of k, so the root is level 1 and the leaves are level L.
  * Interfaces: a separator point q of node B is pushed to the adjacent layer
    of each child (coordinate m-1 on the low side, m+2 on the high side) and
    descended to the deepest node containing it (desc_low, desc_high).
    key_k(q) = (anc_k(desc_low), anc_k(desc_high)) with anc_k(X) the level-k
    ancestor of X (X itself if level(X) <= k).  At stage k the clusters of a
    separator of level < k are the classes of key_k; a node of level k is a
    single cluster.  The merge parent of a stage-k cluster is the stage-(k-1)
    cluster containing it.
  * perm (new -> old) sorts points by level descending, node id ascending,
    then (key_2, ..., key_L) lexicographically (low side before high side),
    then the natural index.  Every cluster of every stage is a contiguous
    range of perm.

All arithmetic here is integer.
"""

from __future__ import annotations

import numpy as np


class GridOrderingError(ValueError):
    pass


def _level(ids):
    ids = np.asarray(ids, dtype=np.int64)
    # bit length of positive ints
    out = np.zeros(ids.shape, dtype=np.int64)
    v = ids.copy()
    while np.any(v > 0):
        nz = v > 0
        out[nz] += 1
        v[nz] >>= 1
    return out


def build_tree(dims, L):
    """Split boxes recursively.  Returns arrays indexed by heap id (size 2^L):
    axis, msplit (for internal nodes, level < L), lo, hi (boxes)."""
    d = len(dims)
    nnodes = 1 << L
    lo = np.zeros((nnodes, d), dtype=np.int64)
    hi = np.zeros((nnodes, d), dtype=np.int64)
    axis = np.full(nnodes, -1, dtype=np.int64)
    msplit = np.full(nnodes, -1, dtype=np.int64)
    hi[1] = dims
    for node in range(1, 1 << (L - 1)):
        ext = hi[node] - lo[node]
        ax = int(np.argmax(ext))          # first maximum -> lowest axis on ties
        w = int(ext[ax])
        if w < 4:
            raise GridOrderingError(
                f"node {node}: longest extent {w} < 4, too many levels for this grid")
        m = int(lo[node, ax]) + (w - 2) // 2
        axis[node] = ax
        msplit[node] = m
        lo[2 * node] = lo[node]
        hi[2 * node] = hi[node]
        hi[2 * node, ax] = m
        lo[2 * node + 1] = lo[node]
        hi[2 * node + 1] = hi[node]
        lo[2 * node + 1, ax] = m + 2
    return axis, msplit, lo, hi


def _descend(coords, start, axis, msplit, L):
    """Deepest node containing each point, starting from node ids `start`."""
    node = start.copy()
    done = _level(node) >= L
    while not np.all(done):
        act = np.nonzero(~done)[0]
        nd = node[act]
        ax = axis[nd]
        m = msplit[nd]
        c = coords[act, ax]
        in_slab = (c == m) | (c == m + 1)
        done[act[in_slab]] = True
        go = act[~in_slab]
        node[go] = 2 * node[go] + (coords[go, ax[~in_slab]] >= m[~in_slab] + 2)
        done[go] = _level(node[go]) >= L
    return node


def _anc(ids, k):
    lev = _level(ids)
    sh = np.maximum(0, lev - k)
    return ids >> sh


class Ordering:
    """Result of the grid MND: perm, node of each point, and per-stage clusters."""

    def __init__(self, dims, L):
        self.dims = tuple(int(x) for x in dims)
        self.L = int(L)
        d = len(self.dims)
        N = int(np.prod(self.dims))
        self.N = N
        axis, msplit, lo, hi = build_tree(self.dims, self.L)
        self.axis, self.msplit = axis, msplit
        strides = [1]
        for x in self.dims[:-1]:
            strides.append(strides[-1] * x)
        idx = np.arange(N, dtype=np.int64)
        coords = np.stack([(idx // strides[a]) % self.dims[a] for a in range(d)], axis=1)
        node = _descend(coords, np.ones(N, dtype=np.int64), axis, msplit, self.L)
        level = _level(node)
        self.node = node
        self.level = level
        # interface keys for separator points
        sep = level < self.L
        keys = np.zeros((self.L + 1, 2, N), dtype=np.int64)
        if np.any(sep):
            sp_idx = np.nonzero(sep)[0]
            B = node[sp_idx]
            ax = axis[B]
            m = msplit[B]
            cl = coords[sp_idx].copy()
            cl[np.arange(sp_idx.size), ax] = m - 1
            ch = coords[sp_idx].copy()
            ch[np.arange(sp_idx.size), ax] = m + 2
            dlow = _descend(cl, 2 * B, axis, msplit, self.L)
            dhigh = _descend(ch, 2 * B + 1, axis, msplit, self.L)
            for k in range(1, self.L + 1):
                keys[k, 0, sp_idx] = _anc(dlow, k)
                keys[k, 1, sp_idx] = _anc(dhigh, k)
        self.keys = keys
        self._build_perm()

    def _build_perm(self):
        """perm from node, level and keys; every cluster of every stage is a
        contiguous range of it."""
        N, keys, node, level = self.N, self.keys, self.node, self.level
        idx = np.arange(N, dtype=np.int64)
        # perm: level desc, node asc, key_2..key_L (low, high), natural index
        sort_keys = [idx]
        for k in range(self.L, 1, -1):
            sort_keys.append(keys[k, 1])
            sort_keys.append(keys[k, 0])
        sort_keys.append(node)
        sort_keys.append(-level)
        perm = np.lexsort(sort_keys)
        self.perm = perm.astype(np.int64)
        self.iperm = np.empty(N, dtype=np.int64)
        self.iperm[self.perm] = np.arange(N)
        self._stage_cache = {}

    # ------------------------------------------------------------------
    def stage_clusters(self, k):
        """Clusters at stage k as arrays (start, end, node, level), sorted by start.

        Points of nodes at level > k are already eliminated; a node at level k
        is one cluster; a separator of level < k is split by key_k."""
        if k in self._stage_cache:
            return self._stage_cache[k]
        p = self.perm
        lev = self.level[p]
        act = np.nonzero(lev <= k)[0]
        first = act[0] if act.size else self.N
        nd = self.node[p[first:]]
        lv = lev[first:]
        kl = np.where(lv < k, self.keys[k, 0, p[first:]], 0)
        kh = np.where(lv < k, self.keys[k, 1, p[first:]], 0)
        M = nd.size
        if M == 0:
            out = (np.zeros(0, np.int64),) * 4
        else:
            brk = np.ones(M, dtype=bool)
            brk[1:] = (nd[1:] != nd[:-1]) | (kl[1:] != kl[:-1]) | (kh[1:] != kh[:-1])
            starts = np.nonzero(brk)[0]
            ends = np.append(starts[1:], M)
            out = (starts + first, ends + first, nd[starts], lv[starts])
        self._stage_cache[k] = out
        return out

    def merge_parents(self, k):
        """For each stage-k cluster of a node at level < k, the index of the
        stage-(k-1) cluster that contains it; -1 for eliminated clusters."""
        s, e, nd, lv = self.stage_clusters(k)
        s2, e2, _, _ = self.stage_clusters(k - 1)
        par = np.full(s.size, -1, dtype=np.int64)
        keep = lv < k
        j = np.searchsorted(s2, s[keep], side="right") - 1
        par[keep] = j
        return par

    def is_ancestor(self, a, b):
        """True where node a is a proper ancestor of node b."""
        la, lb = _level(a), _level(b)
        return (la < lb) & ((b >> np.maximum(0, lb - la)) == a)


def order_grid(dims, L):
    return Ordering(dims, L)


# ----------------------------------------------------------------------------
# Algebraic MND for matrices without a grid (Section 2.3).
#
# The paper partitions general matrices with a hypergraph partitioner on the
# structure of A (HUND, an external library) and defines interfaces by the
# modified ND of Fig. "mnd".  The readings here, with the graph of A^T A in
# place of the hypergraph:
#   G1 the graph: i ~ j (i != j) iff some row r has A_ri != 0 and A_rj != 0,
#      the pattern of A^T A, whose ND the paper's column ordering is.
#   G2 node X of level l < L with vertex set V_X is split between two far
#      vertices of the subgraph induced on V_X: the root r starts at min(V_X);
#      up to four times, if the BFS from u = the smallest vertex of r's last
#      level has more levels than the BFS from r, r <- u.  Then u is the
#      smallest vertex of r's last level, and every vertex v of r's component
#      gets key(v) = d_r(v) - d_u(v) (BFS distances in the induced subgraph):
#      the classes of key are bands across the line from r to u, not rings
#      around r.  Vertices outside r's component go to the high child.
#   G3 keys run from kmin to kmax; with kmax - kmin >= 3 the separator is the
#      key pair {t, t+1}, t in [kmin+1, kmax-2] minimizing (|#low - #high|,
#      |separator|, t), low = key < t (child 2X), high = key > t+1 and the
#      other components (child 2X+1).  Along an edge each distance changes by
#      at most one, so key by at most two: the separator cuts A^T A inside V_X.
#      The pair is then thinned: its vertices without a neighbour in the high
#      part join the low part, then those without a neighbour in the low part
#      join the high part (a band of equal keys can be wide in a graph
#      metric; what remains still separates).
#      kmax - kmin < 3 at a node above the leaves: too many levels.
#   G4 interfaces: for a separator vertex q of node B and each child C of B,
#      desc_C(q) is the deepest common ancestor of the nodes of q's
#      neighbours inside C's subtree (C if there are none);
#      key_k(q) = (anc_k(desc_2B(q)), anc_k(desc_2B+1(q))), as in the grid
#      version, where desc is the deepest node touched on each side.
#   G5 perm and the clusters of every stage follow the grid version.
#   G6 the default number of levels is ceil(log2(N/64)) (at least 1), capped
#      at the deepest tree whose nodes above the leaves all split.
# ----------------------------------------------------------------------------
def ata_graph(A):
    """Pattern of A^T A without its diagonal, as CSR (indptr, indices) with
    sorted neighbour lists (G1)."""
    import scipy.sparse as sp
    P = sp.csr_matrix((np.ones(A.nnz), A.indices, A.indptr), shape=A.shape)
    G = (P.T @ P).tocsr()
    G.setdiag(0)
    G.eliminate_zeros()
    G.sort_indices()
    return G.indptr.astype(np.int64), G.indices.astype(np.int64)


def _bfs_levels(indptr, indices, inset, root):
    """BFS level sets (ascending arrays) from root inside the vertex mask inset."""
    levels = []
    seen = {int(root)}
    front = np.array([root], dtype=np.int64)
    while front.size:
        levels.append(np.sort(front))
        nb = np.concatenate([indices[indptr[v]:indptr[v + 1]] for v in front]) if front.size else front
        nb = np.unique(nb)
        nb = nb[inset[nb]]
        nb = np.array([v for v in nb if int(v) not in seen], dtype=np.int64)
        seen.update(int(v) for v in nb)
        front = nb
    return levels


def _bisect(indptr, indices, V, N):
    """G2/G3 for the sorted vertex set V: (low, separator, high, (r, u, t)),
    or None when V cannot be split."""
    inset = np.zeros(N, dtype=bool)
    inset[V] = True
    r = int(V[0])
    lev = _bfs_levels(indptr, indices, inset, r)
    for _ in range(4):
        u = int(lev[-1][0])
        lu = _bfs_levels(indptr, indices, inset, u)
        if len(lu) > len(lev):
            r, lev = u, lu
        else:
            break
    u = int(lev[-1][0])
    dr = np.full(N, -1, dtype=np.int64)
    for d, x in enumerate(lev):
        dr[x] = d
    du = np.full(N, -1, dtype=np.int64)
    for d, x in enumerate(_bfs_levels(indptr, indices, inset, u)):
        du[x] = d
    comp = V[dr[V] >= 0]
    other = V[dr[V] < 0]
    key = dr[comp] - du[comp]
    kmin, kmax = int(key.min()), int(key.max())
    if kmax - kmin < 3:
        return None
    counts = np.bincount(key - kmin, minlength=kmax - kmin + 1)
    t = kmin + _split_keys(counts.tolist(), int(other.size))
    side = np.zeros(N, dtype=np.int64)  # -1 low, 0 separator, 1 high (vertices of comp)
    side[comp] = np.where(key < t, -1, np.where(key > t + 1, 1, 0))
    band = comp[side[comp] == 0]
    # thinning (G3): a separator vertex with no neighbour in the high part
    # joins the low part, then one with no neighbour in the low part joins
    # the high part
    for want, to in ((1, -1), (-1, 1)):
        move = [v for v in band if side[v] == 0 and
                not np.any(side[indices[indptr[v]:indptr[v + 1]][inset[indices[indptr[v]:indptr[v + 1]]]]] == want)]
        side[np.array(move, dtype=np.int64)] = to
    low = comp[side[comp] == -1]
    sep = comp[side[comp] == 0]
    high = np.sort(np.concatenate([comp[side[comp] == 1], other]))
    return low, sep, high, (r, u, t)


def _split_keys(counts, n_other):
    """G3 on key class sizes counts[0..] (keys kmin, kmin+1, ...) and n_other
    vertices outside the root's component: the offset t - kmin of the chosen
    separator pair."""
    h = len(counts)
    best = None
    for q in range(1, h - 2):
        lo, sep, hi = sum(counts[:q]), counts[q] + counts[q + 1], sum(counts[q + 2:]) + n_other
        cand = (abs(lo - hi), sep, q)
        if best is None or cand < best:
            best = cand
    return best[2]


def _lca(a, b):
    la, lb = int(a).bit_length(), int(b).bit_length()
    a >>= max(0, la - lb)
    b >>= max(0, lb - la)
    while a != b:
        a >>= 1
        b >>= 1
    return a


class GraphOrdering(Ordering):
    """Algebraic MND of a square sparse matrix (readings G1-G6)."""

    def __init__(self, A, L=0):
        import scipy.sparse as sp
        A = sp.csr_matrix(A)
        N = A.shape[0]
        self.N = N
        self.dims = (N,)
        indptr, indices = ata_graph(A)
        self.graph = (indptr, indices)
        if L <= 0:
            L = 0
            while (64 << L) < N:
                L += 1
            L = max(1, L)
            cap = True
        else:
            cap = False
        node = np.ones(N, dtype=np.int64)
        sets = {1: np.arange(N, dtype=np.int64)}
        # (r, u, t) of every split node (a record only)
        self.splits = {}
        depth = 1
        while depth < L:
            new = {}
            ok = True
            for X in range(1 << (depth - 1), 1 << depth):
                V = sets[X]
                got = _bisect(indptr, indices, V, N) if V.size else None
                if got is None:
                    ok = False
                    break
                low, sep, high, rec = got
                self.splits[X] = rec
                new[2 * X] = low
                new[2 * X + 1] = high
                node[sep] = X
            if not ok:
                if cap:
                    L = depth
                    break
                raise GridOrderingError(f"too many levels: a node of level {depth} cannot be split")
            for X, V in new.items():
                node[V] = X
            sets = new
            depth += 1
        self.L = int(L)
        level = _level(node)
        self.node, self.level = node, level
        keys = np.zeros((self.L + 1, 2, N), dtype=np.int64)
        for q in np.nonzero(level < self.L)[0]:
            B = int(node[q])
            nb = node[indices[indptr[q]:indptr[q + 1]]]
            for side in (0, 1):
                C = 2 * B + side
                lc = C.bit_length()
                lv = _level(nb)
                inside = nb[(lv >= lc) & ((nb >> np.maximum(0, lv - lc)) == C)]
                d = C
                if inside.size:
                    d = int(inside[0])
                    for x in inside[1:]:
                        d = _lca(d, int(x))
                for k in range(1, self.L + 1):
                    keys[k, side, q] = d >> max(0, d.bit_length() - k)
        self.keys = keys
        self._build_perm()


def order_graph(A, L=0):
    return GraphOrdering(A, L)
