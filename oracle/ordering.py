"""Geometric modified nested dissection (MND) on a regular grid -- oracle.

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
