"""spaQR factorization and preconditioner apply -- FP64 oracle.

Implements Algorithm 2 (Section 2.8) step by step on a dictionary of dense
blocks over clusters:

  pre-scale columns to unit 2-norm                          (Section 2.8)
  for stage k = L .. 1:
    block Householder QR of every front at level k          (Section 2.4)
    if sparsifying at this stage:
      block-diagonal scaling of every remaining interface   (Section 2.6)
      scaled sparsification (CPQR, ratio rule) per interface (Sections 2.5, 2.6, 4)
    merge interfaces one level up the cluster hierarchy     (Section 2.7)

and the apply of the preconditioner M^{-1} = D_c P^T W^{-1} Q^T P, with
Q^T = the left factors in elimination order and W^{-1} = the right factors in
reverse order (Section 2.8; the printed products are read this way, see
the readings list below).

Readings where the paper is silent or ambiguous (each is listed in the design
notes of the repository):
  R1 rows are clustered exactly like columns (upwind grids are diagonally
     dominant, Section 2.3).
  R2 column pre-scaling to 2-norm 1: A_hat = P A D_c P^T, x = D_c P^T y.
  R3 stage k: factor level k; if k <= L - skip and k > 1, scale then sparsify
     every interface of the separators of level < k; merge to stage k-1.
     skip = 2 ("skip sparsification for two levels", Fig. runtime_per_level).
  R4 front of s: rows [s; n1(s) ascending], n1(s) = clusters i != s holding a
     block (i, s); columns cols(s) = {s} u {j : the node of j is a proper
     ancestor of the node of s and some front row holds a block (i, j)}.
     H_s^T is not applied to non-ancestor columns (it acts as the identity on
     them up to O(eps), Lemma 2 and Theorem well_sep, Appendix).
  R5 order of the fronts of one level: greedy colouring (ascending id, lowest
     free colour) of the graph "f1 ~ f2 iff some block (i, j), i in n1, j in
     cols minus the pivots, is updated by both"; fronts run colour by colour,
     ascending id inside a colour.  Fronts of one colour touch disjoint blocks,
     so a colour may run in parallel with identical results.
  R6 scaling: A_pp = U_pp R_pp (Householder QR), A_pj <- U_pp^T A_pj,
     A_ip <- A_ip R_pp^{-1}, A_pp := I; left before right; an interface whose
     R_pp has an exactly zero diagonal entry is neither scaled nor sparsified.
  R7 sparsification of a scaled interface p: C = [A_np^T | A_pn] with columns
     ordered as the row-neighbour blocks (i, p) by ascending i, then the
     column-neighbour blocks (p, j) by ascending j; partial CPQR with the ratio
     rule gives r and Q_pp; W = Q_pp^T C; A_cj := W[:r, cols of j],
     A_ic := W[:r, rows of i]^T, A_cc := I_r; W[r:, :] is dropped and the
     fine unknowns are final.  Coarse first in storage.  If r = |p| nothing is
     dropped and nothing is stored.
  R8 order of sparsification inside a stage: greedy colouring (ascending id)
     of the interface graph "p ~ q iff block (p, q) or (q, p) exists"; colours
     in order, ascending id inside a colour.
  R9 merge: a stage-(k-1) cluster takes the surviving unknowns of its stage-k
     children in ascending child order; blocks are assembled from the child
     blocks with zeros elsewhere; the block pattern is symbolic (a block of
     size zero still exists).

The variant without scaling (Section 2.5, scale=False) replaces R6 and R7:
  R10 no interface is scaled; interfaces are sparsified in the order of R8 and
     sigma = 1 / sigma_min(A_p) is taken from the current blocks when p is
     reached (A_p = [A_pp; A_np], the row-neighbour blocks (i, p) stacked
     under A_pp by ascending i), so it sees the neighbours of earlier colours
     already sparsified.  sigma_min(A_p) = 0 leaves p alone.
  R11 C = [A_np^T | sigma A_pp^T A_pn], columns ordered as in R7; the partial
     CPQR with the ratio rule gives r and Q_pp.  The first r columns of Q_pp
     are the coarse unknowns c, the other |p| - r the fine ones f.  A_ip :=
     A_ip Q_pp restricted to c (W_cn^T; the f part is dropped).  Householder
     QR of the f columns of A_pp Q_pp gives H and R_ff; H^T is applied to the
     rows of p: its first |p| - r rows hold [R_fc R_ff R_fn] (R_fn dropped),
     its last r rows the new A_cc and A_cj.  The right factor R_f^{-1} makes
     the f rows [0 I] and leaves the c columns unchanged.  If r = |p| nothing
     is dropped and nothing is stored.
  R12 the rows of p after H^T are stored coarse first: the forward sweep
     applies H^T to b_p and moves its last r entries to the front, so rows and
     columns of the new cluster share its first r slots.

Vectors live in a fixed slot space of length N (the permuted index).  Each
cluster owns a list of slots; after sparsification its first r slots carry
the coarse unknowns and the rest hold final values.  A merge concatenates
slot lists and moves no data.
"""

from __future__ import annotations

from collections import defaultdict

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg  # noqa: F401  (sp.linalg.norm)
from scipy.linalg import lapack

from .cpqr import cpqr_ratio, apply_reflectors


# ----------------------------------------------------------------------------
# LAPACK wrappers (library primitives used as single steps)
def _geqrf(F):
    qr, tau, _, info = lapack.dgeqrf(np.asfortranarray(F))
    if info != 0:
        raise RuntimeError("dgeqrf failed")
    return qr, tau


def _ormqr_lt(qr, tau, C):
    """C <- H^T C for the reflectors stored by dgeqrf."""
    if C.size == 0:
        return C.copy()
    lwork = max(1, C.shape[1]) * 64
    out, _, info = lapack.dormqr("L", "T", qr, tau, np.asfortranarray(C), lwork)
    if info != 0:
        raise RuntimeError("dormqr failed")
    return out


def _reflectors(qr, tau):
    """Explicit Householder vectors (unit diagonal) from dgeqrf output."""
    m, n = qr.shape
    k = min(m, n)
    V = np.tril(qr[:, :k], -1)
    V[np.arange(k), np.arange(k)] = 1.0
    return V, np.asarray(tau[:k], dtype=np.float64)


def _greedy_colour(n_items, neighbours):
    """Greedy colouring in ascending order; neighbours[i] is a set."""
    colour = np.full(n_items, -1, dtype=np.int64)
    for i in range(n_items):
        used = {colour[j] for j in neighbours[i] if colour[j] >= 0}
        c = 0
        while c in used:
            c += 1
        colour[i] = c
    return colour


class BlockMatrix:
    """Dense blocks over clusters with row and column adjacency sets."""

    def __init__(self):
        self.blk = {}
        self.rows = defaultdict(set)   # i -> {j}
        self.cols = defaultdict(set)   # j -> {i}

    def get(self, i, j):
        return self.blk.get((i, j))

    def set(self, i, j, B):
        self.blk[(i, j)] = B
        self.rows[i].add(j)
        self.cols[j].add(i)

    def drop_cluster(self, s):
        for j in list(self.rows[s]):
            del self.blk[(s, j)]
            self.cols[j].discard(s)
        for i in list(self.cols[s]):
            if (i, s) in self.blk:
                del self.blk[(i, s)]
            self.rows[i].discard(s)
        self.rows.pop(s, None)
        self.cols.pop(s, None)

    def pattern(self):
        return sorted(self.blk.keys())


class OracleFactorization:
    """Factors and per-stage records of one spaQR factorization."""

    def __init__(self):
        self.ops = []        # elimination-order list of factor records
        self.stages = {}     # k -> dict of per-stage records


def _initial_blocks(Ahp, starts, ends):
    """Dense blocks of the permuted, pre-scaled matrix over stage-L clusters."""
    bm = BlockMatrix()
    Ahp = Ahp.tocsr()
    for i in range(starts.size):
        sub = Ahp[starts[i]:ends[i]]
        if sub.nnz == 0:
            continue
        cl = np.searchsorted(starts, sub.indices, side="right") - 1
        for j in np.unique(cl):
            bm.set(i, int(j), sub[:, starts[j]:ends[j]].toarray())
    return bm


def _sparsify_unscaled(bm, p, rowN, colN, eps):
    """Sparsification of interface p without scaling (Section 2.5, Lemma 1),
    in place on the block dictionary; readings R10-R12.

    Returns None when sigma_min(A_p) = 0 (p is left alone), else
    (r, op, info): op = (Vq, tq, r, VH, tH, R_ff, R_fc) for the apply and info
    the record of sigma, R_ff, the dropped R_fn and the f rows of Q_pp^T C."""
    App = bm.get(p, p)
    sz = App.shape[0]
    rows = [bm.get(i, p) for i in rowN]
    Ap = np.vstack([App] + rows)
    smin = float(np.linalg.svd(Ap, compute_uv=False)[-1])
    if smin == 0.0:
        return None
    sigma = 1.0 / smin
    parts = [B.T for B in rows] + [sigma * (App.T @ bm.get(p, j)) for j in colN]
    widths = [x.shape[1] for x in parts]
    C = np.hstack(parts) if parts else np.zeros((sz, 0))
    mr = int(sum(B.shape[0] for B in rows))
    r, Vq, tq, W, rdiag, piv = cpqr_ratio(C, eps)
    QtC = apply_reflectors(Vq, tq, C, transpose=True)
    info = {"sigma": sigma, "m": int(C.shape[1]), "W_f1": QtC[r:, :mr].copy(), "W_f2": QtC[r:, mr:].copy()}
    if r == sz:
        return r, None, info
    f = sz - r
    # A_pp Q_pp: Q_pp acts on the columns of p
    AQ = apply_reflectors(Vq, tq, App.T, transpose=True).T
    # Householder QR of the f columns (rows of p only: A_np Q_pf is dropped)
    qrH, tauH = _geqrf(AQ[:, r:])
    VH, tH = _reflectors(qrH, tauH)
    Rff = np.triu(qrH[:f, :f])
    Hc = _ormqr_lt(qrH, tauH, AQ[:, :r])  # [R_fc; A_cc]
    off = np.concatenate([[0], np.cumsum(widths)]).astype(np.int64)
    for a, i in enumerate(rowN):
        bm.set(i, p, np.ascontiguousarray(W[:, off[a]:off[a + 1]].T))
    rfn = []
    for j in colN:
        Hj = _ormqr_lt(qrH, tauH, bm.get(p, j))
        rfn.append(Hj[:f])
        bm.set(p, j, np.ascontiguousarray(Hj[f:]))
    bm.set(p, p, np.ascontiguousarray(Hc[f:]))
    info["R_ff"] = Rff
    info["R_fn"] = np.hstack(rfn) if rfn else np.zeros((f, 0))
    return r, (Vq, tq, r, VH, tH, Rff, np.ascontiguousarray(Hc[:f])), info


def factor(A, ordering, eps, skip=2, scale=True, check_skipped=False, within_colour="ascending", trace=None):
    """Factorize A with spaQR (Algorithm 2).  A: scipy sparse, N x N.

    Returns an OracleFactorization with .ops (for apply), .perm, .Dc and
    per-stage records in .stages[k].

    within_colour: order of the fronts (R5) and interfaces (R8) inside one
    colour class, "ascending" (the reading) or "descending"; by the colouring
    the result must not depend on it.
    trace: optional callable trace(k, event, blocks) receiving a copy of the
    block dictionary {(i, j): array} at events "before_scaling" and
    "after_scaling" of every sparsified stage, or "before_sparsification"
    without scaling (a record only).
    scale: True for the scaled variant (Sections 2.6, 2.8), False for the
    sparsification without scaling of Section 2.5 (readings R10-R12)."""
    if within_colour not in ("ascending", "descending"):
        raise ValueError("within_colour is 'ascending' or 'descending'")
    wsign = 1 if within_colour == "ascending" else -1
    A = sp.csr_matrix(A, dtype=np.float64)
    N = A.shape[0]
    L = ordering.L
    F = OracleFactorization()
    F.N, F.L, F.eps, F.skip = N, L, float(eps), int(skip)
    # Section 2.8: pre-process so that every column has the same 2-norm (1).
    colnorm = np.sqrt(np.asarray(A.multiply(A).sum(axis=0)).ravel())
    if np.any(colnorm == 0.0):
        raise ValueError("A has a zero column")
    Dc = 1.0 / colnorm
    perm = ordering.perm
    Ah = (A @ sp.diags(Dc)).tocsr()
    Ahp = Ah[perm][:, perm]
    F.perm, F.Dc = perm, Dc
    F.anorm = float(sp.linalg.norm(Ahp))

    st, en, nd, lv = ordering.stage_clusters(L)
    bm = _initial_blocks(Ahp, st, en)
    slots = [np.arange(st[c], en[c], dtype=np.int64) for c in range(st.size)]
    max_skipped = 0.0

    for k in range(L, 0, -1):
        st, en, nd, lv = ordering.stage_clusters(k)
        rec = {"clusters": (st.copy(), en.copy(), nd.copy(), lv.copy()),
               "pattern_in": bm.pattern(),
               "sizes_in": np.array([len(s) for s in slots], dtype=np.int64)}
        # ---------------- fronts of level k (Section 2.4) ----------------
        fronts = [int(c) for c in np.nonzero(lv == k)[0]]
        fstruct = {}
        for s in fronts:
            n1 = sorted(i for i in bm.cols[s] if i != s)
            rows = [s] + n1
            cand = set()
            for r in rows:
                cand |= bm.rows[r]
            cand.discard(s)
            cand = np.array(sorted(cand), dtype=np.int64)
            if cand.size:
                anc = ordering.is_ancestor(nd[cand], np.full(cand.size, nd[s]))
                cols = [int(j) for j in cand[anc]]
                nonanc = [int(j) for j in cand[~anc]]
            else:
                cols, nonanc = [], []
            fstruct[s] = (n1, cols, nonanc)
        # conflict graph between fronts (R5)
        upd = {s: {(i, j) for i in fstruct[s][0] for j in fstruct[s][1]} for s in fronts}
        fidx = {s: t for t, s in enumerate(fronts)}
        owners = defaultdict(list)
        for s in fronts:
            for key in upd[s]:
                owners[key].append(fidx[s])
        nbr = [set() for _ in fronts]
        for lst in owners.values():
            for a in lst:
                nbr[a].update(lst)
        for t in range(len(fronts)):
            nbr[t].discard(t)
        fcol = _greedy_colour(len(fronts), nbr)
        rec["fronts"] = {s: (fstruct[s][0], fstruct[s][1], int(fcol[fidx[s]])) for s in fronts}
        order = sorted(fronts, key=lambda s: (fcol[fidx[s]], wsign * s))
        for s in order:
            n1, cols, nonanc = fstruct[s]
            rows = [s] + n1
            rsz = [len(slots[r]) for r in rows]
            roff = np.concatenate([[0], np.cumsum(rsz)])
            n = len(slots[s])
            csz = [len(slots[j]) for j in cols]
            coff = np.concatenate([[0], np.cumsum(csz)]).astype(np.int64)
            m = int(roff[-1])
            rowslots = np.concatenate([slots[r] for r in rows]) if rows else np.zeros(0, np.int64)
            colslots = (np.concatenate([slots[j] for j in cols]) if cols
                        else np.zeros(0, np.int64))
            if n > 0:
                Fp = np.vstack([bm.get(r, s) for r in rows])
                T = np.zeros((m, int(coff[-1])))
                for a, r in enumerate(rows):
                    for b, j in enumerate(cols):
                        B = bm.get(r, j)
                        if B is not None:
                            T[roff[a]:roff[a + 1], coff[b]:coff[b + 1]] = B
                qr, tau = _geqrf(Fp)
                HT = _ormqr_lt(qr, tau, T)
                V, tauv = _reflectors(qr, tau)
                Rss = np.triu(qr[:n, :n])
                if check_skipped and nonanc:
                    for j in nonanc:
                        X = np.zeros((m, len(slots[j])))
                        for a, r in enumerate(rows):
                            B = bm.get(r, j)
                            if B is not None:
                                X[roff[a]:roff[a + 1]] = B
                        if X.size:
                            dX = _ormqr_lt(qr, tau, X) - X
                            max_skipped = max(max_skipped, float(np.abs(dX).max()))
                F.ops.append(("front", k, s, rowslots, n, V, tauv, Rss, colslots, HT[:n].copy()))
                Tn = HT[n:]
            else:
                Tn = np.zeros((m, int(coff[-1])))
                F.ops.append(("front", k, s, rowslots, 0, np.zeros((m, 0)), np.zeros(0),
                              np.zeros((0, 0)), colslots, np.zeros((0, colslots.size))))
            bm.drop_cluster(s)
            for a, i in enumerate(n1):
                r0, r1 = roff[a + 1] - n, roff[a + 2] - n
                for b, j in enumerate(cols):
                    bm.set(i, j, Tn[r0:r1, coff[b]:coff[b + 1]].copy())
        rec["pattern_post"] = bm.pattern()
        remaining = [int(c) for c in np.nonzero(lv < k)[0]]
        rec["sparsified"] = False
        # ---------------- scaling + sparsification (Sections 2.5, 2.6) -----
        if k <= L - skip and k > 1 and remaining:
            rec["sparsified"] = True
            Uf = {}
            if scale:
                for p in remaining:
                    sz = len(slots[p])
                    if sz == 0:
                        continue
                    qrU, tauU = _geqrf(bm.get(p, p))
                    Rpp = np.triu(qrU[:sz, :sz])
                    if np.any(np.diag(Rpp) == 0.0):
                        continue
                    Uf[p] = (qrU, tauU, Rpp)
                if trace is not None:
                    trace(k, "before_scaling", {key: B.copy() for key, B in bm.blk.items()})
                for (i, j), B in list(bm.blk.items()):
                    if i == j and i in Uf:
                        bm.blk[(i, j)] = np.eye(B.shape[0])
                        continue
                    if B.size == 0:
                        continue
                    if i in Uf:
                        B = _ormqr_lt(Uf[i][0], Uf[i][1], B)
                    if j in Uf:
                        B = sla.solve_triangular(Uf[j][2], B.T, trans="T", lower=False).T
                    bm.blk[(i, j)] = np.ascontiguousarray(B)
                if trace is not None:
                    trace(k, "after_scaling", {key: B.copy() for key, B in bm.blk.items()})
                for p in remaining:
                    if p in Uf:
                        V, tauv = _reflectors(Uf[p][0], Uf[p][1])
                        F.ops.append(("scale", k, p, slots[p].copy(), V, tauv, Uf[p][2]))
            elif trace is not None:
                trace(k, "before_sparsification", {key: B.copy() for key, B in bm.blk.items()})
            # colouring of the interface graph (R8)
            ridx = {p: t for t, p in enumerate(remaining)}
            nbr = [set() for _ in remaining]
            for p in remaining:
                for q in (bm.rows[p] | bm.cols[p]):
                    if q != p:
                        nbr[ridx[p]].add(ridx[q])
            icol = _greedy_colour(len(remaining), nbr)
            rec["iface_colour"] = {p: int(icol[ridx[p]]) for p in remaining}
            ranks = {}
            shapes = {}
            unscaled = {}
            for p in sorted(remaining, key=lambda p: (icol[ridx[p]], wsign * p)):
                sz = len(slots[p])
                if scale and p not in Uf:
                    ranks[p] = sz
                    continue
                rowN = sorted(i for i in bm.cols[p] if i != p)
                colN = sorted(j for j in bm.rows[p] if j != p)
                if not scale:
                    if sz == 0:
                        ranks[p] = 0
                        continue
                    got = _sparsify_unscaled(bm, p, rowN, colN, eps)
                    if got is None:
                        ranks[p] = sz
                        continue
                    r, op, info = got
                    ranks[p] = r
                    shapes[p] = (sz, info["m"], r)
                    unscaled[p] = info
                    if r < sz:
                        F.ops.append(("sparsify_u", k, p, slots[p].copy()) + op)
                        slots[p] = slots[p][:r]
                    continue
                parts = [bm.get(i, p).T for i in rowN] + [bm.get(p, j) for j in colN]
                widths = [x.shape[1] for x in parts]
                C = np.hstack(parts) if parts else np.zeros((sz, 0))
                r, Vq, tq, W, rdiag, piv = cpqr_ratio(C, eps)
                ranks[p] = r
                shapes[p] = (sz, C.shape[1], r)
                if r == sz:
                    continue
                off = np.concatenate([[0], np.cumsum(widths)]).astype(np.int64)
                for a, i in enumerate(rowN):
                    bm.set(i, p, np.ascontiguousarray(W[:, off[a]:off[a + 1]].T))
                for b, j in enumerate(colN):
                    a = len(rowN) + b
                    bm.set(p, j, np.ascontiguousarray(W[:, off[a]:off[a + 1]]))
                bm.set(p, p, np.eye(r))
                F.ops.append(("sparsify", k, p, slots[p].copy(), Vq, tq, r))
                slots[p] = slots[p][:r]
            rec["ranks"] = ranks
            # (|p|, m, r) of every CPQR taken: the interface size, the columns
            # of C and the rank (a record only; no arithmetic depends on it)
            rec["cpqr_shapes"] = shapes
            if not scale:
                # sigma, R_ff, the dropped R_fn and W_fn blocks of every
                # interface without scaling (a record only)
                rec["unscaled"] = unscaled
        rec["sizes_post"] = np.array([len(s) for s in slots], dtype=np.int64)
        # ---------------- merge (Section 2.7) ----------------
        if k > 1:
            par = ordering.merge_parents(k)
            rec["merge_parent"] = par.copy()
            st2, en2, _, _ = ordering.stage_clusters(k - 1)
            nslots = [[] for _ in range(st2.size)]
            for c in range(st.size):
                if par[c] >= 0:
                    nslots[par[c]].append(slots[c])
            nslots = [np.concatenate(x) if x else np.zeros(0, np.int64) for x in nslots]
            # offset of each child inside its parent
            off = np.zeros(st.size, dtype=np.int64)
            fill = np.zeros(st2.size, dtype=np.int64)
            for c in range(st.size):
                if par[c] >= 0:
                    off[c] = fill[par[c]]
                    fill[par[c]] += len(slots[c])
            nbm = BlockMatrix()
            for (i, j), B in bm.blk.items():
                P, Q = int(par[i]), int(par[j])
                if P < 0 or Q < 0:
                    raise RuntimeError("block of an eliminated cluster survived")
                D = nbm.get(P, Q)
                if D is None:
                    D = np.zeros((len(nslots[P]), len(nslots[Q])))
                    nbm.set(P, Q, D)
                D[off[i]:off[i] + B.shape[0], off[j]:off[j] + B.shape[1]] = B
            bm = nbm
            slots = nslots
        F.stages[k] = rec
    F.max_skipped_update = max_skipped
    return F


def _forward_unscaled(op, yp):
    """H^T on the rows of p, then the last r rows (coarse) moved to the front (R12)."""
    _, k, p, sl, Vq, tq, r, VH, tH, Rff, Rfc = op
    z = apply_reflectors(VH, tH, yp, transpose=True)
    f = len(sl) - r
    return np.vstack([z[f:], z[:f]])


def apply(F, b):
    """x = M^{-1} b = D_c P^T W^{-1} Q^T P b (Section 2.8), b of shape (N,) or (N, nrhs)."""
    b = np.asarray(b, dtype=np.float64)
    one = b.ndim == 1
    X = b.reshape(F.N, -1)
    y = X[F.perm].copy()
    # forward sweep: left factors in elimination order
    for op in F.ops:
        kind = op[0]
        if kind == "front":
            _, k, s, rows, n, V, tau, Rss, cols, Rsj = op
            if n:
                y[rows] = apply_reflectors(V, tau, y[rows], transpose=True)
        elif kind == "scale":
            _, k, p, sl, V, tau, Rpp = op
            y[sl] = apply_reflectors(V, tau, y[sl], transpose=True)
        elif kind == "sparsify_u":
            y[op[3]] = _forward_unscaled(op, y[op[3]])
        else:
            _, k, p, sl, V, tau, r = op
            y[sl] = apply_reflectors(V, tau, y[sl], transpose=True)
    # backward sweep: right factors in reverse order
    for op in reversed(F.ops):
        kind = op[0]
        if kind == "front":
            _, k, s, rows, n, V, tau, Rss, cols, Rsj = op
            if n:
                ss = rows[:n]
                rhs = y[ss] - (Rsj @ y[cols] if cols.size else 0.0)
                y[ss] = sla.solve_triangular(Rss, rhs, lower=False)
        elif kind == "scale":
            _, k, p, sl, V, tau, Rpp = op
            y[sl] = sla.solve_triangular(Rpp, y[sl], lower=False)
        elif kind == "sparsify_u":
            # R_f^{-1} on [x_c; z_f], then Q_pp
            _, k, p, sl, Vq, tq, r, VH, tH, Rff, Rfc = op
            z = y[sl]
            xf = sla.solve_triangular(Rff, z[r:] - Rfc @ z[:r], lower=False)
            y[sl] = apply_reflectors(Vq, tq, np.vstack([z[:r], xf]), transpose=False)
        else:
            _, k, p, sl, V, tau, r = op
            y[sl] = apply_reflectors(V, tau, y[sl], transpose=False)
    x = np.empty_like(y)
    x[F.perm] = y
    x *= F.Dc[:, None]
    return x[:, 0] if one else x


def factor_bytes(F, itemsize=8):
    """Bytes of stored factors (V, tau, R blocks, U, Q) in the given precision."""
    tot = 0
    for op in F.ops:
        if op[0] == "front":
            _, k, s, rows, n, V, tau, Rss, cols, Rsj = op
            tot += (V.size + tau.size + Rss.size + Rsj.size) * itemsize
        elif op[0] == "scale":
            tot += (op[4].size + op[5].size + op[6].size) * itemsize
        elif op[0] == "sparsify_u":
            tot += sum(op[t].size for t in (4, 5, 7, 8, 9, 10)) * itemsize
        else:
            tot += (op[4].size + op[5].size) * itemsize
    return tot


def apply_qt(F, y):
    """Forward sweep only: y <- Q^T y in the permuted slot space (y: N x nrhs);
    an interface sparsified without scaling contributes its H^T and the
    coarse-first row order."""
    y = np.array(y, dtype=np.float64, copy=True).reshape(F.N, -1)
    for op in F.ops:
        if op[0] == "front":
            if op[4]:
                y[op[3]] = apply_reflectors(op[5], op[6], y[op[3]], transpose=True)
        elif op[0] == "sparsify_u":
            y[op[3]] = _forward_unscaled(op, y[op[3]])
        else:
            y[op[3]] = apply_reflectors(op[4], op[5], y[op[3]], transpose=True)
    return y


def assembled_r(F):
    """Dense block upper-triangular R (permuted index) assembled from the front
    factors; meaningful when no interface was scaled or sparsified."""
    R = np.zeros((F.N, F.N))
    for op in F.ops:
        if op[0] != "front":
            raise ValueError("scaled/sparsified factorization has no single R")
        _, k, s, rows, n, V, tau, Rss, cols, Rsj = op
        if n:
            ss = rows[:n]
            R[np.ix_(ss, ss)] = Rss
            if cols.size:
                R[np.ix_(ss, cols)] = Rsj
    return R
