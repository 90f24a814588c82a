"""Pins for the oracle's spaQR factorization, apply, CPQR and GMRES.

Each pin checks the oracle against something other than itself: exactness of
the factorization at eps = 0 (Section 3: with no sparsification spaQR is
nested-dissection Householder QR), a dense Householder QR of the whole
matrix, LAPACK's column-pivoted QR, numpy's dense solve, orthogonality, the
truncation bound of the ratio rule, and SciPy's GMRES.
"""

import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from problems import convdiff, config_problem, make_rhs
from oracle.ordering import order_grid
from oracle import spaqr, gmres
from oracle.cpqr import cpqr_ratio, apply_reflectors


def _ahat(A, F):
    Dc = F.Dc
    Ah = (sp.csr_matrix(A) @ sp.diags(Dc)).tocsr()
    return Ah[F.perm][:, F.perm].toarray()


@pytest.mark.parametrize("dims,L,beta", [((32, 32), 5, (10.0, 10.0)),
                                          ((8, 8, 8), 4, (20.0, -5.0, 3.0)),
                                          ((24, 24), 5, (-40.0, 7.0))])
def test_eps0_exact_solve(dims, L, beta):
    """eps = 0: M^{-1} = A^{-1} up to roundoff (relative residual <= 1e-13)."""
    A = convdiff(dims, beta)
    o = order_grid(dims, L)
    F = spaqr.factor(A, o, 0.0, check_skipped=True)
    b = make_rhs(A.shape[0], 2, seed=3)
    x = spaqr.apply(F, b)
    res = np.linalg.norm(A @ x - b, axis=0) / np.linalg.norm(b, axis=0)
    assert res.max() <= 1e-13
    # the skipped non-ancestor updates are zero up to roundoff (Lemma 2)
    assert F.max_skipped_update <= 1e-13


@pytest.mark.parametrize("dims,L", [((16, 16), 4), ((6, 6, 6), 3)])
def test_solution_matches_dense_solve(dims, L):
    A = convdiff(dims, (7.0,) * len(dims))
    o = order_grid(dims, L)
    F = spaqr.factor(A, o, 0.0)
    b = make_rhs(A.shape[0], 1, seed=1)[:, 0]
    x = spaqr.apply(F, b)
    xd = np.linalg.solve(A.toarray(), b)
    assert np.linalg.norm(x - xd) <= 1e-12 * np.linalg.norm(xd)


@pytest.mark.parametrize("dims,L", [((16, 16), 4), ((12, 12), 4), ((6, 6, 6), 3)])
def test_direct_r_matches_dense_qr(dims, L):
    """No scaling, no sparsification (skip >= L): the assembled block R equals
    the R of a dense Householder QR of the permuted, pre-scaled matrix up to
    row signs (QR is unique up to signs; R^T R = A^T A)."""
    A = convdiff(dims, (5.0, -9.0, 2.0)[:len(dims)])
    o = order_grid(dims, L)
    F = spaqr.factor(A, o, 0.0, skip=L + 1)
    R = spaqr.assembled_r(F)
    Ah = _ahat(A, F)
    Rd = np.linalg.qr(Ah, mode="r")
    assert np.allclose(np.abs(R), np.abs(Rd), rtol=0, atol=1e-12 * np.abs(Rd).max())
    # and R^T R = A^T A
    assert np.allclose(R.T @ R, Ah.T @ Ah, atol=1e-12)


def test_front_reflectors_orthogonal():
    A = convdiff((16, 16), (3.0, 4.0))
    o = order_grid((16, 16), 4)
    F = spaqr.factor(A, o, 1e-3)
    worst = 0.0
    for op in F.ops:
        V, tau = (op[5], op[6]) if op[0] == "front" else (op[4], op[5])
        if V.shape[1] == 0:
            continue
        Q = apply_reflectors(V, tau, np.eye(V.shape[0]), transpose=False)
        worst = max(worst, np.abs(Q.T @ Q - np.eye(Q.shape[0])).max())
    assert worst <= 1e-13


def test_qt_preserves_norms():
    A = convdiff((24, 24), (30.0, -10.0))
    o = order_grid((24, 24), 5)
    F = spaqr.factor(A, o, 1e-2)
    v = make_rhs(A.shape[0], 3, seed=9)
    w = spaqr.apply_qt(F, v)
    assert np.allclose(np.linalg.norm(w, axis=0), np.linalg.norm(v, axis=0), rtol=1e-13)


def _dense_u(V, tau):
    """U = H_0 H_1 ... H_{r-1} as a dense matrix, H_t = I - tau_t v_t v_t^T
    (formed here with plain matrix products, independently of the oracle)."""
    P = V.shape[0]
    U = np.eye(P)
    for t in range(V.shape[1]):
        v = V[:, t:t + 1]
        U = U @ (np.eye(P) - tau[t] * (v @ v.T))
    return U


def test_scaling_transforms_the_prescaling_blocks():
    """Section 2.6 on the real blocks of a factorization: with the block
    dictionary captured just before and just after the scaling step of every
    sparsified stage,
      * the diagonal block before scaling satisfies U_pp^T A_pp R_pp^{-1} = I
        (A_pp from the snapshot; U_pp built densely from the stored
        reflectors, R_pp the stored factor);
      * a block (p, j) became U_pp^T A_pj, a block (i, p) became A_ip R_pp^{-1},
        a block between two scaled interfaces U_p^T A_pq R_q^{-1} (left
        before right), and A_pp became I;
      * blocks of clusters that were not scaled are untouched (none occur
        here: after the fronts of level k every remaining cluster is an
        interface of a separator above k, and all of them scale)."""
    A = convdiff((24, 24), (30.0, -10.0))
    o = order_grid((24, 24), 5)
    snaps = {}

    def trace(k, event, blocks):
        snaps[(k, event)] = blocks

    F = spaqr.factor(A, o, 1e-2, trace=trace)
    stages = sorted({k for k, _ in snaps})
    assert stages
    nblk = nboth = 0
    for k in stages:
        pre, post = snaps[(k, "before_scaling")], snaps[(k, "after_scaling")]
        assert set(pre) == set(post)
        fac = {op[2]: (_dense_u(op[4], op[5]), op[6]) for op in F.ops if op[0] == "scale" and op[1] == k}
        assert fac
        for p, (U, R) in fac.items():
            M = np.linalg.solve(R.T, (U.T @ pre[(p, p)]).T).T
            assert np.abs(M - np.eye(R.shape[0])).max() <= 1e-12 * np.linalg.cond(R)
        for (i, j), B in pre.items():
            if i == j and i in fac:
                assert np.array_equal(post[(i, j)], np.eye(B.shape[0]))
                continue
            want = B
            if i in fac:
                want = fac[i][0].T @ want
            if j in fac:
                want = np.linalg.solve(fac[j][1].T, want.T).T
            scale = max(1.0, np.abs(want).max()) * (np.linalg.cond(fac[j][1]) if j in fac else 1.0)
            assert np.abs(post[(i, j)] - want).max() <= 1e-13 * scale, (k, i, j)
            nblk += 1
            nboth += (i in fac) and (j in fac)
    assert nblk > 0 and nboth > 0


def test_same_colour_items_touch_disjoint_blocks():
    """R5 and R8: fronts of one colour update disjoint blocks and none of
    them reads a block another one of the colour writes; interfaces of one
    colour read and write disjoint sets of blocks."""
    A = convdiff((12, 12, 12), (5.0, 5.0, 5.0))
    o = order_grid((12, 12, 12), 6)
    F = spaqr.factor(A, o, 1e-2)
    checked_f = checked_i = 0
    for k, rec in F.stages.items():
        by_c = {}
        for s, (n1, cols, c) in rec["fronts"].items():
            writes = {(i, j) for i in n1 for j in cols}
            reads = {(r, j) for r in [s] + n1 for j in [s] + cols}
            by_c.setdefault(c, []).append((writes, reads))
        for items in by_c.values():
            for a in range(len(items)):
                for b in range(len(items)):
                    if a != b:
                        assert not (items[a][0] & items[b][0])
                        assert not (items[a][0] & items[b][1])
                        checked_f += 1
        if not rec["sparsified"]:
            continue
        pattern = set(rec["pattern_post"])
        touch = {}
        for p, c in rec["iface_colour"].items():
            t = {(i, j) for (i, j) in pattern if i == p or j == p}
            touch.setdefault(c, []).append(t)
        for items in touch.values():
            for a in range(len(items)):
                for b in range(a + 1, len(items)):
                    assert not (items[a] & items[b])
                    checked_i += 1
    assert checked_f > 0 and checked_i > 0


def test_order_inside_a_colour_does_not_change_the_result():
    """O8 / R5: processing the fronts and interfaces of every colour in
    descending instead of ascending id gives bitwise the same factors and the
    same M^{-1} b."""
    A = convdiff((12, 12, 12), (5.0, 5.0, 5.0))
    o = order_grid((12, 12, 12), 6)
    Fa = spaqr.factor(A, o, 1e-2)
    Fd = spaqr.factor(A, o, 1e-2, within_colour="descending")
    key = lambda op: (op[0], -op[1], op[2])  # noqa: E731
    oa, od = sorted(Fa.ops, key=key), sorted(Fd.ops, key=key)
    assert len(oa) == len(od)
    for x, y in zip(oa, od):
        assert key(x) == key(y)
        for u, v in zip(x[3:], y[3:]):
            assert np.array_equal(np.asarray(u), np.asarray(v))
    b = make_rhs(A.shape[0], 2, seed=4)
    assert np.array_equal(spaqr.apply(Fa, b), spaqr.apply(Fd, b))


# ----------------------------------------------------------------------------
# CPQR with the ratio rule (Section 4 setup: |R_ii| / |R_11| >= eps)
def _decaying(rng, P, m, rate):
    U, _ = np.linalg.qr(rng.standard_normal((P, P)))
    Vt, _ = np.linalg.qr(rng.standard_normal((m, m)))
    k = min(P, m)
    s = rate ** np.arange(k)
    S = np.zeros((P, m))
    S[np.arange(k), np.arange(k)] = s
    return U @ S @ Vt.T


@pytest.mark.parametrize("P,m,rate,eps", [(30, 80, 0.7, 1e-3), (40, 25, 0.5, 1e-6),
                                          (12, 200, 0.9, 1e-2), (25, 60, 0.6, 0.0)])
def test_cpqr_rank_matches_lapack(P, m, rate, eps):
    rng = np.random.default_rng(P * m)
    C = _decaying(rng, P, m, rate)
    r, V, tau, W, rdiag, piv = cpqr_ratio(C, eps)
    # LAPACK dgeqp3 (norm downdating) under the same rule
    _, Rl, pl = sla.qr(C, pivoting=True)
    d = np.abs(np.diag(Rl))
    if eps == 0.0:
        rl = min(P, m)
    else:
        ok = d >= eps * d[0]
        rl = int(np.argmin(ok)) if not ok.all() else ok.size
    assert r == rl
    assert np.allclose(rdiag, d[:r], rtol=1e-10)
    assert np.all(np.diff(rdiag) <= 1e-12 * rdiag[0])
    # Q orthogonal
    Q = apply_reflectors(V, tau, np.eye(P), transpose=False)
    assert np.abs(Q.T @ Q - np.eye(P)).max() <= 1e-13
    # W = first r rows of Q^T C, and the dropped rows obey the stopping rule
    QtC = apply_reflectors(V, tau, C, transpose=True)
    assert np.allclose(QtC[:r], W, atol=1e-13 * np.abs(C).max())
    if eps > 0 and r < min(P, m):
        dropped = np.linalg.norm(QtC[r:])
        assert dropped <= math.sqrt(m - r) * eps * rdiag[0] * (1 + 1e-12)


def test_cpqr_degenerate():
    r, V, tau, W, rdiag, piv = cpqr_ratio(np.zeros((5, 0)), 1e-2)
    assert r == 0 and W.shape == (0, 0)
    r, *_ = cpqr_ratio(np.zeros((5, 7)), 1e-2)
    assert r == 0
    # exact rank 2, eps tiny
    rng = np.random.default_rng(0)
    C = rng.standard_normal((6, 2)) @ rng.standard_normal((2, 9))
    r, *_ = cpqr_ratio(C, 1e-10)
    assert r == 2
    # ties resolve to the lowest index
    r, V, tau, W, rdiag, piv = cpqr_ratio(np.eye(4), 0.5)
    assert r == 4 and list(piv) == [0, 1, 2, 3]


# ----------------------------------------------------------------------------
def test_preconditioner_error_shrinks_with_eps():
    """||I - M^{-1} A|| = O(eps) (Section 3.3): it must shrink as eps does."""
    dims = (20, 20)
    A = convdiff(dims, (25.0, 12.0))
    o = order_grid(dims, 5)
    Ad = A.toarray()
    errs = []
    for eps in (1e-2, 1e-4, 1e-6):
        F = spaqr.factor(A, o, eps)
        MA = spaqr.apply(F, Ad)
        errs.append(np.linalg.norm(np.eye(A.shape[0]) - MA, 2))
    assert errs[0] > errs[1] > errs[2]
    assert errs[1] < 0.1 * errs[0] and errs[2] < 0.1 * errs[1]
    E = errs[1]
    if E < 1:
        # kappa(M^{-1}A) <= (1 + ||E||) / (1 - ||E||)
        F = spaqr.factor(A, o, 1e-4)
        s = np.linalg.svd(spaqr.apply(F, Ad), compute_uv=False)
        assert s[0] / s[-1] <= (1 + E) / (1 - E) * (1 + 1e-8)


def test_gmres_one_iteration_at_eps0():
    P = config_problem("c1")
    A = P["A"]
    o = order_grid(P["dims"], P["levels"])
    F = spaqr.factor(A, o, 0.0)
    b = make_rhs(A.shape[0], 1, seed=0)[:, 0]
    x, it, rel = gmres.fgmres(lambda v: A @ v, lambda v: spaqr.apply(F, v), b, 1e-10)
    assert it == 1 and np.linalg.norm(A @ x - b) / np.linalg.norm(b) <= 1e-12


@pytest.mark.parametrize("eps", [1e-2, 1e-3])
def test_gmres_matches_scipy(eps):
    """Iteration counts equal SciPy's GMRES on the right-preconditioned operator
    A M^{-1} (same Krylov space) within +-1."""
    dims = (32, 32)
    A = convdiff(dims, (60.0, -25.0))
    o = order_grid(dims, 5)
    F = spaqr.factor(A, o, eps)
    b = make_rhs(A.shape[0], 1, seed=2)[:, 0]
    x, it, rel = gmres.fgmres(lambda v: A @ v, lambda v: spaqr.apply(F, v), b, 1e-10)
    assert np.linalg.norm(A @ x - b) / np.linalg.norm(b) <= 1e-10
    N = A.shape[0]
    op = spla.LinearOperator((N, N), matvec=lambda u: A @ spaqr.apply(F, u))
    count = [0]

    def cb(_):
        count[0] += 1

    u, info = spla.gmres(op, b, rtol=1e-10, atol=0.0, restart=100, maxiter=10,
                         callback=cb, callback_type="pr_norm")
    assert info == 0
    assert abs(count[0] - it) <= 1


def test_iterations_flat_in_n():
    """Counts stay nearly flat as the grid grows at eps = 1e-2 (Section 4.2)."""
    its = []
    for n in (64, 128, 192):
        A = convdiff((n, n), (50.0, 50.0))
        o = order_grid((n, n), max(1, math.ceil(math.log2(n * n / 64))))
        F = spaqr.factor(A, o, 1e-2)
        b = make_rhs(A.shape[0], 1, seed=0)[:, 0]
        _, it, rel = gmres.fgmres(lambda v: A @ v, lambda v: spaqr.apply(F, v), b, 1e-10)
        assert rel <= 1e-10
        its.append(it)
    assert max(its) <= 2 * min(its) + 2


def test_symbolic_pattern_invariants():
    """Blocks only ever join ancestor-related clusters, and the fronts of one
    colour update disjoint blocks."""
    dims = (32, 32)
    A = convdiff(dims, (10.0, 10.0))
    o = order_grid(dims, 5)
    F = spaqr.factor(A, o, 1e-3)
    for k, rec in F.stages.items():
        st, en, nd, lv = rec["clusters"]
        for (i, j) in rec["pattern_post"]:
            a, b = nd[i], nd[j]
            assert a == b or o.is_ancestor(a, b) or o.is_ancestor(b, a)
        byc = {}
        for s, (n1, cols, c) in rec["fronts"].items():
            touched = {(i, j) for i in n1 for j in cols}
            for other in byc.get(c, []):
                assert not (touched & other)
            byc.setdefault(c, []).append(touched)


# ----------------------------------------------------------------------------
# sparsification without scaling (Section 2.5, Lemma 1)
def _unscaled_case(eps=1e-4, dims=(24, 24), L=5):
    A = convdiff(dims, (25.0, 12.0))
    o = order_grid(dims, L)
    return A, o, spaqr.factor(A, o, eps, scale=False)


def test_unscaled_sigma_is_the_inverse_smallest_singular_value():
    """sigma = 1/sigma_min(A_p) (Lemma 1), checked against A_p assembled
    densely: at the first sparsified stage the p columns of A_p are the p
    columns of Q^T A_hat (the front reflectors applied to the dense permuted,
    pre-scaled matrix) over the rows not yet eliminated.  Interfaces of the
    first colour see no earlier sparsification."""
    A, o, F = _unscaled_case()
    k0 = max(k for k, rec in F.stages.items() if rec["sparsified"])
    rec = F.stages[k0]
    Ah = _ahat(A, F)
    fronts = [op for op in F.ops if op[0] == "front" and op[1] >= k0]
    Y = Ah.copy()
    for op in fronts:
        if op[4]:
            Y[op[3]] = apply_reflectors(op[5], op[6], Y[op[3]], transpose=True)
    elim = np.zeros(F.N, dtype=bool)
    for op in fronts:
        elim[op[3][:op[4]]] = True
    st, en, _, _ = rec["clusters"]
    checked = 0
    for p, info in rec["unscaled"].items():
        if rec["iface_colour"][p] != 0:
            continue
        cols = np.arange(st[p], en[p])  # stage-k0 clusters still own their initial slots here
        cols = cols[~elim[cols]]
        Ap = Y[np.ix_(~elim, cols)]
        smin = np.linalg.svd(Ap, compute_uv=False)[-1]
        assert abs(info["sigma"] * smin - 1.0) <= 1e-10
        checked += 1
    assert checked >= 2


def test_unscaled_lemma1_identity_and_bound():
    """Proof of Lemma 1: sigma R_ff^T R_fn = W_fn^(2) exactly (A_pp Q_pf = H_ff
    R_ff), and ||R_fn|| <= ||W_fn^(2)|| / (1 - sigma ||W_fn^(1)||) because
    sigma_min(R_ff) >= sigma_min(A_p) - ||A_np Q_pf||."""
    n = 0
    for eps in (1e-2, 1e-4):
        A, o, F = _unscaled_case(eps)
        for k, rec in F.stages.items():
            for p, info in rec.get("unscaled", {}).items():
                if "R_ff" not in info:
                    continue
                sig, Rff, Rfn, W1, W2 = info["sigma"], info["R_ff"], info["R_fn"], info["W_f1"], info["W_f2"]
                if Rfn.size == 0:
                    continue
                lhs = sig * Rff.T @ Rfn
                scale = sig * np.linalg.norm(Rff, 2) * np.linalg.norm(Rfn, 2) + np.linalg.norm(W2, 2) + 1e-300
                assert np.abs(lhs - W2).max() <= 1e-12 * scale
                w1 = sig * np.linalg.norm(W1, 2) if W1.size else 0.0
                if w1 < 0.5:
                    assert np.linalg.norm(Rfn, 2) <= np.linalg.norm(W2, 2) / (1.0 - w1) * (1 + 1e-10) + 1e-15
                n += 1
    assert n >= 6


def test_unscaled_preconditioner_error_shrinks_with_eps():
    """||I - M^{-1} A|| = O(eps) without scaling too; at eps = 0 M^{-1} = A^{-1}."""
    dims = (20, 20)
    A = convdiff(dims, (25.0, 12.0))
    o = order_grid(dims, 5)
    Ad = A.toarray()
    errs = []
    for eps in (1e-2, 1e-4, 1e-6, 1e-8):
        F = spaqr.factor(A, o, eps, scale=False)
        assert any(op[0] == "sparsify_u" for op in F.ops)
        errs.append(np.linalg.norm(np.eye(A.shape[0]) - spaqr.apply(F, Ad), 2))
    assert all(errs[t + 1] < 0.1 * errs[t] for t in range(3))
    assert errs[3] <= 1e-4
    F = spaqr.factor(A, o, 0.0, scale=False)
    b = make_rhs(A.shape[0], 2, seed=5)
    x = spaqr.apply(F, b)
    assert (np.linalg.norm(A @ x - b, axis=0) / np.linalg.norm(b, axis=0)).max() <= 1e-13


def test_unscaled_gmres_converges_and_scaling_helps():
    """Both variants precondition FGMRES to 1e-10 (Section 4 setup); on this
    advection-dominated case the scaled variant needs no more iterations
    (the comparison of Section 4.1)."""
    dims = (32, 32)
    A = convdiff(dims, (40.0, -25.0))
    o = order_grid(dims, 5)
    b = make_rhs(A.shape[0], 1, seed=2)[:, 0]
    its = {}
    for sc in (True, False):
        F = spaqr.factor(A, o, 1e-2, scale=sc)
        x, it, rel = gmres.fgmres(lambda v: A @ v, lambda v: spaqr.apply(F, v), b, 1e-10)
        assert np.linalg.norm(A @ x - b) <= 1e-9 * np.linalg.norm(b)
        its[sc] = it
    assert its[True] <= its[False]


def test_unscaled_ranks_move_under_roundoff_level_perturbation():
    """Without scaling, at eps = 1e-6 the ranks of later sparsified stages
    change when A's entries are perturbed by 1e-13 relative, while the scaled
    variant's do not (the robustness Section 2.6's scaling buys).  This sets
    the GPU parity bar for the unscaled FP64 path at small eps to +-1."""
    dims, L, eps = (96, 96), 7, 1e-6
    A = sp.csr_matrix(convdiff(dims, (25.0, 12.0)))
    A1 = A.copy()
    A1.data = A1.data * (1 + 1e-13 * np.random.default_rng(0).standard_normal(A1.data.size))
    o = order_grid(dims, L)
    moved = {}
    for sc in (True, False):
        F0, F1 = spaqr.factor(A, o, eps, scale=sc), spaqr.factor(A1, o, eps, scale=sc)
        moved[sc] = [abs(F1.stages[k]["ranks"][p] - r) for k, rec in F0.stages.items() if rec["sparsified"]
                     for p, r in rec["ranks"].items()]
    assert max(moved[True]) == 0
    assert 0 < max(moved[False]) <= 1
