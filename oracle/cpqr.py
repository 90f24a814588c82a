"""Partial column-pivoted Householder QR with the ratio rank rule -- oracle.

Businger-Golub pivoting, as LAPACK's xLAQPS/xGEQP3 perform it, stopped by the
rule of Section 4 (setup): the rank r is the number of leading steps i with
|R_ii| / |R_11| >= eps.  Readings:
  * column norms are recomputed exactly at every step (no downdating);
  * the pivot is the trailing column of largest norm, ties -> lowest current
    position (the first maximum, as IDAMAX returns);
  * r = 0 if there are no columns or |R_11| = 0; with eps = 0 all
    min(rows, cols) steps are taken;
  * reflectors follow LAPACK's xLARFG convention: beta = -sign(alpha)*||x||,
    tau = (beta - alpha)/beta, v = [1, x_tail/(alpha - beta)], tau = 0 when the
    tail is zero.
"""

from __future__ import annotations

import math

import numpy as np


def householder(x):
    """Return (v, tau, beta) with (I - tau v v^T) x = beta e_1 and v[0] = 1."""
    alpha = float(x[0])
    tail = x[1:]
    xn = float(np.sqrt(np.dot(tail, tail)))
    v = np.zeros_like(x, dtype=np.float64)
    v[0] = 1.0
    if xn == 0.0:
        return v, 0.0, alpha
    beta = -math.copysign(math.hypot(alpha, xn), alpha)
    tau = (beta - alpha) / beta
    v[1:] = tail / (alpha - beta)
    return v, tau, beta


def cpqr_ratio(C, eps):
    """Partial CPQR of C (P x m) stopped by the ratio rule.

    Returns (r, V, tau, W, rdiag, piv):
      r      rank
      V      P x r Householder vectors (unit first entry on the diagonal)
      tau    r scalars
      W      r x m, the first r rows of Q^T C in the ORIGINAL column order
      rdiag  |R_ii| for i < r
      piv    column permutation of the first r steps (piv[k] = original column)
    """
    C = np.array(C, dtype=np.float64, copy=True)
    P, m = C.shape
    piv = np.arange(m)
    kmax = min(P, m)
    V = np.zeros((P, kmax))
    tau = np.zeros(kmax)
    rdiag = []
    r = 0
    R11 = 0.0
    for k in range(kmax):
        norms = np.einsum("ij,ij->j", C[k:, k:], C[k:, k:])
        j = k + int(np.argmax(norms))
        rkk = math.sqrt(float(norms[j - k]))
        if k == 0:
            R11 = rkk
            if R11 == 0.0:
                break
        if eps > 0.0 and rkk < eps * R11:
            break
        if j != k:
            C[:, [k, j]] = C[:, [j, k]]
            piv[[k, j]] = piv[[j, k]]
        v, t, beta = householder(C[k:, k])
        C[k, k] = beta
        C[k + 1:, k] = 0.0
        if k + 1 < m:
            w = v @ C[k:, k + 1:]
            C[k:, k + 1:] -= t * np.outer(v, w)
        V[k:, k] = v
        tau[k] = t
        rdiag.append(abs(beta))
        r = k + 1
    W = np.zeros((r, m))
    W[:, piv] = C[:r, :]
    return r, V[:, :r].copy(), tau[:r].copy(), W, np.array(rdiag), piv[:r].copy()


def apply_reflectors(V, tau, X, transpose):
    """X <- Q^T X (transpose=True) or Q X, with Q = H_0 H_1 ... H_{r-1},
    H_t = I - tau_t v_t v_t^T and v_t = V[:, t] (zero above row t)."""
    X = np.array(X, dtype=np.float64, copy=True)
    r = V.shape[1]
    order = range(r) if transpose else range(r - 1, -1, -1)
    for t in order:
        if tau[t] == 0.0:
            continue
        v = V[t:, t]
        X[t:] -= tau[t] * np.outer(v, v @ X[t:])
    return X
