"""Right-preconditioned flexible GMRES -- FP64 oracle.

The paper solves Ax = b with GMRES preconditioned by the spaQR factors and
stops at ||Ax - b|| / ||b|| <= tol (Section 4).  Readings: flexible GMRES
(stores z_j = M^{-1} v_j, identical to right-preconditioned GMRES for a fixed
linear M), x0 = 0, modified Gram-Schmidt, Givens rotations, restart 100,
at most 1000 Arnoldi steps; the restart loop stops on the estimate
|g_{j+1}| / ||b|| <= tol, then recomputes the true residual and restarts from
x if that misses tol.  The iteration count is the total number of Arnoldi
steps.
"""

from __future__ import annotations

import math

import numpy as np


def fgmres(matvec, precond, b, tol=1e-10, restart=100, maxit=1000):
    b = np.asarray(b, dtype=np.float64)
    N = b.shape[0]
    x = np.zeros(N)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return x, 0, 0.0
    it = 0
    r = b.copy()
    rel = 1.0
    while True:
        beta = float(np.linalg.norm(r))
        rel = beta / bnorm
        if rel <= tol or it >= maxit:
            break
        m = restart
        V = np.zeros((N, m + 1))
        Z = np.zeros((N, m))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[:, 0] = r / beta
        jend = 0
        for j in range(m):
            Z[:, j] = precond(V[:, j])
            w = matvec(Z[:, j])
            it += 1
            for i in range(j + 1):
                H[i, j] = float(V[:, i] @ w)
                w = w - H[i, j] * V[:, i]
            H[j + 1, j] = float(np.linalg.norm(w))
            if H[j + 1, j] > 0.0:
                V[:, j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = math.hypot(H[j, j], H[j + 1, j])
            if den == 0.0:
                cs[j], sn[j] = 1.0, 0.0
            else:
                cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            jend = j + 1
            if abs(g[j + 1]) / bnorm <= tol or it >= maxit or H[j, j] == 0.0:
                break
        y = np.zeros(jend)
        for i in range(jend - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:jend] @ y[i + 1:jend]) / H[i, i]
        x = x + Z[:, :jend] @ y
        r = b - matvec(x)
    return x, it, rel
