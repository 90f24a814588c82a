"""Estimate of ||A^{-1}||_2 for a sparse square A -- test infrastructure.

Used to turn the stopping rule of GMRES (Section 4: ||A x - b|| / ||b|| <= tol)
into a bound on the distance between two converged solutions:
||x - x'|| <= ||A^{-1}||_2 (||r|| + ||r'||).  Inverse power iteration on
A^T A with a sparse LU of A (SuperLU through SciPy, a library primitive):
v <- A^{-1} A^{-T} v, normalized; the Rayleigh quotient after `iters` steps
is a lower estimate of ||A^{-1}||_2^2 that converges from below.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def inv_norm2_estimate(A, iters=30, seed=0):
    A = sp.csc_matrix(A, dtype=np.float64)
    lu = spla.splu(A)
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(A.shape[0])
    v /= np.linalg.norm(v)
    est = 0.0
    for _ in range(iters):
        w = lu.solve(lu.solve(v, trans="T"))
        nw = float(np.linalg.norm(w))
        if nw == 0.0:
            break
        est = nw
        v = w / nw
    return float(np.sqrt(est))
