"""Seeded sparse matrices without a grid, for the algebraic ordering.

  delaunay_convdiff  convection-diffusion on the Delaunay triangulation of
                     uniform random points in the unit square: for every
                     mesh edge (i, j) a diffusion weight 1 plus an upwind
                     convection weight max(0, -beta . (p_j - p_i) / |p_j - p_i|),
                     a_ij = -(that sum); the diagonal is the sum of the row's
                     off-diagonal magnitudes plus 1e-2 (strictly diagonally
                     dominant, so nonsingular and unsymmetric for beta != 0)
  permuted           P A P^T for a seeded random permutation P: a grid matrix
                     whose index carries no geometry

Inputs only: no arithmetic of the method lives here.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def delaunay_convdiff(npts, beta=(10.0, 5.0), seed=0):
    from scipy.spatial import Delaunay
    rng = np.random.default_rng([seed, 11])
    pts = rng.random((int(npts), 2))
    tri = Delaunay(pts)
    s = tri.simplices
    e = np.concatenate([s[:, [0, 1]], s[:, [1, 2]], s[:, [2, 0]]])
    e = np.concatenate([e, e[:, ::-1]])
    e = np.unique(e, axis=0)
    i, j = e[:, 0], e[:, 1]
    d = pts[j] - pts[i]
    dn = d / np.linalg.norm(d, axis=1)[:, None]
    conv = np.maximum(0.0, -(dn @ np.asarray(beta, dtype=np.float64)))
    off = -(1.0 + conv)
    n = pts.shape[0]
    A = sp.csr_matrix((off, (i, j)), shape=(n, n))
    diag = np.asarray(abs(A).sum(axis=1)).ravel() + 1e-2
    A = (A + sp.diags(diag)).tocsr()
    A.sort_indices()
    return A


def permuted(A, seed=0):
    """P A P^T with a seeded random permutation; returns (matrix, perm) with
    row/column t of the result = row/column perm[t] of A."""
    rng = np.random.default_rng([seed, 13])
    p = rng.permutation(A.shape[0])
    B = sp.csr_matrix(A)[p][:, p].tocsr()
    B.sort_indices()
    return B, p
