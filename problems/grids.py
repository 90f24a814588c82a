"""Upwind finite-difference convection-diffusion matrices on unit-square / unit-cube grids.

The paper's test problems are advection-diffusion equations
-div(a grad u) + q div(b u) = f on [0,1]^d with u = 0 on the boundary
(Section 4.1.1 and Section 4.2).  The workloads used here discretize
-div(a grad u) + beta . grad u with a 5-point (2D) or 7-point (3D) *upwind*
stencil, which keeps every row weakly diagonally dominant, so rows can be
clustered exactly like columns (Section 2.3).

Conventions (shared by the oracle and the engine; no spaQR arithmetic here):
  * n^d interior points, spacing h = 1/(n+1), lexicographic index
    i = x + n*y (+ n*n*z).  (Box grids use h_d = 1/(n_d+1) per axis and
    scale by min h_d^2; only pattern tests use them.)
  * diffusion uses face coefficients a_f = (a_i + a_j)/2; a face that leads to
    a Dirichlet neighbour uses a_f = a_i.
  * convection per axis d: beta_d > 0 -> h*beta_d*(u_i - u_{i-e_d});
    beta_d < 0 -> h*|beta_d|*(u_i - u_{i+e_d}).  The whole row is multiplied
    by h^2 so entries are O(1).
  * Dirichlet neighbours are dropped (their value is zero).
"""

from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


def _strides(dims):
    s = [1]
    for d in dims[:-1]:
        s.append(s[-1] * d)
    return s


def convdiff(dims, beta, a=None):
    """Assemble the upwind convection-diffusion matrix on a box grid.

    dims : tuple of ints, (nx, ny) or (nx, ny, nz); spacing h_d = 1/(n_d+1)
           per axis and the row is scaled by min_d h_d^2 (h^2 on cubic grids)
    beta : sequence of floats, one per axis
    a    : None (a = 1) or an array with prod(dims) entries, flattened so
           that a.ravel()[x + nx*y (+ nx*ny*z)] is the diffusivity at (x, y[, z]).
    Returns a CSR matrix with int32 column indices, int64 row pointers and
    sorted columns, no duplicates.
    """
    dims = tuple(int(d) for d in dims)
    d = len(dims)
    if d not in (2, 3):
        raise ValueError("2D or 3D grids only")
    hs = [1.0 / (n + 1) for n in dims]
    scale = min(hs) ** 2
    N = int(np.prod(dims))
    idx = np.arange(N, dtype=np.int64)
    strides = _strides(dims)
    coords = [(idx // strides[ax]) % dims[ax] for ax in range(d)]
    if a is None:
        af = np.ones(N)
    else:
        af = np.asarray(a, dtype=np.float64).reshape(-1)
        if af.shape[0] != N:
            raise ValueError("a has the wrong size")
    beta = [float(b) for b in beta]
    if len(beta) != d:
        raise ValueError("beta needs one entry per axis")

    diag = np.zeros(N)
    rows, cols, vals = [], [], []
    for ax in range(d):
        for sgn in (-1, +1):
            nb_coord = coords[ax] + sgn
            inside = (nb_coord >= 0) & (nb_coord < dims[ax])
            j = idx + sgn * strides[ax]
            # diffusion face coefficient
            face = af.copy()
            face[inside] = 0.5 * (af[inside] + af[j[inside]])
            face *= scale / hs[ax] ** 2
            hb = scale / hs[ax]
            diag += face
            off = -face
            # upwind convection
            b = beta[ax]
            if sgn < 0 and b > 0:
                diag += hb * b
                off = off - hb * b
            if sgn > 0 and b < 0:
                diag += hb * (-b)
                off = off - hb * (-b)
            rows.append(idx[inside])
            cols.append(j[inside])
            vals.append(off[inside])
    rows.append(idx)
    cols.append(idx)
    vals.append(diag)
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    A = sp.csr_matrix((v, (r, c)), shape=(N, N))
    A.sum_duplicates()
    A.sort_indices()
    A.indptr = A.indptr.astype(np.int64)
    A.indices = A.indices.astype(np.int32)
    return A


def smoothed_gaussian_field(n, d, corr_frac, rng):
    """White N(0,1) noise on an n^d grid, smoothed by a periodic Gaussian filter
    (FFT) of standard deviation corr_frac * n grid spacings, then standardized
    to mean 0 and standard deviation 1.  Shape (n,)*d in C order (z, y, x)."""
    w = rng.standard_normal((n,) * d)
    sigma = corr_frac * n
    freqs = [np.fft.fftfreq(n) for _ in range(d)]
    grids = np.meshgrid(*freqs, indexing="ij")
    k2 = sum(g * g for g in grids)
    filt = np.exp(-2.0 * (math.pi ** 2) * (sigma ** 2) * k2)
    g = np.real(np.fft.ifftn(np.fft.fftn(w) * filt))
    g = (g - g.mean()) / g.std()
    return g


def perturb_offdiagonals(A, frac, lo, hi, rng):
    """Multiply each off-diagonal entry, independently with probability `frac`,
    by a factor drawn from U[lo, hi].  Draws happen in CSR order."""
    A = A.copy()
    rowid = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    off = np.nonzero(A.indices != rowid)[0]
    mask = rng.random(off.shape[0]) < frac
    fac = rng.uniform(lo, hi, off.shape[0])
    sel = off[mask]
    A.data[sel] *= fac[mask]
    return A


def make_rhs(N, nrhs=1, seed=0):
    """b ~ U[-1, 1], column-major (N, nrhs) float64, from PCG64 seeded with (seed, 1)."""
    rng = np.random.default_rng([int(seed), 1])
    return np.asfortranarray(rng.uniform(-1.0, 1.0, size=(N, nrhs)))


def default_levels(N):
    """Number of nested-dissection levels ceil(log2(N/64)) (Section 4, setup)."""
    return max(1, int(math.ceil(math.log(N / 64.0) / math.log(2.0))))


# Workload definitions.  Each returns a dict with the CSR matrix, grid dims,
# number of ND levels and the tolerances the workload is quoted at.
def _c1(seed):
    n = 32
    A = convdiff((n, n), (10.0, 10.0))
    return dict(name="c1", A=A, dims=(n, n), levels=5, eps=(0.0, 1e-3))


def _c2(seed):
    n = 256
    rng = np.random.default_rng(int(seed))
    t = rng.uniform(0.0, 2.0 * math.pi)
    g = smoothed_gaussian_field(n, 2, 1.0 / 16.0, rng)
    A = convdiff((n, n), (50.0 * math.cos(t), 50.0 * math.sin(t)), a=np.exp(g))
    return dict(name="c2", A=A, dims=(n, n), levels=default_levels(n * n),
                eps=(1e-2, 1e-4, 1e-6))


def _c3(seed):
    n = 64
    A = convdiff((n, n, n), (20.0, 20.0, 20.0))
    return dict(name="c3", A=A, dims=(n, n, n), levels=12, eps=(1e-2,))


def _c4(seed):
    n = 1024
    rng = np.random.default_rng(int(seed))
    A = convdiff((n, n), (500.0, -300.0))
    A = perturb_offdiagonals(A, 0.05, 0.5, 1.5, rng)
    return dict(name="c4", A=A, dims=(n, n), levels=14, eps=(1e-2,))


def _grid(dim, side, beta, seed=0):
    dims = (side,) * dim
    A = convdiff(dims, beta)
    return dict(name=f"grid{dim}d_{side}", A=A, dims=dims,
                levels=default_levels(side ** dim), eps=(1e-2,))


CONFIGS = {"c1": _c1, "c2": _c2, "c3": _c3, "c4": _c4}


def config_problem(name, seed=0, **kw):
    """Build one of the named workloads ('c1'..'c4'), or a plain grid
    ('grid', dim=.., side=.., beta=..)."""
    if name == "grid":
        return _grid(kw["dim"], kw["side"], kw["beta"], seed)
    return CONFIGS[name](seed)
