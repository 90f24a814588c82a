"""The paper's own advection-diffusion test problems (Section 4), re-synthesized.

-div(a grad u) + q div(b u) = f on the unit square / cube, u = 0 on the
boundary, n^d interior points, h = 1/(n+1), lexicographic index
x + n y (+ n^2 z), every row multiplied by h^2:

  * centered differences for both terms (Section 4.2: "centered finite
    difference scheme"): diffusion with face coefficients (a_i + a_j)/2, and
    q div(b u) ~ q (b_{i+1} u_{i+1} - b_{i-1} u_{i-1}) / (2h) per axis with
    b evaluated at the neighbouring grid points;
  * b is a vector field: "b = 1" is read as b = (1, ..., 1) and
    "b = e^{x+y}" as b = e^{x+y} (1, 1) (the paper writes a scalar);
  * the high-contrast diffusivity of Section 4.1.1: a uniform U[0,1] field,
    smoothed by a Gaussian of unit width (one grid spacing, periodic FFT
    filter), then a = rho where the smoothed value is >= 0.5 and 1/rho
    elsewhere; b = 1, q = 1.

Inputs only: no spaQR arithmetic here.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


def _coords(dims):
    N = int(np.prod(dims))
    idx = np.arange(N, dtype=np.int64)
    strides = [1]
    for d in dims[:-1]:
        strides.append(strides[-1] * d)
    return N, idx, strides, [(idx // strides[ax]) % dims[ax] for ax in range(len(dims))]


def advdiff_centered(dims, q=1.0, b="one", a=None):
    """Centered-difference matrix of -div(a grad u) + q div(b u).

    dims: (n, n) or (n, n, n); q: convection magnitude; b: "one" (b = 1 in
    every direction), "exp" (b = e^{x+y} (1, 1), 2D) or a callable
    b(axis, coords_list) -> values at the points; a: None (a = 1) or an array
    of prod(dims) diffusivities.  CSR, int64 rowptr, int32 sorted columns."""
    dims = tuple(int(d) for d in dims)
    d = len(dims)
    if d not in (2, 3):
        raise ValueError("2D or 3D grids only")
    N, idx, strides, coords = _coords(dims)
    h = 1.0 / (dims[0] + 1)
    if any(abs(1.0 / (n + 1) - h) > 0 for n in dims):
        raise ValueError("the paper's grids are cubic: equal sides")
    af = np.ones(N) if a is None else np.asarray(a, dtype=np.float64).reshape(-1)
    xs = [(c + 1) * h for c in coords]          # point coordinates
    if b == "one":
        bval = [np.ones(N) for _ in range(d)]
    elif b == "exp":
        if d != 2:
            raise ValueError("b = e^{x+y} is the 2D problem")
        e = np.exp(xs[0] + xs[1])
        bval = [e, e]
    else:
        bval = [np.asarray(b(ax, xs), dtype=np.float64) for ax in range(d)]
    diag = np.zeros(N)
    rows, cols, vals = [], [], []
    for ax in range(d):
        for sgn in (-1, +1):
            nb = coords[ax] + sgn
            inside = (nb >= 0) & (nb < dims[ax])
            j = idx + sgn * strides[ax]
            face = af.copy()
            face[inside] = 0.5 * (af[inside] + af[j[inside]])
            diag += face                       # h^2 * (face / h^2)
            off = -face
            # q d(b u)/dx_ax ~ q (b_j u_j - b_k u_k) / (2h), times h^2
            conv = np.zeros(N)
            conv[inside] = sgn * q * bval[ax][j[inside]] * h / 2.0
            rows.append(idx[inside])
            cols.append(j[inside])
            vals.append((off + conv)[inside])
    rows.append(idx)
    cols.append(idx)
    vals.append(diag)
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))
    A.sum_duplicates()
    A.sort_indices()
    A.indptr = A.indptr.astype(np.int64)
    A.indices = A.indices.astype(np.int32)
    return A


def high_contrast_field(n, rho, rng, d=2):
    """a = rho where a unit-width Gaussian smoothing of U[0,1] noise is >= 0.5,
    1/rho elsewhere (n^d points, flattened with x fastest)."""
    w = rng.random((n,) * d)
    freqs = [np.fft.fftfreq(n) for _ in range(d)]
    grids = np.meshgrid(*freqs, indexing="ij")
    k2 = sum(g * g for g in grids)
    sm = np.real(np.fft.ifftn(np.fft.fftn(w) * np.exp(-2.0 * math.pi ** 2 * k2)))
    a = np.where(sm >= 0.5, float(rho), 1.0 / float(rho))
    # index (z, y, x) in C order -> flatten so that x is fastest
    return a.reshape(-1)


def paper_problem(kind, n, q=1.0, b="one", rho=1.0, seed=0):
    """kind 'ad2' (Section 4.2.1, centered FD, a = 1), 'ad3' (Section 4.2.2,
    a = b = q = 1) or 'hc' (Section 4.1.1, high contrast rho, b = q = 1)."""
    if kind == "ad2":
        return dict(A=advdiff_centered((n, n), q=q, b=b), dims=(n, n))
    if kind == "ad3":
        return dict(A=advdiff_centered((n, n, n), q=1.0, b="one"), dims=(n, n, n))
    if kind == "hc":
        a = high_contrast_field(n, rho, np.random.default_rng(seed))
        return dict(A=advdiff_centered((n, n), q=1.0, b="one", a=a), dims=(n, n))
    raise ValueError(kind)
