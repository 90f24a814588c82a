"""Seeded request trace for the serving workload: Poisson arrivals of fresh
2D/3D convection-diffusion problems with several right-hand sides each."""

from __future__ import annotations

import math

import numpy as np

from .grids import convdiff, make_rhs


def serving_trace(nreq=512, seed=0, rate=100.0, side2d=(64, 512), side3d=(16, 48),
                  beta_mag=(1.0, 200.0), nrhs=(1, 32), eps=1e-2):
    """Return a list of request descriptors (the matrices are built lazily by
    `build_request`).  Arrival gaps are exponential with the given rate (1/s).
    A request is 2D or 3D with probability 1/2, side uniform on the integer
    range, |beta| ~ U[beta_mag], direction uniform (angle in 2D, sphere in 3D),
    a = 1, nrhs ~ U{nrhs}."""
    rng = np.random.default_rng([int(seed), 7])
    t = 0.0
    reqs = []
    for r in range(nreq):
        t += rng.exponential(1.0 / rate)
        dim = 2 if rng.random() < 0.5 else 3
        lo, hi = side2d if dim == 2 else side3d
        side = int(rng.integers(lo, hi + 1))
        mag = rng.uniform(*beta_mag)
        if dim == 2:
            th = rng.uniform(0.0, 2.0 * math.pi)
            beta = (mag * math.cos(th), mag * math.sin(th))
        else:
            v = rng.standard_normal(3)
            v /= np.linalg.norm(v)
            beta = tuple(mag * v)
        k = int(rng.integers(nrhs[0], nrhs[1] + 1))
        reqs.append(dict(id=r, arrival=t, dim=dim, side=side, beta=tuple(float(b) for b in beta),
                         nrhs=k, eps=eps, rhs_seed=int(rng.integers(0, 2**31 - 1))))
    return reqs


def build_request(req):
    dims = (req["side"],) * req["dim"]
    A = convdiff(dims, req["beta"])
    N = A.shape[0]
    b = make_rhs(N, req["nrhs"], req["rhs_seed"])
    # levels 0: the solver's default depth, ceil(log2(N / 64)) capped at the
    # deepest tree the grid allows (some 3D sides cannot take the full depth)
    return dict(A=A, dims=dims, levels=0, b=b)
