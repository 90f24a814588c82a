"""Pins for the synthetic input generators (upwind convection-diffusion)."""

import numpy as np
import pytest

from problems import convdiff, make_rhs, config_problem, serving_trace


def _brute_force(n, d, beta, a=None):
    """Entry-by-entry stencil, written point by point (independent of the
    vectorized assembly)."""
    N = n ** d
    h = 1.0 / (n + 1)
    A = np.zeros((N, N))
    af = np.ones(N) if a is None else a.reshape(-1)

    def idx(c):
        return sum(c[t] * n ** t for t in range(d))

    for i in range(N):
        c = [(i // n ** t) % n for t in range(d)]
        for ax in range(d):
            for s in (-1, 1):
                cc = list(c)
                cc[ax] += s
                inside = 0 <= cc[ax] < n
                if inside:
                    j = idx(cc)
                    face = 0.5 * (af[i] + af[j])
                    A[i, j] -= face
                else:
                    face = af[i]
                A[i, i] += face
            b = beta[ax]
            if b > 0:
                A[i, i] += h * b
                if c[ax] - 1 >= 0:
                    cc = list(c)
                    cc[ax] -= 1
                    A[i, idx(cc)] -= h * b
            elif b < 0:
                A[i, i] += h * -b
                if c[ax] + 1 < n:
                    cc = list(c)
                    cc[ax] += 1
                    A[i, idx(cc)] -= h * -b
    return A


@pytest.mark.parametrize("n,d,beta", [(5, 2, (10.0, -3.0)), (4, 3, (2.0, -1.0, 5.0)), (6, 2, (0.0, 0.0))])
def test_stencil_matches_pointwise(n, d, beta):
    rng = np.random.default_rng(1)
    a = np.exp(rng.standard_normal((n,) * d))
    for field in (None, a):
        A = convdiff((n,) * d, beta, a=field).toarray()
        B = _brute_force(n, d, beta, a=field)
        assert np.allclose(A, B, rtol=0, atol=1e-14)


@pytest.mark.parametrize("n,d", [(7, 2), (16, 2), (5, 3), (9, 3)])
def test_nnz_and_dominance(n, d):
    A = convdiff((n,) * d, (3.0,) * d)
    nnz = 5 * n * n - 4 * n if d == 2 else 7 * n ** 3 - 6 * n ** 2
    assert A.nnz == nnz
    D = np.abs(A.diagonal())
    off = np.asarray(abs(A).sum(axis=1)).ravel() - D
    assert np.all(D >= off - 1e-12)
    assert A.indices.dtype == np.int32 and A.indptr.dtype == np.int64


def test_pure_diffusion_is_laplacian():
    n = 6
    A = convdiff((n, n), (0.0, 0.0)).toarray()
    assert np.allclose(A, A.T)
    assert np.allclose(np.diag(A), 4.0)
    # interior rows sum to zero (conservation)
    assert abs(A[n + 1].sum()) < 1e-14


def test_configs_and_rhs():
    c1 = config_problem("c1")
    assert c1["A"].shape == (1024, 1024) and c1["levels"] == 5
    b = make_rhs(100, 3, seed=4)
    assert b.shape == (100, 3) and b.flags.f_contiguous
    assert np.all(np.abs(b) <= 1.0)
    assert np.array_equal(b, make_rhs(100, 3, seed=4))
    tr = serving_trace(20, seed=0)
    assert len(tr) == 20 and all(16 <= r["side"] <= 512 for r in tr)
    assert all(tr[i]["arrival"] < tr[i + 1]["arrival"] for i in range(19))
