"""The paper's advection-diffusion problems (problems/paper_ad.py): the
centered-difference discretization of -div(a grad u) + q div(b u) pinned by
its symmetric and antisymmetric parts, consistency with the exact operator
on smooth functions, and the high-contrast field's two values."""

import math

import numpy as np

from problems.paper_ad import advdiff_centered, high_contrast_field, paper_problem
from problems.grids import convdiff


def test_constant_b_splits_into_diffusion_and_antisymmetric_convection():
    for dims in [(12, 12), (6, 6, 6)]:
        n = dims[0]
        q = 25.0
        A = advdiff_centered(dims, q=q, b="one")
        D = convdiff(dims, (0.0,) * len(dims))     # the same diffusion, no convection
        S = 0.5 * (A + A.T)
        K = 0.5 * (A - A.T)
        assert abs(S - D).max() <= 1e-15
        h = 1.0 / (n + 1)
        # every off-diagonal entry of the antisymmetric part is +-q h / 2
        Kc = K.tocoo()
        nz = Kc.data[np.abs(Kc.data) > 0]
        assert np.allclose(np.abs(nz), q * h / 2.0, rtol=1e-14)
        assert abs(K.diagonal()).max() == 0.0
        assert A.nnz == (5 * n * n - 4 * n if len(dims) == 2 else 7 * n ** 3 - 6 * n * n)


def test_consistent_with_the_exact_operator():
    """A applied to samples of u = sin(pi x) sin(pi y), divided by h^2, tends
    to -lap u + q div(b u) at second order (b = e^{x+y} (1, 1))."""
    q = 3.0
    errs = []
    for n in (31, 63):
        h = 1.0 / (n + 1)
        x = (np.arange(n) + 1) * h
        X, Y = np.meshgrid(x, x, indexing="xy")
        u = np.sin(math.pi * X) * np.sin(math.pi * Y)
        e = np.exp(X + Y)
        # -lap u + q (d/dx + d/dy)(e u)
        exact = (2 * math.pi ** 2 * u + q * (e * u + e * math.pi * np.cos(math.pi * X) * np.sin(math.pi * Y)
                                             + e * u + e * math.pi * np.sin(math.pi * X) * np.cos(math.pi * Y)))
        A = advdiff_centered((n, n), q=q, b="exp")
        got = (A @ u.reshape(-1)) / h ** 2
        errs.append(np.abs(got - exact.reshape(-1)).max())
    assert errs[1] < errs[0] / 3.0   # second order: ~4x per halving of h


def test_high_contrast_field_takes_two_values():
    rng = np.random.default_rng(0)
    a = high_contrast_field(64, 100.0, rng)
    assert set(np.unique(a)) == {0.01, 100.0}
    frac = np.mean(a == 100.0)
    assert 0.3 < frac < 0.7
    p = paper_problem("hc", 32, rho=10.0)
    assert p["A"].shape == (1024, 1024)
    # rho = 1 is the constant-coefficient problem
    assert abs(paper_problem("hc", 16, rho=1.0)["A"] - advdiff_centered((16, 16), q=1.0)).max() == 0.0
