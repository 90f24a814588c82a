"""spaqr_apply_noalloc against spaqr_apply through the C ABI: the same
M^{-1} b (the two share every kernel, so bit for bit), on two calls in a
row, the second with a smaller input; sizes above the fixed workspace are
refused before any GPU work."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2010_06807_amd as P
from paper_2010_06807_amd import _abi
from problems import convdiff, make_rhs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _dev(b):
    return torch.from_numpy(np.asfortranarray(b).T.copy()).to(DEV).T


def test_noalloc_apply_matches_apply():
    cases = [((48, 48), 6, (35.0, -12.0), 3, 32), ((24, 24), 5, (10.0, 5.0), 1, 64)]
    for dims, L, beta, nrhs, prec in cases:   # the second call is the smaller input
        print(f"case noalloc dims={dims} nrhs={nrhs} precision={prec}", flush=True)
        A = convdiff(dims, beta)
        N = A.shape[0]
        fac = P.factor(A, P.order_grid(dims, L), eps=1e-2, precision=prec)
        b = _dev(make_rhs(N, nrhs, seed=4))
        ref = fac.apply(b)
        out = torch.full_like(b, float("nan"))
        fac.apply_noalloc(b, out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        res = np.linalg.norm(A @ out.cpu().numpy() - b.cpu().numpy()) / np.linalg.norm(b.cpu().numpy())
        assert res < 1.0


def test_noalloc_apply_refuses_sizes_beyond_the_workspace():
    A = convdiff((32, 32), (10.0, 10.0))
    N = A.shape[0]
    fac = P.factor(A, P.order_grid((32, 32), 5), eps=1e-2, precision=32)
    cap = _abi.load().spaqr_apply_noalloc_max()
    assert cap == 1 << 23
    too_many = cap // N + 1
    lib = _abi.load()
    b = torch.zeros(1, device=DEV, dtype=torch.float64)
    st = lib.spaqr_apply_noalloc(fac._h, b.data_ptr(), b.data_ptr(), too_many, N)
    assert st == _abi.EINVAL
