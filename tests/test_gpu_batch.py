"""Cross-request batching through the C-ABI: spaqr_factor_batch advances
several factorizations stage by stage in shared launches, spaqr_solve_batch
runs their FGMRES steps together (one launch per apply phase for all of
them).  Each problem's result must be the one it gets alone, within the
stated tolerances: interface ranks within +-1, the same iteration count
within +-1, ||Ax - b|| / ||b|| <= 1e-10 and solutions that agree to the solve
tolerance."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2010_06807_amd as P
from problems import convdiff, make_rhs
from problems.grids import default_levels

pytestmark = pytest.mark.gpu

# dims, beta, eps: uneven sizes (padding of the batched vectors), 2D and 3D
PROBS = [
    ((48, 48), (10.0, 5.0), 1e-2),
    ((64, 40), (-30.0, 20.0), 1e-3),
    ((12, 12, 12), (5.0, 5.0, 5.0), 1e-2),
    ((32, 32), (1.0, 1.0), 0.0),
]


def _setup(i, dims, beta, eps, nrhs):
    A = convdiff(dims, beta)
    N = A.shape[0]
    o = P.order_grid(dims, default_levels(N))
    return dict(A=A, o=o, sym=P.analyze(A, o), eps=eps, b=make_rhs(N, nrhs, seed=200 + i))


def _ranks(fac, L):
    return [fac.stage_sizes(k) for k in range(L, 0, -1)]


def _compare(jobs, facs_b, xs, infos, precision):
    for j, fb, xb, ib in zip(jobs, facs_b, xs, infos):
        print(f"  case batch n={j['A'].shape[0]} eps={j['eps']} precision={precision}", flush=True)
        alone = P.factor_device(j["A"], j["sym"], P.DeviceCSR(j["A"]), eps=j["eps"], precision=precision)
        L = j["o"].levels
        for ra, rb in zip(_ranks(alone, L), _ranks(fb, L)):
            assert ra.shape == rb.shape
            if ra.size:
                assert int(np.max(np.abs(ra.astype(np.int64) - rb))) <= 1
        b = j["b"]
        xa, ia = alone.solve(b, tol=1e-10)
        xb = xb.cpu().numpy() if hasattr(xb, "cpu") else xb
        xb = xb.reshape(b.shape)
        for c in range(b.shape[1]):
            r = np.linalg.norm(j["A"] @ xb[:, c] - b[:, c]) / np.linalg.norm(b[:, c])
            assert r <= 1e-10, r
            assert ib[c]["converged"]
            assert abs(ib[c]["iterations"] - ia[c]["iterations"]) <= 1
            d = np.linalg.norm(xb[:, c] - xa[:, c]) / np.linalg.norm(xa[:, c])
            assert d <= 1e-7, d


@pytest.mark.parametrize("precision", [32, 64])
def test_factor_and_solve_batch_device(precision):
    jobs = [_setup(i, d, bt, e, 1 + (i % 2)) for i, (d, bt, e) in enumerate(PROBS)]
    dcsrs = [P.DeviceCSR(j["A"]) for j in jobs]
    # one eps per batch call: group by eps
    facs = [None] * len(jobs)
    for eps in sorted({j["eps"] for j in jobs}):
        idx = [i for i, j in enumerate(jobs) if j["eps"] == eps]
        out = P.factor_batch([jobs[i]["A"] for i in idx], [jobs[i]["sym"] for i in idx], [dcsrs[i] for i in idx],
                             eps=eps, precision=precision)
        for i, f in zip(idx, out):
            facs[i] = f
    bs = [torch.from_numpy(np.asfortranarray(j["b"])).cuda() for j in jobs]  # column-major
    xs, infos = P.solve_batch(facs, bs, tol=1e-10)
    torch.cuda.synchronize()
    _compare(jobs, facs, xs, infos, precision)


def test_solve_batch_mixed_precision_host_arrays():
    jobs = [_setup(i, d, bt, 1e-2, 2 if i == 0 else 1) for i, (d, bt, _) in enumerate(PROBS[:3])]
    facs = [P.factor_device(j["A"], j["sym"], P.DeviceCSR(j["A"]), eps=1e-2, precision=32 if i != 1 else 64)
            for i, j in enumerate(jobs)]
    xs, infos = P.solve_batch(facs, [j["b"] for j in jobs], tol=[1e-10, 1e-10, 1e-10])
    for j, x, inf in zip(jobs, xs, infos):
        b = j["b"]
        x = x.reshape(b.shape)
        for c in range(b.shape[1]):
            r = np.linalg.norm(j["A"] @ x[:, c] - b[:, c]) / np.linalg.norm(b[:, c])
            assert r <= 1e-10, r
            assert inf[c]["converged"]


def test_batch_of_one_matches_plain_solve_exactly():
    j = _setup(0, (40, 40), (10.0, -5.0), 1e-2, 1)
    dA = P.DeviceCSR(j["A"])
    (fb,) = P.factor_batch([j["A"]], [j["sym"]], [dA], eps=1e-2, precision=32)
    fa = P.factor_device(j["A"], j["sym"], dA, eps=1e-2, precision=32)
    L = j["o"].levels
    for ra, rb in zip(_ranks(fa, L), _ranks(fb, L)):
        assert np.array_equal(ra, rb)
    xa, ia = fa.solve(j["b"], tol=1e-10)
    (xb,), (ib,) = P.solve_batch([fb], [j["b"]], tol=1e-10)
    # same launches, same kernels: bit-identical factors and iterates
    assert ia[0]["iterations"] == ib[0]["iterations"]
    assert np.array_equal(xa.reshape(-1), xb.reshape(-1))


def test_factor_batch_mixed_shapes_one_eps():
    """Five problems of different shapes (2D and 3D, different depths) in one
    batched factorization and one batched solve: every problem must match
    its factorization alone."""
    probs = [((40, 40), (10.0, 5.0)), ((12, 12, 12), (5.0, 5.0, 5.0)), ((64, 40), (-30.0, 20.0)),
             ((10, 10, 14), (2.0, -3.0, 1.0)), ((56, 56), (1.0, 20.0))]
    jobs = [_setup(i, d, bt, 1e-2, 1) for i, (d, bt) in enumerate(probs)]
    dcsrs = [P.DeviceCSR(j["A"]) for j in jobs]
    facs = P.factor_batch([j["A"] for j in jobs], [j["sym"] for j in jobs], dcsrs, eps=1e-2, precision=32)
    xs, infos = P.solve_batch(facs, [j["b"] for j in jobs], tol=1e-10)
    _compare(jobs, facs, xs, infos, 32)
