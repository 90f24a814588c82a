"""Continuous-batching server on the GPU: every result of a mixed batch is the
same, within the solve tolerance, as the same request factored and solved
alone; requests that arrive while others are half-way through their
factorization join the running batch."""

import numpy as np
import pytest

pytest.importorskip("torch")

import paper_2010_06807_amd as P
from paper_2010_06807_amd.server import Server, serve_trace
from problems import convdiff, make_rhs
from problems.grids import default_levels

pytestmark = pytest.mark.gpu

# dims, beta, eps, nrhs, precision: 2D and 3D, mixed sizes, tolerances and
# right-hand side counts, FP32 and FP64 factors in one server
MIX = [
    ((40, 40), (10.0, 5.0), 1e-2, 2, 32),
    ((64, 48), (-30.0, 20.0), 1e-3, 1, 32),
    ((12, 12, 12), (5.0, 5.0, 5.0), 1e-2, 3, 32),
    ((24, 24), (1.0, 1.0), 0.0, 1, 32),
    ((10, 10, 14), (2.0, -3.0, 1.0), 1e-2, 2, 64),
    ((96, 96), (50.0, -20.0), 1e-2, 1, 32),
]


def _job(i, dims, beta, eps, nrhs):
    A = convdiff(dims, beta)
    N = A.shape[0]
    L = default_levels(N)
    return dict(A=A, dims=dims, ordering=P.order_grid(dims, L), b=make_rhs(N, nrhs, seed=100 + i), eps=eps)


def _alone(j, precision):
    fac = P.factor(j["A"], j["ordering"], eps=j["eps"], precision=precision)
    return fac.solve(j["b"], tol=1e-10)


def _check(j, x_mix, info_mix, x_one, info_one):
    A, b = j["A"], j["b"]
    for c in range(b.shape[1]):
        r = np.linalg.norm(A @ x_mix[:, c] - b[:, c]) / np.linalg.norm(b[:, c])
        assert r <= 1e-10, r
        assert abs(info_mix[c]["iterations"] - info_one[c]["iterations"]) <= 1
        # both solutions are within the solve tolerance of A^{-1} b
        d = np.linalg.norm(x_mix[:, c] - x_one[:, c]) / np.linalg.norm(x_one[:, c])
        assert d <= 1e-7, d


def test_mix_submitted_together():
    jobs = [_job(i, *m[:4]) for i, m in enumerate(MIX)]
    srv = Server(mem_budget=8 << 30)
    tickets = [srv.submit(j["A"], j["ordering"], j["b"], eps=j["eps"], precision=m[4]) for j, m in zip(jobs, MIX)]
    out = {}
    for _ in range(200):
        srv.step()
        for t in tickets:
            if t not in out:
                r = srv.poll(t)
                if r is not None:
                    out[t] = r
        if len(out) == len(tickets):
            break
    assert len(out) == len(tickets)
    for j, m, t in zip(jobs, MIX, tickets):
        x_one, info_one = _alone(j, m[4])
        _check(j, out[t][0], out[t][1], x_one, info_one)


def test_late_arrivals_join_the_batch():
    jobs = [_job(10 + i, *m[:4]) for i, m in enumerate(MIX)]
    srv = Server(mem_budget=8 << 30)
    tickets = {}
    out = {}
    # two requests start; the others arrive one per step while they factor
    for i in range(2):
        tickets[i] = srv.submit(jobs[i]["A"], jobs[i]["ordering"], jobs[i]["b"], eps=jobs[i]["eps"],
                                precision=MIX[i][4])
    nxt = 2
    for _ in range(300):
        srv.step()
        if nxt < len(jobs):
            tickets[nxt] = srv.submit(jobs[nxt]["A"], jobs[nxt]["ordering"], jobs[nxt]["b"], eps=jobs[nxt]["eps"],
                                      precision=MIX[nxt][4])
            nxt += 1
        for i, t in tickets.items():
            if i not in out:
                r = srv.poll(t)
                if r is not None:
                    out[i] = r
        if len(out) == len(jobs):
            break
    assert len(out) == len(jobs)
    for i, j in enumerate(jobs):
        x_one, info_one = _alone(j, MIX[i][4])
        _check(j, out[i][0], out[i][1], x_one, info_one)


def _estimate(j, nrhs, precision=32):
    return P.analyze(j["A"], j["ordering"]).estimate_bytes(precision=precision, nrhs=nrhs)


def test_admission_by_memory_budget():
    """A budget that holds one request at a time: the server never has two
    requests resident (its occupancy is read after every step) and still
    serves them all."""
    jobs = [_job(20 + i, *m[:4]) for i, m in enumerate(MIX[:3])]
    est = [_estimate(j, j["b"].shape[1]) for j in jobs]
    budget = max(est) + min(est) // 2   # the largest fits, no two do
    assert all(a + b > budget for a in est for b in est)
    srv = Server(mem_budget=budget)
    tickets = [srv.submit(j["A"], j["ordering"], j["b"], eps=j["eps"]) for j in jobs]
    out = {}
    seen = 0
    for _ in range(300):
        srv.step()
        queued, resident, used = srv.status()
        assert resident <= 1 and used <= budget, (queued, resident, used)
        seen = max(seen, resident)
        for t in tickets:
            if t not in out:
                r = srv.poll(t)
                if r is not None:
                    out[t] = r
        if len(out) == len(tickets):
            break
    assert len(out) == len(tickets) and seen == 1
    assert srv.status()[:2] == (0, 0)
    for j, t in zip(jobs, tickets):
        x, info = out[t]
        for c in range(j["b"].shape[1]):
            r = np.linalg.norm(j["A"] @ x[:, c] - j["b"][:, c]) / np.linalg.norm(j["b"][:, c])
            assert r <= 1e-10


def test_admission_estimate_bounds_measured_factor_bytes():
    """The analysis's device-memory bound covers what a factorization really
    stores, in both precisions, for 2D and 3D grids and eps = 0 (nothing
    compressed, the bound's own worst case)."""
    for i, (dims, beta, eps) in enumerate([((64, 48), (-30.0, 20.0), 1e-3), ((12, 12, 12), (5.0,) * 3, 0.0),
                                           ((96, 96), (50.0, -20.0), 0.0), ((16, 16, 16), (2.0, 1.0, -1.0), 1e-2)]):
        j = _job(40 + i, dims, beta, eps, 1)
        for prec in (32, 64):
            fac = P.factor(j["A"], j["ordering"], eps=eps, precision=prec)
            fb = fac.stats()["factor_bytes"]
            assert 0 < fb <= _estimate(j, 1, prec), (dims, prec, fb)


def test_trace_replay():
    jobs = []
    for i, m in enumerate(MIX[:4]):
        j = _job(30 + i, *m[:4])
        j["arrival"] = 0.002 * i
        jobs.append(j)
    res, summ = serve_trace(jobs, mem_budget=8 << 30)
    assert summ["requests"] == len(jobs) and summ["p99_ms"] >= summ["p50_ms"] > 0
    for j, r in zip(jobs, res):
        assert max(r["relres"]) <= 1e-10
