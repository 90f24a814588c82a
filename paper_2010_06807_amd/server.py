"""Continuous-batching server binding (spaqr_server_*)."""

from __future__ import annotations

import ctypes as C

import numpy as np

from . import _abi
from ._abi import SolveInfo, check


class Server:
    def __init__(self, mem_budget, stream=None):
        from . import _stream_ptr
        lib = _abi.load()
        h = C.c_void_p()
        check(lib.spaqr_server_create(int(mem_budget), _stream_ptr(stream), C.byref(h)), "spaqr_server_create")
        self._h = h
        self._keep = {}
        _abi.track("server", self)

    def close(self):
        if getattr(self, "_h", None) and _abi is not None and not _abi.released():
            _abi.load().spaqr_server_destroy(self._h)
        self._h = None

    def __del__(self):
        self.close()

    def submit(self, A, ordering, b, tol=1e-10, eps=1e-2, precision=32, skip=2):
        from . import _csr_struct, make_opts
        lib = _abi.load()
        csr, keep = _csr_struct(A)
        b = np.asarray(b, dtype=np.float64, order="F")
        nrhs = 1 if b.ndim == 1 else b.shape[1]
        o = make_opts(eps, skip, precision)
        t = C.c_uint64()
        check(lib.spaqr_submit(self._h, C.byref(csr), ordering.handle, C.byref(o), b.ctypes.data_as(C.c_void_p),
                               nrhs, float(tol), C.byref(t)), "spaqr_submit")
        self._keep[t.value] = (A.shape[0], nrhs)
        return t.value

    def step(self):
        a = C.c_int()
        check(_abi.load().spaqr_server_step(self._h, C.byref(a)), "spaqr_server_step")
        return a.value

    def status(self):
        """(queued, resident, estimated bytes of the resident requests)."""
        q, r, b = C.c_int64(), C.c_int64(), C.c_size_t()
        check(_abi.load().spaqr_server_status(self._h, C.byref(q), C.byref(r), C.byref(b)), "spaqr_server_status")
        return q.value, r.value, b.value

    def poll(self, ticket):
        n, nrhs = self._keep[ticket]
        x = np.empty((n, nrhs), dtype=np.float64, order="F")
        info = (SolveInfo * nrhs)()
        st = check(_abi.load().spaqr_poll(self._h, ticket, x.ctypes.data_as(C.c_void_p), info), "spaqr_poll")
        if st == _abi.PENDING:
            return None
        del self._keep[ticket]
        return x, [dict(iterations=i.iterations, converged=bool(i.converged), relres=i.relres,
                        seconds=i.seconds) for i in info]


def _percentile(v, q):
    v = sorted(v)
    if not v:
        return None
    i = min(len(v) - 1, max(0, int(np.ceil(q / 100.0 * len(v))) - 1))
    return v[i]


def serve_trace(jobs, mem_budget, tol=1e-10, precision=32, stream=None, time_scale=1.0, log=None):
    """Replay a request trace through the continuous-batching server.

    jobs: list of dicts with `arrival` (seconds from the start), `A` (scipy
    CSR), `ordering` (GridOrdering), `b` (n x nrhs) and `eps`.  Each request is
    submitted once the wall clock passes its arrival time (scaled by
    time_scale); the loop steps the server while requests are in flight.
    Returns per-request dicts (latency_s = completion - arrival, iterations,
    relres) and a summary with throughput (unknowns x right-hand sides per
    second over the makespan) and p50/p99 latency.  log(str), if given, is
    called as each request completes and after any server step longer than
    5 s."""
    import time
    srv = Server(mem_budget, stream)
    order = sorted(range(len(jobs)), key=lambda i: jobs[i]["arrival"])
    res = [None] * len(jobs)
    pending = {}
    t0 = time.perf_counter()
    nxt = 0
    while nxt < len(order) or pending:
        now = time.perf_counter() - t0
        while nxt < len(order) and jobs[order[nxt]]["arrival"] * time_scale <= now:
            j = jobs[order[nxt]]
            t = srv.submit(j["A"], j["ordering"], j["b"], tol=tol, eps=j.get("eps", 1e-2), precision=precision)
            pending[t] = order[nxt]
            nxt += 1
        if not pending:
            time.sleep(max(0.0, jobs[order[nxt]]["arrival"] * time_scale - (time.perf_counter() - t0)))
            continue
        ts = time.perf_counter()
        srv.step()
        dt = time.perf_counter() - ts
        if log and dt > 5.0:
            log(f"server step took {dt:.1f} s with {len(pending)} requests in flight")
        for t in list(pending):
            out = srv.poll(t)
            if out is None:
                continue
            i = pending.pop(t)
            x, info = out
            res[i] = dict(latency_s=time.perf_counter() - t0 - jobs[i]["arrival"] * time_scale, x=x,
                          iterations=[d["iterations"] for d in info], relres=[d["relres"] for d in info])
            if log:
                log(f"request {i} done, latency {res[i]['latency_s']:.3f} s")
    span = time.perf_counter() - t0
    work = sum(j["A"].shape[0] * (1 if np.ndim(j["b"]) == 1 else np.shape(j["b"])[1]) for j in jobs)
    lat = [r["latency_s"] for r in res]
    return res, dict(makespan_s=span, throughput=work / span, p50_ms=1e3 * _percentile(lat, 50),
                     p99_ms=1e3 * _percentile(lat, 99), requests=len(jobs))


def serve_sequential(jobs, tol=1e-10, precision=64, time_scale=1.0, log=None):
    """The same trace without batching: requests run one at a time in arrival
    order (factor, then solve all of the request's right-hand sides), each
    starting no earlier than its arrival."""
    import time
    from . import factor
    order = sorted(range(len(jobs)), key=lambda i: jobs[i]["arrival"])
    res = [None] * len(jobs)
    t0 = time.perf_counter()
    for i in order:
        j = jobs[i]
        wait = j["arrival"] * time_scale - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        fac = factor(j["A"], j["ordering"], eps=j.get("eps", 1e-2), precision=precision)
        x, info = fac.solve(j["b"], tol=tol)
        del fac
        res[i] = dict(latency_s=time.perf_counter() - t0 - j["arrival"] * time_scale, x=x,
                      iterations=[d["iterations"] for d in info], relres=[d["relres"] for d in info])
        if log:
            log(f"request {i} done, latency {res[i]['latency_s']:.3f} s")
    span = time.perf_counter() - t0
    work = sum(j["A"].shape[0] * (1 if np.ndim(j["b"]) == 1 else np.shape(j["b"])[1]) for j in jobs)
    lat = [r["latency_s"] for r in res]
    return res, dict(makespan_s=span, throughput=work / span, p50_ms=1e3 * _percentile(lat, 50),
                     p99_ms=1e3 * _percentile(lat, 99), requests=len(jobs))
