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

    def __del__(self):
        if getattr(self, "_h", None):
            _abi.load().spaqr_server_destroy(self._h)
            self._h = None

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
