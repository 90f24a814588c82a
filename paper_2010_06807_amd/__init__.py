"""MI355X spaQR engine: Python binding over the C ABI of libspaqr.so.

Only argument marshalling lives here; ordering, symbolic analysis,
factorization, apply and GMRES all run in the native library (host C++ and
HIP kernels for gfx950).  PyTorch supplies device buffers and the stream.

    ord = order_grid((256, 256))
    fac = factor(A, ord, eps=1e-2, precision=32)   # A: scipy CSR (FP64)
    x, info = fac.solve(b, tol=1e-10)              # b: torch CUDA tensor or numpy
"""

from __future__ import annotations

import ctypes as C

import numpy as np

from . import _abi
from ._abi import CSR, Opts, SolveInfo, SpaqrError, check

__all__ = ["order_grid", "analyze", "factor", "factor_device", "factor_batch", "solve_batch", "DeviceCSR",
           "GridOrdering", "Symbolic", "Factorization", "Server", "SpaqrError", "load_library", "profile_enable",
           "profile_query", "kernel_launches", "get_tuning", "set_tuning"]


def load_library():
    return _abi.load()


def _csr_struct(A):
    indptr = np.ascontiguousarray(A.indptr, dtype=np.int64)
    indices = np.ascontiguousarray(A.indices, dtype=np.int32)
    data = np.ascontiguousarray(A.data, dtype=np.float64)
    s = CSR(A.shape[0], data.shape[0], indptr.ctypes.data_as(C.POINTER(C.c_int64)),
            indices.ctypes.data_as(C.POINTER(C.c_int32)), data.ctypes.data_as(C.POINTER(C.c_double)))
    return s, (indptr, indices, data)


def make_opts(eps=1e-2, skip=2, precision=32, restart=100, maxit=1000, scale=True):
    """spaqr_opts; scale=False selects the sparsification without scaling of
    Section 2.5 (sigma = 1/sigma_min(A_p), Householder on the fine unknowns)."""
    lib = _abi.load()
    o = lib.spaqr_opts_default()
    o.eps, o.skip, o.scale, o.precision, o.restart, o.maxit = float(eps), int(skip), 1 if scale else 0, \
        int(precision), int(restart), int(maxit)
    return o


class GridOrdering:
    """Geometric modified nested dissection of a grid (spaqr_order_grid)."""

    def __init__(self, dims, levels=0):
        lib = _abi.load()
        dims = tuple(int(d) for d in dims)
        sides = (C.c_int32 * 3)(*(list(dims) + [1] * (3 - len(dims))))
        h = C.c_void_p()
        check(lib.spaqr_order_grid(len(dims), sides, int(levels), C.byref(h)), "spaqr_order_grid")
        self._h = h
        self.dims = dims
        self.n = lib.spaqr_ordering_n(h)
        self.levels = lib.spaqr_ordering_levels(h)
        _abi.track("ordering", self)

    def close(self):
        # after the exit hook (or once module globals are gone) the handle
        # was already released
        if getattr(self, "_h", None) and _abi is not None and not _abi.released():
            _abi.load().spaqr_ordering_free(self._h)
        self._h = None

    def __del__(self):
        self.close()

    @property
    def handle(self):
        return self._h

    def perm(self):
        out = np.empty(self.n, dtype=np.int64)
        check(_abi.load().spaqr_ordering_perm(self._h, out.ctypes.data_as(C.POINTER(C.c_int64))),
              "spaqr_ordering_perm")
        return out

    def clusters(self, stage):
        lib = _abi.load()
        nc = lib.spaqr_ordering_num_clusters(self._h, int(stage))
        if nc < 0:
            raise ValueError("bad stage")
        s, e, nd = (np.empty(nc, dtype=np.int64) for _ in range(3))
        lv = np.empty(nc, dtype=np.int32)
        p64 = C.POINTER(C.c_int64)
        check(lib.spaqr_ordering_clusters(self._h, int(stage), s.ctypes.data_as(p64), e.ctypes.data_as(p64),
                                          nd.ctypes.data_as(p64), lv.ctypes.data_as(C.POINTER(C.c_int32))),
              "spaqr_ordering_clusters")
        return s, e, nd, lv

    def merge_parents(self, stage):
        lib = _abi.load()
        nc = lib.spaqr_ordering_num_clusters(self._h, int(stage))
        out = np.empty(nc, dtype=np.int64)
        check(lib.spaqr_ordering_merge_parents(self._h, int(stage), out.ctypes.data_as(C.POINTER(C.c_int64))),
              "spaqr_ordering_merge_parents")
        return out


def order_grid(dims, levels=0):
    return GridOrdering(dims, levels)


class GraphOrdering(GridOrdering):
    """Algebraic modified nested dissection of a square sparse matrix without a
    grid (spaqr_order_graph): bisection of the graph of A^T A between two far
    vertices, with separator thinning."""

    def __init__(self, A, levels=0):
        lib = _abi.load()
        csr, keep = _csr_struct(A)
        h = C.c_void_p()
        check(lib.spaqr_order_graph(C.byref(csr), int(levels), C.byref(h)), "spaqr_order_graph")
        del keep
        self._h = h
        self.dims = (A.shape[0],)
        self.n = lib.spaqr_ordering_n(h)
        self.levels = lib.spaqr_ordering_levels(h)
        _abi.track("ordering", self)


def order_graph(A, levels=0):
    return GraphOrdering(A, levels)


class Symbolic:
    """Host-only symbolic analysis (spaqr_analyze)."""

    def __init__(self, A, ordering, skip=2):
        lib = _abi.load()
        csr, self._keep = _csr_struct(A)
        o = make_opts(skip=skip)
        h = C.c_void_p()
        check(lib.spaqr_analyze(C.byref(csr), ordering.handle, C.byref(o), C.byref(h)), "spaqr_analyze")
        self._h = h
        self.levels = ordering.levels
        _abi.track("symbolic", self)

    def close(self):
        if getattr(self, "_h", None) and _abi is not None and not _abi.released():
            _abi.load().spaqr_symbolic_free(self._h)
        self._h = None

    def __del__(self):
        self.close()

    @property
    def handle(self):
        return self._h

    def estimate_bytes(self, precision=32, nrhs=1, restart=100):
        """Upper bound on the device bytes of a factorization of this analysis
        and a solve of nrhs right-hand sides (spaqr_estimate_bytes)."""
        o = make_opts(precision=precision, restart=restart)
        out = C.c_size_t()
        check(_abi.load().spaqr_estimate_bytes(self._h, C.byref(o), int(nrhs), C.byref(out)),
              "spaqr_estimate_bytes")
        return out.value

    def stage_info(self, stage, what):
        lib = _abi.load()
        n = C.c_int64()
        check(lib.spaqr_symbolic_stage_info(self._h, int(stage), int(what), None, 0, C.byref(n)), "stage_info")
        buf = np.empty(max(1, n.value), dtype=np.int32)
        check(lib.spaqr_symbolic_stage_info(self._h, int(stage), int(what),
                                            buf.ctypes.data_as(C.POINTER(C.c_int32)), buf.size, C.byref(n)),
              "stage_info")
        return buf[:n.value]

    def pattern(self, stage, post=False):
        v = self.stage_info(stage, 1 if post else 0)
        return [tuple(x) for x in v.reshape(-1, 2).tolist()]

    def fronts(self, stage):
        v = self.stage_info(stage, 2).tolist()
        out, i = {}, 0
        while i < len(v):
            s, col, nn1 = v[i], v[i + 1], v[i + 2]
            n1 = v[i + 3:i + 3 + nn1]
            i += 3 + nn1
            nc = v[i]
            cols = v[i + 1:i + 1 + nc]
            i += 1 + nc
            out[s] = (n1, cols, col)
        return out

    def iface_colours(self, stage):
        v = self.stage_info(stage, 3).reshape(-1, 2)
        return {int(a): int(b) for a, b in v}


def analyze(A, ordering, skip=2):
    return Symbolic(A, ordering, skip)


def _stream_ptr(stream):
    if stream is None:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
        return C.c_void_p(0)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


class Factorization:
    """A spaQR factorization resident on the GPU (spaqr_factor)."""

    def __init__(self, A, ordering=None, symbolic=None, eps=1e-2, skip=2, precision=32, restart=100,
                 maxit=1000, stream=None, device_csr=None, scale=True, _handle=None):
        if _handle is not None:          # made by factor_batch
            self._h = _handle
            self._sym = symbolic
            self.n = A.shape[0]
            _abi.track("factor", self)
            return
        lib = _abi.load()
        csr, keep = _csr_struct(A)
        o = make_opts(eps, skip, precision, restart, maxit, scale)
        h = C.c_void_p()
        sp = _stream_ptr(stream)
        if device_csr is not None:
            if symbolic is None:
                raise ValueError("the device path needs a symbolic analysis")
            dev = _abi.CSRDev(device_csr.rowptr.data_ptr(), device_csr.col.data_ptr(), device_csr.val.data_ptr())
            st = lib.spaqr_factor_device(C.byref(csr), C.byref(dev), symbolic.handle, C.byref(o), sp, C.byref(h))
        elif symbolic is not None:
            st = lib.spaqr_factor_symbolic(C.byref(csr), symbolic.handle, C.byref(o), sp, C.byref(h))
        else:
            st = lib.spaqr_factor(C.byref(csr), ordering.handle, C.byref(o), sp, C.byref(h))
        check(st, "spaqr_factor")
        del keep
        self._h = h
        self._sym = symbolic   # the handle reads the analysis it was made from
        self.n = A.shape[0]
        _abi.track("factor", self)

    def close(self):
        if getattr(self, "_h", None) and _abi is not None and not _abi.released():
            _abi.load().spaqr_free(self._h)
        self._h = None

    def __del__(self):
        self.close()

    # vectors: numpy (host) or torch CUDA tensors (device), shape (n,) or (n, nrhs)
    @staticmethod
    def _layout(b, n):
        if b.ndim == 1 or b.shape[1] == 1:
            return 1, n     # the stride of a single column is irrelevant
        if hasattr(b, "stride"):           # torch
            if b.stride(0) != 1:
                raise ValueError("device arrays must be column-major (stride(0) == 1)")
            return b.shape[1], b.stride(1)
        if not b.flags.f_contiguous:
            raise ValueError("host arrays must be column-major")
        return b.shape[1], n

    def apply(self, b, out=None):
        lib = _abi.load()
        if hasattr(b, "is_cuda") and b.is_cuda:
            import torch
            if out is None:
                out = torch.empty_like(b)
            nrhs, ld = self._layout(b, self.n)
            check(lib.spaqr_apply(self._h, C.c_void_p(b.data_ptr()), C.c_void_p(out.data_ptr()), nrhs, ld, 1),
                  "spaqr_apply")
            return out
        b = np.asarray(b, dtype=np.float64, order="F")
        out = np.empty_like(b, order="F") if out is None else out
        nrhs, ld = self._layout(b, self.n)
        check(lib.spaqr_apply(self._h, b.ctypes.data_as(C.c_void_p), out.ctypes.data_as(C.c_void_p), nrhs, ld, 0),
              "spaqr_apply")
        return out

    def apply_noalloc(self, b, out):
        """out = M^{-1} b through spaqr_apply_noalloc (no device allocation;
        b and out are device tensors, column-major); returns once the work
        is enqueued on the factorization's stream."""
        nrhs, ld = self._layout(b, self.n)
        nrhs_o, ld_o = self._layout(out, self.n)
        if (nrhs_o, ld_o) != (nrhs, ld):
            raise ValueError("b and out must have the same layout")
        check(_abi.load().spaqr_apply_noalloc(self._h, C.c_void_p(b.data_ptr()), C.c_void_p(out.data_ptr()),
                                              nrhs, ld), "spaqr_apply_noalloc")
        return out

    def solve(self, b, tol=1e-10, out=None):
        lib = _abi.load()
        on_dev = hasattr(b, "is_cuda") and b.is_cuda
        if on_dev:
            import torch
            out = torch.empty_like(b) if out is None else out
            nrhs, ld = self._layout(b, self.n)
            info = (SolveInfo * nrhs)()
            st = lib.spaqr_solve(self._h, C.c_void_p(b.data_ptr()), C.c_void_p(out.data_ptr()), nrhs, ld, 1,
                                 float(tol), info)
        else:
            b = np.asarray(b, dtype=np.float64, order="F")
            out = np.empty_like(b, order="F") if out is None else out
            nrhs, ld = self._layout(b, self.n)
            info = (SolveInfo * nrhs)()
            st = lib.spaqr_solve(self._h, b.ctypes.data_as(C.c_void_p), out.ctypes.data_as(C.c_void_p), nrhs, ld,
                                 0, float(tol), info)
        check(st, "spaqr_solve")
        res = [dict(iterations=i.iterations, converged=bool(i.converged), relres=i.relres, seconds=i.seconds)
               for i in info]
        return out, res

    def stats(self):
        s = _abi.Stats()
        check(_abi.load().spaqr_stats(self._h, C.byref(s)), "spaqr_stats")
        d = {k: getattr(s, k) for k, _ in _abi.Stats._fields_ if k != "ms_phase"}
        d["ms_phase"] = list(s.ms_phase)
        return d

    def stage_stats(self, stage):
        """Per-stage statistics of the completed factorization (spaqr_stage_stats)."""
        st = _abi.StageStats()
        check(_abi.load().spaqr_stage_stats(self._h, int(stage), C.byref(st)), "spaqr_stage_stats")
        return {k: getattr(st, k) for k, _ in _abi.StageStats._fields_ if k != "pad"}

    def stage_interfaces(self, stage):
        """(cluster, |p|, m_p, r_p) of every interface sparsified at the stage,
        an int32 array of shape (count, 4)."""
        lib = _abi.load()
        n = C.c_int64()
        check(lib.spaqr_stage_interfaces(self._h, int(stage), None, 0, C.byref(n)), "spaqr_stage_interfaces")
        buf = np.empty(max(1, n.value), dtype=np.int32)
        check(lib.spaqr_stage_interfaces(self._h, int(stage), buf.ctypes.data_as(C.POINTER(C.c_int32)), buf.size,
                                         C.byref(n)), "spaqr_stage_interfaces")
        return buf[:n.value].reshape(-1, 4)

    def solve_history(self):
        """FGMRES residual estimates per Arnoldi step of the last solve's first
        column, then its true relative residual (spaqr_solve_history)."""
        lib = _abi.load()
        n = C.c_int64()
        check(lib.spaqr_solve_history(self._h, None, 0, C.byref(n)), "spaqr_solve_history")
        buf = np.empty(max(1, n.value), dtype=np.float64)
        check(lib.spaqr_solve_history(self._h, buf.ctypes.data_as(C.POINTER(C.c_double)), buf.size, C.byref(n)),
              "spaqr_solve_history")
        return buf[:n.value]

    def stage_sizes(self, stage):
        lib = _abi.load()
        n = C.c_int64()
        check(lib.spaqr_stage_sizes(self._h, int(stage), None, 0, C.byref(n)), "spaqr_stage_sizes")
        buf = np.empty(max(1, n.value), dtype=np.int32)
        check(lib.spaqr_stage_sizes(self._h, int(stage), buf.ctypes.data_as(C.POINTER(C.c_int32)), buf.size,
                                    C.byref(n)), "spaqr_stage_sizes")
        return buf[:n.value]


def factor(A, ordering, eps=1e-2, **kw):
    return Factorization(A, ordering=ordering, eps=eps, **kw)


class DeviceCSR:
    """Device copies (torch CUDA tensors) of a CSR matrix's three arrays."""

    def __init__(self, A, device="cuda:0"):
        import torch
        self.rowptr = torch.from_numpy(np.ascontiguousarray(A.indptr, dtype=np.int64)).to(device)
        self.col = torch.from_numpy(np.ascontiguousarray(A.indices, dtype=np.int32)).to(device)
        self.val = torch.from_numpy(np.ascontiguousarray(A.data, dtype=np.float64)).to(device)


def factor_device(A, symbolic, dcsr, eps=1e-2, **kw):
    """Factorize with A's values taken from device memory (dcsr: DeviceCSR);
    A (host) supplies only the pattern the symbolic analysis was made from."""
    return Factorization(A, symbolic=symbolic, eps=eps, device_csr=dcsr, **kw)


def factor_batch(As, symbolics, dcsrs=None, eps=1e-2, skip=2, precision=32, restart=100, maxit=1000,
                 stream=None, scale=True):
    """Factorize several problems together (spaqr_factor_batch): stage by
    stage, all their fronts, scalings and sparsifications share one launch per
    phase.  As: scipy CSR matrices (the pattern; also the values when dcsrs is
    None); symbolics: their analyses; dcsrs: DeviceCSR copies or None.
    Returns one Factorization per problem."""
    lib = _abi.load()
    n = len(As)
    if n == 0 or len(symbolics) != n or (dcsrs is not None and len(dcsrs) != n):
        raise ValueError("factor_batch: one matrix and one analysis per problem")
    keep, csrs, devs = [], [], []
    for i, A in enumerate(As):
        s, k = _csr_struct(A)
        keep.append(k)
        csrs.append(s)
        if dcsrs is not None:
            d = dcsrs[i]
            devs.append(_abi.CSRDev(d.rowptr.data_ptr(), d.col.data_ptr(), d.val.data_ptr()))
    csr_p = (C.POINTER(CSR) * n)(*[C.pointer(s) for s in csrs])
    dev_p = (C.POINTER(_abi.CSRDev) * n)(*[C.pointer(d) for d in devs]) if dcsrs is not None else None
    sym_p = (C.c_void_p * n)(*[s.handle.value if hasattr(s.handle, "value") else s.handle for s in symbolics])
    out = (C.c_void_p * n)()
    o = make_opts(eps, skip, precision, restart, maxit, scale)
    st = lib.spaqr_factor_batch(n, csr_p, dev_p, sym_p, C.byref(o), _stream_ptr(stream), out)
    facs = [Factorization(As[i], symbolic=symbolics[i], _handle=C.c_void_p(out[i])) if out[i] else None
            for i in range(n)]
    del keep
    check(st, "spaqr_factor_batch")
    return facs


def solve_batch(facs, bs, tol=1e-10):
    """FGMRES for several factorizations at once (spaqr_solve_batch): every
    Arnoldi step applies all their preconditioners in one launch per phase.
    bs: torch CUDA tensors of shape (n_i,) or (n_i, nrhs_i) with contiguous
    columns (all on the device), or numpy arrays (all on the host).
    tol: one value or one per problem.  Returns (xs, infos)."""
    lib = _abi.load()
    n = len(facs)
    if n == 0 or len(bs) != n:
        raise ValueError("solve_batch: one right-hand side block per factorization")
    tols = [float(tol)] * n if np.isscalar(tol) else [float(t) for t in tol]
    on_dev = hasattr(bs[0], "is_cuda") and bs[0].is_cuda
    xs, bp, xp, nr = [], [], [], []
    if on_dev:
        import torch
        for f, b in zip(facs, bs):
            b2 = b if b.ndim == 2 else b.reshape(-1, 1)
            if b2.shape[0] != f.n or (b2.shape[1] > 1 and b2.stride(1) != f.n) or b2.stride(0) != 1:
                raise ValueError("device right-hand sides must be n x nrhs with contiguous columns")
            x = torch.empty_like(b)
            xs.append(x)
            bp.append(b.data_ptr())
            xp.append(x.data_ptr())
            nr.append(b2.shape[1])
    else:
        keep = []
        for f, b in zip(facs, bs):
            b = np.asarray(b, dtype=np.float64, order="F")
            if b.shape[0] != f.n:
                raise ValueError("right-hand side size differs from the factorization")
            x = np.empty_like(b, order="F")
            keep.append(b)
            xs.append(x)
            bp.append(b.ctypes.data)
            xp.append(x.ctypes.data)
            nr.append(1 if b.ndim == 1 else b.shape[1])
    hs = (C.c_void_p * n)(*[f._h.value if hasattr(f._h, "value") else f._h for f in facs])
    info = (SolveInfo * sum(nr))()
    st = lib.spaqr_solve_batch(n, hs, (C.c_void_p * n)(*bp), (C.c_void_p * n)(*xp), (C.c_int64 * n)(*nr),
                               1 if on_dev else 0, (C.c_double * n)(*tols), info)
    check(st, "spaqr_solve_batch")
    infos, c = [], 0
    for k in nr:
        infos.append([dict(iterations=i.iterations, converged=bool(i.converged), relres=i.relres,
                           seconds=i.seconds) for i in info[c:c + k]])
        c += k
    return xs, infos


def profile_enable(on=True, only=None):
    """Record per-launch HIP-event timings of every kernel, or only of `only`
    (one name, or a prefix ending in '*', e.g. 'host_*' for the host phases)."""
    check(_abi.load().spaqr_profile_enable(1 if on else 0, only.encode() if only else None),
          "spaqr_profile_enable")


def get_tuning():
    """The kernel dispatch thresholds (spaqr_get_tuning) as a dict."""
    t = _abi.Tuning()
    check(_abi.load().spaqr_get_tuning(C.byref(t)), "spaqr_get_tuning")
    return {k: getattr(t, k) for k, _ in _abi.Tuning._fields_}


def set_tuning(**kw):
    """Set some dispatch thresholds (the others keep their values); with no
    argument, restore the defaults (spaqr_set_tuning)."""
    lib = _abi.load()
    if not kw:
        check(lib.spaqr_set_tuning(None), "spaqr_set_tuning")
        return
    cur = get_tuning()
    unknown = set(kw) - set(cur)
    if unknown:
        raise ValueError(f"unknown tuning keys {sorted(unknown)}")
    cur.update(kw)
    check(lib.spaqr_set_tuning(C.byref(_abi.Tuning(**cur))), "spaqr_set_tuning")


def kernel_launches(kernel=None):
    """Launches of one kernel family (e.g. 'k_qr', 'k_cpqr_coop') since the
    last reset; kernel=None resets every count."""
    n = C.c_int64()
    check(_abi.load().spaqr_kernel_launches(kernel.encode() if kernel else None, C.byref(n)),
          "spaqr_kernel_launches")
    return n.value


def profile_query(kernel):
    n = C.c_int64()
    ms, fl, by = C.c_double(), C.c_double(), C.c_double()
    check(_abi.load().spaqr_profile_query(kernel.encode(), C.byref(n), C.byref(ms), C.byref(fl), C.byref(by)),
          "spaqr_profile_query")
    return dict(launches=n.value, total_ms=ms.value, flops=fl.value, bytes=by.value)


from .server import Server  # noqa: E402,F401
