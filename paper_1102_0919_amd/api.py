"""Thin Python binding of the slamg C ABI (same names as include/slamg.h without the prefix).

Argument marshalling only: every step of the method runs in libslamg.so.  Matrices are passed as
``workloads.CSR`` (or any object with m, n, indptr, indices, data) or scipy CSR; outputs are numpy
arrays.  PyTorch is used only for device memory in the step-level helpers of the tests.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _lib as L


class SlamgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{L.STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _as_csr(A):
    if hasattr(A, "indptr") and hasattr(A, "m"):
        return A.m, A.n, A.indptr, A.indices, A.data
    A = A.tocsr()
    A.sort_indices()
    return A.shape[0], A.shape[1], A.indptr, A.indices, A.data


def params_init(kind: str = "svd", target: str = "dominant", **overrides) -> L.Params:
    p = L.Params()
    lib = L.load()
    st = lib.slamg_params_init(C.byref(p), L.KIND[kind], L.TARGET[target])
    if st != 0:
        raise SlamgError(st, "params_init")
    names = {f[0] for f in L.Params._fields_}
    for k, v in overrides.items():
        if k == "precision" and isinstance(v, str):
            v = L.PRECISION[v]
        if k == "omega":
            k = "omega_J"
        if k not in names or k.startswith("reserved"):
            raise TypeError(f"params_init: unknown parameter {k!r}")
        setattr(p, k, v)
    return p


class Context:
    """A library context on one HIP device (slamg_create / slamg_destroy)."""

    def __init__(self, device: int = 0, stream: int | None = None, hbm_budget_bytes: int = 0):
        self.lib = L.load()
        self.h = C.c_void_p()
        st = self.lib.slamg_create(C.byref(self.h), device, C.c_void_p(stream) if stream else None,
                                   hbm_budget_bytes)
        if st != 0:
            raise SlamgError(st, "slamg_create failed")

    def close(self):
        if self.h:
            self.lib.slamg_destroy(self.h)
            self.h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self) -> str:
        return self.lib.slamg_last_error(self.h).decode()


def _csr_struct(A):
    m, n, indptr, indices, data = _as_csr(A)
    rp = np.ascontiguousarray(indptr, dtype=np.int64)
    ci = np.ascontiguousarray(indices, dtype=np.int32)
    v = np.ascontiguousarray(data, dtype=np.float64)
    s = L.Csr(m, n, int(rp[-1]), rp.ctypes.data, ci.ctypes.data, v.ctypes.data, 0)
    return s, (rp, ci, v)


@dataclass
class Result:
    sigma: np.ndarray
    U: np.ndarray
    V: np.ndarray | None
    status: int
    report: L.Report

    @property
    def converged(self) -> bool:
        return self.status == 0


def solve(ctx: Context, A, kind: str, target: str, n_b: int, params: L.Params | None = None,
          init_tests: np.ndarray | None = None, allow_not_converged: bool = True) -> Result:
    """slamg_solve: n_b extremal singular triplets (kind 'svd') or eigenpairs (kind 'spd')."""
    s, keep = _csr_struct(A)
    m, n = s.m, s.n
    if params is None:
        params = params_init(kind, target)
    sig = np.zeros(n_b)
    U = np.zeros((n_b, m))            # column-major m x n_b == row-major n_b x m
    V = np.zeros((n_b, n)) if kind == "svd" else None
    rep = L.Report()
    init = None
    if init_tests is not None:
        init = np.asfortranarray(init_tests, dtype=np.float64)
    st = ctx.lib.slamg_solve(ctx.h, C.byref(s), L.KIND[kind], L.TARGET[target], n_b, C.byref(params),
                             _ptr(init) if init is not None else None, _ptr(sig), _ptr(U),
                             _ptr(V) if V is not None else None, C.byref(rep))
    del keep
    if st not in (0, 1) or (st == 1 and not allow_not_converged):
        raise SlamgError(st, ctx.last_error())
    return Result(sig, U.T.copy(), None if V is None else V.T.copy(), st, rep)


class Matrix:
    """A matrix prepared once and kept resident in device memory (slamg_matrix_create)."""

    def __init__(self, ctx: Context, A, kind: str):
        s, keep = _csr_struct(A)
        self.ctx, self.kind, self.m, self.n = ctx, kind, s.m, s.n
        self.h = C.c_void_p()
        st = ctx.lib.slamg_matrix_create(ctx.h, C.byref(s), L.KIND[kind], C.byref(self.h))
        del keep
        if st != 0:
            raise SlamgError(st, ctx.last_error())

    def close(self):
        if self.h:
            self.ctx.lib.slamg_matrix_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_matrix(ctx: Context, M: Matrix, target: str, n_b: int, params: L.Params | None = None,
                 init_tests: np.ndarray | None = None, U_dev=None, V_dev=None, host_vectors: bool = False) -> Result:
    """slamg_solve_matrix.  With U_dev / V_dev (device tensors, column-major m x n_b / n x n_b, e.g.
    torch tensors of shape (n_b, m)) the vectors are written on the device; with host_vectors the
    vectors are returned as numpy arrays; otherwise only sigma and the report are returned."""
    if params is None:
        params = params_init(M.kind, target)
    sig = np.zeros(n_b)
    rep = L.Report()
    init = None if init_tests is None else np.asfortranarray(init_tests, dtype=np.float64)
    U = V = None
    if U_dev is not None or V_dev is not None:
        on_dev = 1
        pu = C.c_void_p(U_dev.data_ptr()) if U_dev is not None else None
        pv = C.c_void_p(V_dev.data_ptr()) if V_dev is not None else None
    elif host_vectors:
        on_dev = 0
        U = np.zeros((n_b, M.m)); V = np.zeros((n_b, M.n)) if M.kind == "svd" else None
        pu, pv = _ptr(U), (_ptr(V) if V is not None else None)
    else:
        on_dev, pu, pv = 0, None, None
    st = ctx.lib.slamg_solve_matrix(ctx.h, M.h, L.TARGET[target], n_b, C.byref(params),
                                    _ptr(init) if init is not None else None, _ptr(sig), pu, pv, on_dev,
                                    C.byref(rep))
    if st not in (0, 1):
        raise SlamgError(st, ctx.last_error())
    return Result(sig, None if U is None else U.T.copy(), None if V is None else V.T.copy(), st, rep)


def submit(ctx: Context, A, kind: str, target: str, n_b: int, params: L.Params | None = None) -> int:
    s, keep = _csr_struct(A)
    if params is None:
        params = params_init(kind, target)
    rid = C.c_uint64()
    st = ctx.lib.slamg_submit(ctx.h, C.byref(s), L.KIND[kind], L.TARGET[target], n_b, C.byref(params),
                              C.byref(rid))
    del keep
    if st != 0:
        raise SlamgError(st, ctx.last_error())
    return rid.value


def poll(ctx: Context, rid: int) -> bool:
    done = C.c_int32()
    st = ctx.lib.slamg_poll(ctx.h, rid, C.byref(done))
    if st != 0:
        raise SlamgError(st, ctx.last_error())
    return bool(done.value)


def wait(ctx: Context, rid: int) -> None:
    """slamg_wait: block until the request is done."""
    st = ctx.lib.slamg_wait(ctx.h, rid)
    if st != 0:
        raise SlamgError(st, ctx.last_error())


def fetch(ctx: Context, rid: int, m: int, n: int, n_b: int, kind: str, raise_errors: bool = True) -> Result:
    """slamg_fetch; with raise_errors False a failed request comes back as a Result with its status."""
    sig = np.zeros(n_b)
    U = np.zeros((n_b, m))
    V = np.zeros((n_b, n)) if kind == "svd" else None
    rep = L.Report()
    st = ctx.lib.slamg_fetch(ctx.h, rid, _ptr(sig), _ptr(U), _ptr(V) if V is not None else None, C.byref(rep))
    if st not in (0, 1) and (raise_errors or st == L.STATUS_BUSY):
        raise SlamgError(st, ctx.last_error())
    return Result(sig, U.T.copy(), None if V is None else V.T.copy(), st, rep)


def serve_start(ctx: Context, slots: int) -> None:
    """slamg_serve_start: solve submitted requests concurrently on `slots` streams."""
    st = ctx.lib.slamg_serve_start(ctx.h, slots)
    if st != 0:
        raise SlamgError(st, ctx.last_error())


def serve_stop(ctx: Context) -> None:
    st = ctx.lib.slamg_serve_stop(ctx.h)
    if st != 0:
        raise SlamgError(st, ctx.last_error())


def status_string(status: int) -> str:
    return L.load().slamg_status_string(status).decode()


def report_dict(rep: L.Report) -> dict:
    lv = rep.levels
    return dict(levels=lv, mult_cycles=rep.mult_cycles, add_iters=rep.add_iters, converged=bool(rep.converged),
                sizes=[(int(rep.rows[i]), int(rep.cols[i])) for i in range(max(lv, 1))],
                nnz=[int(rep.nnz[i]) for i in range(max(lv, 1))],
                colours=[int(rep.colours[i]) for i in range(max(lv, 1))],
                anorm=rep.anorm, t_setup_ms=rep.t_setup_ms, t_solve_ms=rep.t_solve_ms,
                rho_history=[rep.rho_history[i] for i in range(min(rep.add_iters + 1, 256))],
                p_dropped=rep.p_dropped)
