"""Helpers of the GPU tests: device copies (PyTorch tensors as device memory) and pointers."""
import ctypes as C
import os

import numpy as np


def lib():
    from paper_1102_0919_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        from paper_1102_0919_amd import build
        build.build()
    return L.load()


# Device tensors created by dev() stay referenced until release() runs (after each test), so that
# pointers taken inside an argument list stay valid while the library call runs.
_KEEP = []


def release():
    _KEEP.clear()


def dev(a, dtype=None):
    import torch
    a = np.ascontiguousarray(a if dtype is None else np.asarray(a, dtype=dtype))
    t = torch.from_numpy(a.copy()).to("cuda")
    _KEEP.append(t)
    return t


def ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def csr_dev(M):
    """Device (rp, ci, v) of a scipy CSR with int32 indices."""
    import scipy.sparse as sp
    M = sp.csr_matrix(M)
    M.sort_indices()
    return (dev(M.indptr, np.int32), dev(M.indices, np.int32), dev(M.data, np.float64))


def hp(a):
    return a.ctypes.data_as(C.c_void_p)
