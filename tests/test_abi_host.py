"""CPU checks of the C ABI: the library loads and exports every declared symbol, and the host
graph steps of the first multiplicative cycle (strength sets, Algorithm 1, interpolatory sets,
Kaczmarz colouring) agree bit for bit with the oracle."""
import ctypes as C
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import slamg_oracle as O
from paper_1102_0919_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_1102_0919_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        from paper_1102_0919_amd import build
        build.build()
    return L.load()


def _declared_symbols():
    names = []
    for h in ("slamg.h", "slamg_ops.h"):
        txt = open(os.path.join(ROOT, "include", h)).read()
        names += re.findall(r"^\s*(?:slamg_status|void|const char\s*\*)\s*(slamg_[a-z0-9_]+)\s*\(", txt, re.M)
    return sorted(set(names))


def test_every_declared_symbol_is_exported(lib):
    names = _declared_symbols()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings(lib):
    from paper_1102_0919_amd import api
    assert api.status_string(0) == "ok"
    assert api.status_string(-3) == "HBM budget exceeded"


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _strength(lib, N, theta, rule, top_s=4):
    N = sp.csr_matrix(N); N.sort_indices()
    n = N.shape[0]
    rp, ci, v = _i32(N.indptr), _i32(N.indices), np.ascontiguousarray(N.data, dtype=np.float64)
    sp_ = np.zeros(n + 1, np.int32); si = np.zeros(max(N.nnz, 1), np.int32)
    assert lib.slamg_graph_strength(n, _p(rp), _p(ci), _p(v), theta, rule, top_s, _p(sp_), _p(si)) == 0
    return sp_, si[:sp_[-1]], (rp, ci, v)


def _matrices():
    yield "laplace2d", W.laplace2d(14).to_scipy()
    yield "aniso3d", W.aniso3d(7, 0.01).to_scipy()
    G = W.gradient2d(12).to_scipy()
    yield "gradAAt", O.structural_product(G, G.T.tocsr())
    yield "gradAtA", O.structural_product(G.T.tocsr(), G)
    R = W.random_csr(120, 120, seed=11, mean_row=7).to_scipy()
    yield "random", sp.csr_matrix(R + R.T + 10 * sp.identity(120))


@pytest.mark.parametrize("rule,theta", [(0, 0.06), (0, 0.2), (1, 0.25), (2, 0.0)])
def test_strength_rs_interp_bitexact(lib, rule, theta):
    for name, N in _matrices():
        Sp, Si, (rp, ci, v) = _strength(lib, N, theta, rule)
        oSp, oSi = O.strength_sets(N, theta, rule, 4)
        assert np.array_equal(Sp, oSp) and np.array_equal(Si, oSi), name
        n = N.shape[0]
        isc = np.zeros(n, np.int8)
        assert lib.slamg_graph_rs(n, _p(Sp), _p(_i32(Si) if Si.size else np.zeros(1, np.int32)), _p(isc)) == 0
        ois = O.rs_coarsen(oSp, oSi, n)
        assert np.array_equal(isc.astype(bool), ois), name
        ptr = np.zeros(n + 1, np.int32); cols = np.zeros(Si.size + n + 1, np.int32); capped = C.c_int32()
        cap = 3
        assert lib.slamg_graph_interp(n, _p(Sp), _p(_i32(Si) if Si.size else np.zeros(1, np.int32)), _p(rp),
                                      _p(ci), _p(v), _p(isc), cap, _p(ptr), _p(cols), C.byref(capped)) == 0
        optr, ocols, ocap = O.interp_pattern(oSp, oSi, N, ois, cap)
        assert np.array_equal(ptr, optr) and np.array_equal(cols[:ptr[-1]], ocols) and capped.value == ocap, name


@pytest.mark.parametrize("rule,theta", [(0, 0.06), (1, 0.25), (2, 0.0)])
def test_strength_bitexact_row_parallel(lib, rule, theta):
    # above 8192 rows the strength sets are built on several host threads; the sets must equal the
    # oracle's row by row (term-document A A^t pattern with ties in |n_ij|)
    A = W.termdoc(12000, 3000, 20, seed=7).to_scipy()
    N = O.structural_product(A, A.T.tocsr())
    N = sp.csr_matrix((np.round(N.data * 7.0) % 5 + 1.0, N.indices, N.indptr), shape=N.shape)
    assert N.shape[0] >= 8192
    Sp, Si, _ = _strength(lib, N, theta, rule)
    oSp, oSi = O.strength_sets(N, theta, rule, 4)
    assert np.array_equal(Sp, oSp) and np.array_equal(Si, oSi)


def test_colouring_bitexact(lib):
    for M in (W.gradient2d(9).to_scipy(), W.gradient2d(9).to_scipy().T.tocsr(), W.laplace2d(11).to_scipy(),
              W.random_csr(80, 50, seed=4, mean_row=4).to_scipy()):
        M = sp.csr_matrix(M); M.sort_indices()
        m, n = M.shape
        col = np.zeros(m, np.int32)
        assert lib.slamg_graph_colour(m, n, _p(_i32(M.indptr)), _p(_i32(M.indices)), _p(col)) == 0
        assert np.array_equal(col, O.greedy_row_colouring(M))


def test_solve_rejects_invalid_inputs_without_device(lib):
    # argument validation happens before any device work
    from paper_1102_0919_amd import _lib as L
    p = L.Params()
    lib.slamg_params_init(C.byref(p), 0, 0)
    rp = np.array([0, 1, 2], np.int64); ci = np.array([1, 0], np.int32); v = np.array([1.0, 2.0])
    s = L.Csr(2, 2, 2, rp.ctypes.data, ci.ctypes.data, v.ctypes.data, 0)
    sig = np.zeros(1)
    # NULL context
    assert lib.slamg_solve(None, C.byref(s), 0, 0, 1, C.byref(p), None, _p(sig), None, None, None) == -1


def test_bf16_reference_rounding_worked_values():
    # the GPU tests' BF16 reference, pinned on the host: nearest BF16 of the FP32 value, ties to the
    # even pattern, infinity past the halfway point above the largest finite BF16
    from .test_gpu_ops import _bf16_nearest
    cases = [(1.0, 0x3F80), (1 + 2 ** -8, 0x3F80), (1 + 3 * 2 ** -8, 0x3F82), (1 + 2 ** -8 + 2 ** -20, 0x3F81),
             (-2.5, 0xC020), (2.0 ** -133, 0x0001), (2.0 ** -134, 0x0000), (3 * 2.0 ** -135, 0x0001),
             (3.3895313892515355e38, 0x7F7F), (3.4e38, 0x7F80), (np.inf, 0x7F80), (0.0, 0x0000), (-0.0, 0x8000)]
    got = _bf16_nearest(np.array([v for v, _ in cases]))
    assert [int(g) for g in got] == [p for _, p in cases]


def test_colouring_and_coarsening_bitexact_large(lib):
    # colours and the C/F split of Algorithm 1 (buckets by lambda) on larger and wider
    # patterns must equal the oracle's
    A = W.aniso3d(28, 0.01).to_scipy()
    G = sp.csr_matrix(O.structural_product(A, A))          # a wider, Galerkin-like pattern
    R = W.random_csr(20000, 15000, seed=3, mean_row=6).to_scipy()
    for M in (A, G, sp.csr_matrix(R)):
        M.sort_indices()
        m, n = M.shape
        assert m >= 16384
        col = np.zeros(m, np.int32)
        assert lib.slamg_graph_colour(m, n, _p(_i32(M.indptr)), _p(_i32(M.indices)), _p(col)) == 0
        assert np.array_equal(col, O.greedy_row_colouring(M))
    # Algorithm 1 on the stencil, on the wider pattern (many measures grow) and on a random square
    # pattern with the row-sum rule
    Rs = W.random_csr(16384, 16384, seed=5, mean_row=9).to_scipy()
    Rs = sp.csr_matrix(Rs + Rs.T)
    for N, theta, rule in ((sp.csr_matrix(A), 0.25, 1), (G, 0.25, 1), (Rs, 0.06, 0)):
        N.sort_indices()
        Sp, Si, _ = _strength(lib, N, theta, rule)
        isc = np.zeros(N.shape[0], np.int8)
        assert lib.slamg_graph_rs(N.shape[0], _p(Sp), _p(_i32(Si)), _p(isc)) == 0
        oSp, oSi = O.strength_sets(N, theta, rule, 4)
        assert np.array_equal(isc.astype(bool), O.rs_coarsen(oSp, oSi, N.shape[0]))
