"""Step-level parity of the HIP kernels with the oracle (one test per hot-path step).

FP64 tolerance: the kernels and the oracle sum in different orders, so an entry may differ by
(row length) * eps * sum_k |a_ik x_k|; tests use 1e-13 times that magnitude (eps = 2.2e-16 and
rows of at most ~40 entries give < 1e-14), or a stated bound derived the same way.
"""
import ctypes as C

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import slamg_oracle as O
from paper_1102_0919_amd import workloads as W

from .gpu_util import csr_dev, dev, host, hp, lib, ptr, release

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _keepalive():
    yield
    release()


def _close(x, ref, mag, rel=1e-13):
    x, ref, mag = np.asarray(x), np.asarray(ref), np.asarray(mag)
    err = np.abs(x - ref)
    ok = err <= rel * mag + 1e-300
    assert ok.all(), f"max err {err.max():.3e}, max allowed {(rel * mag).max():.3e}"


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available()
    return lib()


@pytest.mark.parametrize("w,mean_row", [(1, 7), (2, 7), (3, 7), (5, 7), (8, 7), (10, 7), (16, 7),
                                        (1, 20), (8, 20), (3, 80), (8, 80), (16, 40)])
def test_spmm_parity(L, w, mean_row):
    # skewed, ragged, empty rows; mean_row >= 20 takes the kernels' split-row variants
    A = W.random_csr(3001, 1777, seed=w, mean_row=mean_row).to_scipy()
    X = W.seeded_block(1777, w, seed=100 + w)
    Y0 = W.seeded_block(3001, w, seed=200 + w)
    rp, ci, v = csr_dev(A)
    dx, dy = dev(X), dev(Y0)
    assert L.slamg_op_spmm(3001, w, ptr(rp), ptr(ci), ptr(v), ptr(dx), ptr(dy), 0.5, None) == 0
    ref = A @ X + 0.5 * Y0
    _close(host(dy), ref, abs(A) @ abs(X) + 0.5 * abs(Y0))


def test_spmm_f32_parity(L):
    import torch
    A = W.random_csr(2000, 2000, seed=3, mean_row=7).to_scipy()
    X = W.seeded_block(2000, 8, seed=4)
    M = sp.csr_matrix(A); M.sort_indices()
    rp, ci = dev(M.indptr, np.int32), dev(M.indices, np.int32)
    v = dev(M.data.astype(np.float32))
    dx = dev(X.astype(np.float32)); dy = dev(np.zeros((2000, 8), np.float32))
    assert L.slamg_op_spmm_f32(2000, 8, ptr(rp), ptr(ci), ptr(v), ptr(dx), ptr(dy), 0.0, None) == 0
    ref = M.astype(np.float64) @ X
    # fp32 storage + fp32 accumulation: |err| <= (len + 2) u32 sum |a||x|, u32 = 6e-8
    _close(host(dy), ref, abs(M) @ abs(X), rel=40 * 6e-8)


def _bf16_nearest(x):
    """BF16 bit patterns of FP64 values by the definition: x rounded to FP32, then the nearer of the
    two BF16 neighbours of that FP32 value (ties to the even pattern; past the largest finite BF16
    the upper neighbour is 2^128, i.e. infinity).  NaN inputs are not handled here."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32)
    sign = u & np.uint32(0x80000000)
    mag = u & np.uint32(0x7FFFFFFF)
    lo = (mag >> 16).astype(np.uint64)                  # truncated pattern (toward zero)
    hi = lo + 1
    def val(pat):
        pat = np.asarray(pat, np.uint64)
        out = (pat.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
        return np.where(pat >= 0x7F80, 2.0 ** 128, out)
    a = np.abs(f.astype(np.float64))
    dlo, dhi = a - val(lo), val(hi) - a
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (lo % 2 == 1))
    pat = np.where(np.isinf(f), 0x7F80, np.where(pick_hi, hi, lo)).astype(np.uint32)
    return ((sign >> 16) | pat).astype(np.uint16)


def test_cast_bf16_bit_exact(L):
    rng = np.random.default_rng(16)
    special = [  # (value, its BF16 pattern)
        (0.0, 0x0000), (-0.0, 0x8000), (1.0, 0x3F80),
        (1 + 2 ** -8, 0x3F80),        # halfway between 1 and 1 + 2^-7: the even pattern, 1
        (1 + 3 * 2 ** -8, 0x3F82),    # halfway between 1 + 2^-7 and 1 + 2^-6: the even one, 1 + 2^-6
        (-(1 + 2 ** -8), 0xBF80),
        (2.0 ** -133, 0x0001),        # smallest subnormal BF16
        (3.3895313892515355e38, 0x7F7F),   # largest finite BF16
        (3.39e38, 0x7F7F),            # below the halfway point to 2^128
        (3.4e38, 0x7F80),             # above it: infinity
        (1e300, 0x7F80), (-1e300, 0xFF80), (np.inf, 0x7F80), (-np.inf, 0xFF80),
    ]
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.uniform(-40, 40, 20000),
                        [v for v, _ in special]])
    d_in = dev(x)
    d_out = dev(np.zeros(x.size, np.int16))
    assert L.slamg_op_cast_bf16(x.size, ptr(d_in), ptr(d_out), None) == 0
    got = host(d_out).view(np.uint16)
    with np.errstate(over="ignore"):
        ref = _bf16_nearest(x)
    assert np.array_equal(got, ref), np.flatnonzero(got != ref)[:10]
    for i, (v, pat) in enumerate(special):
        assert got[20000 + i] == pat, (v, hex(got[20000 + i]))
    nan = dev(np.array([np.nan, -np.nan]))
    d2 = dev(np.zeros(2, np.int16))
    assert L.slamg_op_cast_bf16(2, ptr(nan), ptr(d2), None) == 0
    g = host(d2).view(np.uint16)
    assert np.all((g & 0x7F80) == 0x7F80) and np.all((g & 0x7F) != 0)


@pytest.mark.parametrize("w,mean_row", [(8, 7), (3, 7), (8, 40), (16, 80)])
def test_spmm_bf16_parity(L, w, mean_row):
    A = W.random_csr(2500, 1900, seed=40 + w, mean_row=mean_row).to_scipy()
    M = sp.csr_matrix(A); M.sort_indices()
    bits = _bf16_nearest(M.data)
    vals = (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    X = W.seeded_block(1900, w, seed=41 + w).astype(np.float32)
    Y0 = W.seeded_block(2500, w, seed=42 + w).astype(np.float32)
    rp, ci = dev(M.indptr, np.int32), dev(M.indices, np.int32)
    v = dev(bits.view(np.int16))
    dx, dy = dev(X), dev(Y0)
    assert L.slamg_op_spmm_bf16(2500, w, ptr(rp), ptr(ci), ptr(v), ptr(dx), ptr(dy), 0.5, None) == 0
    Mb = sp.csr_matrix((vals, M.indices, M.indptr), shape=M.shape)
    ref = Mb @ X.astype(np.float64) + 0.5 * Y0.astype(np.float64)
    # FP32 products and sums of exactly representable BF16 values: (len + 2) u32 sum |a||x|
    row_len = np.diff(M.indptr).max()
    _close(host(dy), ref, abs(Mb) @ abs(X.astype(np.float64)) + 0.5 * abs(Y0), rel=(row_len + 3) * 6e-8)


def _svd_level(m, n, seed, coarse):
    rng = np.random.default_rng(seed)
    A = sp.csr_matrix(W.random_csr(m, n, seed=seed, mean_row=5, empty_rows=False).to_scipy())
    if coarse:
        Bh = sp.random(m, m, density=0.05, random_state=seed) ; Bd = sp.csr_matrix(Bh @ Bh.T + 3 * sp.identity(m))
        Ch = sp.random(n, n, density=0.05, random_state=seed + 1); Cd = sp.csr_matrix(Ch @ Ch.T + 3 * sp.identity(n))
    else:
        Bd, Cd = sp.identity(m, format="csr"), sp.identity(n, format="csr")
    for M in (A, Bd, Cd):
        M.sort_indices()
    return O.Level(A, Bd, Cd), rng


@pytest.mark.parametrize("coarse", [False, True])
def test_relaxation_dominant_svd_parity(L, coarse):
    lev, rng = _svd_level(1500, 900, 7, coarse)
    A, B, Cm = lev.A, lev.B, lev.C
    w = 6
    U, V = rng.uniform(-1, 1, (1500, w)), rng.uniform(-1, 1, (900, w))
    a, at = csr_dev(A), csr_dev(A.T.tocsr())
    b = csr_dev(B) if coarse else (None, None, None)
    c = csr_dev(Cm) if coarse else (None, None, None)
    du, dv = dev(U), dev(V)
    assert L.slamg_op_relax_test(0, 1500, 900, w, *map(ptr, a), *map(ptr, at), *map(ptr, b), *map(ptr, c), 0.7,
                                 ptr(du), ptr(dv), None) == 0
    Ur, Vr = O.relax_test_dominant(lev, O.SVD, U, V, 0.7)
    _close(host(du), Ur, np.abs(Ur) + 1e-3, rel=1e-12)
    _close(host(dv), Vr, np.abs(Vr) + 1e-3, rel=1e-12)
    sig = rng.uniform(1.0, 3.0, w)
    kap, tau = rng.normal(size=(1500, w)), rng.normal(size=(900, w))
    du, dv, ds, dk, dt = dev(U), dev(V), dev(sig), dev(kap), dev(tau)
    assert L.slamg_op_relax_boot(0, 1500, 900, w, *map(ptr, a), *map(ptr, at), *map(ptr, b), *map(ptr, c),
                                 ptr(ds), ptr(dk), ptr(dt), 0.7, ptr(du), ptr(dv), None) == 0
    Ub, Vb = O.relax_boot_dominant(lev, O.SVD, U, V, sig, kap, tau, 0.7)
    _close(host(du), Ub, np.abs(Ub) + 10, rel=1e-13)
    _close(host(dv), Vb, np.abs(Vb) + 10, rel=1e-13)


@pytest.mark.parametrize("coarse", [False, True])
def test_relaxation_dominant_spd_parity(L, coarse):
    A = sp.csr_matrix(W.laplace2d(40).to_scipy())
    n = A.shape[0]
    diag_mask = A.indices == np.repeat(np.arange(n), np.diff(A.indptr))
    bdata = np.where(diag_mask, 2.0, 0.1)
    if coarse:
        Bd = sp.csr_matrix((bdata, A.indices.copy(), A.indptr.copy()), shape=A.shape)
    else:
        Bd = sp.identity(n, format="csr")
    lev = O.Level(A, Bd, None)
    rng = np.random.default_rng(1)
    X = rng.uniform(-1, 1, (n, 8))
    a = csr_dev(A)
    bv = dev(bdata) if coarse else None
    dx = dev(X)
    assert L.slamg_op_relax_test(1, n, n, 8, *map(ptr, a), None, None, None, None, None, ptr(bv), None, None,
                                 None, 0.7, ptr(dx), None, None) == 0
    Xr, _ = O.relax_test_dominant(lev, O.SPD, X, None, 0.7)
    _close(host(dx), Xr, np.abs(Xr) + 1e-3, rel=1e-12)
    sig = rng.uniform(4.0, 8.0, 8); kap = rng.normal(size=(n, 8))
    dx, ds, dk = dev(X), dev(sig), dev(kap)
    assert L.slamg_op_relax_boot(1, n, n, 8, *map(ptr, a), None, None, None, None, None, ptr(bv), None, None,
                                 None, ptr(ds), ptr(dk), None, 0.7, ptr(dx), None, None) == 0
    Xb, _ = O.relax_boot_dominant(lev, O.SPD, X, None, sig, kap, None, 0.7)
    _close(host(dx), Xb, np.abs(Xb) + 10, rel=1e-13)


@pytest.mark.parametrize("shifted,dense", [(False, False), (True, False), (False, True), (True, True)])
def test_kaczmarz_parity(L, shifted, dense):
    if dense:
        # Galerkin-like operator: long rows (split-row kernels), shifted by a B on the same pattern
        M = sp.csr_matrix(W.random_csr(700, 700, seed=9, mean_row=35, empty_rows=False).to_scipy()
                          + 4 * sp.identity(700))
    elif shifted:
        M = sp.csr_matrix(W.aniso3d(9, 0.01).to_scipy())
    else:
        M = sp.csr_matrix(W.gradient2d(30).to_scipy())
    M.sort_indices()
    Bv = None
    if dense and shifted:
        Bv = np.where(M.indices == np.repeat(np.arange(M.shape[0]), np.diff(M.indptr)), 2.0,
                      np.random.default_rng(3).uniform(-0.2, 0.2, M.nnz))
    nr, nc = M.shape
    col = O.greedy_row_colouring(M)
    groups = O.colour_groups(col)
    rows = np.concatenate(groups).astype(np.int32)
    cptr = np.concatenate([[0], np.cumsum([g.size for g in groups])]).astype(np.int32)
    rng = np.random.default_rng(5)
    w = 8
    x0 = rng.uniform(-1, 1, (nc, w)); rhs = rng.normal(size=(nr, w))
    lam = rng.uniform(0.0, 0.3, w)
    rp, ci, v = csr_dev(M)
    dx, dr = dev(x0), dev(rhs)
    dl = dev(lam) if shifted else None
    db = dev(Bv) if Bv is not None else None
    assert L.slamg_op_kaczmarz(nr, nc, w, ptr(rp), ptr(ci), ptr(v), ptr(db), ptr(dl), hp(rows), hp(cptr),
                               len(groups), ptr(dr), ptr(dx), None) == 0
    if shifted:
        Bm = sp.csr_matrix((Bv, M.indices, M.indptr), shape=M.shape) if Bv is not None else sp.identity(nr)
        ref = x0.copy()
        for j in range(w):
            Mj = sp.csr_matrix(M - lam[j] * Bm)
            ref[:, j:j + 1] = O.kaczmarz_sweep(Mj, x0[:, j:j + 1], rhs[:, j:j + 1], groups)
    else:
        ref = O.kaczmarz_sweep(M, x0, rhs, groups)
    _close(host(dx), ref, np.abs(ref) + 1.0, rel=1e-12)


@pytest.mark.parametrize("mean_row", [5, 30])
def test_residual_and_dots_parity(L, mean_row):
    lev, rng = _svd_level(1200, 700, 3, True)
    B = lev.B
    A = sp.csr_matrix(W.random_csr(1200, 700, seed=3, mean_row=mean_row, empty_rows=False).to_scipy())
    A.sort_indices()
    w = 5
    U, V = rng.normal(size=(1200, w)), rng.normal(size=(700, w))
    kap = rng.normal(size=(1200, w)); sig = rng.uniform(0.5, 2, w)
    a, b = csr_dev(A), csr_dev(B)
    out = dev(np.zeros((1200, w)))
    assert L.slamg_op_residual(1200, w, *map(ptr, a), ptr(dev(V)), *map(ptr, b), ptr(dev(U)), ptr(dev(kap)),
                               ptr(dev(sig)), ptr(out), None) == 0
    ref = kap - (A @ V - (B @ U) * sig)
    _close(host(out), ref, abs(kap) + abs(A) @ abs(V) + (abs(B) @ abs(U)) * sig)
    h = np.zeros(w)
    assert L.slamg_op_dots(1200, w, ptr(dev(U)), *map(ptr, a), ptr(dev(V)), None, None, hp(h), None) == 0
    refd = np.sum(U * (A @ V), axis=0)
    _close(h, refd, np.sum(np.abs(U) * (abs(A) @ abs(V)), axis=0), rel=1e-12)
    assert L.slamg_op_dots(1200, w, None, *map(ptr, a), ptr(dev(V)), ptr(dev(U)), ptr(dev(sig)), hp(h), None) == 0
    _close(h, np.sum((A @ V - U * sig) ** 2, axis=0), np.sum((abs(A) @ abs(V) + abs(U) * sig) ** 2, axis=0),
           rel=1e-12)


@pytest.mark.parametrize("rows,w", [(1, 3), (37, 8), (5003, 8), (100003, 16), (4096, 10)])
def test_gram_mfma_parity(L, rows, w):
    X = W.seeded_block(rows, w, seed=rows)
    Y = W.seeded_block(rows, w, seed=rows + 1)
    g = np.zeros((w, w))
    assert L.slamg_op_gram(rows, w, ptr(dev(X)), ptr(dev(Y)), hp(g), None) == 0
    _close(g, X.T @ Y, np.abs(X).T @ np.abs(Y), rel=1e-12)     # non-symmetric: checks the lane layout


@pytest.mark.parametrize("kind,target", [("svd", "dominant"), ("svd", "minimal"), ("spd", "minimal"),
                                         ("spd", "dominant")])
def test_ritz_parity(L, kind, target):
    rng = np.random.default_rng(9)
    if kind == "svd":
        A = sp.csr_matrix(W.gradient2d(20).to_scipy())
    else:
        A = sp.csr_matrix(W.laplace2d(25).to_scipy())
    m, n = A.shape
    w = 6
    U, V = rng.normal(size=(m, w)), rng.normal(size=(n, w))
    sig_o, Uo, Vo = O.ritz(A, kind, target, U, V if kind == "svd" else None)
    a = csr_dev(A)
    du, dv = dev(U), dev(V)
    hs = np.zeros(w)
    assert L.slamg_op_ritz(1 if kind == "spd" else 0, 1 if target == "minimal" else 0, m, n, w, *map(ptr, a),
                           ptr(du), ptr(dv) if kind == "svd" else None, hp(hs), None) == 0
    assert np.allclose(hs, sig_o, rtol=1e-11, atol=1e-13 * abs(sig_o).max())
    Ug = host(du)
    # vectors: unique up to sign for simple Ritz values
    for j in range(w):
        s = np.sign(Ug[:, j] @ Uo[:, j])
        assert np.allclose(Ug[:, j] * s, Uo[:, j], atol=1e-9)
    assert np.allclose(Ug.T @ Ug, np.eye(w), atol=1e-12)
    if kind == "svd":
        Vg = host(dv)
        assert np.allclose(A @ Vg - Ug * hs, Uo * 0 + (A @ Vo - Uo * sig_o) * np.sign(np.sum(Ug * Uo, 0)),
                           atol=1e-10)


@pytest.mark.parametrize("nnull,seed", [(1, 0), (1, 2), (1, 3), (3, 1), (6, 2)])
def test_ritz_zero_singular_values(L, nnull, seed):
    # a block V whose span meets null(A) in nnull dimensions makes the w x w Ritz matrix rank
    # deficient: its zero singular values come first for a minimal target with their left vectors
    # completed to an orthonormal set, so the new U and V stay orthonormal, U^t A V is the diagonal
    # of the Ritz values, and the nonzero Ritz values agree with the oracle's.  With 16 columns the
    # complement of the nonzero left vectors can have no unit-vector component above 1/2 (seeds 0, 2
    # and 3 of one null direction, seed 2 of six).
    rng = np.random.default_rng(seed * 10 + nnull)
    m, n, w = 60, 50, 16
    Ad = sp.random(m, n, density=0.3, random_state=np.random.RandomState(seed * 10 + nnull), format="lil")
    Ad[:, :10] = 0.0
    A = sp.csr_matrix(Ad)
    U = rng.normal(size=(m, w))
    V = rng.normal(size=(n, w))
    V[10:, w - nnull:] = 0.0           # the last nnull columns lie in null(A)
    sig_o, _, _ = O.ritz(A, "svd", "minimal", U, V)
    assert np.all(sig_o[:nnull] <= 1e-13 * sig_o[-1]) and sig_o[nnull] > 1e-3 * sig_o[-1]
    a = csr_dev(A)
    du, dv = dev(U), dev(V)
    hs = np.zeros(w)
    assert L.slamg_op_ritz(0, 1, m, n, w, *map(ptr, a), ptr(du), ptr(dv), hp(hs), None) == 0
    Ug, Vg = host(du), host(dv)
    smax = sig_o[-1]
    assert np.all(hs[:nnull] <= 1e-13 * smax)
    assert np.allclose(hs[nnull:], sig_o[nnull:], rtol=1e-11)
    assert np.allclose(Ug.T @ Ug, np.eye(w), atol=1e-12)
    assert np.allclose(Vg.T @ Vg, np.eye(w), atol=1e-12)
    assert np.allclose(Ug.T @ (A @ Vg), np.diag(hs), atol=1e-12 * smax)


@pytest.mark.parametrize("boots", [False, True])
def test_ls_fit_parity(L, boots):
    N = W.laplace2d(30).to_scipy()
    Sp, Si = O.strength_sets(N, 0.06, 0)
    is_c = O.rs_coarsen(Sp, Si, N.shape[0])
    ptr_, cols, _ = O.interp_pattern(Sp, Si, N, is_c, 7)
    rng = np.random.default_rng(3)
    n = N.shape[0]
    U1 = rng.normal(size=(n, 8)); U2 = rng.normal(size=(n, 4)) if boots else None
    B1 = U1 + 0.01 * rng.normal(size=U1.shape)
    wts = rng.uniform(0.1, 2.0, 12 if boots else 8)
    Uf = np.hstack([U1, U2]) if boots else U1
    Bf = np.hstack([B1, U2]) if boots else B1
    P = O.ls_interpolation(ptr_, cols, is_c, Uf, Bf, wts)
    pv = np.zeros(ptr_[-1])
    assert L.slamg_op_ls_fit(n, hp(ptr_.astype(np.int32)), hp(cols.astype(np.int32)), hp(is_c.astype(np.int8)), 8,
                             ptr(dev(U1)), ptr(dev(B1)), 4 if boots else 0, ptr(dev(U2)) if boots else None, None,
                             ptr(dev(wts)), hp(pv), None) == 0
    # normal equations solved by LU (oracle) and Cholesky (kernel): both backward stable
    assert np.allclose(pv, P.data, rtol=1e-8, atol=1e-10)


def test_galerkin_spgemm_parity(L):
    A = sp.csr_matrix(W.gradient2d(25).to_scipy())
    rng = np.random.default_rng(2)
    m, n = A.shape
    P = sp.csr_matrix(sp.random(m, m // 3, density=3.0 / (m // 3), random_state=1) + sp.eye(m, m // 3))
    Q = sp.csr_matrix(sp.random(n, n // 2, density=3.0 / (n // 2), random_state=2) + sp.eye(n, n // 2))
    for M in (P, Q):
        M.sort_indices()
    Pt, At, Qt = P.T.tocsr(), A.T.tocsr(), Q.T.tocsr()
    S1 = O.structural_product(Pt, A)
    Ac = O.structural_product(S1, Q)
    # S1 = P^t A: rows of P^t . rows of A^t ; Ac = S1 Q: rows of S1 . rows of Q^t
    def run(Cpat, Lm, Rt):
        rowc = np.repeat(np.arange(Cpat.shape[0]), np.diff(Cpat.indptr)).astype(np.int32)
        out = dev(np.zeros(Cpat.nnz))
        assert L.slamg_op_spgemm(Cpat.nnz, ptr(dev(rowc)), ptr(dev(Cpat.indices, np.int32)), *map(ptr, csr_dev(Lm)),
                                 *map(ptr, csr_dev(Rt)), ptr(out), None) == 0
        return host(out)
    s1 = run(S1, Pt, At)
    assert np.allclose(s1, S1.data, rtol=1e-13, atol=1e-14)
    S1g = sp.csr_matrix((s1, S1.indices, S1.indptr), shape=S1.shape)
    ac = run(Ac, S1g, Qt)
    assert np.allclose(ac, Ac.data, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("s", [1, 4, 16])
def test_topsel_parity(L, s):
    # the top-s rule of §3.7 on the device (one workgroup per row, per-thread lists merged in LDS)
    # against the oracle's strength sets: values from a small integer set (ties broken to the lower
    # column), explicit zeros and the diagonal left out, rows longer than a workgroup and empty rows
    rng = np.random.default_rng(11 + s)
    m, n = 300, 2000
    rows = []
    for i in range(m):
        k = 0 if i % 37 == 0 else int(rng.integers(1, 900 if i % 5 == 0 else 40))
        cols = np.sort(rng.choice(n, size=k, replace=False))
        rows.append(cols)
    indptr = np.concatenate([[0], np.cumsum([len(c) for c in rows])]).astype(np.int32)
    indices = np.concatenate(rows).astype(np.int32) if indptr[-1] else np.zeros(0, np.int32)
    data = rng.integers(-4, 5, size=indices.size).astype(np.float64) * 0.5
    N = sp.csr_matrix((data, indices, indptr), shape=(m, n))
    oc = dev(np.zeros(m * s, np.int32))
    ov = dev(np.zeros(m * s))
    assert L.slamg_op_topsel(m, ptr(dev(indptr)), ptr(dev(indices)), ptr(dev(data)), s, ptr(oc), ptr(ov), None) == 0
    gc, gv = host(oc).reshape(m, s), host(ov).reshape(m, s)
    Sp, Si = O.strength_sets(N, 0.0, 2, top_s=s)
    for i in range(m):
        want = np.asarray(Si[Sp[i]:Sp[i + 1]])
        got = gc[i][gc[i] >= 0]
        assert np.array_equal(got, want), (i, got, want)
        assert np.array_equal(gv[i][: got.size], np.array([N[i, j] for j in got]))
        assert np.all(gc[i][got.size:] == -1)
    assert L.slamg_op_topsel(m, ptr(dev(indptr)), ptr(dev(indices)), ptr(dev(data)), 17, ptr(oc), ptr(ov), None) != 0


@pytest.mark.parametrize("kind,target,m,n", [("svd", "dominant", 70, 40), ("svd", "minimal", 70, 40),
                                             ("svd", "dominant", 40, 70), ("svd", "minimal", 40, 70),
                                             ("svd", "minimal", 33, 32), ("spd", "minimal", 90, 90),
                                             ("spd", "dominant", 90, 90)])
def test_coarse_gsvd_parity(L, kind, target, m, n):
    # m < n: min(m, n) generalized singular values (Theorem 3.2); the n - m directions of the null
    # space of A are not triplets and a minimal solve must not return them
    rng = np.random.default_rng(4)
    if kind == "svd":
        Ad = rng.uniform(-1, 1, (m, n))
        Bh = rng.uniform(-1, 1, (m, m)); Bd = Bh @ Bh.T / m + np.eye(m)
        Ch = rng.uniform(-1, 1, (n, n)); Cd = Ch @ Ch.T / n + np.eye(n)
        lev = O.Level(sp.csr_matrix(Ad), sp.csr_matrix(Bd), sp.csr_matrix(Cd))
    else:
        Ah = rng.uniform(-1, 1, (m, m)); Ad = Ah @ Ah.T / m + 0.1 * np.eye(m)
        Bh = rng.uniform(-1, 1, (m, m)); Bd = Bh @ Bh.T / m + np.eye(m)
        Cd = None
        lev = O.Level(sp.csr_matrix(Ad), sp.csr_matrix(Bd), None)
    nb = 6
    so, Uo, Vo = O.coarsest_gsvd(lev, kind, target, nb)
    hs, hu, hv = np.zeros(nb), np.zeros((m, nb)), np.zeros((n, nb))
    assert L.slamg_op_coarse_gsvd(1 if kind == "spd" else 0, 1 if target == "minimal" else 0, m, n, nb,
                                  hp(np.ascontiguousarray(Ad)), hp(np.ascontiguousarray(Bd)),
                                  hp(np.ascontiguousarray(Cd)) if Cd is not None else None, hp(hs), hp(hu),
                                  hp(hv)) == 0
    # eigen-decomposition of D^t D: sigma accurate to eps * sigma_max^2 / sigma
    smax = np.linalg.svd(Ad, compute_uv=False)[0] * 10
    # sigma_k = ||X w_k||: an error delta in w_k enters only as delta^2, so sigma is accurate to a
    # few eps sigma_max, including the smallest ones
    assert np.all(np.abs(hs - so) <= 1e-12 * smax), np.abs(hs - so) / smax
    for j in range(nb):
        s = np.sign(hu[:, j] @ Bd @ Uo[:, j])
        assert np.allclose(hu[:, j] * s, Uo[:, j], atol=1e-7)
        if kind == "svd":
            assert np.allclose(hv[:, j] * s, Vo[:, j], atol=1e-7)


@pytest.mark.parametrize("m,n", [(50, 30), (30, 50), (31, 31)])
def test_coarse_gsvd_zero_singular_value(L, m, n):
    # a rank-deficient A (one row and one column are combinations of the others) has a genuine zero
    # generalized singular value; its triplet is not unique, so the test checks that the returned
    # one satisfies A v = 0, A^t u = 0 and the B / C orthonormality, and that the others match the
    # oracle's
    rng = np.random.default_rng(9)
    Ad = rng.uniform(-1, 1, (m, n))
    Ad[:, -1] = Ad[:, :-1] @ rng.uniform(-1, 1, n - 1) / n
    Ad[-1, :] = rng.uniform(-1, 1, m - 1) @ Ad[:-1, :] / m
    Bh = rng.uniform(-1, 1, (m, m)); Bd = Bh @ Bh.T / m + np.eye(m)
    Ch = rng.uniform(-1, 1, (n, n)); Cd = Ch @ Ch.T / n + np.eye(n)
    lev = O.Level(sp.csr_matrix(Ad), sp.csr_matrix(Bd), sp.csr_matrix(Cd))
    nb = 4
    so, Uo, Vo = O.coarsest_gsvd(lev, "svd", "minimal", nb)
    assert so[0] < 1e-12 and so[1] > 1e-3          # the zero is simple among the min(m, n) values
    hs, hu, hv = np.zeros(nb), np.zeros((m, nb)), np.zeros((n, nb))
    assert L.slamg_op_coarse_gsvd(0, 1, m, n, nb, hp(np.ascontiguousarray(Ad)), hp(np.ascontiguousarray(Bd)),
                                  hp(np.ascontiguousarray(Cd)), hp(hs), hp(hu), hp(hv)) == 0
    smax = np.linalg.svd(Ad, compute_uv=False)[0] * 10
    assert hs[0] <= 1e-7 * smax
    assert np.linalg.norm(Ad @ hv[:, 0]) <= 1e-10 * smax
    assert np.linalg.norm(Ad.T @ hu[:, 0]) <= 1e-10 * smax
    assert np.allclose(hu.T @ Bd @ hu, np.eye(nb), atol=1e-9)
    assert np.allclose(hv.T @ Cd @ hv, np.eye(nb), atol=1e-9)
    assert np.allclose(hs[1:], so[1:], rtol=1e-9)
    for j in range(1, nb):
        s = np.sign(hu[:, j] @ Bd @ Uo[:, j])
        assert np.allclose(hu[:, j] * s, Uo[:, j], atol=1e-7)
        assert np.allclose(hv[:, j] * s, Vo[:, j], atol=1e-7)


def _proj_svd(L, M, nb, minimal):
    k = M.shape[0]
    hs, hy, hz = np.zeros(nb), np.zeros((k, nb)), np.zeros((k, nb))
    assert L.slamg_op_proj_svd(1 if minimal else 0, k, nb, hp(np.ascontiguousarray(M)), hp(hs), hp(hy), hp(hz)) == 0
    return hs, hy, hz


@pytest.mark.parametrize("k,nb", [(1, 1), (2, 1), (7, 7), (16, 8), (17, 8), (24, 8), (31, 12), (32, 8), (32, 32)])
@pytest.mark.parametrize("target", ["dominant", "minimal"])
def test_proj_svd_parity(L, k, nb, target):
    # the projected problem of the LOBPCG step for SVD targets (§7): the oracle takes it by a dense
    # SVD of the k x k matrix; singular values agree to a few eps sigma_max, the triplets satisfy
    # M z = sigma y and M^t y = sigma z with orthonormal y and z, and vectors of well separated
    # values agree up to sign
    rng = np.random.default_rng(k * 100 + nb)
    M = rng.standard_normal((k, k))
    hs, hy, hz = _proj_svd(L, M, nb, target == "minimal")
    Yo, so, Zto = np.linalg.svd(M)
    order = np.argsort(so) if target == "minimal" else np.argsort(-so)
    sel = order[:nb]
    smax = so[0]
    assert np.all(np.abs(hs - so[sel]) <= 1e-13 * smax), np.abs(hs - so[sel]) / smax
    assert np.linalg.norm(M @ hz - hy * hs[None, :]) <= 1e-13 * smax
    assert np.linalg.norm(M.T @ hy - hz * hs[None, :]) <= 1e-13 * smax
    assert np.allclose(hy.T @ hy, np.eye(nb), atol=1e-13)
    assert np.allclose(hz.T @ hz, np.eye(nb), atol=1e-13)
    for j, src in enumerate(sel):
        gap = np.min(np.abs(np.delete(so, src) - so[src])) if k > 1 else smax
        if gap < 1e-3 * smax:
            continue
        sgn = np.sign(hz[:, j] @ Zto[src])
        assert np.allclose(hz[:, j] * sgn, Zto[src], atol=1e-10)
        assert np.allclose(hy[:, j] * sgn, Yo[:, src], atol=1e-10)


@pytest.mark.parametrize("k,nb,nzero", [(9, 4, 2), (20, 6, 3), (32, 32, 5), (16, 16, 1), (32, 8, 1), (32, 32, 31),
                                        (5, 5, 5)])
def test_proj_svd_zero_singular_values(L, k, nb, nzero):
    # a projected matrix of rank k - nzero: its zero singular values come first for a minimal target,
    # with y completed to an orthonormal set in the left null space, and the rest agree with the
    # dense SVD
    rng = np.random.default_rng(k + nzero)
    Uq, _ = np.linalg.qr(rng.standard_normal((k, k)))
    Vq, _ = np.linalg.qr(rng.standard_normal((k, k)))
    s = np.concatenate([np.zeros(nzero), np.linspace(0.5, 3.0, k - nzero)])
    M = (Uq * s[None, :]) @ Vq.T
    hs, hy, hz = _proj_svd(L, M, nb, True)
    so = np.sort(np.linalg.svd(M, compute_uv=False))[:nb]
    smax = 3.0
    assert np.all(np.abs(hs - so) <= 1e-13 * smax), np.abs(hs - so) / smax
    nz = min(nzero, nb)
    assert np.all(hs[:nz] <= 1e-13 * smax)
    assert np.linalg.norm(M @ hz[:, :nz]) <= 1e-13 * smax
    assert np.linalg.norm(M.T @ hy[:, :nz]) <= 1e-13 * smax
    assert np.linalg.norm(M @ hz - hy * hs[None, :]) <= 1e-13 * smax
    assert np.allclose(hy.T @ hy, np.eye(nb), atol=1e-13)
    assert np.allclose(hz.T @ hz, np.eye(nb), atol=1e-13)


def test_proj_svd_rejects_sizes(L):
    M = np.eye(33)
    hs, hy, hz = np.zeros(33), np.zeros((33, 33)), np.zeros((33, 33))
    assert L.slamg_op_proj_svd(0, 33, 8, hp(M), hp(hs), hp(hy), hp(hz)) == -1
    assert L.slamg_op_proj_svd(0, 8, 9, hp(M), hp(hs), hp(hy), hp(hz)) == -1
    assert L.slamg_op_proj_svd(0, 8, 0, hp(M), hp(hs), hp(hy), hp(hz)) == -1
    assert L.slamg_op_proj_svd(0, 0, 0, hp(M), hp(hs), hp(hy), hp(hz)) == -1


@pytest.mark.parametrize("variant,m,n", [(0, 30, 20), (1, 30, 20), (2, 30, 20), (3, 30, 20), (4, 30, 20), (5, 30, 20),
                                         (5, 60, 40), (2, 34, 30),
                                         (3, 33, 30), (4, 34, 30), (2, 40, 25), (3, 40, 25), (0, 60, 40), (2, 60, 40),
                                         (3, 60, 40), (4, 60, 40), (0, 120, 90), (2, 120, 90), (3, 120, 90),
                                         (1, 120, 90)])
def test_coarse_solve_parity(L, variant, m, n):
    # N = m + n: up to 74 keeps all three eigensolve arrays in LDS (up to 64 with the dense products
    # on the matrix cores and the fourth array of the Newton-type steps: 63 and 64 are a ragged and a
    # full 64 x 64 tile set, 65 the scalar products), 100 the matrix only (up to 128), 210 none;
    # variants 2-5 are warm starts (Newton-type steps where they fit, else Jacobi sweeps /
    # first-order update / Jacobi sweeps / Newton after re-orthonormalising)
    import scipy.linalg as sla
    rng = np.random.default_rng(6)
    Ad = rng.uniform(-1, 1, (m, n))
    Bh = rng.uniform(-1, 1, (m, m)); Bd = Bh @ Bh.T / m + np.eye(m)
    Ch = rng.uniform(-1, 1, (n, n)); Cd = Ch @ Ch.T / n + np.eye(n)
    lev = O.Level(sp.csr_matrix(Ad), sp.csr_matrix(Bd), sp.csr_matrix(Cd))
    X, Y = O.pencil_matrices(lev, O.SVD)
    mu = sla.eigh(X, Y, eigvals_only=True)
    # one shift next to a generalized singular value: X - sigma Y nearly singular there
    sig = np.array([mu[-1] * (1 + 1e-9), 0.7, 1.3, 2.1])
    rhs = rng.normal(size=(m + n, 4))
    if variant in (2, 3, 4, 5):
        # the inputs take the intended branch: in the eigenbasis at sigma (1 + delta), the largest
        # first-order ratio |E_pq| / |d_q - d_p| is far inside 2^-26 (variant 3), inside 1e-4
        # (variant 2) or above it (variant 4)
        delta = {2: 1e-6, 3: 1e-12, 4: 1e-3, 5: 1e-6}[variant]
        worst = 0.0
        for s in sig:
            lam2, Q2 = np.linalg.eigh(X - s * (1 + delta) * Y)
            Mq = Q2.T @ (X - s * Y) @ Q2
            gap = np.abs(lam2[:, None] - lam2[None, :]) + np.eye(m + n)
            worst = max(worst, (np.abs(Mq - np.diag(np.diag(Mq))) / gap).max())
        assert {2: 1e-7 < worst < 1e-4, 3: worst < 2.0 ** -30, 4: worst > 1e-3, 5: 1e-7 < worst < 1e-4}[variant], worst
    ref = (O.coarse_pencil_solve if variant == 1 else O.coarse_pinv_solve)(X, Y, sig, rhs)
    out = np.zeros_like(rhs)
    assert L.slamg_op_coarse_solve(variant, m + n, 4, hp(np.ascontiguousarray(X)), hp(np.ascontiguousarray(Y)),
                                   hp(sig), hp(np.ascontiguousarray(rhs)), hp(out)) == 0
    assert np.allclose(out, ref, rtol=1e-8, atol=1e-9 * np.abs(ref).max())
