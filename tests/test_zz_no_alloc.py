"""The no-allocation Gram entry point against slamg_op_gram, through the C ABI."""
import ctypes as C

import numpy as np
import pytest

from .gpu_util import dev, host, hp, lib, ptr, release

pytestmark = pytest.mark.gpu


def _gram(L, X, Y, w):
    rows = X.shape[0]
    g = np.zeros((w, w))
    st = L.slamg_op_gram(rows, w, ptr(dev(X)), ptr(dev(Y)), hp(g), None)
    assert st == 0
    return g


def _gram_noalloc(L, X, Y, w):
    import torch
    rows = X.shape[0]
    dg = torch.full((w, w), np.nan, dtype=torch.float64, device="cuda")
    st = L.slamg_op_gram_noalloc(rows, w, ptr(dev(X)), ptr(dev(Y)), ptr(dg), None)
    assert st == 0
    return host(dg)


def test_gram_noalloc_equals_gram_on_two_calls():
    import torch
    assert torch.cuda.is_available()
    L = lib()
    assert L.slamg_op_gram_noalloc_scratch_bytes() == 2048 * 256 * 8
    rng = np.random.default_rng(7)
    # a large call (the full 2048-workgroup reduction) and then a smaller one: the second reads only
    # the scratch slots it writes, whatever the first left there
    for rows, w in ((300000, 16), (3001, 5)):
        X = rng.uniform(-1, 1, (rows, w)); Y = rng.uniform(-1, 1, (rows, w))
        g_ref = _gram(L, X, Y, w)
        g = _gram_noalloc(L, X, Y, w)
        assert np.array_equal(g, g_ref)                       # same kernels, same summation order
        assert np.allclose(g, X.T @ Y, rtol=1e-12, atol=1e-9)
        gx = _gram_noalloc(L, X, X, w)
        assert np.array_equal(gx, _gram(L, X, X, w))
        release()
    # bad sizes are rejected before anything is launched
    assert L.slamg_op_gram_noalloc(10, 17, None, None, None, None) != 0
    assert L.slamg_op_gram_noalloc(-1, 4, C.c_void_p(1), C.c_void_p(1), C.c_void_p(1), None) != 0
