"""Serving loop (slamg_serve_start): requests solved concurrently on several streams give the same
results as each request solved alone, admission respects the HBM budget, and a request that can
never fit is refused at submission."""
import numpy as np
import pytest

from paper_1102_0919_amd import workloads as W

from .gpu_util import lib

pytestmark = pytest.mark.gpu


def _mix():
    reqs = []
    for name, scale, over in [("laplace2d_31_min4", None, {}), ("gradient2d_256_dom8", 32, {}),
                              ("laplace2d_32_dom8", 20, {}), ("gradient2d_256_dom8", 24, {"n_mult": 6}),
                              ("laplace2d_31_min4", 25, {"precision": "mixed_fp32"}),
                              ("laplace2d_31_min4", 28, {"coarse_pinv": 1})]:
        wl = W.WORKLOADS[name]
        A = W.build_workload_matrix(name, scale).to_scipy()
        prm = dict(wl["params"]); prm.update(over)
        reqs.append((A, wl["kind"], wl["target"], wl["n_b"], prm))
    return reqs


def test_serving_results_equal_alone(tmp_path):
    import torch
    assert torch.cuda.is_available()
    lib()
    from paper_1102_0919_amd import api
    reqs = _mix()
    with api.Context(0) as ctx:
        alone = [api.solve(ctx, A, k, t, nb, api.params_init(k, t, **prm)) for A, k, t, nb, prm in reqs]
    with api.Context(0) as ctx:
        api.serve_start(ctx, 3)
        ids = [api.submit(ctx, A, k, t, nb, api.params_init(k, t, **prm)) for A, k, t, nb, prm in reqs]
        for rid in ids:
            api.wait(ctx, rid)
        mix = [api.fetch(ctx, rid, A.shape[0], A.shape[1], nb, k)
               for rid, (A, k, t, nb, prm) in zip(ids, reqs)]
        api.serve_stop(ctx)
    for a, b in zip(alone, mix):
        assert a.status == b.status
        assert b.report.add_iters == a.report.add_iters
        assert np.array_equal(a.sigma, b.sigma)
        assert np.array_equal(a.U, b.U)
        if a.V is not None:
            assert np.array_equal(a.V, b.V)
        assert 0.0 <= b.report.t_queue_ms <= b.report.t_latency_ms
        assert b.report.device_bytes > 0


def test_serving_budget_admission():
    import torch
    assert torch.cuda.is_available()
    lib()
    from paper_1102_0919_amd import api
    A = W.laplace2d(31).to_scipy()
    wl = W.WORKLOADS["laplace2d_31_min4"]
    p = api.params_init("spd", "minimal", **wl["params"])
    # the estimate of this request is about 230 MB: a 300 MB budget admits one at a time
    with api.Context(0, hbm_budget_bytes=300 << 20) as ctx:
        api.serve_start(ctx, 4)
        ids = [api.submit(ctx, A, "spd", "minimal", 4, p) for _ in range(3)]
        res = []
        for rid in ids:
            api.wait(ctx, rid)
            res.append(api.fetch(ctx, rid, 961, 961, 4, "spd"))
        api.serve_stop(ctx)
        for r in res:
            assert r.converged
            assert np.array_equal(r.sigma, res[0].sigma)
        # one at a time: each request starts after the previous one ended
        q = sorted(r.report.t_queue_ms for r in res)
        assert q[1] > 0.5 * (res[0].report.t_latency_ms - res[0].report.t_queue_ms)
        big = W.laplace2d(200).to_scipy()
        with pytest.raises(api.SlamgError, match="E_BUDGET"):
            api.submit(ctx, big, "spd", "minimal", 16, api.params_init("spd", "minimal"))
