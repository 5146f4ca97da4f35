"""Serving-stream measurement: a seeded Poisson stream of solve requests through the serving loop.

    python -m paper_1102_0919_amd.serve_bench [--requests 200] [--slots 8] [--n-max 2e5] ...

Requests come from ``workloads.serving_requests`` (three matrix families, n log-uniform, n_b in
{1, 4, 8, 16}, dominant or minimal, tolerance 1e-8).  A closed-loop run of ``--calib`` requests
submitted at once measures the capacity (requests/s with every slot busy); the stream then
arrives at ``--load`` x that capacity.  Each request's latency runs from its submission (at its
arrival time) to its result, measured inside the library.  A few requests are solved again alone
on another context and compared bit for bit with their result from the stream.  Prints one JSON
line.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def _build(api, W, req, max_add):
    """The request's matrix (scipy CSR), kind and parameters, built before the clock starts."""
    A, kind = W.serving_matrix(req)
    # verbose: each solve reports its progress every 50 additive iterations on stderr
    prm = dict(W.FAMILY_PARAMS[(req["family"], req["target"])], max_add=max_add, verbose=50)
    # the block holds at most 16 pairs: guard pairs fill what n_b leaves
    prm["n_guard"] = max(0, min(prm.get("n_guard", 0), 16 - req["n_b"]))
    return A.to_scipy(), kind, api.params_init(kind, req["target"], **prm)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--n-max", type=float, default=2e5)
    ap.add_argument("--calib", type=int, default=32)
    ap.add_argument("--load", type=float, default=0.7)
    ap.add_argument("--max-add", type=int, default=200)
    ap.add_argument("--check", type=int, default=5)
    ap.add_argument("--seed", type=int, default=1102)
    a = ap.parse_args(argv)

    import torch
    from paper_1102_0919_amd import api, workloads as W
    if not torch.cuda.is_available():
        print("serve_bench: needs a HIP device", file=sys.stderr)
        return 2
    budget = int(a.budget_gb * (1 << 30))
    reqs = W.serving_requests(a.requests, seed=a.seed, n_hi=a.n_max, rate=1.0)
    calib = W.serving_requests(a.calib, seed=a.seed + 7919, n_hi=a.n_max, rate=1.0)

    built = [_build(api, W, r, a.max_add) for r in reqs]
    cbuilt = [_build(api, W, r, a.max_add) for r in calib]
    print(f"[serve] built {len(built)} + {len(cbuilt)} request matrices", file=sys.stderr, flush=True)

    with api.Context(0, hbm_budget_bytes=budget) as ctx:
        api.serve_start(ctx, a.slots)
        # closed loop: every request at once
        t0 = time.perf_counter()
        ids = [(api.submit(ctx, S, kind, r["target"], r["n_b"], p), r, S, kind) for r, (S, kind, p) in
               zip(calib, cbuilt)]
        for k, (rid, r, S, kind) in enumerate(ids):
            api.wait(ctx, rid)
            api.fetch(ctx, rid, S.shape[0], S.shape[1], r["n_b"], kind, raise_errors=False)
            print(f"[serve] calibration {k + 1}/{len(ids)} done at {time.perf_counter() - t0:.1f} s "
                  f"({r['family']}, n={r['n']:.0f}, n_b={r['n_b']}, {r['target']})", file=sys.stderr, flush=True)
        cap = len(calib) / (time.perf_counter() - t0)
        rate = a.load * cap
        print(f"[serve] capacity {cap:.3f} req/s with {a.slots} slots; stream at {rate:.3f} req/s", file=sys.stderr,
              flush=True)

        # open loop: Poisson arrivals at `rate`
        t0 = time.perf_counter()
        live = []
        for k, r in enumerate(reqs):
            due = t0 + r["arrival"] / rate
            now = time.perf_counter()
            if due > now:
                time.sleep(due - now)
            S, kind, p = built[k]
            rid = api.submit(ctx, S, kind, r["target"], r["n_b"], p)
            live.append((rid, r, S.shape, kind, p))
            if (k + 1) % 20 == 0:
                print(f"[serve] submitted {k + 1}/{len(reqs)}", file=sys.stderr, flush=True)
        out = [None] * len(live)
        left = set(range(len(live)))
        while left:
            for k in sorted(left):
                rid, r, shape, kind, p = live[k]
                if not api.poll(ctx, rid):
                    continue
                res = api.fetch(ctx, rid, shape[0], shape[1], r["n_b"], kind, raise_errors=False)
                out[k] = (r, res, kind, p)
                left.discard(k)
                run = res.report.t_latency_ms - res.report.t_queue_ms
                print(f"[serve] done {len(live) - len(left)}/{len(live)} at {time.perf_counter() - t0:.1f} s: "
                      f"{r['family']} n={r['n']:.0f} n_b={r['n_b']} {r['target']} status={res.status} "
                      f"iters={res.report.add_iters} queue={res.report.t_queue_ms:.0f} ms run={run:.0f} ms",
                      file=sys.stderr, flush=True)
            if left:
                time.sleep(0.05)
        elapsed = time.perf_counter() - t0
        api.serve_stop(ctx)

    lat = np.array([res.report.t_latency_ms for _, res, _, _ in out])
    conv = np.array([res.status == 0 for _, res, _, _ in out])
    names = {0: "ok", 1: "not_converged"}
    counts: dict = {}
    for r, res, _, _ in out:
        key = f"{r['family']}/{r['target']}/{names.get(res.status, api.status_string(res.status))}"
        counts[key] = counts.get(key, 0) + 1
    triplets = sum(r["n_b"] for (r, res, _, _) in out if res.status == 0)

    # alone versus in the mix, bit for bit
    same, checked = 0, 0
    picks = [i for i, (_, res, _, _) in enumerate(out) if res.status in (0, 1)][: a.check]
    with api.Context(0) as solo:
        for i in picks:
            r, res, kind, p = out[i]
            alone = api.solve(solo, built[i][0], kind, r["target"], r["n_b"], p, allow_not_converged=True)
            checked += 1
            same += int(np.array_equal(alone.sigma, res.sigma) and np.array_equal(alone.U, res.U))

    line = {
        "metric": "serving stream: requests/s, p50/p99 latency", "requests": len(out), "slots": a.slots,
        "hbm_budget_gb": a.budget_gb, "n_range": [1e3, a.n_max], "max_add": a.max_add, "tol": 1e-8,
        "capacity_req_per_s": round(cap, 4), "arrival_rate_req_per_s": round(rate, 4),
        "throughput_req_per_s": round(len(out) / elapsed, 4),
        "converged_triplets_per_s": round(triplets / elapsed, 4),
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 2), "p99": round(float(np.percentile(lat, 99)), 2),
                       "p50_converged": round(float(np.percentile(lat[conv], 50)), 2) if conv.any() else None,
                       "p99_converged": round(float(np.percentile(lat[conv], 99)), 2) if conv.any() else None},
        "outcomes": dict(sorted(counts.items())),
        "alone_vs_mix_bitwise_equal": f"{same}/{checked}",
    }
    print(json.dumps(line))
    return 0


if __name__ == "__main__":
    sys.exit(main())
