#!/usr/bin/env python
"""Benchmark of the self-learning AMG solver on one MI355X.

One step = one complete solve (multiplicative set-up phase + additive phase with Ritz steps down
to relative residual 1e-8) of the named workload, with the matrix resident in device memory when
the timed region starts.  Prints ONE JSON line:

  value      triplets/s = n_b / (seconds per solve)
  roofline   the dominant kernel class, timed live with HIP events on the library's stream over the
             timed steps: algorithmic bytes per launch / average launch duration, against 8 TB/s
  cpu_baseline  the FP64 oracle on the host cores, on a bounded sample of the same workload
             (the multiplicative phase plus a few additive iterations, scaled to the iteration
             count of the GPU solve)
  compare    the same workload timed in a second precision (default: the mixed FP32 V-cycle with
             the FP64 refinement around it), with its accuracy
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CLASS_NAMES = {0: "k_rowop, finest-level relaxation sweeps",
               1: "k_kacz, finest-level Kaczmarz colour sweeps", 2: "k_gram (MFMA FP64 Gram)",
               3: "k_spgemm_dot (Galerkin SpGEMM)", 4: "coarsest dense solves (k_pinv_solve / k_pencil_solve)",
               5: "k_spmm, finest-level block SpMM", 6: "k_dots, finest-level operator reductions",
               7: "k_rowop, finest-level residuals"}
NCLS = 8
ALL_CLASSES = (1 << NCLS) - 1
DEFAULT_WORKLOAD = "aniso3d_128_min8"
# roofline kernel classes whose achieved bandwidth the line reports next to the dominant one
REPORTED = {1: "relaxation (finest-level Kaczmarz sweeps)", 0: "relaxation (finest-level row kernel)",
            5: "block SpMM (finest level)", 3: "Galerkin SpGEMM (all levels)"}

# HBM traffic of the dominant kernel class, from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs
# (profiles/pmc_*_<workload>.md), per dispatch in KiB, scaled by the same counters of a 1 GiB device
# copy (profiles/pmc_*_copy_1GiB.md: FETCH 524304.5 KiB, WRITE 1048576.0 KiB per 1 GiB).  Valid
# only for the kernel source the counters were taken with.
TRAFFIC = {
    # the two finest-level k_rowop launch shapes (u rows, v rows)
    ("gradient2d_256_dom8", 0): dict(
        kernels_sha256="56df206b3531e9b5594c229e089abdefcc35af292738dcdd46269dfbf4342271",
        fetch_kib=(12230.1, 10374.9), write_kib=(8160.0, 4096.0),
        copy_fetch_kib=524304.5, copy_write_kib=1048576.0, copy_bytes=1 << 30,
        note="mean of the finest-level u-row and v-row launches"),
    # every finest-level k_kacz launch of the multiplicative phase and one additive iteration
    ("aniso3d_128_min8", 1): dict(
        kernels_sha256="f910d07505489c0af19a2c36b9cd904ffbc5434d5678dffd5a5bfb7076029ec4",
        fetch_kib=(117662.2,), write_kib=(154376.8,),
        copy_fetch_kib=524304.5, copy_write_kib=1048576.0, copy_bytes=1 << 30,
        note="mean over the 1240 finest-level Kaczmarz colour launches of the multiplicative phase and "
             "one additive iteration"),
}


def _traffic(name, cls):
    import hashlib
    t = TRAFFIC.get((name, cls))
    if t is None:
        return None, "no counter run for this workload and kernel"
    with open(os.path.join(ROOT, "paper_1102_0919_amd", "csrc", "kernels.hip"), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != t["kernels_sha256"]:
            return None, "kernel source changed since the counter runs"
    ff = t["copy_bytes"] / (t["copy_fetch_kib"] * 1024.0)
    fw = t["copy_bytes"] / (t["copy_write_kib"] * 1024.0)
    per = [(fk * ff + wk * fw) * 1024.0 for fk, wk in zip(t["fetch_kib"], t["write_kib"])]
    return sum(per) / len(per), (f"rocprofv3 FETCH_SIZE x {ff:.4f} + WRITE_SIZE x {fw:.4f} (copy-calibrated), "
                                 + t["note"])


def _closed_form(name, n_b, target):
    from paper_1102_0919_amd import workloads as W
    if name.startswith("gradient2d_256"):
        s = W.gradient2d_singular_values(256)
        return s[::-1][:n_b] if target == "dominant" else s[:n_b]
    if name.startswith("laplace2d_31"):
        e = W.laplace2d_eigs(31)
        return e[:n_b] if target == "minimal" else e[::-1][:n_b]
    if name.startswith("aniso3d_128"):
        return W.aniso3d_eigs_smallest(128, 0.01, n_b)
    return None


def cpu_baseline(name, A, wl, gpu_add_iters, budget_s=30.0):
    """Oracle timing on a bounded sample.  The oracle's multiplicative phase plus up to 5 additive
    iterations are timed; the additive time is extrapolated to the GPU solve's iteration count.  For
    the 3-D anisotropic workload the oracle runs on the 24^3 grid of the same family (its
    multiplicative phase on 128^3 alone would take hours in pure-Python coarsening and colouring)
    and both parts are scaled by the unknown count (the cost of a cycle grows linearly with the
    number of unknowns, §6.1); for the term-document workload on the same generator at 4000 x 1000,
    scaled by the nonzero count."""
    import numpy as np
    from oracle import slamg_oracle as O
    from paper_1102_0919_amd import workloads as W
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = 1
    p = O.Params(**wl["params"])
    scale, what = 1.0, "the same matrix"
    if name.startswith("aniso3d_128"):
        k = 24
        As = W.aniso3d(k, 0.01).to_scipy()
        scale = A.shape[0] / As.shape[0]
        what = f"the {k}^3 grid of the same family ({As.shape[0]} unknowns), scaled by {scale:.1f} (unknown count)"
        A = As
    elif name == "termdoc_200k_dom10":
        # the same generator at 4000 x 1000 (the oracle's pure-Python coarsening of the full matrix
        # takes tens of minutes), scaled by the nonzero count
        As = W.termdoc(4000, 1000, 60, seed=1102).to_scipy().tocsr()
        As = As[As.getnnz(axis=1) > 0][:, As.getnnz(axis=0) > 0]
        scale = A.nnz / As.nnz
        what = (f"the same Zipf generator at {As.shape[0]} x {As.shape[1]} (empty rows removed, {As.nnz} "
                f"nonzeros), scaled by {scale:.1f} (nonzero count)")
        A = As
    print(f"[bench] cpu baseline: oracle on {what}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    s = O.Solver(A, wl["kind"], wl["target"], wl["n_b"], p)
    for c in range(1, p.n_mult + 1):
        s.mult_cycle(c)
    t_setup = time.perf_counter() - t0
    k = 0
    t1 = time.perf_counter()
    while k < 5 and time.perf_counter() - t0 < budget_s:
        s.additive_vcycle()
        s.sig, s.Ub, s.Vb = s._ritz(s.Ub, s.Vb)
        O.residuals(s.levels[0].A, s.kind, s.Ub, s.Vb, s.sig, s.anorm)
        k += 1
    t_iter = (time.perf_counter() - t1) / max(k, 1)
    t_total = (t_setup + t_iter * gpu_add_iters) * scale
    return {"value": wl["n_b"] / t_total, "unit": "triplets/s", "cores": int(threads), "kind": "oracle",
            "sample": f"oracle multiplicative phase ({p.n_mult} cycles, {t_setup:.1f} s) + {k} additive "
                      f"iterations ({t_iter:.3f} s each) on {what}, extrapolated to the GPU's "
                      f"{gpu_add_iters} additive iterations; scipy sparse kernels are single-threaded"}


def _run_steps(api, ctx, mat, target, n_b, p, U_dev, V_dev, steps, label):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    for k in range(steps):
        r = api.solve_matrix(ctx, mat, target, n_b, p, U_dev=U_dev, V_dev=V_dev)
        reps.append(r)
        print(f"[bench] {label} step {k}: add_iters={r.report.add_iters} converged={r.converged}", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    return reps, (time.perf_counter() - t0) * 1e3 / steps


def _class_totals(reps):
    import numpy as np
    tot_ms = np.zeros(NCLS); tot_n = np.zeros(NCLS); tot_b = np.zeros(NCLS)
    for r in reps:
        for c in range(NCLS):
            tot_ms[c] += r.report.prof_ms[c]; tot_n[c] += r.report.prof_launches[c]
            tot_b[c] += r.report.prof_bytes[c]
    return tot_ms, tot_n, tot_b


def _accuracy(last, ref, n_b):
    import numpy as np
    acc = {"max_rel_residual": float(max(last.report.resid[j] for j in range(n_b))),
           "levels": int(last.report.levels), "add_iters": int(last.report.add_iters),
           "mult_cycles": int(last.report.mult_cycles), "converged": bool(last.converged)}
    if ref is not None:
        err = np.abs(last.sigma - ref) / np.maximum(np.abs(ref), 1e-8 * last.report.anorm)
        acc["max_rel_sigma_err_vs_closed_form"] = float(err.max())
    return acc


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed_fp32", "mixed_bf16"])
    ap.add_argument("--compare", default="mixed_fp32", choices=["none", "fp64", "mixed_fp32", "mixed_bf16"],
                    help="second precision timed on the same workload and reported next to the headline")
    ap.add_argument("--solve-phase", type=int, default=0, choices=[0, 1],
                    help="0 the multigrid-Ritz additive phase (the method's own), 1 LOBPCG on the learned hierarchy")
    ap.add_argument("--no-alt-phase", action="store_true",
                    help="skip timing the other solve phase (FP64) next to the headline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--max-add", type=int, default=6000,
                    help="additive iteration cap (the solve stops earlier once every residual is below 1e-8)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this benchmark runs on one GPU only (asked for --gpus {args.gpus}); the single-GPU "
              "figure is the whole measurement", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1102_0919_amd import api, workloads as W

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    name = args.workload
    wl = W.WORKLOADS[name]
    A = W.build_workload_matrix(name).to_scipy()
    kind, target, n_b = wl["kind"], wl["target"], wl["n_b"]
    stream = torch.cuda.current_stream()

    def params(precision, mask, graphs=1, phase=None):
        prm = dict(wl["params"])
        prm["precision"] = precision
        prm["solve_phase"] = args.solve_phase if phase is None else phase
        prm["profile_mask"] = mask
        prm["max_add"] = args.max_add
        prm["graphs"] = graphs
        return api.params_init(kind, target, **prm)

    ctx = api.Context(0, stream=stream.cuda_stream)
    mat = api.Matrix(ctx, A, kind)          # validated, prepared and resident in device memory
    # the singular vectors are written to device arrays (column-major m x n_b, n x n_b)
    U_dev = torch.empty((n_b, A.shape[0]), dtype=torch.float64, device="cuda")
    V_dev = torch.empty((n_b, A.shape[1]), dtype=torch.float64, device="cuda") if kind == "svd" else None
    print(f"[bench] workload {name}: {A.shape[0]}x{A.shape[1]} nnz={A.nnz} n_b={n_b} {args.precision}",
          file=sys.stderr, flush=True)
    p = params(args.precision, 0 if args.no_profile else ALL_CLASSES)
    # the untimed warmup runs every additive iteration eagerly (no graph replay), so that its
    # class times cover every launch of the solve: they pick the dominant kernel class
    pw = params(args.precision, 0 if args.no_profile else ALL_CLASSES, graphs=0)
    warm_ms = np.zeros(NCLS)
    warm_n = np.zeros(NCLS)
    warm_b = np.zeros(NCLS)
    for _ in range(max(args.warmup, 1 if not args.no_profile else 0)):
        w = api.solve_matrix(ctx, mat, target, n_b, pw, U_dev=U_dev, V_dev=V_dev)
        warm_ms = np.array([w.report.prof_ms[c] for c in range(NCLS)])
        warm_n = np.array([w.report.prof_launches[c] for c in range(NCLS)], dtype=float)
        warm_b = np.array([w.report.prof_bytes[c] for c in range(NCLS)])
        print(f"[bench] warmup: add_iters={w.report.add_iters} converged={w.converged}", file=sys.stderr, flush=True)
    reps, ms = _run_steps(api, ctx, mat, target, n_b, p, U_dev, V_dev, args.steps, args.precision)
    value = n_b / (ms / 1e3)
    last = reps[-1]
    ref = _closed_form(name, n_b, target)
    # roofline: the profiled kernel class with the largest device time over the whole warmup solve;
    # its bytes and launch durations from the launches sampled in the timed steps
    tot_ms, tot_n, tot_b = _class_totals(reps)
    roof = None
    if tot_ms.sum() > 0:
        c = int(np.argmax(np.where(tot_b > 0, warm_ms if warm_ms.sum() > 0 else tot_ms, 0)))
        avg_ms = tot_ms[c] / tot_n[c]
        per_launch = tot_b[c] / tot_n[c]
        ach = per_launch / (avg_ms * 1e-3) / 1e9
        traffic, tnote = _traffic(name, c)
        kernels = {}
        for k2, label in REPORTED.items():
            if tot_n[k2] > 0 and tot_b[k2] > 0:
                kernels[label] = {"GB/s": round(tot_b[k2] / tot_n[k2] / (tot_ms[k2] / tot_n[k2] * 1e-3) / 1e9, 1),
                                  "frac": round(tot_b[k2] / (tot_ms[k2] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                  "launches": int(tot_n[k2]), "avg_launch_us": round(tot_ms[k2] / tot_n[k2] * 1e3, 2)}
        roof = {"bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else int(traffic), "traffic_note": tnote,
                "kernel": CLASS_NAMES[c],
                "timed_launches_per_step": int(tot_n[c] / args.steps), "avg_launch_us": round(avg_ms * 1e3, 3),
                "timing_sample": "a HIP event pair around every launch of the profiled kernel classes on the "
                                 "library stream in the eagerly launched additive iterations (every 32nd; the "
                                 "others replay a HIP graph of the iteration) and in the multiplicative phase",
                "algorithmic_bytes_per_launch": int(per_launch),
                "graph_iters_per_step": int(last.report.graph_iters),
                "kernels": kernels,
                "class_ms_in_warmup_solve": {CLASS_NAMES[i]: round(warm_ms[i], 3) for i in range(NCLS)}}
        if warm_n[c] > 0:
            # every launch of the class in one whole solve (the warmup runs every iteration
            # eagerly, each launch between HIP events): the sample rocprofv3's average covers
            wa = warm_ms[c] / warm_n[c]
            wb = warm_b[c] / warm_n[c]
            roof["whole_solve_sample"] = {
                "launches": int(warm_n[c]), "avg_launch_us": round(wa * 1e3, 3),
                "algorithmic_bytes_per_launch": int(wb), "GB/s": round(wb / (wa * 1e-3) / 1e9, 2),
                "frac": round(wb / (wa * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "note": "the untimed warmup solve, all additive iterations eager: graph replays in the timed "
                        "solves cannot be timed per launch (HIP does not time events recorded by graph nodes)"}
    compare = None
    if args.compare != "none" and args.compare != args.precision:
        p2 = params(args.compare, 0)
        w2 = api.solve_matrix(ctx, mat, target, n_b, p2, U_dev=U_dev, V_dev=V_dev)
        print(f"[bench] {args.compare} warmup: add_iters={w2.report.add_iters} converged={w2.converged}",
              file=sys.stderr, flush=True)
        reps2, ms2 = _run_steps(api, ctx, mat, target, n_b, p2, U_dev, V_dev, args.steps, args.compare)
        last2 = reps2[-1]
        compare = {"precision": args.compare, "value": round(n_b / (ms2 / 1e3), 4), "unit": "triplets/s",
                   "ms_per_step": round(ms2, 3), "speedup_vs_headline": round(ms / ms2, 4),
                   "setup_ms": round(last2.report.t_setup_ms, 3), "solve_ms": round(last2.report.t_solve_ms, 3),
                   "accuracy": _accuracy(last2, ref, n_b)}
        if ref is not None:
            compare["accuracy"]["max_rel_sigma_diff_vs_headline"] = float(
                np.max(np.abs(last2.sigma - last.sigma) / np.abs(ref)))
    alt = None
    if not args.no_alt_phase:
        ph = 1 - args.solve_phase
        p3 = params("fp64", 0, phase=ph)
        w3 = api.solve_matrix(ctx, mat, target, n_b, p3, U_dev=U_dev, V_dev=V_dev)
        print(f"[bench] solve phase {ph} warmup: add_iters={w3.report.add_iters} converged={w3.converged}",
              file=sys.stderr, flush=True)
        reps3, ms3 = _run_steps(api, ctx, mat, target, n_b, p3, U_dev, V_dev, args.steps, f"phase {ph}")
        last3 = reps3[-1]
        alt = {"solve_phase": ph, "name": ["multigrid-Ritz", "LOBPCG"][ph], "precision": "fp64",
               "value": round(n_b / (ms3 / 1e3), 4), "unit": "triplets/s", "ms_per_step": round(ms3, 3),
               "speedup_vs_headline": round(ms / ms3, 4), "setup_ms": round(last3.report.t_setup_ms, 3),
               "solve_ms": round(last3.report.t_solve_ms, 3), "accuracy": _accuracy(last3, ref, n_b)}
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(name, A, wl, int(last.report.add_iters))
    line = {"metric": "triplets/s at resid 1e-8", "value": round(value, 4), "unit": "triplets/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None,
            "dtype": {"fp64": "f64", "mixed_fp32": "f32+f64", "mixed_bf16": "bf16+f32+f64"}[args.precision],
            "data": "synthetic",
            "config": {"workload": name, "description": wl["desc"], "rows": int(A.shape[0]),
                       "cols": int(A.shape[1]), "nnz": int(A.nnz), "n_b": n_b, "kind": kind, "target": target,
                       "precision": args.precision, "tol": 1e-8,
                       "solve_phase": ["multigrid-Ritz", "LOBPCG"][args.solve_phase]},
            "roofline": roof, "cpu_baseline": cpu, "accuracy": _accuracy(last, ref, n_b),
            "setup_ms": round(last.report.t_setup_ms, 3), "solve_ms": round(last.report.t_solve_ms, 3),
            "compare": compare, "alt_phase": alt}
    mat.close()
    ctx.close()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
