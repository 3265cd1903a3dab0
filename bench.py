#!/usr/bin/env python
"""Benchmark: converged eigenpairs per second of the MI355X ARRABIT solver.

Workload (one step = one whole solve, A resident in HBM before timing):
3D 7-point Dirichlet Laplacian on a 100^3 grid plus a diagonal potential drawn
U[0, 1) (seed 1): n = 1e6, nnz = 6.94e6; the k = 200 smallest eigenpairs with a
block of 240 columns, tolerance 1e-10 on the residual of eq. resi
(||Ax - lambda x|| / max(1, |lambda|)). The starting block is drawn on the
device from the counter-based generator (seed 2) at the start of every solve.

Prints ONE JSON line. `roofline` is the HBM roofline of the dominant kernel
(the fused filter SpMM), measured with HIP events on the solver's stream over
the timed solves; `cpu_baseline` is the plain FP64 CPU oracle timed on a
bounded sample (see cpu_baseline()).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = ("3D 7-point Laplacian 100^3 + U[0,1) diagonal potential (seed 1), n=1e6, nnz=6.94e6, "
            "k=200 smallest, block 240, tol 1e-10")


def cpu_baseline(A, k, w, spmm_cols_per_solve, a, b):
    """Time the CPU oracle's Algorithm 7 (poly, degree 3, on the shifted
    operator as Algorithm 8 calls it) on the full workload with a 240-column
    block, and scale by the number of block-degree columns the GPU solve
    needed. This counts only the filter work the paper reports as dominant, so
    the oracle's true solve time is longer and the derived rate is an upper
    bound of the oracle's throughput."""
    import numpy as np
    from oracle import arrabit as O
    from paper_1507_06078_amd import workloads as W

    B = -A.to_scipy()
    X = W.gaussian_block(A.n, w, seed=2)
    g = O.interpolant_coefficients(3)
    t = time.perf_counter()
    Y = O.poly(O.shifted(B, a), X, 0.0, b - a, g)
    dt = time.perf_counter() - t
    del Y
    per_col = dt / (3 * w)
    est = per_col * spmm_cols_per_solve
    return {"value": k / est, "unit": "eigenpairs/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle poly (Algorithm 7, 3 degrees, scipy CSR x {w}-column FP64 block, single thread) "
                       f"on the full n=1e6 workload took {dt:.2f} s; scaled to the GPU solve's "
                       f"{spmm_cols_per_solve} block-degree columns -> {est:.0f} s per solve "
                       "(filter work only: a lower bound of the oracle's solve time)"),
            "seconds_measured": dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--mixed-switch", type=float, default=None)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only; --gpus {args.gpus} is not supported "
              "(the row-sharded multi-GPU design is documented but not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1507_06078_amd import arr, workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    A = W.laplacian_3d(100, potential_seed=1)
    k, w, tol = 200, 240, 1e-10
    o = arr.arr_options_default()
    o.w = w
    o.precision = arr.MIXED if args.precision == "mixed" else arr.FP64
    o.timing = 1
    if args.mixed_switch is not None:
        o.mixed_switch = args.mixed_switch
    o.verbose = 1 if args.verbose else 0
    h = arr.arr_create(A, A.n, k, arr.SMALLEST, tol, o)
    print(f"[bench] handle ready (n={A.n}, nnz={A.nnz}); warmup {args.warmup}, steps {args.steps}",
          file=sys.stderr, flush=True)
    for i in range(args.warmup):
        st = arr.arr_solve(h)
        print(f"[bench] warmup {i}: status {st}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for i in range(args.steps):
        st = arr.arr_solve(h)
        stats.append(arr.arr_get_stats(h))
        print(f"[bench] step {i}: status {st} t {stats[-1]['t_total']:.3f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ev, _, res = arr.arr_get_eigpairs(h, k, A.n, vectors=False)
    sec = (t1 - t0) / args.steps
    ok = all(s["status"] == 0 for s in stats) and float(res.max()) <= tol
    spmm_ms = sum(s["spmm_ms"] for s in stats)
    spmm_bytes = sum(s["spmm_bytes"] for s in stats)
    launches = sum(s["spmm_launches"] for s in stats)
    achieved = spmm_bytes / (spmm_ms * 1e-3) / 1e9 if spmm_ms > 0 else None
    last = stats[-1]
    out = {
        "metric": "converged eigenpairs/s at res<=1e-10",
        "value": (k / sec) if ok else 0.0,
        "unit": "eigenpairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "precision": args.precision},
        "converged": ok,
        "max_res": float(res.max()),
        "roofline": {
            "bound": "hbm",
            "kernel": f"k_filter_spmm<{'double' if args.precision == 'fp64' else 'float'},"
                      f"{last['spmm_cols_per_lane']}>",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
            "traffic": None,
            "launches": launches,
            "avg_launch_us": spmm_ms * 1e3 / max(1, launches),
            "algorithmic_bytes_per_launch": spmm_bytes / max(1, launches),
        },
        "solve": {key: last[key] for key in ("outer_iters", "arr_calls", "poly_calls", "final_p", "final_d",
                                             "n_locked", "fp32_outer", "spmm_degrees", "spmm_cols", "t_total",
                                             "t_setup", "t_filter", "t_arr", "t_dense")},
    }
    h.close()
    if not args.no_cpu_baseline:
        # interval of the working operator (-A) as the solver estimated it
        a_w, b_w = -last["a"], -last["b"]
        out["cpu_baseline"] = cpu_baseline(A, k, w, int(last["spmm_cols"]), a_w, b_w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
