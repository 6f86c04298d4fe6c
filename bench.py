#!/usr/bin/env python3
"""Benchmark of the profile-likelihood hot path on one MI355X.

A step is one pl_profile_loglik call over the whole anisotropic workload
(n = 2000 locations, p = 4 covariates, K = 1024 omega points x M = 8 Box-Cox
values = 8192 profile log-likelihoods; Matern build, bordered Cholesky,
solves, cross products and the p x p stage), with the inputs already resident
in HBM.  Prints one JSON line (rank 0, one GPU).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("profile-loglik points/sec at n=2000 (FP64 vs mixed, |Δℓ|≤1e-2); "
          "p99 latency")
PEAK_FP64_TFLOPS = 78.6    # MI355X dense FP64 matrix peak
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(pr, n_omega, gpu_ll):
    """The oracle as it stands, on a bounded sample of the same workload."""
    import numpy as np

    import oracle
    try:
        from threadpoolctl import threadpool_info
        blas = [i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"]
        cores = int(max(blas)) if blas else 1
    except Exception:
        cores = 1
    idx = np.arange(n_omega)
    t0 = time.perf_counter()
    ref = oracle.profile_loglik(pr.locs, pr.y, pr.X, pr.omega[idx], pr.lam)
    dt = time.perf_counter() - t0
    pts = n_omega * pr.M
    err = float(np.max(np.abs(gpu_ll[idx] - ref["loglik"]) /
                       np.maximum(np.abs(ref["loglik"]), pr.n)))
    return {"value": pts / dt, "unit": "points/s", "cores": cores, "kind": "oracle",
            "sample": (f"first {n_omega} of the {pr.K} omega points x {pr.M} lambdas at n={pr.n} "
                       f"({pts} points, {dt:.1f} s; SciPy Bessel on one thread, LAPACK with "
                       f"{cores} BLAS threads)")}, err


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-sample", type=int, default=8, help="omega points timed on the oracle")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n", type=int, default=2000)
    ap.add_argument("--K", type=int, default=1024)
    ap.add_argument("--M", type=int, default=8)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(omega points shard across GPUs by design only)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_2305_04318_amd as pl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    pl.load()
    pr = synth.config_aniso(n=args.n, K=args.K, M=args.M)
    n, p, K, M = pr.n, pr.p, pr.K, pr.M
    log(f"workload {pr.name}, p={p}")
    inp = pl.Inputs(pr.locs, pr.y, pr.X, device="cuda")
    out = torch.empty((K, M, 10), dtype=torch.float64, device="cuda")
    work = torch.empty(pl.workspace_size(n, p, K, M), dtype=torch.uint8, device="cuda")
    log(f"workspace {work.numel() / 2**30:.2f} GiB")

    def step():
        pl.profile_loglik(None, None, None, pr.omega, pr.lam, inputs=inp, out=out, work=work)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")

    pl.profiling_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = pl.profiling_read()
    pl.profiling_enable(False)
    ms = (t1 - t0) / args.steps * 1e3
    value = K * M / (ms / 1e3)
    log(f"timed {args.steps} steps: {ms:.2f} ms/step, {value:.0f} points/s")

    g = prof["gemm"]
    gemm_tflops = g["flops"] / (g["ms"] / 1e3) / 1e12 if g["ms"] > 0 else 0.0
    chol_flops = K * n ** 3 / 3.0
    per_class = {c: round(v["ms"] / args.steps, 3) for c, v in prof.items()}
    info = pl.unpack_records(out)["info"].cpu().numpy()
    gpu_ll = pl.unpack_records(out)["loglik"].cpu().numpy()

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"anisotropic Matern, n={n}, p={p}, K={K} omega x M={M} lambda, FP64",
                   "n": n, "p": p, "K": K, "M": M, "precision": "fp64"},
        "roofline": {"bound": "mfma", "achieved": gemm_tflops, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": gemm_tflops / PEAK_FP64_TFLOPS, "traffic": None,
                     "kernel": "k_gemm_col (left-looking block-column update, MFMA f64)",
                     "launches_per_step": g["launches"] // args.steps},
        "omega_per_s": K / (ms / 1e3),
        "chol_path_tflops": chol_flops / (ms / 1e3) / 1e12,
        "kernel_ms_per_step": per_class,
        "failed_points": int(np.sum(info != 0)),
    }
    if not args.no_cpu_baseline:
        log(f"timing the oracle on {args.cpu_sample} omega points")
        cb, err = cpu_baseline(pr, args.cpu_sample, gpu_ll)
        line["cpu_baseline"] = cb
        line["oracle_max_rel_err"] = err
        log(f"oracle {cb['value']:.1f} points/s, max rel err vs GPU {err:.2e}")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
