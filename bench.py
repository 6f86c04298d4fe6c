#!/usr/bin/env python3
"""Benchmark of the profile-likelihood hot path on one MI355X.

A step is one pl_profile_loglik call over the whole anisotropic workload
(n = 2000 locations, p = 4 covariates, K = 1024 omega points x M = 8 Box-Cox
values = 8192 profile log-likelihoods; Matern build, bordered Cholesky,
solves, cross products and the p x p stage) in FP64, with the inputs already
resident in HBM.  Prints one JSON line (one GPU).

Beside the headline the line carries the other forms of the path, each on
seeded synthetic inputs of the stated shape:
  mixed_n2000   the mixed-precision form on the same inputs, with its
                log-likelihood error against the FP64 records;
  n4000, n8000  FP64 and mixed at n = 4000 (K = 256) and n = 8000 (K = 256);
  uneven_batch  2048 datasets of n in [100, 1500] in one persistent launch;
  serving       Poisson arrivals of requests of n in [500, 8000], p50/p99
                latency and points/s for both forms.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("profile-loglik points/sec at n=2000 (FP64 vs mixed, |Δℓ|≤1e-2); "
          "p99 latency")
PEAK_FP64_TFLOPS = 78.6     # MI355X dense FP64 matrix peak
PEAK_FP32_TFLOPS = 157.3    # MI355X dense FP32 matrix peak
EXTRAS = ("mixed", "n4000", "n8000", "batch", "serve")
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "block_column_update_hbm_traffic_aniso_n2000_K1024.md")
GEMM_SOURCES = ("common.h", "tiles.h", "chol.hip")


COV_PROFILE = os.path.join(ROOT, "profiles", "covariance_build_aniso_n2000_K1024.md")
COV_SOURCES = ("common.h", "matern_dev.h", "matern.hip")


def profile_value(path, key, sources):
    """A figure from the machine-readable lines of a committed rocprofv3
    summary, or None when the kernel sources (sha256 over `sources`, in that
    order) changed since the counters were taken."""
    import hashlib
    try:
        text = open(path).read()
        want = {}
        for line in text.splitlines():
            k, _, v = line.strip().partition(": ")
            if k in (key, "sources_sha256"):
                want[k] = v.strip()
        h = hashlib.sha256()
        for f in sources:
            with open(os.path.join(ROOT, "paper_2305_04318_amd", "csrc", f), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest() != want.get("sources_sha256"):
            return None
        return float(want[key])
    except (OSError, KeyError, ValueError):
        return None


def measured_traffic():
    """HBM bytes per block-column update launch from the committed FETCH_SIZE/WRITE_SIZE
    summary, or None when the kernel sources changed since it was taken."""
    return profile_value(TRAFFIC_PROFILE, "traffic_bytes_per_launch", GEMM_SOURCES)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# --------------------------------------------------------------------------
# CPU baseline: the oracle, one omega point per task on a process pool with
# one BLAS thread per worker.  Runs before the process touches the GPU.
# --------------------------------------------------------------------------
_CPU_PR = None


def _oracle_point(k):
    from threadpoolctl import threadpool_limits

    import oracle
    pr = _CPU_PR
    with threadpool_limits(1):
        return k, oracle.profile_loglik(pr.locs, pr.y, pr.X, pr.omega[k:k + 1], pr.lam)["loglik"][0]


def host_cpu():
    """Host processor model and logical core count, as nproc and lscpu show them."""
    import subprocess
    model = ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    if not model:
        try:
            with open("/proc/cpuinfo") as f:
                for line in f:
                    if line.startswith("model name"):
                        model = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count() or 1
    return {"nproc": nproc, "model": model}


def cpu_single_core(pr, n_omega):
    """The oracle on one core (this process, one BLAS thread): points/s."""
    from threadpoolctl import threadpool_limits

    import oracle
    t0 = time.perf_counter()
    with threadpool_limits(1):
        for k in range(n_omega):
            oracle.profile_loglik(pr.locs, pr.y, pr.X, pr.omega[k:k + 1], pr.lam)
    dt = time.perf_counter() - t0
    return {"points_per_s": n_omega * pr.M / dt, "omega": n_omega, "seconds": dt}


def cpu_baseline(pr, n_omega, workers):
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    import numpy as np
    global _CPU_PR
    _CPU_PR = pr
    t0 = time.perf_counter()
    ll = np.empty((n_omega, pr.M))
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
        for k, row in ex.map(_oracle_point, range(n_omega)):
            ll[k] = row
    dt = time.perf_counter() - t0
    pts = n_omega * pr.M
    return {"value": pts / dt, "unit": "points/s", "cores": workers, "kind": "oracle",
            "sample": (f"first {n_omega} of the {pr.K} omega points x {pr.M} lambdas at n={pr.n} "
                       f"({pts} points in {dt:.1f} s; one omega per task on {workers} processes, "
                       f"one BLAS thread each; SciPy Bessel, LAPACK dpotrf)")}, ll


# --------------------------------------------------------------------------
# GPU legs
# --------------------------------------------------------------------------

def _pct(a, q):
    import numpy as np
    return float(np.percentile(a, q))


def time_steps(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(steps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    return ts


def run_form(pl, pr, precision, steps, warmup, chunk=0):
    """Time `steps` calls of one form over problem `pr`; returns stats, records."""
    import numpy as np
    import torch
    n, p, K, M = pr.n, pr.p, pr.K, pr.M
    inp = pl.Inputs(pr.locs, pr.y, pr.X, device="cuda")
    out = torch.empty((K, M, 10), dtype=torch.float64, device="cuda")
    beta = torch.empty((K, M, p), dtype=torch.float64, device="cuda")
    work = torch.empty(pl.workspace_size(n, p, K, M, precision, chunk), dtype=torch.uint8,
                       device="cuda")

    def step():
        pl.profile_loglik(None, None, None, pr.omega, pr.lam, inputs=inp, out=out, beta=beta,
                          return_beta=True, work=work, precision=precision, chunk=chunk)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    pl.profiling_enable(True)
    ts = time_steps(step, steps, 0)
    prof = pl.profiling_read()
    pl.profiling_enable(False)
    rec = {k: v.cpu().numpy() for k, v in pl.unpack_records(out).items()}
    rec["beta"] = beta.cpu().numpy()
    med = float(np.median(ts))
    st = {"precision": precision, "n": n, "K": K, "M": M,
          "ms_median": med, "ms_p10": _pct(ts, 10), "ms_p90": _pct(ts, 90),
          "points_per_s": K * M / (med / 1e3), "omega_per_s": K / (med / 1e3),
          "chol_path_tflops": K * n ** 3 / 3.0 / (med / 1e3) / 1e12,
          "workspace_gib": work.numel() / 2 ** 30,
          "kernel_ms_per_step": {c: round(v["ms"] / steps, 3) for c, v in prof.items()},
          "gemm_tflops": (prof["gemm"]["flops"] / (prof["gemm"]["ms"] / 1e3) / 1e12
                          if prof["gemm"]["ms"] > 0 else 0.0)}
    del inp, out, beta, work
    torch.cuda.empty_cache()
    return st, rec


def mixed_error(rec_mx, rec_64, n):
    """|dl| of mixed against FP64 records (FP64 matches the oracle to 1e-8)."""
    import numpy as np
    from paper_2305_04318_amd import PL_INFO_FALLBACK
    ok = (rec_64["info"] == 0)
    d = np.abs(rec_mx["loglik"][ok] - rec_64["loglik"][ok])
    db = np.abs(rec_mx["beta"][ok] - rec_64["beta"][ok])
    inf = rec_mx["info"][:, 0]
    fb = int(np.sum((inf > 0) & ((inf & PL_INFO_FALLBACK) != 0)))
    return {"max_abs_dl": float(d.max()), "p99_abs_dl": _pct(d, 99), "median_abs_dl": _pct(d, 50),
            "frac_over_1e-2": float(np.mean(d > 1e-2)), "max_abs_dbeta": float(db.max()),
            "fallback_points": fb}


GOLDEN = os.path.join(ROOT, "tests", "golden", "large_samples.json")


def oracle_sample_error(rec, pr, name):
    """Records of the sampled omega points against the oracle values stored in
    tests/golden/large_samples.json (written by the oracle alone): max |dl|,
    max |dl| / max(|l|, 1), and the sample size."""
    import numpy as np
    with open(GOLDEN) as f:
        g = json.load(f)[name]
    fp = g["fingerprint"]
    if (pr.n, pr.p, pr.K, pr.M) != (fp["n"], fp["p"], fp["K"], fp["M"]) or \
            abs(float(np.sum(pr.y)) - fp["sum_y"]) > 1e-12 * max(1.0, abs(fp["sum_y"])):
        return None
    idx = np.asarray(g["omega_index"])
    ref = np.asarray(g["records"]["loglik"])
    got = rec["loglik"][idx]
    ok = np.asarray(g["records"]["info"]) == 0
    d = np.abs(got - ref)[ok]
    return {"oracle_points": int(ok.sum()), "oracle_max_abs_dl": float(d.max()),
            "oracle_max_rel_dl": float((d / np.maximum(np.abs(ref[ok]), 1.0)).max())}


def tune(pl, pr, tol=1e-3, sample=0):
    """pl_autotune's choice of form for this workload under an error budget,
    timed on `sample` omega points (0: all K of the workload)."""
    sample = sample or pr.K
    choice, report = pl.autotune(pr.locs, pr.y, pr.X, pr.omega, pr.lam, tol=tol, sample=sample)
    return {"choice": choice, "report": report, "sample": sample}


def _run_batch(pl, probs, runs, **kw):
    import numpy as np
    import torch
    b = pl.batch.Batch(probs, probs[0].lam, **kw)
    b.run()
    torch.cuda.synchronize()
    err = b.error()
    ts = []
    for _ in range(runs):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.run()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    rec = {k: v.cpu().numpy() for k, v in b.records().items()}
    med = float(np.median(ts))
    pts = b.units * probs[0].M
    flops = sum(p.K * p.n ** 3 / 3.0 for p in probs)
    st = {"ms_median": med, "ms_p10": _pct(ts, 10), "ms_p90": _pct(ts, 90),
          "points_per_s": pts / (med / 1e3), "omega_per_s": b.units / (med / 1e3),
          "chol_path_tflops": flops / (med / 1e3) / 1e12,
          "chol_path_frac_fp64_peak": flops / (med / 1e3) / 1e12 / PEAK_FP64_TFLOPS,
          "workspace_gib": b.work.numel() / 2 ** 30, "device_error": err,
          "failed_points": int(np.sum((rec["info"][:, 0] & ~pl.PL_INFO_FALLBACK) != 0)),
          "fallback_points": int(np.sum((rec["info"][:, 0] & pl.PL_INFO_FALLBACK) != 0))}
    if b.schedule == "persistent":
        st.update({"tasks": b.tasks, "slabs": b.slabs})
    else:
        st.update({"passes": b.passes, "streams": b.lanes})
    b.close()
    del b
    torch.cuda.empty_cache()
    return st, rec


def bench_uneven(pl, runs, forms=("tune", "persistent", "calls")):
    import numpy as np
    import torch

    import synth
    t0 = time.perf_counter()
    probs = synth.config_uneven()
    log(f"uneven: generated {len(probs)} datasets in {time.perf_counter() - t0:.1f} s")
    st = {"datasets": len(probs), "units": sum(p.K for p in probs),
          "points": sum(p.K for p in probs) * probs[0].M}
    # the size-bucketed schedule in both forms (one graph launch each), then
    # the persistent kernel (FP64)
    s64, r64 = _run_batch(pl, probs, runs)
    st["fp64"] = s64
    log(f"uneven bucketed fp64: {s64['ms_median']:.0f} ms")
    smx, rmx = _run_batch(pl, probs, runs, precision="mixed")
    ok = r64["info"] == 0
    d = np.abs(rmx["loglik"][ok] - r64["loglik"][ok])
    smx.update({"max_abs_dl_vs_fp64": float(d.max()), "p99_abs_dl_vs_fp64": _pct(d, 99)})
    st["mixed"] = smx
    log(f"uneven bucketed mixed: {smx['ms_median']:.0f} ms, max |dl| {d.max():.2e}")
    if "tune" in forms:
        # the autotuner's choice for this workload (budget 1e-3 against FP64),
        # measured like the others
        t0 = time.perf_counter()
        choice, report = pl.batch.autotune(probs, probs[0].lam, tol=1e-3)
        log(f"uneven autotune ({time.perf_counter() - t0:.0f} s): {choice}")
        stt, rtt = _run_batch(pl, probs, runs, **choice)
        stt["max_abs_dl_vs_fp64"] = float(np.max(np.abs(rtt["loglik"][ok] - r64["loglik"][ok])))
        st["tuned"] = {"choice": choice, "candidates": report, **stt}
        log(f"uneven tuned: {stt['ms_median']:.0f} ms")
    if "persistent" in forms:
        spe, rpe = _run_batch(pl, probs, runs, schedule="persistent")
        spe["max_rel_diff_vs_bucketed"] = float(np.max(
            np.abs(rpe["loglik"][ok] - r64["loglik"][ok]) / np.maximum(np.abs(r64["loglik"][ok]), 1)))
        st["persistent_fp64"] = spe
        log(f"uneven persistent fp64: {spe['ms_median']:.0f} ms")
    if "calls" not in forms:
        return st
    pts = st["points"]
    # the same datasets as independent calls on four streams (the serving
    # executor with every request present at the start), in both forms
    from paper_2305_04318_amd import serve as sv
    for prec in ("fp64", "mixed"):
        reqs = [sv.Request(i, 0.0, p.locs, p.y, p.X, p.omega, p.lam, prec)
                for i, p in enumerate(probs)]
        ex = sv.GpuExecutor(64 << 30, slots=4)
        sv.Server(ex).run(reqs[:8])  # untimed: first use of this form's kernels
        reqs = [sv.Request(i, 0.0, p.locs, p.y, p.X, p.omega, p.lam, prec)
                for i, p in enumerate(probs)]
        t0 = time.perf_counter()
        done = sv.Server(ex).run(reqs)
        dt = time.perf_counter() - t0
        ex.close()
        del ex
        torch.cuda.empty_cache()
        bad = int(sum(np.sum((r.result["info"] != 0) & (r.result["info"] != pl.PL_INFO_FALLBACK))
                      for r in done))
        st[f"per_dataset_calls_{prec}"] = {"ms": dt * 1e3, "points_per_s": pts / dt,
                                           "failed_points": bad}
        log(f"uneven as {len(done)} calls on 4 streams, {prec}: {dt * 1e3:.0f} ms")
    return st


def _gen_requests(arrivals):
    from concurrent.futures import ThreadPoolExecutor

    import synth

    def mk(a):
        t, n, K, seed = a
        return synth.serving_problem(n, K, seed, 4)

    with ThreadPoolExecutor(max_workers=16) as ex:
        probs = list(ex.map(mk, arrivals))
    return probs


def bench_serving(pl, seconds, rate, slots, budget_gib):
    import numpy as np
    import torch

    import synth
    from paper_2305_04318_amd import serve as sv
    arrivals = synth.serving_requests(duration_s=seconds, rate=rate)
    t0 = time.perf_counter()
    probs = _gen_requests(arrivals)
    log(f"serving: generated {len(probs)} requests in {time.perf_counter() - t0:.1f} s")
    offered = sum(pr.K * pr.n ** 3 / 3.0 for pr in probs) / seconds / 1e12
    out = {"rate_per_s": rate, "arrival_window_s": seconds, "requests": len(probs),
           "slots": slots, "hbm_budget_gib": budget_gib, "offered_chol_tflops": offered}
    for prec in ("fp64", "mixed"):
        reqs = [sv.Request(i, t, pr.locs, pr.y, pr.X, pr.omega, pr.lam, prec)
                for i, ((t, _, _, _), pr) in enumerate(zip(arrivals, probs))]
        ex = sv.GpuExecutor(budget_gib << 30, slots=slots, max_request_work=48 << 30)
        # untimed warm-up of the kernels for this form on a small request
        warm = sv.Request(-1, 0.0, probs[0].locs, probs[0].y, probs[0].X, probs[0].omega[:4],
                          probs[0].lam, prec)
        sv.Server(ex).run([warm])
        srv = sv.Server(ex)
        done = srv.run(reqs)
        ex.close()
        del ex
        torch.cuda.empty_cache()
        s = sv.latency_summary(done)
        s["achieved_chol_tflops"] = sum(r.K * r.n ** 3 / 3.0 for r in done) / s["span_s"] / 1e12
        s["max_inflight"] = srv.max_inflight
        s["peak_arena_gib"] = srv.peak_bytes / 2 ** 30
        s["failed_points"] = int(sum(np.sum((r.result["info"] != 0) &
                                            (r.result["info"] != pl.PL_INFO_FALLBACK))
                                     for r in done))
        # the largest sustainable arrival rate: the first `cap_n` requests all
        # present at time 0; the service rate at saturation bounds any stable rate
        cap_n = min(len(probs), 120)
        ex = sv.GpuExecutor(budget_gib << 30, slots=slots, max_request_work=48 << 30)
        sat = [sv.Request(i, 0.0, pr.locs, pr.y, pr.X, pr.omega, pr.lam, prec)
               for i, pr in enumerate(probs[:cap_n])]
        t0 = time.perf_counter()
        sv.Server(ex).run(sat)
        span = time.perf_counter() - t0
        ex.close()
        del ex
        torch.cuda.empty_cache()
        s["max_sustainable_rate_per_s"] = cap_n / span
        s["saturation_sample"] = (f"first {cap_n} requests of the stream, all present at t=0: "
                                  f"{span:.2f} s")
        s["stable"] = bool(rate < cap_n / span)
        out[prec] = s
        log(f"serving {prec}: p50 {s['p50_s'] * 1e3:.0f} ms p99 {s['p99_s'] * 1e3:.0f} ms "
            f"{s['points_per_s']:.0f} points/s over {s['span_s']:.1f} s; "
            f"max sustainable {cap_n / span:.1f} req/s")
    return out


def copy_calibration(mib):
    """Three device-to-device copies of `mib` MiB: each reads and writes
    exactly mib MiB, the scale for FETCH_SIZE / WRITE_SIZE readings."""
    import torch
    n = mib * 2 ** 20 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n * 8, "copies": 3}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="omega points timed on the oracle (default 6 per worker)")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="oracle processes (default min(16, cores): 16 cores is the host "
                         "share of one GPU on the measured boxes)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n", type=int, default=2000)
    ap.add_argument("--K", type=int, default=1024)
    ap.add_argument("--M", type=int, default=8)
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="fp64",
                    help="form of the headline steps (the metric is quoted on fp64)")
    ap.add_argument("--extras", default=",".join(EXTRAS),
                    help=f"comma list from {EXTRAS}, or 'none'")
    ap.add_argument("--batch-forms", default="tune,persistent,calls",
                    help="uneven batch extras beyond the bucketed FP64 and mixed runs: comma "
                         "list of tune, persistent, calls (per-dataset calls), or 'none'")
    ap.add_argument("--serve-seconds", type=float, default=30.0)
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device three times (the known-size "
                         "reference for HBM byte counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(omega points would shard across GPUs; only the single-GPU share is built)",
              file=sys.stderr)
        sys.exit(2)
    extras = [] if args.extras == "none" else [e for e in args.extras.split(",") if e]
    for e in extras:
        if e not in EXTRAS:
            sys.exit(f"unknown extra {e!r}")

    import numpy as np

    import synth
    pr = synth.config_aniso(n=args.n, K=args.K, M=args.M)
    n, p, K, M = pr.n, pr.p, pr.K, pr.M
    log(f"workload {pr.name}, p={p}")

    cb = None
    if not args.no_cpu_baseline:
        workers = args.cpu_workers or min(16, os.cpu_count() or 1)
        n_omega = args.cpu_sample or 6 * workers
        log(f"timing the oracle on {n_omega} omega points, {workers} processes")
        cb, cpu_ll = cpu_baseline(pr, n_omega, workers)
        cb["host"] = host_cpu()
        cb["single_core"] = cpu_single_core(pr, 2)
        log(f"oracle {cb['value']:.1f} points/s on {workers} processes, "
            f"{cb['single_core']['points_per_s']:.1f} on one core "
            f"(nproc {cb['host']['nproc']}, {cb['host']['model']})")

    import torch

    import paper_2305_04318_amd as pl
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    pl.load()

    # ---- headline: FP64, with per-kernel-class HIP-event timing -------------
    inp = pl.Inputs(pr.locs, pr.y, pr.X, device="cuda")
    out = torch.empty((K, M, 10), dtype=torch.float64, device="cuda")
    beta = torch.empty((K, M, p), dtype=torch.float64, device="cuda")
    prec = args.precision
    work = torch.empty(pl.workspace_size(n, p, K, M, prec), dtype=torch.uint8, device="cuda")
    log(f"workspace {work.numel() / 2**30:.2f} GiB")

    def step():
        pl.profile_loglik(None, None, None, pr.omega, pr.lam, inputs=inp, out=out, beta=beta,
                          return_beta=True, work=work, precision=prec)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    pl.profiling_enable(True)
    torch.cuda.synchronize()
    ts = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a = time.perf_counter()
        step()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - a) * 1e3)
    t1 = time.perf_counter()
    prof = pl.profiling_read()
    pl.profiling_enable(False)
    ms = (t1 - t0) / args.steps * 1e3
    value = K * M / (ms / 1e3)
    log(f"timed {args.steps} steps: {ms:.2f} ms/step, {value:.0f} points/s")

    g = prof["gemm"]
    gemm_ms = g["ms"] / max(1, g["launches"])
    gemm_flops = g["flops"] / max(1, g["launches"])
    gemm_tflops = g["flops"] / (g["ms"] / 1e3) / 1e12 if g["ms"] > 0 else 0.0
    if prec == "fp64":
        peak = PEAK_FP64_TFLOPS
        kernel_name = ("k_col_update (left-looking block-column update, bordered row folded "
                       "into the diagonal tile's workgroup, MFMA f64)")
        # counters were taken on this workload's launches only
        default_shape = (n, K, M) == (2000, 1024, 8)
        traffic = measured_traffic() if default_shape else None
    else:
        peak = PEAK_FP32_TFLOPS
        kernel_name = ("k_col_update_mx (block-column update: FP32 MFMA with FP64 flushes off "
                       "the diagonal, FP64 MFMA on the diagonal tile and the bordered row)")
        traffic = None
    rec64 = {k: v.cpu().numpy() for k, v in pl.unpack_records(out).items()}
    rec64["beta"] = beta.cpu().numpy()
    del inp, out, beta, work
    torch.cuda.empty_cache()

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
        "dtype": "f64" if prec == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": (f"anisotropic Matern, n={n}, p={p}, K={K} omega x M={M} lambda, "
                                f"{prec.upper() if prec == 'fp64' else 'mixed precision'}"),
                   "n": n, "p": p, "K": K, "M": M, "precision": prec},
        "roofline": {"bound": "mfma", "achieved": gemm_tflops, "peak": peak,
                     "unit": "TFLOP/s", "frac": gemm_tflops / peak, "traffic": traffic,
                     "kernel": kernel_name,
                     "launches_per_step": g["launches"] // args.steps,
                     "avg_launch_ms": gemm_ms, "alg_flops_per_launch": gemm_flops},
        "ms_p10": _pct(ts, 10), "ms_median": float(np.median(ts)), "ms_p90": _pct(ts, 90),
        "omega_per_s": K / (ms / 1e3),
        "chol_path_tflops": K * n ** 3 / 3.0 / (ms / 1e3) / 1e12,
        "kernel_ms_per_step": {c: round(v["ms"] / args.steps, 3) for c, v in prof.items()},
        "failed_points": int(np.sum(rec64["info"] != 0)),
    }
    # covariance build: the VALU-bound row; algorithmic bytes are the stored
    # lower triangle (8 B per element in FP64; the mixed form also stores 4 B)
    mt = prof["matern"]["ms"] / args.steps / 1e3
    if mt > 0:
        elems = K * n * (n + 1) / 2.0
        nbytes = elems * (8 if prec == "fp64" else 12)
        line["covariance_build"] = {
            "ms_per_step": mt * 1e3, "correlations_per_s": K * n * (n - 1) / 2.0 / mt,
            "alg_bytes_per_step": nbytes, "gb_per_s": nbytes / mt / 1e9,
            "hbm_frac": nbytes / mt / 8e12,
            "valu_busy": (profile_value(COV_PROFILE, "valu_busy_frac", COV_SOURCES)
                          if (prec == "fp64" and (n, K, M) == (2000, 1024, 8)) else None)}
    if cb is not None:
        k = cpu_ll.shape[0]
        ref = cpu_ll
        err = float(np.max(np.abs(rec64["loglik"][:k] - ref) / np.maximum(np.abs(ref), 1.0)))
        line["cpu_baseline"] = cb
        line["oracle_max_rel_err"] = err
        log(f"max rel err vs oracle {err:.2e}")
    if prec == "fp64" and (n, K, M) == (2000, 1024, 8):
        line["vs_oracle_sample"] = oracle_sample_error(rec64, pr, "aniso_n2000")

    def guarded(name, fn):
        try:
            line[name] = fn()
        except Exception as e:  # an extra must not lose the headline line
            log(f"{name} failed: {type(e).__name__}: {e}")
            line[name] = {"error": f"{type(e).__name__}: {e}"}
        torch.cuda.empty_cache()

    if "mixed" in extras and prec == "fp64":
        def mixed2000():
            st, rec = run_form(pl, pr, "mixed", args.steps, args.warmup)
            st.update(mixed_error(rec, rec64, n))
            st["vs_oracle"] = oracle_sample_error(rec, pr, "aniso_n2000")
            st["autotune_tol_1e-3"] = tune(pl, pr)
            log(f"mixed n={n}: {st['ms_median']:.1f} ms, max |dl| {st['max_abs_dl']:.2e}")
            return st
        guarded("mixed_n2000", mixed2000)

    for big, key in ((4000, "n4000"), (8000, "n8000")):
        if key not in extras:
            continue

        def both(big=big):
            q = synth.config_mixed() if big == 4000 else synth.config_aniso(n=8000, K=256, M=8)
            res = {}
            s64, r64 = run_form(pl, q, "fp64", max(2, args.steps // 2), 1)
            s64["vs_oracle"] = oracle_sample_error(r64, q, f"aniso_n{big}")
            res["fp64"] = s64
            smx, rmx = run_form(pl, q, "mixed", max(2, args.steps // 2), 1)
            # error statistics over every point against the FP64 records (which
            # match the oracle to 1e-8), and on the stored oracle sample itself
            smx.update(mixed_error(rmx, r64, q.n))
            smx["vs_oracle"] = oracle_sample_error(rmx, q, f"aniso_n{big}")
            res["mixed"] = smx
            res["autotune_tol_1e-3"] = tune(pl, q, sample=64 if big == 8000 else 0)
            log(f"n={big}: fp64 {s64['ms_median']:.1f} ms, mixed {smx['ms_median']:.1f} ms, "
                f"max |dl| {smx['max_abs_dl']:.2e}")
            return res
        guarded(key, both)

    if "batch" in extras:
        forms = () if args.batch_forms == "none" else tuple(args.batch_forms.split(","))
        guarded("uneven_batch", lambda: bench_uneven(pl, max(3, args.steps // 2), forms))
    if "serve" in extras:
        guarded("serving", lambda: bench_serving(pl, args.serve_seconds, args.serve_rate, 4, 160))

    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
