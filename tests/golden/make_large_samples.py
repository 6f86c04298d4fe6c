#!/usr/bin/env python3
"""Write tests/golden/large_samples.json: oracle records for seeded samples of
omega points of the full-size anisotropic workloads, so that GPU tests and the
benchmark can compare full-size runs with the oracle without spending minutes
of CPU time per run.

Only `oracle` (the FP64 reference) and `synth` (the seeded input generator)
are called; nothing here touches the HIP library.  The inputs are regenerated
from their seeds wherever the file is used; the fingerprints stored with each
workload (sums of y, locations and X) let a reader check that it regenerated
the same data.

Workloads (equation "profile" per (omega, lambda); Section 3.3, Step 3):
  aniso_n2000  n=2000, p=4, K=1024, M=8 (the headline workload), 48 omega
  aniso_n4000  n=4000, K=256, M=8 (the mixed-precision workload), 16 omega
  aniso_n8000  n=8000, K=256, M=8 (the anisotropic generator at n=8000), 8 omega

Usage: python tests/golden/make_large_samples.py [--workers W]
"""
import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "large_samples.json")
FIELDS = ("loglik", "logdet_v", "logdet_xvx", "ssq_y", "ssq_betahat", "ssq_resid",
          "sigma2_hat", "jacobian", "loglik_reml", "info")

# name -> (synth function, keyword arguments, omega points sampled, sample seed)
WORKLOADS = {
    "aniso_n2000": ("config_aniso", {"n": 2000, "K": 1024, "M": 8}, 48, 20),
    "aniso_n4000": ("config_mixed", {"n": 4000, "K": 256, "M": 8}, 16, 40),
    "aniso_n8000": ("config_aniso", {"n": 8000, "K": 256, "M": 8}, 8, 80),
}


def make_problem(fn, kwargs):
    import synth
    return getattr(synth, fn)(**kwargs)


def fingerprint(pr):
    return {"sum_y": float(np.sum(pr.y)), "sum_locs": float(np.sum(pr.locs)),
            "sum_X": float(np.sum(pr.X)), "n": pr.n, "p": pr.p, "K": pr.K, "M": pr.M}


def sample_indices(K, count, seed):
    return sorted(int(i) for i in np.random.default_rng(seed).choice(K, count, replace=False))


_PR = None


def _init(fn, kwargs):
    global _PR
    _PR = make_problem(fn, kwargs)


def _point(k):
    from threadpoolctl import threadpool_limits

    import oracle
    with threadpool_limits(1):
        rec, beta = oracle.profile_loglik(_PR.locs, _PR.y, _PR.X, _PR.omega[k:k + 1], _PR.lam,
                                          return_beta=True)
    return k, {f: np.asarray(rec[f])[0].tolist() for f in FIELDS}, beta[0].tolist()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("--only", default="", help="comma list of workload names")
    args = ap.parse_args()
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    names = [w for w in args.only.split(",") if w] or list(WORKLOADS)
    for name in names:
        fn, kwargs, count, seed = WORKLOADS[name]
        pr = make_problem(fn, kwargs)
        idx = sample_indices(pr.K, count, seed)
        t0 = time.time()
        workers = args.workers if pr.n < 8000 else max(1, min(args.workers, 6))
        recs, betas = {}, {}
        with ProcessPoolExecutor(max_workers=workers, initializer=_init,
                                 initargs=(fn, kwargs)) as ex:
            for k, rec, beta in ex.map(_point, idx):
                recs[k], betas[k] = rec, beta
        data[name] = {
            "generator": {"function": f"synth.{fn}", "kwargs": kwargs},
            "fingerprint": fingerprint(pr),
            "omega_index": idx,
            "lambda": pr.lam.tolist(),
            "records": {f: [recs[k][f] for k in idx] for f in FIELDS},
            "beta": [betas[k] for k in idx],
        }
        print(f"{name}: {len(idx)} omega in {time.time() - t0:.1f} s", flush=True)
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
