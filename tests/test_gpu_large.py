"""Full-size anisotropic workloads against the oracle, through the C ABI.

The GPU evaluates the whole workload in the launch configuration of the
benchmark (all K omega points in one device pass); the records of a seeded
sample of omega points are compared with oracle values stored in
tests/golden/large_samples.json, which tests/golden/make_large_samples.py
wrote from the oracle alone (equation "profile"; Section 3.3, Step 3).

Bars: FP64 |dl| <= 1e-8 |l| (relative to the log-likelihood itself, floored
at 1 for values near 0) and <= 1e-8 n; mixed |dl| <= 1e-2 absolute."""
import json
import os

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "large_samples.json")
TOL_FP64 = 1e-8
TOL_MIXED = 1e-2


def golden(name):
    with open(GOLDEN) as f:
        g = json.load(f)[name]
    fn = getattr(synth, g["generator"]["function"].split(".", 1)[1])
    pr = fn(**g["generator"]["kwargs"])
    fp = g["fingerprint"]
    # the same seeded inputs as when the oracle values were written
    assert (pr.n, pr.p, pr.K, pr.M) == (fp["n"], fp["p"], fp["K"], fp["M"])
    for key, arr in (("sum_y", pr.y), ("sum_locs", pr.locs), ("sum_X", pr.X)):
        assert abs(float(np.sum(arr)) - fp[key]) <= 1e-12 * max(1.0, abs(fp[key])), key
    np.testing.assert_array_equal(pr.lam, np.asarray(g["lambda"]))
    idx = np.asarray(g["omega_index"])
    ref = {f: np.asarray(v) for f, v in g["records"].items()}
    return pr, idx, ref, np.asarray(g["beta"])


def run(pl, pr, precision):
    res = pl.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, pr.lam, precision=precision,
                            return_beta=True)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in res.items()}
    del res
    torch.cuda.empty_cache()
    return out


def check_fp64(got, ref, refb, n):
    assert np.all(got["info"] == ref["info"])
    for f in ("loglik", "loglik_reml"):
        d = np.abs(got[f] - ref[f])
        rel = d / np.maximum(np.abs(ref[f]), 1.0)
        assert rel.max() <= TOL_FP64, (f, rel.max())
        assert d.max() <= TOL_FP64 * n, (f, d.max())
    np.testing.assert_allclose(got["logdet_v"], ref["logdet_v"], rtol=TOL_FP64, atol=0)
    for f in ("ssq_y", "ssq_resid", "ssq_betahat", "sigma2_hat", "logdet_xvx"):
        np.testing.assert_allclose(got[f], ref[f], rtol=1e-8, atol=1e-10 * np.max(np.abs(ref[f])))
    np.testing.assert_allclose(got["beta"], refb, rtol=1e-7, atol=1e-7)


@pytest.mark.parametrize("name", ["aniso_n2000", "aniso_n4000", "aniso_n8000"])
def test_full_size_fp64_matches_oracle(plprof_lib, name):
    pl = plprof_lib
    pr, idx, ref, refb = golden(name)
    print(f"{name}: n={pr.n} K={pr.K} M={pr.M}, FP64, {len(idx)} sampled omega", flush=True)
    got = run(pl, pr, "fp64")
    assert np.all(got["info"] == 0)
    sub = {k: v[idx] for k, v in got.items()}
    check_fp64(sub, ref, refb, pr.n)
    rel = np.abs(sub["loglik"] - ref["loglik"]) / np.abs(ref["loglik"])
    print(f"{name}: max relative |dl| {rel.max():.2e}")


@pytest.mark.parametrize("name", ["aniso_n2000", "aniso_n4000", "aniso_n8000"])
def test_full_size_mixed_matches_oracle(plprof_lib, name):
    pl = plprof_lib
    pr, idx, ref, refb = golden(name)
    print(f"{name}: n={pr.n} K={pr.K} M={pr.M}, mixed, {len(idx)} sampled omega", flush=True)
    got = run(pl, pr, "mixed")
    assert np.all((got["info"] & ~pl.PL_INFO_FALLBACK) == 0)
    sub = {k: v[idx] for k, v in got.items()}
    dl = np.abs(sub["loglik"] - ref["loglik"])
    dr = np.abs(sub["loglik_reml"] - ref["loglik_reml"])
    db = np.abs(sub["beta"] - refb)
    print(f"{name}: max |dl| {dl.max():.2e}, max |dl reml| {dr.max():.2e}, max |dbeta| {db.max():.2e}")
    assert dl.max() <= TOL_MIXED
    assert dr.max() <= TOL_MIXED
    np.testing.assert_allclose(sub["beta"], refb, rtol=0, atol=1e-3 * max(1.0, np.abs(refb).max()))
