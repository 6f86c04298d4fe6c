"""Mixed-precision form against the FP64 oracle: |delta l| <= 1e-2 absolute
(well inside the 1.92 half-width of a 95% chi-square(1) likelihood interval),
the effect of the FP64 refinement of the cross products, and the FP64
fallback for points whose FP32 factorisation breaks down."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu
TOL_LL = 1e-2


def _run(pl, pr, **kw):
    res = pl.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, pr.lam, return_beta=True, **kw)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in res.items()}


@pytest.mark.parametrize("n,p,K,M,seed", [(300, 2, 4, 3, 11), (700, 4, 4, 8, 12), (1100, 3, 3, 4, 13),
                                          (500, 4, 3, 24, 14)])
def test_mixed_parity(plprof_lib, n, p, K, M, seed):
    pl = plprof_lib
    pr = synth.small_problem(n, p=p, K=K, M=M, seed=seed)
    got = _run(pl, pr, precision="mixed")
    ref, refb = oracle.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, pr.lam, return_beta=True)
    assert np.all((got["info"] & ~pl.PL_INFO_FALLBACK) == 0)
    dll = np.abs(got["loglik"] - ref["loglik"])
    print(f"n={n}: max |dl| = {dll.max():.2e}, max |d logdet| = "
          f"{np.abs(got['logdet_v'] - ref['logdet_v']).max():.2e}, max |d beta| = "
          f"{np.abs(got['beta'] - refb).max():.2e}")
    assert dll.max() <= TOL_LL
    assert np.abs(got["loglik_reml"] - ref["loglik_reml"]).max() <= TOL_LL
    np.testing.assert_allclose(got["beta"], refb, rtol=0, atol=1e-3 * max(1.0, np.abs(refb).max()))


def test_refinement_reduces_error(plprof_lib):
    pl = plprof_lib
    pr = synth.small_problem(900, p=3, K=4, M=4, seed=21)
    ref = oracle.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, pr.lam)
    e1 = np.abs(_run(pl, pr, precision="mixed", refine=1)["ssq_resid"] - ref["ssq_resid"]) / ref["ssq_resid"]
    e0 = np.abs(_run(pl, pr, precision="mixed", refine=0)["ssq_resid"] - ref["ssq_resid"]) / ref["ssq_resid"]
    print(f"relative SSR error: refined {e1.max():.2e}, unrefined {e0.max():.2e}")
    assert e1.max() < e0.max()


def test_mixed_full_size_sampled(plprof_lib):
    # n=4000, K=256, M=8 (the mixed-precision workload), a seeded sample of
    # omega points against the oracle
    pl = plprof_lib
    pr = synth.config_mixed()
    got = _run(pl, pr, precision="mixed")
    ok = (got["info"] & ~pl.PL_INFO_FALLBACK) == 0
    assert np.all(ok)
    idx = np.random.default_rng(1).choice(pr.K, 3, replace=False)
    ref, refb = oracle.profile_loglik(pr.locs, pr.y, pr.X, pr.omega[idx], pr.lam, return_beta=True)
    dll = np.abs(got["loglik"][idx] - ref["loglik"])
    print(f"n=4000 sample: max |dl| = {dll.max():.2e}, fallbacks = "
          f"{int(np.sum((got['info'][:, 0] & pl.PL_INFO_FALLBACK) != 0))}")
    assert dll.max() <= TOL_LL


def test_fallback_redoes_fp32_breakdowns_in_fp64(plprof_lib):
    # duplicated locations in different tiles with a tiny nugget: V is SPD in
    # FP64 but the FP32 Schur complements lose positivity
    pl = plprof_lib
    pr = synth.small_problem(260, p=2, K=3, M=2, seed=31)
    locs = pr.locs.copy()
    for i in range(0, 40):
        locs[130 + i] = locs[i] + 1e-9
    om = pr.omega.copy()
    om[1] = [2.0, 2.5, 1e-7, 1.0, 0.0]
    got = pl.profile_loglik(locs, pr.y, pr.X, om, pr.lam, precision="mixed")
    torch.cuda.synchronize()
    info = got["info"].cpu().numpy()
    ll = got["loglik"].cpu().numpy()
    ref = oracle.profile_loglik(locs, pr.y, pr.X, om, pr.lam)
    assert ref["info"][1, 0] == 0, "the constructed point must be SPD in FP64"
    fb = (info[1] & pl.PL_INFO_FALLBACK) != 0
    assert np.all(fb), "expected the FP32 factorisation of point 1 to break down"
    assert np.all((info[1] & ~pl.PL_INFO_FALLBACK) == 0)
    scale = np.maximum(np.abs(ref["loglik"][1]), pr.n)
    assert np.max(np.abs(ll[1] - ref["loglik"][1]) / scale) <= 1e-8
    assert np.max(np.abs(ll[[0, 2]] - ref["loglik"][[0, 2]])) <= TOL_LL


@pytest.mark.parametrize("flush", [1, 2, 4])
def test_mixed_parity_each_flush(plprof_lib, flush):
    """Every FP32 partial-sum depth the autotuner may pick stays within the
    mixed tolerance of the oracle; shorter partial sums are not less accurate
    here than the longest."""
    pl = plprof_lib
    pr = synth.small_problem(1000, p=3, K=3, M=4, seed=31)
    ref = oracle.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, pr.lam)
    got = _run(pl, pr, precision="mixed", flush=flush)
    d = np.abs(got["loglik"] - ref["loglik"]).max()
    print(f"flush {flush}: max |dl| = {d:.2e}")
    assert d <= TOL_LL


def test_autotune_respects_error_budget(plprof_lib):
    pl = plprof_lib
    pr = synth.small_problem(900, p=3, K=10, M=4, seed=41)
    # a zero budget admits only the FP64 form
    choice, rep = pl.autotune(pr.locs, pr.y, pr.X, pr.omega, pr.lam, tol=0.0)
    assert choice == {"precision": "fp64", "flush": 0}
    assert rep["fp64"]["max_abs_dl"] == 0.0 and rep["fp64"]["ms_per_omega"] > 0
    for key in ("mixed/flush4", "mixed/flush2", "mixed/flush1"):
        assert rep[key]["ms_per_omega"] > 0 and 0 < rep[key]["max_abs_dl"] < TOL_LL
    # a loose budget picks the fastest candidate, and the chosen form meets it
    choice, rep = pl.autotune(pr.locs, pr.y, pr.X, pr.omega, pr.lam, tol=1e-2)
    key = "fp64" if choice["precision"] == "fp64" else f"mixed/flush{choice['flush']}"
    assert rep[key]["ms_per_omega"] == min(v["ms_per_omega"] for v in rep.values())
    ref = oracle.profile_loglik(pr.locs, pr.y, pr.X, pr.omega[:3], pr.lam)
    got = pl.profile_loglik(pr.locs, pr.y, pr.X, pr.omega[:3], pr.lam, **choice)
    torch.cuda.synchronize()
    assert np.abs(got["loglik"].cpu().numpy() - ref["loglik"]).max() <= 1e-2
    print("autotune report", rep, "->", choice)


# bordered heights above 32: the bordered row is updated as a tile row of its
# own and the back substitution and refined cross products run at 48 and 64
# right-hand sides; the shapes of the paper's examples (Swiss rainfall:
# 34 Box-Cox values and 2 covariates at n = 100; soil mercury: 31 values and
# 18 covariates at n = 829, Sections 6 and 7) among them
@pytest.mark.parametrize("n,p,K,M,seed", [(100, 2, 4, 34, 90), (829, 18, 3, 31, 91),
                                          (300, 2, 3, 36, 92), (420, 4, 3, 60, 93)])
def test_mixed_tall_border_matches_oracle(plprof_lib, n, p, K, M, seed):
    pl = plprof_lib
    pr = synth.small_problem(n, p=p, K=K, M=M, seed=seed)
    print(f"mixed n={n} M+p={M + p}", flush=True)
    got = _run(pl, pr, precision="mixed")
    ref, refb = oracle.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, pr.lam, return_beta=True)
    assert np.all((got["info"] & ~pl.PL_INFO_FALLBACK) == 0)
    dll = np.abs(got["loglik"] - ref["loglik"])
    print(f"  max |dl| = {dll.max():.2e}")
    assert dll.max() <= TOL_LL
    assert np.abs(got["loglik_reml"] - ref["loglik_reml"]).max() <= TOL_LL
    np.testing.assert_allclose(got["beta"], refb, rtol=0, atol=1e-3 * max(1.0, np.abs(refb).max()))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_workspace_contents_do_not_leak_into_results(plprof_lib, precision):
    """The padding of the last block column (rows past n) is never read as
    data: a workspace filled with all-ones bytes (NaN in FP32 and FP64) gives
    the same records, bit for bit, as one filled with zeros."""
    pl = plprof_lib
    pr = synth.small_problem(300, p=2, K=3, M=2, seed=77, aniso=True)
    size = pl.workspace_size(300, 2, 3, 2, precision, 0)
    print(f"workspace fill: {precision}, n = 300, {size} bytes", flush=True)
    recs = []
    for fill in (0, 255):
        work = torch.full((size,), fill, dtype=torch.uint8, device="cuda")
        recs.append(_run(pl, pr, precision=precision, work=work))
    for key in ("loglik", "loglik_reml", "logdet_v", "info", "beta"):
        np.testing.assert_array_equal(recs[0][key], recs[1][key], err_msg=key)
    assert np.all(np.isfinite(recs[0]["loglik"]))
