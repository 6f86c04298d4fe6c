"""Parity of the HIP path with the FP64 oracle, through the C ABI.

Tolerances: covariance elements 1e-12 absolute (rho <= 1; the oracle's own
Bessel route is good to ~1e-13); log|V| and l_p within
1e-8 * max(|l_p|, n) (the FP64 criterion for this path); beta-hat within
1e-7 relative to max(1, |beta|)."""
import dataclasses
import math

import numpy as np
from scipy.linalg import lapack
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

FIELDS = ("loglik", "logdet_v", "logdet_xvx", "ssq_y", "ssq_betahat", "ssq_resid",
          "sigma2_hat", "jacobian", "loglik_reml")


def _gpu(pl, pr, **kw):
    res = pl.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, pr.lam, return_beta=True, **kw)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in res.items()}


def _check(got, ref, refb, n, tol=1e-8):
    # relative to the log-likelihood itself (floored at 1 for values near 0),
    # and absolute per location
    assert np.all(got["info"] == ref["info"]), (got["info"], ref["info"])
    for f in ("loglik", "loglik_reml"):
        d = np.abs(got[f] - ref[f])
        rel = d / np.maximum(np.abs(ref[f]), 1.0)
        assert np.max(rel) <= tol, f"max rel {f} err {np.max(rel):.3e}"
        assert np.max(d) <= tol * n, f"max abs {f} err {np.max(d):.3e}"
    err = np.abs(got["loglik"] - ref["loglik"]) / np.maximum(np.abs(ref["loglik"]), 1.0)
    np.testing.assert_allclose(got["logdet_v"], ref["logdet_v"], rtol=0, atol=tol * n)
    np.testing.assert_allclose(got["jacobian"], ref["jacobian"], rtol=1e-13, atol=1e-12)
    for f in ("ssq_y", "ssq_resid", "ssq_betahat", "sigma2_hat"):
        np.testing.assert_allclose(got[f], ref[f], rtol=1e-8, atol=1e-10 * np.max(np.abs(ref[f])))
    np.testing.assert_allclose(got["beta"], refb, rtol=1e-7, atol=1e-7)
    return float(np.max(err))


def test_mfma_layout_via_small_chol(plprof_lib):
    # n = 300: three tile rows with a ragged tail of 44; exercises every
    # kernel's fragment layout against LAPACK on the oracle's V
    pl = plprof_lib
    pr = synth.small_problem(300, p=2, K=3, M=1, seed=3)
    Vs = np.stack([oracle.build_V(pr.locs, om) for om in pr.omega])
    V = torch.tensor(np.ascontiguousarray(np.transpose(Vs, (0, 2, 1))), device="cuda")
    logdet, info = pl.chol_batched(V)
    torch.cuda.synchronize()
    L = np.transpose(V.cpu().numpy(), (0, 2, 1))
    for k in range(pr.K):
        Lr = np.linalg.cholesky(Vs[k])
        np.testing.assert_allclose(np.tril(L[k]), Lr, rtol=0, atol=1e-11)
        assert abs(logdet[k].item() - 2 * np.sum(np.log(np.diag(Lr)))) < 1e-10 * pr.n
    assert np.all(info.cpu().numpy() == 0)


@pytest.mark.parametrize("n,aniso", [(7, True), (128, False), (300, True), (520, True)])
def test_matern_cov_elementwise(plprof_lib, n, aniso):
    pl = plprof_lib
    pr = synth.small_problem(n, p=2, K=8, M=1, seed=n, aniso=aniso,
                             kappas=[0.05, 0.2, 0.5, 1.0, 1.5, 2.37, 4.5, 9.8])
    V = pl.matern_cov(pr.locs, pr.omega)
    torch.cuda.synchronize()
    Vg = np.transpose(V.cpu().numpy(), (0, 2, 1))
    for k in range(pr.K):
        ref = oracle.build_V(pr.locs, pr.omega[k])
        lo = np.tril_indices(n)
        err = np.max(np.abs(Vg[k][lo] - ref[lo]))
        assert err <= 1e-12, (k, pr.omega[k], err)


def test_matern_close_points_and_duplicates(plprof_lib):
    # pairs closer than the table's lower end go through the direct quadrature;
    # duplicates give rho = 1 exactly
    pl = plprof_lib
    rng = np.random.default_rng(5)
    base = rng.uniform(0, 1, (40, 2))
    locs = np.concatenate([base, base[:10] + rng.uniform(-1e-6, 1e-6, (10, 2)), base[10:14]])
    om = np.array([[0.5, k, 0.1, 2.0, 0.3] for k in (0.05, 0.3, 1.0, 3.3, 12.0, 60.0)])
    V = pl.matern_cov(locs, om)
    torch.cuda.synchronize()
    Vg = np.transpose(V.cpu().numpy(), (0, 2, 1))
    lo = np.tril_indices(locs.shape[0])
    for k in range(om.shape[0]):
        ref = oracle.build_V(locs, om[k])
        err = np.max(np.abs(Vg[k][lo] - ref[lo]))
        assert err <= 2e-12, (om[k], err)


# M + p up to 16 and to 32 (the bordered row folded into the diagonal tile's
# workgroup, one or two block rows) and beyond 32 (bordered tiles of their
# own), up to 60 (four block rows in the bordered row's panel solve)
@pytest.mark.parametrize("n,p,K,M,seed", [(50, 1, 3, 1, 0), (128, 2, 4, 3, 1), (300, 3, 5, 4, 2),
                                          (700, 4, 4, 8, 3), (257, 6, 3, 5, 4),
                                          (400, 5, 3, 20, 5), (300, 4, 2, 40, 6),
                                          (270, 4, 2, 56, 7)])
def test_profile_loglik_parity(plprof_lib, n, p, K, M, seed):
    pl = plprof_lib
    pr = synth.small_problem(n, p=p, K=K, M=M, seed=seed)
    got = _gpu(pl, pr)
    ref, refb = oracle.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, pr.lam, return_beta=True)
    _check(got, ref, refb, n)


def test_config_iso_grid_full(plprof_lib):
    # n=200, 4x4x4 grid x 3 lambdas: every record against the oracle
    pl = plprof_lib
    pr = synth.config_iso_grid()
    got = _gpu(pl, pr)
    ref, refb = oracle.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, pr.lam, return_beta=True)
    _check(got, ref, refb, pr.n)


def test_chunking_is_bitwise_invariant(plprof_lib):
    pl = plprof_lib
    pr = synth.small_problem(260, p=2, K=7, M=3, seed=8)
    a = _gpu(pl, pr)
    b = _gpu(pl, pr, chunk=2)
    c = _gpu(pl, pr, chunk=1)
    for f in FIELDS:
        assert np.array_equal(a[f], b[f]) and np.array_equal(a[f], c[f]), f


def test_non_pd_point_isolated(plprof_lib):
    pl = plprof_lib
    pr = synth.small_problem(150, p=2, K=3, M=2, seed=9)
    locs = pr.locs
    om = pr.omega.copy()
    # range 50, shape 50, no nugget on a domain of side 5: numerical rank ~16,
    # so any FP64 factorisation meets a non-positive pivot (a singular V that
    # is only singular in exact arithmetic, e.g. a duplicate location without
    # nugget, can factor with a tiny positive pivot in either implementation)
    om[1] = [50.0, 50.0, 0.0, 1.0, 0.0]
    assert lapack.dpotrf(oracle.build_V(locs, om[1]), lower=1)[1] > 0
    got = pl.profile_loglik(locs, pr.y, pr.X, om, pr.lam)
    torch.cuda.synchronize()
    info = got["info"].cpu().numpy()
    ll = got["loglik"].cpu().numpy()
    assert np.all(info[1] > 0) and np.all(ll[1] == -np.inf)
    ref = oracle.profile_loglik(locs, pr.y, pr.X, om[[0, 2]], pr.lam)
    np.testing.assert_allclose(ll[[0, 2]], ref["loglik"], rtol=1e-9)
    assert np.all(info[[0, 2]] == 0)


def test_bad_y_flags_every_record(plprof_lib):
    pl = plprof_lib
    pr = synth.small_problem(100, p=2, K=2, M=2, seed=10)
    y = pr.y.copy()
    y[5] = -1.0
    got = pl.profile_loglik(pr.locs, y, pr.X, pr.omega, pr.lam)
    torch.cuda.synchronize()
    assert np.all(got["info"].cpu().numpy() == pl.PL_INFO_BAD_Y)
    assert np.all(np.isnan(got["loglik"].cpu().numpy()))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_profile_close_pairs_take_the_quadrature(plprof_lib, precision):
    """Pairs closer than the tables' lower end (w < 2^-20), spread over
    several tiles of the packed build, one exact duplicate among them: their
    elements come from the build's quadrature launch (or are 1), and the
    records match the oracle."""
    pl = plprof_lib
    pr = synth.small_problem(300, p=2, K=3, M=2, seed=21, aniso=True)
    rng = np.random.default_rng(21)
    idx = rng.permutation(300)[:24]
    locs = pr.locs.copy()
    locs[idx[12:]] = locs[idx[:12]] + rng.uniform(-1e-6, 1e-6, (12, 2))
    locs[idx[23]] = locs[idx[11]]
    pr = dataclasses.replace(pr, locs=locs)
    print(f"close pairs: {precision}, n = 300, 12 pairs", flush=True)
    got = _gpu(pl, pr, precision=precision)
    ref, refb = oracle.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, pr.lam, return_beta=True)
    if precision == "fp64":
        _check(got, ref, refb, pr.n)
    else:
        assert np.all((got["info"] & ~pl.PL_INFO_FALLBACK) == 0)
        assert np.max(np.abs(got["loglik"] - ref["loglik"])) <= 1e-2
