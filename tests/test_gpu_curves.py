"""Profile curves of sigma and of single coefficients (pl_profile_curves) and
(X^T V^-1 X)^-1 (pl_profile_loglik's xvx_inv) against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


def _setup(pl, pr, locs=None, omega=None, precision="fp64"):
    locs = pr.locs if locs is None else locs
    omega = pr.omega if omega is None else omega
    res = pl.profile_loglik(locs, pr.y, pr.X, omega, pr.lam, return_beta=True,
                            return_xvx_inv=True, precision=precision)
    ref, rb = oracle.profile_loglik(locs, pr.y, pr.X, omega, pr.lam, return_beta=True)
    ll = np.where(ref["info"] == 0, ref["loglik"], -np.inf)
    k, m = np.unravel_index(int(np.argmax(ll)), ll.shape)
    s_hat = np.sqrt(ref["sigma2_hat"][k, m])
    sgrid = s_hat * np.linspace(0.6, 1.6, 21)
    bgrid = np.stack([rb[k, m, j] + np.linspace(-1.5, 1.5, 17) for j in range(pr.p)])
    return res, sgrid, bgrid, locs, omega


def _check(pl, pr, res, sgrid, bgrid, locs, omega, tol_rel=None, tol_abs=None):
    cv = pl.profile_curves(res, pr.lam, pr.n, sigma_grid=sgrid, beta_grid=bgrid)
    torch.cuda.synchronize()
    sig, sarg, bet, barg, sall, ball = oracle.curves(locs, pr.y, pr.X, omega, pr.lam, sgrid,
                                                     bgrid, per_record=True)
    gs, gsa = cv["sigma"].cpu().numpy(), cv["sigma_arg"].cpu().numpy()
    gb, gba = cv["beta"].cpu().numpy(), cv["beta_arg"].cpu().numpy()
    lim = lambda ref: (tol_rel * np.maximum(np.abs(ref), pr.n)) if tol_rel else tol_abs
    assert np.all(np.abs(gs - sig) <= lim(sig)), np.abs(gs - sig).max()
    assert np.all(np.abs(gb - bet) <= lim(bet)), np.abs(gb - bet).max()
    # the record the GPU picked attains the maximum (ties may pick another)
    for g in range(sgrid.shape[0]):
        assert np.abs(sall[g, gsa[g]] - sig[g]) <= lim(sig[g])
    for j in range(pr.p):
        for g in range(bgrid.shape[1]):
            assert np.abs(ball[j, g, gba[j, g]] - bet[j, g]) <= lim(bet[j, g])
    return gs, gb


def test_xvx_inverse_matches_oracle(plprof_lib):
    pl = plprof_lib
    pr = synth.small_problem(260, p=4, K=5, M=3, seed=51)
    res = pl.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, pr.lam, return_xvx_inv=True)
    torch.cuda.synchronize()
    got = res["xvx_inv"].cpu().numpy()
    ssq, _ = oracle.cross_products(pr.locs, pr.y, pr.X, pr.omega, pr.lam)
    for k in range(pr.K):
        want = np.linalg.inv(ssq[k][pr.M:, pr.M:])
        np.testing.assert_allclose(got[k], want, rtol=1e-9, atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("n,p,K,M,seed", [(180, 2, 8, 3, 52), (420, 4, 6, 4, 53), (700, 1, 5, 2, 54)])
def test_curves_match_oracle(plprof_lib, n, p, K, M, seed):
    pl = plprof_lib
    pr = synth.small_problem(n, p=p, K=K, M=M, seed=seed)
    res, sgrid, bgrid, locs, om = _setup(pl, pr)
    gs, gb = _check(pl, pr, res, sgrid, bgrid, locs, om, tol_rel=1e-8)
    # the curves peak at the largest profile log-likelihood
    top = float(res["loglik"].max().item())
    assert gs.max() <= top + 1e-8 * abs(top) and gb.max() <= top + 1e-8 * abs(top)


def test_curves_skip_non_pd_points(plprof_lib):
    pl = plprof_lib
    pr = synth.small_problem(150, p=2, K=4, M=2, seed=55)
    om = pr.omega.copy()
    # range 50, shape 50, no nugget on a domain of side 5: numerical rank ~16,
    # so any FP64 factorisation meets a non-positive pivot
    om[1] = [50.0, 50.0, 0.0, 1.0, 0.0]
    res, sgrid, bgrid, locs, om = _setup(pl, pr, omega=om)
    info = res["info"].cpu().numpy()
    assert np.all(info[1] > 0)
    cv = pl.profile_curves(res, pr.lam, pr.n, sigma_grid=sgrid, beta_grid=bgrid)
    torch.cuda.synchronize()
    bad = {1 * pr.M + m for m in range(pr.M)}
    assert not (set(cv["sigma_arg"].cpu().numpy().tolist()) & bad)
    assert not (set(cv["beta_arg"].cpu().numpy().ravel().tolist()) & bad)
    _check(pl, pr, res, sgrid, bgrid, locs, om, tol_rel=1e-8)


def test_mixed_form_curves_within_mixed_tolerance(plprof_lib):
    pl = plprof_lib
    pr = synth.small_problem(900, p=3, K=4, M=3, seed=56)
    res, sgrid, bgrid, locs, om = _setup(pl, pr, precision="mixed")
    _check(pl, pr, res, sgrid, bgrid, locs, om, tol_abs=1e-2)


def test_step4_profiles_match_oracle(plprof_lib):
    """Univariate profiles of every correlation parameter and of lambda from
    GPU records equal those the oracle extracts from its own records."""
    from oracle.extract import profile as oracle_profile
    pl = plprof_lib
    pr = synth.small_problem(240, p=2, K=40, M=5, seed=61)
    res = pl.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, pr.lam)
    torch.cuda.synchronize()
    ref = oracle.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, pr.lam)
    for which in range(6):
        got = pl.profile_param(res, pr.omega, pr.lam, which)
        ox, oy, am, lo, hi, op = oracle_profile(ref["loglik"], ref["info"] == 0, pr.omega, pr.lam,
                                                which)
        np.testing.assert_array_equal(got["x"], ox)
        np.testing.assert_allclose(got["y"], oy, rtol=1e-9)
        assert got["argmax"] == am and got["open"] == op
        scale = max(1.0, abs(ox).max())
        np.testing.assert_allclose([got["lower"], got["upper"]], [lo, hi], rtol=0, atol=1e-6 * scale)
