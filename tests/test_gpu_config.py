"""Step 2 on the GPU: the numerical Hessian (pl_hessian, one batched
likelihood call) against the oracle's, and the configuration end to end."""
import numpy as np
import pytest
import torch

import synth
from oracle import config as oc

pytestmark = pytest.mark.gpu


def _fit(pl, pr, **kw):
    fit = pl.mle(pr.locs, pr.y, pr.X, pr.lam, **kw)
    print(pr.name, fit, flush=True)
    return fit


def _hessian_parity(pl, pr, omega_hat, lam_hat, st, fix, delta=0.05):
    got = pl.hessian(pr.locs, pr.y, pr.X, omega_hat, lam_hat, shape_transform=st,
                     fix_shape=fix, delta=delta)
    H, curv, f0, _ = oc.hessian_at(pr.locs, pr.y, pr.X, omega_hat, lam_hat, st, fix, delta)
    # FP64 likelihoods agree to ~1e-12 relative; the stencil divides by delta^2
    scale = 1e-10 * max(abs(f0), pr.n) / delta ** 2
    assert got["H"].shape == H.shape
    np.testing.assert_allclose(got["H"], H, rtol=0, atol=10 * scale)
    assert abs(got["lambda_curv"] - curv) <= 10 * scale
    assert abs(got["loglik"] - f0) <= 1e-8 * max(abs(f0), pr.n)
    return got


def test_hessian_matches_oracle_at_the_mle(plprof_lib):
    pl = plprof_lib
    pr = synth.small_problem(220, p=2, K=4, M=5, seed=71)
    fit = _fit(pl, pr)
    for st in (0, 1):
        h = _hessian_parity(pl, pr, fit["omega"], fit["lambda"], st, False)
    # at a maximum the quadratic approximation opens downwards in lambda
    assert h["lambda_curv"] < 0


def test_hessian_with_shape_fixed(plprof_lib):
    pl = plprof_lib
    pr = synth.small_problem(200, p=3, K=4, M=4, seed=72)
    for kappa in (0.5, 10.0):
        starts = pl.default_starts(pr.locs, shapes=(kappa,))
        fit = _fit(pl, pr, omega0=starts, fixed=("shape",))
        h = _hessian_parity(pl, pr, fit["omega"], fit["lambda"], 1 if kappa >= 4 else 0, True)
        assert h["H"].shape == (4, 4)


def test_configuration_end_to_end(plprof_lib):
    pl = plprof_lib
    pr = synth.small_problem(260, p=2, K=4, M=5, seed=73)
    fit = _fit(pl, pr)
    fits = [dict(fit, fixed_shape=False)]
    starts = pl.default_starts(pr.locs, shapes=(0.5,))
    fits.append(dict(_fit(pl, pr, omega0=starts, fixed=("shape",)), fixed_shape=True))
    alpha = (0.999, 0.8, 0.5, 0.2, 0.05)
    cfg = pl.configure(pr.locs, pr.y, pr.X, fits, alpha=alpha, npts=40, seed=5,
                       sphere_iters=100)
    om = cfg["omega"]
    assert om.shape == (2 * len(alpha) * 40, 5)
    assert np.all(om[:, 0] > 0) and np.all(om[:, 2] >= 0) and np.all(om[:, 3] >= 1.0)
    assert np.all((om[:, 1] >= 0.05) & (om[:, 1] <= 100.0))
    assert np.all(om[len(alpha) * 40:, 1] == 0.5)
    lam = cfg["lambda"]
    assert lam.shape == (30,) and abs(0.5 * (lam[0] + lam[-1]) - fit["lambda"]) < 1e-12
    # the same points from the oracle's map, given the library's Hessian
    sph = pl.sphere_points(5, 40, init=np.random.Generator(np.random.PCG64(5))
                           .standard_normal((40, 5)), iters=100)[0]
    h0 = cfg["fits"][0]
    u = np.random.Generator(np.random.PCG64(5))
    u.standard_normal((40, 5))
    uu = u.uniform(size=len(alpha) * 40)
    want, _, _ = oc.config_points(fit["omega"], h0["shape_transform"], False, h0["H"], alpha,
                                  sph, uu)
    np.testing.assert_allclose(om[:len(alpha) * 40], want, rtol=1e-9, atol=1e-12)
    # the likelihood falls further on the outer contours: the mean drop at
    # lambda_hat grows with the level's chi-square quantile
    res = pl.profile_loglik(pr.locs, pr.y, pr.X, om[:len(alpha) * 40], [fit["lambda"]])
    torch.cuda.synchronize()
    ll = res["loglik"].cpu().numpy().reshape(len(alpha), 40)
    drop = np.nanmean(fit["loglik"] - np.where(np.isfinite(ll), ll, np.nan), axis=1)
    print("mean drop per level", drop, flush=True)
    assert np.all(np.diff(drop) > 0)
    assert np.all(drop > -1e-6)
