"""Pins of the oracle's sigma and single-coefficient profile curves
(Sections 3.4 and 3.5, the profile likelihoods for beta_p and for sigma)."""
import math

import numpy as np

import oracle
import synth
from oracle.curves import cross_products, curves, ssr_fixed_coefficient
from oracle.likelihood import full_loglik, gauss_jordan_inverse, lu_logdet, transformed_columns
from oracle.model import build_V


def _problem(n=40, p=3, K=3, M=2, seed=5):
    return synth.small_problem(n, p=p, K=K, M=M, seed=seed)


def test_fixed_coefficient_ssr_matches_constrained_gls_brute_force():
    """SSR from the subsetting identities equals the residual quadratic form
    of a direct constrained GLS fit (explicit Gauss-Jordan inverse of V):
    regress y' - X_j b on the other columns."""
    pr = _problem()
    n, p = pr.X.shape
    ssq, _ = cross_products(pr.locs, pr.y, pr.X, pr.omega, pr.lam)
    Yt = transformed_columns(pr.y, pr.lam)
    for k in range(pr.K):
        Vi = gauss_jordan_inverse(build_V(pr.locs, pr.omega[k]))
        for m in range(pr.M):
            for j in range(p):
                for b in (-1.3, 0.2, 2.5):
                    rest = [i for i in range(p) if i != j]
                    yo = Yt[:, m] - pr.X[:, j] * b
                    Xr = pr.X[:, rest]
                    br = np.linalg.solve(Xr.T @ Vi @ Xr, Xr.T @ Vi @ yo)
                    r = yo - Xr @ br
                    want = float(r @ Vi @ r)
                    got = ssr_fixed_coefficient(ssq[k], pr.M, m, j, b)
                    assert abs(got - want) <= 1e-9 * max(1.0, abs(want))


def test_fixed_coefficient_ssr_closed_form():
    """The minimal SSR grows by (b - betahat_j)^2 / [(X^T V^-1 X)^-1]_jj (a
    block-inverse identity), for every coefficient and lambda."""
    pr = _problem(p=4, seed=6)
    ssq, _ = cross_products(pr.locs, pr.y, pr.X, pr.omega, pr.lam)
    M = pr.M
    for k in range(pr.K):
        xx, Ainv = ssq[k][M:, M:], np.linalg.inv(ssq[k][M:, M:])
        for m in range(M):
            bh = np.linalg.solve(xx, ssq[k][M:, m])
            ssr = ssq[k][m, m] - ssq[k][M:, m] @ bh
            for j in range(pr.p):
                for b in (bh[j], bh[j] + 0.7, bh[j] - 2.0):
                    got = ssr_fixed_coefficient(ssq[k], M, m, j, b)
                    want = ssr + (b - bh[j]) ** 2 / Ainv[j, j]
                    assert abs(got - want) <= 1e-10 * max(1.0, abs(want))


def test_curve_values_are_equation_2_at_the_constrained_estimates():
    """Every curve value is equation (2) evaluated at the fixed parameter and
    the remaining closed-form estimates (brute-force inverse/determinant)."""
    pr = _problem(n=30, K=2, M=2, seed=7)
    n, p = pr.X.shape
    Yt = transformed_columns(pr.y, pr.lam)
    J = float(np.sum(np.log(pr.y)))
    sgrid = np.array([0.6, 1.1])
    bgrid = np.array([[0.3, 1.4], [-0.5, 0.5], [0.0, 0.9]])
    sig, sarg, bet, barg = curves(pr.locs, pr.y, pr.X, pr.omega, pr.lam, sgrid, bgrid)
    best_s = np.full(2, -np.inf)
    best_b = np.full((p, 2), -np.inf)
    for k in range(pr.K):
        V = build_V(pr.locs, pr.omega[k])
        Vi = gauss_jordan_inverse(V)
        ldv = lu_logdet(V)[1]
        for m in range(pr.M):
            bh = np.linalg.solve(pr.X.T @ Vi @ pr.X, pr.X.T @ Vi @ Yt[:, m])
            for g, s in enumerate(sgrid):
                v = full_loglik(bh, s * s, Yt[:, m], pr.X, Vi, ldv, pr.lam[m], J)
                best_s[g] = max(best_s[g], v)
            for j in range(p):
                rest = [i for i in range(p) if i != j]
                for g, b in enumerate(bgrid[j]):
                    yo = Yt[:, m] - pr.X[:, j] * b
                    Xr = pr.X[:, rest]
                    br = np.linalg.solve(Xr.T @ Vi @ Xr, Xr.T @ Vi @ yo)
                    beta = np.empty(p)
                    beta[j] = b
                    beta[rest] = br
                    r = Yt[:, m] - pr.X @ beta
                    s2 = float(r @ Vi @ r) / n
                    best_b[j, g] = max(best_b[j, g],
                                       full_loglik(beta, s2, Yt[:, m], pr.X, Vi, ldv, pr.lam[m], J))
    np.testing.assert_allclose(sig, best_s, rtol=1e-10, atol=1e-9)
    np.testing.assert_allclose(bet, best_b, rtol=1e-10, atol=1e-9)


def test_curves_touch_the_profile_maximum():
    """At sigma-hat and at betahat_j of the best record the curves equal the
    largest profile log-likelihood of the points, and never exceed it."""
    pr = _problem(n=60, p=2, K=4, M=3, seed=8)
    ref, beta = oracle.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, pr.lam, return_beta=True)
    ll = ref["loglik"]
    k, m = np.unravel_index(int(np.argmax(ll)), ll.shape)
    s_hat = math.sqrt(ref["sigma2_hat"][k, m])
    sgrid = np.array([0.5 * s_hat, s_hat, 2.0 * s_hat])
    bgrid = np.array([[beta[k, m, 0] - 1.0, beta[k, m, 0], beta[k, m, 0] + 1.0],
                      [beta[k, m, 1] - 1.0, beta[k, m, 1], beta[k, m, 1] + 1.0]])
    sig, sarg, bet, barg = curves(pr.locs, pr.y, pr.X, pr.omega, pr.lam, sgrid, bgrid)
    top = ll.max()
    assert abs(sig[1] - top) <= 1e-9 * abs(top) and sarg[1] == k * pr.M + m
    assert np.all(np.abs(bet[:, 1] - top) <= 1e-9 * abs(top))
    assert np.all(sig <= top + 1e-9 * abs(top)) and np.all(bet <= top + 1e-9 * abs(top))
    assert sig[0] < top and sig[2] < top and np.all(bet[:, 0] < top) and np.all(bet[:, 2] < top)


def test_single_covariate_has_no_remaining_coefficients():
    pr = _problem(n=25, p=1, K=2, M=2, seed=9)
    ssq, _ = cross_products(pr.locs, pr.y, pr.X, pr.omega, pr.lam)
    got = ssr_fixed_coefficient(ssq[0], pr.M, 1, 0, 0.4)
    want = ssq[0][1, 1] - 0.8 * ssq[0][2, 1] + 0.16 * ssq[0][2, 2]
    assert abs(got - want) <= 1e-12 * abs(want)
