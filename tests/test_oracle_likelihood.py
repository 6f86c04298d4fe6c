"""Pins of the oracle's likelihood against routes that do not go through it:
brute-force inverse and determinant, the GLS normal equations, maximality of
the profile, closed forms at range -> 0, invariances of the Box-Cox Jacobian,
the REML identity, and the parameter conventions printed in the paper."""
import math
import os

import numpy as np
import pytest

import oracle
import synth
from oracle.likelihood import gauss_jordan_inverse, lu_logdet

HERE = os.path.dirname(os.path.abspath(__file__))


def _prob(n=30, p=3, K=4, M=3, seed=0, aniso=True):
    return synth.small_problem(n, p=p, K=K, M=M, seed=seed, aniso=aniso)


def test_bruteforce_helpers_against_numpy():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((12, 12)) + 12 * np.eye(12)
    np.testing.assert_allclose(gauss_jordan_inverse(A) @ A, np.eye(12), atol=1e-12)
    s, ld = lu_logdet(A)
    s2, ld2 = np.linalg.slogdet(A)
    assert s == s2 and abs(ld - ld2) < 1e-12


@pytest.mark.parametrize("seed,aniso", [(0, True), (1, False), (2, True)])
def test_cholesky_route_matches_bruteforce(seed, aniso):
    pr = _prob(seed=seed, aniso=aniso)
    out, beta = oracle.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, pr.lam, return_beta=True)
    ll_bf, beta_bf = oracle.profile_loglik_bruteforce(pr.locs, pr.y, pr.X, pr.omega, pr.lam)
    np.testing.assert_allclose(out["loglik"], ll_bf, rtol=1e-10, atol=1e-9)
    np.testing.assert_allclose(beta, beta_bf, rtol=1e-8, atol=1e-9)


def test_gls_normal_equations():
    pr = _prob(n=40, p=3, seed=3)
    out, beta = oracle.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, pr.lam, return_beta=True)
    for k in range(pr.K):
        V = oracle.build_V(pr.locs, pr.omega[k])
        Vi_X = np.linalg.solve(V, pr.X)
        for m, lam in enumerate(pr.lam):
            yt = oracle.boxcox(pr.y, lam)
            lhs = pr.X.T @ Vi_X @ beta[k, m]
            rhs = Vi_X.T @ yt
            np.testing.assert_allclose(lhs, rhs, rtol=1e-9, atol=1e-9)


def test_profile_is_maximum_over_beta_and_sigma():
    pr = _prob(n=35, p=2, K=2, M=2, seed=4)
    out, beta = oracle.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, pr.lam, return_beta=True)
    jac = float(np.sum(np.log(pr.y)))
    rng = np.random.default_rng(1)
    for k in range(pr.K):
        V = oracle.build_V(pr.locs, pr.omega[k])
        Vi = np.linalg.inv(V)
        _, ld = np.linalg.slogdet(V)
        for m, lam in enumerate(pr.lam):
            yt = oracle.boxcox(pr.y, lam)
            b, s2 = beta[k, m], out["sigma2_hat"][k, m]
            at_hat = oracle.full_loglik(b, s2, yt, pr.X, Vi, ld, lam, jac)
            assert abs(at_hat - out["loglik"][k, m]) < 1e-9 * abs(at_hat)
            for _ in range(5):
                db = 1e-3 * rng.standard_normal(pr.p)
                assert oracle.full_loglik(b + db, s2, yt, pr.X, Vi, ld, lam, jac) < at_hat
            # d l / d sigma^2 = 0 at sigma-hat^2 (central difference)
            h = 1e-6 * s2
            g = (oracle.full_loglik(b, s2 + h, yt, pr.X, Vi, ld, lam, jac)
                 - oracle.full_loglik(b, s2 - h, yt, pr.X, Vi, ld, lam, jac)) / (2 * h)
            assert abs(g) < 1e-4 * pr.n / s2


def test_range_to_zero_closed_form():
    # range -> 0: R = I, V = (1 + nu^2) I; l_p follows from ordinary least squares
    pr = _prob(n=50, p=3, K=1, M=2, seed=5)
    nug = 0.3
    om = np.array([[1e-9, 1.3, nug, 1.0, 0.0]])
    out = oracle.profile_loglik(pr.locs, pr.y, pr.X, om, pr.lam)
    n = pr.n
    for m, lam in enumerate(pr.lam):
        yt = oracle.boxcox(pr.y, lam)
        b, *_ = np.linalg.lstsq(pr.X, yt, rcond=None)
        rss = float(np.sum((yt - pr.X @ b) ** 2))
        ssr = rss / (1 + nug)
        ll = (-0.5 * (n * math.log(ssr / n) + n * math.log(1 + nug) + n * math.log(2 * math.pi) + n)
              + (lam - 1) * np.sum(np.log(pr.y)))
        assert abs(out["loglik"][0, m] - ll) < 1e-10 * abs(ll)
        assert abs(out["logdet_v"][0, m] - n * math.log(1 + nug)) < 1e-10 * n


def test_boxcox_special_cases():
    y = np.array([0.01, 0.5, 1.0, 2.0, 37.0])
    np.testing.assert_allclose(oracle.boxcox(y, 1.0), y - 1.0, rtol=1e-15, atol=1e-16)
    np.testing.assert_allclose(oracle.boxcox(y, 0.0), np.log(y), rtol=1e-15)
    np.testing.assert_allclose(oracle.boxcox(y, 1e-10), np.log(y), rtol=1e-9)
    np.testing.assert_allclose(oracle.boxcox(y, -1.0), 1.0 - 1.0 / y, rtol=1e-14)
    with pytest.raises(ValueError):
        oracle.boxcox(np.array([1.0, 0.0]), 0.5)


def test_lambda_one_is_shift_invariant():
    # with an intercept, l_p(lambda=1) does not change when y is shifted
    pr = _prob(n=30, p=2, K=3, M=1, seed=6)
    a = oracle.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, [1.0])
    b = oracle.profile_loglik(pr.locs, pr.y + 5.0, pr.X, pr.omega, [1.0])
    np.testing.assert_allclose(a["loglik"], b["loglik"], rtol=1e-11)


def test_lambda_zero_scale_jacobian():
    # lambda = 0: y -> c y shifts y' by log c (absorbed by the intercept) and
    # the Jacobian term (lambda - 1) sum log y by -n log c
    pr = _prob(n=30, p=2, K=3, M=1, seed=7)
    c = 3.7
    a = oracle.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, [0.0])
    b = oracle.profile_loglik(pr.locs, c * pr.y, pr.X, pr.omega, [0.0])
    np.testing.assert_allclose(b["loglik"], a["loglik"] - pr.n * math.log(c), rtol=1e-11)


def test_ssq_identities():
    # Step 8: ssqResidual = ssqY - ssqBetahat; Table tab:tocpu components
    pr = _prob(n=40, p=3, seed=8)
    out = oracle.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, pr.lam)
    np.testing.assert_allclose(out["ssq_resid"], out["ssq_y"] - out["ssq_betahat"], rtol=1e-9)
    k = 1
    V = oracle.build_V(pr.locs, pr.omega[k])
    _, ld = np.linalg.slogdet(V)
    _, ldx = np.linalg.slogdet(pr.X.T @ np.linalg.solve(V, pr.X))
    assert abs(out["logdet_v"][k, 0] - ld) < 1e-10 * abs(ld)
    assert abs(out["logdet_xvx"][k, 0] - ldx) < 1e-9 * max(1, abs(ldx))


def test_reml_against_contrast_likelihood():
    # REML via an explicit error contrast A (orthonormal rows with A X = 0):
    # -2 l* = (n-p) log(q/(n-p)) + log|A V A^T| + (n-p) log 2 pi + n - p - 2(lam-1)J.
    # Searle: |A V A^T| = |V| |X^T V^-1 X| / |X^T X|, so the paper's form differs by
    # -0.5 log|X^T X| - 0.5 p log 2 pi, the same for every omega.
    pr = _prob(n=30, p=3, K=3, M=2, seed=9)
    out = oracle.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, pr.lam)
    n, p = pr.n, pr.p
    Qf, _ = np.linalg.qr(pr.X, mode="complete")
    A = Qf[:, p:].T
    jac = float(np.sum(np.log(pr.y)))
    _, ldxx = np.linalg.slogdet(pr.X.T @ pr.X)
    for k in range(pr.K):
        V = oracle.build_V(pr.locs, pr.omega[k])
        AVA = A @ V @ A.T
        _, ld = np.linalg.slogdet(AVA)
        for m, lam in enumerate(pr.lam):
            ys = A @ oracle.boxcox(pr.y, lam)
            q = float(ys @ np.linalg.solve(AVA, ys))
            ll = -0.5 * ((n - p) * math.log(q / (n - p)) + ld + (n - p) * math.log(2 * math.pi)
                         + n - p) + (lam - 1) * jac
            diff = out["loglik_reml"][k, m] - ll
            assert abs(diff - (-0.5 * ldxx - 0.5 * p * math.log(2 * math.pi))) < 1e-9 * abs(ll)


def test_non_pd_point_reports_info():
    pr = _prob(n=20, p=2, K=1, M=2, seed=10)
    locs = pr.locs.copy()
    locs[5] = locs[4]                       # duplicate location, nugget 0 -> singular V
    om = np.array([[2.0, 2.0, 0.0, 1.0, 0.0]])
    out = oracle.profile_loglik(locs, pr.y, pr.X, om, pr.lam)
    assert np.all(out["info"] > 0) and np.all(out["loglik"] == -np.inf)


def _golden():
    rows = {}
    with open(os.path.join(HERE, "golden", "swiss_soil_params.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                name, *vals = line.split()
                rows[name] = [float(v) for v in vals]
    return rows


def test_parameter_conventions_from_paper_tables():
    # The printed combined range sqrt(phi_X phi_Y) equals phi_X / sqrt(phi_R) within the
    # rounding of the printed ratio: phi_Y = phi_X / phi_R, which aniso_ranges encodes.
    # The printed tau equals sigma * sqrt(nu^2): nu^2 is the nugget relative to sigma^2,
    # as in V = R + nu^2 I.
    for name, (rng_, comb, ratio, sigma, nug, tau, *_angle_gammas) in _golden().items():
        lo = hi = None
        for r in (ratio - 0.005, ratio + 0.005):
            phi_x, phi_y = oracle.aniso_ranges([rng_, 1.0, nug, r, 0.0])
            c = math.sqrt(phi_x * phi_y)
            lo = c if lo is None else min(lo, c)
            hi = c if hi is None else max(hi, c)
        assert lo - 0.01 <= comb <= hi + 0.01, (name, lo, hi, comb)
        taus = [sigma * math.sqrt(v) for v in (nug - 0.005, nug + 0.005)]
        assert min(taus) - 0.01 <= tau <= max(taus) + 0.01, (name, taus, tau)


def test_rotation_and_isotropy_invariance():
    pr = _prob(n=25, p=2, seed=11)
    om = np.array([1.3, 1.7, 0.1, 2.5, 0.4])
    theta = 0.9
    rot = np.array([[math.cos(theta), -math.sin(theta)], [math.sin(theta), math.cos(theta)]])
    V1 = oracle.build_V(pr.locs, om)
    om2 = om.copy()
    om2[4] -= theta
    V2 = oracle.build_V(pr.locs @ rot.T, om2)
    np.testing.assert_allclose(V1, V2, rtol=1e-12, atol=1e-14)
    iso = om.copy()
    iso[3] = 1.0
    Va = oracle.build_V(pr.locs, iso)
    iso[4] = 2.2
    np.testing.assert_allclose(Va, oracle.build_V(pr.locs, iso), rtol=1e-13, atol=1e-15)
