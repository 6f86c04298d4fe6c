"""Pins of the oracle's Bessel-K and Matern routines against mathematics that
does not go through them: an independent quadrature, mpmath at 40 digits,
terminating closed forms, the recurrence and the Wronskian."""
import math

import mpmath
import numpy as np
import pytest
from scipy import special

import oracle
from oracle.bessel import kv_quadrature_log, log_kv, log_matern, matern_halfint

NUS = [0.05, 0.2, 0.5, 1.0, 1.37, 2.5, 4.5, 9.7, 30.0]
TS = [1e-3, 0.1, 1.0, 2.0, 5.0, 20.0, 100.0, 600.0]


@pytest.mark.parametrize("nu", NUS)
def test_kv_scipy_vs_mpmath(nu):
    mpmath.mp.dps = 40
    for t in TS:
        ref = float(mpmath.log(mpmath.besselk(nu, t)))
        got = float(log_kv(nu, t))
        assert abs(got - ref) <= 1e-13 * max(1.0, abs(ref)), (nu, t, got, ref)


@pytest.mark.parametrize("nu", NUS)
def test_kv_quadrature_vs_mpmath(nu):
    mpmath.mp.dps = 40
    for t in TS:
        ref = float(mpmath.log(mpmath.besselk(nu, t)))
        got = kv_quadrature_log(nu, t)
        assert abs(got - ref) <= 1e-13 * max(1.0, abs(ref)), (nu, t, got, ref)


def test_kv_overflow_falls_back_to_log_space():
    # K_100(1e-3) ~ 1e485 overflows double; log K must stay finite and right
    mpmath.mp.dps = 40
    ref = float(mpmath.log(mpmath.besselk(100, mpmath.mpf("1e-3"))))
    got = float(log_kv(100.0, 1e-3))
    assert np.isfinite(got) and abs(got - ref) <= 1e-13 * abs(ref)


@pytest.mark.parametrize("m", [0, 1, 2, 3, 4])
def test_halfinteger_closed_forms(m):
    t = np.array([1e-6, 1e-3, 0.05, 0.7, 1.9, 2.1, 6.0, 35.0, 300.0])
    closed = matern_halfint(m, t)
    via_k = np.exp(log_matern(m + 0.5, t))
    # log-space evaluation: relative error grows like eps * |log rho| (~3e-14 at t=300)
    np.testing.assert_allclose(via_k, closed, rtol=1e-13, atol=1e-300)


def test_halfinteger_named_cases():
    t = np.linspace(0.0, 8.0, 41)
    np.testing.assert_allclose(matern_halfint(0, t), np.exp(-t), rtol=1e-15)
    np.testing.assert_allclose(matern_halfint(1, t), (1 + t) * np.exp(-t), rtol=1e-15)
    np.testing.assert_allclose(matern_halfint(2, t), (1 + t + t * t / 3) * np.exp(-t), rtol=1e-15)
    np.testing.assert_allclose(
        matern_halfint(4, t),
        (1 + t + 3 * t**2 / 7 + 2 * t**3 / 21 + t**4 / 105) * np.exp(-t), rtol=1e-14)


@pytest.mark.parametrize("nu", [0.3, 1.0, 2.75, 8.1])
def test_three_term_recurrence(nu):
    # K_{nu+1}(t) = K_{nu-1}(t) + (2 nu / t) K_nu(t)   (DLMF 10.29.1)
    for t in [0.01, 0.5, 3.0, 40.0]:
        lhs = math.exp(log_kv(nu + 1, t) - log_kv(nu, t))
        rhs = math.exp(log_kv(nu - 1, t) - log_kv(nu, t)) + 2 * nu / t
        assert abs(lhs - rhs) <= 1e-13 * abs(rhs)


@pytest.mark.parametrize("nu", [0.2, 1.5, 3.3])
def test_wronskian(nu):
    # I_nu K_{nu+1} + I_{nu+1} K_nu = 1/t   (DLMF 10.28.2)
    for t in [0.05, 1.0, 7.0, 30.0]:
        w = (special.iv(nu, t) * math.exp(log_kv(nu + 1, t))
             + special.iv(nu + 1, t) * math.exp(log_kv(nu, t)))
        assert abs(w * t - 1.0) <= 1e-13


def test_matern_at_zero_and_monotone():
    for kappa in [0.05, 0.2, 0.5, 1.0, 3.7, 10.0, 60.0]:
        d = np.array([0.0, 1e-250, 1e-8, 1e-3, 0.1, 0.5, 1.0, 3.0])
        r = oracle.matern_corr(d, kappa)
        # at t ~ 1e-250 the log-space terms are ~kappa*575 in size, so the
        # oracle is good to ~1e-12 there; monotone to that tolerance
        assert r[0] == 1.0 and abs(r[1] - 1.0) < 2e-12
        assert np.all(np.diff(r) <= 2e-12) and np.all(r > 0.0) and np.all(r <= 1.0)


def test_matern_shape_half_is_exp_minus_2d():
    # under the sqrt(8 kappa) scaling of Section 2.1, kappa = 1/2 gives exp(-2d)
    d = np.linspace(0.0, 5.0, 51)
    np.testing.assert_allclose(oracle.matern_corr(d, 0.5), np.exp(-2 * d), rtol=1e-15)


def test_matern_large_shape_tends_to_gaussian():
    # kappa -> infinity gives exp(-2 d^2) (Section 2.1)
    d = np.linspace(0.0, 1.5, 16)
    errs = [np.max(np.abs(oracle.matern_corr(d, k) - np.exp(-2 * d * d))) for k in (5.0, 20.0, 80.0)]
    assert errs[0] > errs[1] > errs[2] and errs[2] < 0.01
