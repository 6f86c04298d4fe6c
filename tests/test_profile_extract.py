"""Step 4 profile extraction (pl_profile_param, host code) and its oracle:
upper convex hull of the point cloud, interpolation, likelihood interval."""
import ctypes

import numpy as np
import pytest

import paper_2305_04318_amd as pl
from oracle.extract import point_cloud, profile, upper_hull
from paper_2305_04318_amd import _lib

Z975 = 1.959963984540054   # chi^2_1 0.95 quantile = 1.95996^2 = 3.8415; c/2 = 1.92


def _records(ll, info=None):
    """(K, M) loglik -> host pl_result array."""
    K, M = ll.shape
    arr = (_lib.PlResult * (K * M))()
    for k in range(K):
        for m in range(M):
            r = arr[k * M + m]
            r.loglik = ll[k, m]
            r.info = 0 if info is None else int(info[k, m])
    return arr


def _lib_profile(ll, omega, lam, which, drop=1.92, info=None):
    K, M = ll.shape
    arr = _records(ll, info)
    om = np.ascontiguousarray(omega, dtype=np.float64)
    lm = np.ascontiguousarray(lam, dtype=np.float64)
    cx, cy = np.empty(max(K, M)), np.empty(max(K, M))
    n = ctypes.c_int64(0)
    iv = np.empty(3)
    op = ctypes.c_int32(0)
    P = ctypes.c_void_p
    rc = pl.load().pl_profile_param(arr, K, M, om.ctypes.data_as(P), lm.ctypes.data_as(P), which,
                                    drop, cx.ctypes.data_as(P), cy.ctypes.data_as(P),
                                    ctypes.byref(n), iv.ctypes.data_as(P), ctypes.byref(op))
    assert rc == 0
    return cx[:n.value], cy[:n.value], iv, op.value


def test_oracle_hull_of_concave_points_with_interior_noise():
    rng = np.random.default_rng(1)
    xs = np.linspace(-3, 3, 41)
    top = -0.5 * xs ** 2
    xi = rng.uniform(-3, 3, 200)
    yi = -0.5 * xi ** 2 - rng.uniform(0.01, 2.0, 200)
    x = np.concatenate([xs, xi])
    y = np.concatenate([top, yi])
    order = np.argsort(x)
    h = upper_hull(x[order], y[order])
    np.testing.assert_allclose(x[order][h], xs)


def test_oracle_interval_of_a_quadratic_profile_is_the_normal_quantile():
    """A profile exactly quadratic in theta with curvature 1/s^2 has the
    likelihood interval theta0 +- z_0.975 s; the densely sampled hull recovers
    it to the chord error."""
    theta0, s = 1.3, 0.4
    th = np.linspace(theta0 - 5 * s, theta0 + 5 * s, 2001)
    ll = (-0.5 * ((th - theta0) / s) ** 2)[:, None] + np.array([[0.0, -3.0]])  # M = 2
    om = np.zeros((th.size, 5))
    om[:, 1] = th
    # drop = z^2 / 2 exactly (the paper's 1.92 is this value rounded)
    x, y, am, lo, hi, op = profile(ll, np.ones_like(ll, bool), om, np.array([0.0, 1.0]), 1,
                                   drop=Z975 ** 2 / 2)
    assert op == 0 and abs(am - theta0) <= th[1] - th[0]
    # chord error of the sampled parabola: (h^2/8)/s^2 in l, over slope z/s
    assert abs(lo - (theta0 - Z975 * s)) < 1e-6 and abs(hi - (theta0 + Z975 * s)) < 1e-6


def test_library_matches_oracle_on_random_clouds():
    rng = np.random.default_rng(2)
    for trial in range(20):
        K, M = int(rng.integers(5, 120)), int(rng.integers(1, 6))
        om = rng.uniform(0.1, 5.0, (K, 5))
        om[rng.integers(0, K, K // 4), 1] = 1.5          # repeated abscissae
        ll = -rng.gamma(2.0, 3.0, (K, M)) - 100.0
        info = np.where(rng.random((K, M)) < 0.05, 3, 0)  # some unusable records
        lam = np.linspace(-0.5, 1.0, M)
        for which in range(6):
            if which == 5 and M < 2:
                continue
            cx, cy, iv, op = _lib_profile(ll, om, lam, which, 1.92, info)
            ox, oy, am, lo, hi, oop = profile(ll, info == 0, om, lam, which)
            np.testing.assert_array_equal(cx, ox)
            np.testing.assert_array_equal(cy, oy)
            assert iv[0] == am and op == oop
            np.testing.assert_allclose([iv[1], iv[2]], [lo, hi], rtol=1e-13, atol=1e-13)


def test_open_ends_and_lambda_interpolation():
    K, M = 3, 5
    lam = np.linspace(0, 1, M)
    ll = np.tile(-(lam - 1.0) ** 2 * 10.0, (K, 1))   # increasing in lambda: open on the right
    om = np.ones((K, 5))
    cx, cy, iv, op = _lib_profile(ll, om, lam, 5)
    np.testing.assert_array_equal(cx, lam)
    assert iv[0] == 1.0 and iv[2] == 1.0 and op == 2
    # the curve is -10 (lambda - 1)^2 at the vertices: -2.5 at 0.5, -0.625 at
    # 0.75; the threshold -1.92 is crossed between them
    want_lo = 0.75 - (-0.625 + 1.92) / (-0.625 + 2.5) * 0.25
    assert abs(iv[1] - want_lo) < 1e-12


def test_argument_errors():
    lib = pl.load()
    P = ctypes.c_void_p
    arr = _records(np.zeros((2, 2)))
    om = np.zeros((2, 5))
    buf = np.zeros(4)
    n = ctypes.c_int64(0)

    def call(rec=arr, K=2, M=2, omega=om, which=0, drop=1.92, cx=buf, npts=True):
        return lib.pl_profile_param(rec, K, M, omega.ctypes.data_as(P) if omega is not None else None,
                                    buf.ctypes.data_as(P), which, drop,
                                    cx.ctypes.data_as(P) if cx is not None else None,
                                    buf.ctypes.data_as(P), ctypes.byref(n) if npts else None,
                                    buf.ctypes.data_as(P), None)
    assert call(rec=None) == -1
    assert call(K=0) == -2 and call(M=0) == -3
    assert call(omega=None) == -4
    assert call(which=6) == -6 and call(drop=0.0) == -7
    assert call(cx=None) == -8 and call(npts=False) == -10
