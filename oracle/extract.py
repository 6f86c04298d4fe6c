"""Univariate profile curves of the correlation parameters and of lambda from
evaluated points, and likelihood intervals.  TEST INFRASTRUCTURE ONLY (see the
package docstring).

Section 3.6, "Profile likelihood for correlation parameters": for parameter
theta the point cloud is (theta_k, max over lambda of l_p(omega_k, lambda));
the points on its upper convex hull are the best likelihoods and the profile
curve interpolates them linearly.  For lambda the curve interpolates
(lambda_m, max over omega of l_p).  Section 2's likelihood-based interval,
read as {theta : l_p(theta) >= max l_p - c/2} with c the chi^2_1 quantile.

The hull vertices are found point by point from the supporting-line
characterisation: with the points sorted by x, point i is a vertex exactly
when some line through it has every other point strictly below, i.e. when the
smallest slope from a point on its left exceeds the largest slope to a point
on its right (the two end points always qualify).
"""
from __future__ import annotations

import numpy as np


def point_cloud(loglik, info_ok, omega, lam, which):
    """(x, y) of the cloud; loglik and info_ok are (K, M)."""
    ll = np.where(info_ok, loglik, -np.inf)
    if which == 5:
        x, y = np.asarray(lam, dtype=float), ll.max(axis=0)
    else:
        x, y = np.asarray(omega, dtype=float)[:, which], ll.max(axis=1)
    keep = np.isfinite(y) & np.isfinite(x)
    x, y = x[keep], y[keep]
    # equal abscissae keep their largest value
    ux = np.unique(x)
    uy = np.array([y[x == v].max() for v in ux])
    return ux, uy


def upper_hull(x, y):
    """Indices of the upper-hull vertices of points sorted by distinct x."""
    n = x.shape[0]
    keep = []
    for i in range(n):
        left = (y[i] - y[:i]) / (x[i] - x[:i]) if i > 0 else np.array([np.inf])
        right = (y[i + 1:] - y[i]) / (x[i + 1:] - x[i]) if i < n - 1 else np.array([-np.inf])
        if left.min() > right.max():
            keep.append(i)
    return np.array(keep, dtype=int)


def profile(loglik, info_ok, omega, lam, which, drop=1.92):
    """(curve x, curve y, argmax, lower, upper, open bits)."""
    x, y = point_cloud(loglik, info_ok, omega, lam, which)
    if which != 5:
        h = upper_hull(x, y)
        x, y = x[h], y[h]
    im = int(np.argmax(y))
    thr = y[im] - drop
    lo, hi, open_ = x[0], x[-1], 3
    for i in range(im, 0, -1):
        if y[i - 1] < thr:
            lo = x[i] - (y[i] - thr) / (y[i] - y[i - 1]) * (x[i] - x[i - 1])
            open_ &= ~1
            break
    for i in range(im, x.shape[0] - 1):
        if y[i + 1] < thr:
            hi = x[i] + (y[i] - thr) / (y[i] - y[i + 1]) * (x[i + 1] - x[i])
            open_ &= ~2
            break
    return x, y, x[im], lo, hi, open_
