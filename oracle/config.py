"""Representative parameter points of Step 2, FP64.  TEST INFRASTRUCTURE ONLY
(see the package docstring).

Section 3.2, "Hessian matrix": the Hessian of l_p(omega', lambda_hat) in the
internal parameters omega' (oracle.mle), by numerical differentiation on
51 points for the five-dimensional case and 33 for the four-dimensional one
(shape held fixed), each at lambda_hat and lambda_hat +- delta -- the counts
51 x 3 and 33 x 3 the paper gives, which are those of the central-difference
stencil {centre, +-delta e_i, (+-delta e_i, +-delta e_j)}.  The lambda values
give the second derivative in lambda at the centre.

Eigen-repair: -H = E D E^T; negative eigenvalues become their absolute
values; when the largest exceeds 100 the small ones are raised to 0.1
(reading: every eigenvalue below 0.1).

"Obtaining representative points": unit-sphere points x are mapped to
  omega' = omega_hat' + sqrt(q) E D^(-1/2) x
(reading of the garbled printed map: with this form (omega' - omega_hat')^T
(-H) (omega' - omega_hat') = q, the ellipsoid of the quadratic
approximation), q the chi-square quantile with d degrees of freedom and
upper-tail probability alpha (the paper's definition of chi^2_p(alpha)).
Nugget repair: a point with nu < 0 has a negative nugget; half of them get
0 and half a uniform draw on (0, 2) (reading: alternately, in output order,
starting with 0; the draws are inputs).  Box-Cox grid: m values evenly
spaced between the 0.01 and 0.99 quantiles of the normal approximation
N(lambda_hat, 1/|d^2 l / d lambda^2|).

The spread of the unit-sphere points (a maximin design found by an
unspecified stochastic optimiser) has no oracle: parity unpinned; its tests
check properties only.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import stats

from .likelihood import profile_loglik
from .mle import from_internal, to_internal

MIN_SHAPE, MAX_SHAPE = 0.05, 100.0


def free_coords(fix_shape):
    return [0, 2, 3, 4] if fix_shape else [0, 1, 2, 3, 4]


def stencil(d):
    """Offsets (in units of delta) of the central-difference stencil."""
    pts = [np.zeros(d)]
    for i in range(d):
        for s in (1.0, -1.0):
            e = np.zeros(d)
            e[i] = s
            pts.append(e)
    for i in range(d):
        for j in range(i + 1, d):
            for si, sj in ((1, 1), (1, -1), (-1, 1), (-1, -1)):
                e = np.zeros(d)
                e[i], e[j] = si, sj
                pts.append(e)
    return np.array(pts)


def central_hessian(fvals, d, delta):
    """Hessian from f on stencil(d) (same order)."""
    f0 = fvals[0]
    H = np.empty((d, d))
    for i in range(d):
        H[i, i] = (fvals[1 + 2 * i] - 2.0 * f0 + fvals[2 + 2 * i]) / delta ** 2
    k = 1 + 2 * d
    for i in range(d):
        for j in range(i + 1, d):
            fpp, fpm, fmp, fmm = fvals[k:k + 4]
            H[i, j] = H[j, i] = (fpp - fpm - fmp + fmm) / (4.0 * delta ** 2)
            k += 4
    return H


def hessian_at(locs, y, X, omega_hat, lam_hat, shape_transform, fix_shape, delta):
    """(H, d^2 l / d lambda^2, l at the centre); the likelihood of a stencil
    point uses nugget nu^2 whatever the sign of nu."""
    idx = free_coords(fix_shape)
    d = len(idx)
    w0 = to_internal([omega_hat], shape_transform)[0]
    rows = []
    for off in stencil(d):
        w = w0.copy()
        w[idx] += delta * off
        w[2] = abs(w[2])
        om = from_internal([w], shape_transform)[0]
        if fix_shape:
            om[1] = omega_hat[1]
        rows.append(om)
    lam = [lam_hat - delta, lam_hat, lam_hat + delta]
    rec = profile_loglik(locs, y, X, np.array(rows), lam)
    ll = rec["loglik"]
    H = central_hessian(ll[:, 1], d, delta)
    curv = (ll[0, 0] - 2.0 * ll[0, 1] + ll[0, 2]) / delta ** 2
    return H, curv, ll[0, 1], np.array(rows)


def repair(H):
    """Eigen-decomposition of -H with the repair: (D, E), columns in the
    ascending order of the eigenvalues of -H before the repair, each column of
    E with its largest-magnitude entry positive."""
    A = -0.5 * (H + H.T)
    D, E = np.linalg.eigh(A)
    for j in range(E.shape[1]):
        if E[np.argmax(np.abs(E[:, j])), j] < 0:
            E[:, j] = -E[:, j]
    D = np.abs(D)
    if D.max() > 100.0:
        D = np.maximum(D, 0.1)
    return D, E


def chisq_upper(alpha, d):
    return float(stats.chi2.isf(alpha, d))


def config_points(omega_hat, shape_transform, fix_shape, H, alpha, sphere, uniforms):
    """(omega rows level-major, repaired eigenvalues ascending, number of
    repaired nuggets)."""
    idx = free_coords(fix_shape)
    d = len(idx)
    D, E = repair(np.asarray(H, dtype=np.float64))
    w0 = to_internal([omega_hat], shape_transform)[0]
    M = E @ np.diag(1.0 / np.sqrt(D))
    out = []
    negatives = 0
    t = 0
    for a in alpha:
        rq = math.sqrt(chisq_upper(a, d))
        for x in np.asarray(sphere, dtype=np.float64).reshape(-1, d):
            w = w0.copy()
            w[idx] += rq * (M @ x)
            nu, ks = w[2], w[1]
            w[2] = abs(nu)
            beyond = shape_transform == 1 and ks <= 0.0   # 1/sqrt(kappa) <= 0: kappa "infinite"
            if beyond:
                w[1] = 1.0                                # any valid value; replaced below
            om = from_internal([w], shape_transform)[0]
            if fix_shape:
                om[1] = omega_hat[1]
            elif beyond:
                om[1] = MAX_SHAPE
            else:
                om[1] = min(MAX_SHAPE, max(MIN_SHAPE, om[1]))
            if nu < 0.0:
                om[2] = 0.0 if negatives % 2 == 0 else 2.0 * uniforms[t]
                negatives += 1
            out.append(om)
            t += 1
    return np.array(out), np.sort(D), negatives


def lambda_grid(lam_hat, curv, m=30, tail=0.01):
    half = stats.norm.isf(tail) / math.sqrt(abs(curv))
    return np.linspace(lam_hat - half, lam_hat + half, m)
