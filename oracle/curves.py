"""Profile curves of sigma and of single regression coefficients, FP64, from
the cross products of Table "tab:tocpu".  TEST INFRASTRUCTURE ONLY (see the
package docstring).

Section 3.4, "Profile likelihood for beta_p": with beta_j fixed at b the other
coefficients and sigma take their closed-form maximum-likelihood values, and
the residual quadratic form is assembled from rows and columns of ssqYX:
  (y' - X_j b)^T V^-1 (y' - X_j b)
      = y'^T V^-1 y' - 2 b (X^T V^-1 y')_j + b^2 (X^T V^-1 X)_jj,
  (X_-j bhat_-j)^T V^-1 (X_-j bhat_-j)
      = u^T G^-1 u,  u = (X^T V^-1 y')_-j - b (X^T V^-1 X)_-j,j,
                     G = (X^T V^-1 X)_-j,-j,
SSR(b) is the first minus the second; sigma-hat^2 = SSR(b)/n and the
likelihood is equation (2) at those values, i.e. equation "profile" with
SSR(b) in place of SSR.  Section 3.5, "Profile likelihood for sigma": beta at
its MLE, sigma fixed (equation "profileSigma").  Both curves are maximised
over the evaluated (omega_k, lambda_m), as in Step 6.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import lapack, solve_triangular

from .likelihood import transformed_columns
from .model import build_V

LOG2PI = math.log(2.0 * math.pi)


def cross_products(locs, y, X, omega, lam):
    """Per omega: ssqYX = [Y'_1..Y'_M | X]^T V^-1 [Y'_1..Y'_M | X] ((M+p) x
    (M+p)) and log|V| (Step 4 of Section 3.3), NaN for a non-PD V."""
    omega = np.atleast_2d(np.asarray(omega, dtype=np.float64))
    lam = np.atleast_1d(np.asarray(lam, dtype=np.float64))
    B = np.column_stack([transformed_columns(y, lam), X])
    q = B.shape[1]
    out = np.full((omega.shape[0], q, q), np.nan)
    ldv = np.full(omega.shape[0], np.nan)
    for k in range(omega.shape[0]):
        L, info = lapack.dpotrf(build_V(locs, omega[k]), lower=1, clean=1)
        if info != 0:
            continue
        Z = solve_triangular(L, B, lower=True)
        out[k] = Z.T @ Z
        ldv[k] = 2.0 * np.sum(np.log(np.diag(L)))
    return out, ldv


def ssr_fixed_coefficient(ssq, M, m, j, b):
    """SSR with coefficient j fixed at b, for lambda index m, from ssqYX by
    the subsetting identities above."""
    p = ssq.shape[0] - M
    yy = ssq[m, m]
    xy = ssq[M:, m]                  # X^T V^-1 y'_m
    xx = ssq[M:, M:]                 # X^T V^-1 X
    first = yy - 2.0 * b * xy[j] + b * b * xx[j, j]
    rest = [i for i in range(p) if i != j]
    if not rest:
        return first
    G = xx[np.ix_(rest, rest)]
    u = xy[rest] - b * xx[rest, j]
    second = u @ np.linalg.solve(G, u)
    return first - second


def curves(locs, y, X, omega, lam, sigma_grid, beta_grid, per_record=False):
    """(sigma curve (Gs,), its argmax records, beta curves (p, Gb), argmax)
    with records indexed k*M + m; -inf / -1 where nothing is usable.  With
    per_record, also every record's value: (Gs, K*M) and (p, Gb, K*M), -inf
    for unusable records."""
    n, p = X.shape
    lam = np.atleast_1d(np.asarray(lam, dtype=np.float64))
    M = lam.shape[0]
    J = float(np.sum(np.log(y)))
    ssq, ldv = cross_products(locs, y, X, omega, lam)
    K = ssq.shape[0]
    sigma_grid = np.asarray(sigma_grid, dtype=np.float64)
    beta_grid = np.atleast_2d(np.asarray(beta_grid, dtype=np.float64))
    sig = np.full(sigma_grid.shape[0], -np.inf)
    sig_arg = np.full(sigma_grid.shape[0], -1, dtype=np.int64)
    bet = np.full(beta_grid.shape, -np.inf)
    bet_arg = np.full(beta_grid.shape, -1, dtype=np.int64)
    sig_all = np.full((sigma_grid.shape[0], K * M), -np.inf)
    bet_all = np.full(beta_grid.shape + (K * M,), -np.inf)
    for k in range(K):
        if not np.isfinite(ldv[k]):
            continue
        xx = ssq[k][M:, M:]
        for m in range(M):
            xy = ssq[k][M:, m]
            bh = np.linalg.solve(xx, xy)
            ssr = ssq[k][m, m] - xy @ bh
            jt = (lam[m] - 1.0) * J
            r = k * M + m
            for g, s in enumerate(sigma_grid):
                v = -0.5 * (ssr / s ** 2 + n * math.log(s ** 2) + ldv[k] + n * LOG2PI) + jt
                sig_all[g, r] = v
                if v > sig[g]:
                    sig[g], sig_arg[g] = v, r
            for j in range(p):
                for g, b in enumerate(beta_grid[j]):
                    sb = ssr_fixed_coefficient(ssq[k], M, m, j, b)
                    v = -0.5 * (n * math.log(sb / n) + ldv[k] + n * LOG2PI + n) + jt
                    bet_all[j, g, r] = v
                    if v > bet[j, g]:
                        bet[j, g], bet_arg[j, g] = v, r
    if per_record:
        return sig, sig_arg, bet, bet_arg, sig_all, bet_all
    return sig, sig_arg, bet, bet_arg
