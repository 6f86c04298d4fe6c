"""Profile log-likelihood, per (omega, lambda), in plain FP64.

Cholesky route (the timed oracle): Section 3.3's Step 3 in the paper's order,
with LAPACK's textbook dpotrf/dtrtrs as steps:
  1. V = R(omega) + nu^2 I                                    (Step 1)
  2. V = L L^T, log|V| = 2 sum log L_ii                        (Step 2; the paper
     uses L D L^T, which has the same determinant)
  3. Z = L^{-1} [Y'_1 .. Y'_M | X]                             (Step 3)
  4. ssqYX = Z^T Z, i.e. (y, X)^T V^{-1} (y, X)                (Step 4)
  5. X^T V^{-1} X = Q Q^T, log|X^T V^{-1} X|                   (Step 5)
  6. c = Q^{-1} X^T V^{-1} y                                   (Step 6)
  7. ssqBetahat = c^T c                                        (Step 7)
  8. ssqResidual = y^T V^{-1} y - ssqBetahat                   (Step 8)
then beta-hat = Q^{-T} c (equation "betahat"), sigma-hat^2 = SSR/n (the
display after it) and
  -2 l_p = n log(SSR/n) + log|V| - 2 (lambda - 1) sum log y + n log(2 pi) + n
(equation "profile"); the routine returns l_p itself.  The REML form of the
Appendix (equation "remlpro") is returned beside it.

Brute-force route (pins the Cholesky route on small n): Gauss-Jordan inverse
and LU determinant written out, then equation (2) evaluated at the closed-form
(beta-hat, sigma-hat^2).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import lapack, solve_triangular

from .model import boxcox, build_V

LOG2PI = math.log(2.0 * math.pi)

RESULT_FIELDS = ("loglik", "logdet_v", "logdet_xvx", "ssq_y", "ssq_betahat",
                 "ssq_resid", "sigma2_hat", "jacobian", "loglik_reml", "info")


def _empty_records(M):
    rec = {f: np.full(M, np.nan) for f in RESULT_FIELDS}
    rec["info"] = np.zeros(M, dtype=np.int64)
    return rec


def profile_point(V, Yt, X, lam, jac):
    """All records for one omega given V (n x n), the transformed columns
    Yt (n x M), X (n x p), the M lambdas and J = sum log y."""
    n, p = X.shape
    M = Yt.shape[1]
    rec = _empty_records(M)
    beta = np.full((M, p), np.nan)
    c_fac, info = lapack.dpotrf(V, lower=1, clean=1)
    if info != 0:
        rec["info"][:] = info
        rec["loglik"][:] = -np.inf
        rec["loglik_reml"][:] = -np.inf
        rec["jacobian"][:] = jac
        return rec, beta
    L = c_fac
    logdet_v = 2.0 * np.sum(np.log(np.diag(L)))
    B = np.column_stack([Yt, X])
    Z = solve_triangular(L, B, lower=True)
    ZY, ZX = Z[:, :M], Z[:, M:]
    A = ZX.T @ ZX                                   # X^T V^-1 X
    Bxy = ZX.T @ ZY                                 # X^T V^-1 y'   (p x M)
    s = np.sum(ZY * ZY, axis=0)                     # y'^T V^-1 y'  (diagonal)
    Q, qinfo = lapack.dpotrf(A, lower=1, clean=1)
    if qinfo != 0:
        rec["info"][:] = -1                          # rank-deficient X^T V^-1 X
        rec["logdet_v"][:] = logdet_v
        rec["jacobian"][:] = jac
        return rec, beta
    logdet_xvx = 2.0 * np.sum(np.log(np.diag(Q)))
    C = solve_triangular(Q, Bxy, lower=True)         # c = Q^-1 X^T V^-1 y'
    ssq_bh = np.sum(C * C, axis=0)
    bh = solve_triangular(Q.T, C, lower=False)       # beta-hat = Q^-T c
    # residual quadratic form computed directly, (y' - X b)^T V^-1 (y' - X b)
    R = ZY - ZX @ bh
    ssr = np.sum(R * R, axis=0)
    sig2 = ssr / n
    lam = np.asarray(lam, dtype=np.float64)
    ll = -0.5 * (n * np.log(sig2) + logdet_v + n * LOG2PI + n) + (lam - 1.0) * jac
    ll_reml = -0.5 * ((n - p) * np.log(ssr / (n - p)) + logdet_v + logdet_xvx
                      + n * LOG2PI + n - p) + (lam - 1.0) * jac
    rec.update(loglik=ll, logdet_v=np.full(M, logdet_v), logdet_xvx=np.full(M, logdet_xvx),
               ssq_y=s, ssq_betahat=ssq_bh, ssq_resid=ssr, sigma2_hat=sig2,
               jacobian=np.full(M, jac), loglik_reml=ll_reml)
    return rec, bh.T


def transformed_columns(y, lam):
    return np.column_stack([boxcox(y, float(l)) for l in lam])


def profile_loglik(locs, y, X, omega, lam, return_beta=False):
    """Records for every (omega_k, lambda_m): dict of (K, M) arrays, and
    optionally beta-hat as (K, M, p)."""
    locs = np.asarray(locs, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    omega = np.atleast_2d(np.asarray(omega, dtype=np.float64))
    lam = np.atleast_1d(np.asarray(lam, dtype=np.float64))
    K, M, p = omega.shape[0], lam.shape[0], X.shape[1]
    jac = float(np.sum(np.log(y)))
    Yt = transformed_columns(y, lam)
    out = {f: np.empty((K, M), dtype=np.int64 if f == "info" else np.float64) for f in RESULT_FIELDS}
    betas = np.empty((K, M, p))
    for k in range(K):
        V = build_V(locs, omega[k])
        rec, bh = profile_point(V, Yt, X, lam, jac)
        for f in RESULT_FIELDS:
            out[f][k] = rec[f]
        betas[k] = bh
    if return_beta:
        return out, betas
    return out


# --------------------------------------------------------------------------
# Brute-force route (small n only)
# --------------------------------------------------------------------------

def gauss_jordan_inverse(A):
    """Inverse by Gauss-Jordan elimination with partial pivoting."""
    A = np.array(A, dtype=np.float64)
    n = A.shape[0]
    aug = np.hstack([A, np.eye(n)])
    for col in range(n):
        piv = col + int(np.argmax(np.abs(aug[col:, col])))
        if aug[piv, col] == 0.0:
            raise np.linalg.LinAlgError("singular")
        if piv != col:
            aug[[col, piv]] = aug[[piv, col]]
        aug[col] /= aug[col, col]
        for r in range(n):
            if r != col:
                aug[r] -= aug[r, col] * aug[col]
    return aug[:, n:]


def lu_logdet(A):
    """(sign, log|det A|) by Doolittle LU with partial pivoting."""
    U = np.array(A, dtype=np.float64)
    n = U.shape[0]
    sign = 1.0
    logdet = 0.0
    for col in range(n):
        piv = col + int(np.argmax(np.abs(U[col:, col])))
        if U[piv, col] == 0.0:
            return 0.0, -np.inf
        if piv != col:
            U[[col, piv]] = U[[piv, col]]
            sign = -sign
        d = U[col, col]
        sign *= math.copysign(1.0, d)
        logdet += math.log(abs(d))
        U[col + 1:, col:] -= np.outer(U[col + 1:, col] / d, U[col, col:])
    return sign, logdet


def full_loglik(beta, sigma2, yt, X, Vinv, logdet_v, lam, jac):
    """Equation (2): -2 l = (y'-X b)^T (s2 V)^-1 (y'-X b) + log|s2 V|
    - 2 (lam - 1) sum log y + n log 2 pi; returns l."""
    n = X.shape[0]
    r = yt - X @ beta
    q = float(r @ Vinv @ r) / sigma2
    m2l = q + n * math.log(sigma2) + logdet_v - 2.0 * (lam - 1.0) * jac + n * LOG2PI
    return -0.5 * m2l


def profile_loglik_bruteforce(locs, y, X, omega, lam):
    """l_p(omega_k, lambda_m) through an explicit inverse and determinant:
    beta-hat = (X^T V^-1 X)^-1 X^T V^-1 y', sigma-hat^2 = r^T V^-1 r / n, then
    equation (2) at those values.  Returns (ll (K, M), beta (K, M, p))."""
    omega = np.atleast_2d(omega)
    lam = np.atleast_1d(lam)
    n, p = X.shape
    jac = float(np.sum(np.log(y)))
    ll = np.empty((omega.shape[0], lam.shape[0]))
    betas = np.empty((omega.shape[0], lam.shape[0], p))
    for k, om in enumerate(omega):
        V = build_V(locs, om)
        Vinv = gauss_jordan_inverse(V)
        sgn, logdet = lu_logdet(V)
        if sgn <= 0:
            raise np.linalg.LinAlgError("V not positive definite")
        XtVi = X.T @ Vinv
        G = gauss_jordan_inverse(XtVi @ X)
        for m, l in enumerate(lam):
            yt = boxcox(y, float(l))
            b = G @ (XtVi @ yt)
            r = yt - X @ b
            s2 = float(r @ Vinv @ r) / n
            ll[k, m] = full_loglik(b, s2, yt, X, Vinv, logdet, float(l), jac)
            betas[k, m] = b
    return ll, betas
