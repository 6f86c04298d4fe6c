"""Modified Bessel function of the second kind, K_nu, three ways.

The Matern correlation of Section 2.1 needs K_kappa(t) for real kappa > 0 and
t > 0.  The oracle evaluates it in log space because K_kappa(t) overflows FP64
at small t and large kappa while the normalised product t^kappa K_kappa(t)
stays bounded.

Routes (independent of one another and of the GPU library):
  1. log_kv: SciPy's exponentially scaled kve (Amos' algorithm), log K = log kve - t.
     Where kve overflows, the quadrature route below is used instead.
  2. kv_quadrature_log: the trapezoid rule applied to the integral
     K_nu(t) = int_0^inf exp(-t cosh u) cosh(nu u) du (DLMF 10.32.9).  The
     integrand is even and analytic, so the trapezoid sum over the whole line
     converges geometrically in the step.
  3. matern_halfint: for kappa = m + 1/2 the series for K_{m+1/2} terminates
     (DLMF 10.49.12), giving rho(t) = exp(-t) m!/(2m)! sum_{i=0}^m
     (m+i)!/(i!(m-i)!) (2t)^(m-i).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special


def log_kv(nu, t):
    """log K_nu(t) elementwise for t > 0 (array-valued)."""
    nu = np.asarray(nu, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    nu_b, t_b = np.broadcast_arrays(nu, t)
    with np.errstate(over="ignore", divide="ignore"):
        kve = special.kve(nu_b, t_b)
        out = np.log(kve) - t_b
    bad = ~np.isfinite(out)
    if np.any(bad):
        idx = np.flatnonzero(bad)
        flat = out.reshape(-1)
        nf, tf = nu_b.reshape(-1), t_b.reshape(-1)
        for i in idx:
            flat[i] = kv_quadrature_log(float(nf[i]), float(tf[i]))
        out = flat.reshape(out.shape)
    return out


def kv_quadrature_log(nu: float, t: float) -> float:
    """log K_nu(t) by the trapezoid rule on DLMF 10.32.9, in log space.

    The log-integrand f(u) = -t (cosh u - 1) + log cosh(nu u) has its peak
    where t sinh u = nu tanh(nu u); its width is about 1/sqrt(max(nu, t, 1)),
    so a step of a quarter of that width puts the discretisation error far
    below double precision.  The sum is truncated once f drops 60 below its
    maximum.  Returns log K_nu(t) = -t + log(sum).
    """
    if t <= 0.0:
        raise ValueError("t must be positive")
    nu = abs(nu)
    h = 0.25 / math.sqrt(max(nu, t, 1.0))

    def f(u):
        # log cosh(nu u) written to avoid overflow
        a = nu * u
        # cosh u - 1 = 2 sinh^2(u/2) keeps precision near u = 0
        return -2.0 * t * np.sinh(0.5 * u) ** 2 + a + np.log1p(np.exp(-2.0 * a)) - math.log(2.0)

    # locate the peak: f'(u) = -t sinh u + nu tanh(nu u)
    if nu == 0.0:
        u_star = 0.0
    else:
        lo, hi = 0.0, max(1.0, math.asinh(nu / t) + 1.0)
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if -t * math.sinh(mid) + nu * math.tanh(nu * mid) > 0.0:
                lo = mid
            else:
                hi = mid
        u_star = 0.5 * (lo + hi)
    f_star = float(f(np.array([u_star]))[0])
    # extend the grid until the integrand is negligible
    u_end = u_star + 1.0
    while float(f(np.array([u_end]))[0]) > f_star - 60.0:
        u_end = u_star + 2.0 * (u_end - u_star)
    k = np.arange(0, int(math.ceil(u_end / h)) + 1, dtype=np.float64)
    vals = f(k * h)
    w = np.ones_like(vals)
    w[0] = 0.5
    m = vals.max()
    s = np.sum(w * np.exp(vals - m))
    return -t + m + math.log(s * h)


def log_matern(kappa, t):
    """log rho(t) = (1-kappa) log 2 - lgamma(kappa) + kappa log t + log K_kappa(t).

    Uses the normalising constant 2^(1-kappa)/Gamma(kappa), the only value
    for which rho(0) = 1 (the paper prints 2^(kappa-1); see the reading in the
    design notes).  t = 0 returns log rho = 0.
    """
    kappa = np.asarray(kappa, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    k_b, t_b = np.broadcast_arrays(kappa, t)
    out = np.zeros(k_b.shape)
    pos = t_b > 1e-300
    if np.any(pos):
        kk, tt = k_b[pos], t_b[pos]
        out[pos] = ((1.0 - kk) * math.log(2.0) - special.gammaln(kk)
                    + kk * np.log(tt) + log_kv(kk, tt))
    return np.minimum(out, 0.0)


def matern_halfint(m: int, t):
    """rho(t) for kappa = m + 1/2 from the terminating series (DLMF 10.49.12)."""
    t = np.asarray(t, dtype=np.float64)
    total = np.zeros_like(t)
    for i in range(m + 1):
        coef = math.factorial(m + i) / (math.factorial(i) * math.factorial(m - i))
        total = total + coef * (2.0 * t) ** (m - i)
    return np.exp(-t) * total * math.factorial(m) / math.factorial(2 * m)
