"""Seeded synthetic inputs for the profile-likelihood path.

This module is shared by the oracle's tests and by the GPU path's tests and
benchmark.  It generates locations, covariates, positive observations and
parameter sets; it contains none of the likelihood arithmetic (no Box-Cox
forward transform, no Matern correlation, no Bessel function, no
factorisation).

Gaussian fields are drawn by random Fourier features: a stationary field with
spectral density proportional to (8*kappa + |w|^2)^-(kappa+1) in the scaled
coordinates has the Matern correlation of the paper's parametrisation
(Section 2.1, the equation defining rho with argument sqrt(8 kappa) d).  That
density is a bivariate Student-t with 2*kappa degrees of freedom and scale 2,
so frequencies are w = 2 z / sqrt(g / (2 kappa)) with z ~ N(0, I_2) and
g ~ chi^2(2 kappa).  The field is then sqrt(2/F) sum_f cos(w_f . A s + b_f)
with A = diag(1/phi_X, 1/phi_Y) Rot(phi_A) the anisotropy map of the same
equation.  Observations are y' = X beta + sigma (U + nu eps) (the model of
equation (1)) mapped back to the positive scale by the inverse Box-Cox map.

Seeds follow numpy's PCG64 fed by SeedSequence([2305, 4318, cfg, rep]).

Parameter vectors omega are rows (range phi_X, shape kappa, nugget nu^2,
anisotropy ratio phi_R, angle phi_A) with phi_Y = phi_X / phi_R.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np

N_FEATURES = 2048


def rng_for(cfg: int, rep: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([2305, 4318, cfg, rep])))


@dataclass
class Problem:
    """One dataset plus the (omega, lambda) points to evaluate."""
    locs: np.ndarray          # (n, 2) float64
    y: np.ndarray             # (n,) float64, > 0
    X: np.ndarray             # (n, p) float64
    omega: np.ndarray         # (K, 5) float64 natural parameters
    lam: np.ndarray           # (M,) float64 Box-Cox values
    truth: dict = field(default_factory=dict)
    name: str = ""

    @property
    def n(self) -> int:
        return self.locs.shape[0]

    @property
    def p(self) -> int:
        return self.X.shape[1]

    @property
    def K(self) -> int:
        return self.omega.shape[0]

    @property
    def M(self) -> int:
        return self.lam.shape[0]


def _aniso_map(phi_x: float, ratio: float, angle: float) -> np.ndarray:
    phi_y = phi_x / ratio
    c, s = math.cos(angle), math.sin(angle)
    rot = np.array([[c, -s], [s, c]])
    return np.diag([1.0 / phi_x, 1.0 / phi_y]) @ rot


def field_draws(rng, kappa, n_features=N_FEATURES):
    """Random frequencies and phases of one random-Fourier-feature field
    (see module docstring); drawn in the order z, g, b."""
    z = rng.standard_normal((n_features, 2))
    g = rng.chisquare(2.0 * kappa, size=n_features)
    w = 2.0 * z / np.sqrt(g / (2.0 * kappa))[:, None]
    b = rng.uniform(0.0, 2.0 * math.pi, size=n_features)
    return w, b


def field_eval(locs, A, w, b):
    """sqrt(2/F) sum_f cos(w_f . A s + b_f) at every location."""
    scaled = locs @ A.T                       # (n, 2) scaled coordinates
    return math.sqrt(2.0 / w.shape[0]) * np.cos(scaled @ w.T + b).sum(axis=1)


def gaussian_field(rng, locs, phi_x, kappa, ratio=1.0, angle=0.0, n_features=N_FEATURES):
    """Zero-mean, unit-variance stationary field with (approximately) Matern
    correlation, drawn by random Fourier features (see module docstring)."""
    A = _aniso_map(phi_x, ratio, angle)
    w, b = field_draws(rng, kappa, n_features)
    return field_eval(locs, A, w, b)


def inverse_boxcox(yt, lam, floor=0.01):
    """Map transformed values back to positive observations."""
    if lam == 0.0:
        return np.exp(yt)
    base = np.maximum(1.0 + lam * yt, floor)
    return base ** (1.0 / lam)


def _finish_obs(u, eps, X, beta, sigma, nugget, lam_true):
    yt = X @ np.asarray(beta) + sigma * (u + math.sqrt(nugget) * eps)
    floored = int(np.sum(1.0 + lam_true * yt <= 0.01)) if lam_true != 0.0 else 0
    return inverse_boxcox(yt, lam_true), floored


def simulate(rng, locs, X, beta, sigma, phi_x, kappa, nugget, ratio, angle, lam_true):
    u = gaussian_field(rng, locs, phi_x, kappa, ratio, angle)
    eps = rng.standard_normal(locs.shape[0])
    return _finish_obs(u, eps, X, beta, sigma, nugget, lam_true)


def omega_box(rng, K, range_lo=0.5, range_hi=4.5, ratio_lo=1.0, ratio_hi=6.0,
              nug_lo=0.02, nug_hi=1.0, kappa_lo=0.2, kappa_hi=10.0):
    """K parameter points: log-uniform range/ratio/nugget, uniform shape/angle."""
    om = np.empty((K, 5))
    om[:, 0] = np.exp(rng.uniform(math.log(range_lo), math.log(range_hi), K))
    om[:, 1] = rng.uniform(kappa_lo, kappa_hi, K)
    om[:, 2] = np.exp(rng.uniform(math.log(nug_lo), math.log(nug_hi), K))
    om[:, 3] = np.exp(rng.uniform(math.log(ratio_lo), math.log(ratio_hi), K))
    om[:, 4] = rng.uniform(0.0, math.pi, K)
    return om


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

def config_iso_grid(rep: int = 0) -> Problem:
    """n=200 on [0,1]^2, X=[1, x], field range 0.2, shape 1.5, nugget 0.1,
    y = exp(y'); 4x4x4 grid over (range, shape, nugget), lambda in {0, .5, 1}."""
    rng = rng_for(1, rep)
    n = 200
    locs = rng.uniform(0.0, 1.0, (n, 2))
    X = np.column_stack([np.ones(n), locs[:, 0]])
    y, _ = simulate(rng, locs, X, (1.0, 0.5), 1.0, 0.2, 1.5, 0.1, 1.0, 0.0, 0.0)
    ranges = np.linspace(0.05, 0.5, 4)
    shapes = np.array([0.5, 1.5, 2.5, 4.5])
    nuggets = np.linspace(0.01, 0.5, 4)
    grid = np.array([(r, k, v, 1.0, 0.0) for r in ranges for k in shapes for v in nuggets])
    return Problem(locs, y, X, grid, np.array([0.0, 0.5, 1.0]),
                   truth=dict(range=0.2, shape=1.5, nugget=0.1, lam=0.0), name="iso-grid n=200")


def config_aniso(n: int = 2000, K: int = 1024, M: int = 8, rep: int = 0, cfg: int = 2) -> Problem:
    """n locations on [0,10]^2, X = [1, z1, z2, z3], beta=(1,.5,-.3,.2); field
    range 1.5, shape 1.0, nugget 0.2, ratio 2, angle pi/6; lambda_true=0.5;
    K omega points from the box around the truth; M lambdas on [0, 1]."""
    rng = rng_for(cfg, rep)
    locs = rng.uniform(0.0, 10.0, (n, 2))
    X = np.column_stack([np.ones(n), rng.standard_normal((n, 3))])
    y, floored = simulate(rng, locs, X, (1.0, 0.5, -0.3, 0.2), 1.0, 1.5, 1.0, 0.2,
                          2.0, math.pi / 6.0, 0.5)
    om = omega_box(rng, K)
    lam = np.linspace(0.0, 1.0, M)
    return Problem(locs, y, X, om, lam,
                   truth=dict(range=1.5, shape=1.0, nugget=0.2, ratio=2.0,
                              angle=math.pi / 6, lam=0.5, floored=floored),
                   name=f"aniso n={n} K={K} M={M}")


def config_mixed(n: int = 4000, K: int = 256, M: int = 8, rep: int = 0) -> Problem:
    """The anisotropic generator at n=4000, K=256, M=8."""
    return config_aniso(n=n, K=K, M=M, rep=rep, cfg=3)


def config_uneven(n_datasets: int = 2048, k_per: int = 16, rep: int = 0,
                  n_lo: int = 100, n_hi: int = 1500):
    """Independent isotropic datasets of uneven size n ~ U{n_lo..n_hi} on
    [0,5]^2, X=[1, z], shape in {0.5, 1.5, 3}, range U[0.2, 1], nugget 0.1,
    y = exp(y'), 16 omega points jittered around each truth, lambda in {0,1}."""
    rng = rng_for(4, rep)
    # all random draws in sequence (the same order as simulate), then the
    # field sums, which dominate the cost, on a thread pool
    drawn = []
    for _ in range(n_datasets):
        n = int(rng.integers(n_lo, n_hi + 1))
        locs = rng.uniform(0.0, 5.0, (n, 2))
        X = np.column_stack([np.ones(n), rng.standard_normal(n)])
        kap = float(rng.choice([0.5, 1.5, 3.0]))
        rng_ = float(rng.uniform(0.2, 1.0))
        w, b = field_draws(rng, kap)
        eps = rng.standard_normal(n)
        om = np.empty((k_per, 5))
        om[:, 0] = rng_ * np.exp(rng.uniform(-0.7, 0.7, k_per))
        om[:, 1] = kap * np.exp(rng.uniform(-0.7, 0.7, k_per))
        om[:, 2] = 0.1 * np.exp(rng.uniform(-1.0, 1.0, k_per))
        om[:, 3] = 1.0
        om[:, 4] = 0.0
        drawn.append((locs, X, kap, rng_, w, b, eps, om))

    def make(d):
        locs, X, kap, rng_, w, b, eps, om = d
        u = field_eval(locs, _aniso_map(rng_, 1.0, 0.0), w, b)
        y, _ = _finish_obs(u, eps, X, (1.0, 0.5), 1.0, 0.1, 0.0)
        return Problem(locs, y, X, om, np.array([0.0, 1.0]),
                       truth=dict(range=rng_, shape=kap, nugget=0.1, lam=0.0),
                       name=f"uneven n={locs.shape[0]}")

    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as pool:
        return list(pool.map(make, drawn))


def serving_requests(duration_s: float = 30.0, rate: float = 20.0, rep: int = 0,
                     n_lo: int = 500, n_hi: int = 8000, k_lo: int = 32, k_hi: int = 200, M: int = 4):
    """Poisson arrival times plus a lazily generated anisotropic dataset per
    request: n log-uniform on [n_lo, n_hi], K ~ U{k_lo..k_hi}, M lambdas."""
    rng = rng_for(5, rep)
    t, arrivals = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration_s:
            break
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        K = int(rng.integers(k_lo, k_hi + 1))
        seed = int(rng.integers(0, 2**31 - 1))
        arrivals.append((t, n, K, seed))
    return arrivals


def serving_problem(n: int, K: int, seed: int, M: int = 4) -> Problem:
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([2305, 4318, 5, seed])))
    locs = rng.uniform(0.0, 10.0, (n, 2))
    X = np.column_stack([np.ones(n), rng.standard_normal((n, 3))])
    y, _ = simulate(rng, locs, X, (1.0, 0.5, -0.3, 0.2), 1.0, 1.5, 1.0, 0.2,
                    2.0, math.pi / 6.0, 0.5)
    om = omega_box(rng, K)
    return Problem(locs, y, X, om, np.linspace(0.0, 1.0, M), name=f"serve n={n} K={K}")


def small_problem(n: int, p: int = 2, K: int = 6, M: int = 3, seed: int = 0,
                  aniso: bool = True, extent: float = 5.0, kappas=None) -> Problem:
    """A small seeded problem for parity tests; omega from a box scaled to the
    domain, optionally with fixed shape values."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([2305, 4318, 99, seed, n, p])))
    locs = rng.uniform(0.0, extent, (n, 2))
    X = np.column_stack([np.ones(n), rng.standard_normal((n, p - 1))]) if p > 1 else np.ones((n, 1))
    beta = np.concatenate([[1.0], 0.3 * rng.standard_normal(p - 1)])
    y, _ = simulate(rng, locs, X, beta, 1.0, 0.3 * extent, 1.2, 0.2,
                    1.8 if aniso else 1.0, 0.4 if aniso else 0.0, 0.0)
    om = omega_box(rng, K, range_lo=0.05 * extent, range_hi=0.6 * extent,
                   ratio_lo=1.0, ratio_hi=4.0 if aniso else 1.0)
    if not aniso:
        om[:, 3] = 1.0
        om[:, 4] = 0.0
    if kappas is not None:
        om[:, 1] = np.resize(np.asarray(kappas, dtype=float), K)
    lam = np.linspace(-0.25, 1.0, M) if M > 1 else np.array([0.5])
    return Problem(locs, y, X, om, lam, name=f"small n={n} p={p} K={K} M={M}")
