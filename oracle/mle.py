"""Internal parameters of Step 2 and checks of a maximum-likelihood estimate,
FP64.  TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 3.2, "Reparameterization": the internal parameters are
  omega' = (gamma1, kappa~, nu, gamma2, gamma3),
  gamma1 = log phi_X + log phi_Y,
  gamma2 = sqrt(phi_X/phi_Y - 1) cos(2 phi_A),
  gamma3 = sqrt(phi_X/phi_Y - 1) sin(2 phi_A),
  kappa~ = log kappa when kappa-hat < 4, 1/sqrt(kappa) otherwise,
  nu = sqrt(nu^2).
gamma2, gamma3 are real only for phi_X >= phi_Y.  Reading taken here: a
natural omega with phi_X < phi_Y is first written as the same model with the
axes exchanged -- phi_X' = phi_Y, phi_Y' = phi_X, phi_A' = phi_A + pi/2 -- which
gives the same scaled distance and so the same V.  The inverse follows from
the definitions: phi_X/phi_Y = 1 + gamma2^2 + gamma3^2, phi_X phi_Y =
exp(gamma1), 2 phi_A = the polar angle of (gamma2, gamma3).

Step 1 (Section 3.1) is the numerical maximisation of the profile likelihood
(equation "profile") over omega and lambda; the helpers below evaluate the
objective at given points, by the oracle's likelihood, so that a maximiser's
answer can be checked: its value, a brute-force grid it must beat, and the
absence of ascent around it.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from .likelihood import profile_loglik


def to_internal(omega, shape_transform=0):
    """Natural (K x 5: range phi_X, shape, nugget, ratio phi_X/phi_Y, angle)
    -> internal (K x 5: gamma1, kappa~, nu, gamma2, gamma3)."""
    om = np.atleast_2d(np.asarray(omega, dtype=np.float64))
    out = np.empty_like(om)
    for k, (phi_x, kappa, nugget, ratio, angle) in enumerate(om):
        phi_y = phi_x / ratio
        if phi_x < phi_y:  # exchange the axes
            phi_x, phi_y, angle = phi_y, phi_x, angle + math.pi / 2.0
        r = math.sqrt(phi_x / phi_y - 1.0)
        out[k, 0] = math.log(phi_x) + math.log(phi_y)
        out[k, 1] = math.log(kappa) if shape_transform == 0 else 1.0 / math.sqrt(kappa)
        out[k, 2] = math.sqrt(nugget)
        out[k, 3] = r * math.cos(2.0 * angle)
        out[k, 4] = r * math.sin(2.0 * angle)
    return out


def from_internal(internal, shape_transform=0):
    """Internal -> natural, with phi_X >= phi_Y and phi_A in (-pi/2, pi/2].
    A negative nu is returned as the negative nugget -nu^2 (points drawn
    from the quadratic approximation of Step 2 can land there)."""
    w = np.atleast_2d(np.asarray(internal, dtype=np.float64))
    out = np.empty_like(w)
    for k, (g1, ks, nu, g2, g3) in enumerate(w):
        ratio = 1.0 + g2 * g2 + g3 * g3          # phi_X / phi_Y
        # phi_X phi_Y = exp(g1) and phi_X = ratio phi_Y
        phi_y = math.sqrt(math.exp(g1) / ratio)
        out[k, 0] = ratio * phi_y
        out[k, 1] = math.exp(ks) if shape_transform == 0 else 1.0 / (ks * ks)
        out[k, 2] = math.copysign(nu * nu, nu)
        out[k, 3] = ratio
        out[k, 4] = 0.5 * math.atan2(g3, g2)
    return out


def objective(locs, y, X, omega, lam, reml=False):
    """Per omega_k: the largest (restricted) profile log-likelihood over the
    lambda values, -inf where no record is usable, and the lambda attaining
    it (NaN then)."""
    rec = profile_loglik(locs, y, X, omega, lam)
    ll = np.where(rec["info"] == 0, rec["loglik_reml" if reml else "loglik"], -np.inf)
    lam = np.atleast_1d(np.asarray(lam, dtype=np.float64))
    best = ll.max(axis=1)
    arg = np.where(np.isfinite(best), lam[np.argmax(ll, axis=1)], np.nan)
    return best, arg


def grid(center, half_widths, points):
    """Brute-force grid (natural omega rows) in the search coordinates
    (gamma1, log kappa, log nu^2, gamma2, gamma3): `points` evenly spaced
    values over center_i +- half_widths_i in every coordinate."""
    c = np.asarray(center, dtype=np.float64)
    axes = [np.linspace(c[i] - half_widths[i], c[i] + half_widths[i], points)
            if half_widths[i] > 0 else np.array([c[i]]) for i in range(5)]
    rows = []
    for g1, lk, ln2, g2, g3 in itertools.product(*axes):
        rows.append(from_search([g1, lk, ln2, g2, g3]))
    return np.array(rows)


def to_search(omega):
    """Natural omega -> (gamma1, log kappa, log nu^2, gamma2, gamma3)."""
    w = to_internal(omega, 0)[0]
    return np.array([w[0], w[1], 2.0 * math.log(w[2]), w[3], w[4]])


def from_search(s):
    """(gamma1, log kappa, log nu^2, gamma2, gamma3) -> natural omega."""
    return from_internal([[s[0], s[1], math.exp(0.5 * s[2]), s[3], s[4]]], 0)[0]


def ascent_around(locs, y, X, omega_hat, lam_hat, delta, reml=False, coords=range(5)):
    """Largest increase of the objective over the points omega_hat +- delta
    along each search coordinate in `coords` (lambda at lam_hat, lam_hat +-
    delta searched jointly) and lambda_hat +- delta at omega_hat; <= 0 at a
    local maximum that is resolved on the scale delta."""
    lam3 = [lam_hat - delta, lam_hat, lam_hat + delta]
    f0, _ = objective(locs, y, X, omega_hat, [lam_hat], reml)
    s = to_search(omega_hat)
    pts = []
    for i in coords:
        for sg in (-1.0, 1.0):
            t = s.copy()
            t[i] += sg * delta
            pts.append(from_search(t))
    f, _ = objective(locs, y, X, np.array(pts), lam3, reml)
    fl, _ = objective(locs, y, X, omega_hat, lam3, reml)
    return float(max(f.max(), fl.max()) - f0[0])
