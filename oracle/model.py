"""Box-Cox transform, anisotropic distance, Matern correlation and V.

Section 2 (Box-Cox display), Section 2.1 (Matern with geometric anisotropy)
and equation (1) (V = R + nu^2 I).
"""
from __future__ import annotations

import math

import numpy as np

from .bessel import log_matern


def boxcox(y, lam: float):
    """y' = (y^lam - 1)/lam for lam != 0 and log y for lam = 0 (Section 2).

    Written as expm1(lam log y)/lam, which is the same value without the
    cancellation of y^lam - 1 at small |lam|.  Requires y > 0.
    """
    y = np.asarray(y, dtype=np.float64)
    if np.any(~(y > 0.0)) or np.any(~np.isfinite(y)):
        raise ValueError("Box-Cox needs positive, finite observations")
    ly = np.log(y)
    if lam == 0.0:
        return ly
    return np.expm1(lam * ly) / lam


def aniso_ranges(omega):
    """(phi_X, phi_Y) from natural omega = (range, shape, nugget, ratio, angle).

    The fourth slot is the anisotropy ratio phi_R = phi_X / phi_Y; the
    paper's parameter tables (combined range = sqrt(phi_X phi_Y)) fix this
    convention.
    """
    phi_x = float(omega[0])
    return phi_x, phi_x / float(omega[3])


def scaled_distance(locs, omega):
    """d(s_i - s_j) = || diag(1/phi_X, 1/phi_Y) Rot(phi_A) (s_i - s_j) || for all
    pairs (Section 2.1).  The rotation matrix [[cos, -sin], [sin, cos]] is
    applied to the difference vector as printed."""
    locs = np.asarray(locs, dtype=np.float64)
    phi_x, phi_y = aniso_ranges(omega)
    a = float(omega[4])
    dx = locs[:, 0][:, None] - locs[:, 0][None, :]
    dy = locs[:, 1][:, None] - locs[:, 1][None, :]
    u1 = math.cos(a) * dx - math.sin(a) * dy
    u2 = math.sin(a) * dx + math.cos(a) * dy
    return np.sqrt((u1 / phi_x) ** 2 + (u2 / phi_y) ** 2)


def matern_corr(d, kappa: float):
    """rho = 2^(1-kappa)/Gamma(kappa) (sqrt(8 kappa) d)^kappa K_kappa(sqrt(8 kappa) d),
    with rho = 1 at d = 0 (Section 2.1)."""
    t = math.sqrt(8.0 * kappa) * np.asarray(d, dtype=np.float64)
    return np.exp(log_matern(kappa, t))


def build_V(locs, omega):
    """V = R(omega) + nu^2 I (equation (1) and the display before it)."""
    d = scaled_distance(locs, omega)
    R = matern_corr(d, float(omega[1]))
    n = R.shape[0]
    return R + float(omega[2]) * np.eye(n)
