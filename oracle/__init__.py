"""Plain FP64 CPU oracle for the profile log-likelihood of a Box-Cox
transformed Gaussian geostatistical model with anisotropic Matern correlation.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The GPU library does
not use it, shares no code with it, and must never fall back to it.

Every function is written from the paper's statement of the method:
  * Box-Cox transform (Section 2, first display),
  * the model Y' ~ MVN(X beta, sigma^2 V), V = R + nu^2 I (equation (1)),
  * the Matern correlation with geometric anisotropy (Section 2.1),
  * the log-likelihood (equation (2)), the closed-form beta-hat and sigma-hat^2
    (the two displays after it) and the profile log-likelihood (equation
    "profile"), plus the sufficient statistics of Table "tab:tocpu" and the
    Step 3 sub-steps (Section 3.3),
  * the restricted (REML) profile log-likelihood of the Appendix,
  * the profile curves of sigma and of single regression coefficients
    (Sections 3.4 and 3.5, the profile likelihoods for beta_p and for sigma).

Readings of points where the paper is garbled or silent are listed in the
project's design notes; the ones that change arithmetic are repeated where
they are used (normalising constant 2^(1-kappa)/Gamma(kappa); kappa=0.5 gives
exp(-2d) under the sqrt(8 kappa) scaling; phi_Y = phi_X / phi_R).

Pins (tests/test_oracle_*.py): three independent Bessel-K routes (SciPy's
Amos library, trapezoid quadrature of an integral representation, mpmath at
high precision), the terminating closed forms at half-integer order, the
three-term recurrence and Wronskian, a brute-force Gauss-Jordan/LU route for
the likelihood on small n, the GLS normal equations, maximality of the
profile in (beta, sigma^2), the range->0 closed form, Box-Cox special cases,
and the Swiss-rainfall parameter table printed in the paper.
"""
from .bessel import log_kv, kv_quadrature_log, matern_halfint, log_matern
from .model import boxcox, scaled_distance, matern_corr, build_V, aniso_ranges
from .likelihood import (profile_loglik, profile_point, full_loglik,
                         profile_loglik_bruteforce, RESULT_FIELDS)
from .curves import cross_products, curves

__all__ = [
    "log_kv", "kv_quadrature_log", "matern_halfint", "log_matern",
    "boxcox", "scaled_distance", "matern_corr", "build_V", "aniso_ranges",
    "profile_loglik", "profile_point", "full_loglik", "profile_loglik_bruteforce",
    "RESULT_FIELDS", "cross_products", "curves",
]
