"""Covariance functions of Section 2.1 (oracle; test infrastructure only).

* Matern, eq. (matern-cov-function): C(t) = sigma2 2^{1-nu}/Gamma(nu)
  x^nu K_nu(x) with x = sqrt(2 nu) |t|_2 / lambda, and C(0) = sigma2
  (the limit of x^nu K_nu(x) 2^{1-nu}/Gamma(nu) as x -> 0 is 1).
* Separable exponential, eq. (p-norm-cov-function) with p = 1:
  C(t) = sigma2 exp(-|t|_1 / lambda).

Pins (tests/test_oracle_covariance.py): the closed forms of the Matern
family at nu = 1/2 (sigma2 e^{-x}) and nu = 3/2 (sigma2 (1+x) e^{-x});
C(0) = sigma2; continuity at 0; nu = 1/2 Matern differs from the
separable exponential away from the axes.
"""

import numpy as np
from scipy.special import kv, gamma

MATERN = 0
SEPEXP = 1


def matern(t1, t2, nu, lam, sigma2):
    """Matern covariance at lag (t1, t2), eq. (matern-cov-function)."""
    t1 = np.asarray(t1, dtype=np.float64)
    t2 = np.asarray(t2, dtype=np.float64)
    r = np.sqrt(t1 * t1 + t2 * t2)
    x = np.sqrt(2.0 * nu) * r / lam
    out = np.full(np.broadcast(t1, t2).shape, float(sigma2))
    nz = x > 0
    xn = x[nz]
    out[nz] = sigma2 * 2.0 ** (1.0 - nu) / gamma(nu) * xn ** nu * kv(nu, xn)
    return out


def sepexp(t1, t2, lam, sigma2):
    """Separable exponential covariance, eq. (p-norm-cov-function), p = 1."""
    t1 = np.asarray(t1, dtype=np.float64)
    t2 = np.asarray(t2, dtype=np.float64)
    return sigma2 * np.exp(-(np.abs(t1) + np.abs(t2)) / lam)


def covariance(kind, nu, lam, sigma2):
    """Return C(t1, t2) for the descriptor fields (kind, nu, lambda, sigma2)."""
    if kind == MATERN:
        return lambda a, b: matern(a, b, nu, lam, sigma2)
    if kind == SEPEXP:
        return lambda a, b: sepexp(a, b, lam, sigma2)
    raise ValueError("unknown covariance kind %r" % (kind,))
