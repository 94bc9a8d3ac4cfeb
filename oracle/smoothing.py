"""Smoothing parameter rule and smoothing-error statistic (oracle; test
infrastructure only).

Section 3.5: the number tau of eigenvalues to drop on a mesh h = 1/m is
chosen so that the smoothing error bound equals the discretisation error
C_alpha h^alpha.  With c = C_s / C_alpha and s = n^2 = 4 (m + J)^2:

* separable exponential (Corollary error-1-norm-cov, no padding, J = 0):
  eq. (k-values-p-norm-cov), tau = (s + 1) / ((c / 2^alpha) s^(alpha/2) + 1);
* Matern (Corollary error-matern-cov, s with the padding J): tau solves
  eq. (tau-values-matern),
  (s - tau + 1)^(-(1 + nu)/2) tau = (2 / c) h^(alpha + 1) (1/h + J),
  found here with scipy's Brent root finder on [0, s] (s when the right
  side is at least s, the value of the left side at tau = s).

The integer count is the root rounded to the nearest integer.

Section 4.1: the smoothing error of one mesh is Q_h - Q~_h with both terms
computed from the same normals (the same realisation of the field): Q_h
with every eigenvalue kept, Q~_h with tau dropped.  smoothing_error
returns the sample mean, mean absolute value and variance of the
differences and the two sample means, over samples first .. first+count-1.

Pins (tests/test_oracle_smoothing.py): the separable exponential closed
form satisfies the balance C_alpha h^alpha = C_s tau / (s - tau + 1) it
comes from; the Matern root balances C_alpha h^alpha against C_s times the
bound of Corollary (error-matern-cov) evaluated in its general
d-dimensional form (s = 2^d prod (m_i + J_i), exponent -(1 + 2 nu/d)/2),
and the embedding's sorted eigenvalues decay at the rate j^-(1 + nu) that
exponent rests on; the root lies in [0, s];
tau decreases as C_s / C_alpha grows and tends to s as it vanishes; tau = 0
gives identically zero differences; tau = s gives Q~_h equal to the
constant-coefficient QoI (k = exp(0) = 1) for every sample; the statistics
equal numpy's on the per-sample differences.
"""

import math

import numpy as np
from scipy import optimize

from . import fem, qoi, sampler

SEPEXP = 1
MATERN = 0


def tau_rule(cov, m, alpha, cs_over_calpha, nu=0.5, J=0):
    """(tau rounded to the nearest integer, real root)."""
    if m < 1 or J < 0 or alpha <= 0 or cs_over_calpha <= 0:
        raise ValueError("m >= 1, J >= 0, alpha > 0 and C_s / C_alpha > 0 required")
    s = 4.0 * (m + J) ** 2
    c = cs_over_calpha
    if cov == SEPEXP:
        if J != 0:
            raise ValueError("the separable exponential rule assumes no padding")
        t = (s + 1.0) / (c / 2.0 ** alpha * s ** (alpha / 2.0) + 1.0)
    else:
        h = 1.0 / m
        rhs = 2.0 / c * h ** (alpha + 1.0) * (1.0 / h + J)
        p = 0.5 * (1.0 + nu)

        def g(t):
            return (s - t + 1.0) ** (-p) * t - rhs

        t = s if g(s) <= 0 else optimize.brentq(g, 0.0, s, xtol=1e-13, rtol=1e-15, maxiter=500)
    t = min(max(t, 0.0), s)
    return int(math.floor(t + 0.5)), t


def smoothing_error(desc, tau, seed, first, count):
    """Statistics of Q_h - Q~_h for a single-level descriptor (its tau_f
    is replaced by 0 for Q_h and by tau for Q~_h)."""
    d_full = dict(desc, level=sampler.SINGLE, tau_f=0, tau_c=0)
    d_sm = dict(desc, level=sampler.SINGLE, tau_f=tau, tau_c=tau)
    pf, ps = sampler.Plan(d_full), sampler.Plan(d_sm)
    q = np.array([pf.sample(seed, first + i)[1] for i in range(count)])
    qs = np.array([ps.sample(seed, first + i)[1] for i in range(count)])
    d = q - qs
    return {"n": count, "mean": float(np.mean(d)), "mean_abs": float(np.mean(np.abs(d))),
            "var": float(np.var(d, ddof=1)), "mean_q": float(np.mean(q)), "mean_q_smoothed": float(np.mean(qs)),
            "diff": d, "q": q, "q_smoothed": qs}


def constant_coefficient_qoi(desc):
    """QoI of the solve with k = 1 (a zero field), for the tau = s pin."""
    m = desc["m"]
    k = np.ones((m + 1, m + 1))
    u, A, b = fem.solve(k, m, desc.get("bc", fem.DIRICHLET0), desc.get("f", 1.0))
    return qoi.evaluate(desc.get("qoi", qoi.INTEGRAL), u, m, A, b, desc.get("qx", 7.0 / 15.0),
                        desc.get("qy", 7.0 / 15.0))
