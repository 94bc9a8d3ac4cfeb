"""Adaptive MLMC estimator over level samples (test infrastructure).

Section 3.3: the MLMC estimator is the sum over levels of the sample mean
of Y_l (eq. (mlmc-estimator); with smoothing eq. (mlmc-estimator-smoothed),
where the finest level uses the unsmoothed fine field).  Sample sizes follow
eq. (optimal-nl): N_l = ceil(2 eps^-2 (sum_k sqrt(C_k V_k)) sqrt(V_l / C_l)),
written here with the variance share theta of eps^2 (theta = 1/2 gives the
factor 2).  Section 4: the bias |E[Q_h - Q]| is estimated by Richardson
extrapolation with extrapolant Q_2h, |E[Y_L]| / (2^alpha - 1), and alpha,
beta, gamma are the slopes of the best linear fits of log2 |E[Y_l]|,
log2 V[Y_l], log2 C_l against l.  The paper names the adaptive choice of
the number of levels without spelling it out; the loop here is: sample
what is missing, recompute N_l, and once no level lacks samples, stop if
the squared bias estimate is within (1 - theta) eps^2, else add a level.
Section 3.5: the coarsest-mesh rules h_0 <= lambda (separable exponential,
eq. (mlmc-h0-bound-exp-covariance)) and h_0 <= sqrt(8 nu) lambda (Matern,
eq. (mlmc-h0-bound-matern-covariance)).

Pins (tests/test_oracle_mlmc.py): hand-computed sample sizes, exact fits on
exact data, the Richardson formula on a constructed sequence, the variance
recursion against numpy, and a statistical run on synthetic levels with
known means and variances.
"""

import math

import numpy as np


def optimal_samples(var, cost, eps, theta=0.5):
    """Eq. (optimal-nl) with the variance budget theta eps^2."""
    s = sum(math.sqrt(v * c) for v, c in zip(var, cost))
    return [max(2, math.ceil(s * math.sqrt(v / c) / (theta * eps * eps))) for v, c in zip(var, cost)]


def fit_slope(ls, values):
    """Least-squares slope of values against ls."""
    x = np.asarray(ls, dtype=float)
    y = np.asarray(values, dtype=float)
    n = len(x)
    den = n * np.sum(x * x) - np.sum(x) ** 2
    return float((n * np.sum(x * y) - np.sum(x) * np.sum(y)) / den) if den != 0 else 0.0


def richardson_bias(mean_finest, alpha):
    """|E[Q_h - Q]| from E[Q_h - Q_2h] (Section 4)."""
    return abs(mean_finest) / (2.0 ** alpha - 1.0)


def coarsest_mesh(cov, nu, lam):
    """m_0 = 1/h_0 with h_0 = 2^-k the largest with the Section 3.5 bound."""
    hmax = lam if cov == "sepexp" else math.sqrt(8.0 * nu) * lam
    m = 1
    while 1.0 / m > hmax:
        m *= 2
    return m


class RunningStats:
    """Mean and variance of a stream of numbers taken in order."""

    def __init__(self):
        self.n = 0
        self.mean = 0.0
        self.m2 = 0.0

    def add(self, y):
        self.n += 1
        d = y - self.mean
        self.mean += d / self.n
        self.m2 += d * (y - self.mean)

    def var(self):
        return self.m2 / (self.n - 1) if self.n > 1 else 0.0


def run(sample, cost, nlevels, eps, l_start=2, n_pilot=100, theta=0.5, alpha=0.0, max_rounds=50,
        finest_differs=False):
    """Adaptive MLMC.  sample(l, finest, first, count) returns the Y values
    of level l (finest: sampled in its finest-level form) for sample
    indices first .. first+count-1; cost[l] is the cost of one sample."""
    L = min(l_start, nlevels - 1)
    stats = [RunningStats() for _ in range(nlevels)]
    want = [0] * nlevels
    nxt = [0] * nlevels
    for l in range(L + 1):
        want[l] = n_pilot
    a, b, g, bias, varsum, converged, rounds = alpha, 0.0, 0.0, 0.0, 0.0, False, 0
    while rounds < max_rounds:
        for l in range(L + 1):
            c = want[l] - stats[l].n
            if c > 0:
                for y in sample(l, finest_differs and l == L, nxt[l], c):
                    stats[l].add(float(y))
                nxt[l] += c
        rounds += 1
        var = [stats[l].var() for l in range(L + 1)]
        nl = optimal_samples(var, cost[:L + 1], eps, theta)
        more = False
        for l in range(L + 1):
            want[l] = max(nl[l], stats[l].n)
            more = more or want[l] > stats[l].n
        ls = list(range(1, L + 1))
        if len(ls) >= 2:
            if alpha <= 0:
                a = max(0.5, -fit_slope(ls, [math.log2(max(abs(stats[l].mean), 1e-300)) for l in ls]))
            b = -fit_slope(ls, [math.log2(max(stats[l].var(), 1e-300)) for l in ls])
            g = fit_slope(ls, [math.log2(cost[l]) for l in ls])
        elif alpha <= 0:
            a = 1.0
        varsum = sum(stats[l].var() / stats[l].n for l in range(L + 1))
        bias = richardson_bias(stats[L].mean, a) if L >= 1 else 0.0
        if more:
            continue
        if L >= 1 and bias * bias <= (1 - theta) * eps * eps:
            converged = True
            break
        # a level is added only when a round is left to sample it, so that
        # every level of the result has samples
        if L + 1 >= nlevels or rounds >= max_rounds:
            break
        if finest_differs:
            stats[L] = RunningStats()
            nxt[L] = 0
            want[L] = n_pilot
        L += 1
        want[L] = n_pilot
    return {"estimate": sum(stats[l].mean for l in range(L + 1)), "variance": varsum, "bias": bias,
            "alpha": a, "beta": b, "gamma": g, "levels": L + 1, "converged": converged, "rounds": rounds,
            "n": [stats[l].n for l in range(L + 1)], "mean": [stats[l].mean for l in range(L + 1)],
            "var": [stats[l].var() for l in range(L + 1)]}


def unknowns(m, bc="dirichlet0"):
    """Unknowns of the mesh with m intervals per side (the cost model)."""
    return (m - 1) * ((m + 1) if bc == "flowcell" else (m - 1))
