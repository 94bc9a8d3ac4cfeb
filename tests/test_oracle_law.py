"""Law of the oracle's field samples against dense Cholesky sampling.

Section 2.1, eq. (sample-from-Z): a sample of the grid field is Theta xi
for any factor R = Theta Theta^T of the grid covariance matrix.  The dense
Cholesky factor of R (built from the covariance function alone, none of
the embedding code) with independent normals from numpy's generator gives
reference samples; the oracle's circulant-embedding samples (Philox
normals, the DFT, the restriction) must have the same law.  Checked on
tiny grids by two-sample Kolmogorov-Smirnov tests on fixed random
projections, by whitening (L^-1 Z must be standard normal with identity
covariance) and, in PAIR mode, by the independence of the two fields of
one complex xi.  Deterministic seeds; the bars are several standard errors
wide at the sample sizes used.
"""

import numpy as np
import pytest
from scipy import stats

from oracle import sampler
from oracle.covariance import MATERN, SEPEXP, covariance

N = 6000   # samples per law


def grid_cov(kind, nu, lam, sigma2, m):
    h = 1.0 / m
    i = np.arange(m + 1) * h
    x1, x2 = np.meshgrid(i, i, indexing="xy")   # node (i1, i2) at row i2
    x1, x2 = x1.ravel(), x2.ravel()
    return covariance(kind, nu, lam, sigma2)(x1[:, None] - x1[None, :], x2[:, None] - x2[None, :])


CASES = [
    dict(cov=MATERN, nu=1.0, lam=0.3, sigma2=1.0, m=4, field_mode=0),        # PAIR, J = 0
    dict(cov=SEPEXP, nu=0.5, lam=0.3, sigma2=2.0, m=4, field_mode=1),        # HARTLEY
    dict(cov=MATERN, nu=1.5, lam=0.4, sigma2=1.0, m=4, field_mode=0),        # padded (J > 0)
]


def ce_samples(d, seed=11):
    p = sampler.Plan(dict(d, level=sampler.SINGLE))
    return np.array([p.fields(seed, i)[0].ravel() for i in range(N)]), p


@pytest.mark.parametrize("d", CASES, ids=["matern1-pair", "sepexp-hartley", "matern15-padded"])
def test_field_law_matches_dense_cholesky(d):
    R = grid_cov(d["cov"], d["nu"], d["lam"], d["sigma2"], d["m"])
    L = np.linalg.cholesky(R)
    z_ce, plan = ce_samples(d)
    if d is CASES[2]:
        assert plan.J > 0, "the case is meant to exercise the periodised embedding"
    rng = np.random.default_rng(2024)
    z_ch = (L @ rng.standard_normal((R.shape[0], N))).T
    # (1) one-dimensional laws along fixed random directions
    dirs = rng.standard_normal((16, R.shape[0]))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    for w in dirs:
        p = stats.ks_2samp(z_ce @ w, z_ch @ w).pvalue
        assert p > 1e-4, p
    # (2) whitened: standard normal coordinates with identity covariance
    wz = np.linalg.solve(L, z_ce.T).T
    C = wz.T @ wz / N
    assert np.max(np.abs(C - np.eye(C.shape[0]))) <= 6.0 / np.sqrt(N)
    assert np.max(np.abs(wz.mean(axis=0))) <= 5.0 / np.sqrt(N)
    assert stats.kstest(wz.ravel()[: 20 * N], "norm").pvalue > 1e-4


def test_pair_fields_of_one_xi_are_independent():
    d = CASES[0]
    z, _ = ce_samples(d, seed=5)
    a, b = z[0::2], z[1::2]          # Re v and Im v of the same xi
    n = a.shape[0]
    cross = (a - a.mean(0)).T @ (b - b.mean(0)) / n
    scale = np.sqrt(np.outer(a.var(0), b.var(0)))
    assert np.max(np.abs(cross / scale)) <= 5.0 / np.sqrt(n)
