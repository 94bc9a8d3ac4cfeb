"""Pins of oracle.field (Algorithm 1 step 4; Section 2.1; Theorem 1)."""

import math

import numpy as np
import pytest

from oracle import embedding as em, field as fd
from oracle.covariance import covariance, MATERN, SEPEXP


def grid_cov(cov, m):
    h = 1.0 / m
    i = np.arange(m + 1)
    X1, X2 = np.meshgrid(i * h, i * h, indexing="xy")
    x1, x2 = X1.ravel(), X2.ravel()
    return cov(x1[:, None] - x1[None, :], x2[:, None] - x2[None, :])


def linear_maps(a, m, mode):
    """Columns of the map xi -> restricted field for unit real xi."""
    n = a.shape[0]
    cols = []
    for j in range(n * n):
        e = np.zeros(n * n, dtype=complex)
        e[j] = 1.0
        v = fd.dft_plus(a * e.reshape(n, n))[: m + 1, : m + 1]
        cols.append((v.real.ravel(), v.imag.ravel()))
    A = np.stack([c[0] for c in cols], axis=1)
    B = np.stack([c[1] for c in cols], axis=1)
    return A, B


@pytest.mark.parametrize("kind,nu,lam,m,psd", [(SEPEXP, 0.5, 0.3, 4, 0), (MATERN, 1.0, 0.3, 4, 0),
                                               (MATERN, 1.5, 0.25, 6, 0)])
def test_sampler_covariance_identity(kind, nu, lam, m, psd):
    d = dict(cov=kind, nu=nu, lam=lam, sigma2=1.2, m=m, psd=psd)
    st = em.setup(d)
    assert st["n_clamped"] == 0 or st["lam_min"] >= -1e-13 * st["lam_max"]
    a = em.amplitudes(st["lam"])
    A, B = linear_maps(a, m, fd.PAIR)
    R = grid_cov(covariance(kind, nu, lam, 1.2), m)
    # PAIR: each of Re v, Im v has covariance A A^T + B B^T;
    np.testing.assert_allclose(A @ A.T + B @ B.T, R, atol=1e-13)
    # HARTLEY: Re v + Im v with real xi has covariance (A+B)(A+B)^T.
    np.testing.assert_allclose((A + B) @ (A + B).T, R, atol=1e-13)
    # Re v and Im v of one complex xi are uncorrelated: B A^T - A B^T = 0
    np.testing.assert_allclose(B @ A.T - A @ B.T, 0, atol=1e-13)


def test_smoothing_extremes():
    d = dict(cov=MATERN, nu=0.5, lam=0.1, sigma2=1.0, m=8)
    st = em.setup(d)
    lam = st["lam"]
    n = lam.shape[0]
    xi = fd.xi(3, 5, 0, n, fd.PAIR)
    z0 = fd.fields(em.amplitudes(lam), xi, 8, fd.PAIR)
    zt = fd.fields(em.amplitudes(lam, em.mask(lam, 0)), xi, 8, fd.PAIR)
    for a, b in zip(z0, zt):
        np.testing.assert_array_equal(a, b)
    zs = fd.fields(em.amplitudes(lam, em.mask(lam, n * n)), xi, 8, fd.PAIR)
    assert all(np.abs(z).max() == 0 for z in zs)


@pytest.mark.slow
def test_empirical_covariance_matches_matern():
    m = 8
    cov = covariance(MATERN, 1.0, 0.3, 1.0)
    st = em.setup(dict(cov=MATERN, nu=1.0, lam=0.3, sigma2=1.0, m=m))
    a = em.amplitudes(st["lam"])
    n = st["n"]
    zs = []
    for q in range(3000):
        zs.extend(fd.fields(a, fd.xi(11, q, 0, n, fd.PAIR), m, fd.PAIR))
    Z = np.stack([z.ravel() for z in zs])
    emp = Z.T @ Z / Z.shape[0]
    R = grid_cov(cov, m)
    N = Z.shape[0]
    se = np.sqrt((R ** 2 + np.outer(np.diag(R), np.diag(R))) / N)
    assert np.max(np.abs(emp - R) / se) < 6.0


@pytest.mark.slow
def test_theorem1_explicit_bound_hartley():
    # E||Z - Z~||_inf <= max|g_ij| sqrt(Lambda_ord[s-tau+1]) E sum|xi| with
    # |g_ij| <= sqrt(2/s) and E|xi| = sqrt(2/pi) (proof of Theorem 1).
    m = 16
    st = em.setup(dict(cov=MATERN, nu=0.5, lam=0.1, sigma2=1.0, m=m))
    lam = st["lam"]
    n = st["n"]
    s = n * n
    a = em.amplitudes(lam)
    order = np.sort(lam.ravel())[::-1]
    for tau in (32, 128, 512):
        at = em.amplitudes(lam, em.mask(lam, tau))
        errs = []
        for q in range(150):
            xi = fd.xi(21, q, 0, n, fd.HARTLEY)
            errs.append(np.abs(fd.fields(a, xi, m, fd.HARTLEY)[0]
                               - fd.fields(at, xi, m, fd.HARTLEY)[0]).max())
        bound = 2.0 / math.sqrt(math.pi * s) * math.sqrt(order[s - tau]) * tau
        assert np.mean(errs) < bound
        assert np.mean(errs) > 0


def test_dft_plus_matches_naive_definition():
    rng = np.random.default_rng(8)
    n = 6
    w = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    ref = np.zeros((n, n), dtype=complex)
    for p2 in range(n):
        for p1 in range(n):
            for j2 in range(n):
                for j1 in range(n):
                    ang = 2 * math.pi * (j1 * p1 + j2 * p2) / n
                    ref[p2, p1] += w[j2, j1] * complex(math.cos(ang), math.sin(ang))
    np.testing.assert_allclose(fd.dft_plus(w), ref, atol=1e-12)
