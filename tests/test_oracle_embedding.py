"""Pins of oracle.embedding (Sections 2.1.2, 2.2, 2.4; Algorithms 1-2)."""

import math

import numpy as np
import pytest

from oracle import embedding as em
from oracle.covariance import covariance, MATERN, SEPEXP


def naive_dft_plus(s):
    n = s.shape[0]
    out = np.zeros((n, n), dtype=complex)
    for k2 in range(n):
        for k1 in range(n):
            acc = 0j
            for j2 in range(n):
                for j1 in range(n):
                    acc += s[j2, j1] * complex(math.cos(2 * math.pi * (j1 * k1 + j2 * k2) / n),
                                               math.sin(2 * math.pi * (j1 * k1 + j2 * k2) / n))
            out[k2, k1] = acc
    return out


def bccb(s):
    """Explicit block-circulant S with circulant blocks, first column s."""
    n = s.shape[0]
    N = n * n
    S = np.zeros((N, N))
    for p2 in range(n):
        for p1 in range(n):
            for q2 in range(n):
                for q1 in range(n):
                    S[p1 + n * p2, q1 + n * q2] = s[(p2 - q2) % n, (p1 - q1) % n]
    return S


def grid_covariance(cov, m):
    """R of Section 2.1.2: C(x_p - x_q) over the (m+1)^2 grid, x fastest."""
    h = 1.0 / m
    i = np.arange(m + 1)
    X1, X2 = np.meshgrid(i * h, i * h, indexing="xy")
    x1 = X1.ravel()
    x2 = X2.ravel()
    return cov(x1[:, None] - x1[None, :], x2[:, None] - x2[None, :])


@pytest.mark.parametrize("m,J,reading", [(3, 0, 0), (4, 0, 0), (4, 2, 1), (4, 4, 0), (4, 4, 1)])
def test_eigenvalues_equal_naive_dft_and_dense_spectrum(m, J, reading):
    cov = covariance(MATERN, 1.5, 0.3, 1.0)
    s = em.first_column(cov, m, J, reading)
    lam, imag = em.eigenvalues(s)
    ref = naive_dft_plus(s)
    scale = np.abs(ref).max()
    assert imag < 1e-12 * scale
    np.testing.assert_allclose(lam, ref.real, atol=1e-12 * scale)
    assert np.abs(ref.imag).max() < 1e-12 * scale
    S = bccb(s)
    np.testing.assert_allclose(S, S.T, atol=0)
    ev = np.sort(np.linalg.eigvalsh(S))
    np.testing.assert_allclose(np.sort(lam.ravel()), ev, atol=1e-12 * scale)


@pytest.mark.parametrize("cov_kind,nu,m,J,reading",
                         [(MATERN, 0.5, 4, 0, 0), (MATERN, 1.0, 4, 2, 1), (MATERN, 1.5, 4, 4, 0),
                          (SEPEXP, 0.5, 3, 0, 0), (MATERN, 1.0, 6, 6, 1)])
def test_embedding_contains_grid_covariance(cov_kind, nu, m, J, reading):
    # The block of S on the grid nodes (first m+1 per axis) is R itself;
    # for J > 0 this is the statement C^ext = C on [-1, 1]^2.
    cov = covariance(cov_kind, nu, 0.2, 1.3)
    s = em.first_column(cov, m, J, reading)
    n = s.shape[0]
    S = bccb(s)
    idx = np.array([i1 + n * i2 for i2 in range(m + 1) for i1 in range(m + 1)])
    R = grid_covariance(cov, m)
    np.testing.assert_allclose(S[np.ix_(idx, idx)], R, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("reading", [em.PERIOD_EUCLID, em.PERIOD_INF])
def test_periodised_column_is_even_and_exact_on_unit_box(reading):
    cov = covariance(MATERN, 1.0, 0.25, 1.0)
    m, J = 16, 16
    s = em.first_column(cov, m, J, reading)
    n = s.shape[0]
    j = np.arange(n)
    # even up to rounding of the node coordinates
    np.testing.assert_allclose(s, s[:, (n - j) % n], rtol=0, atol=1e-15)
    np.testing.assert_allclose(s, s[(n - j) % n, :], rtol=0, atol=1e-15)
    i = np.arange(m + 1) / m
    X1, X2 = np.meshgrid(i, i, indexing="xy")
    np.testing.assert_allclose(s[: m + 1, : m + 1], cov(X1, X2), rtol=1e-15)


def test_cutoff_plateaus():
    t = np.linspace(0, 3, 3001)
    phi = em.cutoff(t, 1.0, 2.0)
    assert np.all(phi[t <= 1.0] == 1.0)
    assert np.all(phi[t >= 2.0] == 0.0)
    mid = (t > 1.1) & (t < 1.9)  # near the plateaus phi rounds to exactly 0 or 1
    assert np.all((phi[mid] > 0) & (phi[mid] < 1)) and np.all(np.diff(phi) <= 0)
    np.testing.assert_allclose(em.cutoff(1.5, 1.0, 2.0), 0.5, rtol=1e-15)


def one_d_sepexp_eigenvalues(m, lam, h):
    """Closed form of the 1-D mirrored exponential embedding (n = 2m)."""
    n = 2 * m
    rho = math.exp(-h / lam)
    k = np.arange(n)
    w = rho * np.exp(2j * np.pi * k / n)
    sgn = (-1.0) ** k
    return 1.0 + 2.0 * ((w - rho ** m * sgn) / (1.0 - w)).real + rho ** m * sgn


@pytest.mark.parametrize("m,lam", [(8, 0.3), (32, 0.1), (64, 0.05)])
def test_separable_exponential_positive_and_kronecker(m, lam):
    sigma2 = 1.7
    cov = covariance(SEPEXP, 0.5, lam, sigma2)
    s = em.first_column(cov, m, 0)
    L2, _ = em.eigenvalues(s)
    L1 = one_d_sepexp_eigenvalues(m, lam, 1.0 / m)
    # Lemma 2: Lambda^{2D} = Lambda^{1D} (x) Lambda^{1D} / sigma^2 with sigma^2 = 1 per axis
    ref = sigma2 * np.outer(L1, L1)
    np.testing.assert_allclose(L2, ref, rtol=1e-11, atol=1e-12 * ref.max())
    assert L2.min() > 0


def test_psd_policies_on_fixed_size_matern_half():
    d = dict(cov=MATERN, nu=0.5, lam=0.3, sigma2=1.0, m=32)
    st = em.setup(dict(d, psd=em.PSD_CLAMP))
    assert st["n"] == 64 and st["n_clamped"] > 0 and st["lam"].min() == 0.0
    assert st["lam_min"] < -1e-6 * st["lam_max"]
    with pytest.raises(em.NotPSD):
        em.setup(dict(d, psd=em.PSD_FAIL))
    g = em.setup(dict(d, psd=em.PSD_GROW))
    assert g["n"] == 96 and g["J"] == 16 and g["lam_min"] >= -em.PSD_TOL * g["lam_max"]
    with pytest.raises(em.NotPSD):
        em.setup(dict(d, psd=em.PSD_GROW, max_pad=2))


def test_symmetrise_orbits():
    cov = covariance(MATERN, 1.0, 0.1, 1.0)
    s = em.first_column(cov, 16, 0)
    lam, _ = em.eigenvalues(s)
    sym = em.symmetrise(lam)
    n = lam.shape[0]
    np.testing.assert_allclose(sym, lam, rtol=0, atol=1e-13 * lam.max())
    k = np.arange(n)
    np.testing.assert_array_equal(sym, sym.T)
    np.testing.assert_array_equal(sym, sym[:, (n - k) % n])
    np.testing.assert_array_equal(sym, sym[(n - k) % n, :])


def test_mask_counts_and_order():
    rng = np.random.default_rng(3)
    lam = em.symmetrise(rng.uniform(0, 1, (12, 12)))
    s = lam.size
    assert em.mask(lam, 0).min() == 1.0
    assert em.mask(lam, s).max() == 0.0
    for tau in (1, 7, 40, 100):
        keep = em.mask(lam, tau)
        assert int((keep == 0).sum()) == tau
        assert lam[keep == 1].min() >= lam[keep == 0].max()
    # ties broken by linear index: among equal values the larger indices go first
    keep = em.mask(lam, 1)
    flat = lam.ravel()
    dropped = np.flatnonzero(keep.ravel() == 0)[0]
    ties = np.flatnonzero(flat == flat.min())
    assert dropped == ties.max()
