"""Pins of the EMBED coupling of the oracle (coarse term of a pair level
drawn from the coarse mesh's own embedding with the fine normals of the
same signed frequencies)."""

import numpy as np
import pytest

from oracle import embedding as em, field as fd, sampler as osm
from oracle.covariance import covariance, MATERN, SEPEXP


def signed(k, n):
    return np.where(k < n // 2, k, k - n)


@pytest.mark.parametrize("n_c,n_f", [(8, 16), (12, 24), (16, 32), (8, 24), (32, 96), (16, 64), (24, 64)])
def test_selection_is_injective_and_takes_the_nearest_frequency(n_c, n_f):
    idx = fd.embedded_index(n_c, n_f)
    assert len(set(idx.tolist())) == n_c and idx.min() >= 0 and idx.max() < n_f
    # physical frequencies: coarse k / (n_c 2h), fine f / (n_f h); the
    # chosen fine frequency is the nearest (within half a fine spacing)
    k = signed(np.arange(n_c), n_c)
    f = signed(idx, n_f)
    assert np.all(np.abs(f / n_f - k / (2.0 * n_c)) <= 0.5 / n_f + 1e-15)
    if n_f == 2 * n_c:
        np.testing.assert_array_equal(f, k)


def grid_cov(cov, m):
    h = 1.0 / m
    i = np.arange(m + 1)
    X1, X2 = np.meshgrid(i * h, i * h, indexing="xy")
    x1, x2 = X1.ravel(), X2.ravel()
    return cov(x1[:, None] - x1[None, :], x2[:, None] - x2[None, :])


@pytest.mark.parametrize("kind,nu,lam,m", [(SEPEXP, 0.5, 0.3, 8), (MATERN, 1.0, 0.3, 8)])
def test_embedded_coarse_field_has_the_coarse_grid_law(kind, nu, lam, m):
    # the map fine xi -> coarse field: its covariance is the covariance
    # matrix of the coarse grid (A A^T + B B^T = R_c, as for a level of its own)
    d = dict(cov=kind, nu=nu, lam=lam, sigma2=1.1, m=m, level=osm.PAIR_LEVEL, coupling=osm.EMBED)
    p = osm.Plan(d)
    c = p.coarse_plan
    assert c is not None and p.n == 2 * c.n and c.desc["m"] == m // 2
    n = p.n
    A, B = [], []
    for j in range(n * n):
        e = np.zeros(n * n, dtype=complex)
        e[j] = 1.0
        z = fd.fields(c.a_f, fd.embedded_xi(e.reshape(n, n), c.n), m // 2, fd.PAIR)
        A.append(z[0].ravel())
        e[j] = 1j
        z = fd.fields(c.a_f, fd.embedded_xi(e.reshape(n, n), c.n), m // 2, fd.PAIR)
        B.append(z[0].ravel())
    A, B = np.stack(A, axis=1), np.stack(B, axis=1)
    R = grid_cov(covariance(kind, nu, lam, 1.1), m // 2)
    np.testing.assert_allclose(A @ A.T + B @ B.T, R, atol=1e-13)


def test_embedded_coarse_term_equals_the_coarser_level_on_selected_normals():
    # a pair level's coarse field is the field of the next coarser single
    # level when that level draws the selected normals; with RESTRICT it is
    # the fine field's even nodes instead
    base = dict(cov=MATERN, nu=1.5, lam=0.2, sigma2=1.0, m=16, level=osm.PAIR_LEVEL)
    pe = osm.Plan(dict(base, coupling=osm.EMBED))
    pr = osm.Plan(dict(base, coupling=osm.RESTRICT))
    single = osm.Plan(dict(base, m=8, level=osm.SINGLE))
    for i in (0, 1, 5):
        zf_e, zc_e = pe.fields(4, i)
        zf_r, zc_r = pr.fields(4, i)
        np.testing.assert_array_equal(zf_e, zf_r)
        xi = fd.xi(4, i // 2, 0, pe.n, fd.PAIR)
        want = fd.fields(single.a_f, fd.embedded_xi(xi, single.n), 8, fd.PAIR)[i % 2]
        np.testing.assert_array_equal(zc_e, want)
        np.testing.assert_array_equal(zc_r, fd.restrict_coarse(zf_r))
        # the two couplings differ, but both follow the fine field closely
        assert not np.array_equal(zc_e, zc_r)
        assert np.max(np.abs(zc_e - zc_r)) < 0.5 * np.max(np.abs(zc_r))


def test_embed_plans_padded_differently():
    # lambda = 0.3 needs padding on 32^2 (n = 96) but not on 16^2 (n = 32):
    # the coarse xi takes the nearest of the fine frequencies
    d = dict(cov=MATERN, nu=0.5, lam=0.3, sigma2=1.0, m=32, level=osm.PAIR_LEVEL, coupling=osm.EMBED)
    p = osm.Plan(d)
    assert (p.n, p.coarse_plan.n) == (96, 32)
    zf, zc = p.fields(1, 3)
    xi = fd.xi(1, 1, 0, p.n, fd.PAIR)
    want = fd.fields(p.coarse_plan.a_f, fd.embedded_xi(xi, p.coarse_plan.n), 16, fd.PAIR)[1]
    np.testing.assert_array_equal(zc, want)
