"""Pins of oracle.sampler (Algorithms 1-2, MLMC telescoping of Section 3.4)."""

import numpy as np
import pytest

from oracle import sampler, field, embedding


BASE = dict(cov=0, nu=0.5, lam=0.3, sigma2=1.0, psd=0, qoi=0, bc=0)


def test_pair_components_share_one_xi():
    p = sampler.Plan(dict(BASE, m=8, level=0))
    z0, _ = p.fields(5, 6)
    z1, _ = p.fields(5, 7)
    n = p.n
    v = field.dft_plus(p.a_f * field.xi(5, 3, 0, n, field.PAIR))[:9, :9]
    np.testing.assert_array_equal(z0, v.real)
    np.testing.assert_array_equal(z1, v.imag)


def test_coarse_field_is_even_node_restriction_and_one_dft_when_taus_equal():
    p = sampler.Plan(dict(BASE, m=8, level=1, tau_f=10, tau_c=10))
    zf, zc = p.fields(1, 3)
    np.testing.assert_array_equal(zc, zf[::2, ::2])
    assert zc.shape == (5, 5)


def test_finest_level_uses_unsmoothed_fine_field():
    d = dict(BASE, m=8, level=1, tau_f=0, tau_c=-1)
    p = sampler.Plan(d)
    q = sampler.Plan(dict(d, level=0, tau_f=0))
    zf, zc = p.fields(2, 9)
    zf_single, _ = q.fields(2, 9)
    np.testing.assert_array_equal(zf, zf_single)
    assert p.tau_c == p.n
    r = sampler.Plan(dict(d, level=0, tau_f=-1))
    zs, _ = r.fields(2, 9)
    np.testing.assert_array_equal(zc, zs[::2, ::2])


@pytest.mark.slow
def test_mlmc_telescoping_in_expectation():
    # E[Y_1] = E[Q_{h_1}] - E[Q_{h_0}] (Section 3.4), estimated with
    # independent streams; unsmoothed, so the identity is exact in law.
    N = 1500
    d1 = dict(BASE, m=8, level=1, tau_f=0, tau_c=0, stream=1)
    y1, qf, qc = sampler.level_samples(d1, 0, 0, N)
    d0 = dict(BASE, m=4, level=0, tau_f=0, stream=2)
    q0, _, _ = sampler.level_samples(d0, 0, 0, N)
    diff = y1.mean() - (qf.mean() - q0.mean())
    se = np.sqrt(q0.var() / N + qc.var() / N)
    assert abs(diff) < 5 * se
    np.testing.assert_allclose(y1, qf - qc, rtol=0, atol=0)
