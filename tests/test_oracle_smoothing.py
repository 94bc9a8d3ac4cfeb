"""Pins of the oracle's smoothing rule and smoothing-error statistic
(oracle/smoothing.py), and parity of the library's host-side tau rule
(ces_tau_rule, no device needed) with it."""

import math

import numpy as np
import pytest

from oracle import smoothing as osm
from paper_2306_13493_amd import workloads as W


@pytest.mark.parametrize("m,alpha,c", [(16, 1.0, 0.5), (64, 1.0, 3.0), (128, 2.0, 0.2), (256, 0.5, 10.0)])
def test_sepexp_closed_form_balances_the_two_errors(m, alpha, c):
    # eq. (k-values-p-norm-cov) comes from C_alpha h^alpha = C_s tau / (s - tau + 1)
    # with s = 4 h^-2; take C_alpha = 1, C_s = c
    _, t = osm.tau_rule(osm.SEPEXP, m, alpha, c)
    s = 4.0 * m * m
    h = 2.0 / math.sqrt(s)
    assert h ** alpha == pytest.approx(c * t / (s - t + 1.0), rel=1e-12)
    assert 0.0 <= t <= s


@pytest.mark.parametrize("m,J,nu,alpha,c", [(32, 0, 1.5, 1.0, 1.0), (64, 32, 1.5, 1.0, 0.3), (128, 64, 1.0, 2.0, 5.0),
                                            (256, 0, 0.5, 1.0, 50.0)])
def test_matern_root_solves_its_equation(m, J, nu, alpha, c):
    _, t = osm.tau_rule(osm.MATERN, m, alpha, c, nu=nu, J=J)
    s = 4.0 * (m + J) ** 2
    h = 1.0 / m
    rhs = 2.0 / c * h ** (alpha + 1.0) * (1.0 / h + J)
    assert 0.0 <= t <= s
    if t < s:
        assert (s - t + 1.0) ** (-(1.0 + nu) / 2.0) * t == pytest.approx(rhs, rel=1e-9)


@pytest.mark.parametrize("cov", [osm.SEPEXP, osm.MATERN])
def test_tau_falls_as_the_smoothing_constant_grows(cov):
    taus = [osm.tau_rule(cov, 64, 1.0, c, nu=1.5)[1] for c in (1e-3, 1e-1, 1.0, 10.0, 1e3)]
    assert all(a > b for a, b in zip(taus, taus[1:])), taus
    # a vanishing smoothing constant drops (almost) everything
    s = 4.0 * 64 * 64
    assert osm.tau_rule(cov, 64, 1.0, 1e-12, nu=1.5)[0] >= s - 1


SMALL = dict(cov="sepexp", lam=0.3, m=16, qoi="point", precision="fp64")


def test_tau_zero_gives_zero_smoothing_error():
    d = W.to_oracle(SMALL)
    st = osm.smoothing_error(d, 0, seed=2, first=0, count=6)
    assert np.all(st["diff"] == 0.0) and st["mean"] == 0.0 and st["var"] == 0.0


def test_dropping_every_eigenvalue_gives_the_constant_coefficient_qoi():
    d = W.to_oracle(SMALL)
    n = 2 * d["m"]     # separable exponential: classical embedding, no padding
    st = osm.smoothing_error(d, n * n, seed=2, first=0, count=6)
    qc = osm.constant_coefficient_qoi(d)
    assert np.allclose(st["q_smoothed"], qc, rtol=1e-12, atol=0)
    assert np.allclose(st["diff"], st["q"] - qc, rtol=0, atol=1e-15)


@pytest.mark.parametrize("cov,m,J,nu,alpha,c", [(osm.SEPEXP, 16, 0, 0.5, 1.0, 0.5), (osm.SEPEXP, 256, 0, 0.5, 2.0, 0.1),
                                                (osm.MATERN, 64, 32, 1.5, 1.0, 0.3), (osm.MATERN, 128, 0, 1.0, 1.0, 4.0),
                                                (osm.MATERN, 32, 0, 2.5, 0.5, 1e-9)])
def test_library_tau_rule_matches_the_oracle(cov, m, J, nu, alpha, c):
    import paper_2306_13493_amd as ces
    try:
        ces.load()
    except ImportError:
        pytest.skip("library not built")
    tau, t = ces.tau_rule("sepexp" if cov == osm.SEPEXP else "matern", m, alpha, c, nu=nu, J=J)
    tau_o, t_o = osm.tau_rule(cov, m, alpha, c, nu=nu, J=J)
    assert t == pytest.approx(t_o, rel=1e-9, abs=1e-9)
    if abs(t_o - math.floor(t_o) - 0.5) > 1e-6:
        assert tau == tau_o


def test_library_tau_rule_rejects_bad_arguments():
    import paper_2306_13493_amd as ces
    try:
        ces.load()
    except ImportError:
        pytest.skip("library not built")
    for args in [("sepexp", 16, 1.0, 1.0, 0.5, 4), ("matern", 16, 0.0, 1.0), ("matern", 16, 1.0, -1.0),
                 ("matern", 0, 1.0, 1.0)]:
        with pytest.raises(ces.CesError):
            ces.tau_rule(*args)


def matern_smoothing_bound(m, J, nu, tau, d=2):
    """The constant-free bound of Corollary (error-matern-cov) for p = 1 in
    d dimensions with m_i = m and J_i = J:
    s^(-1/2) (prod m_i)^(1/2) (s - tau + 1)^(-(1 + 2 nu / d) / 2) tau,
    s = 2^d prod (m_i + J_i)."""
    s = 2.0 ** d * float(m + J) ** d
    return s ** -0.5 * float(m) ** (d / 2.0) * (s - tau + 1.0) ** (-0.5 * (1.0 + 2.0 * nu / d)) * tau


@pytest.mark.parametrize("m,J,nu,alpha,c", [(32, 0, 1.5, 1.0, 1.0), (64, 32, 1.5, 1.0, 0.3), (128, 64, 1.0, 2.0, 5.0),
                                            (256, 0, 0.5, 1.0, 50.0), (64, 64, 2.5, 1.5, 0.02)])
def test_matern_root_balances_the_corollary_bound(m, J, nu, alpha, c):
    # the rule of Section 3.5: the discretisation error C_alpha h^alpha equals
    # the smoothing error C_s x (bound of Corollary (error-matern-cov)); here
    # C_alpha = 1, C_s = c.  Evaluated from the corollary's general form, so
    # a wrong exponent or a dropped (1/h + J) factor in the oracle's equation
    # fails.
    _, t = osm.tau_rule(osm.MATERN, m, alpha, c, nu=nu, J=J)
    s = 4.0 * (m + J) ** 2
    assert 0.0 < t <= s
    if t < s:
        assert (1.0 / m) ** alpha == pytest.approx(c * matern_smoothing_bound(m, J, nu, t), rel=1e-9)
    else:
        assert (1.0 / m) ** alpha >= c * matern_smoothing_bound(m, J, nu, s) * (1 - 1e-12)


@pytest.mark.parametrize("nu", [0.5, 1.0, 1.5, 2.5])
def test_embedding_eigenvalues_decay_at_the_rate_the_rule_assumes(nu):
    # the corollary's exponent comes from the Matern eigenvalue decay
    # Lambda^ord_j ~ j^-(1 + 2 nu / d) (d = 2: j^-(1 + nu)); the oracle's
    # sorted embedding eigenvalues decay at that rate (log-log slope over
    # s/64 <= j <= s/4, within the pre-asymptotic band of 15%), and not at
    # the rates a dropped 1/2 or 2 / d would give
    from oracle import embedding as em
    from oracle.covariance import MATERN
    st = em.setup(dict(cov=MATERN, nu=nu, lam=0.05, sigma2=1.0, m=128))
    lam = np.sort(np.maximum(st["lam"].ravel(), 0.0))[::-1]
    j = np.arange(1, lam.size + 1)
    sel = (j >= lam.size // 64) & (j <= lam.size // 4)
    slope = np.polyfit(np.log(j[sel]), np.log(lam[sel]), 1)[0]
    want = -(1.0 + nu)
    assert abs(slope - want) <= 0.15 * abs(want), slope
    others = [-(1.0 + nu) / 2.0, -(1.0 + 2.0 * nu)]
    assert all(abs(slope - want) < abs(slope - o) for o in others), slope
