"""Pins of the oracle's quasi-Monte Carlo module (oracle/qmc.py) against
closed forms and brute force that do not reuse its formulas:

* e^2 for one coordinate: gamma / (6 N^2) for every odd z;
* e^2 as the sum over the dual lattice of the Fourier weights
  gamma_j / (2 pi^2 h_j^2), grouped by residues mod N with the closed forms
  sum_k 1/(a + kN)^2 = (pi / (N sin(pi a / N)))^2 and sum_{k!=0} 1/(kN)^2 =
  pi^2 / (3 N^2);
* the first 2^m points of the sequence integrate exp(2 pi i h.x) exactly:
  the sum vanishes unless h.z = 0 mod 2^m, and has modulus 1 if it is;
* each CBC component minimises e^2 over all candidates (brute force);
* the multilevel QMC estimator on synthetic levels whose decisions are
  computed by hand.
"""

import math

import numpy as np
import pytest

from oracle import qmc
from oracle import sampler as osm
from oracle import field as ofield


@pytest.mark.parametrize("p", [1, 2, 4, 6])
def test_error_one_coordinate_closed_form(p):
    N = 1 << p
    g = 0.7
    for z in range(1, N, 2):
        assert abs(qmc.error2([z], p, [g]) - g / (6.0 * N * N)) <= 1e-15


def dual_sum(z, p, gamma):
    """sum over h != 0 with h.z = 0 mod N of prod_j r_j(h_j), by residues."""
    N = 1 << p
    s = len(z)

    def S(a, g):
        if a % N == 0:
            return 1.0 + g / (6.0 * N * N)
        return g / (2.0 * N * N * math.sin(math.pi * a / N) ** 2)

    tot = 0.0
    for a in np.ndindex(*([N] * s)):
        if sum(int(ai) * int(zi) for ai, zi in zip(a, z)) % N == 0:
            tot += math.prod(S(ai, g) for ai, g in zip(a, gamma))
    return tot - 1.0


@pytest.mark.parametrize("z,p,gamma", [([1, 5], 4, [1.0, 0.5]), ([1, 3, 7], 4, [0.9, 0.4, 0.2]),
                                       ([1, 11, 5], 5, [1.0, 1.0, 1.0])])
def test_error_equals_dual_lattice_sum(z, p, gamma):
    assert abs(qmc.error2(z, p, gamma) - dual_sum(z, p, gamma)) <= 1e-13


@pytest.mark.parametrize("m", [0, 1, 3, 5])
def test_sequence_prefix_integrates_characters_exactly(m):
    z = [1, 13, 27, 5]
    D = qmc.shifts(11, 2, 3, len(z))
    n = 1 << m
    pts = np.array([qmc.lattice_points(i, z, D) for i in range(n)])
    assert np.all(pts > 0) and np.all(pts < 1)
    rng = np.random.default_rng(0)
    for _ in range(40):
        h = rng.integers(-9, 10, size=len(z))
        v = np.exp(2j * np.pi * (pts @ h)).mean()
        if sum(int(a) * b for a, b in zip(h, z)) % n == 0:
            assert abs(abs(v) - 1.0) <= 1e-9
        else:
            assert abs(v) <= 1e-9


def test_points_are_the_shifted_lattice():
    # point i of the sequence is frac(phi_2(i) z + Delta), phi_2 the van der Corput radical inverse
    z = [1, 7]
    D = [1 << 63, 3 << 61]
    for i in range(16):
        phi = sum(((i >> b) & 1) * 2.0 ** -(b + 1) for b in range(8))
        want = [(phi * zj + dj / 2.0 ** 64) % 1.0 for zj, dj in zip(z, D)]
        assert np.allclose(qmc.lattice_points(i, z, D), want, atol=2.0 ** -51)


@pytest.mark.parametrize("p,gamma", [(5, [1.0, 0.6, 0.3]), (6, [0.5, 0.5, 0.25, 0.1])])
def test_cbc_components_minimise_the_error(p, gamma):
    N = 1 << p
    z = qmc.cbc(p, gamma)
    assert z[0] == 1 and all(v % 2 == 1 and v <= N // 2 for v in z)
    for j in range(1, len(z)):
        errs = {c: qmc.error2(z[:j] + [c], p, gamma[: j + 1]) for c in range(1, N, 2)}
        best = min(errs.values())
        # the criterion's terms are truncated to 2^-40: optimal to that resolution
        assert errs[z[j]] <= best + 1e-11


def test_cbc_beats_the_worst_candidate_and_plain_mc():
    p, gamma = 8, list(0.5 ** np.arange(6))
    z = qmc.cbc(p, gamma)
    N = 1 << p
    e_cbc = qmc.error2(z, p, gamma)
    # Monte Carlo mean squared error of the same integrand class: (prod(1 + gamma/180) - 1) / N
    e_mc = (math.prod(1 + g * g / 180.0 for g in gamma) - 1.0) / N
    assert e_cbc < e_mc
    assert e_cbc < qmc.error2([1] * len(gamma), p, gamma)


def test_eigen_order_and_weights():
    lam = np.array([0.5, 2.0, -1e-18, 2.0, 1.0])
    assert list(qmc.eigen_order(lam, 4)) == [1, 3, 4, 0]
    w = qmc.default_weights(lam[[1, 3, 4]])
    assert abs(w.sum() - 1.0) <= 1e-15 and w[0] == w[1] == 0.4


def test_lattice_xi_replaces_only_the_lattice_coordinates():
    n = 8
    lat = qmc.Lattice([1, 3, 5], [9, 0, 40], 4)
    g = 13
    x = qmc.lattice_xi(lat, 5, g, 1, n).reshape(-1)
    ref = ofield.xi(5, g, 1, n, ofield.HARTLEY).reshape(-1)
    other = np.setdiff1d(np.arange(n * n), lat.dims)
    assert np.array_equal(x[other], ref[other])
    u = qmc.lattice_points(g // 4, lat.z, qmc.shifts(5, 1, g % 4, 3))
    # Phi(xi) = u at the lattice coordinates
    from scipy.special import ndtr
    assert np.allclose(ndtr(x[lat.dims].real), u, rtol=1e-13, atol=0)


def test_plan_lattice_needs_hartley():
    d = dict(cov="matern", nu=0.5, lam=0.2, sigma2=1.0, m=8, level=0, field_mode=ofield.PAIR)
    with pytest.raises(ValueError):
        osm.Plan(d).set_lattice(qmc.Lattice([1], [0], 2))


def test_run_constant_levels_hand_computed():
    # Y_l = c_l exactly: every shift mean equals c_l, V_l = 0, nothing is doubled;
    # alpha is fitted from |c_1| = 1/4, |c_2| = 1/16 (slope -2), so the bias of
    # level 2 is (1/16) / 3 and eps decides whether level 3 is added
    c = [1.0, 0.25, 1.0 / 16, 1.0 / 64]

    def sample(l, finest, first, count):
        return [c[l]] * count

    r = qmc.run(sample, [1.0, 2.0, 4.0, 8.0], 4, eps=0.06, shifts_=4, l_start=2, n_pilot=2)
    assert r["levels"] == 3 and r["converged"] == 1 and r["points"] == [2, 2, 2]
    assert r["estimate"] == sum(c[:3]) and r["variance"] == 0.0
    assert abs(r["alpha"] - 2.0) <= 1e-12
    r = qmc.run(sample, [1.0, 2.0, 4.0, 8.0], 4, eps=0.02, shifts_=4, l_start=2, n_pilot=2)
    assert r["levels"] == 4 and r["converged"] == 1 and r["n"] == [8, 8, 8, 8]


def test_run_doubling_rule_hand_computed():
    # level l's shift means are c_l + a_l w_r whatever the points: V_l = a_l^2 var(w) / R.
    # With R = 2, w = (-1, 1): var(w) = 2, V = (a0^2, a1^2).  eps^2 theta = 0.5 * 0.1^2 = 0.005
    a = [0.1, 0.04]
    cost = [1.0, 4.0]

    def sample(l, finest, first, count):
        return [(1.0 if l == 0 else 0.0) + a[l] * (-1.0 if (first + t) % 2 == 0 else 1.0) for t in range(count)]

    r = qmc.run(sample, cost, 2, eps=0.1, shifts_=2, l_start=1, n_pilot=1, max_rounds=1)
    # V = (0.01, 0.0016), points (1, 1): ratios 0.01 and 0.0004 -> double level 0 (V0 -> 0.005,
    # sum 0.0066); ratios 0.0025 and 0.0004 -> level 0 again (0.0025, sum 0.0041 <= 0.005: stop)
    assert r["rounds"] == 1 and r["points"] == [1, 1]
    assert abs(r["variance"] - (0.01 + 0.0016)) <= 1e-15
    r2 = qmc.run(sample, cost, 2, eps=0.1, shifts_=2, l_start=1, n_pilot=1, max_rounds=2)
    assert r2["points"] == [4, 1] and r2["n"] == [8, 2]


def test_run_round_cap_adds_no_unsampled_level():
    # shift means equal c_l on every shift (no variance); the bias after the
    # pilot round exceeds eps, and with no round left no level is added
    c = [1.0, 0.25, 0.0625, 0.015625]

    def sample(l, finest, first, count):
        return [c[l]] * count

    r = qmc.run(sample, [1.0, 2.0, 4.0, 8.0], 4, eps=1e-3, shifts_=4, l_start=1, n_pilot=2, alpha=2.0,
                max_rounds=1)
    assert r["rounds"] == 1 and r["levels"] == 2 and r["converged"] == 0 and r["points"] == [2, 2]
    r = qmc.run(sample, [1.0, 2.0, 4.0, 8.0], 4, eps=1e-3, shifts_=4, l_start=1, n_pilot=2, alpha=2.0,
                max_rounds=2)
    assert r["levels"] == 3 and r["points"] == [2, 2, 2]


def exact_error2(z, p, gamma):
    """e^2 of the rank-1 rule in exact rational arithmetic (the definition,
    B2(x) = x^2 - x + 1/6 at x = {k z / N}, with the float weights taken
    exactly)."""
    from fractions import Fraction
    N = 1 << p
    g = [Fraction(float(v)) for v in gamma]
    tot = Fraction(0)
    for k in range(N):
        prod = Fraction(1)
        for zj, gj in zip(z, g):
            x = Fraction((k * int(zj)) % N, N)
            prod *= 1 + gj * (x * x - x + Fraction(1, 6))
        tot += prod
    return tot / N - 1


@pytest.mark.parametrize("p,gamma", [(4, [1.0, 1e-13, 0.3]), (5, [0.8, 3e-12, 1e-12]), (4, [0.5, 0.0, 0.25]),
                                     (6, [1.0, 0.6, 2e-12]), (5, [1.0, 0.9, 0.8])])
def test_cbc_choice_is_the_exact_argmin_up_to_its_truncation(p, gamma):
    # the CBC criterion truncates every term to a multiple of 2^-40 (so that
    # any summation order gives the same choice); each term moves by less
    # than 2^-40, so e^2 of the chosen candidate is within 2^-40 (plus the
    # float rounding of the products, far smaller) of the exact minimum,
    # and the choice is the exact argmin wherever that is ahead by more.
    # Weights near 1e-12 build near-ties below that resolution.
    from fractions import Fraction
    N = 1 << p
    tol = Fraction(2) ** -40 + Fraction(1, 10 ** 14)
    z = qmc.cbc(p, gamma)
    cand = list(range(1, N // 2 + 1, 2))
    for j in range(len(gamma)):
        e = {c: exact_error2(z[:j] + [c], p, gamma[: j + 1]) for c in cand}
        best = min(e.values())
        assert e[z[j]] - best <= tol, (j, float(e[z[j]] - best))
        winners = [c for c in cand if e[c] == best]
        runner_up = min((v for c, v in e.items() if v != best), default=None)
        if len(winners) == 1 and runner_up is not None and runner_up - best > tol:
            assert z[j] == winners[0]
        if gamma[j] == 0.0:
            assert z[j] == 1      # exact tie over every candidate: the smallest
