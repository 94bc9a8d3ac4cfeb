"""Pins of the oracle's adaptive MLMC estimator (oracle/mlmc.py) against
values fixed by the paper's formulas and by construction."""

import math

import numpy as np
import pytest

from oracle import mlmc


def test_optimal_samples_hand_computed():
    # sum sqrt(V C) = 1 + 1 + 1 = 3; N_l = ceil(3 sqrt(V_l/C_l) / (0.5 * 0.01))
    assert mlmc.optimal_samples([1.0, 0.25, 0.0625], [1.0, 4.0, 16.0], 0.1) == [600, 150, 38]
    # the paper's factor 2 eps^-2 is theta = 1/2; theta = 1/4 doubles every N_l
    assert mlmc.optimal_samples([1.0], [1.0], 0.1, theta=0.25) == [400]
    assert mlmc.optimal_samples([0.0, 1.0], [1.0, 1.0], 0.1) == [2, 200]   # at least 2 samples


def test_fit_slope_exact_and_richardson():
    ls = [1, 2, 3, 4]
    assert mlmc.fit_slope(ls, [3.0 - 2.0 * l for l in ls]) == pytest.approx(-2.0, abs=1e-14)
    # E[Y_L] = c 4^-L with alpha = 2: Richardson gives sum_{l>L} c 4^-l = c 4^-L / 3
    c, L = 0.7, 3
    assert mlmc.richardson_bias(c * 4.0 ** -L, 2.0) == pytest.approx(c * 4.0 ** -L / 3.0, rel=1e-14)


def test_running_stats_against_numpy():
    y = np.random.default_rng(3).normal(5.0, 0.01, 1000)
    s = mlmc.RunningStats()
    for v in y:
        s.add(v)
    assert abs(s.mean - y.mean()) <= 1e-13 * abs(y.mean())
    assert abs(s.var() - y.var(ddof=1)) <= 1e-10 * y.var(ddof=1)


def test_coarsest_mesh_rules():
    # Matern: h_0 <= sqrt(8 nu) lambda; nu = 1/2, lambda = 0.03: 0.06 -> h_0 = 1/32
    assert mlmc.coarsest_mesh("matern", 0.5, 0.03) == 32
    # separable exponential: h_0 <= lambda = 0.1 -> 1/16
    assert mlmc.coarsest_mesh("sepexp", 0.5, 0.1) == 16
    # sqrt(12) 0.1 = 0.346: 1/2 is too coarse, 1/4 is the largest admissible
    assert mlmc.coarsest_mesh("matern", 1.5, 0.1) == 4


def synthetic(seed, shift_finest=0.0):
    # E[Y_0] = 1, E[Y_l] = 4^-l (alpha = 2), V[Y_l] = 0.1 8^-l (beta = 3), C_l = 4^l
    def sample(l, finest, first, count):
        rng = np.random.default_rng([seed, l, first, int(finest)])
        mean = 1.0 if l == 0 else 4.0 ** -l
        return rng.normal(mean + (shift_finest if finest else 0.0), math.sqrt(0.1 * 8.0 ** -l), count)
    return sample


def test_synthetic_levels_reach_the_target_error():
    eps = 0.01
    cost = [4.0 ** l for l in range(8)]
    errs = []
    for seed in range(30):
        r = mlmc.run(synthetic(seed), cost, 8, eps, l_start=1, n_pilot=50)
        assert r["converged"]
        assert r["variance"] <= 0.5 * eps * eps * 1.0000001
        assert r["bias"] ** 2 <= 0.5 * eps * eps
        errs.append(r["estimate"] - 4.0 / 3.0)        # limit of sum_l E[Y_l]
    rmse = math.sqrt(np.mean(np.square(errs)))
    assert rmse <= 1.5 * eps, rmse


def test_finest_level_form_is_replaced_when_a_level_is_added():
    # the finest level is sampled in a different form (mean shifted by 0.5);
    # only the level that ends up finest may contribute that form
    cost = [4.0 ** l for l in range(8)]
    r = mlmc.run(synthetic(1, shift_finest=0.5), cost, 8, 0.01, l_start=1, n_pilot=50, finest_differs=True,
                 alpha=2.0)
    L = r["levels"] - 1
    for l in range(L):
        target = 1.0 if l == 0 else 4.0 ** -l
        assert abs(r["mean"][l] - target) < 0.05
    assert abs(r["mean"][L] - (4.0 ** -L + 0.5)) < 0.05


def test_round_cap_adds_no_unsampled_level():
    # levels with E[Y_l] = 4^-l and no variance: after the pilot round the
    # bias |E[Y_1]| / 3 = 1/12 exceeds eps, so a level would be added; with
    # no round left the run stops with the sampled levels only
    def sample(l, finest, first, count):
        return [4.0 ** -l] * count

    cost = [4.0 ** l for l in range(6)]
    r = mlmc.run(sample, cost, 6, 1e-3, l_start=1, n_pilot=4, alpha=2.0, max_rounds=1)
    assert r["rounds"] == 1 and r["levels"] == 2 and not r["converged"]
    assert r["n"] == [4, 4] and all(n > 0 for n in r["n"])
    # one more round samples the added level (pilot only: no variance)
    r = mlmc.run(sample, cost, 6, 1e-3, l_start=1, n_pilot=4, alpha=2.0, max_rounds=2)
    assert r["levels"] == 3 and r["n"] == [4, 4, 4]
    assert r["estimate"] == 1.0 + 0.25 + 0.0625
