"""Seeded synthetic inputs shared by the GPU path and the oracle in tests.

Holds no arithmetic of the method: only random coefficient arrays.
"""

import numpy as np


def lognormal_k(m, count, seed, sigma=1.0):
    """count x (m+1) x (m+1) positive coefficients exp(N(0, sigma^2)),
    smoothed by a 3-point average per axis so neighbouring values correlate."""
    rng = np.random.default_rng(seed)
    z = rng.normal(0.0, sigma, size=(count, m + 3, m + 3))
    z = (z[:, :-2, :] + z[:, 1:-1, :] + z[:, 2:, :]) / 3.0
    z = (z[:, :, :-2] + z[:, :, 1:-1] + z[:, :, 2:]) / 3.0
    return np.exp(z * 3.0 / np.sqrt(3.0))
