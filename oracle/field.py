"""Per-sample Gaussian field, Algorithm 1 step 4(a)-(f) (oracle; test only).

w = a (.) xi with a = sqrt(Lambda)/n (reading of step 4(b): the
factorisation S = G Lambda G^T needs the square root of the eigenvalues;
the unitary 1/sqrt(s) of F is folded into a), v = sum_j w_j e^{+2 pi i j.p/n}
(step 4(c)), then

* HARTLEY mode (steps 4(a)-(d) as printed): xi real, Z = Re v + Im v.
* PAIR mode: xi = g0 + i g1 complex; Re v and Im v are two independent
  fields with the same law (samples 2q and 2q+1).

Restriction (step 4(e)): the fine field is v[p1, p2] for 0 <= p1, p2 <= m
(Section 2.1.2: the first m+1 entries along each axis); the coarse field
of the mesh with spacing 2h takes the even nodes (2 i1, 2 i2).  Step 4(f):
k = exp(Z).

EMBED coupling (the coarse term drawn from the coarse mesh's own
embedding, so that the smoothed estimator telescopes): the coarse
embedding's xi takes the fine xi at the nearest signed frequencies
(embedded_xi); the selection is injective when n_f >= 2 n_c, so its law is
that of an independent draw.

Pins (tests/test_oracle_field.py, tests/test_oracle_law.py): the linear
map xi -> Z satisfies A A^T = R exactly (covariance identity of Section
2.1); the emitted samples (Philox normals included) have the law of dense
Cholesky samples of R (eq. (sample-from-Z)) by two-sample tests on tiny
grids, and the two fields of one complex xi are independent; tau = 0 gives the
unsmoothed field bitwise; tau = s gives zero; empirical covariance of many
samples against C within Monte Carlo error; the smoothing error against
the explicit constant of Theorem 1's proof.
"""

import numpy as np

from .normals import normals

PAIR = 0
HARTLEY = 1


def xi(seed, q, stream, n, mode):
    """xi on the n x n embedding (indexed [j2, j1]) for pair / sample q.

    PAIR: entry e is g0 + i g1 of draw e.  HARTLEY: entry e is output e & 1
    of draw e >> 1 (both Box-Muller outputs used, a real normal per entry)."""
    e = np.arange(n * n, dtype=np.uint64)
    if mode == PAIR:
        g0, g1 = normals(seed, q, stream, e)
        return (g0 + 1j * g1).reshape(n, n)
    g0, g1 = normals(seed, q, stream, e >> np.uint64(1))
    return np.where((e & np.uint64(1)) == 1, g1, g0).reshape(n, n).astype(np.complex128)


def dft_plus(w):
    """v[p2, p1] = sum_j w[j2, j1] exp(+2 pi i (j1 p1 + j2 p2)/n)."""
    n = w.shape[0]
    return np.fft.ifft2(w) * float(n * n)


def fields(a, xi_, m, mode):
    """Restricted fine fields Z for one xi: list of one (HARTLEY) or two
    (PAIR: components 0 and 1) arrays of shape (m+1, m+1) indexed [i2, i1]."""
    v = dft_plus(a * xi_)[: m + 1, : m + 1]
    if mode == PAIR:
        return [v.real.copy(), v.imag.copy()]
    return [v.real + v.imag]


def embedded_index(n_c, n_f):
    """Fine embedding index (per axis) of each coarse embedding index of
    the EMBED coupling: the fine signed frequency nearest to the coarse one
    (coarse period n_c * 2h, fine period n_f * h), ties upwards, mod n_f."""
    j = np.arange(n_c, dtype=np.int64)
    k = np.where(j < n_c // 2, j, j - n_c)
    # round(k * n_f / (2 n_c)) with ties upwards, in integers
    f = np.floor_divide(2 * k * n_f + 2 * n_c, 4 * n_c)
    return np.where(f >= 0, f, f + n_f)


def embedded_xi(xi_f, n_c):
    """Normals of the coarse embedding taken from the fine embedding's xi
    (indexed [j2, j1]) at the same signed frequencies."""
    idx = embedded_index(n_c, xi_f.shape[0])
    return xi_f[np.ix_(idx, idx)]


def restrict_coarse(z):
    """Coarse mesh (spacing 2h) values of a fine nodal array: even nodes."""
    return z[::2, ::2].copy()
