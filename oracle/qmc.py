"""Randomised quasi-Monte Carlo level sampling (oracle; test infrastructure
only).

The paper's outlook (Section 5) names multilevel quasi-Monte Carlo as the
direct extension of the smoothed sampler, and Sections 2.1.1-2.1.2 note
that QMC uses the real (Hartley) factorisation of the embedding; the paper
fixes no QMC method.  The method built here is the usual one of the QMC
literature for PDEs with random coefficients, restated from the published
definitions:

* Rank-1 lattice rule, N = 2^p points, generating vector z by the
  component-by-component (CBC) construction of Sloan, Kuo and Joe (2002):
  coordinate j takes the candidate that minimises the shift-averaged
  worst-case error of the weighted unanchored Sobolev space (first-order
  mixed smoothness, product weights gamma_j) given z_1..z_{j-1},
      e^2(z) = -1 + (1/N) sum_k prod_j (1 + gamma_j B2({k z_j / N})),
      B2(x) = x^2 - x + 1/6.
  Candidates are the odd z <= N/2 (z and N - z give the same error; N = 2
  has the single candidate 1); ties go to the smaller z.  Each candidate's
  sum is taken with every term truncated to a multiple of 2^-40 and added
  exactly in integers, so the choice does not depend on summation order.
* Points in radical-inverse order (a lattice sequence: Hickernell, Hong,
  L'Ecuyer and Lemieux, 2000): point i is {phi_2(i) z}, so the first 2^m
  points form the lattice rule with N = 2^m for every m.  In 64-bit fixed
  point the shifted point is U = (bitrev64(i) z + D) mod 2^64 and the
  uniform is u = (floor(U / 2^12) + 1/2) 2^-52, in (0, 1).
* R independent uniform shifts: D_{r,j} = x0 + 2^32 x1 from Philox4x32-10
  with counter (j, r, 2^32 - 1, stream) and the sampling seed as key (the
  Monte Carlo normals use counters (e, q mod 2^32, q >> 32, stream), which
  meet these only for sample indices of at least 2^64 - 2^32).
* xi_e = Phi^{-1}(u) at the eigen indices e = dims[j] (coordinate j); every
  other xi_e is the Monte Carlo sampler's Philox normal.  Sample index g is
  point floor(g / R) of shift g mod R.
* Multilevel estimator of Giles and Waterhouse (2009, "Multilevel
  quasi-Monte Carlo path simulation"): on each level the R shift averages
  give the level mean and the variance V_l of its estimate; while
  sum_l V_l exceeds theta eps^2 the level with the largest V_l / (C_l N_l)
  has its points per shift doubled; levels are added as in the Monte Carlo
  estimator (Richardson bias).

Parity status: lattice_points, cbc, error2 and run are pinned in
tests/test_oracle_qmc.py (closed forms, the dual-lattice sum, exact
integration of trigonometric polynomials, brute-force argmin, the exact
rational argmin up to the truncation's resolution 2^-40 on constructed
near-ties, synthetic levels).  Phi^{-1} is scipy.special.ndtri (a library
primitive).
"""

import numpy as np
from scipy.special import ndtri

from . import field
from .mlmc import fit_slope
from .normals import philox4x32_10

FRAC_BITS = 40
M64 = (1 << 64) - 1


def b2(x):
    """Bernoulli polynomial B2(x) = x (x - 1) + 1/6 (x(x-1) exact for x = a/N)."""
    x = np.asarray(x, dtype=np.float64)
    return x * (x - 1.0) + (1.0 / 6.0)


def error2(z, log2n, gamma):
    """Shift-averaged squared worst-case error e^2(z) (real arithmetic)."""
    N = 1 << log2n
    k = np.arange(N, dtype=np.int64)
    prod = np.ones(N)
    for zj, gj in zip(z, gamma):
        prod *= 1.0 + gj * b2(((k * int(zj)) % N) / N)
    return float(prod.mean() - 1.0)


def _exact_sum(t):
    """sum_k floor(t_k 2^40), exactly (t_k >= 0, t_k < 2^23)."""
    v = np.floor(np.ldexp(t, FRAC_BITS)).astype(np.uint64)
    hi = (v >> np.uint64(32)).astype(np.int64)
    lo = (v & np.uint64(0xFFFFFFFF)).astype(np.int64)
    return (int(hi.sum(dtype=np.int64)) << 32) + int(lo.sum(dtype=np.int64))


def cbc(log2n, gamma):
    """Generating vector (list of ints) for N = 2^log2n and weights gamma."""
    N = 1 << log2n
    k = np.arange(N, dtype=np.int64)
    cand = [1] if N <= 2 else list(range(1, N // 2 + 1, 2))
    P = np.ones(N)
    z = []
    for gj in gamma:
        best, best_s = None, None
        for c in cand:
            f = 1.0 + gj * b2(((k * c) % N) / N)
            s = _exact_sum(P * f)
            if best_s is None or s < best_s:
                best, best_s = c, s
        z.append(best)
        P = P * (1.0 + gj * b2(((k * best) % N) / N))
    return z


def bitrev64(i):
    return int("{:064b}".format(int(i))[::-1], 2)


def shifts(seed, stream, r, s):
    """64-bit shifts D_{r,j}, j = 0..s-1 (Python ints)."""
    j = np.arange(s, dtype=np.uint64)
    x0, x1, _, _ = philox4x32_10(j, np.uint64(r), np.uint64(0xFFFFFFFF), np.uint64(int(stream) & 0xFFFFFFFF),
                                 np.uint64(int(seed) & 0xFFFFFFFF), np.uint64((int(seed) >> 32) & 0xFFFFFFFF))
    return [int(a) + (int(b) << 32) for a, b in zip(x0, x1)]


def lattice_points(i, z, D):
    """Uniforms u_j in (0,1) of point i (radical-inverse order), shift D."""
    bi = bitrev64(i)
    out = np.empty(len(z))
    for j, (zj, dj) in enumerate(zip(z, D)):
        U = (bi * int(zj) + int(dj)) & M64
        out[j] = (float(U >> 12) + 0.5) * 2.0 ** -52
    return out


class Lattice:
    """Lattice attached to a level: s coordinates, generating vector z,
    eigen indices dims, R shifts."""

    def __init__(self, z, dims, shifts_):
        self.z = [int(v) for v in z]
        self.dims = [int(v) for v in dims]
        self.R = int(shifts_)
        if len(self.z) != len(self.dims) or len(set(self.dims)) != len(self.dims):
            raise ValueError("z and dims must have one entry per coordinate, dims distinct")


def lattice_xi(lat, seed, g, stream, n):
    """Hartley xi (n x n complex, imaginary part zero) of sample g."""
    x = field.xi(seed, g, stream, n, field.HARTLEY).reshape(-1).copy()
    i, r = divmod(int(g), lat.R)
    u = lattice_points(i, lat.z, shifts(seed, stream, r, len(lat.z)))
    x[np.asarray(lat.dims, dtype=np.int64)] = ndtri(u)
    return x.reshape(n, n)


def eigen_order(lam, s):
    """Indices of the s largest eigenvalues (value descending, index ascending)."""
    lam = np.maximum(np.asarray(lam, dtype=np.float64).reshape(-1), 0.0)
    idx = np.lexsort((np.arange(lam.size), -lam))
    return idx[:s]


def default_weights(lam_sel):
    """Product weights: the selected eigenvalues scaled to sum to one."""
    lam_sel = np.maximum(np.asarray(lam_sel, dtype=np.float64), 0.0)
    t = lam_sel.sum()
    return lam_sel / t if t > 0 else np.full(lam_sel.size, 1.0 / max(lam_sel.size, 1))


def run(sample, cost, nlevels, eps, shifts_, l_start=2, n_pilot=1, theta=0.5, alpha=0.0, max_rounds=50,
        finest_differs=False):
    """Multilevel QMC estimator.  sample(l, finest, first, count) returns
    the level samples Y_l of indices first .. first+count-1 (index g is
    point g // R of shift g % R); cost[l] is the cost of one sample."""
    R = int(shifts_)
    L = min(l_start, nlevels - 1)
    pts = [0] * nlevels
    want = [0] * nlevels
    sums = [np.zeros(R) for _ in range(nlevels)]
    for l in range(L + 1):
        want[l] = n_pilot
    alpha_fit = alpha
    bias = 0.0
    converged = False
    rounds = 0

    def stats(l):
        means = sums[l] / pts[l]
        mu = means.sum() / R
        v = float(((means - mu) ** 2).sum() / (R - 1))
        return float(mu), v

    while rounds < max_rounds:
        for l in range(L + 1):
            if want[l] > pts[l]:
                first = pts[l] * R
                ys = sample(l, finest_differs and l == L, first, (want[l] - pts[l]) * R)
                for t, y in enumerate(ys):
                    sums[l][(first + t) % R] += y
                pts[l] = want[l]
        rounds += 1
        st = [stats(l) for l in range(L + 1)]
        V = [v / R for _, v in st]
        # doublings planned with the Monte Carlo rate (V halves)
        proj = list(V)
        newp = list(pts[: L + 1])
        while sum(proj) > theta * eps * eps:
            ratios = [proj[l] / (cost[l] * newp[l]) for l in range(L + 1)]
            ls = int(np.argmax(ratios))
            newp[ls] *= 2
            proj[ls] /= 2.0
        more = False
        for l in range(L + 1):
            want[l] = newp[l]
            more = more or want[l] > pts[l]
        if L >= 2 and alpha <= 0.0:
            alpha_fit = max(0.5, -fit_slope(list(range(1, L + 1)),
                                            [np.log2(max(abs(st[l][0]), 1e-300)) for l in range(1, L + 1)]))
        elif alpha <= 0.0:
            alpha_fit = 1.0
        bias = abs(st[L][0]) / (2.0 ** alpha_fit - 1.0) if L >= 1 else 0.0
        if more:
            continue
        if L >= 1 and bias * bias <= (1.0 - theta) * eps * eps:
            converged = True
            break
        if L + 1 >= nlevels or rounds >= max_rounds:
            break
        if finest_differs:
            sums[L] = np.zeros(R)
            pts[L] = 0
            want[L] = n_pilot
        L += 1
        want[L] = n_pilot
    st = [stats(l) for l in range(L + 1)]
    return {
        "levels": L + 1, "converged": int(converged), "rounds": rounds,
        "points": pts[: L + 1], "n": [p * R for p in pts[: L + 1]],
        "mean": [mu for mu, _ in st], "var": [v for _, v in st],
        "estimate": sum(mu for mu, _ in st), "variance": sum(v / R for _, v in st),
        "bias": bias, "alpha": alpha_fit,
    }
