"""Circulant embedding set-up (oracle; test infrastructure only).

Follows Section 2.1.2 (two-dimensional embedding), Section 2.2 (padding and
smooth periodisation), Algorithm 1 steps 1-3 and Algorithm 2 step 4(b).

Array convention: a 2-D array ``a`` of the embedding (size n x n) is indexed
``a[j2, j1]`` -- x index fastest, the lexicographic order of Section 2.1.2.

Readings of the paper taken here:
* J = 0 is the classical mirrored embedding (the cutoff is undefined there).
* J > 0 evaluates the periodised covariance C^ext of eq. (periodic-cov-fun)
  at every embedding node; the cutoff phi is the paper's eta-quotient with
  two readings of the norm and plateau:
    PERIOD_INF    (literal text): |.|_inf, plateau 1, kappa = 2 ell - 1
    PERIOD_EUCLID (default): |.|_2, plateau sqrt(2), kappa = 2 ell - sqrt(2),
                  i.e. the exactness condition ell >= (kappa + sqrt(d))/2
                  taken with equality.
  Both give C^ext = C on [-1, 1]^2.
* Eigenvalues are the unnormalised DFT with + sign of the first column
  (Lambda = sqrt(s) F s with unitary F of positive exponent).
* Nonnegativity test: accept iff min Lambda >= -1e-13 max Lambda; then the
  remaining (round-off) negatives are set to zero.  GROW tries
  J = 0, m/2, m while n = 2(m + J) <= max_pad_factor * m.
* Eigenvalues are orbit-symmetrised before ordering: every index takes the
  value of its representative (min(k1, n-k1), min(k2, n-k2)) with the pair
  sorted, so symmetric entries are bitwise equal.
* tau counts the dropped (smallest) eigenvalues; the order is Lambda
  descending, then linear index k1 + n k2 ascending.

Pins (tests/test_oracle_embedding.py): naive DFT; dense eigen-decomposition
of the explicit block-circulant matrix S; the top-left block of S equals
the covariance matrix R of the grid; separable-exponential positivity and
Kronecker structure with the 1-D geometric-sum closed form; C^ext = C on
[-1, 1]^2; tau = 0 keeps everything, tau = s drops everything.
"""

import math

import numpy as np

from .covariance import covariance

PSD_GROW = 0
PSD_CLAMP = 1
PSD_FAIL = 2
PERIOD_EUCLID = 0
PERIOD_INF = 1
PSD_TOL = 1e-13


class NotPSD(RuntimeError):
    pass


def _eta(x):
    """eta(x) = exp(-1/x) for x > 0, else 0 (Section 2.2)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    pos = x > 0
    out[pos] = np.exp(-1.0 / x[pos])
    return out


def cutoff(t, lo, kappa):
    """Smooth cutoff phi(t): 1 for t <= lo, 0 for t >= kappa (Section 2.2)."""
    t = np.abs(np.asarray(t, dtype=np.float64))
    w = kappa - lo
    a = _eta((kappa - t) / w)
    b = _eta((t - lo) / w)
    return a / (a + b)


def first_column(cov, m, J, reading=PERIOD_EUCLID):
    """First column s of the embedding matrix S as an n x n array, n = 2(m+J).

    J = 0: s[j2, j1] = C(min(j1, n-j1) h, min(j2, n-j2) h) (mirroring,
    Section 2.1.2).  J > 0: s[j2, j1] = C^ext(j1 h, j2 h) with the
    2 ell-periodic extension of eq. (periodic-cov-fun), ell = 1 + J/m.
    """
    n = 2 * (m + J)
    h = 1.0 / m
    j = np.arange(n)
    if J == 0:
        jh = np.minimum(j, n - j) * h
        x1 = jh[None, :]
        x2 = jh[:, None]
        return cov(np.broadcast_to(x1, (n, n)), np.broadcast_to(x2, (n, n)))
    ell = 1.0 + J / m
    if reading == PERIOD_INF:
        lo, kappa = 1.0, 2.0 * ell - 1.0
    elif reading == PERIOD_EUCLID:
        lo, kappa = math.sqrt(2.0), 2.0 * ell - math.sqrt(2.0)
        if not kappa > lo:
            raise ValueError("Euclidean periodisation needs ell > sqrt(2)")
    else:
        raise ValueError("unknown periodisation reading")
    x = j * h
    s = np.zeros((n, n))
    # Images x + 2 ell n with n in {0, -1}^2 are the only ones that can
    # reach the support [-kappa, kappa]^2 of C phi_kappa for x in [0, 2 ell).
    for a in (0, -1):
        for b in (0, -1):
            y1 = np.broadcast_to((x + 2.0 * ell * a)[None, :], (n, n))
            y2 = np.broadcast_to((x + 2.0 * ell * b)[:, None], (n, n))
            if reading == PERIOD_INF:
                t = np.maximum(np.abs(y1), np.abs(y2))
            else:
                t = np.sqrt(y1 * y1 + y2 * y2)
            s = s + cov(y1, y2) * cutoff(t, lo, kappa)
    return s


def eigenvalues(s):
    """Lambda[k2, k1] = sum_j s[j2, j1] exp(+2 pi i (j1 k1 + j2 k2)/n).

    Algorithm 1 step 3.  numpy's inverse FFT carries the + sign and a 1/n^2
    factor, which is undone here.  Returns (real part, max |imag part|).
    """
    n = s.shape[0]
    lam = np.fft.ifft2(s) * float(n * n)
    return lam.real.copy(), float(np.max(np.abs(lam.imag)))


def symmetrise(lam):
    """Orbit symmetrisation: every index takes its representative's value."""
    n = lam.shape[0]
    k = np.arange(n)
    r = np.minimum(k, n - k)
    a = np.broadcast_to(r[None, :], (n, n))  # from k1
    b = np.broadcast_to(r[:, None], (n, n))  # from k2
    lo = np.minimum(a, b)
    hi = np.maximum(a, b)
    # representative (k1, k2) = (lo, hi): value lam[hi, lo]
    return lam[hi, lo].copy()


def setup(desc):
    """Algorithm 1 steps 1-3 with the nonnegativity policy.

    Returns a dict: n, J, lam (symmetrised, negatives clamped), lam_min,
    lam_max (before clamping), n_clamped, imag_max.
    """
    m = desc["m"]
    cov = covariance(desc["cov"], desc.get("nu", 0.5), desc["lam"], desc["sigma2"])
    policy = desc.get("psd", PSD_GROW)
    reading = desc.get("period", PERIOD_EUCLID)
    maxpad = desc.get("max_pad", 4)
    if policy == PSD_GROW:
        cands = [J for J in (0, m // 2, m) if 2 * (m + J) <= maxpad * m]
    else:
        cands = [0]
    last = None
    for J in cands:
        s = first_column(cov, m, J, reading)
        lam, imag = eigenvalues(s)
        lam = symmetrise(lam)
        lmin, lmax = float(lam.min()), float(lam.max())
        ok = lmin >= -PSD_TOL * lmax
        last = (J, lam, lmin, lmax, imag)
        if ok or policy == PSD_CLAMP:
            break
    J, lam, lmin, lmax, imag = last
    if not (lmin >= -PSD_TOL * lmax) and policy != PSD_CLAMP:
        raise NotPSD("embedding not nonnegative (min/max = %g)" % (lmin / lmax))
    neg = lam < 0
    lam = np.where(neg, 0.0, lam)
    return dict(n=2 * (m + J), J=J, lam=lam, lam_min=lmin, lam_max=lmax,
                n_clamped=int(neg.sum()), imag_max=imag)


def tau_default(n):
    """Default number of dropped eigenvalues, tau = sqrt(s) = n (Section 4)."""
    return n


def mask(lam, tau):
    """Algorithm 2 step 4(b): zero the tau smallest of the ordered eigenvalues.

    Order: Lambda descending, ties by linear index k1 + n k2 ascending.
    Returns a float64 array of 0/1 with the same shape as lam.
    """
    n = lam.shape[0]
    s = n * n
    tau = int(tau)
    if tau < 0 or tau > s:
        raise ValueError("tau out of range")
    flat = lam.reshape(-1)
    idx = np.arange(s)
    order = np.lexsort((idx, -flat))  # primary key -lam, secondary index
    keep = np.ones(s)
    if tau > 0:
        keep[order[s - tau:]] = 0.0
    return keep.reshape(n, n)


def amplitudes(lam, keep=None):
    """a = sqrt(Lambda)/n (the unitary 1/sqrt(s) folded in), times the mask."""
    n = lam.shape[0]
    a = np.sqrt(np.maximum(lam, 0.0)) / n
    if keep is not None:
        a = a * keep
    return a
