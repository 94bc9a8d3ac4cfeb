"""Seeded standard normals for Algorithm 1 step 4(a) (oracle; test only).

The paper does not name its generator.  Reading used here: Philox4x32-10 of Salmon, Moraes, Dror and Shaw (SC'11,
"Parallel random numbers: as easy as 1, 2, 3"), written from that paper's
definition: two 32x32->64 multiplies per round with multipliers
0xD2511F53 and 0xCD9E8D57, key schedule bumped by the Weyl constants
0x9E3779B9 and 0xBB67AE85, ten rounds.

key     = (seed mod 2^32, seed >> 32)
counter = (e, q mod 2^32, q >> 32, stream)
  e      draw index: the element index j1 + n j2 of the embedding in PAIR
         mode (one complex normal per element), half of it in HARTLEY
         mode (elements 2d and 2d+1 take the two outputs of draw d)
  q      pair index (PAIR mode) or sample index (HARTLEY mode)
  stream level tag of the request

Words x0..x3 give two uniforms with 53 random bits each
  U1 = (x1 2^21 + floor(x0 / 2^11) + 1) 2^-53   in (0, 1]
  U2 = (x3 2^21 + floor(x2 / 2^11)) 2^-53       in [0, 1)
and the Box-Muller pair g0 = rho cos(theta), g1 = rho sin(theta) with
rho = sqrt(-2 ln U1) and theta = 2 pi U2.

ln, sqrt, cos and sin below are written from their series / Newton
definitions with IEEE float64 +, -, * and exact scalings by powers of two
only (no division, no library call, no fused multiply-add), so any IEEE
machine that performs the same operations in the same order gets the same
bits.  The GPU path implements the same definitions independently.

Pins (tests/test_oracle_normals.py): Philox words against rocRAND's
Philox4x32-10 engine compiled for the host; ln within 4 ulp, sqrt within
2 ulp, cos/sin within 4 units of 2^-52
of libm; moments and Kolmogorov-Smirnov of the normals.
"""

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32-10 on uint32 arrays (as uint64 holders); returns 4 arrays."""
    c0 = np.asarray(c0, dtype=np.uint64) & MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & MASK32
    k0 = np.asarray(k0, dtype=np.uint64) & MASK32
    k1 = np.asarray(k1, dtype=np.uint64) & MASK32
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + W0) & MASK32
            k1 = (k1 + W1) & MASK32
        p0 = M0 * c0  # < 2^64, exact in uint64
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return c0, c1, c2, c3


# ---- float64 constants (hex literals of correctly rounded values) --------
_f = float.fromhex
LN2_HI = _f("0x1.62e42fe000000p-1")   # ln 2 truncated to 28 bits
LN2_LO = _f("0x1.f473de6af278fp-30")  # ln 2 - LN2_HI
SQRT2 = _f("0x1.6a09e667f3bcdp+0")
PI_2 = _f("0x1.921fb54442d18p+0")     # pi / 2
# 1/(2k+1), k = 1..11: atanh series of ln
INV_ODD = [_f(x) for x in (
    "0x1.5555555555555p-2", "0x1.999999999999ap-3", "0x1.2492492492492p-3",
    "0x1.c71c71c71c71cp-4", "0x1.745d1745d1746p-4", "0x1.3b13b13b13b14p-4",
    "0x1.1111111111111p-4", "0x1.e1e1e1e1e1e1ep-5", "0x1.af286bca1af28p-5",
    "0x1.8618618618618p-5", "0x1.642c8590b2164p-5")]
# (-1)^k/(2k+1)!, k = 1..9: sine series
SIN_C = [(-1.0) ** k * _f(x) for k, x in enumerate((
    "0x1.5555555555555p-3", "0x1.1111111111111p-7", "0x1.a01a01a01a01ap-13",
    "0x1.71de3a556c734p-19", "0x1.ae64567f544e4p-26", "0x1.6124613a86d09p-33",
    "0x1.ae7f3e733b81fp-41", "0x1.952c77030ad4ap-49", "0x1.2f49b46814157p-57"),
    start=1)]
# (-1)^k/(2k)!, k = 1..10: cosine series
COS_C = [(-1.0) ** k * _f(x) for k, x in enumerate((
    "0x1.0000000000000p-1", "0x1.5555555555555p-5", "0x1.6c16c16c16c17p-10",
    "0x1.a01a01a01a01ap-16", "0x1.27e4fb7789f5cp-22", "0x1.1eed8eff8d898p-29",
    "0x1.93974a8c07c9dp-37", "0x1.ae7f3e733b81fp-45", "0x1.6827863b97d97p-53",
    "0x1.e542ba4020225p-62"), start=1)]
RSQRT_MAGIC = np.uint64(0x5FE6EB50C7B537A9)


def _bits(x):
    return np.asarray(x, dtype=np.float64).view(np.uint64)


def _from_bits(b):
    return np.asarray(b, dtype=np.uint64).view(np.float64)


def ln(u):
    """Natural log of u in (0, 2^1023) for normal u.

    u = 2^e f with f in [sqrt(2)/2, sqrt(2)];  ln u = e ln 2 + 2 atanh(t),
    t = (f-1)/(f+1).  1/(f+1) by Newton's iteration r <- r + r (1 - d r)
    from r = 1/2 (five steps: relative error 0.21 -> 1e-22).
    """
    u = np.asarray(u, dtype=np.float64)
    b = _bits(u)
    e = ((b >> np.uint64(52)) & np.uint64(0x7FF)).astype(np.int64) - 1023
    f = _from_bits((b & np.uint64(0x000FFFFFFFFFFFFF)) | np.uint64(0x3FF0000000000000))
    big = f > SQRT2
    f = np.where(big, f * 0.5, f)
    e = np.where(big, e + 1, e)
    d = f + 1.0
    r = np.full_like(d, 0.5)
    for _ in range(5):
        r = r + r * (1.0 - d * r)
    t = (f - 1.0) * r
    z = t * t
    p = INV_ODD[10]
    for c in INV_ODD[9::-1]:
        p = c + z * p
    lnf = (t + t * (z * p)) * 2.0
    ef = e.astype(np.float64)
    return ef * LN2_HI + (ef * LN2_LO + lnf)


def sqrt(x):
    """sqrt(x) for x >= 0 by x * rsqrt(x); rsqrt by four Newton steps
    y <- y (3/2 - (x/2) y y) from the classical exponent-halving seed, then
    one Newton step on the root itself, s <- s + (x - s s) (y/2)."""
    x = np.asarray(x, dtype=np.float64)
    y = _from_bits(RSQRT_MAGIC - (_bits(x) >> np.uint64(1)))
    hx = x * 0.5
    for _ in range(4):
        y = y * (1.5 - (hx * y) * y)
    s = x * y
    return s + (x - s * s) * (y * 0.5)


def sincos_2pi(u):
    """(cos(2 pi u), sin(2 pi u)) for u in [0, 1).

    Quadrant q = floor(4u + 1/2) and remainder r = 4u - q in [-1/2, 1/2]
    are exact; phi = r pi/2 in [-pi/4, pi/4]; Taylor series of sin and cos.
    """
    u = np.asarray(u, dtype=np.float64)
    v = u * 4.0
    q = np.floor(v + 0.5)
    r = v - q
    phi = r * PI_2
    z = phi * phi
    ps = SIN_C[8]
    for c in SIN_C[7::-1]:
        ps = c + z * ps
    s = phi + phi * (z * ps)
    pc = COS_C[9]
    for c in COS_C[8::-1]:
        pc = c + z * pc
    c = 1.0 + z * pc
    qi = q.astype(np.int64) & 3
    cos_t = np.select([qi == 0, qi == 1, qi == 2], [c, -s, -c], s)
    sin_t = np.select([qi == 0, qi == 1, qi == 2], [s, c, -s], -c)
    return cos_t, sin_t


def uniforms(x0, x1, x2, x3):
    """Two 53-bit uniforms U1 in (0,1], U2 in [0,1) from four Philox words."""
    two21 = np.uint64(1 << 21)
    a = (x1 * two21 + (x0 >> np.uint64(11))) + np.uint64(1)
    b = x3 * two21 + (x2 >> np.uint64(11))
    scale = 2.0 ** -53
    return a.astype(np.float64) * scale, b.astype(np.float64) * scale


def box_muller(u1, u2):
    """g0 = sqrt(-2 ln u1) cos(2 pi u2), g1 = sqrt(-2 ln u1) sin(2 pi u2)."""
    rho = sqrt(ln(u1) * -2.0)
    c, s = sincos_2pi(u2)
    return rho * c, rho * s


def normals(seed, q, stream, e):
    """(g0, g1) for elements e (array), pair/sample index q, level tag."""
    e = np.asarray(e, dtype=np.uint64)
    seed = int(seed)
    q = int(q)
    x0, x1, x2, x3 = philox4x32_10(
        e, np.uint64(q & 0xFFFFFFFF), np.uint64((q >> 32) & 0xFFFFFFFF),
        np.uint64(int(stream) & 0xFFFFFFFF),
        np.uint64(seed & 0xFFFFFFFF), np.uint64((seed >> 32) & 0xFFFFFFFF))
    u1, u2 = uniforms(x0, x1, x2, x3)
    return box_muller(u1, u2)
