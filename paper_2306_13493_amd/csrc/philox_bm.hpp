// Counter-based normals for the field sample (Algorithm 1 step 4(a)).
//
// Philox4x32-10 as defined by Salmon, Moraes, Dror and Shaw, "Parallel
// random numbers: as easy as 1, 2, 3" (SC'11): per round two 32x32->64-bit
// products with multipliers 0xD2511F53 and 0xCD9E8D57, the key bumped by
// 0x9E3779B9 and 0xBB67AE85 between rounds, ten rounds.
//
// key = (seed mod 2^32, seed >> 32); counter = (e, q mod 2^32, q >> 32,
// stream) with e the embedding element, q the pair (or sample) index and
// stream the level tag.  Words x0..x3 become U1 = (x1 2^21 + x0/2^11 + 1)
// 2^-53 in (0,1] and U2 = (x3 2^21 + x2/2^11) 2^-53 in [0,1), then the
// Box-Muller pair (rho cos 2piU2, rho sin 2piU2), rho = sqrt(-2 ln U1).
//
// ln, sqrt, cos, sin are evaluated from their series / Newton definitions
// with IEEE double +, -, * and exact power-of-two scalings only: no
// division, no library call and no contraction into fused multiply-adds,
// so the values are reproducible bit for bit by any IEEE double machine
// that performs the same operations in the same order.
//   ln u   = e ln2 + 2 atanh t, u = 2^e f, f in [sqrt2/2, sqrt2],
//            t = (f-1)/(f+1), 1/(f+1) by five Newton steps from 1/2,
//            atanh by its odd series to t^23
//   sqrt x = x rsqrt(x): four Newton steps from the exponent-halving seed,
//            one Newton step on the root
//   cos, sin of 2 pi u: exact quadrant q = floor(4u + 1/2), r = 4u - q,
//            Taylor series in phi = r pi/2 to phi^20 / phi^19
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ces {

__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                              uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c0 = n0;
        c1 = (uint32_t)p1;
        c2 = n2;
        c3 = (uint32_t)p0;
    }
}

namespace bm {
__device__ __forceinline__ double ln(double u) {
#pragma clang fp contract(off)
    const long long b = __double_as_longlong(u);
    long long e = ((b >> 52) & 0x7FF) - 1023;
    double f = __longlong_as_double((b & 0x000FFFFFFFFFFFFFll) | 0x3FF0000000000000ll);
    if (f > 0x1.6a09e667f3bcdp+0) {
        f = f * 0.5;
        e = e + 1;
    }
    const double d = f + 1.0;
    double r = 0.5;
#pragma unroll
    for (int i = 0; i < 5; ++i) r = r + r * (1.0 - d * r);
    const double t = (f - 1.0) * r;
    const double z = t * t;
    double p = 0x1.642c8590b2164p-5;  // 1/23
    p = 0x1.8618618618618p-5 + z * p;  // 1/21
    p = 0x1.af286bca1af28p-5 + z * p;  // 1/19
    p = 0x1.e1e1e1e1e1e1ep-5 + z * p;  // 1/17
    p = 0x1.1111111111111p-4 + z * p;  // 1/15
    p = 0x1.3b13b13b13b14p-4 + z * p;  // 1/13
    p = 0x1.745d1745d1746p-4 + z * p;  // 1/11
    p = 0x1.c71c71c71c71cp-4 + z * p;  // 1/9
    p = 0x1.2492492492492p-3 + z * p;  // 1/7
    p = 0x1.999999999999ap-3 + z * p;  // 1/5
    p = 0x1.5555555555555p-2 + z * p;  // 1/3
    const double lnf = (t + t * (z * p)) * 2.0;
    const double ef = (double)e;
    return ef * 0x1.62e42fe000000p-1 + (ef * 0x1.f473de6af278fp-30 + lnf);
}

__device__ __forceinline__ double sqrt_nr(double x) {
#pragma clang fp contract(off)
    const unsigned long long xb = (unsigned long long)__double_as_longlong(x);
    double y = __longlong_as_double((long long)(0x5FE6EB50C7B537A9ull - (xb >> 1)));
    const double hx = x * 0.5;
#pragma unroll
    for (int i = 0; i < 4; ++i) y = y * (1.5 - (hx * y) * y);
    const double s = x * y;
    return s + (x - s * s) * (y * 0.5);
}

__device__ __forceinline__ void sincos_2pi(double u, double& c_out, double& s_out) {
#pragma clang fp contract(off)
    const double v = u * 4.0;
    const double q = floor(v + 0.5);
    const double r = v - q;
    const double phi = r * 0x1.921fb54442d18p+0;
    const double z = phi * phi;
    // sine series, Horner from the highest coefficient (-1)^k/(2k+1)!
    double sp = -0x1.2f49b46814157p-57;     // k=9: -1/19!
    sp = 0x1.952c77030ad4ap-49 + z * sp;    // k=8: +1/17!
    sp = -0x1.ae7f3e733b81fp-41 + z * sp;   // k=7: -1/15!
    sp = 0x1.6124613a86d09p-33 + z * sp;    // k=6: +1/13!
    sp = -0x1.ae64567f544e4p-26 + z * sp;   // k=5: -1/11!
    sp = 0x1.71de3a556c734p-19 + z * sp;    // k=4: +1/9!
    sp = -0x1.a01a01a01a01ap-13 + z * sp;   // k=3: -1/7!
    sp = 0x1.1111111111111p-7 + z * sp;     // k=2: +1/5!
    sp = -0x1.5555555555555p-3 + z * sp;    // k=1: -1/3!
    const double s = phi + phi * (z * sp);
    // cosine series, (-1)^k/(2k)!
    double cp = 0x1.e542ba4020225p-62;      // k=10: +1/20!
    cp = -0x1.6827863b97d97p-53 + z * cp;   // k=9: -1/18!
    cp = 0x1.ae7f3e733b81fp-45 + z * cp;    // k=8: +1/16!
    cp = -0x1.93974a8c07c9dp-37 + z * cp;   // k=7: -1/14!
    cp = 0x1.1eed8eff8d898p-29 + z * cp;    // k=6: +1/12!
    cp = -0x1.27e4fb7789f5cp-22 + z * cp;   // k=5: -1/10!
    cp = 0x1.a01a01a01a01ap-16 + z * cp;    // k=4: +1/8!
    cp = -0x1.6c16c16c16c17p-10 + z * cp;   // k=3: -1/6!
    cp = 0x1.5555555555555p-5 + z * cp;     // k=2: +1/4!
    cp = -0x1.0000000000000p-1 + z * cp;    // k=1: -1/2!
    const double c = 1.0 + z * cp;
    const int qi = ((int)q) & 3;
    if (qi == 0) { c_out = c;  s_out = s; }
    else if (qi == 1) { c_out = -s; s_out = c; }
    else if (qi == 2) { c_out = -c; s_out = -s; }
    else { c_out = s; s_out = -c; }
}
}  // namespace bm

// (g0, g1) of element e for pair/sample q, level tag `stream`, key `seed`.
__device__ __forceinline__ void normal_pair(uint64_t seed, uint64_t q, uint32_t stream, uint32_t e,
                                            double& g0, double& g1) {
#pragma clang fp contract(off)
    uint32_t c0 = e, c1 = (uint32_t)q, c2 = (uint32_t)(q >> 32), c3 = stream;
    philox4x32_10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
    const uint64_t a = (((uint64_t)c1 << 21) + (uint64_t)(c0 >> 11)) + 1ull;
    const uint64_t b = ((uint64_t)c3 << 21) + (uint64_t)(c2 >> 11);
    const double u1 = (double)a * 0x1.0p-53;
    const double u2 = (double)b * 0x1.0p-53;
    const double rho = bm::sqrt_nr(bm::ln(u1) * -2.0);
    double c, s;
    bm::sincos_2pi(u2, c, s);
    g0 = rho * c;
    g1 = rho * s;
}

}  // namespace ces
