// Modified Bessel function of the second kind K_nu(x) for real nu and
// x > 0, needed by the Matern covariance (Section 2.1) for general nu.
//
// Method: the integral representation
//     K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt
// summed with the trapezoidal rule of step h.  The integrand is even and
// smooth, so the rule's relative error is about the ratio of its Fourier
// transform at 2 pi / h to its integral, i.e. |K_{nu + 2 pi i / h}(x)| /
// K_nu(x): like w^(nu - 1/2) exp(-pi w / 2) with w = 2 pi / h when x is
// small, and like exp(-w^2 / (2 x)) when x is large (the integrand is then
// a narrow bump of width 1/sqrt(x)).  h = min(0.15, 0.6 / sqrt(x)) keeps
// both below double rounding for the nu <= 5 of covariance models
// (checked against an independent implementation in the tests).  Terms
// are summed until the integrand is past its maximum (x sinh t >= nu) and
// below 1e-18 of the sum.  Overflow: nu t stays below 710 for nu <= 5.
//
// Plain C++ so that the same routine serves the device (covariance
// kernel) and a host build for testing.
#pragma once

#include <cmath>

#if defined(__HIPCC__)
#define CES_HD __host__ __device__
#else
#define CES_HD
#endif

namespace ces {

CES_HD inline double bessel_k(double nu, double x) {
    // exp(-x) is factored out and cosh t - 1 = 2 sinh^2(t/2) is formed
    // without cancellation, so large x loses no accuracy in the exponent
    const double h = fmin(0.15, 0.6 / sqrt(x));
    double sum = 0.5;   // t = 0, half weight
    for (int k = 1; k < 4000; ++k) {
        const double t = k * h;
        const double sh = sinh(0.5 * t);
        const double g = 2.0 * x * sh * sh;
        const double term = 0.5 * (exp(nu * t - g) + exp(-nu * t - g));
        sum += term;
        if (x * sinh(t) >= nu && term <= 1e-18 * sum) break;
    }
    return h * sum * exp(-x);
}

}  // namespace ces
