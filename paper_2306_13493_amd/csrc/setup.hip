// Plan set-up on the device (Algorithm 1 steps 1-3): the first column of
// the circulant embedding from the covariance function, the orbit
// symmetrisation of its eigenvalues with their extremes and count of
// negatives, and the amplitudes sqrt(Lambda)/n of Algorithm 1 step 4(b)
// with the smoothing masks of Algorithm 2.
#include "besselk.hpp"
#include "internal.hpp"

namespace ces {

namespace {

// Matern, eq. (matern-cov-function), with the closed forms of nu = 1/2,
// 3/2, 5/2; separable exponential, eq. (p-norm-cov-function) with p = 1.
__device__ double cov_eval(const CovParams& c, double t1, double t2) {
    if (c.kind == COV_SEPEXP) return c.sigma2 * exp(-(fabs(t1) + fabs(t2)) / c.lam);
    const double r = sqrt(t1 * t1 + t2 * t2);
    const double x = sqrt(2.0 * c.nu) * r / c.lam;
    if (x == 0.0) return c.sigma2;
    if (c.nu == 0.5) return c.sigma2 * exp(-x);
    if (c.nu == 1.5) return c.sigma2 * (1.0 + x) * exp(-x);
    if (c.nu == 2.5) return c.sigma2 * (1.0 + x + x * x / 3.0) * exp(-x);
    if (x > 700.0) return 0.0;
    return c.pref * pow(x, c.nu) * bessel_k(c.nu, x);
}

__device__ double eta(double x) { return x > 0.0 ? exp(-1.0 / x) : 0.0; }

// One thread per quadrant offset (a, b), 0 <= a, b <= n/2; the column is
// even in each index, so the value is written at (+-a, +-b) mod n.
__global__ __launch_bounds__(kBlock) void k_cov_column(double* __restrict__ s, int n, int m, int J, int reading,
                                                       CovParams c) {
    const int nh = n / 2;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)(nh + 1) * (nh + 1)) return;
    const int b = (int)(t / (nh + 1)), a = (int)(t - (long long)b * (nh + 1));
    const double h = 1.0 / m;
    double v;
    if (J == 0) {
        v = cov_eval(c, a * h, b * h);
    } else {
        // smooth periodisation with period 2 ell (Section 2.2): the four
        // images of the offset that can lie inside the cutoff radius kappa
        const double ell = 1.0 + (double)J / m;
        const double lo = reading == PERIOD_INF ? 1.0 : sqrt(2.0);
        const double kappa = reading == PERIOD_INF ? 2.0 * ell - 1.0 : 2.0 * ell - sqrt(2.0);
        const double wdt = kappa - lo;
        v = 0.0;
        for (int s2 = 0; s2 >= -1; --s2)
            for (int s1 = 0; s1 >= -1; --s1) {
                const double y1 = a * h + 2.0 * ell * s1, y2 = b * h + 2.0 * ell * s2;
                const double r = reading == PERIOD_INF ? fmax(fabs(y1), fabs(y2)) : sqrt(y1 * y1 + y2 * y2);
                if (r >= kappa) continue;
                const double ea = eta((kappa - r) / wdt), eb = eta((r - lo) / wdt);
                v += cov_eval(c, y1, y2) * (ea / (ea + eb));
            }
    }
    const int a2 = (n - a) % n, b2 = (n - b) % n;
    s[(size_t)b * n + a] = v;
    if (a2 != a) s[(size_t)b * n + a2] = v;
    if (b2 != b) {
        s[(size_t)b2 * n + a] = v;
        if (a2 != a) s[(size_t)b2 * n + a2] = v;
    }
}

constexpr int kSymPerThread = 4;

__global__ __launch_bounds__(kBlock) void k_symmetrise(const double* __restrict__ lam, double* __restrict__ out,
                                                       int n, double* bmin, double* bmax, int* bneg) {
    __shared__ double red[kBlock / 64];
    const long long nn = (long long)n * n;
    const long long base = (long long)blockIdx.x * kBlock * kSymPerThread;
    double lo = 1e308, hi = -1e308;
    double neg = 0.0;
    for (int i = 0; i < kSymPerThread; ++i) {
        const long long k = base + (long long)i * kBlock + threadIdx.x;
        if (k >= nn) break;
        const int k2 = (int)(k / n), k1 = (int)(k - (long long)k2 * n);
        const int p = min(k1, n - k1), q = min(k2, n - k2);
        const int r1 = min(p, q), r2 = max(p, q);
        const double v = lam[(size_t)r2 * n + r1];
        out[k] = v;
        lo = fmin(lo, v);
        hi = fmax(hi, v);
        neg += v < 0.0 ? 1.0 : 0.0;
    }
    hi = block_max(hi, red);
    lo = -block_max(-lo, red);
    neg = block_sum(neg, red);
    if (threadIdx.x == 0) {
        bmin[blockIdx.x] = lo;
        bmax[blockIdx.x] = hi;
        bneg[blockIdx.x] = (int)neg;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_amplitudes(double* __restrict__ lam, long long nn, double n,
                                                       const uint8_t* __restrict__ keep_f,
                                                       const uint8_t* __restrict__ keep_c, T* __restrict__ af,
                                                       T* __restrict__ ac) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nn) return;
    const double v = fmax(lam[k], 0.0);
    lam[k] = v;
    const double a = sqrt(v) / n;
    af[k] = (T)((keep_f == nullptr || keep_f[k]) ? a : 0.0);
    if (ac) ac[k] = (T)((keep_c == nullptr || keep_c[k]) ? a : 0.0);
}

}  // namespace

hipError_t launch_cov_column(double* s, int n, int m, int J, int reading, const CovParams& c, hipStream_t st) {
    const long long q = (long long)(n / 2 + 1) * (n / 2 + 1);
    hipLaunchKernelGGL(k_cov_column, dim3(cdiv(q, kBlock)), dim3(kBlock), 0, st, s, n, m, J, reading, c);
    return hipGetLastError();
}

int symmetrise_blocks(int n) { return (int)cdiv((long long)n * n, (long long)kBlock * kSymPerThread); }

hipError_t launch_symmetrise(const double* lam, double* out, int n, double* bmin, double* bmax, int* bneg,
                             int* nblk, hipStream_t st) {
    const int nb = symmetrise_blocks(n);
    hipLaunchKernelGGL(k_symmetrise, dim3(nb), dim3(kBlock), 0, st, lam, out, n, bmin, bmax, bneg);
    *nblk = nb;
    return hipGetLastError();
}

template <typename T>
hipError_t launch_amplitudes(double* lam, int n, const uint8_t* keep_f, const uint8_t* keep_c, T* af, T* ac,
                             hipStream_t st) {
    const long long nn = (long long)n * n;
    hipLaunchKernelGGL(k_amplitudes<T>, dim3(cdiv(nn, kBlock)), dim3(kBlock), 0, st, lam, nn, (double)n, keep_f,
                       keep_c, af, ac);
    return hipGetLastError();
}
template hipError_t launch_amplitudes<float>(double*, int, const uint8_t*, const uint8_t*, float*, float*,
                                             hipStream_t);
template hipError_t launch_amplitudes<double>(double*, int, const uint8_t*, const uint8_t*, double*, double*,
                                              hipStream_t);

}  // namespace ces
