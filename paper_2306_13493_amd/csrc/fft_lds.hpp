// Workgroup-local 1-D DFTs in LDS (the transforms of Algorithm 1 steps 3
// and 4(c), taken one axis at a time as in Section 2.1.2).
//
// Sign: V_p = sum_j v_j exp(+2 pi i j p / N) (the Fourier matrix of the
// paper has a positive exponent); no normalisation.
//
// Mixed-radix (8, 4, 2, 3) Stockham autosort: stage with radix R over
// sub-length Ns takes inputs v_r = x[j + r N/R], twiddles them by
// W_{Ns R}^{r k} (k = j mod Ns), applies the R-point DFT and writes
// y[(j - k) R + k + r Ns].  One LDS buffer: each thread first reads all its
// butterflies of the stage into registers, the workgroup synchronises, then
// writes -- so L lines of N points need only L N complex words of LDS.
// Twiddles come from a table tw[t] = exp(+2 pi i t / N) computed in double
// on the host (rounded once to float for the float transforms).
#pragma once

#include "common.hpp"

namespace ces {

// nr[s], ns[s]: divisions by N / R and by Ns of stage s (the butterfly
// indices stay below lines * N <= E * blockDim <= 8192 and the divisors
// below 8192: within FastDiv's exact range)
struct FftPlan {
    int n;
    int nst;
    int rad[24];
    FastDiv nr[24], ns[24];
};

inline FftPlan make_fft_plan(int n) {
    FftPlan p{};
    p.n = n;
    int r = n;
    while (r % 8 == 0 && r > 1) { p.rad[p.nst++] = 8; r /= 8; }
    while (r % 4 == 0 && r > 1) { p.rad[p.nst++] = 4; r /= 4; }
    if (r % 2 == 0) { p.rad[p.nst++] = 2; r /= 2; }
    while (r % 3 == 0) { p.rad[p.nst++] = 3; r /= 3; }
    if (r != 1) {
        p.nst = -1;  // unsupported size
        return p;
    }
    int Ns = 1;
    for (int s = 0; s < p.nst; ++s) {
        p.nr[s] = FastDiv((unsigned)(n / p.rad[s]));
        p.ns[s] = FastDiv((unsigned)Ns);
        Ns *= p.rad[s];
    }
    return p;
}

template <typename T, int R>
__device__ __forceinline__ void dft_small(cplx<T>* v) {
    if constexpr (R == 2) {
        const cplx<T> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 4) {
        const cplx<T> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
        const cplx<T> t2 = cadd(v[1], v[3]), t3 = csub(v[1], v[3]);
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, cmuli(t3));
        v[3] = csub(t1, cmuli(t3));
    } else if constexpr (R == 8) {
        // two 4-point DFTs (even, odd inputs), odd ones twiddled by
        // W8^k = exp(+2 pi i k / 8), then 2-point butterflies
        cplx<T> e[4] = {v[0], v[2], v[4], v[6]};
        cplx<T> o[4] = {v[1], v[3], v[5], v[7]};
        dft_small<T, 4>(e);
        dft_small<T, 4>(o);
        const T c = T(0.70710678118654752440);   // 1/sqrt(2)
        const cplx<T> o1 = {c * (o[1].x - o[1].y), c * (o[1].x + o[1].y)};     // (1+i)/sqrt2
        const cplx<T> o2 = cmuli(o[2]);                                        // i
        const cplx<T> o3 = {-c * (o[3].x + o[3].y), c * (o[3].x - o[3].y)};    // (-1+i)/sqrt2
        v[0] = cadd(e[0], o[0]);
        v[4] = csub(e[0], o[0]);
        v[1] = cadd(e[1], o1);
        v[5] = csub(e[1], o1);
        v[2] = cadd(e[2], o2);
        v[6] = csub(e[2], o2);
        v[3] = cadd(e[3], o3);
        v[7] = csub(e[3], o3);
    } else {  // R == 3, W = exp(+2 pi i / 3)
        const T h = T(0.5);
        const T s3 = T(0.86602540378443864676);  // sqrt(3)/2
        const cplx<T> a = v[0];
        const cplx<T> sum = cadd(v[1], v[2]);
        const cplx<T> dif = csub(v[1], v[2]);
        const cplx<T> m = {a.x - h * sum.x, a.y - h * sum.y};
        const cplx<T> rot = {-s3 * dif.y, s3 * dif.x};  // i sqrt(3)/2 (b - c)
        v[0] = cadd(a, sum);
        v[1] = cadd(m, rot);
        v[2] = csub(m, rot);
    }
}

// One Stockham stage over `lines` lines of length n in buf, line l at
// buf + l * ld (ld >= n; a padded stride spreads lines over the LDS banks).
// MB = maximum butterflies per thread (compile time, registers).
template <typename T, int R, int MB>
__device__ __forceinline__ void fft_stage(cplx<T>* buf, int n, int ld, int lines, int Ns, FastDiv dnr,
                                          FastDiv dns, const cplx<T>* __restrict__ tw) {
    const int NR = n / R;
    const int total = NR * lines;
    const int stride = n / (Ns * R);
    // index arithmetic once per butterfly, before the barrier (all indices
    // and products stay below 2^24: lines * n <= 8192, ld <= 8193)
    cplx<T> v[MB][R];
    int yo[MB], kt[MB];
#pragma unroll
    for (int b = 0; b < MB; ++b) {
        const int g = threadIdx.x + b * (int)blockDim.x;
        if (g < total) {
            const int line = dnr.div(g);
            const int j = g - mul24(line, NR);
            const int k = j - mul24(dns.div(j), Ns);
            const int lo = mul24(line, ld);
            const cplx<T>* x = buf + lo;
#pragma unroll
            for (int r = 0; r < R; ++r) v[b][r] = x[j + mul24(r, NR)];
            yo[b] = lo + (j - k) * R + k;
            kt[b] = mul24(k, stride);
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < MB; ++b) {
        const int g = threadIdx.x + b * (int)blockDim.x;
        if (g < total) {
            if (Ns > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) v[b][r] = cmul(v[b][r], tw[mul24(r, kt[b])]);
            }
            dft_small<T, R>(v[b]);
            cplx<T>* y = buf + yo[b];
#pragma unroll
            for (int r = 0; r < R; ++r) y[mul24(r, Ns)] = v[b][r];
        }
    }
    __syncthreads();
}

// In-place DFT of `lines` lines of length fp.n in LDS, line l at buf + l * ld.
// E bounds the complex values per thread: lines * n <= E * blockDim.x.
template <typename T, int E>
__device__ void fft_lines(cplx<T>* buf, int lines, int ld, const FftPlan& fp, const cplx<T>* __restrict__ tw) {
    int Ns = 1;
    for (int s = 0; s < fp.nst; ++s) {
        const int R = fp.rad[s];
        if (R == 8)
            fft_stage<T, 8, (E + 7) / 8>(buf, fp.n, ld, lines, Ns, fp.nr[s], fp.ns[s], tw);
        else if (R == 4)
            fft_stage<T, 4, (E + 3) / 4>(buf, fp.n, ld, lines, Ns, fp.nr[s], fp.ns[s], tw);
        else if (R == 2)
            fft_stage<T, 2, (E + 1) / 2>(buf, fp.n, ld, lines, Ns, fp.nr[s], fp.ns[s], tw);
        else
            fft_stage<T, 3, (E + 2) / 3>(buf, fp.n, ld, lines, Ns, fp.nr[s], fp.ns[s], tw);
        Ns *= R;
    }
}

}  // namespace ces
