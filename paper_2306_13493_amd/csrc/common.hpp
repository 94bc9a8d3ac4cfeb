// Shared device/host helpers of the cesmlmc HIP library (gfx950).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace ces {

template <typename T>
struct alignas(2 * sizeof(T)) cplx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// multiply by +i
template <typename T>
__device__ __forceinline__ cplx<T> cmuli(cplx<T> a) { return {-a.y, a.x}; }

constexpr int kBlock = 256;  // threads per workgroup of every kernel here

// Deterministic block-wide sum (fixed shuffle tree within each wave64, then
// waves in order).  `red` must hold kBlock/64 values.  All threads get it.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    T s = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    __syncthreads();
    return s;
}

// Two block-wide sums in one pass (same order as block_sum for each).
template <typename T>
__device__ __forceinline__ void block_sum2(T& a, T& b, T* red2) {
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off, 64);
        b += __shfl_down(b, off, 64);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (int)(blockDim.x >> 6);
    __syncthreads();
    if (lane == 0) {
        red2[wid] = a;
        red2[nw + wid] = b;
    }
    __syncthreads();
    T sa = red2[0], sb = red2[nw];
    for (int w = 1; w < nw; ++w) {
        sa += red2[w];
        sb += red2[nw + w];
    }
    __syncthreads();
    a = sa;
    b = sb;
}

template <typename T>
__device__ __forceinline__ T block_max(T v, T* red) {
    for (int off = 32; off > 0; off >>= 1) {
        T o = __shfl_down(v, off, 64);
        v = o > v ? o : v;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    T s = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) s = red[w] > s ? red[w] : s;
    __syncthreads();
    return s;
}

// Work-item index of workgroup b in a 1-D grid of nb workgroups such that
// each of the 8 XCDs (which receive workgroups round-robin, each with its
// own L2) processes one contiguous range of work items: neighbouring tiles
// of a sample then share an L2 and their halo rows are fetched once.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    constexpr int NX = 8;
    const int per = nb / NX, rem = nb - per * NX;
    const int x = b % NX, j = b / NX;
    return x * per + (x < rem ? x : rem) + j;
}

inline unsigned cdiv(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

// Division by a runtime divisor d >= 1 as one multiply-high: with
// M = ceil(2^32 / d), umulhi(x, M) = floor(x / d) whenever x (M d - 2^32)
// < 2^32, and M d - 2^32 < d, so every x with x d < 2^32 is exact (d = 1
// keeps M = 0 and returns x).  Replaces the ~15-instruction integer
// division sequence in per-element index arithmetic.
struct FastDiv {
    unsigned d, M;
    FastDiv() = default;   // trivial, so that LDS arrays of it are allowed
    __host__ __device__ explicit FastDiv(unsigned dv) : d(dv), M(dv <= 1u ? 0u : 0xFFFFFFFFu / dv + 1u) {}
    __device__ __forceinline__ int div(int x) const { return M ? (int)__umulhi((unsigned)x, M) : x; }
};

// a * b for 0 <= a, b < 2^24 with a product below 2^31, on the full-rate
// 24-bit multiplier (a 32-bit integer multiply issues at a quarter rate)
__device__ __forceinline__ int mul24(int a, int b) { return (int)__umul24((unsigned)a, (unsigned)b); }

// Opt a kernel in to more than 64 KiB of dynamic LDS (gfx950 has 160 KiB).
template <typename KernelT>
hipError_t allow_lds(KernelT kernel, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace ces
