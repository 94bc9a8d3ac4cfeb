// Field sampling kernels: Algorithm 1 step 3 (FP64 eigenvalue DFT of the
// embedding's first column) and step 4(a)-(f) (normals, scaling by the
// square-root eigenvalues, 2-D DFT, Hartley / pair combination,
// restriction to the fine and coarse meshes, exponential).
//
// The 2-D DFT is two passes of workgroup-local 1-D DFTs (fft_lds.hpp):
//   y pass:  for each embedding column j1 (a workgroup takes L adjacent
//            ones), draw the normals, scale, transform along j2 and keep
//            only the m+1 outputs p2 <= m that the restriction reads; store
//            them as work[p2][j1] (L adjacent j1 per store: aligned 8L-byte
//            runs of complex values).
//   x pass:  for each kept p2 (a row of the mesh), transform along j1, keep
//            p1 <= m, combine and write exp(Z) at the mesh nodes: whole
//            mesh rows (and whole coarse rows at even p2) per store.
// Pruning the first pass to m+1 of n outputs cuts the intermediate and the
// second pass to (m+1)/n ~ 1/2..1/4 of a full transform.  LDS lines are
// padded by one complex value so that lines written across threads do not
// share a bank.
#include "internal.hpp"
#include "philox_bm.hpp"

namespace ces {

namespace {

int lowbit(int n) { return n & (-n); }
int pow2floor(int v) {
    int p = 1;
    while (p * 2 <= v) p *= 2;
    return p;
}

template <typename T>
__device__ __forceinline__ T dev_exp(T z);
template <>
__device__ __forceinline__ float dev_exp<float>(float z) {
#pragma clang fp contract(off)
    // e^z = 2^(z log2 e) on the hardware exp2 (v_exp_f32), with the
    // rounding error of the float product z log2 e (recovered by an FMA,
    // log2 e split into l2e + l2e_lo) applied to first order: about 2 ulp,
    // against ~10 instructions of the library expf's range reduction
    const float l2e = 0x1.715476p+0f, l2e_lo = 0x1.4ae0bep-26f;
    const float h = z * l2e;
    const float lo = fmaf(z, l2e_lo, fmaf(z, l2e, -h));
    const float r = __builtin_amdgcn_exp2f(h);
    return fmaf(r, lo * 0x1.62e430p-1f, r);
}
template <>
__device__ __forceinline__ double dev_exp<double>(double z) { return exp(z); }

// Index of the source embedding (size ns, period ns h_s) whose signed
// frequency is nearest to that of index j of an embedding of size n on the
// mesh of twice the spacing (period 2 n h_s): round(k * ns / (2 n)) with
// k = j or j - n, ties upwards, taken mod ns.  Injective for ns >= 2 n.
__device__ __forceinline__ int src_index(int j, int n, int ns) {
    const long long k = j < n / 2 ? j : j - n;
    const long long num = 2 * k * ns + 2LL * n, den = 4LL * n;
    const long long f = num >= 0 ? num / den : -((-num + den - 1) / den);
    return (int)(f >= 0 ? f : f + ns);
}

// Randomly shifted lattice coordinate j of the point whose radical inverse
// is qpt (64-bit fraction), shift r: U = (qpt z + D) mod 2^64 with D from
// Philox counter (j, r, 2^32-1, stream); u = (floor(U/2^12) + 1/2) 2^-52 in
// (0,1); the normal is Phi^-1(u).
__device__ __noinline__ double lattice_normal(uint64_t seed, uint32_t stream, uint64_t r, uint64_t qpt,
                                                 uint32_t z, uint32_t j) {
    uint32_t c0 = j, c1 = (uint32_t)r, c2 = 0xFFFFFFFFu, c3 = stream;
    philox4x32_10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
    const uint64_t D = (uint64_t)c0 | ((uint64_t)c1 << 32);
    const uint64_t U = qpt * (uint64_t)z + D;
    const double u = ((double)(U >> 12) + 0.5) * 0x1.0p-52;
    return normcdfinv(u);
}

// Embeddings up to this size keep their twiddle table in LDS behind the
// lines (n complex values), so that the DFT stages read twiddles at LDS
// latency; larger ones read the global table.
constexpr int kTwLds = 1024;

// line stride of the field kernels' LDS buffer (one slot of padding: the
// odd stride spreads the lines over the banks)
__host__ __device__ constexpr int field_ld(int n) { return n + 1; }

template <typename T>
inline size_t field_lds_bytes(int lines, int n) {
    return (size_t)lines * field_ld(n) * sizeof(cplx<T>) + (n <= kTwLds ? (size_t)n * sizeof(cplx<T>) : 0);
}

// DFT of the lines in buf, with the twiddles staged into LDS at twl (the
// workgroup synchronises first: the caller's stores into buf are complete)
template <typename T, int E>
__device__ __forceinline__ void field_fft(cplx<T>* buf, int lines, int ld, const FieldBatch<T>& b, cplx<T>* twl) {
    const int n = b.n;
    if (n <= kTwLds) {
        for (int t = threadIdx.x; t < n; t += blockDim.x) twl[t] = b.tw[t];
        __syncthreads();
        fft_lines<T, E>(buf, lines, ld, b.fp, twl);
    } else {
        __syncthreads();
        fft_lines<T, E>(buf, lines, ld, b.fp, b.tw);
    }
}

template <typename T, int E, int MODE, int NF>
__global__ __launch_bounds__(kBlock) void k_field_y(FieldBatch<T> b, int L) {
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
    const int n = b.n, ld = field_ld(n);
    const int u = blockIdx.y;
    const uint64_t q = b.q0 + (uint64_t)u;
    const int j1_0 = blockIdx.x * L;
    // lattice point (radical-inverse order, as a 64-bit fraction) and shift
    uint64_t qpt = 0, qsh = 0;
    if (MODE == MODE_HARTLEY && b.qrank) {
        const uint64_t i = q / (uint64_t)b.qshifts;
        qsh = q - i * (uint64_t)b.qshifts;
        qpt = __builtin_bitreverse64(i);
    }
    // scaled normal into line `line`, row j2 of the LDS buffer (and of the
    // coarse lines when a pair level takes two fields from one xi)
    // (mul24 operands below 2^24 and products below 2^31 throughout:
    // n <= 8192, L <= 16)
    auto put = [&](int line, int j2, uint32_t ia, double xr, double xi) {
        const double a = (double)b.af[ia];
        buf[mul24(line, ld) + j2] = cplx<T>{(T)(a * xr), (T)(a * xi)};
        if constexpr (NF == 2) {
            const double c = (double)b.ac[ia];
            buf[mul24(L + line, ld) + j2] = cplx<T>{(T)(c * xr), (T)(c * xi)};
        }
    };
    auto counter = [&](int j1, int j2) -> uint32_t {
        if (b.n_src > 0) return (uint32_t)src_index(j1, n, b.n_src) + (uint32_t)b.n_src * (uint32_t)src_index(j2, n, b.n_src);
        return (uint32_t)(j1 + mul24(n, j2));
    };
    if constexpr (MODE == MODE_PAIR) {
        // adjacent threads take adjacent j1 of one row j2 (coalesced
        // amplitude reads); line `line` of the LDS buffer is column j1_0 + line
        const FastDiv dL((unsigned)L);
        for (int t = threadIdx.x; t < L * n; t += blockDim.x) {
            const int j2 = dL.div(t);
            const int line = t - j2 * L;
            const int j1 = j1_0 + line;
            double g0, g1;
            normal_pair(b.seed, q, b.stream, counter(j1, j2), g0, g1);
            put(line, j2, (uint32_t)(j1 + mul24(n, j2)), g0, g1);
        }
    } else {
        // real xi: entry e takes output e & 1 of draw e >> 1, or a lattice
        // coordinate where the plan carries a lattice rule.  A thread takes
        // two adjacent lines when L >= 2: entries e, e + 1 with e even then
        // share one draw.
        const int W = L >= 2 ? 2 : 1;
        const int per = L / W;
        const FastDiv dper((unsigned)per);
        for (int t = threadIdx.x; t < per * n; t += blockDim.x) {
            const int j2 = dper.div(t);
            const int line = W * (t - j2 * per);
            const int j1 = j1_0 + line;
            const uint32_t e0 = counter(j1, j2);
            const uint32_t e1 = W == 2 ? counter(j1 + 1, j2) : e0;
            double x0, x1;
            {
                double g0, g1;
                normal_pair(b.seed, q, b.stream, e0 >> 1, g0, g1);
                x0 = (e0 & 1u) ? g1 : g0;
                x1 = g1;
            }
            if (W == 2 && !((e0 & 1u) == 0u && e1 == e0 + 1u)) {
                double g0, g1;
                normal_pair(b.seed, q, b.stream, e1 >> 1, g0, g1);
                x1 = (e1 & 1u) ? g1 : g0;
            }
            if (b.qrank) {
                const int jq0 = b.qrank[e0];
                if (jq0 >= 0) x0 = lattice_normal(b.seed, b.stream, qsh, qpt, b.qz[jq0], (uint32_t)jq0);
                const int jq1 = W == 2 ? b.qrank[e1] : -1;
                if (jq1 >= 0) x1 = lattice_normal(b.seed, b.stream, qsh, qpt, b.qz[jq1], (uint32_t)jq1);
            }
            const uint32_t ia = (uint32_t)(j1 + mul24(n, j2));
            put(line, j2, ia, x0, 0.0);
            if (W == 2) put(line + 1, j2, ia + 1u, x1, 0.0);
        }
    }
    field_fft<T, E>(buf, NF * L, ld, b, buf + (size_t)NF * L * ld);
    const int mp1 = b.m + 1;
    const FastDiv dL((unsigned)L), dm((unsigned)mp1);
    for (int t = threadIdx.x; t < NF * mp1 * L; t += blockDim.x) {
        const int rest = dL.div(t);
        const int line = t - rest * L;
        const int f = dm.div(rest);
        const int p2 = rest - f * mp1;
        cplx<T>* wf = b.work + (size_t)(f * b.units + u) * mp1 * n;
        wf[mul24(p2, n) + j1_0 + line] = buf[mul24(f * L + line, ld) + p2];
    }
}

template <typename T, int E, int MODE, int NF, bool ZOUT>
__global__ __launch_bounds__(kBlock) void k_field_x(FieldBatch<T> b, int L) {
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
    const int n = b.n, ld = field_ld(n);
    const int mp1 = b.m + 1;
    const int p2_0 = blockIdx.x * L;
    const int u = blockIdx.y;
    const int f = blockIdx.z;
    const int lines = min(L, mp1 - p2_0);
    const cplx<T>* src = b.work + ((size_t)(f * b.units + u) * mp1 + p2_0) * n;
    // all of the thread's loads are issued before the first LDS store, so
    // that their latencies overlap (lines * n <= E * kBlock)
    {
        const FastDiv dn((unsigned)n);
        cplx<T> v[E];
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int t = threadIdx.x + i * kBlock;
            if (t < lines * n) v[i] = src[t];
        }
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int t = threadIdx.x + i * kBlock;
            if (t < lines * n) {
                const int l = dn.div(t);
                buf[mul24(l, ld) + (t - mul24(l, n))] = v[i];
            }
        }
    }
    field_fft<T, E>(buf, lines, ld, b, buf + (size_t)L * ld);
    const bool fine = (f == 0);
    const bool coarse = b.coarse && (f == NF - 1);
    const int mcp1 = b.m / 2 + 1;
    // adjacent threads write adjacent p1 of one mesh row p2
    const FastDiv dm((unsigned)mp1);
    for (int t = threadIdx.x; t < lines * mp1; t += blockDim.x) {
        const int l = dm.div(t);
        const int p1 = t - mul24(l, mp1);
        const int p2 = p2_0 + l;
        const cplx<T> v = buf[mul24(l, ld) + p1];
        const bool even = ((p1 | p2) & 1) == 0;
        if (MODE == MODE_PAIR) {
            const T z0 = v.x, z1 = v.y;
            const size_t s0 = 2 * (size_t)u, s1 = s0 + 1;
            if (fine) {
                const int o = p1 + mul24(mp1, p2);
                if (ZOUT) {
                    b.zf[s0 * mp1 * mp1 + o] = (double)z0;
                    b.zf[s1 * mp1 * mp1 + o] = (double)z1;
                } else {
                    b.kf[s0 * b.kf_stride + o] = dev_exp<T>(z0);
                    b.kf[s1 * b.kf_stride + o] = dev_exp<T>(z1);
                }
            }
            if (coarse && even) {
                const int o = (p1 >> 1) + mul24(mcp1, p2 >> 1);
                if (ZOUT) {
                    b.zc[s0 * mcp1 * mcp1 + o] = (double)z0;
                    b.zc[s1 * mcp1 * mcp1 + o] = (double)z1;
                } else {
                    b.kc[s0 * b.kc_stride + o] = dev_exp<T>(z0);
                    b.kc[s1 * b.kc_stride + o] = dev_exp<T>(z1);
                }
            }
        } else {
            const T z = v.x + v.y;
            const size_t s0 = (size_t)u;
            if (fine) {
                const int o = p1 + mul24(mp1, p2);
                if (ZOUT) b.zf[s0 * mp1 * mp1 + o] = (double)z;
                else b.kf[s0 * b.kf_stride + o] = dev_exp<T>(z);
            }
            if (coarse && even) {
                const int o = (p1 >> 1) + mul24(mcp1, p2 >> 1);
                if (ZOUT) b.zc[s0 * mcp1 * mcp1 + o] = (double)z;
                else b.kc[s0 * b.kc_stride + o] = dev_exp<T>(z);
            }
        }
    }
}

template <int E>
__global__ __launch_bounds__(kBlock) void k_eig_rows(const double* __restrict__ s, int L, FftPlan fp,
                                                     const cplx<double>* __restrict__ tw,
                                                     cplx<double>* __restrict__ work) {
    extern __shared__ unsigned char smem_raw[];
    cplx<double>* buf = reinterpret_cast<cplx<double>*>(smem_raw);
    const int n = fp.n;
    const int j2_0 = blockIdx.x * L;
    for (int t = threadIdx.x; t < L * n; t += blockDim.x) {
        buf[t] = cplx<double>{s[(size_t)j2_0 * n + t], 0.0};
    }
    __syncthreads();
    fft_lines<double, E>(buf, L, n, fp, tw);
    for (int t = threadIdx.x; t < L * n; t += blockDim.x) {
        const int line = t % L;
        const int p1 = t / L;
        work[(size_t)p1 * n + j2_0 + line] = buf[line * n + p1];
    }
}

template <int E>
__global__ __launch_bounds__(kBlock) void k_eig_cols(const cplx<double>* __restrict__ work, int L, FftPlan fp,
                                                     const cplx<double>* __restrict__ tw,
                                                     double* __restrict__ lam, double* __restrict__ imag_blk) {
    extern __shared__ unsigned char smem_raw[];
    __shared__ double red[kBlock / 64];
    cplx<double>* buf = reinterpret_cast<cplx<double>*>(smem_raw);
    const int n = fp.n;
    const int p1_0 = blockIdx.x * L;
    for (int t = threadIdx.x; t < L * n; t += blockDim.x) buf[t] = work[(size_t)p1_0 * n + t];
    __syncthreads();
    fft_lines<double, E>(buf, L, n, fp, tw);
    double im = 0.0;
    for (int t = threadIdx.x; t < L * n; t += blockDim.x) {
        const int l = t % L;
        const int p2 = t / L;
        const cplx<double> v = buf[l * n + p2];
        lam[(size_t)p2 * n + p1_0 + l] = v.x;
        im = fmax(im, fabs(v.y));
    }
    im = block_max(im, red);
    if (threadIdx.x == 0) imag_blk[blockIdx.x] = im;
}

__global__ __launch_bounds__(kBlock) void k_normals(uint64_t seed, uint64_t q, uint32_t stream,
                                                    uint64_t first_e, long long count, double* out) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    double g0, g1;
    normal_pair(seed, q, stream, (uint32_t)(first_e + (uint64_t)t), g0, g1);
    out[2 * t] = g0;
    out[2 * t + 1] = g1;
}

__global__ __launch_bounds__(kBlock) void k_convert_d2f(const double* __restrict__ in, float* __restrict__ out,
                                                        long long count) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) out[t] = (float)in[t];
}

template <typename T, int E, int MODE, int NF>
hipError_t field_launch_e(const FieldBatch<T>& b, hipStream_t st, int L1, int L2) {
    const size_t lds1 = field_lds_bytes<T>(NF * L1, b.n);
    const size_t lds2 = field_lds_bytes<T>(L2, b.n);
    auto kr = k_field_y<T, E, MODE, NF>;
    hipError_t e = allow_lds(kr, lds1);
    if (e != hipSuccess) return e;
    // algorithmic bytes: amplitudes once, the pruned intermediate written
    // then read, k written at the fine (and coarse) nodes
    const double sT = sizeof(T);
    const double inter = (double)b.units * NF * (b.m + 1) * b.n * 2.0 * sT;
    const double slots = (double)b.units * (MODE == MODE_PAIR ? 2 : 1);
    const double kout = slots * sT * ((double)(b.m + 1) * (b.m + 1) +
                                      (b.coarse ? (double)(b.m / 2 + 1) * (b.m / 2 + 1) : 0.0));
    Profiler& P = Profiler::get();
    Profiler::Slot ps = P.begin("field_y");
    hipExtLaunchKernelGGL(kr, dim3(b.n / L1, b.units), dim3(kBlock), lds1, st, ps.a, ps.b, 0, b, L1);
    P.end(ps, "field_y", (double)NF * b.n * b.n * sT + inter, 1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    dim3 g2(cdiv(b.m + 1, L2), b.units, NF);
    ps = P.begin("field_x");
    if (b.zf) {
        auto kc = k_field_x<T, E, MODE, NF, true>;
        if ((e = allow_lds(kc, lds2)) != hipSuccess) return e;
        hipExtLaunchKernelGGL(kc, g2, dim3(kBlock), lds2, st, ps.a, ps.b, 0, b, L2);
    } else {
        auto kc = k_field_x<T, E, MODE, NF, false>;
        if ((e = allow_lds(kc, lds2)) != hipSuccess) return e;
        hipExtLaunchKernelGGL(kc, g2, dim3(kBlock), lds2, st, ps.a, ps.b, 0, b, L2);
    }
    P.end(ps, "field_x", inter + kout, 1);
    return hipGetLastError();
}

template <typename T, int MODE, int NF>
hipError_t field_launch_nf(const FieldBatch<T>& b, hipStream_t st) {
    // lines per workgroup: a power of two dividing n, with NF*L*n <= 16*256
    // values per workgroup (E = 16) when possible, else one line (E = 32).
    // The row pass takes as many lines as fit (its stores are runs of L
    // adjacent values); the column pass half as many, so that twice the
    // workgroups share a CU and overlap their loads with the others' DFT
    // stages (4 lines of n = 512: 3.6 -> 3.9 TB/s; 2 lines are slower again).
    const int cap = 16 * kBlock;
    int L1 = pow2floor(std::max(1, cap / (NF * b.n)));
    L1 = std::min(L1, lowbit(b.n));
    int L2 = pow2floor(std::max(1, cap / (2 * b.n)));
    if (NF * L1 * b.n <= cap && L2 * b.n <= cap) return field_launch_e<T, 16, MODE, NF>(b, st, L1, L2);
    if (NF * b.n <= 2 * cap) return field_launch_e<T, 32, MODE, NF>(b, st, 1, 1);
    return hipErrorInvalidValue;
}

}  // namespace

template <typename T>
hipError_t launch_field(const FieldBatch<T>& b, hipStream_t st) {
    if (b.units <= 0) return hipSuccess;
    if (b.mode == MODE_PAIR)
        return b.nf == 2 ? field_launch_nf<T, MODE_PAIR, 2>(b, st) : field_launch_nf<T, MODE_PAIR, 1>(b, st);
    return b.nf == 2 ? field_launch_nf<T, MODE_HARTLEY, 2>(b, st) : field_launch_nf<T, MODE_HARTLEY, 1>(b, st);
}
template hipError_t launch_field<float>(const FieldBatch<float>&, hipStream_t);
template hipError_t launch_field<double>(const FieldBatch<double>&, hipStream_t);

hipError_t launch_eigen_fft(const double* s, int n, const FftPlan& fp, const cplx<double>* tw,
                            cplx<double>* work, double* lam, double* imag_blk, int* nblk, hipStream_t st) {
    const int cap = 16 * kBlock;
    int L = std::min(pow2floor(std::max(1, cap / n)), lowbit(n));
    hipError_t e;
    if (L * n <= cap) {
        const size_t lds = (size_t)L * n * sizeof(cplx<double>);
        if ((e = allow_lds(k_eig_rows<16>, lds)) != hipSuccess) return e;
        if ((e = allow_lds(k_eig_cols<16>, lds)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_eig_rows<16>, dim3(n / L), dim3(kBlock), lds, st, s, L, fp, tw, work);
        hipLaunchKernelGGL(k_eig_cols<16>, dim3(n / L), dim3(kBlock), lds, st, work, L, fp, tw, lam, imag_blk);
    } else if (n <= 2 * cap) {
        L = 1;
        const size_t lds = (size_t)n * sizeof(cplx<double>);
        if ((e = allow_lds(k_eig_rows<32>, lds)) != hipSuccess) return e;
        if ((e = allow_lds(k_eig_cols<32>, lds)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_eig_rows<32>, dim3(n), dim3(kBlock), lds, st, s, 1, fp, tw, work);
        hipLaunchKernelGGL(k_eig_cols<32>, dim3(n), dim3(kBlock), lds, st, work, 1, fp, tw, lam, imag_blk);
    } else {
        return hipErrorInvalidValue;
    }
    *nblk = n / L;
    return hipGetLastError();
}

hipError_t launch_normals(uint64_t seed, uint64_t q, uint32_t stream, uint64_t first_e, long long count,
                          double* out, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_normals, dim3(cdiv(count, kBlock)), dim3(kBlock), 0, st, seed, q, stream, first_e,
                       count, out);
    return hipGetLastError();
}

hipError_t launch_convert_d2f(const double* in, float* out, long long count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_convert_d2f, dim3(cdiv(count, kBlock)), dim3(kBlock), 0, st, in, out, count);
    return hipGetLastError();
}

}  // namespace ces
