// Batched solver for -div(k grad u) = f on the unit square (Section 3.1),
// P1 elements on the right-diagonal mesh with nodal (trapezoidal)
// quadrature of k (Section 3.2).  With that quadrature the stiffness
// matrix couples only axis-neighbours (the diagonal couplings cancel), so
// A is a 5-point operator with edge conductances
//   c_E(i,j) = [T above] (k_ij + k_i+1,j + k_i+1,j+1)/6 + [T below] (k_i,j-1 + k_i+1,j + k_ij)/6
//   c_N(i,j) = [T right] (k_ij + k_i+1,j+1 + k_i,j+1)/6 + [T left] (k_i-1,j + k_ij + k_i,j+1)/6
// ([T ...] = the adjacent triangle exists), (A u)_p = sum_q c_pq (u_p - u_q)
// and load b_p = f (#triangles at p) h^2/6.
//
// Method: conjugate gradients in double (beta = r.z / r_old.z_old),
// preconditioned by one geometric multigrid V(2,2) cycle in T (float on
// the mixed path, double on the plain path): red-black SOR, relaxation
// 1.25 (red, black, red, black before the coarse correction, the reverse
// after, so the preconditioner is symmetric), restriction = transpose of bilinear
// prolongation, coarse edge conductances from the series (harmonic) means
// of the fine edges they span (exact for constant k), exact solve on the
// 2 x 2 mesh.
//
// Work layout: one launch handles a whole batch of samples; fine levels
// are tiled (64 x 64 or 64 x 32 node regions per workgroup) and the four
// half-sweeps of a smoothing step run in LDS on the tile plus a 4-node
// halo (temporal blocking: one HBM read of z, rhs and k and one write of z
// per smoothing step); a level that fits one region is smoothed by one
// workgroup per sample without halo; all levels with m <= 32 (16 in
// double) run in one workgroup per sample entirely in LDS.  Dot products are
// per-tile partial sums reduced in a fixed order, so every result is
// independent of the batch composition.  Converged samples switch their
// workgroups off (per-sample active flag).
#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "internal.hpp"

// kernel launch inside a profiled launch(...) lambda: the slot's events (or
// none) are stamped with the kernel's start and end
#define PLAUNCH(kernel, grid, block, shmem, stream, ...) \
    hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, ps.a, ps.b, 0, __VA_ARGS__)

namespace ces {

namespace {

struct Scal {
    double bb, rz, rz_old, pq, rr;
    double qacc;   // sum over iterations of alpha w.p = w.(x - x0)
    int it, active, status, pad;
};

struct Lvl {
    int m, w;
    long long ss;   // per-sample stride of this level's arrays
    int ylo, yhi;   // unknown rows (columns are always 1 .. m-1)
};

__device__ __forceinline__ bool is_unknown(int gx, int gy, int m, int bc) {
    return gx >= 1 && gx <= m - 1 && (bc == BC_FLOWCELL ? (gy >= 0 && gy <= m) : (gy >= 1 && gy <= m - 1));
}

// Dirichlet data of the flow cell: u = 1 on x1 = 0, 0 elsewhere.
__device__ __forceinline__ double dirichlet_value(int gx, int bc) {
    return (bc == BC_FLOWCELL && gx == 0) ? 1.0 : 0.0;
}

template <typename T, typename KF>
__device__ __forceinline__ T cond_e(int gx, int gy, int m, const KF& K) {
    if (gx < 0 || gx >= m || gy < 0 || gy > m) return T(0);
    const T up = (gy < m) ? K(gx, gy) + K(gx + 1, gy) + K(gx + 1, gy + 1) : T(0);
    const T dn = (gy > 0) ? K(gx, gy - 1) + K(gx + 1, gy) + K(gx, gy) : T(0);
    return (up + dn) * T(1.0 / 6.0);
}
template <typename T, typename KF>
__device__ __forceinline__ T cond_n(int gx, int gy, int m, const KF& K) {
    if (gx < 0 || gx > m || gy < 0 || gy >= m) return T(0);
    const T rt = (gx < m) ? K(gx, gy) + K(gx + 1, gy + 1) + K(gx, gy + 1) : T(0);
    const T lf = (gx > 0) ? K(gx - 1, gy) + K(gx, gy) + K(gx, gy + 1) : T(0);
    return (rt + lf) * T(1.0 / 6.0);
}

// number of triangles touching vertex (i, j) (load weight = cnt h^2 / 6)
__device__ __forceinline__ int tri_count(int i, int j, int m) {
    int c = 0;
    if (i < m && j < m) c += 2;
    if (i >= 1 && j < m) c += 1;
    if (i >= 1 && j >= 1) c += 2;
    if (i < m && j >= 1) c += 1;
    return c;
}

// ------------------------------------------------------- multigrid tiles
// One tile of one sample's level.  The region is 64 columns x 8*SH rows:
// the tile plus an H-node halo on every side.  A workgroup is 8 half-waves
// of 32 lanes; half-wave hw owns region rows [hw*SH, hw*SH + SH) and lane k
// owns the two columns 2k, 2k+1 of them, keeping z, rhs, inverse diagonal
// and conductances of its 2*SH nodes in registers.  In a red-black
// half-sweep exactly one of a lane's two nodes per row has the active
// colour, and which one is the same for every lane of the workgroup, so the
// update runs without masked-off lanes.  Neighbours come from registers
// except the column across the lane boundary and the rows across the strip
// boundary, which go through LDS.
//
// Conductances from per-triangle sums: for the square (i, j) (existing iff
// 0 <= i, j <= m-1) let S1 = k_ij + k_i+1,j + k_i+1,j+1 (triangle below the
// diagonal) and S2 = k_ij + k_i+1,j+1 + k_i,j+1 (above); then
// c_E(i,j) = (S1(i,j) + S2(i,j-1))/6 and c_N(i,j) = (S2(i,j) + S1(i-1,j))/6,
// with S = 0 for squares outside the mesh -- which is exactly the boundary
// rule (only existing triangles contribute).
//
// PRE (H = 6): two sweeps (red, black, red, black) from z = 0, z written on
// the tile, then the residual r - A z on the tile plus one ring and its
// restriction P^T to the coarse nodes whose fine centre lies in the tile.
// POST (H = 4): z_pre + P z_coarse, two sweeps (black, red, black, red),
// z written on the tile; on level 0 also the partial sum r.z.
template <typename T>
struct MgArgs {
    Lvl L, C;            // this level, the next coarser level
    int bc, tiles_x, ntiles;
    const T* k;          // level 0: nodal k
    long long kss;
    const T* ce;         // coarser levels: stored edge conductances (stride L.ss)
    const T* cn;
    const void* rhs;     // level rhs: double (level 0) or T
    T* za;               // pre-smoothed z (PRE output, POST input)
    T* rhs_c;            // PRE: coarse rhs output
    const T* zc;         // POST: coarse correction
    T* zout;             // POST: smoothed z
    double* dot;         // POST level 0: partial r.z per tile
    const Scal* scal;
};

// Red-black SOR relaxation of the smoother: each half-sweep moves a node
// by kSorOmega times its Gauss-Seidel correction.  The pre- and
// post-smoothing visit the colours in mirrored order with the same factor,
// so the V-cycle stays a symmetric positive definite preconditioner (for
// 0 < omega < 2).  Measured: 1.25 takes C2 from 10.26 to 9.97 mean CG
// iterations, C5 from 12.48 to 10.73 (1.0, 1.1 ... 1.6 tried; 1.2 - 1.3 best).
constexpr double kSorOmega = 1.25;

template <typename T>
__device__ __forceinline__ T fast_rcp(T v) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_amdgcn_rcpf(v);
    } else {
        return T(1) / v;
    }
}

template <typename T, int SH, int Q0, int PX>
__device__ __forceinline__ void mg_half_sweep(T (&z)[SH][2], const T (&rhs)[SH][2], const T (&id)[SH][2],
                                              const T (&ce)[SH][2], const T (&cw0)[SH], const T (&cn)[SH + 1][2],
                                              T* sz0) {
    // sz0 points at this lane's node (row 0 of its strip, left column) in the
    // padded LDS array; the one-node ring keeps every neighbour in range
#pragma unroll
    for (int r = 0; r < SH; ++r) {
        const int q = Q0 ^ (r & 1);
        T* p = sz0 + r * PX + q;
        const T zE = q == 0 ? z[r][1] : p[1];
        const T zW = q == 1 ? z[r][0] : p[-1];
        const T zN = (r < SH - 1) ? z[r + 1][q] : p[PX];
        const T zS = (r > 0) ? z[r - 1][q] : p[-PX];
        const T cW = q == 0 ? cw0[r] : ce[r][0];
        const T gs = (rhs[r][q] + ce[r][q] * zE + cW * zW + cn[r + 1][q] * zN + cn[r][q] * zS) * id[r][q];
        const T v = z[r][q] + T(kSorOmega) * (gs - z[r][q]);
        z[r][q] = v;
        p[0] = v;
    }
    __syncthreads();
}

// WHOLE: the level's unknowns fit in one region (Dirichlet boundary, m - 1
// <= 64 columns and rows), so one workgroup per sample takes the level with
// no halo: every sweep is exact on the region and nothing is recomputed.
// RXW = 128 (float only): the same with 128 x 128 regions, a workgroup of
// 16 waves of 64 lanes (lane k owns columns 2k, 2k+1 of its wave's SH
// rows), for Dirichlet levels with 64 < m - 1 <= 128.
// MID (POST, coarser levels): the step between the two coarse corrections
// of a level visited twice per cycle: z = z_pre + P z_c, then the residual
// restricted to the coarse rhs (no smoothing); z goes to zout, which a
// whole level may point at z_pre itself (one workgroup holds the level).
template <typename T, int SH, bool POST, bool L0, bool WHOLE, int RXW = 64, bool MID = false>
__global__ __launch_bounds__(RXW == 64 ? kBlock : 1024) void k_mg(MgArgs<T> a) {
    static_assert(RXW == 64 || (RXW == 128 && WHOLE), "128-wide regions: whole levels only");
    static_assert(!MID || (POST && !L0), "MID: coarser levels");
    constexpr int NT = RXW == 64 ? kBlock : 1024, LW = RXW / 2;
    constexpr int RX = RXW, NH = NT / LW, RY = NH * SH;
    constexpr int H = WHOLE ? 0 : (POST ? 4 : 6);
    constexpr int TX = RX - 2 * H, TY = RY - 2 * H;
    constexpr int PX = RX + 2, PY = RY + 2;   // padded: one-node ring on every side
    __shared__ T sz[PY * PX];
    __shared__ T sk[(L0 || !POST || MID) ? PY * PX : 1];    // level 0: k; PRE and MID: the residual
    constexpr int CX = RX / 2 + 3, CY = RY / 2 + 3;
    __shared__ T szc[POST ? CY * CX : 1];
    __shared__ double red[NT / 64];
    const int wi = xcd_remap(blockIdx.x, gridDim.x);
    const int s = wi / a.ntiles;
    const int tile = wi - s * a.ntiles;
    if (!a.scal[s].active) return;
    const int ty = tile / a.tiles_x, tx = tile - ty * a.tiles_x;
    const int x0 = 1 + tx * TX, y0 = a.L.ylo + ty * TY;
    const int ox = x0 - H, oy = y0 - H;
    const int m = a.L.m, w = a.L.w, bc = a.bc;
    const size_t sbase = (size_t)s * a.L.ss;
    // this lane's nodes: rhs (and the pre-smoothed z of POST); tiles load
    // them first, so that their latency overlaps the k tile's (the
    // 1024-thread whole-level workgroups, alone on their CU, load them
    // after the conductances instead)
    const int lane = threadIdx.x % LW, hw = threadIdx.x / LW;
    const int lx0 = 2 * lane, ly0 = hw * SH;
    const int gx0 = ox + lx0;
    using RT = typename std::conditional<L0, double, T>::type;   // level 0: r in double
    RT rhs_raw[SH][2];
    T zv[SH][2];
    auto load_rhs = [&]() {
        const RT* rin = reinterpret_cast<const RT*>(a.rhs) + sbase;
        const T* zin = a.za + sbase;
        const int gxc0 = min(max(gx0, 0), m), gxc1 = min(max(gx0 + 1, 0), m);
#pragma unroll
        for (int r = 0; r < SH; ++r) {
            const int gyc = min(max(oy + ly0 + r, 0), m);
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int o = gyc * w + (q == 0 ? gxc0 : gxc1);
                rhs_raw[r][q] = rin[o];
                if constexpr (POST) zv[r][q] = zin[o];
            }
        }
    };
    if constexpr (RXW == 64) load_rhs();
    // POST: the coarse correction of the region (with its ring), prefetched
    // into registers by the tiles for the same reason, except where the
    // registers would push the float level-0 kernel below four waves per SIMD
    const int cox = ox >> 1, coy = oy >> 1;  // floor, also for negative origins
    constexpr bool kEarlyZc = POST && RXW == 64 && !(L0 && sizeof(T) == 4);
    constexpr int NZC = POST ? (CY * CX + NT - 1) / NT : 1;
    T zcv[NZC];
    auto load_zc = [&]() {
        const T* zc = a.zc + (size_t)s * a.C.ss;
        const int cm = a.C.m, cw = a.C.w;
#pragma unroll
        for (int i = 0; i < NZC; ++i) {
            const int t = threadIdx.x + i * NT;
            const int y = t / CX, x = t - y * CX;
            const int I = cox + x, J = coy + y;
            const int Ic = min(max(I, 0), cm), Jc = min(max(J, 0), cm);
            zcv[i] = zc[Jc * cw + Ic];
        }
    };
    if constexpr (kEarlyZc) load_zc();
    // k tile (level 0): lane l of wave wv loads padded column l for rows wv, wv+4, ...
    if constexpr (L0) {
        // all loads are issued before any is used (addresses clamped into
        // the mesh, values masked afterwards) so their latencies overlap
        // lane l of wave wv takes padded columns l, l + 64, ... of rows
        // wv, wv + NW, ... (the last chunk only where it is inside PX)
        const T* kk = a.k + (size_t)s * a.kss;
        constexpr int NW = NT / 64, NIT = (PY + NW - 1) / NW, NCW = (PX + 63) / 64;
        const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
        int gxc[NCW];
        bool okx[NCW];
#pragma unroll
        for (int c = 0; c < NCW; ++c) {
            const int gx = ox - 1 + 64 * c + l;
            gxc[c] = min(max(gx, 0), m);
            okx[c] = gx >= 0 && gx <= m;
        }
        T kv[NIT][NCW];
#pragma unroll
        for (int i = 0; i < NIT; ++i) {
            const int gyc = min(max(oy - 1 + wv + i * NW, 0), m);
#pragma unroll
            for (int c = 0; c < NCW; ++c) kv[i][c] = kk[gyc * w + gxc[c]];
        }
#pragma unroll
        for (int i = 0; i < NIT; ++i) {
            const int y = wv + i * NW, gy = oy - 1 + y;
            const bool oky = gy >= 0 && gy <= m;
            if (y < PY) {
#pragma unroll
                for (int c = 0; c < NCW; ++c) {
                    const int col = 64 * c + l;
                    if (col < PX) sk[y * PX + col] = (okx[c] && oky) ? kv[i][c] : T(0);
                }
            }
        }
    }
    // zero ring of the z array (never updated, read as neighbours of the edge)
    for (int t = threadIdx.x; t < 2 * PX + 2 * RY; t += blockDim.x) {
        if (t < PX) sz[t] = T(0);
        else if (t < 2 * PX) sz[(PY - 1) * PX + t - PX] = T(0);
        else if (t < 2 * PX + RY) sz[(t - 2 * PX + 1) * PX] = T(0);
        else sz[(t - 2 * PX - RY + 1) * PX + PX - 1] = T(0);
    }
    if constexpr (POST) {
        if constexpr (!kEarlyZc) load_zc();
        const int cm = a.C.m;
#pragma unroll
        for (int i = 0; i < NZC; ++i) {
            const int t = threadIdx.x + i * NT;
            if (t >= CY * CX) break;
            const int y = t / CX, x = t - y * CX;
            const int I = cox + x, J = coy + y;
            szc[t] = is_unknown(I, J, cm, bc) ? zcv[i] : T(0);
        }
    }
    __syncthreads();
    // column masks of this lane
    const bool unk_c0 = gx0 >= 1 && gx0 <= m - 1, unk_c1 = gx0 + 1 >= 1 && gx0 + 1 <= m - 1;
    const bool sqc_m = gx0 - 1 >= 0 && gx0 - 1 <= m - 1, sqc_a = gx0 >= 0 && gx0 <= m - 1,
               sqc_b = gx0 + 1 >= 0 && gx0 + 1 <= m - 1;
    const int ylo = a.L.ylo, yhi = a.L.yhi;
    T ce[SH][2], cw0[SH], cn[SH + 1][2];
    if constexpr (!L0) {
        // coarser levels: stored conductances (zero outside the mesh)
        const T* CEg = a.ce + sbase;
        const T* CNg = a.cn + sbase;
        auto ld = [&](const T* g, int gx, int gy) -> T {
            const T v = g[min(max(gy, 0), m) * w + min(max(gx, 0), m)];
            return (gx >= 0 && gx <= m && gy >= 0 && gy <= m) ? v : T(0);
        };
#pragma unroll
        for (int q = 0; q < 2; ++q) cn[0][q] = ld(CNg, gx0 + q, oy + ly0 - 1);
#pragma unroll
        for (int r = 0; r < SH; ++r) {
            const int gy = oy + ly0 + r;
            cw0[r] = ld(CEg, gx0 - 1, gy);
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                ce[r][q] = ld(CEg, gx0 + q, gy);
                cn[r + 1][q] = ld(CNg, gx0 + q, gy);
            }
        }
    } else {
        // triangle sums S1, S2 of the squares at columns gx0-1, gx0, gx0+1
        const T* k0 = sk + ly0 * PX + lx0;   // padded (lx0 - 1, ly0 - 1)
        T p2m = T(0), p2a = T(0), p2b = T(0);
        const T sixth = T(1.0 / 6.0);
#pragma unroll
        for (int r = -1; r < SH; ++r) {
            const T* kr = k0 + (r + 1) * PX;
            const T k_m = kr[0], k_a = kr[1], k_b = kr[2], k_c = kr[3];
            const T u_m = kr[PX], u_a = kr[PX + 1], u_b = kr[PX + 2], u_c = kr[PX + 3];
            const int gy = oy + ly0 + r;
            const bool sqr = gy >= 0 && gy <= m - 1;
            const T s1m = (sqr && sqc_m) ? k_m + k_a + u_a : T(0);
            const T s2m = (sqr && sqc_m) ? k_m + u_a + u_m : T(0);
            const T s1a = (sqr && sqc_a) ? k_a + k_b + u_b : T(0);
            const T s2a = (sqr && sqc_a) ? k_a + u_b + u_a : T(0);
            const T s1b = (sqr && sqc_b) ? k_b + k_c + u_c : T(0);
            const T s2b = (sqr && sqc_b) ? k_b + u_c + u_b : T(0);
            if (r >= 0) {
                ce[r][0] = (s1a + p2a) * sixth;
                ce[r][1] = (s1b + p2b) * sixth;
                cw0[r] = (s1m + p2m) * sixth;
            }
            cn[r + 1][0] = (s2a + s1m) * sixth;
            cn[r + 1][1] = (s2b + s1a) * sixth;
            p2m = s2m;
            p2a = s2a;
            p2b = s2b;
        }
    }
    T z[SH][2], rhs[SH][2], id[SH][2];
    T* sz0 = sz + (ly0 + 1) * PX + lx0 + 1;
    if constexpr (RXW != 64) load_rhs();
#pragma unroll
    for (int r = 0; r < SH; ++r)
#pragma unroll
        for (int q = 0; q < 2; ++q) rhs[r][q] = (T)rhs_raw[r][q];
#pragma unroll
    for (int r = 0; r < SH; ++r) {
        const int gy = oy + ly0 + r;
        const bool ur = gy >= ylo && gy <= yhi;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int gx = gx0 + q;
            T rr = T(0), zz = T(0), d = T(0);
            if (ur && (q == 0 ? unk_c0 : unk_c1)) {
                rr = rhs[r][q];
                const T cW = q == 0 ? cw0[r] : ce[r][0];
                d = fast_rcp(ce[r][q] + cW + cn[r + 1][q] + cn[r][q]);
                if constexpr (POST) {
                    const int I = (gx >> 1) - cox, J = (gy >> 1) - coy;
                    const bool ox1 = gx & 1, oy1 = gy & 1;
                    const T* c0 = szc + J * CX + I;
                    T p;
                    if (!ox1 && !oy1) p = c0[0];
                    else if (ox1 && !oy1) p = T(0.5) * (c0[0] + c0[1]);
                    else if (!ox1 && oy1) p = T(0.5) * (c0[0] + c0[CX]);
                    else p = T(0.25) * ((c0[0] + c0[1]) + (c0[CX] + c0[CX + 1]));
                    zz = zv[r][q] + p;
                }
            }
            z[r][q] = zz;
            rhs[r][q] = rr;
            id[r][q] = d;
            sz0[r * PX + q] = zz;
        }
    }
    __syncthreads();
    // the active column of row 0 for colour c is (c - ox - oy) & 1 (ly0 is even)
    const int par = (ox + oy) & 1;
    const int c0 = POST ? 1 : 0;
    if constexpr (!MID) {
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const int c = (h & 1) ? 1 - c0 : c0;
            if (((c - par) & 1) == 0)
                mg_half_sweep<T, SH, 0, PX>(z, rhs, id, ce, cw0, cn, sz0);
            else
                mg_half_sweep<T, SH, 1, PX>(z, rhs, id, ce, cw0, cn, sz0);
        }
    }
    // outputs on the tile (margin >= H); id != 0 marks unknown nodes
    double acc = 0.0;
    T* out = POST ? a.zout + sbase : a.za + sbase;
#pragma unroll
    for (int r = 0; r < SH; ++r) {
        const int ly = ly0 + r, gy = oy + ly;
        const bool iny = ly >= H && ly < H + TY;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int lx = lx0 + q;
            const bool in = iny && lx >= H && lx < H + TX && id[r][q] != T(0);
            if (in) out[gy * w + gx0 + q] = z[r][q];
            if constexpr (POST && L0) {
                if (in) acc += (double)rhs[r][q] * (double)z[r][q];
            }
        }
    }
    if constexpr (POST && !MID) {
        if constexpr (L0) {
            acc = block_sum(acc, red);
            if (threadIdx.x == 0) a.dot[(size_t)s * a.ntiles + tile] = acc;
        }
        return;
    } else {
        // residual r - A z (difference form) into sk, on every region node
        T* sres0 = sk + (ly0 + 1) * PX + lx0 + 1;
#pragma unroll
        for (int r = 0; r < SH; ++r) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const T* p = sz0 + r * PX + q;
                const T zp = z[r][q];
                const T zE = q == 0 ? z[r][1] : p[1];
                const T zW = q == 1 ? z[r][0] : p[-1];
                const T zN = (r < SH - 1) ? z[r + 1][q] : p[PX];
                const T zS = (r > 0) ? z[r - 1][q] : p[-PX];
                const T cW = q == 0 ? cw0[r] : ce[r][0];
                const T az = (ce[r][q] * (zp - zE) + cW * (zp - zW)) + (cn[r + 1][q] * (zp - zN) + cn[r][q] * (zp - zS));
                sres0[r * PX + q] = id[r][q] != T(0) ? rhs[r][q] - az : T(0);
            }
        }
        __syncthreads();
        // coarse nodes whose fine centre (2I, 2J) lies in the tile
        const int I0 = (x0 + 1) >> 1, J0 = (y0 + 1) >> 1;
        const int nI = ((x0 + TX + 1) >> 1) - I0, nJ = ((y0 + TY + 1) >> 1) - J0;
        const int cm = a.C.m, cwid = a.C.w;
        T* rc = a.rhs_c + (size_t)s * a.C.ss;
        for (int t = threadIdx.x; t < nI * nJ; t += blockDim.x) {
            const int jj = t / nI, ii = t - jj * nI;
            const int I = I0 + ii, J = J0 + jj;
            if (!is_unknown(I, J, cm, bc)) continue;
            const T* c0 = sk + (2 * J - oy + 1) * PX + (2 * I - ox + 1);
            const T v = c0[0] + T(0.5) * ((c0[-1] + c0[1]) + (c0[-PX] + c0[PX])) +
                        T(0.25) * ((c0[-PX - 1] + c0[-PX + 1]) + (c0[PX - 1] + c0[PX + 1]));
            rc[J * cwid + I] = v;
        }
    }
}

// ------------------------------------------------ whole-V-cycle bottom ---
// ------------------------------------------------- LDS-resident multigrid
// Levels with m <= 32 (16 in double) of one sample live in one workgroup's
// LDS: z, rhs and edge conductances of every level,
// stored level after level (level l at off[l], row pitch m_l + 1), plus a
// scratch array the size of the finest of them.
// Level l has m0 >> l intervals; its arrays start at off[l] (an LDS table,
// so that no per-level array sits in private memory).
// fw[l], fh[l] (LDS too): division by the row pitch w_l and by the
// (w_l + 1) / 2 nodes of one colour in a row.
template <typename T>
struct LdsMg {
    T *z, *rhs, *ce, *cn, *tmp;
    int* off;
    FastDiv *fw, *fh;
    int nl, bc, m0;
    __device__ int m(int l) const { return m0 >> l; }
    __device__ int w(int l) const { return (m0 >> l) + 1; }
    __device__ int ylo(int) const { return bc == BC_FLOWCELL ? 0 : 1; }
    __device__ int yhi(int l) const { return bc == BC_FLOWCELL ? (m0 >> l) : (m0 >> l) - 1; }
};

__host__ __device__ constexpr int lds_mg_nodes(int m) {
    int t = 0;
    for (int mm = m; mm >= 2; mm /= 2) t += (mm + 1) * (mm + 1);
    return t;
}

// Threads per workgroup of the whole-solve kernel: fixed by m, because the
// workgroup's dot products sum in an order that depends on it.
__host__ __device__ constexpr int small_threads(int m) { return m <= 16 ? 256 : 512; }

// fills the offset table (call before the first barrier of the kernel)
template <typename T>
__device__ void lds_mg_layout(const LdsMg<T>& g) {
    if (threadIdx.x == 0) {
        int o = 0;
        for (int l = 0; l < g.nl; ++l) {
            g.off[l] = o;
            o += g.w(l) * g.w(l);
            g.fw[l] = FastDiv((unsigned)g.w(l));
            g.fh[l] = FastDiv((unsigned)(g.w(l) + 1) / 2);
        }
    }
}

// diagonal of unknown p (x, y) from the edge conductances
template <typename T>
__device__ __forceinline__ T lds_diag(const T* ce, const T* cn, int p, int y, int w) {
    return ce[p] + ce[p - 1] + cn[p] + (y >= 1 ? cn[p - w] : T(0));
}

// one red-black half-sweep of colour c (parity of x + y) on one level; the
// inverse diagonal is formed where it is used (not stored: the LDS it
// would take decides how many samples a CU holds)
template <typename T>
__device__ void lds_sweep(T* z, const T* rhs, const T* ce, const T* cn, int m, int bc, int c, FastDiv fh) {
    const int w = m + 1;
    const int half = (w + 1) / 2;
    for (int t = threadIdx.x; t < half * w; t += blockDim.x) {
        const int y = fh.div(t);
        const int x = 2 * (t - mul24(y, half)) + ((c - y) & 1);
        if (x >= w) continue;
        if (!is_unknown(x, y, m, bc)) continue;
        const int p = mul24(y, w) + x;
        const T d = fast_rcp(lds_diag(ce, cn, p, y, w));
        T s = rhs[p];
        if (x + 1 < w) s += ce[p] * z[p + 1];
        if (x >= 1) s += ce[p - 1] * z[p - 1];
        if (y + 1 < w) s += cn[p] * z[p + w];
        if (y >= 1) s += cn[p - w] * z[p - w];
        z[p] = z[p] + T(kSorOmega) * (s * d - z[p]);
    }
    __syncthreads();
}

// One V(2,2) cycle from z = 0 with the level-0 rhs in place; z of every
// level is overwritten, level 0's holds the result.
template <typename T>
__device__ void lds_vcycle(const LdsMg<T>& g) {
    const int tot = g.off[g.nl - 1] + g.w(g.nl - 1) * g.w(g.nl - 1);
    for (int t = threadIdx.x; t < tot; t += blockDim.x) g.z[t] = T(0);
    __syncthreads();
    T *z = g.z, *rhs = g.rhs, *tmp = g.tmp;
    const T *ce = g.ce, *cn = g.cn;
    // down: pre-smooth, residual, restriction (transpose of bilinear)
    for (int l = 0; l + 1 < g.nl; ++l) {
        const int m = g.m(l), w = g.w(l), o = g.off[l];
        const FastDiv fw = g.fw[l], fh = g.fh[l];
        for (int c = 0; c < 4; ++c) lds_sweep<T>(z + o, rhs + o, ce + o, cn + o, m, g.bc, c & 1, fh);
        for (int t = threadIdx.x; t < w * w; t += blockDim.x) {
            const int y = fw.div(t), x = t - mul24(y, w);
            T r = T(0);
            if (is_unknown(x, y, m, g.bc)) {
                const int p = o + t;
                const T zp = z[p];
                const T zN = y + 1 < w ? z[p + w] : T(0), zS = y >= 1 ? z[p - w] : T(0);
                const T cS = y >= 1 ? cn[p - w] : T(0);
                const T az = (ce[p] * (zp - z[p + 1]) + ce[p - 1] * (zp - z[p - 1])) +
                             (cn[p] * (zp - zN) + cS * (zp - zS));
                r = rhs[p] - az;
            }
            tmp[t] = r;
        }
        __syncthreads();
        const int cm = g.m(l + 1), cwid = g.w(l + 1), co = g.off[l + 1];
        const FastDiv fwc = g.fw[l + 1];
        for (int t = threadIdx.x; t < cwid * cwid; t += blockDim.x) {
            const int J = fwc.div(t), I = t - mul24(J, cwid);
            T v = T(0);
            if (is_unknown(I, J, cm, g.bc)) {
                const int x = 2 * I, y = 2 * J;
                auto R = [&](int xx, int yy) -> T {
                    return (xx >= 0 && xx < w && yy >= 0 && yy < w) ? tmp[mul24(yy, w) + xx] : T(0);
                };
                v = R(x, y) + T(0.5) * ((R(x - 1, y) + R(x + 1, y)) + (R(x, y - 1) + R(x, y + 1))) +
                    T(0.25) * ((R(x - 1, y - 1) + R(x + 1, y - 1)) + (R(x - 1, y + 1) + R(x + 1, y + 1)));
            }
            rhs[co + t] = v;
        }
        __syncthreads();
    }
    // coarsest (m = 2): exact tridiagonal solve along the unknown column x = 1
    if (threadIdx.x == 0) {
        const int l = g.nl - 1, w = g.w(l), o = g.off[l];
        const int ylo = g.ylo(l), yhi = g.yhi(l);
        T beta[3] = {T(1), T(1), T(1)}, yv[3] = {T(0), T(0), T(0)};
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            if (j < ylo || j > yhi) continue;
            const int p = o + j * w + 1;
            const T d = lds_diag(ce, cn, p, j, w);
            if (j == ylo) {
                beta[j] = d;
                yv[j] = rhs[p];
            } else {
                const T cS = cn[p - w];
                beta[j] = d - cS * cS / beta[j - 1];
                yv[j] = rhs[p] + cS * yv[j - 1] / beta[j - 1];
            }
        }
        T zn = T(0);
#pragma unroll
        for (int j = 2; j >= 0; --j) {
            if (j < ylo || j > yhi) continue;
            const int p = o + j * w + 1;
            const T cN = (j < yhi) ? cn[p] : T(0);
            const T v = (yv[j] + cN * zn) / beta[j];
            z[p] = v;
            zn = v;
        }
    }
    __syncthreads();
    // up: bilinear prolongation of the correction, post-smooth
    for (int l = g.nl - 2; l >= 0; --l) {
        const int m = g.m(l), w = g.w(l), o = g.off[l];
        const int cm = g.m(l + 1), cwid = g.w(l + 1), co = g.off[l + 1];
        const FastDiv fw = g.fw[l], fh = g.fh[l];
        for (int t = threadIdx.x; t < w * w; t += blockDim.x) {
            const int y = fw.div(t), x = t - mul24(y, w);
            if (!is_unknown(x, y, m, g.bc)) continue;
            const int I = x >> 1, J = y >> 1;
            auto C = [&](int ci, int cj) -> T {
                return is_unknown(ci, cj, cm, g.bc) ? z[co + mul24(cj, cwid) + ci] : T(0);
            };
            T p;
            const bool ox1 = x & 1, oy1 = y & 1;
            if (!ox1 && !oy1) p = C(I, J);
            else if (ox1 && !oy1) p = T(0.5) * (C(I, J) + C(I + 1, J));
            else if (!ox1 && oy1) p = T(0.5) * (C(I, J) + C(I, J + 1));
            else p = T(0.25) * ((C(I, J) + C(I + 1, J)) + (C(I, J + 1) + C(I + 1, J + 1)));
            z[o + t] += p;
        }
        __syncthreads();
        for (int c = 0; c < 4; ++c) lds_sweep<T>(z + o, rhs + o, ce + o, cn + o, m, g.bc, 1 - (c & 1), fh);
    }
}

// Bottom of the tiled V-cycle: the levels with m <= MB of each sample in
// one workgroup (stored conductances, rhs from the next finer level).
template <typename T>
struct BottomArgs {
    int nl;            // levels handled here: m0, m0/2, ..., 2
    int bc, m0;
    long long ss[8];   // per-sample stride of each level's arrays
    const T* ce[8];    // stored edge conductances
    const T* cn[8];
    const T* rhs;      // rhs of the first bottom level
    T* zout;           // its z
    const Scal* scal;
};

// NT threads per workgroup; the result does not depend on NT.
template <typename T, int MB, int NT>
__global__ __launch_bounds__(NT) void k_bottom(BottomArgs<T> a) {
    constexpr int TOT = lds_mg_nodes(MB);
    __shared__ T z[TOT], rhs[TOT], ce[TOT], cn[TOT];
    __shared__ T tmp[(MB + 1) * (MB + 1)];
    __shared__ int off[8];
    __shared__ FastDiv fdw[8], fdh[8];
    const int s = blockIdx.x;
    if (!a.scal[s].active) return;
    LdsMg<T> g;
    g.z = z; g.rhs = rhs; g.ce = ce; g.cn = cn; g.tmp = tmp;
    g.off = off;
    g.fw = fdw;
    g.fh = fdh;
    g.nl = a.nl;
    g.bc = a.bc;
    g.m0 = a.m0;
    lds_mg_layout(g);
    __syncthreads();
    {
        // every level's conductances and the first level's rhs, all loads
        // issued before the LDS stores (node t of the stacked levels)
        const int total = off[a.nl - 1] + g.w(a.nl - 1) * g.w(a.nl - 1);
        const int m0 = g.m(0), w0 = g.w(0);
        constexpr int NLD = (TOT + NT - 1) / NT;
        T cev[NLD], cnv[NLD], rv[NLD];
#pragma unroll
        for (int i = 0; i < NLD; ++i) {
            const int t = threadIdx.x + i * NT;
            cev[i] = cnv[i] = rv[i] = T(0);
            if (t < total) {
                int l = 0;
                while (l + 1 < a.nl && t >= off[l + 1]) ++l;
                const int u = t - off[l];
                cev[i] = a.ce[l][(size_t)s * a.ss[l] + u];
                cnv[i] = a.cn[l][(size_t)s * a.ss[l] + u];
                if (l == 0) {
                    const int uy = fdw[0].div(u);
                    if (is_unknown(u - mul24(uy, w0), uy, m0, a.bc)) rv[i] = a.rhs[(size_t)s * a.ss[0] + u];
                }
            }
        }
#pragma unroll
        for (int i = 0; i < NLD; ++i) {
            const int t = threadIdx.x + i * NT;
            if (t < total) {
                ce[t] = cev[i];
                cn[t] = cnv[i];
                if (t < w0 * w0) rhs[t] = rv[i];
            }
        }
    }
    __syncthreads();
    lds_vcycle(g);
    const int m = g.m(0), w = g.w(0);
    const FastDiv fw0 = fdw[0];
    for (int t = threadIdx.x; t < w * w; t += blockDim.x) {
        const int y = fw0.div(t), x = t - mul24(y, w);
        if (is_unknown(x, y, m, a.bc)) a.zout[(size_t)s * a.ss[0] + t] = z[t];
    }
}

// Coarse operators from the fine edge conductances: along the coarse edge
// the two fine edges it spans act in series (harmonic mean 2ab/(a+b)); the
// coarse control volume also covers half of each parallel fine line beside
// it, so the series means of the three fine lines are averaged with weights
// 1/2 (the line itself) and 1/4 (each neighbour).  Exact for constant k
// (also on boundary lines, whose missing neighbour counts as zero where the
// fine boundary edge has half the interior conductance).  Computed from
// level 0's nodal k or from a stored level.
// harmonic mean 2ab/(a+b), zero when both conductances vanish; in float
// (the mixed path's coarse operators) with the hardware reciprocal
template <typename V>
__device__ __forceinline__ V hmean2(V a, V b) {
    const V s = a + b;
    if constexpr (sizeof(V) == 4) return s > V(0) ? V(2) * a * b * fast_rcp(s) : V(0);
    else return s > V(0) ? V(2) * a * b / s : V(0);
}

// E(x, y), N(x, y): fine east / north edge conductances, zero outside the
// mesh; the arithmetic takes their value type
template <typename EF>
__device__ __forceinline__ auto coarse_e(int I, int J, const EF& E) -> decltype(E(0, 0)) {
    using V = decltype(E(0, 0));
    const int x = 2 * I, y = 2 * J;
    return V(0.5) * hmean2(E(x, y), E(x + 1, y)) +
           V(0.25) * (hmean2(E(x, y - 1), E(x + 1, y - 1)) + hmean2(E(x, y + 1), E(x + 1, y + 1)));
}
template <typename NF>
__device__ __forceinline__ auto coarse_n(int I, int J, const NF& N) -> decltype(N(0, 0)) {
    using V = decltype(N(0, 0));
    const int x = 2 * I, y = 2 * J;
    return V(0.5) * hmean2(N(x, y), N(x, y + 1)) +
           V(0.25) * (hmean2(N(x - 1, y), N(x - 1, y + 1)) + hmean2(N(x + 1, y), N(x + 1, y + 1)));
}

// Coarse nodes in tiles of at most CCX x CCY per workgroup (each thread
// takes two rows of a column); the fine k
// they read (fine nodes 2I-2 .. 2I+2 by 2J-2 .. 2J+2) is staged in LDS
// first.  The tile width ctw <= CCX splits the coarse rows into equal
// parts (129 coarse columns: 5 tiles of 26, not 5 of 32).  The level-1
// operator is computed in T (float on the mixed path, which stores it in
// float anyway).
constexpr int CCX = 32, CCR = kBlock / CCX, CCY = 2 * CCR;   // CCR rows per pass, two passes

template <typename T>
__global__ __launch_bounds__(kBlock) void k_coarsen_k(const T* __restrict__ kf, long long kfss, Lvl F,
                                                      T* __restrict__ cec, T* __restrict__ cnc, Lvl C,
                                                      int tiles_x, int ntiles, int ctw) {
    constexpr int KX = 2 * CCX + 3, KY = 2 * CCY + 3;
    __shared__ T kt[KY * KX];
    // one sample's tiles on one XCD: their overlapping fine rows share its L2
    const int wi = xcd_remap(blockIdx.x, gridDim.x);
    const int s = wi / ntiles, tile = wi - s * ntiles;
    const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
    const int I0 = tx * ctw, J0 = ty * CCY;
    const int fx0 = 2 * I0 - 2, fy0 = 2 * J0 - 2;
    const T* k = kf + (size_t)s * kfss;
    const int m = F.m, w = F.w;
    const int kx = 2 * ctw + 3;   // fine columns the tile reads
    // fine rows of the tile, 64 lanes along each; every load of the tile
    // (address clamped into the mesh) is issued before the first is stored
    constexpr int NW = kBlock / 64, NYP = (KY + NW - 1) / NW, NXP = (KX + 63) / 64;
    const int ly = (int)threadIdx.x >> 6, lx = (int)threadIdx.x & 63;
    T v[NYP][NXP];
#pragma unroll
    for (int i = 0; i < NYP; ++i) {
        const int gy = min(max(fy0 + ly + NW * i, 0), m);
#pragma unroll
        for (int c = 0; c < NXP; ++c) {
            const int x = lx + 64 * c;
            v[i][c] = (ly + NW * i < KY && x < kx) ? k[(size_t)gy * w + min(max(fx0 + x, 0), m)] : T(0);
        }
    }
#pragma unroll
    for (int i = 0; i < NYP; ++i) {
        const int y = ly + NW * i, gy = fy0 + y;
#pragma unroll
        for (int c = 0; c < NXP; ++c) {
            const int x = lx + 64 * c, gx = fx0 + x;
            if (y < KY && x < kx) kt[y * KX + x] = (gx >= 0 && gx <= m && gy >= 0 && gy <= m) ? v[i][c] : T(0);
        }
    }
    __syncthreads();
    const int ix = (int)threadIdx.x % CCX;
    const int I = I0 + ix;
    if (ix >= ctw || I >= C.w) return;
    // the conductance formulas read only nodes inside the mesh
    auto K = [&](int gx, int gy) -> T { return kt[(gy - fy0) * KX + (gx - fx0)]; };
    auto E = [&](int x, int y) -> T { return cond_e<T>(x, y, m, K); };
    auto N = [&](int x, int y) -> T { return cond_n<T>(x, y, m, K); };
#pragma unroll
    for (int r = 0; r < CCY / CCR; ++r) {
        const int J = J0 + (int)threadIdx.x / CCX + r * CCR;
        if (J >= C.w) break;
        const size_t t = (size_t)J * C.w + I;
        cec[(size_t)s * C.ss + t] = coarse_e(I, J, E);
        cnc[(size_t)s * C.ss + t] = coarse_n(I, J, N);
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_coarsen_c(const T* __restrict__ cef, const T* __restrict__ cnf, Lvl F,
                                                      T* __restrict__ cec, T* __restrict__ cnc, Lvl C) {
    const int s = blockIdx.y;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= C.w * C.w) return;
    const int J = t / C.w, I = t - J * C.w;
    const T* ce = cef + (size_t)s * F.ss;
    const T* cn = cnf + (size_t)s * F.ss;
    const int m = F.m, w = F.w;
    // loads clamped into the mesh and masked afterwards, so that all twelve
    // are issued before the first is used; the arithmetic is in T, as in
    // k_coarsen_k
    auto E = [&](int x, int y) -> T {
        const T v = ce[min(max(y, 0), m) * w + min(max(x, 0), m)];
        return (x >= 0 && y >= 0 && x <= m && y <= m) ? v : T(0);
    };
    auto N = [&](int x, int y) -> T {
        const T v = cn[min(max(y, 0), m) * w + min(max(x, 0), m)];
        return (x >= 0 && y >= 0 && x <= m && y <= m) ? v : T(0);
    };
    cec[(size_t)s * C.ss + t] = coarse_e(I, J, E);
    cnc[(size_t)s * C.ss + t] = coarse_n(I, J, N);
}

// ------------------------------------------- whole solve of a small mesh
// Meshes with m <= 32: one workgroup runs one sample's entire PCG solve
// (same method as the tiled path: CG in double, one V(2,2) cycle in T per
// iteration, harmonic-mean coarse operators) with every vector in LDS or
// registers, so a batch of small solves is a single launch with no host
// round trips.  Thread t owns nodes t, t + NT, ... (at most NPT of them):
// their x, r and q stay in registers; p (which the operator
// needs at neighbours), the double conductances of the CG operator and the
// multigrid hierarchy live in LDS.
template <typename T>
struct SmallArgs {
    int nl, bc, maxit, m;
    long long xss;     // per-sample stride of X
    double f, h2, rtol2;
    const T* k;        // nodal k (stride kss)
    long long kss;
    double* X;         // nodal solution out (stride L[0].ss)
    Scal* scal;        // per-sample scalars out (it, status, bb, rr)
    int S;             // samples in the launch
};

constexpr int kSmallMax = 32;   // largest mesh solved by one workgroup

template <typename T>
size_t small_lds_bytes(int m) {
    const size_t n0 = (size_t)(m + 1) * (m + 1);
    return 3 * n0 * sizeof(double) + (4 * (size_t)lds_mg_nodes(m) + n0) * sizeof(T);
}

// NT threads for meshes with m <= MB: thread t owns nodes t, t + NT, ...
template <typename T, int NT, int MB>
__global__ __launch_bounds__(NT) void k_small_pcg(SmallArgs<T> a) {
    constexpr int kSmallNpt = ((MB + 1) * (MB + 1) + NT - 1) / NT;   // nodes per thread
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[2 * (NT / 64)];
    __shared__ int off[8];
    __shared__ FastDiv fdw[8], fdh[8];
    const int s = blockIdx.x;
    const int m = a.m, w = m + 1, n0 = w * w, bc = a.bc;
    const int tot = lds_mg_nodes(m);
    double* P = reinterpret_cast<double*>(smem);
    double* cE = P + n0;
    double* cN = cE + n0;
    LdsMg<T> g;
    g.z = reinterpret_cast<T*>(cN + n0);
    g.rhs = g.z + tot;
    g.ce = g.rhs + tot;
    g.cn = g.ce + tot;
    g.tmp = g.cn + tot;
    g.off = off;
    g.fw = fdw;
    g.fh = fdh;
    g.nl = a.nl;
    g.bc = bc;
    g.m0 = m;
    lds_mg_layout(g);
    // nodal k, then the conductances of every level
    const T* kg = a.k + (size_t)s * a.kss;
    for (int t = threadIdx.x; t < n0; t += NT) g.tmp[t] = kg[t];
    __syncthreads();
    {
        auto KT = [&](int gx, int gy) -> T { return g.tmp[gy * w + gx]; };
        auto KD = [&](int gx, int gy) -> double { return (double)g.tmp[gy * w + gx]; };
        for (int t = threadIdx.x; t < n0; t += NT) {
            const int y = t / w, x = t - y * w;
            g.ce[t] = cond_e<T>(x, y, m, KT);
            g.cn[t] = cond_n<T>(x, y, m, KT);
            cE[t] = cond_e<double>(x, y, m, KD);
            cN[t] = cond_n<double>(x, y, m, KD);
        }
        if (a.nl > 1) {
            const int cw = g.w(1), o = g.off[1];
            for (int t = threadIdx.x; t < cw * cw; t += NT) {
                const int J = t / cw, I = t - J * cw;
                auto E = [&](int x, int y) -> double { return cond_e<double>(x, y, m, KD); };
                auto N = [&](int x, int y) -> double { return cond_n<double>(x, y, m, KD); };
                g.ce[o + t] = (T)coarse_e(I, J, E);
                g.cn[o + t] = (T)coarse_n(I, J, N);
            }
        }
        __syncthreads();
    }
    for (int l = 2; l < a.nl; ++l) {
        const int fm = g.m(l - 1), fw = g.w(l - 1), fo = g.off[l - 1];
        const int cw = g.w(l), o = g.off[l];
        auto E = [&](int x, int y) -> double {
            return (x >= 0 && y >= 0 && x <= fm && y <= fm) ? (double)g.ce[fo + y * fw + x] : 0.0;
        };
        auto N = [&](int x, int y) -> double {
            return (x >= 0 && y >= 0 && x <= fm && y <= fm) ? (double)g.cn[fo + y * fw + x] : 0.0;
        };
        for (int t = threadIdx.x; t < cw * cw; t += NT) {
            const int J = t / cw, I = t - J * cw;
            g.ce[o + t] = (T)coarse_e(I, J, E);
            g.cn[o + t] = (T)coarse_n(I, J, N);
        }
        __syncthreads();
    }
    // x = Dirichlet lifting, r = b - A x at the unknowns
    double xr[kSmallNpt], rr_[kSmallNpt], qr[kSmallNpt];
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < kSmallNpt; ++i) {
        const int t = threadIdx.x + i * NT;
        xr[i] = rr_[i] = qr[i] = 0.0;
        if (t >= n0) continue;
        const int y = t / w, x = t - y * w;
        if (is_unknown(x, y, m, bc)) {
            double rv = a.f * (double)tri_count(x, y, m) * a.h2 * (1.0 / 6.0);
            if (!is_unknown(x + 1, y, m, bc) && x + 1 <= m) rv += cE[t] * dirichlet_value(x + 1, bc);
            if (!is_unknown(x - 1, y, m, bc) && x - 1 >= 0) rv += cE[t - 1] * dirichlet_value(x - 1, bc);
            if (!is_unknown(x, y + 1, m, bc) && y + 1 <= m) rv += cN[t] * dirichlet_value(x, bc);
            if (!is_unknown(x, y - 1, m, bc) && y - 1 >= 0) rv += cN[t - w] * dirichlet_value(x, bc);
            rr_[i] = rv;
            acc += rv * rv;
        } else {
            xr[i] = dirichlet_value(x, bc);
        }
        P[t] = 0.0;
    }
    const double bb = block_sum(acc, red);
    int it = 0, status = 0;
    double rr = bb, rz_old = 0.0;
    bool active = bb > 0.0;
    while (active) {
        // z = V-cycle(r) in T
#pragma unroll
        for (int i = 0; i < kSmallNpt; ++i) {
            const int t = threadIdx.x + i * NT;
            if (t < n0) g.rhs[t] = (T)rr_[i];   // r is zero off the unknowns
        }
        __syncthreads();
        lds_vcycle(g);
        double rz = 0.0;
        double zr[kSmallNpt];
#pragma unroll
        for (int i = 0; i < kSmallNpt; ++i) {
            const int t = threadIdx.x + i * NT;
            zr[i] = t < n0 ? (double)g.z[t] : 0.0;
            rz += rr_[i] * zr[i];
        }
        rz = block_sum(rz, red);
        const double beta = it == 0 ? 0.0 : rz / rz_old;
        rz_old = rz;
#pragma unroll
        for (int i = 0; i < kSmallNpt; ++i) {
            const int t = threadIdx.x + i * NT;
            if (t >= n0) continue;
            const int y = t / w, x = t - y * w;
            if (is_unknown(x, y, m, bc)) P[t] = zr[i] + beta * P[t];
        }
        __syncthreads();
        double pq = 0.0;
#pragma unroll
        for (int i = 0; i < kSmallNpt; ++i) {
            const int t = threadIdx.x + i * NT;
            qr[i] = 0.0;
            if (t >= n0) continue;
            const int y = t / w, x = t - y * w;
            if (!is_unknown(x, y, m, bc)) continue;
            const double pc = P[t];
            double q = cE[t] * (pc - P[t + 1]) + cE[t - 1] * (pc - P[t - 1]);
            if (y < m) q += cN[t] * (pc - P[t + w]);
            if (y > 0) q += cN[t - w] * (pc - P[t - w]);
            qr[i] = q;
            pq += pc * q;
        }
        pq = block_sum(pq, red);
        const double alpha = rz / pq;
        double racc = 0.0;
#pragma unroll
        for (int i = 0; i < kSmallNpt; ++i) {
            const int t = threadIdx.x + i * NT;
            if (t < n0) xr[i] += alpha * P[t];
            rr_[i] -= alpha * qr[i];
            racc += rr_[i] * rr_[i];
        }
        rr = block_sum(racc, red);
        ++it;
        if (rr <= a.rtol2 * bb) {
            active = false;
        } else if (it >= a.maxit) {
            active = false;
            status = -4;
        }
    }
    double* X = a.X + (size_t)s * a.xss;
#pragma unroll
    for (int i = 0; i < kSmallNpt; ++i) {
        const int t = threadIdx.x + i * NT;
        if (t < n0) X[t] = xr[i];
    }
    if (threadIdx.x == 0) {
        Scal& sc = a.scal[s];
        sc.bb = bb;
        sc.rr = rr;
        sc.it = it;
        sc.status = status;
        sc.active = 0;
    }
}

// ------------------------------------------- direct solve of a tiny mesh
// Meshes with m <= kDirectMax: one wave per sample factorises the band of
// the 5-point operator (unknowns numbered x fastest, half-bandwidth
// bw = m - 1) as L D L^T in double, with the right-hand side eliminated
// along, then back-substitutes.  The operator is the PCG path's: double
// conductances from the nodal k, Dirichlet lifting x0, and x = x0 + A^-1
// (b - A x0).  The band is held in LDS, row i at Bd[i * m] (m = bw + 1, a
// power of two); elimination is right-looking and in place, so after step
// j row j holds D(j) and the multipliers' numerators W(j, j + t), which
// the back substitution reuses.  Exact up to rounding: the solve reports
// one iteration and never the iteration cap.
constexpr int kDirectMax = 16;

__host__ __device__ constexpr int direct_unknowns(int m, int bc) {
    return (m - 1) * (bc == BC_FLOWCELL ? m + 1 : m - 1);
}

template <typename T>
size_t direct_lds_bytes(int m, int bc) {
    const size_t N = (size_t)direct_unknowns(m, bc);
    const size_t n0 = (size_t)(m + 1) * (m + 1);
    return (N * (size_t)m + N) * sizeof(double) + ((n0 * sizeof(T) + 7) / 8) * 8;
}

template <typename T>
__global__ __launch_bounds__(64) void k_small_direct(SmallArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int s = blockIdx.x, lane = threadIdx.x;
    const int m = a.m, w = m + 1, n0 = w * w, bc = a.bc;
    const int ylo = bc == BC_FLOWCELL ? 0 : 1, yhi = bc == BC_FLOWCELL ? m : m - 1;
    const int bw = m - 1, N = bw * (yhi - ylo + 1);
    double* Bd = reinterpret_cast<double*>(smem);    // band, Bd[i * m + d] = W(i, i + d)
    double* rv = Bd + (size_t)N * m;                 // b - A x0, then the solution update
    T* kk = reinterpret_cast<T*>(rv + N);            // nodal k
    const T* kg = a.k + (size_t)s * a.kss;
    for (int t = lane; t < n0; t += 64) kk[t] = kg[t];
    __syncthreads();
    // band rows (unknown i <-> node (1 + i mod bw, ylo + i / bw)) and the
    // right-hand side r0 = b - A x0 (x0: the Dirichlet lifting)
    {
        auto KD = [&](int gx, int gy) -> double { return (double)kk[gy * w + gx]; };
        for (int i = lane; i < N; i += 64) {
            const int yr = ylo + i / bw, xr = 1 + i % bw;
            const double ce = cond_e<double>(xr, yr, m, KD), cw = cond_e<double>(xr - 1, yr, m, KD);
            const double cn = cond_n<double>(xr, yr, m, KD), cs = cond_n<double>(xr, yr - 1, m, KD);
            double* row = Bd + (size_t)i * m;
            double d = ce + cw;
            if (yr < m) d += cn;
            if (yr > 0) d += cs;
            row[0] = d;
            for (int dd = 1; dd < m; ++dd) row[dd] = 0.0;
            if (xr + 1 <= m - 1) row[1] = -ce;
            if (i + bw < N) row[bw] -= cn;
            double v = a.f * (double)tri_count(xr, yr, m) * a.h2 * (1.0 / 6.0);
            if (xr == 1) v += cw * dirichlet_value(0, bc);
            if (xr == m - 1) v += ce * dirichlet_value(m, bc);
            if (bc != BC_FLOWCELL) {
                if (yr == 1) v += cs * dirichlet_value(xr, bc);
                if (yr == m - 1) v += cn * dirichlet_value(xr, bc);
            }
            rv[i] = v;
        }
    }
    __syncthreads();
    // this lane's entries (a, b), 1 <= a <= b <= bw, of the trailing update:
    // pair q = lane + 64 i, the b-th row of the triangle holding a = 1 .. b
    constexpr int NPL = (kDirectMax - 1) * kDirectMax / 2 / 64 + 1;
    int pa[NPL], pb[NPL];
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
        const int q = lane + 64 * i;
        int b = 1;
        while (b * (b + 1) / 2 <= q) ++b;
        pb[i] = q < bw * (bw + 1) / 2 ? b : 0;
        pa[i] = q - (b - 1) * b / 2 + 1;
    }
    for (int j = 0; j < N; ++j) {
        const double* rj = Bd + (size_t)j * m;
        const double inv = 1.0 / rj[0];
        // W(j+a, j+b) -= W(j, j+a) W(j, j+b) / D(j)
#pragma unroll
        for (int i = 0; i < NPL; ++i) {
            const int aa = pa[i], b = pb[i];
            if (b == 0 || j + b >= N) continue;
            Bd[(size_t)(j + aa) * m + (b - aa)] -= rj[aa] * rj[b] * inv;
        }
        // elimination of the right-hand side by L(j + t, j) = W(j, j + t) / D(j)
        if (lane >= 1 && lane <= bw && j + lane < N) rv[j + lane] -= rj[lane] * inv * rv[j];
        __syncthreads();
    }
    // D z = y, then L^T x = z by columns from the last unknown
    for (int i = lane; i < N; i += 64) rv[i] /= Bd[(size_t)i * m];
    __syncthreads();
    for (int j = N - 1; j >= 1; --j) {
        const double xj = rv[j];
        if (lane >= 1 && lane <= bw && j - lane >= 0) {
            const double* ri = Bd + (size_t)(j - lane) * m;
            rv[j - lane] -= ri[lane] / ri[0] * xj;
        }
        __syncthreads();
    }
    // x = x0 + update at every node (Dirichlet values on the boundary)
    double* X = a.X + (size_t)s * a.xss;
    for (int t = lane; t < n0; t += 64) {
        const int y = t / w, x = t - y * w;
        double v = dirichlet_value(x, bc);
        if (is_unknown(x, y, m, bc)) v = rv[(y - ylo) * bw + (x - 1)];
        X[t] = v;
    }
    if (lane == 0) {
        Scal& sc = a.scal[s];
        sc.bb = 0.0;
        sc.rr = 0.0;
        sc.it = 1;
        sc.status = 0;
        sc.active = 0;
    }
}

// ----------------------------------------------------------- PCG (double)
constexpr int PTX = 64, PTY = 16;

// A QoI that is linear in u, Q(x) = Q(x0) + w.(x - x0), needs no iterate:
// with x0 the Dirichlet lifting and x - x0 = sum_k alpha_k p_k, the solve
// accumulates alpha_k w.p_k per sample and never stores x.  Weights w:
// integral, the load weights tri_count h^2 / 6; point value, the three P1
// barycentric weights of the triangle holding the point; outflux through
// x1 = 1, the conductance of the edge from (m-1, j) to the boundary node
// (m, j) (there b - A x is linear in the neighbouring unknown).
struct QoiLin {
    int on, kind;
    int pi, pj;                     // point: lower-left node of its square
    double w00, w10, w11, w01;      // point: weights of (pi,pj), (pi+1,pj), (pi+1,pj+1), (pi,pj+1)
};

template <typename T>
struct PcgArgs {
    Lvl L;
    int bc, tiles_x, ntiles;
    double f, h2;
    const T* k;
    long long kss;
    double *X, *R, *Pold, *Pnew, *Q;
    T* Z;   // preconditioned residual (precision of the multigrid)
    double* part;
    double* part2;   // partial w.p (linear QoI)
    Scal* scal;
    QoiLin ql;
};

// weight of unknown (gx, gy) in a linear QoI; ce is the conductance of the
// east edge of the node
__device__ __forceinline__ double qoi_weight(const QoiLin& q, int gx, int gy, int m, double h2, double ce) {
    if (q.kind == Q_INTEGRAL) return (double)tri_count(gx, gy, m) * h2 * (1.0 / 6.0);
    if (q.kind == Q_OUTFLUX) return gx == m - 1 ? ce : 0.0;
    double w = 0.0;
    if (gy == q.pj) w = gx == q.pi ? q.w00 : (gx == q.pi + 1 ? q.w10 : 0.0);
    else if (gy == q.pj + 1) w = gx == q.pi + 1 ? q.w11 : (gx == q.pi ? q.w01 : 0.0);
    return w;
}

// ------------------------------- direct solve for a linear QoI, m <= 32
// A QoI linear in u needs no x: with A = L D L^T,
// w.(x - x0) = w^T A^-1 r0 = (L^-1 w)^T D^-1 (L^-1 r0), and L^-1 r0 and
// L^-1 w are eliminated along with the factorisation, so nothing behind the
// pivot is kept.  The band's active window -- rows j .. j + MB - 1 at pivot
// j, half-bandwidth m - 1 < MB -- lives in registers: 16 lanes per sample
// (four samples per wave), lane kap holding the columns c = kap + 16 h
// (h < MB / 16) of every window row, with rows and columns numbered mod MB
// (a ring: once row j is eliminated its slot takes row j + MB).  Register
// R[h][rho] holds W(r, r + d) for the window row r = rho (mod MB) and
// d = (c - rho) mod MB; the update of step j,
// W(j+a, j+b) -= W(j, j+a) W(j, j+b) / D(j) for 1 <= a <= b <= m - 1, is then
// register (h, j+a) -= [pivot entry at column j+a, broadcast] x [own pivot
// entry W(j, j+b)] / D(j), masked to the lanes with b >= a.  A row of 16
// lanes is one sample, so the broadcasts are DPP row broadcasts: no LDS and
// no barriers in the elimination.  The ring is renumbered every 16 pivots
// (for MB = 32 by swapping its halves), so every register index is a
// compile-time constant.  Exact up to rounding: one iteration, never the cap.
template <int L>
__device__ __forceinline__ double row_bcast(double v) {
    return __longlong_as_double(__builtin_amdgcn_mov_dpp(__double_as_longlong(v), 0x150 + L, 0xF, 0xF, false));
}

// b on the lanes whose bit of the compile-time lane pattern M is set, a on
// the others: a v_cndmask with the pattern as a scalar operand.  z is a
// scalar zero defined where the blend is used, so that the pattern is
// formed there (as M ^ z) and not hoisted out of the loop: the patterns of
// all pivots together would not fit in SGPRs.
template <unsigned long long M>
__device__ __forceinline__ double lane_blend(double a, double b, unsigned long long z) {
    if constexpr (M == ~0ull) {
        return b;
    } else if constexpr (M == 0ull) {
        return a;
    } else {
        const unsigned long long mz = M ^ z;
        int lo, hi;
        asm("v_cndmask_b32 %0, %1, %2, %3" : "=v"(lo) : "v"(__double2loint(a)), "v"(__double2loint(b)), "s"(mz));
        asm("v_cndmask_b32 %0, %1, %2, %3" : "=v"(hi) : "v"(__double2hiint(a)), "v"(__double2hiint(b)), "s"(mz));
        return __hiloint2double(hi, lo);
    }
}

__device__ __forceinline__ unsigned long long scalar_zero() {
    unsigned long long z;
    asm volatile("s_mov_b64 %0, 0" : "=s"(z));
    return z;
}

// lanes (in every row of 16) whose window column c = kap + 16 h has
// (c - rho) mod MB in [lo, hi]
template <int MB>
constexpr unsigned long long ring_lanes(int rho, int h, int lo, int hi) {
    unsigned long long m = 0;
    for (int k = 0; k < 16; ++k) {
        const int d = (k + 16 * h - rho) & (MB - 1);
        if (d >= lo && d <= hi) m |= 1ull << k;
    }
    return m * 0x0001000100010001ull;
}

template <int I, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (I < E) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, E>(f);
    }
}

constexpr int kDirectLinMax = 32;

template <typename T>
size_t direct_lin_lds_bytes(int m) {
    return 4 * (size_t)(m + 1) * (m + 1) * sizeof(T);
}

template <typename T, int MB, bool FULL>
__global__ __launch_bounds__(64) void k_direct_lin(SmallArgs<T> a, QoiLin ql) {
    static_assert(MB == 16 || MB == 32, "window of 16 or 32 rows");
    constexpr int C = MB / 16;
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x, sub = lane >> 4, kap = lane & 15;
    const int s = blockIdx.x * 4 + sub;
    const bool live = s < a.S;
    const int m = FULL ? MB : a.m, w = m + 1, n0 = w * w, bc = a.bc;
    const int ylo = bc == BC_FLOWCELL ? 0 : 1, yhi = bc == BC_FLOWCELL ? m : m - 1;
    const int bw = m - 1, N = bw > 0 ? bw * (yhi - ylo + 1) : 0;
    T* kk = reinterpret_cast<T*>(smem) + (size_t)sub * n0;
    {
        const T* kg = a.k + (size_t)(live ? s : a.S - 1) * a.kss;
        for (int t = kap; t < n0; t += 16) kk[t] = kg[t];
    }
    __syncthreads();
    auto KD = [&](int gx, int gy) -> double { return (double)kk[gy * w + gx]; };
    auto node = [&](int r, int& x, int& y) {
        const int q = r / bw;
        y = ylo + q;
        x = 1 + r - q * bw;
    };
    // per column: diagonal, right-hand side r0 = b - A x0 and QoI weight of
    // row J0 + c, the east entry that row J0 + (c - 1 mod MB) has in column
    // c, and the north entry of row J0 + (c - bw mod MB)
    double nd[C], ne[C], nn[C], ny[C], nw[C];
    auto prep = [&](int J0) {
#pragma unroll
        for (int h = 0; h < C; ++h) {
            const int c = kap + 16 * h;
            nd[h] = 1.0;
            ny[h] = nw[h] = ne[h] = nn[h] = 0.0;
            int r = J0 + c, x, y;
            if (r < N) {
                node(r, x, y);
                const double ce = cond_e<double>(x, y, m, KD), cw = cond_e<double>(x - 1, y, m, KD);
                const double cn = cond_n<double>(x, y, m, KD), cs = cond_n<double>(x, y - 1, m, KD);
                double d = ce + cw;
                if (y < m) d += cn;
                if (y > 0) d += cs;
                nd[h] = d;
                double v = a.f * (double)tri_count(x, y, m) * a.h2 * (1.0 / 6.0);
                if (x == 1) v += cw * dirichlet_value(0, bc);
                if (x == m - 1) v += ce * dirichlet_value(m, bc);
                if (bc != BC_FLOWCELL) {
                    if (y == 1) v += cs * dirichlet_value(x, bc);
                    if (y == m - 1) v += cn * dirichlet_value(x, bc);
                }
                ny[h] = v;
                nw[h] = qoi_weight(ql, x, y, m, a.h2, ce);
            }
            r = J0 + ((c - 1) & (MB - 1));
            if (r < N) {
                node(r, x, y);
                if (x + 1 <= m - 1) ne[h] = -cond_e<double>(x, y, m, KD);
            }
            r = J0 + ((c - bw) & (MB - 1));
            if (r + bw < N) {
                node(r, x, y);
                nn[h] = -cond_n<double>(x, y, m, KD);
            }
        }
    };
    double R[C][MB], Y[C] = {}, YW[C] = {};
    // ring slot RHO takes the prepared row: the diagonal in column RHO, the
    // east entry in column RHO + 1, the north entry in column RHO + bw
    auto load_row = [&](auto rho_ic) {
        constexpr int RHO = decltype(rho_ic)::value;
        const unsigned long long z = scalar_zero();
        static_for<0, C>([&](auto h_ic) {
            constexpr int h = decltype(h_ic)::value;
            constexpr unsigned long long M0 = ring_lanes<MB>(RHO, h, 0, 0), M1 = ring_lanes<MB>(RHO, h, 1, 1);
            double v = lane_blend<M1>(lane_blend<M0>(0.0, nd[h], z), ne[h], z);
            if constexpr (FULL) {
                v = lane_blend<ring_lanes<MB>(RHO, h, MB - 1, MB - 1)>(v, nn[h], z);
            } else {
                int d = (kap + 16 * h - RHO) & (MB - 1);
                asm volatile("" : "+v"(d));
                if (d == bw) v += nn[h];
            }
            R[h][RHO] = v;
            Y[h] = lane_blend<M0>(Y[h], ny[h], z);
            YW[h] = lane_blend<M0>(YW[h], nw[h], z);
        });
    };
    prep(0);
    static_for<0, MB>(load_row);
    double qacc = 0.0;
    for (int J = 0; J < N; J += 16) {
        prep(J + MB);
        static_for<0, 16>([&](auto rj_ic) {
            constexpr int RJ = decltype(rj_ic)::value;
            if (J + RJ >= N) return;
            // pivot row J + RJ: ring slot RJ, its diagonal in lane RJ of h = 0
            const double D = row_bcast<RJ>(R[0][RJ]);
            const double inv = 1.0 / D;
            const double yj = row_bcast<RJ>(Y[0]), ywj = row_bcast<RJ>(YW[0]);
            const unsigned long long z = scalar_zero();
            // own pivot entry W(j, j + b), b = (c - RJ) mod MB, over -D(j)
            double pmn[C];
#pragma unroll
            for (int h = 0; h < C; ++h) pmn[h] = -R[h][RJ] * inv;
            static_for<1, MB>([&](auto a_ic) {
                constexpr int A = decltype(a_ic)::value;
                constexpr int CS = (RJ + A) & (MB - 1);
                if (!FULL && A > bw) return;
                const double u = row_bcast<CS & 15>(R[CS >> 4][RJ]);   // W(j, j + A)
                static_for<0, C>([&](auto h_ic) {
                    constexpr int h = decltype(h_ic)::value;
                    // lanes with b >= A take the update
                    constexpr unsigned long long M = ring_lanes<MB>(RJ, h, A, MB - 1);
                    if constexpr (M != 0ull) R[h][CS] = fma(u, lane_blend<M>(0.0, pmn[h], z), R[h][CS]);
                });
            });
            static_for<0, C>([&](auto h_ic) {
                constexpr int h = decltype(h_ic)::value;
                const double f = lane_blend<ring_lanes<MB>(RJ, h, 1, MB - 1)>(0.0, pmn[h], z);
                Y[h] = fma(f, yj, Y[h]);
                YW[h] = fma(f, ywj, YW[h]);
            });
            qacc = fma(yj * ywj, inv, qacc);
            load_row(rj_ic);
        });
        if constexpr (MB == 32) {
            static_for<0, 16>([&](auto r_ic) {
                constexpr int r = decltype(r_ic)::value;
                const double t0 = R[0][r];
                R[0][r] = R[1][r + 16];
                R[1][r + 16] = t0;
                const double t1 = R[0][r + 16];
                R[0][r + 16] = R[1][r];
                R[1][r] = t1;
            });
            const double ty = Y[0], tw = YW[0];
            Y[0] = Y[1];
            Y[1] = ty;
            YW[0] = YW[1];
            YW[1] = tw;
        }
    }
    if (live && kap == 0) {
        Scal& sc = a.scal[s];
        sc.bb = 0.0;
        sc.rr = 0.0;
        sc.qacc = qacc;
        sc.it = 1;
        sc.status = 0;
        sc.active = 0;
    }
}

template <typename T>
struct KTile {
    double k[PTY + 2][PTX + 2];
};

template <typename T>
__device__ void load_ktile(KTile<T>& K, const T* __restrict__ k, int x0, int y0, int m, int w) {
    for (int t = threadIdx.x; t < (PTX + 2) * (PTY + 2); t += blockDim.x) {
        const int y = t / (PTX + 2), x = t - y * (PTX + 2);
        const int gx = x0 - 1 + x, gy = y0 - 1 + y;
        K.k[y][x] = (gx >= 0 && gx <= m && gy >= 0 && gy <= m) ? (double)k[(size_t)gy * w + gx] : 0.0;
    }
}

// init over the full (m+1)^2 grid: x = Dirichlet lifting, r = b - A x at
// unknowns (zero elsewhere); partial ||r||^2.  p, q and z need no reset:
// off the unknowns (boundary nodes, stride padding) they are zero from the
// workspace's allocation and never written, z is written before it is
// read, and the first direction does not read p_old.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pcg_init(PcgArgs<T> a) {
    __shared__ KTile<T> K;
    __shared__ double red[kBlock / 64];
    const int wi = xcd_remap(blockIdx.x, gridDim.x);
    const int s = wi / a.ntiles, tile = wi - s * a.ntiles;
    const int ty = tile / a.tiles_x, tx = tile - ty * a.tiles_x;
    const int x0 = tx * PTX, y0 = ty * PTY;
    const int m = a.L.m, w = a.L.w;
    // only the flow cell carries nonzero Dirichlet data (u = 1 at x1 = 0),
    // so only it needs k for the lifting's contribution to r
    const bool lift = a.bc == BC_FLOWCELL;
    if (lift) load_ktile(K, a.k + (size_t)s * a.kss, x0, y0, m, w);
    __syncthreads();
    auto KF = [&](int gx, int gy) -> double { return K.k[gy - y0 + 1][gx - x0 + 1]; };
    const size_t base = (size_t)s * a.L.ss;
    double acc = 0.0;
    for (int t = threadIdx.x; t < PTX * PTY; t += blockDim.x) {
        const int yy = t / PTX, xx = t - yy * PTX;
        const int gx = x0 + xx, gy = y0 + yy;
        if (gx > m || gy > m) continue;
        const size_t o = base + (size_t)gy * w + gx;
        double xv = 0.0, rv = 0.0;
        if (is_unknown(gx, gy, m, a.bc)) {
            rv = a.f * (double)tri_count(gx, gy, m) * a.h2 * (1.0 / 6.0);
            if (lift) {
                // neighbours carrying Dirichlet data
                if (!is_unknown(gx + 1, gy, m, a.bc) && gx + 1 <= m) rv += cond_e<double>(gx, gy, m, KF) * dirichlet_value(gx + 1, a.bc);
                if (!is_unknown(gx - 1, gy, m, a.bc) && gx - 1 >= 0) rv += cond_e<double>(gx - 1, gy, m, KF) * dirichlet_value(gx - 1, a.bc);
                if (!is_unknown(gx, gy + 1, m, a.bc) && gy + 1 <= m) rv += cond_n<double>(gx, gy, m, KF) * dirichlet_value(gx, a.bc);
                if (!is_unknown(gx, gy - 1, m, a.bc) && gy - 1 >= 0) rv += cond_n<double>(gx, gy - 1, m, KF) * dirichlet_value(gx, a.bc);
            }
            acc += rv * rv;
        } else {
            xv = dirichlet_value(gx, a.bc);
        }
        if (a.X) a.X[o] = xv;   // not kept by linear-QoI solves
        a.R[o] = rv;
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) a.part[(size_t)s * a.ntiles + tile] = acc;
}

// p_new = z + beta p_old; q = A p_new; partial p_new.q (unknown-region tiles).
// Lane l of wave wv owns column x0 + l, rows y0 + 4 wv .. y0 + 4 wv + 3.
// Conductances from the triangle sums of the k tile (double).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pcg_dir(PcgArgs<T> a, int first) {
    constexpr int KX = PTX + 2, KY = PTY + 2, NR = PTY / (kBlock / 64);
    __shared__ double K[KY * KX];
    __shared__ double P[KY * KX];
    __shared__ double red[2 * (kBlock / 64)];
    const int wi = xcd_remap(blockIdx.x, gridDim.x);
    const int s = wi / a.ntiles, tile = wi - s * a.ntiles;
    const Scal sc = a.scal[s];
    if (!sc.active) return;
    // beta = r.z / r_old.z_old: the multigrid preconditioner is symmetric
    // (its sweeps are mirrored) and fixed, so plain PCG applies; measured to
    // take the same iterations as the flexible (Polak-Ribiere) form, whose
    // z.q_old would cost a read of q_old per unknown and iteration
    const double beta = first ? 0.0 : sc.rz / sc.rz_old;
    const int ty = tile / a.tiles_x, tx = tile - ty * a.tiles_x;
    const int x0 = 1 + tx * PTX, y0 = a.L.ylo + ty * PTY;
    const int m = a.L.m, w = a.L.w, bc = a.bc;
    const size_t base = (size_t)s * a.L.ss;
    const T* kk = a.k + (size_t)s * a.kss;
    const T* Z = a.Z + base;
    const double* Po = a.Pold + base;
    // tile + one-node ring: flat index, loads first (clamped), then masked stores
    constexpr int NT = (KX * KY + kBlock - 1) / kBlock;
    double kv[NT], zv[NT], pv[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) {
        const int t = threadIdx.x + i * kBlock;
        const int y = t / KX, x = t - y * KX;
        const int gx = min(max(x0 - 1 + x, 0), m), gy = min(max(y0 - 1 + y, 0), m);
        const int o = gy * w + gx;
        kv[i] = (double)kk[o];
        zv[i] = (double)Z[o];
        pv[i] = Po[o];
    }
#pragma unroll
    for (int i = 0; i < NT; ++i) {
        const int t = threadIdx.x + i * kBlock;
        if (t >= KX * KY) break;
        const int y = t / KX, x = t - y * KX;
        const int gx = x0 - 1 + x, gy = y0 - 1 + y;
        const bool in = gx >= 0 && gx <= m && gy >= 0 && gy <= m;
        K[t] = in ? kv[i] : 0.0;
        P[t] = is_unknown(gx, gy, m, bc) ? (first ? zv[i] : zv[i] + beta * pv[i]) : 0.0;
    }
    __syncthreads();
    const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int gx = x0 + l;
    const bool sqm = gx - 1 >= 0 && gx - 1 <= m - 1, sqa = gx >= 0 && gx <= m - 1;
    const bool unkc = gx >= 1 && gx <= m - 1;
    double acc = 0.0;
    // triangle sums S1 (below the diagonal), S2 (above) of squares (gx-1, y) and (gx, y)
    const double* k0 = K + (NR * wv) * KX + l;   // tile coords (l-1, row-1) -> padded (l, row)
    double s1m_p, s2m_p, s2a_p;
    {
        const int gy = y0 + NR * wv - 1;
        const bool sqr = gy >= 0 && gy <= m - 1;
        const double km = k0[0], ka = k0[1], um = k0[KX], ua = k0[KX + 1], ub = k0[KX + 2];
        s1m_p = (sqr && sqm) ? km + ka + ua : 0.0;
        s2m_p = (sqr && sqm) ? km + ua + um : 0.0;
        s2a_p = (sqr && sqa) ? ka + ub + ua : 0.0;
    }
    const double sixth = 1.0 / 6.0;
    double cS = (s2a_p + s1m_p) * sixth;
    double accw = 0.0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int yy = NR * wv + r, gy = y0 + yy;
        const bool sqr = gy >= 0 && gy <= m - 1;
        const double* kr = k0 + (r + 1) * KX;
        const double km = kr[0], ka = kr[1], kb = kr[2], um = kr[KX], ua = kr[KX + 1], ub = kr[KX + 2];
        const double s1m = (sqr && sqm) ? km + ka + ua : 0.0;
        const double s2m = (sqr && sqm) ? km + ua + um : 0.0;
        const double s1a = (sqr && sqa) ? ka + kb + ub : 0.0;
        const double s2a = (sqr && sqa) ? ka + ub + ua : 0.0;
        const double cE = (s1a + s2a_p) * sixth, cW = (s1m + s2m_p) * sixth, cN = (s2a + s1m) * sixth;
        const double* pp = P + (yy + 1) * KX + l + 1;
        const double pc = pp[0];
        const double q = (cE * (pc - pp[1]) + cW * (pc - pp[-1])) + (cN * (pc - pp[KX]) + cS * (pc - pp[-KX]));
        if (unkc && gy >= a.L.ylo && gy <= a.L.yhi) {
            const size_t o = base + (size_t)gy * w + gx;
            a.Pnew[o] = pc;
            a.Q[o] = q;
            acc += pc * q;
            if (a.ql.on) accw += qoi_weight(a.ql, gx, gy, m, a.h2, cE) * pc;
        }
        s1m_p = s1m; s2m_p = s2m; s2a_p = s2a;
        cS = cN;
    }
    if (a.ql.on) {
        block_sum2(acc, accw, red);
        if (threadIdx.x == 0) a.part2[(size_t)s * a.ntiles + tile] = accw;
    } else {
        acc = block_sum(acc, red);
    }
    if (threadIdx.x == 0) a.part[(size_t)s * a.ntiles + tile] = acc;
}

// x += alpha p; r -= alpha q; partial ||r||^2.  Elementwise over each
// sample's whole padded node range, two nodes per lane per access (16 bytes):
// off the unknowns p, q and r are zero (x keeps its boundary values), so no
// masks are needed.  Every access is non-temporal: a chunk's vectors are far
// larger than the caches and are next read by another kernel, so caching
// them only evicts useful lines.  Block b of a sample covers nodes
// [b * kUpdChunk, (b+1) * kUpdChunk); its partial sum goes to part[b].
constexpr int kUpdChunk = 4 * 2 * kBlock;   // nodes per workgroup
typedef double dvec2 __attribute__((ext_vector_type(2)));

// KEEPX = false (a linear QoI accumulated per iteration) skips x and p.
template <bool KEEPX>
__global__ __launch_bounds__(kBlock) void k_pcg_update(double* __restrict__ X, double* __restrict__ R,
                                                       const double* __restrict__ P, const double* __restrict__ Q,
                                                       long long ss, int nb, double* __restrict__ part,
                                                       const Scal* __restrict__ scal) {
    __shared__ double red[kBlock / 64];
    const int s = blockIdx.y, b = blockIdx.x;
    const Scal sc = scal[s];
    if (!sc.active) return;
    const double alpha = sc.rz / sc.pq;
    const size_t base = (size_t)s * ss;
    constexpr int V = kUpdChunk / (2 * kBlock);
    dvec2 xv[V], rv[V], pv[V], qv[V];
    long long o[V];
#pragma unroll
    for (int i = 0; i < V; ++i) {
        o[i] = (long long)b * kUpdChunk + 2LL * (i * kBlock + threadIdx.x);
        const long long oc = o[i] < ss ? o[i] : 0;   // ss is even: pairs never straddle the end
        if (KEEPX) {
            xv[i] = __builtin_nontemporal_load(reinterpret_cast<const dvec2*>(X + base + oc));
            pv[i] = __builtin_nontemporal_load(reinterpret_cast<const dvec2*>(P + base + oc));
        }
        rv[i] = __builtin_nontemporal_load(reinterpret_cast<const dvec2*>(R + base + oc));
        qv[i] = __builtin_nontemporal_load(reinterpret_cast<const dvec2*>(Q + base + oc));
    }
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < V; ++i) {
        if (o[i] >= ss) continue;
        dvec2 rn;
        if (KEEPX) {
            dvec2 xn;
            xn.x = xv[i].x + alpha * pv[i].x;
            xn.y = xv[i].y + alpha * pv[i].y;
            __builtin_nontemporal_store(xn, reinterpret_cast<dvec2*>(X + base + o[i]));
        }
        rn.x = rv[i].x - alpha * qv[i].x;
        rn.y = rv[i].y - alpha * qv[i].y;
        __builtin_nontemporal_store(rn, reinterpret_cast<dvec2*>(R + base + o[i]));
        acc += rn.x * rn.x + rn.y * rn.y;
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) part[(size_t)s * nb + b] = acc;
}

enum { RED_BB = 0, RED_RZ = 1, RED_PQ = 2, RED_RR = 3 };

template <int WHAT>
__global__ __launch_bounds__(kBlock) void k_reduce(const double* __restrict__ part, const double* __restrict__ part2,
                                                   int np, Scal* scal, double rtol2, int maxit, int* active_count) {
    __shared__ double red[kBlock / 64];
    const int s = blockIdx.x;
    if (WHAT != RED_BB && !scal[s].active) return;
    double acc = 0.0, acc2 = 0.0;
    for (int t = threadIdx.x; t < np; t += blockDim.x) acc += part[(size_t)s * np + t];
    acc = block_sum(acc, red);
    if (WHAT == RED_PQ && part2) {
        for (int t = threadIdx.x; t < np; t += blockDim.x) acc2 += part2[(size_t)s * np + t];
        acc2 = block_sum(acc2, red);
    }
    if (threadIdx.x != 0) return;
    Scal& sc = scal[s];
    if (WHAT == RED_BB) {
        sc.bb = acc;
        sc.it = 0;
        sc.rz = sc.rz_old = sc.pq = sc.qacc = 0.0;
        sc.rr = acc;
        sc.status = 0;
        sc.active = acc > 0.0 ? 1 : 0;
        if (sc.active) atomicAdd(active_count, 1);
    } else if (WHAT == RED_RZ) {
        sc.rz = acc;
    } else if (WHAT == RED_PQ) {
        sc.pq = acc;
        if (part2) {
            // the step alpha = rz / pq of this iteration, as the update takes it
            sc.qacc += (sc.rz / sc.pq) * acc2;
        }
    } else {
        sc.rr = acc;
        sc.it += 1;
        sc.rz_old = sc.rz;
        if (acc <= rtol2 * sc.bb) {
            sc.active = 0;
            sc.status = 0;
            atomicSub(active_count, 1);
        } else if (sc.it >= maxit) {
            sc.active = 0;
            sc.status = -4;
            atomicSub(active_count, 1);
        }
    }
}

// QoI of the P1 solution x (double) per sample; one workgroup per sample.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_qoi(const double* __restrict__ X, Lvl L, int bc, double f, int qoi,
                                                double qx, double qy, const T* __restrict__ k, long long kss,
                                                const Scal* scal, int lin, double* q, int* iters) {
    __shared__ double red[kBlock / 64];
    const int s = blockIdx.x;
    const int m = L.m, w = L.w;
    const double h = 1.0 / m, h2 = h * h;
    // a linear-QoI solve keeps no iterate: x is the lifting x0 here, taken
    // from its definition
    const double* xs = X + (size_t)s * L.ss;
    auto xat = [&](int t) -> double { return lin ? dirichlet_value(t % w, bc) : xs[t]; };
    double acc = 0.0;
    if (qoi == Q_INTEGRAL) {
        for (int t = threadIdx.x; t < w * w; t += blockDim.x) {
            const int j = t / w, i = t - j * w;
            acc += xat(t) * (double)tri_count(i, j, m);
        }
        acc = block_sum(acc, red) * (h2 / 6.0);
    } else if (qoi == Q_L2) {
        for (int t = threadIdx.x; t < m * m; t += blockDim.x) {
            const int j = t / m, i = t - j * m;
            const double a00 = xat(j * w + i), a10 = xat(j * w + i + 1), a11 = xat((j + 1) * w + i + 1),
                         a01 = xat((j + 1) * w + i);
            const double s1 = a00 + a10 + a11, s2 = a00 + a11 + a01;
            acc += (a00 * a00 + a10 * a10 + a11 * a11 + s1 * s1) + (a00 * a00 + a11 * a11 + a01 * a01 + s2 * s2);
        }
        acc = sqrt(block_sum(acc, red) * (h2 / 24.0));
    } else if (qoi == Q_POINT) {
        int i = min((int)floor(qx / h), m - 1), j = min((int)floor(qy / h), m - 1);
        const double sx = qx / h - i, sy = qy / h - j;
        if (sx >= sy)
            acc = (1 - sx) * xat(j * w + i) + (sx - sy) * xat(j * w + i + 1) + sy * xat((j + 1) * w + i + 1);
        else
            acc = (1 - sy) * xat(j * w + i) + sx * xat((j + 1) * w + i + 1) + (sy - sx) * xat((j + 1) * w + i);
    } else {  // outflux through x1 = 1: sum_j (b - A x) at (m, j)
        const T* kk = k + (size_t)s * kss;
        auto KF = [&](int gx, int gy) -> double { return (double)kk[(size_t)gy * w + gx]; };
        for (int j = threadIdx.x; j <= m; j += blockDim.x) {
            const int i = m;
            const double xp = xat(j * w + i);
            double ax = cond_e<double>(i - 1, j, m, KF) * (xp - xat(j * w + i - 1));
            if (j < m) ax += cond_n<double>(i, j, m, KF) * (xp - xat((j + 1) * w + i));
            if (j > 0) ax += cond_n<double>(i, j - 1, m, KF) * (xp - xat((j - 1) * w + i));
            acc += f * (double)tri_count(i, j, m) * h2 / 6.0 - ax;
        }
        acc = block_sum(acc, red);
    }
    if (threadIdx.x == 0) {
        // linear QoI: x holds the lifting x0, the solve accumulated w.(x - x0)
        if (lin) acc += scal[s].qacc;
        if (q) q[s] = acc;
        if (iters) iters[s] = scal[s].status == 0 ? scal[s].it : -scal[s].it;
    }
}

__global__ __launch_bounds__(kBlock) void k_zero(uint4* __restrict__ dst, long long n16, unsigned* __restrict__ tail,
                                               int ntail) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        dst[i] = make_uint4(0u, 0u, 0u, 0u);
    if (blockIdx.x == 0 && (int)threadIdx.x < ntail) tail[threadIdx.x] = 0u;
}

__global__ void k_set_int(int* dst, int v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = v;
}

__global__ __launch_bounds__(kBlock) void k_finalize(const double* qf, const double* qc, const int* itf,
                                                     const int* itc, int slot0, int nslots, long long out0,
                                                     double* y, double* yf, double* yc, int* iters, int* status) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nslots) return;
    const int sl = slot0 + t;
    const double a = qf[sl];
    const double b = qc ? qc[sl] : 0.0;
    const long long o = out0 + t;
    y[o] = a - b;
    if (yf) yf[o] = a;
    if (yc) yc[o] = b;
    const int i1 = itf[sl];
    const int i2 = itc ? itc[sl] : 1;
    if (iters) iters[o] = i1;
    if (status) status[o] = (i1 < 0 || i2 < 0) ? -4 : 0;
}

// ---------------------------------------------------------------- host --
size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

template <typename T>
class SolverImpl final : public Solver {
public:
    // tile shapes by precision (LDS <= 64 KiB per workgroup)
    // multigrid tile: 64 columns x 8*SH rows region (SH rows per half-wave)
    static constexpr int SH = sizeof(T) == 4 ? 8 : 4;
    static constexpr int RYT = (kBlock / 32) * SH;
    static constexpr int PRE_TX = 64 - 12, PRE_TY = RYT - 12;   // halo 6
    static constexpr int POST_TX = 64 - 8, POST_TY = RYT - 8;   // halo 4
    static constexpr int MB = sizeof(T) == 4 ? 32 : 16;
    static constexpr int RING = 4;   // iterations that may be unconfirmed

    SolverCfg cfg_;
    int cap_;

    SolverImpl(const SolverCfg& cfg, int cap) : cfg_(cfg), cap_(cap) {
        for (int mm = cfg.m; mm >= 2; mm /= 2) {
            Lvl l;
            l.m = mm;
            l.w = mm + 1;
            l.ss = (long long)align_up((size_t)l.w * l.w, 64);
            l.ylo = cfg.bc == BC_FLOWCELL ? 0 : 1;
            l.yhi = cfg.bc == BC_FLOWCELL ? mm : mm - 1;
            lv_.push_back(l);
        }
        nlev_ = (int)lv_.size();
        small_ = cfg.m <= kSmallMax;
        size_t off = 0;
        auto take = [&](size_t bytes) {
            size_t o = off;
            off = align_up(off + bytes, 256);
            return o;
        };
        const Lvl& L0 = lv_[0];
        const size_t n0 = (size_t)cap * L0.ss;
        if (small_) {
            o_X_ = take(n0 * 8);
            o_scal_ = take((size_t)cap * sizeof(Scal));
            o_q_ = take((size_t)cap * 8);
            o_it_ = take((size_t)cap * 4);
            bytes_ = off;
            return;
        }
        lb_ = 0;
        while (lv_[lb_].m > MB) ++lb_;
        ptx_ = cdiv(L0.m - 1, PTX);
        pty_ = cdiv(L0.yhi - L0.ylo + 1, PTY);
        ptiles_ = ptx_ * pty_;
        itx_ = cdiv(L0.m + 1, PTX);
        ity_ = cdiv(L0.m + 1, PTY);
        itiles_ = itx_ * ity_;
        stx_ = cdiv(L0.m - 1, POST_TX);
        sty_ = cdiv(L0.yhi - L0.ylo + 1, POST_TY);
        rz_parts_ = (whole(0) || whole128(0)) ? 1 : stx_ * sty_;
        ublocks_ = (int)cdiv(L0.ss, kUpdChunk);
        max_parts_ = std::max(std::max(std::max(ptiles_, itiles_), rz_parts_), ublocks_);
        o_X_ = take(n0 * 8); o_R_ = take(n0 * 8); o_P0_ = take(n0 * 8); o_P1_ = take(n0 * 8);
        o_Q_ = take(n0 * 8); o_Z_ = take(n0 * sizeof(T));
        o_za0_ = take(n0 * sizeof(T));
        for (int l = 1; l < nlev_; ++l) {
            const size_t nl = (size_t)cap * lv_[l].ss * sizeof(T);
            o_ce_.push_back(take(nl));
            o_cn_.push_back(take(nl));
            o_rhs_.push_back(take(nl));
            o_za_.push_back(take(nl));
            o_zb_.push_back(take(nl));
        }
        if (twice1_tiled()) o_zm_ = take((size_t)cap * lv_[1].ss * sizeof(T));
        o_part_ = take((size_t)cap * max_parts_ * 8);
        o_part2_ = take((size_t)cap * max_parts_ * 8);
        o_scal_ = take((size_t)cap * sizeof(Scal));
        o_q_ = take((size_t)cap * 8);
        o_it_ = take((size_t)cap * 4);
        o_cnt_ = take(64);
        bytes_ = off;
    }
    ~SolverImpl() override {
        for (auto& G : graphs_)
            for (auto& x : G.exec)
                if (x) (void)hipGraphExecDestroy(x);
        if (cap_stream_) (void)hipStreamDestroy(cap_stream_);
        if (base_) alloc_->release(base_);
        if (hcnt_) pinned_slot_release(hcnt_);
        for (auto& e : ev_)
            if (e) (void)hipEventDestroy(e);
    }
    bool alloc(DeviceAllocator* a, hipStream_t st, std::string* err, bool zero) {
        alloc_ = a;
        hipError_t e = alloc_->alloc(bytes_, &base_);
        if (e != hipSuccess) {
            base_ = nullptr;
            *err = std::string("solver workspace allocation failed: ") + hipGetErrorString(e);
            return false;
        }
        if (zero) e = launch_zero(base_, bytes_, st);
        if (e == hipSuccess) {
            hcnt_ = pinned_slot_acquire();
            if (!hcnt_) e = hipErrorOutOfMemory;
        }
        for (auto& ev : ev_)
            if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess && small_) {
            e = cfg_.m > kDirectMax ? allow_lds(k_small_pcg<T, small_threads(32), 32>, small_lds_bytes<T>(cfg_.m))
                                    : allow_lds(k_small_direct<T>, direct_lds_bytes<T>(cfg_.m, cfg_.bc));
        }
        if (e != hipSuccess) {
            *err = std::string("solver set-up failed: ") + hipGetErrorString(e);
            return false;
        }
        return true;
    }
    int capacity() const override { return cap_; }
    size_t bytes() const override { return bytes_; }
    int mg_levels() const override { return nlev_; }
    const double* x() const override { return ptr<double>(o_X_); }
    long long xstride() const override { return lv_[0].ss; }

    hipError_t begin(const void* kv, long long kss, int S, hipStream_t st, bool keep_x) override {
        k0_ = reinterpret_cast<const T*>(kv);
        lin_ = !keep_x && cfg_.qoi != Q_L2;
        kss_ = kss;
        S_ = S;
        it_next_ = confirmed_ = 0;
        done_ = S <= 0;
        recs_.clear();
        if (done_) return hipSuccess;
        const double sT = sizeof(T);
        if (small_) {
            SmallArgs<T> a{};
            a.nl = nlev_;
            a.bc = cfg_.bc;
            a.maxit = cfg_.maxit;
            a.m = cfg_.m;
            a.xss = lv_[0].ss;
            a.f = cfg_.f;
            a.h2 = 1.0 / ((double)cfg_.m * cfg_.m);
            a.rtol2 = cfg_.rtol * cfg_.rtol;
            a.k = k0_;
            a.kss = kss;
            a.X = ptr<double>(o_X_);
            a.scal = ptr<Scal>(o_scal_);
            a.S = S;
            if (lin_) {
                const QoiLin ql = qoi_lin();
                const dim3 g((unsigned)cdiv(S, 4));
                const size_t lds = direct_lin_lds_bytes<T>(cfg_.m);
                launch("direct_lin", nv(0) * sT, S, -1, st, [&](const Profiler::Slot& ps) {
                    if (cfg_.m == 16)
                        PLAUNCH((k_direct_lin<T, 16, true>), g, dim3(64), lds, st, a, ql);
                    else if (cfg_.m < 16)
                        PLAUNCH((k_direct_lin<T, 16, false>), g, dim3(64), lds, st, a, ql);
                    else if (cfg_.m == 32)
                        PLAUNCH((k_direct_lin<T, 32, true>), g, dim3(64), lds, st, a, ql);
                    else
                        PLAUNCH((k_direct_lin<T, 32, false>), g, dim3(64), lds, st, a, ql);
                });
            } else if (cfg_.m <= kDirectMax) {
                launch("small_direct", nv(0) * (sT + 8.0), S, -1, st, [&](const Profiler::Slot& ps) {
                    PLAUNCH(k_small_direct<T>, dim3(S), dim3(64), direct_lds_bytes<T>(cfg_.m, cfg_.bc), st, a);
                });
            } else {
                const size_t lds = small_lds_bytes<T>(cfg_.m);
                launch("small_pcg", nv(0) * (sT + 8.0), S, -1, st, [&](const Profiler::Slot& ps) {
                    PLAUNCH((k_small_pcg<T, small_threads(32), 32>), dim3(S), dim3(small_threads(32)), lds, st, a);
                });
            }
            done_ = true;
            return hipGetLastError();
        }
        Scal* scal = ptr<Scal>(o_scal_);
        int* cnt = ptr<int>(o_cnt_);
        double* part = ptr<double>(o_part_);
        // coefficient hierarchy
        for (int l = 0; l + 1 < nlev_; ++l) {
            const int ctx = (int)cdiv(lv_[l + 1].w, CCX), cty = (int)cdiv(lv_[l + 1].w, CCY);
            const int ctw = (int)cdiv(lv_[l + 1].w, ctx);
            const dim3 g = l == 0 ? dim3((unsigned)(ctx * cty * S))
                                  : dim3((unsigned)cdiv((long long)lv_[l + 1].w * lv_[l + 1].w, kBlock), S);
            launch("coarsen", (l == 0 ? nv(0) : 2.0 * nv(l)) * sT + 2.0 * nv(l + 1) * sT, S, -1, st, [&](const Profiler::Slot& ps) {
                if (l == 0)
                    PLAUNCH(k_coarsen_k<T>, g, dim3(kBlock), 0, st, k0_, kss, lv_[0], ptr<T>(o_ce_[0]),
                                       ptr<T>(o_cn_[0]), lv_[1], ctx, ctx * cty, ctw);
                else
                    PLAUNCH(k_coarsen_c<T>, g, dim3(kBlock), 0, st, ptr<T>(o_ce_[l - 1]),
                                       ptr<T>(o_cn_[l - 1]), lv_[l], ptr<T>(o_ce_[l]), ptr<T>(o_cn_[l]), lv_[l + 1]);
            });
        }
        hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, cnt, 0);
        PcgArgs<T> pa = pcg_args(0);
        pa.tiles_x = itx_;
        pa.ntiles = itiles_;
        if (lin_) pa.X = nullptr;   // the iterate is not kept
        // k for the flow cell's lifting; x (unless linear QoI) and r out
        const double ib = nv(0) * ((cfg_.bc == BC_FLOWCELL ? sT : 0.0) + (lin_ ? 8.0 : 16.0));
        launch("pcg_init", ib, S, -1, st, [&](const Profiler::Slot& ps) {
            PLAUNCH(k_pcg_init<T>, dim3(itiles_ * S), dim3(kBlock), 0, st, pa);
        });
        hipLaunchKernelGGL(k_reduce<RED_BB>, dim3(S), dim3(kBlock), 0, st, part, part, itiles_, scal,
                           cfg_.rtol * cfg_.rtol, cfg_.maxit, cnt);
        // launch profiler: samples active in each iteration, from the counts
        // read back for the convergence test (iteration 0: all S; a sample
        // with a zero right-hand side, converged from the start, is counted)
        hist_h_.assign(cfg_.maxit + 2, 0);
        hist_h_[0] = S;
        return hipGetLastError();
    }

    hipError_t advance(hipStream_t st, int depth, bool graphs, bool* done, bool* progressed) override {
        *progressed = false;
        depth = std::max(1, std::min(depth, RING));
        // confirm finished iterations in order: the active-sample count
        // after iteration i lands in hcnt_[i % RING]
        while (!done_ && confirmed_ < it_next_) {
            const hipError_t q = hipEventQuery(ev_[confirmed_ % RING]);
            if (q == hipErrorNotReady) {
                (void)hipGetLastError();
                break;
            }
            if (q != hipSuccess) return q;
            const int c = hcnt_[confirmed_ % RING];
            if (confirmed_ + 1 < (int)hist_h_.size()) hist_h_[confirmed_ + 1] = c;
            ++confirmed_;
            if (c == 0) done_ = true;
        }
        if (!done_ && confirmed_ == it_next_ && it_next_ >= cfg_.maxit) done_ = true;
        if (!done_ && it_next_ < cfg_.maxit && it_next_ - confirmed_ < depth) {
            hipError_t e;
            if (graphs && it_next_ >= 1 && !Profiler::get().on()) {
                hipGraphExec_t g = nullptr;
                e = iteration_graph(it_next_ & 1, &g);
                if (e == hipSuccess) e = hipGraphLaunch(g, st);
            } else {
                e = iteration(it_next_, st);
            }
            if (e != hipSuccess) return e;
            const int slot = it_next_ % RING;
            if ((e = hipMemcpyAsync(&hcnt_[slot], ptr<int>(o_cnt_), sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess)
                return e;
            if ((e = hipEventRecord(ev_[slot], st)) != hipSuccess) return e;
            ++it_next_;
            *progressed = true;
        }
        *done = done_;
        return hipSuccess;
    }

    hipError_t wait() override {
        if (done_ || confirmed_ >= it_next_) return hipSuccess;
        return hipEventSynchronize(ev_[confirmed_ % RING]);
    }

    hipError_t finish(hipStream_t) override {
        if (!Profiler::get().on() || small_ || recs_.empty()) return hipSuccess;
        // samples active in iteration it = count read back after iteration
        // it-1 (iterations enqueued past the last confirmed one ran with none)
        for (auto& r : recs_)
            if (r.second >= 0 && r.second < (int)hist_h_.size()) Profiler::get().set_samples(r.first, hist_h_[r.second]);
        return hipSuccess;
    }

    hipError_t qoi(const void* kv, long long kss, int S, double* q, int* iters, hipStream_t st) override {
        if (S <= 0) return hipSuccess;
        launch("qoi", lin_ ? 8.0 : nv(0) * 8.0, S, -1, st, [&](const Profiler::Slot& ps) {
            PLAUNCH(k_qoi<T>, dim3(S), dim3(kBlock), 0, st, ptr<double>(o_X_), lv_[0], cfg_.bc, cfg_.f,
                               cfg_.qoi, cfg_.qx, cfg_.qy, reinterpret_cast<const T*>(kv), kss, ptr<Scal>(o_scal_),
                               lin_ ? 1 : 0, q ? q : ptr<double>(o_q_), iters ? iters : ptr<int>(o_it_));
        });
        return hipGetLastError();
    }

private:
    template <typename U>
    U* ptr(size_t off) const { return reinterpret_cast<U*>(reinterpret_cast<char*>(base_) + off); }

    double nv(int l) const { return (double)lv_[l].w * lv_[l].w; }
    double nu(int l) const { return (double)(lv_[l].m - 1) * (lv_[l].yhi - lv_[l].ylo + 1); }

    // launch with an optional profiler record; it >= 0 ties the record's
    // sample count to the samples active in CG iteration it
    // f(ps) launches the kernel with PLAUNCH, which hands the slot's events
    // to the launch
    template <typename F>
    void launch(const char* name, double bytes_per_sample, int S, int it, hipStream_t st, F&& f) {
        Profiler& P = Profiler::get();
        const Profiler::Slot ps = P.begin(name);
        f(ps);
        if (ps.idx >= 0) {
            P.end(ps, name, bytes_per_sample, S);
            if (it >= 0) recs_.emplace_back(ps.idx, it);
        }
    }

    // one PCG iteration of the tiled path: z = V-cycle(r) and r.z;
    // p, q = A p and p.q; x, r and ||r||^2 with the convergence test
    hipError_t iteration(int it, hipStream_t st) {
        const int S = S_;
        Scal* scal = ptr<Scal>(o_scal_);
        int* cnt = ptr<int>(o_cnt_);
        double* part = ptr<double>(o_part_);
        double* part2 = ptr<double>(o_part2_);
        const double rtol2 = cfg_.rtol * cfg_.rtol;
        const double sT = sizeof(T);
        vcycle(it, st);
        hipLaunchKernelGGL(k_reduce<RED_RZ>, dim3(S), dim3(kBlock), 0, st, part, part, rz_parts_, scal, rtol2, cfg_.maxit, cnt);
        PcgArgs<T> a = pcg_args(it);
        launch("pcg_dir", nu(0) * (24.0 + sT) + nv(0) * sT, S, it, st, [&](const Profiler::Slot& ps) {
            PLAUNCH(k_pcg_dir<T>, dim3(ptiles_ * S), dim3(kBlock), 0, st, a, it == 0 ? 1 : 0);
        });
        hipLaunchKernelGGL(k_reduce<RED_PQ>, dim3(S), dim3(kBlock), 0, st, part, lin_ ? part2 : nullptr, ptiles_,
                           scal, rtol2, cfg_.maxit, cnt);
        launch("pcg_update", nu(0) * (lin_ ? 24.0 : 48.0), S, it, st, [&](const Profiler::Slot& ps) {
            if (lin_)
                PLAUNCH(k_pcg_update<false>, dim3(ublocks_, S), dim3(kBlock), 0, st, a.X, a.R, a.Pnew,
                                   a.Q, lv_[0].ss, ublocks_, part, scal);
            else
                PLAUNCH(k_pcg_update<true>, dim3(ublocks_, S), dim3(kBlock), 0, st, a.X, a.R, a.Pnew,
                                   a.Q, lv_[0].ss, ublocks_, part, scal);
        });
        hipLaunchKernelGGL(k_reduce<RED_RR>, dim3(S), dim3(kBlock), 0, st, part, part, ublocks_, scal, rtol2, cfg_.maxit, cnt);
        return hipGetLastError();
    }

    // Executable graph of one iteration (it >= 1) of a solve of S_ samples
    // with coefficients at k0_: the kernels of iteration(it, .) depend on it
    // only through its parity (which direction buffer is old).  Captured on
    // a private stream on first use; two batch sizes are kept (a plan's full
    // chunks and its last one).
    hipError_t iteration_graph(int parity, hipGraphExec_t* out) {
        ItGraph* G = nullptr;
        for (auto& g : graphs_)
            if (g.S == S_ && g.k == k0_ && g.lin == lin_) G = &g;
        if (!G) {
            G = &graphs_[graph_victim_];
            graph_victim_ ^= 1;
            for (auto& x : G->exec)
                if (x) (void)hipGraphExecDestroy(x);
            G->exec[0] = G->exec[1] = nullptr;
            G->S = S_;
            G->k = k0_;
            G->lin = lin_;
        }
        if (!G->exec[parity]) {
            hipError_t e = hipSuccess;
            if (!cap_stream_) e = hipStreamCreateWithFlags(&cap_stream_, hipStreamNonBlocking);
            if (e != hipSuccess) return e;
            if ((e = hipStreamBeginCapture(cap_stream_, hipStreamCaptureModeRelaxed)) != hipSuccess) return e;
            const hipError_t ei = iteration(parity == 0 ? 2 : 1, cap_stream_);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(cap_stream_, &g);
            if (ei != hipSuccess) e = ei;
            if (e == hipSuccess) e = hipGraphInstantiate(&G->exec[parity], g, nullptr, nullptr, 0);
            if (g) (void)hipGraphDestroy(g);
            if (e != hipSuccess) return e;
        }
        *out = G->exec[parity];
        return hipSuccess;
    }

    PcgArgs<T> pcg_args(int it) {
        PcgArgs<T> a{};
        a.L = lv_[0];
        a.bc = cfg_.bc;
        a.tiles_x = ptx_;
        a.ntiles = ptiles_;
        a.f = cfg_.f;
        a.h2 = 1.0 / ((double)cfg_.m * cfg_.m);
        a.k = k0_;
        a.kss = kss_;
        a.X = ptr<double>(o_X_);
        a.R = ptr<double>(o_R_);
        a.Pold = ptr<double>((it & 1) ? o_P1_ : o_P0_);
        a.Pnew = ptr<double>((it & 1) ? o_P0_ : o_P1_);
        a.Q = ptr<double>(o_Q_);
        a.Z = ptr<T>(o_Z_);
        a.part = ptr<double>(o_part_);
        a.part2 = ptr<double>(o_part2_);
        a.scal = ptr<Scal>(o_scal_);
        a.ql = qoi_lin();
        return a;
    }

    // weights of the linear QoI of this mesh (off when the solve keeps x)
    QoiLin qoi_lin() const {
        QoiLin q{};
        q.on = lin_ ? 1 : 0;
        q.kind = cfg_.qoi;
        q.pi = q.pj = -2;
        if (cfg_.qoi == Q_POINT) {
            // the triangle of the diagonal split that holds the point
            const int m = cfg_.m;
            const double h = 1.0 / m;
            const int i = std::min((int)std::floor(cfg_.qx / h), m - 1), j = std::min((int)std::floor(cfg_.qy / h), m - 1);
            const double sx = cfg_.qx / h - i, sy = cfg_.qy / h - j;
            q.pi = i;
            q.pj = j;
            if (sx >= sy) {
                q.w00 = 1 - sx;
                q.w10 = sx - sy;
                q.w11 = sy;
            } else {
                q.w00 = 1 - sy;
                q.w11 = sx;
                q.w01 = sy - sx;
            }
        }
        return q;
    }

    MgArgs<T> mg_args(int l, int tiles_x, int ntiles) {
        MgArgs<T> a{};
        a.L = lv_[l];
        a.C = lv_[l + 1];
        a.bc = cfg_.bc;
        a.tiles_x = tiles_x;
        a.ntiles = ntiles;
        a.k = k0_;
        a.kss = kss_;
        if (l > 0) {
            a.ce = ptr<T>(o_ce_[l - 1]);
            a.cn = ptr<T>(o_cn_[l - 1]);
        }
        a.rhs = l == 0 ? (const void*)ptr<double>(o_R_) : (const void*)ptr<T>(o_rhs_[l - 1]);
        a.za = l == 0 ? ptr<T>(o_za0_) : ptr<T>(o_za_[l - 1]);
        a.scal = ptr<Scal>(o_scal_);
        return a;
    }

    // a level whose unknowns fit one multigrid region (see k_mg's WHOLE)
    bool whole(int l) const {
        return cfg_.bc == BC_DIRICHLET0 && lv_[l].m - 1 <= 64 && lv_[l].m - 1 <= RYT;
    }
    // a level that fits one 128 x 128 region (float multigrid)
    bool whole128(int l) const {
        return sizeof(T) == 4 && cfg_.bc == BC_DIRICHLET0 && lv_[l].m - 1 > 64 && lv_[l].m - 1 <= 128;
    }

    // Level 1 is visited twice per cycle (a W-cycle at that level) when the
    // configuration asks for it and level 1 has coarser kernel levels or the
    // bottom below it: the second coarse correction costs a fraction of an
    // iteration and cuts the CG iterations (257^2, Matern nu = 1, lambda =
    // 0.1: 10 -> 8), a gain where launches carry many samples.  Both
    // corrections are the same symmetric operator, so the preconditioner
    // stays symmetric.  A tiled level 1 keeps its corrected z_pre in a
    // buffer of its own (tiles read their neighbours' z_pre).
    bool twice1() const { return cfg_.twice1 && lb_ >= 2; }
    bool twice1_tiled() const { return twice1() && !(whole(1) || whole128(1)); }

    void vcycle(int it, hipStream_t st) {
        const int S = S_;
        const double sT = sizeof(T);
        auto pre = [&](int l) {
            const Lvl& L = lv_[l];
            const bool w128 = whole128(l);
            const bool wh = whole(l) || w128;
            const int tx = wh ? 1 : cdiv(L.m - 1, PRE_TX), ty = wh ? 1 : cdiv(L.yhi - L.ylo + 1, PRE_TY);
            MgArgs<T> a = mg_args(l, tx, tx * ty);
            a.rhs_c = ptr<T>(o_rhs_[l]);
            // k, rhs in; z_pre and the coarse rhs out
            const double rb = l == 0 ? 8.0 : sT;
            const double coef = (l == 0 ? 1.0 : 2.0) * nv(l) * sT;   // k, or two conductance arrays
            launch(l == 0 ? "mg_pre_l0" : "mg_pre", coef + nu(l) * (rb + sT) + nu(l + 1) * sT, S, it, st, [&](const Profiler::Slot& ps) {
                const dim3 g(tx * ty * S), b(kBlock);
                if constexpr (sizeof(T) == 4) {
                    if (w128) {
                        if (l == 0) PLAUNCH((k_mg<T, SH, false, true, true, 128>), g, dim3(1024), 0, st, a);
                        else PLAUNCH((k_mg<T, SH, false, false, true, 128>), g, dim3(1024), 0, st, a);
                        return;
                    }
                }
                if (l == 0 && wh) PLAUNCH((k_mg<T, SH, false, true, true>), g, b, 0, st, a);
                else if (l == 0) PLAUNCH((k_mg<T, SH, false, true, false>), g, b, 0, st, a);
                else if (wh) PLAUNCH((k_mg<T, SH, false, false, true>), g, b, 0, st, a);
                else PLAUNCH((k_mg<T, SH, false, false, false>), g, b, 0, st, a);
            });
        };
        auto bottom = [&]() {
            BottomArgs<T> b{};
            b.nl = nlev_ - lb_;
            b.bc = cfg_.bc;
            b.m0 = lv_[lb_].m;
            for (int l = 0; l < b.nl; ++l) {
                b.ss[l] = lv_[lb_ + l].ss;
                b.ce[l] = ptr<T>(o_ce_[lb_ + l - 1]);
                b.cn[l] = ptr<T>(o_cn_[lb_ + l - 1]);
            }
            b.rhs = ptr<T>(o_rhs_[lb_ - 1]);
            b.zout = ptr<T>(o_zb_[lb_ - 1]);
            b.scal = ptr<Scal>(o_scal_);
            double kb = 0.0;
            for (int l = lb_; l < nlev_; ++l) kb += 2.0 * nv(l) * sT;
            launch("mg_bottom", kb + nu(lb_) * 2.0 * sT, S, it, st, [&](const Profiler::Slot& ps) {
                // few samples: more threads per sample shorten each phase;
                // many: more workgroups per CU hide the latency instead
                if (S >= 512)
                    PLAUNCH((k_bottom<T, MB, 256>), dim3(S), dim3(256), 0, st, b);
                else
                    PLAUNCH((k_bottom<T, MB, 1024>), dim3(S), dim3(1024), 0, st, b);
            });
        };
        auto post = [&](int l) {
            const Lvl& L = lv_[l];
            const bool w128 = whole128(l);
            const bool wh = whole(l) || w128;
            const int tx = wh ? 1 : cdiv(L.m - 1, POST_TX), ty = wh ? 1 : cdiv(L.yhi - L.ylo + 1, POST_TY);
            MgArgs<T> a = mg_args(l, tx, tx * ty);
            a.zc = ptr<T>(o_zb_[l]);
            a.zout = l == 0 ? ptr<T>(o_Z_) : ptr<T>(o_zb_[l - 1]);
            a.dot = ptr<double>(o_part_);
            if (l == 1 && twice1_tiled()) a.za = ptr<T>(o_zm_);
            // k, z_pre, rhs, coarse correction in; z out (level 0: r in double)
            const double post = l == 0 ? nv(0) * sT + nu(0) * (sT + 8.0 + sT) + nu(1) * sT
                                       : 2.0 * nv(l) * sT + nu(l) * 3.0 * sT + nu(l + 1) * sT;
            launch(l == 0 ? "mg_post_l0" : "mg_post", post, S, it, st, [&](const Profiler::Slot& ps) {
                const dim3 g(tx * ty * S), b(kBlock);
                if constexpr (sizeof(T) == 4) {
                    if (w128) {
                        if (l == 0) PLAUNCH((k_mg<T, SH, true, true, true, 128>), g, dim3(1024), 0, st, a);
                        else PLAUNCH((k_mg<T, SH, true, false, true, 128>), g, dim3(1024), 0, st, a);
                        return;
                    }
                }
                if (l == 0 && wh) PLAUNCH((k_mg<T, SH, true, true, true>), g, b, 0, st, a);
                else if (l == 0) PLAUNCH((k_mg<T, SH, true, true, false>), g, b, 0, st, a);
                else if (wh) PLAUNCH((k_mg<T, SH, true, false, true>), g, b, 0, st, a);
                else PLAUNCH((k_mg<T, SH, true, false, false>), g, b, 0, st, a);
            });
        };
        // between the two coarse corrections of level l: z = z_pre + P z_c
        // (in place on a whole level, else into its own buffer), coarse
        // rhs = R (rhs - A z)
        auto mid = [&](int l) {
            const Lvl& L = lv_[l];
            const bool w128 = whole128(l);
            const bool wh = whole(l) || w128;
            const int tx = wh ? 1 : cdiv(L.m - 1, POST_TX), ty = wh ? 1 : cdiv(L.yhi - L.ylo + 1, POST_TY);
            MgArgs<T> a = mg_args(l, tx, tx * ty);
            a.zc = ptr<T>(o_zb_[l]);
            a.rhs_c = ptr<T>(o_rhs_[l]);
            a.zout = wh ? a.za : ptr<T>(o_zm_);
            launch("mg_mid", 2.0 * nv(l) * sT + nu(l) * 3.0 * sT + 2.0 * nu(l + 1) * sT, S, it, st,
                   [&](const Profiler::Slot& ps) {
                if constexpr (sizeof(T) == 4) {
                    if (w128) {
                        PLAUNCH((k_mg<T, SH, true, false, true, 128, true>), dim3(S), dim3(1024), 0, st, a);
                        return;
                    }
                }
                if (wh) PLAUNCH((k_mg<T, SH, true, false, true, 64, true>), dim3(S), dim3(kBlock), 0, st, a);
                else PLAUNCH((k_mg<T, SH, true, false, false, 64, true>), dim3(tx * ty * S), dim3(kBlock), 0, st, a);
            });
        };
        const bool w1 = twice1();
        for (int l = 0; l < lb_; ++l) pre(l);
        bottom();
        for (int l = lb_ - 1; l >= 0; --l) {
            if (w1 && l == 1) {
                mid(1);
                for (int k = 2; k < lb_; ++k) pre(k);
                bottom();
                for (int k = lb_ - 1; k >= 2; --k) post(k);
            }
            post(l);
        }
    }

    std::vector<Lvl> lv_;
    int nlev_ = 0, lb_ = 0;
    bool small_ = false;
    int ptx_ = 0, pty_ = 0, ptiles_ = 0, itx_ = 0, ity_ = 0, itiles_ = 0, stx_ = 0, sty_ = 0;
    int rz_parts_ = 0, ublocks_ = 0, max_parts_ = 0;
    size_t o_X_ = 0, o_R_ = 0, o_P0_ = 0, o_P1_ = 0, o_Q_ = 0, o_Z_ = 0, o_za0_ = 0;
    std::vector<size_t> o_ce_, o_cn_, o_rhs_, o_za_, o_zb_;
    size_t o_part_ = 0, o_part2_ = 0, o_scal_ = 0, o_q_ = 0, o_it_ = 0, o_cnt_ = 0, o_zm_ = 0;
    std::vector<int> hist_h_;   // active samples per iteration (launch profiler)
    std::vector<std::pair<int, int>> recs_;
    size_t bytes_ = 0;
    DeviceAllocator* alloc_ = nullptr;
    void* base_ = nullptr;
    int* hcnt_ = nullptr;
    hipEvent_t ev_[RING] = {nullptr, nullptr, nullptr, nullptr};
    struct ItGraph {
        int S = -1;
        const T* k = nullptr;
        bool lin = false;
        hipGraphExec_t exec[2] = {nullptr, nullptr};
    };
    ItGraph graphs_[2];
    int graph_victim_ = 0;
    hipStream_t cap_stream_ = nullptr;
    // state of the solve in progress
    const T* k0_ = nullptr;
    bool lin_ = false;   // the solve accumulates a linear QoI instead of x
    long long kss_ = 0;
    int S_ = 0, it_next_ = 0, confirmed_ = 0;
    bool done_ = true;
};

}  // namespace

size_t solver_bytes(const SolverCfg& cfg, int capacity, bool is_double) {
    if (cfg.m < 4 || (cfg.m & (cfg.m - 1)) != 0) return 0;
    if (is_double) return SolverImpl<double>(cfg, capacity).bytes();
    return SolverImpl<float>(cfg, capacity).bytes();
}

std::unique_ptr<Solver> make_solver(const SolverCfg& cfg, int capacity, bool is_double, DeviceAllocator* alloc,
                                    hipStream_t st, std::string* err, bool zero) {
    if (cfg.m < 4 || (cfg.m & (cfg.m - 1)) != 0) {
        *err = "solver mesh must be a power of two >= 4";
        return nullptr;
    }
    if (is_double) {
        auto s = std::make_unique<SolverImpl<double>>(cfg, capacity);
        if (!s->alloc(alloc, st, err, zero)) return nullptr;
        return s;
    }
    auto s = std::make_unique<SolverImpl<float>>(cfg, capacity);
    if (!s->alloc(alloc, st, err, zero)) return nullptr;
    return s;
}

hipError_t launch_zero(void* dst, size_t bytes, hipStream_t st) {
    if (bytes == 0) return hipSuccess;
    // library buffers are 256-byte aligned: 16-byte stores, then at most
    // three words
    if (((uintptr_t)dst & 15) != 0 || (bytes & 3) != 0) return hipErrorInvalidValue;
    const size_t head = bytes / 16 * 16;
    const long long n16 = (long long)(head / 16);
    const int ntail = (int)((bytes - head) / 4);
    const unsigned blocks = (unsigned)std::max<long long>(1, std::min<long long>(cdiv(n16, kBlock), 4096));
    hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(kBlock), 0, st, reinterpret_cast<uint4*>(dst), n16,
                       reinterpret_cast<unsigned*>(static_cast<char*>(dst) + head), ntail);
    return hipGetLastError();
}

hipError_t launch_finalize(const double* qf, const double* qc, const int* itf, const int* itc, int slot0,
                           int nslots, long long out0, double* y, double* yf, double* yc, int* iters, int* status,
                           hipStream_t st) {
    if (nslots <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize, dim3(cdiv(nslots, kBlock)), dim3(kBlock), 0, st, qf, qc, itf, itc, slot0, nslots,
                       out0, y, yf, yc, iters, status);
    return hipGetLastError();
}

}  // namespace ces
