// Density-fitted assembly of the particle operand (paper Sec. 2.1, eq.
// eri_sym_decomp: (pq|rs) = sum_Q B^Q_pq B^Q_rs).  Instead of reading the
// o*v^3 block (vv|vo), the particle part of the packed rows
//   G[p][x][y][d] = (yd|xp) = sum_Q B^Q_yd B^Q_xp        (d < v)
// is formed on FP64 MFMA from the factors, laid out with Q fastest:
//   bvv[y][d][Q] = B^Q_yd   (v*v*naux),   bvo[x][p][Q] = B^Q_xp   (v*o*naux).
// As a product: rows m = x*o + p of bvo (M = v*o) against rows n = y*v + d
// of bvv (N = v^2), summed over Q (K = naux); element (m, n) goes to row
// G[p][x][y] at kappa = d in the precision's packed format (pack.hip).
//
// Tiles of 128 x 128 per workgroup, 2 x 2 waves of 64 x 64, fragments loaded
// straight from global memory (the FP64 product is matrix-bound: 16 flops
// per byte loaded per tile).  Workgroups walk groups of DF_GM row tiles down
// each column tile, so that a column tile of bvv is fetched once per group.
#include "common.hpp"
#include "pack_out.hpp"

namespace ccsdt {

typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int DF_GM = 16;

// 16-element chunk c of row `row` (length K) for lane group g: k = 16c + 4g + t.
template <bool VEC>
__device__ __forceinline__ f64x4 df_load(const GLOBAL double* row, int c, int g, int K) {
    const int k0 = c * 16 + 4 * g;
    if (VEC && k0 + 4 <= K) return *reinterpret_cast<const GLOBAL f64x4*>(row + k0);
    f64x4 x;
#pragma unroll
    for (int t = 0; t < 4; ++t) x[t] = (k0 + t < K) ? row[k0 + t] : 0.0;
    return x;
}

template <class O, bool VEC>
__global__ __launch_bounds__(256) void assemble_g_df(const double* __restrict__ bvv, const double* __restrict__ bvo,
                                                     int o, int v, int naux, int Kp, typename O::T* __restrict__ g,
                                                     int tiles_m, int tiles_n) {
    const int64_t M = (int64_t)v * o, N = (int64_t)v * v;
    // grouped order: DF_GM row tiles per column tile, then the next column tile
    const int64_t bid = blockIdx.x;
    const int64_t per_group = (int64_t)DF_GM * tiles_n;
    const int grp = (int)(bid / per_group);
    const int first_m = grp * DF_GM;
    const int gm = min(DF_GM, tiles_m - first_m);
    const int64_t in_grp = bid - grp * per_group;
    const int tm = first_m + (int)(in_grp % gm);
    const int tn = (int)(in_grp / gm);

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t m0 = (int64_t)tm * 128 + (wave >> 1) * 64;
    const int64_t n0 = (int64_t)tn * 128 + (wave & 1) * 64;
    if (m0 >= M || n0 >= N) return;  // no barrier in this kernel
    const int gq = lane >> 4;

    const GLOBAL double* pa[4];
    const GLOBAL double* pb[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int64_t m = min(m0 + a * 16 + (lane & 15), M - 1);
        pa[a] = gp(bvo) + m * naux;
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int64_t n = min(n0 + b * 16 + (lane & 15), N - 1);
        pb[b] = gp(bvv) + n * naux;
    }
    f64x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};

    const int nch = (naux + 15) / 16;
    f64x4 fa[4], fb[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) fa[a] = df_load<VEC>(pa[a], 0, gq, naux);
#pragma unroll
    for (int b = 0; b < 4; ++b) fb[b] = df_load<VEC>(pb[b], 0, gq, naux);
    for (int c = 0; c < nch; ++c) {
        f64x4 na[4], nb[4];
        const int cn = min(c + 1, nch - 1);
#pragma unroll
        for (int a = 0; a < 4; ++a) na[a] = df_load<VEC>(pa[a], cn, gq, naux);
#pragma unroll
        for (int b = 0; b < 4; ++b) nb[b] = df_load<VEC>(pb[b], cn, gq, naux);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a][t], fb[b][t], acc[a][b], 0, 0, 0);
            }
#pragma unroll
        for (int a = 0; a < 4; ++a) fa[a] = na[a];
#pragma unroll
        for (int b = 0; b < 4; ++b) fb[b] = nb[b];
    }

    // FP64 MFMA output: lane holds rows (lane >> 4) + 4 r of column lane & 15
    const int64_t rl = O::rowlen(Kp);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int64_t n = n0 + b * 16 + (lane & 15);
        if (n >= N) continue;
        const int y = (int)(n / v), d = (int)(n % v);
#pragma unroll
        for (int a = 0; a < 4; ++a) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t m = m0 + a * 16 + (lane >> 4) + 4 * r;
                if (m < M) {
                    const int x = (int)(m / o), p = (int)(m % o);
                    O::put(g + (((int64_t)p * v + x) * v + y) * rl, d, acc[a][b][r]);
                }
            }
        }
    }
}

template <class O>
static hipError_t assemble_impl(int o, int v, int naux, int Kp, const double* bvv, const double* bvo, void* gc,
                                hipStream_t s) {
    const int64_t M = (int64_t)v * o, N = (int64_t)v * v;
    const int tiles_m = (int)((M + 127) / 128), tiles_n = (int)((N + 127) / 128);
    const int64_t total = (int64_t)tiles_m * tiles_n;
    auto* g = static_cast<typename O::T*>(gc);
    if (naux % 4 == 0)
        hipLaunchKernelGGL((assemble_g_df<O, true>), dim3((unsigned)total), dim3(256), 0, s, bvv, bvo, o, v, naux, Kp,
                           g, tiles_m, tiles_n);
    else
        hipLaunchKernelGGL((assemble_g_df<O, false>), dim3((unsigned)total), dim3(256), 0, s, bvv, bvo, o, v, naux, Kp,
                           g, tiles_m, tiles_n);
    return hipGetLastError();
}

hipError_t launch_assemble_df(int prec, int o, int v, int naux, int Kp, const double* bvv, const double* bvo,
                              void* gc, hipStream_t s) {
    switch (prec) {
        case P_FP64: return assemble_impl<OutF64>(o, v, naux, Kp, bvv, bvo, gc, s);
        case P_FP32: return assemble_impl<OutF32>(o, v, naux, Kp, bvv, bvo, gc, s);
        case P_BF16X3: return assemble_impl<OutB3>(o, v, naux, Kp, bvv, bvo, gc, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ccsdt
