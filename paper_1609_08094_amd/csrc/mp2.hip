// Closed-shell RI-MP2 correlation energy on gfx950 MFMA (paper Sec. 2.1:
// eq. mp2_energy with the denominators of eq. e_orb_diff and the integrals of
// eq. eri_sym_decomp):
//   E = - sum_ij sum_ab g_aibj (2 g_aibj - g_ajbi) / (e_a + e_b - e_i - e_j),
//   g_aibj = sum_Q C^Q_ai C^Q_bj.
// For an ordered pair (i, j) let G_ij[a][b] = g_aibj = <C_i[a], C_j[b]> (rows
// of the fitting coefficients, Q fastest); then g_ajbi = G_ij[b][a], and the
// pair energy e_ij = - sum_ab G(2G - G^T)/D is symmetric in (i, j).  The
// library forms G_ij for i <= j (one batched NT product per chunk of pairs on
// MFMA: FP64, FP32, or the BF16 split with all four hi/lo products, since the
// diagonal g_aiai are sums of squares, the three correction products in an
// accumulator of their own) into a pair buffer; then an FP64
// energy kernel reads each 64 x 64 block of G_ij together with its transposed
// partner, and E = sum_i e_ii + 2 sum_{i<j} e_ij is summed in a fixed order.
#include "common.hpp"
#include "mfma.hpp"
#include "pack_out.hpp"

namespace ccsdt {

// Coefficient rows c_ov[i][a][:] (length naux) into packed rows of Kq.
template <class O>
__global__ __launch_bounds__(256) void mp2_pack_rows(const double* __restrict__ src, int64_t nrows, int K,
                                                     int Kq, typename O::T* __restrict__ dst) {
    const GLOBAL double* s = gp(src);
    for (int64_t row = blockIdx.x; row < nrows; row += gridDim.x) {
        typename O::T* out = dst + row * O::rowlen(Kq);
        for (int k = threadIdx.x; k < Kq; k += 256) O::put(out, k, k < K ? s[row * K + k] : 0.0);
    }
}

// G_ij tiles: workgroup (pair slot, 128 x 128 tile of (a, b)), 2 x 2 waves of
// 64 x 64, operand rows staged through two LDS stages written straight from
// global memory, in the chunk order and swizzle of the (T) contraction.
template <class P>
__global__ __launch_bounds__(256, 2) void mp2_gemm_kernel(const void* __restrict__ cpk, const int2* __restrict__ pairs,
                                                          int v, int Kq, int tiles, int total,
                                                          typename P::W* __restrict__ gbuf) {
    using Wt = typename P::W;
    constexpr int WTM = 64, WTN = 64, BM = 128, BN = 128, RS = 128;
    constexpr int ROWS = BM + BN, TPR = RS / 16, RPP = 256 / TPR, NP = ROWS / RPP;
    constexpr int MB = WTM / 16, NB = WTN / 16;
    __shared__ __attribute__((aligned(16))) char lds[2 * ROWS * RS];

    const int bid = xcd_remap(blockIdx.x, total);
    const int slot = bid / (tiles * tiles);
    const int t = bid - slot * tiles * tiles;
    const int tm = t / tiles, tn = t - tm * tiles;
    const int2 pr = pairs[slot];
    const int mt0 = tm * BM, nt0 = tn * BN;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wm = wave >> 1, wn = wave & 1;
    const int m0 = mt0 + wm * WTM, n0 = nt0 + wn * WTN;
    const int vm = max(0, min(MB, (v - m0 + 15) / 16));
    const int vn = max(0, min(NB, (v - n0 + 15) / 16));

    const int64_t rowbytes = (int64_t)Kq * P::UNITS * sizeof(typename P::E);
    const int nsteps = (int)(rowbytes / RS);
    const char* C = static_cast<const char*>(cpk);
    const int lrow = threadIdx.x / TPR;
    const int pch = (lane & 7) ^ lds_swz(lrow);
    const int src_col = (P::SPLIT ? (((pch & 3) << 1) | (pch >> 2)) : pch) * 16;
    const int wave_row0 = wave * (64 / TPR);
    const char* rbase[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int r = lrow + p * RPP;
        const int64_t row = r < BM ? (int64_t)pr.x * v + min(mt0 + r, v - 1) : (int64_t)pr.y * v + min(nt0 + r - BM, v - 1);
        rbase[p] = C + row * rowbytes + src_col;
    }
    typename P::Acc acc[MB][NB];
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = typename P::Acc{};

#define MP2_GLOAD(c, buf)                                                                      \
    _Pragma("unroll") for (int p = 0; p < NP; ++p) {                                           \
        char* dst = lds + (buf) * (ROWS * RS) + (wave_row0 + p * RPP) * RS;                    \
        __builtin_amdgcn_global_load_lds((const GLOBAL void*)gp(rbase[p] + (int64_t)(c) * RS), \
                                         (__attribute__((address_space(3))) void*)dst, 16, 0, 0); \
    }
    MP2_GLOAD(0, 0);
    lds_dma_barrier();
    const bool active = vm > 0 && vn > 0;
    for (int step = 0; step < nsteps; ++step) {
        const int buf = step & 1;
        // the last step re-requests its own chunk into the idle buffer
        MP2_GLOAD(min(step + 1, nsteps - 1), buf ^ 1);
        __builtin_amdgcn_sched_barrier(0);
        if (active) {
            const char* As = lds + buf * (ROWS * RS) + (wm * WTM + (lane & 15)) * RS;
            const char* Bs = lds + buf * (ROWS * RS) + (BM + wn * WTN + (lane & 15)) * RS;
            const int g = lane >> 4;
            const int sw = lds_swz(lane & 15);
            if (vm == MB && vn == NB)
                lds_stage<P, MB, NB, RS, true>(acc, As, Bs, g, sw, vm, vn);
            else
                lds_stage<P, MB, NB, RS, false>(acc, As, Bs, g, sw, vm, vn);
        }
        lds_dma_barrier();
    }
#undef MP2_GLOAD
    if (!active) return;
    GLOBAL Wt* out = gpw(gbuf) + (int64_t)slot * v * v;
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if (a >= vm || b >= vn) continue;
            const int n = n0 + b * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + a * 16 + P::out_row(lane, r);
                if (m < v && n < v) out[(int64_t)m * v + n] = (Wt)acc[a][b][r];
            }
        }
}

// Energy of one pair slot over one pair of 64 x 64 blocks (A <= B) of G_ij:
// the block (A, B) and its transposed partner (B, A), staged through LDS.
// Each unordered (a, b) in distinct blocks contributes
//   [G_ab (2 G_ab - G_ba) + G_ba (2 G_ba - G_ab)] / D_ab,
// a diagonal block every ordered (a, b) once.  partial = - (sum), FP64.
template <class WT>
__global__ __launch_bounds__(256) void mp2_energy_kernel(const WT* __restrict__ gbuf, const int2* __restrict__ pairs,
                                                         const double* __restrict__ eps_o,
                                                         const double* __restrict__ eps_v, int v, int tiles,
                                                         double* __restrict__ partials) {
    __shared__ double sab[64][65], sba[64][65];
    __shared__ double sh[4];
    __shared__ double ea[64], eb[64];
    const int npt = tiles * (tiles + 1) / 2;
    const int slot = blockIdx.x / npt;
    int q = blockIdx.x - slot * npt;
    // q -> (A, B), A <= B, row-major over the upper triangle
    int A = 0;
    while (q >= tiles - A) {
        q -= tiles - A;
        ++A;
    }
    const int B = A + q;
    const int2 pr = pairs[slot];
    const double eij = eps_o[pr.x] + eps_o[pr.y];
    const GLOBAL WT* G = gp(gbuf) + (int64_t)slot * v * v;
    const int a0 = A * 64, b0 = B * 64;
    if (threadIdx.x < 64) {
        const int a = a0 + threadIdx.x, b = b0 + threadIdx.x;
        ea[threadIdx.x] = a < v ? eps_v[a] : 0.0;
        eb[threadIdx.x] = b < v ? eps_v[b] : 0.0;
    }
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int r = e >> 6, c = e & 63;
        const bool ok1 = a0 + r < v && b0 + c < v, ok2 = b0 + r < v && a0 + c < v;
        sab[r][c] = ok1 ? (double)G[(int64_t)(a0 + r) * v + b0 + c] : 0.0;
        sba[r][c] = ok2 ? (double)G[(int64_t)(b0 + r) * v + a0 + c] : 0.0;
    }
    __syncthreads();
    double acc = 0.0;
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int r = e >> 6, c = e & 63;
        const int a = a0 + r, b = b0 + c;
        if (a >= v || b >= v) continue;
        const double g = sab[r][c];
        const double d = ea[r] + eb[c] - eij;
        if (A == B) {
            acc += g * (2.0 * g - sab[c][r]) / d;
        } else {
            const double gx = sba[c][r];
            acc += (g * (2.0 * g - gx) + gx * (2.0 * gx - g)) / d;
        }
    }
    // block sum in a fixed order
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = -(sh[0] + sh[1] + sh[2] + sh[3]);
}

// e_pair[pair_index[s]] = sum of slot s's partials (fixed order).
__global__ __launch_bounds__(256) void mp2_pair_reduce(const double* __restrict__ partials, int npt,
                                                       const int* __restrict__ pair_index,
                                                       double* __restrict__ e_pair) {
    __shared__ double sh[4];
    const int s = blockIdx.x;
    double acc = 0.0;
    for (int q = threadIdx.x; q < npt; q += 256) acc += partials[(int64_t)s * npt + q];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) e_pair[pair_index[s]] = sh[0] + sh[1] + sh[2] + sh[3];
}

// out[0] = sum_p w_p e_pair[p] with w = 1 for i = j and 2 otherwise.
__global__ __launch_bounds__(256) void mp2_final_reduce(const double* __restrict__ e_pair,
                                                        const int2* __restrict__ all_pairs, int npairs,
                                                        double* __restrict__ out) {
    __shared__ double sh[4];
    double acc = 0.0;
    for (int p = threadIdx.x; p < npairs; p += 256) {
        const int2 pr = all_pairs[p];
        acc += (pr.x == pr.y ? 1.0 : 2.0) * e_pair[p];
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = sh[0] + sh[1] + sh[2] + sh[3];
}

hipError_t launch_mp2_pack(int prec, int o, int v, int naux, int Kq, const double* c_ov, void* cpk, hipStream_t s) {
    const int64_t rows = (int64_t)o * v;
    const dim3 grid((unsigned)std::min<int64_t>(rows, (int64_t)1 << 20));
    switch (prec) {
        case P_FP64:
            hipLaunchKernelGGL(mp2_pack_rows<OutF64>, grid, dim3(256), 0, s, c_ov, rows, naux, Kq,
                               static_cast<double*>(cpk));
            break;
        case P_FP32:
            hipLaunchKernelGGL(mp2_pack_rows<OutF32>, grid, dim3(256), 0, s, c_ov, rows, naux, Kq,
                               static_cast<float*>(cpk));
            break;
        case P_BF16X3:
            hipLaunchKernelGGL(mp2_pack_rows<OutB3>, grid, dim3(256), 0, s, c_ov, rows, naux, Kq,
                               static_cast<uint16_t*>(cpk));
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_mp2_gemm(int prec, const void* cpk, const int2* d_pairs, int nslot, int v, int Kq, void* gbuf,
                           hipStream_t s) {
    const int tiles = (v + 127) / 128;
    const int total = nslot * tiles * tiles;
    if (total <= 0) return hipSuccess;
    switch (prec) {
        case P_FP64:
            hipLaunchKernelGGL(mp2_gemm_kernel<PrecF64>, dim3(total), dim3(256), 0, s, cpk, d_pairs, v, Kq, tiles,
                               total, static_cast<double*>(gbuf));
            break;
        case P_FP32:
            hipLaunchKernelGGL(mp2_gemm_kernel<PrecF32>, dim3(total), dim3(256), 0, s, cpk, d_pairs, v, Kq, tiles,
                               total, static_cast<float*>(gbuf));
            break;
        case P_BF16X3:  // lo*lo kept: see PrecB4
            hipLaunchKernelGGL(mp2_gemm_kernel<PrecB4>, dim3(total), dim3(256), 0, s, cpk, d_pairs, v, Kq, tiles,
                               total, static_cast<float*>(gbuf));
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_mp2_energy(int prec, const void* gbuf, const int2* d_pairs, int nslot, const double* eps_o,
                             const double* eps_v, int v, double* partials, const int* d_pair_index, double* e_pair,
                             hipStream_t s) {
    const int tiles = (v + 63) / 64;
    const int npt = tiles * (tiles + 1) / 2;
    if (nslot <= 0) return hipSuccess;
    if (prec == P_FP64)
        hipLaunchKernelGGL(mp2_energy_kernel<double>, dim3(nslot * npt), dim3(256), 0, s,
                           static_cast<const double*>(gbuf), d_pairs, eps_o, eps_v, v, tiles, partials);
    else
        hipLaunchKernelGGL(mp2_energy_kernel<float>, dim3(nslot * npt), dim3(256), 0, s,
                           static_cast<const float*>(gbuf), d_pairs, eps_o, eps_v, v, tiles, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mp2_pair_reduce, dim3(nslot), dim3(256), 0, s, partials, npt, d_pair_index, e_pair);
    return hipGetLastError();
}

hipError_t launch_mp2_final(const double* e_pair, const int2* d_all_pairs, int npairs, double* out, hipStream_t s) {
    hipLaunchKernelGGL(mp2_final_reduce, dim3(1), dim3(256), 0, s, e_pair, d_all_pairs, npairs, out);
    return hipGetLastError();
}

}  // namespace ccsdt
