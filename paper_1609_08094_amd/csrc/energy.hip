// Denominator-weighted (T) energy of each occupied triple from W, in FP64
// (paper Sec. 2.2: eqs. piecuch_4th_and_5th_order, piecuch_z_coefficients,
// piecuch_tilde_quantity; energy assembly in double precision as in Sec. 4).
//
// For a restricted triple i<=j<=k with multiplicity m (6 or 3):
//   e = m/3 sum_abc W_abc [4V_abc + V_bca + V_cab - 2V_acb - 2V_bac - 2V_cba] / D_abc
// with V = W + Z.  D is symmetric in (a,b,c), so the sum splits into orbits
// of the virtual triple under S3.  Label the orbit's values
//   q: 0=(a,b,c) 1=(a,c,b) 2=(b,a,c) 3=(b,c,a) 4=(c,a,b) 5=(c,b,a);
// the even permutations {0,3,4} and the odd ones {1,2,5}.  The bracket at an
// even point q is 3V_q + Se - 2So, at an odd point 3V_q + So - 2Se
// (Se, So: sums of V over even / odd points), hence the orbit contributes
//   f = 3 sum_q W_q V_q + We (Se - 2 So) + Wo (So - 2 Se)
// divided by D and by the number of times each distinct point is repeated
// (s = 2 when exactly two of a,b,c are equal; a=b=c contributes exactly 0).
// E[4] takes V = W, E[5] takes V = Z; E = E[4] + E[5].
//
// One workgroup handles one block orbit (A <= B <= C) of EB^3 virtual
// blocks and visits each representative a <= b <= c once.  Per-workgroup
// partials go to fixed slots; sums run in a fixed order (deterministic).
#include "common.hpp"

namespace ccsdt {

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    return x;
}

// Sum x over the 256 threads of the block; valid in thread 0.
__device__ __forceinline__ double block_sum(double x, double* sh) {
    x = wave_sum(x);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wave] = x;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    return r;
}

__device__ __forceinline__ void decode_orbit(int q, int& A, int& B, int& C) {
    // orbits are enumerated C-major: all (A<=B<=C) with C fixed are contiguous
    int c = 0;
    while ((int64_t)(c + 1) * (c + 2) * (c + 3) / 6 <= q) ++c;
    int r = q - c * (c + 1) * (c + 2) / 6;
    int b = 0;
    while ((b + 1) * (b + 2) / 2 <= r) ++b;
    A = r - b * (b + 1) / 2;
    B = b;
    C = c;
}

template <class WT>
__global__ __launch_bounds__(256) void energy_kernel(const Slot* __restrict__ slots, int nslot,
                                                     double* __restrict__ partials) {
    __shared__ double sh[4];
    const int bid = blockIdx.x;
    int lo = 0, hi = nslot - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (slots[mid].e_begin <= bid) lo = mid; else hi = mid - 1;
    }
    const Slot* S = slots + lo;
    const int q = bid - S->e_begin;
    int A, B, C;
    decode_orbit(q, A, B, C);
    const int v = S->v, o = S->o, i = S->i, j = S->j, k = S->k;
    const WT* W = static_cast<const WT*>(S->w);
    const double* ev = S->eps_v;
    const double eo = S->eps_o[i] + S->eps_o[j] + S->eps_o[k];
    const double* t1i = S->t1 + (int64_t)i * v;
    const double* t1j = S->t1 + (int64_t)j * v;
    const double* t1k = S->t1 + (int64_t)k * v;
    // (pX|qY) = ovov[p][X][q][Y]; rows of the three slices used by Z
    const double* ov = S->ovov;
    const int64_t rs = (int64_t)o * v;  // stride of X in ovov[p][X][q][:]
    const double* Sjk = ov + ((int64_t)j * v * o + k) * v;  // Sjk[y*rs + z] = (jy|kz)
    const double* Sik = ov + ((int64_t)i * v * o + k) * v;
    const double* Sij = ov + ((int64_t)i * v * o + j) * v;
    const double scale = (double)S->mult / 3.0;
    const int64_t V = v;

    const int c = C * EB + (threadIdx.x & 15);
    const int b = B * EB + (threadIdx.x >> 4);
    double e4 = 0.0, e5 = 0.0;
    if (c < v && b <= c) {
        const double evbc = ev[b] + ev[c];
        for (int aa = 0; aa < EB; ++aa) {
            const int a = A * EB + aa;
            if (a > b) break;
            if (a == c) continue;  // a = b = c
            const double w0 = (double)W[(a * V + b) * V + c];
            const double w1 = (double)W[(a * V + c) * V + b];
            const double w2 = (double)W[(b * V + a) * V + c];
            const double w3 = (double)W[(b * V + c) * V + a];
            const double w4 = (double)W[(c * V + a) * V + b];
            const double w5 = (double)W[(c * V + b) * V + a];
            // Z(x,y,z) = t1[i][x] (jy|kz) + t1[j][y] (ix|kz) + t1[k][z] (ix|jy)
            auto Z = [&](int x, int y, int z) {
                return t1i[x] * Sjk[y * rs + z] + t1j[y] * Sik[x * rs + z] + t1k[z] * Sij[x * rs + y];
            };
            const double z0 = Z(a, b, c), z1 = Z(a, c, b), z2 = Z(b, a, c);
            const double z3 = Z(b, c, a), z4 = Z(c, a, b), z5 = Z(c, b, a);
            const double We = w0 + w3 + w4, Wo = w1 + w2 + w5;
            const double Ze = z0 + z3 + z4, Zo = z1 + z2 + z5;
            const double sww = w0 * w0 + w1 * w1 + w2 * w2 + w3 * w3 + w4 * w4 + w5 * w5;
            const double swz = w0 * z0 + w1 * z1 + w2 * z2 + w3 * z3 + w4 * z4 + w5 * z5;
            const double f4 = 3.0 * sww + We * (We - 2.0 * Wo) + Wo * (Wo - 2.0 * We);
            const double f5 = 3.0 * swz + We * (Ze - 2.0 * Zo) + Wo * (Zo - 2.0 * Ze);
            const double D = eo - ev[a] - evbc;
            const double rep = (a == b || b == c) ? 2.0 : 1.0;
            const double sc = scale / (rep * D);
            e4 += f4 * sc;
            e5 += f5 * sc;
        }
    }
    const double s4 = block_sum(e4, sh);
    const double s5 = block_sum(e5, sh);
    if (threadIdx.x == 0) {
        partials[2 * (S->part_begin + q)] = s4;
        partials[2 * (S->part_begin + q) + 1] = s5;
    }
}

__global__ __launch_bounds__(256) void slot_reduce_kernel(const Slot* __restrict__ slots,
                                                          const double* __restrict__ partials,
                                                          double* __restrict__ e_trip) {
    __shared__ double sh[4];
    const Slot* S = slots + blockIdx.x;
    const int nb = S->nblk;
    const int norb = nb * (nb + 1) * (nb + 2) / 6;
    double e4 = 0.0, e5 = 0.0;
    for (int q = threadIdx.x; q < norb; q += 256) {
        e4 += partials[2 * (S->part_begin + q)];
        e5 += partials[2 * (S->part_begin + q) + 1];
    }
    const double s4 = block_sum(e4, sh);
    const double s5 = block_sum(e5, sh);
    if (threadIdx.x == 0) {
        e_trip[3 * S->trip_index] = s4 + s5;
        e_trip[3 * S->trip_index + 1] = s4;
        e_trip[3 * S->trip_index + 2] = s5;
    }
}

__global__ __launch_bounds__(256) void final_reduce_kernel(const int* __restrict__ trip_begin,
                                                           const double* __restrict__ e_trip,
                                                           double* __restrict__ out) {
    __shared__ double sh[4];
    const int p = blockIdx.x;
    const int t0 = trip_begin[p], t1 = trip_begin[p + 1];
    double e4 = 0.0, e5 = 0.0;
    for (int t = t0 + (int)threadIdx.x; t < t1; t += 256) {
        e4 += e_trip[3 * t + 1];
        e5 += e_trip[3 * t + 2];
    }
    const double s4 = block_sum(e4, sh);
    const double s5 = block_sum(e5, sh);
    if (threadIdx.x == 0) {
        out[3 * p] = s4 + s5;
        out[3 * p + 1] = s4;
        out[3 * p + 2] = s5;
    }
}

template <class WT>
__global__ void widen_kernel(const WT* __restrict__ w, int64_t n, double* __restrict__ out) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        out[e] = (double)w[e];
}

hipError_t launch_energy(int prec, const Slot* d_slots, int nslot, int total, double* partials, hipStream_t s) {
    if (total <= 0) return hipSuccess;
    if (prec == P_FP64)
        hipLaunchKernelGGL(energy_kernel<double>, dim3(total), dim3(256), 0, s, d_slots, nslot, partials);
    else
        hipLaunchKernelGGL(energy_kernel<float>, dim3(total), dim3(256), 0, s, d_slots, nslot, partials);
    return hipGetLastError();
}

hipError_t launch_slot_reduce(const Slot* d_slots, int nslot, int, const double* partials, double* e_trip,
                              hipStream_t s) {
    if (nslot <= 0) return hipSuccess;
    hipLaunchKernelGGL(slot_reduce_kernel, dim3(nslot), dim3(256), 0, s, d_slots, partials, e_trip);
    return hipGetLastError();
}

hipError_t launch_final_reduce(const int* d_trip_begin, int nprob, const double* e_trip, double* out,
                               hipStream_t s) {
    hipLaunchKernelGGL(final_reduce_kernel, dim3(nprob), dim3(256), 0, s, d_trip_begin, e_trip, out);
    return hipGetLastError();
}

hipError_t launch_widen_w(int prec, const void* w, int64_t n, double* out, hipStream_t s) {
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 65536);
    if (prec == P_FP64)
        hipLaunchKernelGGL(widen_kernel<double>, dim3(grid), dim3(256), 0, s, static_cast<const double*>(w), n, out);
    else
        hipLaunchKernelGGL(widen_kernel<float>, dim3(grid), dim3(256), 0, s, static_cast<const float*>(w), n, out);
    return hipGetLastError();
}

}  // namespace ccsdt
