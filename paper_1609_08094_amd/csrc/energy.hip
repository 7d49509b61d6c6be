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
// One workgroup (two waves) handles one orbit (A <= B <= C) of WB^3 blocks
// of W.  The waves take turns over the SB^3 sub-block orbits (x <= y <= z)
// inside it.  For each, a wave first issues every load it needs at once --
// the six permuted sub-blocks W[x][y][z], W[x][z][y], ..., W[z][y][x]
// (each one contiguous SB^3 run of the blocked layout, read with 16-byte
// loads that cover it in lane order; W = W_A + W_B summed on the way, or,
// for a triple taken as (p, p, q), W_A added again at the exchanged
// positions), the 18 SB x SB sub-blocks of the
// ovov slices (jX|kY), (iX|kY), (iX|jY) over ordered pairs of {x,y,z}, and
// the t1 / eps_v segments -- parks them in padded LDS, and then evaluates the
// representatives a <= b <= c of its (b, c) column from LDS alone.
// Per-workgroup partials go to fixed slots; sums run in a fixed order
// (deterministic).
#include "common.hpp"

namespace ccsdt {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int EW = 2;  // waves per energy workgroup

// W = W_A + W_B for one 16-byte pair of global loads, scattered into padded
// (unaligned) LDS elements.  The sum is one rounding in the W precision.
template <class WT> struct Unpack;
template <> struct Unpack<float> {
    static __device__ __forceinline__ void put2(float* d, u32x4 x, u32x4 y) {
        d[0] = __uint_as_float(x.x) + __uint_as_float(y.x);
        d[1] = __uint_as_float(x.y) + __uint_as_float(y.y);
        d[2] = __uint_as_float(x.z) + __uint_as_float(y.z);
        d[3] = __uint_as_float(x.w) + __uint_as_float(y.w);
    }
    static __device__ __forceinline__ void put1(float* d, u32x4 x) {
        d[0] = __uint_as_float(x.x);
        d[1] = __uint_as_float(x.y);
        d[2] = __uint_as_float(x.z);
        d[3] = __uint_as_float(x.w);
    }
    static __device__ __forceinline__ void add1(float* d, u32x4 y) {
        d[0] += __uint_as_float(y.x);
        d[1] += __uint_as_float(y.y);
        d[2] += __uint_as_float(y.z);
        d[3] += __uint_as_float(y.w);
    }
};
template <> struct Unpack<double> {
    static __device__ __forceinline__ void put2(double* d, u32x4 x, u32x4 y) {
        d[0] = __hiloint2double((int)x.y, (int)x.x) + __hiloint2double((int)y.y, (int)y.x);
        d[1] = __hiloint2double((int)x.w, (int)x.z) + __hiloint2double((int)y.w, (int)y.z);
    }
    static __device__ __forceinline__ void put1(double* d, u32x4 x) {
        d[0] = __hiloint2double((int)x.y, (int)x.x);
        d[1] = __hiloint2double((int)x.w, (int)x.z);
    }
    static __device__ __forceinline__ void add1(double* d, u32x4 y) {
        d[0] += __hiloint2double((int)y.y, (int)y.x);
        d[1] += __hiloint2double((int)y.w, (int)y.z);
    }
};

// Each wave of the energy kernel stages into its own LDS region, and the LDS
// operations of one wave complete in issue order, so the staging loop needs
// no workgroup barrier (which would make the two waves alternate loading and
// computing in lockstep); the fence only keeps the compiler from moving LDS
// accesses across the stage boundary.
__device__ __forceinline__ void wave_lds_fence() { asm volatile("" ::: "memory"); }

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    return x;
}

// Sum x over the EW*64 threads of the block; valid in thread 0.
__device__ __forceinline__ double block_sum(double x, double* sh) {
    x = wave_sum(x);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wave] = x;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += sh[w];
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
__global__ __launch_bounds__(EW * 64) void energy_kernel(const Slot* __restrict__ slots, int nslot,
                                                         double* __restrict__ partials) {
    // W sub-block in LDS: element (u, w, t) at u*PS + w*RS + t.  The six
    // permuted reads of the evaluation loop hold one index fixed and spread
    // the other two over the lanes; with rows unpadded (RS = SB) and the plane
    // pitch below, searched over all six patterns for 64 banks of 4 bytes,
    // every such read is at most 2-way (float) or 3-way (double) conflicted.
    constexpr int RS = SB;
    constexpr int PS = sizeof(WT) == 4 ? 69 : 67;
    constexpr int BLK = SB * PS;          // one W sub-block
    constexpr int SRS = SB + 1;           // padded S row
    constexpr int SBLK = SB * SRS;        // one S sub-block
    constexpr int VPR = 16 / sizeof(WT);  // W elements per 16-byte load
    constexpr int NVL = SB / VPR;         // 16-byte loads per W row
    __shared__ WT lw[EW][6][BLK];
    // integral sub-blocks staged in FP64 in every precision, so that Z is
    // formed from the caller's FP64 integrals (only W carries the precision
    // of the contraction)
    __shared__ double ls[EW][18][SBLK];
    __shared__ double lt[EW][4][3][SB];   // t1_i, t1_j, t1_k, eps_v over sub-blocks x, y, z
    __shared__ double sh[EW];
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
    const int v = S->v, o = S->o, i = S->i, j = S->j, k = S->k, nb = S->nbw;
    const GLOBAL WT* W = gp(static_cast<const WT*>(S->w));                 // W_A
    const GLOBAL WT* WBp = W + (int64_t)nb * nb * nb * (WB * WB * WB);       // W_B
    const bool onepass = S->npass == 1;
    const GLOBAL double* eps_o = gp(S->eps_o);
    const double eo = eps_o[i] + eps_o[j] + eps_o[k];
    // (pX|qY) = ovov[p][X][q][Y]; Spq[X * rs + Y] = (pX|qY)
    const double* ov = S->ovov;
    const int64_t rs = (int64_t)o * v;
    const GLOBAL double* S0 = gp(ov + ((int64_t)j * v * o + k) * v);   // (jX|kY)
    const GLOBAL double* S1 = gp(ov + ((int64_t)i * v * o + k) * v);   // (iX|kY)
    const GLOBAL double* S2 = gp(ov + ((int64_t)i * v * o + j) * v);   // (iX|jY)
    const GLOBAL double* T0 = gp(S->t1 + (int64_t)i * v);
    const GLOBAL double* T1 = gp(S->t1 + (int64_t)j * v);
    const GLOBAL double* T2 = gp(S->t1 + (int64_t)k * v);
    const GLOBAL double* ev = gp(S->eps_v);
    const double scale = (double)S->mult / 3.0;
    const int nsb = (v + SB - 1) / SB;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    WT(*L)[BLK] = lw[wave];
    double(*LS)[SBLK] = ls[wave];
    double(*LT)[3][SB] = lt[wave];

    double e4 = 0.0, e5 = 0.0;
    for (int it = 0; it < 8 / EW; ++it) {
        const int s = wave + EW * it;
        const int x = 2 * A + ((s >> 2) & 1), y = 2 * B + ((s >> 1) & 1), z = 2 * C + (s & 1);
        const bool ok = x <= y && y <= z && z < nsb;
        if (ok) {
            const int r = lane >> 3, cc = lane & 7;
            // W sub-blocks, order q: (x,y,z) (x,z,y) (y,x,z) (y,z,x) (z,x,y) (z,y,x)
            const int P[6][3] = {{x, y, z}, {x, z, y}, {y, x, z}, {y, z, x}, {z, x, y}, {z, y, x}};
            u32x4 wa[6][NVL], wb[6][NVL];
            // Each SB^3 sub-block is contiguous: load g of lane l covers
            // elements VPR (l + 64 g) .. + VPR - 1, one coalesced 1 KB
            // read per load across the wave.  Elements past v are never
            // written by the contraction and never used here.
#pragma unroll
            for (int p = 0; p < 6; ++p) {
                const int64_t off = w_index(SB * P[p][0], SB * P[p][1], SB * P[p][2], nb);
                // one-pass slot (i = j): W_B[a][b][c] = W_A[b][a][c], the sub-block
                // with the first two indices exchanged
                const int64_t offB = onepass ? w_index(SB * P[p][1], SB * P[p][0], SB * P[p][2], nb) : off;
                const GLOBAL u32x4* srcA = (const GLOBAL u32x4*)(W + off);
                const GLOBAL u32x4* srcB = (const GLOBAL u32x4*)((onepass ? W : WBp) + offB);
#pragma unroll
                for (int g = 0; g < NVL; ++g) {
                    wa[p][g] = srcA[lane + 64 * g];
                    wb[p][g] = srcB[lane + 64 * g];
                }
            }
            // S sub-blocks: index pq*6 + qq, pairs qq: (y,z) (z,y) (x,z) (z,x) (x,y) (y,x)
            const int QP[6][2] = {{y, z}, {z, y}, {x, z}, {z, x}, {x, y}, {y, x}};
            double sv[18];
#pragma unroll
            for (int qq = 0; qq < 6; ++qq) {
                const int64_t off = (int64_t)min(SB * QP[qq][0] + r, v - 1) * rs + min(SB * QP[qq][1] + cc, v - 1);
                sv[qq] = S0[off];
                sv[6 + qq] = S1[off];
                sv[12 + qq] = S2[off];
            }
            // t1_i, t1_j, t1_k, eps_v over sub-blocks x, y, z: entry e = vec*24 + blk*8 + off
            double tv[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int e = lane + 64 * h;
                double val = 0.0;
                if (e < 96) {
                    const int vec = e / 24, blk = (e / SB) % 3, off = e % SB;
                    const int xb = blk == 0 ? x : (blk == 1 ? y : z);
                    const int g = min(SB * xb + off, v - 1);
                    const GLOBAL double* src = vec == 0 ? T0 : (vec == 1 ? T1 : (vec == 2 ? T2 : ev));
                    val = src[g];
                }
                tv[h] = val;
            }
            if (!onepass) {
#pragma unroll
                for (int p = 0; p < 6; ++p)
#pragma unroll
                    for (int g = 0; g < NVL; ++g) {
                        const int e = VPR * (lane + 64 * g);
                        Unpack<WT>::put2(&L[p][(e >> 6) * PS + ((e >> 3) & 7) * RS + (e & 7)], wa[p][g], wb[p][g]);
                    }
            } else {
                // W_A parts first, then W_B parts added at the exchanged positions
#pragma unroll
                for (int p = 0; p < 6; ++p)
#pragma unroll
                    for (int g = 0; g < NVL; ++g) {
                        const int e = VPR * (lane + 64 * g);
                        Unpack<WT>::put1(&L[p][(e >> 6) * PS + ((e >> 3) & 7) * RS + (e & 7)], wa[p][g]);
                    }
                wave_lds_fence();
#pragma unroll
                for (int p = 0; p < 6; ++p)
#pragma unroll
                    for (int g = 0; g < NVL; ++g) {
                        const int e = VPR * (lane + 64 * g);
                        Unpack<WT>::add1(&L[p][((e >> 3) & 7) * PS + (e >> 6) * RS + (e & 7)], wb[p][g]);
                    }
            }
#pragma unroll
            for (int n = 0; n < 18; ++n) LS[n][r * SRS + cc] = sv[n];
            (&LT[0][0][0])[lane] = tv[0];
            if (lane < 32) (&LT[0][0][0])[lane + 64] = tv[1];
        }
        wave_lds_fence();
        if (ok) {
            const int be = lane >> 3, ga = lane & 7;   // (beta, gamma) column of this lane
            const int b = SB * y + be, c = SB * z + ga;
            if (b < v && c < v && b <= c) {
                // LT[vec][blk][off]: vec 0 t1_i, 1 t1_j, 2 t1_k, 3 eps_v; blk 0 x, 1 y, 2 z
                const double evbc = LT[3][1][be] + LT[3][2][ga];
                const double t1ib = LT[0][1][be], t1ic = LT[0][2][ga];
                const double t1jb = LT[1][1][be], t1jc = LT[1][2][ga];
                const double t1kb = LT[2][1][be], t1kc = LT[2][2][ga];
                // alpha-independent S entries: Q0 = (y,z), Q1 = (z,y)
                const double Sjk_bc = LS[0][be * SRS + ga], Sjk_cb = LS[1][ga * SRS + be];
                const double Sik_bc = LS[6][be * SRS + ga], Sik_cb = LS[7][ga * SRS + be];
                const double Sij_bc = LS[12][be * SRS + ga], Sij_cb = LS[13][ga * SRS + be];
                for (int al = 0; al < SB; ++al) {
                    const int a = SB * x + al;
                    if (a > b) break;
                    if (a == c) continue;  // a = b = c
                    const double w0 = (double)L[0][al * PS + be * RS + ga];
                    const double w1 = (double)L[1][al * PS + ga * RS + be];
                    const double w2 = (double)L[2][be * PS + al * RS + ga];
                    const double w3 = (double)L[3][be * PS + ga * RS + al];
                    const double w4 = (double)L[4][ga * PS + al * RS + be];
                    const double w5 = (double)L[5][ga * PS + be * RS + al];
                    const double t1ia = LT[0][0][al], t1ja = LT[1][0][al], t1ka = LT[2][0][al];
                    // pairs: Q2 (x,z) [al][ga], Q3 (z,x) [ga][al], Q4 (x,y) [al][be], Q5 (y,x) [be][al]
                    const double Sjk_ac = LS[2][al * SRS + ga], Sjk_ca = LS[3][ga * SRS + al];
                    const double Sjk_ab = LS[4][al * SRS + be], Sjk_ba = LS[5][be * SRS + al];
                    const double Sik_ac = LS[8][al * SRS + ga], Sik_ca = LS[9][ga * SRS + al];
                    const double Sik_ab = LS[10][al * SRS + be], Sik_ba = LS[11][be * SRS + al];
                    const double Sij_ac = LS[14][al * SRS + ga], Sij_ca = LS[15][ga * SRS + al];
                    const double Sij_ab = LS[16][al * SRS + be], Sij_ba = LS[17][be * SRS + al];
                    // Z(x,y,z) = t1[i][x] (jy|kz) + t1[j][y] (ix|kz) + t1[k][z] (ix|jy)
                    const double z0 = t1ia * Sjk_bc + t1jb * Sik_ac + t1kc * Sij_ab;   // (a,b,c)
                    const double z1 = t1ia * Sjk_cb + t1jc * Sik_ab + t1kb * Sij_ac;   // (a,c,b)
                    const double z2 = t1ib * Sjk_ac + t1ja * Sik_bc + t1kc * Sij_ba;   // (b,a,c)
                    const double z3 = t1ib * Sjk_ca + t1jc * Sik_ba + t1ka * Sij_bc;   // (b,c,a)
                    const double z4 = t1ic * Sjk_ab + t1ja * Sik_cb + t1kb * Sij_ca;   // (c,a,b)
                    const double z5 = t1ic * Sjk_ba + t1jb * Sik_ca + t1ka * Sij_cb;   // (c,b,a)
                    const double We = w0 + w3 + w4, Wo = w1 + w2 + w5;
                    const double Ze = z0 + z3 + z4, Zo = z1 + z2 + z5;
                    const double sww = w0 * w0 + w1 * w1 + w2 * w2 + w3 * w3 + w4 * w4 + w5 * w5;
                    const double swz = w0 * z0 + w1 * z1 + w2 * z2 + w3 * z3 + w4 * z4 + w5 * z5;
                    const double f4 = 3.0 * sww + We * (We - 2.0 * Wo) + Wo * (Wo - 2.0 * We);
                    const double f5 = 3.0 * swz + We * (Ze - 2.0 * Zo) + Wo * (Zo - 2.0 * Ze);
                    const double D = eo - LT[3][0][al] - evbc;
                    const double rep = (a == b || b == c) ? 2.0 : 1.0;
                    const double sc = scale / (rep * D);
                    e4 += f4 * sc;
                    e5 += f5 * sc;
                }
            }
        }
        wave_lds_fence();
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
    const int nb = S->nbw;
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

__global__ __launch_bounds__(256) void gap_check_kernel(const GapDesc* __restrict__ desc,
                                                        double* __restrict__ flag) {
    __shared__ double smax[256], smin[256];
    __shared__ int sbad;
    const GapDesc g = desc[blockIdx.x];
    if (threadIdx.x == 0) sbad = 0;
    __syncthreads();
    double mo = -INFINITY, mv = INFINITY;
    int bad = 0;
    for (int n = threadIdx.x; n < g.o; n += 256) {
        const double x = g.eps_o[n];
        bad |= !isfinite(x);
        mo = fmax(mo, x);
    }
    for (int n = threadIdx.x; n < g.v; n += 256) {
        const double x = g.eps_v[n];
        bad |= !isfinite(x);
        mv = fmin(mv, x);
    }
    smax[threadIdx.x] = mo;
    smin[threadIdx.x] = mv;
    if (bad) atomicOr(&sbad, 1);
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + h]);
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + h]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) flag[blockIdx.x] = sbad ? 1.0 : (smax[0] < smin[0] ? 0.0 : 2.0);
}

template <class WT>
__global__ void widen_kernel(const WT* __restrict__ w, int v, double* __restrict__ out) {
    const int nb = (v + WB - 1) / WB;
    const int64_t n = (int64_t)v * v * v;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e % v), b = (int)((e / v) % v), a = (int)(e / ((int64_t)v * v));
        const int64_t half = (int64_t)nb * nb * nb * (WB * WB * WB);
        out[e] = (double)(WT)(w[w_index(a, b, c, nb)] + w[half + w_index(a, b, c, nb)]);
    }
}

hipError_t launch_energy(int prec, const Slot* d_slots, int nslot, int total, double* partials, hipStream_t s) {
    if (total <= 0) return hipSuccess;
    if (prec == P_FP64)
        hipLaunchKernelGGL(energy_kernel<double>, dim3(total), dim3(EW * 64), 0, s, d_slots, nslot, partials);
    else
        hipLaunchKernelGGL(energy_kernel<float>, dim3(total), dim3(EW * 64), 0, s, d_slots, nslot, partials);
    return hipGetLastError();
}

hipError_t launch_slot_reduce(const Slot* d_slots, int nslot, const double* partials, double* e_trip,
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

hipError_t launch_gap_check(const GapDesc* d_desc, int nprob, double* flag, hipStream_t s) {
    hipLaunchKernelGGL(gap_check_kernel, dim3(nprob), dim3(256), 0, s, d_desc, flag);
    return hipGetLastError();
}

hipError_t launch_widen_w(int prec, const void* w, int v, double* out, hipStream_t s) {
    const int64_t n = (int64_t)v * v * v;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 65536);
    if (prec == P_FP64)
        hipLaunchKernelGGL(widen_kernel<double>, dim3(grid), dim3(256), 0, s, static_cast<const double*>(w), v, out);
    else
        hipLaunchKernelGGL(widen_kernel<float>, dim3(grid), dim3(256), 0, s, static_cast<const float*>(w), v, out);
    return hipGetLastError();
}

}  // namespace ccsdt
