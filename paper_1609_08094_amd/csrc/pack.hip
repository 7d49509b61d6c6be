// Device-resident operand layout for the (T) contractions.
//
// The connected bracket of eq. analytical_triples_ampl (paper Sec. 2.2) is,
// for an occupied triple (p,q,r) and virtual triple (x,y,z),
//   X^xyz_pqr = sum_d (yd|xp) t^zd_rq  -  sum_l (rz|ql) t^xy_pl .
// Both sums are dot products over one index, so we store each side as one
// row of length Kp = roundup(v + o, 32) with the summation index fastest:
//   G[p][x][y][d]     = (yd|xp) = vvvo[y][d][x][p]     d < v
//   G[p][x][y][v + l] = t^xy_pl = t2[p][l][x][y]       l < o
//   T[r][q][z][d]     = t^zd_rq = t2[r][q][z][d]       d < v
//   T[r][q][z][v + l] = -(rz|ql) = -ovoo[r][z][q][l]   l < o
// and zero beyond v + o.  Then X^xyz_pqr = <G[p][x][y][:], T[r][q][z][:]>:
// the particle and hole terms of one permutation become a single K = v + o
// contraction.
//
// Element formats per precision:
//   FP64   double
//   FP32   float  (round to nearest even)
//   BF16X3 hi = bf16(x), lo = bf16(x - hi), stored in groups of eight
//          elements as [hi x8][lo x8] (16 bf16 = 32 bytes per group), so that
//          one 32-byte load gives a lane both halves of an MFMA fragment.
#include "common.hpp"

namespace ccsdt {

__device__ __forceinline__ uint16_t bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

struct OutF64 {
    using T = double;
    static __device__ __forceinline__ int64_t rowlen(int Kp) { return Kp; }
    static __device__ __forceinline__ void put(T* row, int kappa, double x) { row[kappa] = x; }
};
struct OutF32 {
    using T = float;
    static __device__ __forceinline__ int64_t rowlen(int Kp) { return Kp; }
    static __device__ __forceinline__ void put(T* row, int kappa, double x) { row[kappa] = (float)x; }
};
struct OutB3 {
    using T = uint16_t;
    static __device__ __forceinline__ int64_t rowlen(int Kp) { return 2 * (int64_t)Kp; }
    static __device__ __forceinline__ void put(T* row, int kappa, double x) {
        uint16_t hi = bf16_rne((float)x);
        float hf = __uint_as_float((uint32_t)hi << 16);
        uint16_t lo = bf16_rne((float)(x - (double)hf));
        int base = (kappa >> 3) * 16 + (kappa & 7);
        row[base] = hi;
        row[base + 8] = lo;
    }
};

// G particle part: one workgroup per (y, x); tiles of 64 d x 32 p through LDS.
template <class O>
__global__ __launch_bounds__(256) void pack_g_particle(const double* __restrict__ vvvo, int o, int v,
                                                       int Kp, typename O::T* __restrict__ g) {
    __shared__ double tile[64][33];
    const int y = blockIdx.x / v;
    const int x = blockIdx.x % v;
    const int64_t rl = O::rowlen(Kp);
    for (int d0 = 0; d0 < v; d0 += 64) {
        for (int p0 = 0; p0 < o; p0 += 32) {
            __syncthreads();
            for (int e = threadIdx.x; e < 64 * 32; e += 256) {
                int dd = e >> 5, pp = e & 31;
                int d = d0 + dd, p = p0 + pp;
                double val = 0.0;
                if (d < v && p < o) val = vvvo[(((int64_t)y * v + d) * v + x) * o + p];
                tile[dd][pp] = val;
            }
            __syncthreads();
            for (int e = threadIdx.x; e < 64 * 32; e += 256) {
                int pp = e >> 6, dd = e & 63;
                int d = d0 + dd, p = p0 + pp;
                if (d < v && p < o) {
                    typename O::T* row = g + (((int64_t)p * v + x) * v + y) * rl;
                    O::put(row, d, tile[dd][pp]);
                }
            }
        }
    }
}

// G hole part and zero padding: one workgroup per (p, x).
template <class O>
__global__ __launch_bounds__(256) void pack_g_hole(const double* __restrict__ t2, int o, int v, int Kp,
                                                   typename O::T* __restrict__ g) {
    const int p = blockIdx.x / v;
    const int x = blockIdx.x % v;
    const int64_t rl = O::rowlen(Kp);
    typename O::T* rows = g + ((int64_t)p * v + x) * v * rl;
    const int kext = Kp - v;  // hole entries plus padding per row
    for (int e = threadIdx.x; e < kext * v; e += 256) {
        int l = e / v, y = e % v;
        double val = 0.0;
        if (l < o) val = t2[(((int64_t)p * o + l) * v + x) * v + y];
        O::put(rows + (int64_t)y * rl, v + l, val);
    }
}

// T rows: one workgroup per (r, q, z).
template <class O>
__global__ __launch_bounds__(256) void pack_t(const double* __restrict__ t2, const double* __restrict__ ovoo,
                                              int o, int v, int Kp, typename O::T* __restrict__ t) {
    const int64_t row = blockIdx.x;
    const int z = (int)(row % v);
    const int rq = (int)(row / v);
    const int r = rq / o, q = rq % o;
    typename O::T* out = t + row * O::rowlen(Kp);
    for (int kap = threadIdx.x; kap < Kp; kap += 256) {
        double val = 0.0;
        if (kap < v) val = t2[row * v + kap];
        else if (kap < v + o) val = -ovoo[(((int64_t)r * v + z) * o + q) * o + (kap - v)];
        O::put(out, kap, val);
    }
}

template <class O>
static hipError_t pack_impl(int o, int v, int Kp, const double* vvvo, const double* t2, const double* ovoo,
                            void* gc, void* tc, hipStream_t s) {
    auto* g = static_cast<typename O::T*>(gc);
    auto* t = static_cast<typename O::T*>(tc);
    hipLaunchKernelGGL(pack_g_particle<O>, dim3((unsigned)v * v), dim3(256), 0, s, vvvo, o, v, Kp, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(pack_g_hole<O>, dim3((unsigned)o * v), dim3(256), 0, s, t2, o, v, Kp, g);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(pack_t<O>, dim3((unsigned)((int64_t)o * o * v)), dim3(256), 0, s, t2, ovoo, o, v, Kp, t);
    return hipGetLastError();
}

hipError_t launch_pack(int prec, int o, int v, int Kp, const double* vvvo, const double* t2,
                       const double* ovoo, void* gc, void* tc, hipStream_t s) {
    switch (prec) {
        case P_FP64: return pack_impl<OutF64>(o, v, Kp, vvvo, t2, ovoo, gc, tc, s);
        case P_FP32: return pack_impl<OutF32>(o, v, Kp, vvvo, t2, ovoo, gc, tc, s);
        case P_BF16X3: return pack_impl<OutB3>(o, v, Kp, vvvo, t2, ovoo, gc, tc, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ccsdt
