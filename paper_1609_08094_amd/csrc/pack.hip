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
#include <algorithm>

#include "common.hpp"
#include "pack_out.hpp"

namespace ccsdt {

// G particle part.  For fixed (y, d) the (x, p) plane of vvvo[y][d][x][p]
// is one contiguous run of v*o doubles; with q = x*o + p, a workgroup takes
// 64 values of d and 128 consecutive q, reads 64 runs of 1 KB, transposes
// through LDS and writes, for each q, 64 consecutive kappa = d of row
// G[p][x][y].  Grid: (q tiles) x (d tiles) x y, q tiles fastest.
constexpr int PK_D = 64, PK_Q = 128;

// `vvvo` holds the rows y0 .. y0 + ny - 1 of vvvo[y][d][x][p] (the whole block,
// or one streamed chunk); the grid covers those rows.
template <class O>
__global__ __launch_bounds__(256) void pack_g_particle(const double* __restrict__ vvvo, int o, int v,
                                                       int Kp, typename O::T* __restrict__ g, int y0) {
    __shared__ double tile[PK_D][PK_Q + 1];
    const int64_t nq = (int64_t)v * o;
    const int qtiles = (int)((nq + PK_Q - 1) / PK_Q);
    const int dtiles = (v + PK_D - 1) / PK_D;
    const int64_t bid = blockIdx.x;
    const int qt = (int)(bid % qtiles);
    const int dt = (int)((bid / qtiles) % dtiles);
    const int yl = (int)(bid / ((int64_t)qtiles * dtiles));   // row within the chunk
    const int y = y0 + yl;
    const int64_t q0 = (int64_t)qt * PK_Q;
    const int d0 = dt * PK_D;
    const GLOBAL double* src = gp(vvvo);
    for (int e = threadIdx.x; e < PK_D * PK_Q; e += 256) {
        const int dd = e / PK_Q, qq = e % PK_Q;
        const int d = d0 + dd;
        const int64_t q = q0 + qq;
        double val = 0.0;
        if (d < v && q < nq) val = src[((int64_t)yl * v + d) * nq + q];
        tile[dd][qq] = val;
    }
    __syncthreads();
    const int64_t rl = O::rowlen(Kp);
    for (int e = threadIdx.x; e < PK_D * PK_Q; e += 256) {
        const int qq = e / PK_D, dd = e % PK_D;
        const int d = d0 + dd;
        const int64_t q = q0 + qq;
        if (d < v && q < nq) {
            const int x = (int)(q / o), p = (int)(q % o);
            typename O::T* row = g + (((int64_t)p * v + x) * v + y) * rl;
            O::put(row, d, tile[dd][qq]);
        }
    }
}

// G hole part and zero padding: kappa = v + l of rows G[p][x][y] from
// t2[p][l][x][y].  A workgroup takes (p, x) and 64 values of y; per chunk of
// 64 values of kappa - v it reads the runs t2[p][l][x][y0..y0+63],
// transposes through LDS, and writes for each y consecutive kappa (hole part,
// then zeros up to Kp).
template <class O>
__global__ __launch_bounds__(256) void pack_g_hole(const double* __restrict__ t2, int o, int v, int Kp,
                                                   typename O::T* __restrict__ g) {
    __shared__ double tile[64][65];
    const int ytiles = (v + 63) / 64;
    const int px = blockIdx.x / ytiles;
    const int y0 = (blockIdx.x % ytiles) * 64;
    const int p = px / v, x = px % v;
    const int kext = Kp - v;
    const int64_t rl = O::rowlen(Kp);
    typename O::T* rows = g + ((int64_t)p * v + x) * v * rl;
    for (int l0 = 0; l0 < kext; l0 += 64) {
        const int lc = min(64, kext - l0);
        for (int e = threadIdx.x; e < 64 * 64; e += 256) {
            const int ll = e / 64, yy = e % 64;
            const int l = l0 + ll;
            double val = 0.0;
            if (l < o && y0 + yy < v) val = t2[(((int64_t)p * o + l) * v + x) * v + y0 + yy];
            tile[ll][yy] = val;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < 64 * lc; e += 256) {
            const int yy = e / lc, ll = e % lc;
            if (y0 + yy < v) O::put(rows + (int64_t)(y0 + yy) * rl, v + l0 + ll, tile[ll][yy]);
        }
        __syncthreads();
    }
}

// T rows: one workgroup per row (r, q, z), grid-stride over the o*o*v rows.
template <class O>
__global__ __launch_bounds__(256) void pack_t(const double* __restrict__ t2, const double* __restrict__ ovoo,
                                              int o, int v, int Kp, typename O::T* __restrict__ t) {
    const int64_t nrows = (int64_t)o * o * v;
    for (int64_t row = blockIdx.x; row < nrows; row += gridDim.x) {
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
}

template <class O>
static hipError_t pack_impl(int o, int v, int Kp, const double* vvvo, const double* t2, const double* ovoo,
                            void* gc, void* tc, hipStream_t s) {
    auto* g = static_cast<typename O::T*>(gc);
    auto* t = static_cast<typename O::T*>(tc);
    hipError_t e;
    if (vvvo) {
        const int64_t qtiles = ((int64_t)v * o + PK_Q - 1) / PK_Q, dtiles = (v + PK_D - 1) / PK_D;
        hipLaunchKernelGGL(pack_g_particle<O>, dim3((unsigned)(qtiles * dtiles * v)), dim3(256), 0, s, vvvo, o, v,
                           Kp, g, 0);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(pack_g_hole<O>, dim3((unsigned)((int64_t)o * v * ((v + 63) / 64))), dim3(256), 0, s, t2, o,
                       v, Kp, g);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t trows = (int64_t)o * o * v;
    hipLaunchKernelGGL(pack_t<O>, dim3((unsigned)std::min<int64_t>(trows, (int64_t)1 << 22)), dim3(256), 0, s, t2,
                       ovoo, o, v, Kp, t);
    return hipGetLastError();
}

template <class O>
static hipError_t pack_chunk_impl(int o, int v, int Kp, const double* chunk, int y0, int ny, void* gc, hipStream_t s) {
    const int64_t qtiles = ((int64_t)v * o + PK_Q - 1) / PK_Q, dtiles = (v + PK_D - 1) / PK_D;
    hipLaunchKernelGGL(pack_g_particle<O>, dim3((unsigned)(qtiles * dtiles * ny)), dim3(256), 0, s, chunk, o, v, Kp,
                       static_cast<typename O::T*>(gc), y0);
    return hipGetLastError();
}

hipError_t launch_pack_particle_chunk(int prec, int o, int v, int Kp, const double* chunk, int y0, int ny, void* gc,
                                      hipStream_t s) {
    switch (prec) {
        case P_FP64: return pack_chunk_impl<OutF64>(o, v, Kp, chunk, y0, ny, gc, s);
        case P_FP32: return pack_chunk_impl<OutF32>(o, v, Kp, chunk, y0, ny, gc, s);
        case P_BF16X3: return pack_chunk_impl<OutB3>(o, v, Kp, chunk, y0, ny, gc, s);
        default: return hipErrorInvalidValue;
    }
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
