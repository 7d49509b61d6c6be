// MFMA precision traits and LDS staging helpers shared by the matrix
// kernels (the (T) contraction and the RI-MP2 pair products).
//
// A packed operand row holds the summation index fastest (pack.hip); a
// 16x16 output block is accumulated over chunks of KCH elements:
//   FP64    v_mfma_f64_16x16x4_f64     4 steps per 16-element chunk
//   FP32    v_mfma_f32_16x16x4_f32     4 steps per 16-element chunk
//   BF16X3  v_mfma_f32_16x16x32_bf16   hi*hi + hi*lo + lo*hi per 32-element chunk
// Within a chunk each lane owns a contiguous run of k; A and B use the same
// assignment, so the dot product covers every k exactly once.  Output: lane
// l holds four rows of column l%16 -- rows l/16 + 4r for the FP64
// instruction, 4(l/16) + r for the FP32-accumulating ones.
//
// The *W traits use 32x32 output blocks (v_mfma_f32_32x32x16_bf16,
// v_mfma_f32_32x32x2_f32): the same flops per cycle from half as many
// instructions, each reading half the operand registers per flop.  Lane l
// supplies row l%32 and k-group l/32; it holds sixteen rows of column l%32,
// rows 8(r/4) + 4(l/32) + r%4.
#pragma once

#include "common.hpp"

namespace ccsdt {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));  // HIP uint4 blocks scalar replacement

// Workgroups are dispatched round-robin over the XCDs; give each XCD a
// contiguous range of logical work so tiles sharing operand rows share an L2.
__device__ __forceinline__ int xcd_remap(int bid, int total) {
    const int q = total / NXCD, r = total % NXCD;
    const int x = bid % NXCD, idx = bid / NXCD;
    return x * q + min(x, r) + idx;
}

struct PrecF64 {
    using E = double;
    using W = double;
    using Acc = f64x4;
    static constexpr int KCH = 16;
    static constexpr int UNITS = 1;
    struct Frag { f64x4 x; };
    static constexpr int BS = 16;     // output block edge
    static constexpr int NACC = 4;    // accumulator elements per lane
    static __device__ __forceinline__ int out_row(int lane, int r) { return (lane >> 4) + 4 * r; }
    static __device__ __forceinline__ void load(Frag& f, const E* row, int c, int lane) {
        f.x = *reinterpret_cast<const GLOBAL f64x4*>(gp(row + c * 16 + 4 * (lane >> 4)));
    }
    // LDS staging (128-byte rows of eight 16-byte chunks, see contract_lds_kernel).
    static constexpr int NSUB = 1;     // k sub-steps per 128-byte LDS row chunk set
    static constexpr bool SPLIT = true;  // a lane's 32 bytes live in LDS chunks g and 4 + g
    static __device__ __forceinline__ void load_lds(Frag& f, const char* row, int g, int sub, int sw) {
        const double2 x0 = *reinterpret_cast<const double2*>(row + 16 * (g ^ sw));
        const double2 x1 = *reinterpret_cast<const double2*>(row + 16 * ((4 + g) ^ sw));
        f.x = f64x4{x0.x, x0.y, x1.x, x1.y};
    }
    // the NMMA products of one chunk, in accumulation order
    static constexpr int NMMA = 4;
    template <int T>
    static __device__ __forceinline__ void mma_t(Acc& acc, const Frag& a, const Frag& b) {
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x[T], b.x[T], acc, 0, 0, 0);
    }
    static __device__ __forceinline__ void mma(Acc& acc, const Frag& a, const Frag& b) {
        mma_t<0>(acc, a, b);
        mma_t<1>(acc, a, b);
        mma_t<2>(acc, a, b);
        mma_t<3>(acc, a, b);
    }
};

struct PrecF32 {
    using E = float;
    using W = float;
    using Acc = f32x4;
    static constexpr int KCH = 16;
    static constexpr int UNITS = 1;
    struct Frag { f32x4 x; };
    static constexpr int BS = 16;     // output block edge
    static constexpr int NACC = 4;    // accumulator elements per lane
    static __device__ __forceinline__ int out_row(int lane, int r) { return 4 * (lane >> 4) + r; }
    static __device__ __forceinline__ void load(Frag& f, const E* row, int c, int lane) {
        f.x = *reinterpret_cast<const GLOBAL f32x4*>(gp(row + c * 16 + 4 * (lane >> 4)));
    }
    static constexpr int NSUB = 2;
    static constexpr bool SPLIT = false;  // sub-step s, lane group g reads LDS chunk 4 s + g
    static __device__ __forceinline__ void load_lds(Frag& f, const char* row, int g, int sub, int sw) {
        f.x = *reinterpret_cast<const f32x4*>(row + 16 * ((4 * sub + g) ^ sw));
    }
    static constexpr int NMMA = 4;
    template <int T>
    static __device__ __forceinline__ void mma_t(Acc& acc, const Frag& a, const Frag& b) {
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x[T], b.x[T], acc, 0, 0, 0);
    }
    static __device__ __forceinline__ void mma(Acc& acc, const Frag& a, const Frag& b) {
        mma_t<0>(acc, a, b);
        mma_t<1>(acc, a, b);
        mma_t<2>(acc, a, b);
        mma_t<3>(acc, a, b);
    }
};

struct PrecB3 {
    using E = uint16_t;
    using W = float;
    using Acc = f32x4;
    static constexpr int KCH = 32;
    static constexpr int UNITS = 2;
    struct Frag { bf16x8 hi, lo; };
    static constexpr int BS = 16;     // output block edge
    static constexpr int NACC = 4;    // accumulator elements per lane
    static __device__ __forceinline__ int out_row(int lane, int r) { return 4 * (lane >> 4) + r; }
    static __device__ __forceinline__ void load(Frag& f, const E* row, int c, int lane) {
        const GLOBAL E* p = gp(row + (c * 4 + (lane >> 4)) * 16);
        f.hi = *reinterpret_cast<const GLOBAL bf16x8*>(p);
        f.lo = *reinterpret_cast<const GLOBAL bf16x8*>(p + 8);
    }
    static constexpr int NSUB = 1;
    static constexpr bool SPLIT = true;  // hi of group g in LDS chunk g, lo in chunk 4 + g
    static __device__ __forceinline__ void load_lds(Frag& f, const char* row, int g, int sub, int sw) {
        f.hi = *reinterpret_cast<const bf16x8*>(row + 16 * (g ^ sw));
        f.lo = *reinterpret_cast<const bf16x8*>(row + 16 * ((4 + g) ^ sw));
    }
    static constexpr int NMMA = 3;
    template <int T>
    static __device__ __forceinline__ void mma_t(Acc& acc, const Frag& a, const Frag& b) {
        if constexpr (T == 0) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.lo, b.hi, acc, 0, 0, 0);
        if constexpr (T == 1) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi, b.lo, acc, 0, 0, 0);
        if constexpr (T == 2) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi, b.hi, acc, 0, 0, 0);
    }
    static __device__ __forceinline__ void mma(Acc& acc, const Frag& a, const Frag& b) {
        mma_t<0>(acc, a, b);
        mma_t<1>(acc, a, b);
        mma_t<2>(acc, a, b);
    }
};

// PrecF32 with 32x32 output blocks.  A 128-byte stage row holds 32 k; sub-step
// s, lane group g (0, 1) reads chunk 2 s + g, four k per lane, one per MFMA.
struct PrecF32W : PrecF32 {
    using Acc = f32x16;
    static constexpr int BS = 32;
    static constexpr int NACC = 16;
    static __device__ __forceinline__ int out_row(int lane, int r) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }
    static constexpr int NSUB = 4;
    static __device__ __forceinline__ void load_lds(Frag& f, const char* row, int g, int sub, int sw) {
        f.x = *reinterpret_cast<const f32x4*>(row + 16 * ((2 * sub + g) ^ sw));
    }
    template <int T>
    static __device__ __forceinline__ void mma_t(Acc& acc, const Frag& a, const Frag& b) {
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x[T], b.x[T], acc, 0, 0, 0);
    }
    static __device__ __forceinline__ void mma(Acc& acc, const Frag& a, const Frag& b) {
        mma_t<0>(acc, a, b);
        mma_t<1>(acc, a, b);
        mma_t<2>(acc, a, b);
        mma_t<3>(acc, a, b);
    }
};

// PrecB3 with 32x32 output blocks.  A 128-byte stage row holds four groups of
// 8 k; sub-step s, lane group g (0, 1) takes group q = 2 s + g (hi in LDS
// chunk q, lo in chunk 4 + q).
struct PrecB3W : PrecB3 {
    using Acc = f32x16;
    static constexpr int BS = 32;
    static constexpr int NACC = 16;
    static __device__ __forceinline__ int out_row(int lane, int r) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }
    static constexpr int NSUB = 2;
    static __device__ __forceinline__ void load_lds(Frag& f, const char* row, int g, int sub, int sw) {
        const int q = 2 * sub + g;
        f.hi = *reinterpret_cast<const bf16x8*>(row + 16 * (q ^ sw));
        f.lo = *reinterpret_cast<const bf16x8*>(row + 16 * ((4 + q) ^ sw));
    }
    template <int T>
    static __device__ __forceinline__ void mma_t(Acc& acc, const Frag& a, const Frag& b) {
        if constexpr (T == 0) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.lo, b.hi, acc, 0, 0, 0);
        if constexpr (T == 1) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.hi, b.lo, acc, 0, 0, 0);
        if constexpr (T == 2) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.hi, b.hi, acc, 0, 0, 0);
    }
    static __device__ __forceinline__ void mma(Acc& acc, const Frag& a, const Frag& b) {
        mma_t<0>(acc, a, b);
        mma_t<1>(acc, a, b);
        mma_t<2>(acc, a, b);
    }
};

// The 32x32-block form of a precision (FP64 has no 32x32 MFMA and keeps its own).
template <class P> struct Wide { using T = P; };
template <> struct Wide<PrecF32> { using T = PrecF32W; };
template <> struct Wide<PrecB3> { using T = PrecB3W; };

// BF16 split products with the lo*lo term kept (four MFMAs per chunk), into
// two FP32 accumulators: hi*hi in `big`, the three correction products in
// `small`, added when read.  For sums of squares (the diagonal RI-MP2
// integrals g_aiai) the dropped lo*lo term of PrecB3 is a one-signed bias of
// about 2^-16 relative; kept in the same accumulator as hi*hi it would still
// be lost, since each chunk's lo*lo sum lies below half an ulp of the
// accumulated hi*hi sum.  In a separate accumulator, which stays small, it
// survives; the remaining error is the signed residual of the two-term split
// and the FP32 accumulation.
struct AccPair {
    f32x4 big, small;
    __device__ __forceinline__ float operator[](int r) const { return big[r] + small[r]; }
};

struct PrecB4 : PrecB3 {
    using Acc = AccPair;
    static constexpr int NMMA = 4;
    template <int T>
    static __device__ __forceinline__ void mma_t(Acc& acc, const Frag& a, const Frag& b) {
        if constexpr (T == 0) acc.small = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.lo, b.lo, acc.small, 0, 0, 0);
        if constexpr (T == 1) acc.small = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.lo, b.hi, acc.small, 0, 0, 0);
        if constexpr (T == 2) acc.small = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi, b.lo, acc.small, 0, 0, 0);
        if constexpr (T == 3) acc.big = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi, b.hi, acc.big, 0, 0, 0);
    }
    static __device__ __forceinline__ void mma(Acc& acc, const Frag& a, const Frag& b) {
        mma_t<0>(acc, a, b);
        mma_t<1>(acc, a, b);
        mma_t<2>(acc, a, b);
        mma_t<3>(acc, a, b);
    }
};

// Barrier after which the global_load_lds transfers of every wave have
// landed in LDS.  A global_load_lds is a load whose LDS write completes with
// the vector-memory counter; the fence of __syncthreads need not wait for
// outstanding loads (whether the compiler adds that wait depends on the code
// around the barrier), so the wait is explicit.
__device__ __forceinline__ void lds_dma_barrier() {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
}

// Workgroup-row swizzle of the 16-byte LDS chunks of a 128-byte stage row
// (see the LDS-staged contraction kernel for the layout it serves).
__device__ __forceinline__ int lds_swz(int row) { return (((row >> 1) & 1) << 2) | (((row >> 2) & 1) << 1); }

// The swizzle for fragments of BS rows.  A 128-bit LDS read serves two
// groups of eight lanes per cycle; for 32-row fragments (32x32 blocks) the
// two groups read the same chunk of rows 16 apart, which lds_swz alone maps
// to the same banks (measured: one conflict cycle per read).  Row bit 4 then
// also flips chunk bit 0.
template <int BS>
__device__ __forceinline__ int lds_swz_bs(int row) {
    return BS == 32 ? (lds_swz(row) ^ ((row >> 4) & 1)) : lds_swz(row);
}

// The MFMAs of one chunk for a wave's MB x NB blocks, product by product
// across all blocks, so that consecutive MFMAs never feed each other (each
// accumulator still sees its products in the order of P::mma).
template <class P, int MB, int NB, bool FULL, int T = 0>
__device__ __forceinline__ void mma_blocks(typename P::Acc (&acc)[MB][NB], const typename P::Frag (&fa)[MB],
                                           const typename P::Frag (&fb)[NB], int vm, int vn) {
    if constexpr (T < P::NMMA) {
#pragma unroll
        for (int a = 0; a < MB; ++a)
#pragma unroll
            for (int b = 0; b < NB; ++b)
                if (FULL || (a < vm && b < vn)) P::template mma_t<T>(acc[a][b], fa[a], fb[b]);
        mma_blocks<P, MB, NB, FULL, T + 1>(acc, fa, fb, vm, vn);
    }
}

// MFMAs over one LDS stage for a wave's MB x NB blocks.  FULL skips the
// per-block edge tests (interior tiles), keeping the MFMA stream branch-free.
template <class P, int MB, int NB, int RS, bool FULL>
__device__ __forceinline__ void lds_stage(typename P::Acc (&acc)[MB][NB], const char* As, const char* Bs, int g,
                                          int sw, int vm, int vn) {
    if constexpr (P::BS == 32) {
        // 32x32 blocks: the fragments of every sub-step are read before the
        // stage's first MFMA (as many registers as one 16x16 sub-step), so
        // the LDS latency is exposed once per stage, not once per sub-step.
        typename P::Frag fa[P::NSUB][MB], fb[P::NSUB][NB];
#pragma unroll
        for (int sub = 0; sub < P::NSUB; ++sub) {
#pragma unroll
            for (int a = 0; a < MB; ++a) P::load_lds(fa[sub][a], As + a * P::BS * RS, g, sub, sw);
#pragma unroll
            for (int b = 0; b < NB; ++b) P::load_lds(fb[sub][b], Bs + b * P::BS * RS, g, sub, sw);
        }
#pragma unroll
        for (int sub = 0; sub < P::NSUB; ++sub)
            mma_blocks<P, MB, NB, FULL>(acc, fa[sub], fb[sub], vm, vn);
        return;
    }
#pragma unroll
    for (int sub = 0; sub < P::NSUB; ++sub) {
        typename P::Frag fa[MB], fb[NB];
#pragma unroll
        for (int a = 0; a < MB; ++a) P::load_lds(fa[a], As + a * P::BS * RS, g, sub, sw);
#pragma unroll
        for (int b = 0; b < NB; ++b) P::load_lds(fb[b], Bs + b * P::BS * RS, g, sub, sw);
#pragma unroll
        for (int a = 0; a < MB; ++a)
#pragma unroll
            for (int b = 0; b < NB; ++b)
                if (FULL || (a < vm && b < vn)) P::mma(acc[a][b], fa[a], fb[b]);
    }
}

// As lds_stage with the MFMAs issued product by product across all blocks
// (no MFMA feeds the next one), for kernels with one wave per SIMD, where
// nothing else hides the latency of a dependent MFMA.
template <class P, int MB, int NB, int RS, bool FULL>
__device__ __forceinline__ void lds_stage_pm(typename P::Acc (&acc)[MB][NB], const char* As, const char* Bs, int g,
                                             int sw, int vm, int vn) {
#pragma unroll
    for (int sub = 0; sub < P::NSUB; ++sub) {
        typename P::Frag fa[MB], fb[NB];
#pragma unroll
        for (int a = 0; a < MB; ++a) P::load_lds(fa[a], As + a * P::BS * RS, g, sub, sw);
#pragma unroll
        for (int b = 0; b < NB; ++b) P::load_lds(fb[b], Bs + b * P::BS * RS, g, sub, sw);
        mma_blocks<P, MB, NB, FULL>(acc, fa, fb, vm, vn);
    }
}

}  // namespace ccsdt
