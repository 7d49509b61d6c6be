// Writers of one packed element in each precision's row format (see
// pack.hip for the layouts).  Shared by the pack and DF-assembly kernels.
#pragma once

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

}  // namespace ccsdt
