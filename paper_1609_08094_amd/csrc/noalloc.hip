// Static device workspace of the allocation-free entry point
// (ccsdt_energy_noalloc in api.cpp) and the two small kernels that only that
// path needs: a slot-table builder that enumerates the restricted triples on
// the device, and a finishing kernel that turns a failed denominator check
// into NaN results.
//
// The workspace is one file-scope device array.  Its name is only a
// host-side stand-in for the array, not a device address: the host obtains
// the address once per device with hipGetSymbolAddress (noalloc_scratch) and
// passes that pointer to every kernel.
#include <mutex>

#include "common.hpp"

namespace ccsdt {

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;

hipError_t noalloc_scratch(int dev, void** out) {
    static std::mutex mu;
    static void* addr[NOALLOC_MAX_DEVICES] = {};
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES || !out) return hipErrorInvalidValue;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        // the caller has made `dev` the current device: the symbol resolves
        // to that device's copy of the array
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *out = addr[dev];
    return hipSuccess;
}

// One thread per triple t of the restricted list (i<=j<=k, i=j=k left out, in
// lexicographic order).  Slots are grouped into chunks of `chunk` triples;
// within a chunk every slot is given the grid room of both contraction
// passes and its own W and partial-sum area, so that offsets follow from the
// slot's position alone (no prefix sums).  Both passes always run (no
// (p,p,q) shortcut), so W_B is formed for every triple.
__global__ __launch_bounds__(256) void noalloc_slots_kernel(NoallocPlan a) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) {
        a.trip_begin[0] = 0;
        a.trip_begin[1] = a.ntrip;
        a.desc->eps_o = a.eps_o;
        a.desc->eps_v = a.eps_v;
        a.desc->o = a.o;
        a.desc->v = a.v;
    }
    if (t >= a.ntrip) return;
    const int o = a.o;
    int r = t, i = 0;
    // (j, k) pairs with i <= j <= k < o, minus (i, i)
    for (;; ++i) {
        const int n = (o - i) * (o - i + 1) / 2 - 1;
        if (r < n) break;
        r -= n;
    }
    int j = i;
    for (;; ++j) {
        const int n = (o - j) - (j == i ? 1 : 0);
        if (r < n) break;
        r -= n;
    }
    const int k = (j == i ? j + 1 : j) + r;
    const int l = t % a.chunk;
    Slot S;
    S.i = i;
    S.j = j;
    S.k = k;
    S.mult = (i == j || j == k) ? 3 : 6;
    S.o = o;
    S.v = a.v;
    S.Kp = a.Kp;
    S.prob = 0;
    S.tiles_m = a.tiles_m;
    S.tiles_n = a.tiles_n;
    S.nbw = a.nbw;
    S.bgroups = a.bgroups;
    S.a_begin = l * a.per_triple_wg;
    S.npass = 2;
    S.e_begin = l * a.norb;
    S.trip_index = t;
    S.part_begin = (int64_t)l * a.norb;
    S.gc = a.gc;
    S.tc = a.tc;
    S.w = a.w + (size_t)l * a.w_bytes;
    S.eps_o = a.eps_o;
    S.eps_v = a.eps_v;
    S.t1 = a.t1;
    S.ovov = a.ovov;
    a.slots[t] = S;
}

// out[0..2] = NaN unless the denominator check passed (flag 0).
__global__ void noalloc_finish_kernel(const double* __restrict__ flag, double* __restrict__ out) {
    if (threadIdx.x < 3 && *flag != 0.0) out[threadIdx.x] = __builtin_nan("");
}

hipError_t launch_noalloc_slots(const NoallocPlan& a, hipStream_t s) {
    const int grid = (a.ntrip + 255) / 256;
    hipLaunchKernelGGL(noalloc_slots_kernel, dim3(grid > 0 ? grid : 1), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_noalloc_finish(const double* flag, double* out, hipStream_t s) {
    hipLaunchKernelGGL(noalloc_finish_kernel, dim3(1), dim3(64), 0, s, flag, out);
    return hipGetLastError();
}

}  // namespace ccsdt
