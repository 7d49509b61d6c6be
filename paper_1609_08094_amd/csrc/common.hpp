// Internal definitions shared by the kernels and the host runtime of the
// (T) library.  Not part of the public ABI (include/ccsdt.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccsdt {

// Packed operand rows are padded with zeros to a multiple of KPAD elements.
constexpr int KPAD = 32;
// W is stored in cubic blocks of SB^3 elements, block-major:
//   W[(A*2nb + B)*2nb + C][a%SB][b%SB][c%SB],  A = a/SB, nb = ceil(v/WB),
// so that every SB^3 sub-block is one contiguous 2 KB (FP32) read.  The
// energy kernel walks orbits of WB^3 blocks (one per workgroup) and stages
// their SB^3 sub-blocks through LDS.  The buffer holds (2 nb)^3 SB^3 =
// nb^3 WB^3 elements per pass.
constexpr int WB = 16;
constexpr int SB = 8;
// Number of XCDs on MI355X; workgroups are dispatched round-robin over them.
constexpr int NXCD = 8;

enum Prec { P_FP64 = 0, P_FP32 = 1, P_BF16X3 = 2 };

// Pointers read out of the slot table are generic to the compiler, which
// would then emit flat memory instructions; flat loads share the wait
// counter of LDS reads and would stall every LDS fragment read on the
// in-flight global prefetch.  Accesses to HBM go through global-space
// pointers instead.
#define GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ const GLOBAL T* gp(const T* p) { return (const GLOBAL T*)p; }
template <class T>
__device__ __forceinline__ GLOBAL T* gpw(T* p) { return (GLOBAL T*)p; }

inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// One occupied triple i<=j<=k of one problem, as seen by every kernel of a
// chunk.  All offsets count workgroups of the flattened launch grids.
struct Slot {
    int i, j, k, mult;        // triple and its multiplicity (6 or 3)
    int o, v, Kp, prob;       // sizes and problem index
    int tiles_m, tiles_n;     // ceil(v / tile edge) along m and n
    int nbw, bgroups;         // W blocks per dimension, ceil(v / WB); batch groups per pass
    int a_begin, npass;       // first contraction workgroup of this slot; passes run (2, or 1
                              // when i = j: then W_B[a][b][c] = W_A[b][a][c] and only W_A is formed)
    int e_begin, trip_index;  // first energy workgroup; index into e_trip
    int64_t part_begin;       // first partial-sum entry (2 doubles each)
    const void* gc;           // packed [p][x][y][Kp] operand of the problem
    const void* tc;           // packed [r][q][z][Kp] operand of the problem
    void* w;                  // W_A then W_B of this slot (2 nbw^3 WB^3 elements)
    const double* eps_o;
    const double* eps_v;
    const double* t1;
    const double* ovov;
};

// ---- launchers (defined in the .hip files) ---------------------------------
// Pack one problem's operands into the precision's layout (see pack.hip).
// With vvvo == nullptr the particle part of G is left to launch_assemble_df.
hipError_t launch_pack(int prec, int o, int v, int Kp, const double* vvvo, const double* t2,
                       const double* ovoo, void* gc, void* tc, hipStream_t s);
// Particle part of G from rows y0 .. y0 + ny - 1 of vvvo held in `chunk`
// (ny * v * v * o doubles, device), for vvvo streamed from host memory.
hipError_t launch_pack_particle_chunk(int prec, int o, int v, int Kp, const double* chunk, int y0, int ny, void* gc,
                                      hipStream_t s);
// Particle part of G from density-fitting factors (see df.hip).
hipError_t launch_assemble_df(int prec, int o, int v, int naux, int Kp, const double* bvv, const double* bvo,
                              void* gc, hipStream_t s);
// Both contraction passes over the slots of a chunk (one launch).  `pace`
// (PACE_BYTES of device memory) holds the per-workgroup progress counts of
// the paced configuration (up to 2048 resident workgroups); the launch clears
// them itself.
constexpr size_t PACE_BYTES = 2048 * 128;
hipError_t launch_contract(int prec, int tile_cfg, const Slot* d_slots, int nslot, int total_wg, unsigned* pace,
                           hipStream_t s);
// Energy partials over the block orbits of every slot.
hipError_t launch_energy(int prec, const Slot* d_slots, int nslot, int total_wg,
                         double* partials, hipStream_t s);
// Per-slot deterministic sum of partials into e_trip[trip_index].
hipError_t launch_slot_reduce(const Slot* d_slots, int nslot, const double* partials, double* e_trip,
                              hipStream_t s);
// Per-problem deterministic sum of e_trip ranges into out[3*p].
hipError_t launch_final_reduce(const int* d_trip_begin, int nprob, const double* e_trip,
                               double* out, hipStream_t s);
// W (any precision, blocked layout) of one slot as dense float64 [a][b][c].
hipError_t launch_widen_w(int prec, const void* w, int v, double* out, hipStream_t s);

// RI-MP2 (see mp2.hip).  Pack c_ov rows into Kq-long packed rows; G_ij for
// the nslot pairs d_pairs[0..nslot) into gbuf (v*v per slot); per-slot
// energies into e_pair[d_pair_index[s]]; the weighted final sum into out[0].
hipError_t launch_mp2_pack(int prec, int o, int v, int naux, int Kq, const double* c_ov, void* cpk, hipStream_t s);
hipError_t launch_mp2_gemm(int prec, const void* cpk, const int2* d_pairs, int nslot, int v, int Kq, void* gbuf,
                           hipStream_t s);
hipError_t launch_mp2_energy(int prec, const void* gbuf, const int2* d_pairs, int nslot, const double* eps_o,
                             const double* eps_v, int v, double* partials, const int* d_pair_index, double* e_pair,
                             hipStream_t s);
hipError_t launch_mp2_final(const double* e_pair, const int2* d_all_pairs, int npairs, double* out, hipStream_t s);

// Orbital energies of one problem, for the denominator sign check.
struct GapDesc {
    const double* eps_o;
    const double* eps_v;
    int o, v;
};
// flag[p] = 0 if every eps_o and eps_v of problem p is finite and
// max(eps_o) < min(eps_v) (all denominators negative), 1 if a value is not
// finite, 2 if the gap is not positive.
hipError_t launch_gap_check(const GapDesc* d_desc, int nprob, double* flag, hipStream_t s);

// ---- allocation-free entry point (noalloc.hip) -----------------------------
// Size of the static device workspace (one copy per device).
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)256 << 20;
// Device address of this device's workspace (`dev` must be current); looked
// up once per device.
hipError_t noalloc_scratch(int dev, void** out);
// Everything the device-side slot builder needs: the whole restricted triple
// list of one problem, cut into chunks of `chunk` triples, each slot with
// room for both passes (per_triple_wg contraction workgroups), norb energy
// workgroups and partials, and w_bytes of W.
struct NoallocPlan {
    Slot* slots;
    int* trip_begin;          // [0, ntrip]
    GapDesc* desc;
    int ntrip, chunk;
    int o, v, Kp;
    int tiles_m, tiles_n, nbw, bgroups;
    int per_triple_wg, norb;
    const void* gc;
    const void* tc;
    char* w;
    size_t w_bytes;
    const double* eps_o;
    const double* eps_v;
    const double* t1;
    const double* ovov;
};
hipError_t launch_noalloc_slots(const NoallocPlan& a, hipStream_t s);
// out[0..2] = NaN when *flag != 0 (failed denominator check).
hipError_t launch_noalloc_finish(const double* flag, double* out, hipStream_t s);

__host__ __device__ inline int64_t w_index(int a, int b, int c, int nb) {
    const int64_t n8 = 2 * (int64_t)nb;
    return ((((int64_t)(a >> 3) * n8 + (b >> 3)) * n8 + (c >> 3)) << 9) + ((a & 7) << 6) + ((b & 7) << 3) + (c & 7);
}

// Contraction tile configurations (workgroup tile BM x BN over the (row, col)
// plane of nbat consecutive batch indices).  0-2: operands loaded straight
// from global memory into MFMA fragments, 2x2 waves.  3-5: operands staged
// through double-buffered LDS, 2x2 waves.  6-7: as 3-4 with operands written
// straight from global memory into LDS (global_load_lds), without a register
// round trip.  8-9: direct-to-LDS staging with two batch indices per
// workgroup sharing the batch-independent operand rows (8: four waves of
// 128x64, 9: eight waves of 64x64).  10-11: as 8-9 with the fragments of the
// next stage read into registers while the current stage's MFMAs run.  12:
// that prefetching kernel with one batch index and 2x2 waves of 64x64 (the
// shape of 6).  13-15: batch-shared deep-ring kernels with NSTAGE - 1 stages
// in flight (13: two batch indices, eight waves of 64x64, three stages;
// 14: one batch index, 2x2 waves of 64x64, four stages; 15: two batch
// indices, four waves of 128x64, three stages).  16: configuration 6 as a
// persistent kernel (two resident workgroups per compute unit walking the
// work items in XCD-synchronous order).  17-18: direct-to-LDS staging with
// larger workgroup tiles, 256x256 (2x2 waves of 128x128) and 256x128 (2x2
// waves of 128x64), one workgroup per compute unit, fewer re-reads of shared
// operand rows per flop.  19-20: eight waves of 64x64 staging one copy of
// the rows for a 256x128 (19) or 128x256 (20) tile, two waves per SIMD.
// 21: 64x128 tiles (2x2 waves of 32x64), direct staging, three workgroups
// per compute unit.  22-23: configurations 6 and 7 with 32x32 MFMA output
// blocks (BF16X3 and FP32; FP64, which has no 32x32 MFMA, runs 6 and 7).
// 24: configuration 16 with the workgroups of each XCD paced to within a few
// K stages of each other, so that operand rows shared across tiles are still
// in the XCD's L2 when the other tiles read them.
struct TileCfg { int bm, bn, lds, nbat; };
constexpr int NTILE_CFG = 27;
constexpr TileCfg TILE_CFGS[NTILE_CFG] = {
    {64, 64, 0, 1},   {128, 64, 0, 1},  {128, 128, 0, 1}, {128, 128, 1, 1}, {128, 256, 1, 1},
    {64, 128, 1, 1},  {128, 128, 2, 1}, {128, 256, 2, 1}, {128, 128, 2, 2}, {128, 128, 2, 2},
    {128, 128, 2, 2}, {128, 128, 2, 2}, {128, 128, 2, 1}, {128, 128, 2, 2}, {128, 128, 2, 1},
    {128, 128, 2, 2}, {128, 128, 2, 1}, {256, 256, 2, 1}, {256, 128, 2, 1},
    {256, 128, 2, 1}, {128, 256, 2, 1}, {64, 128, 2, 1}, {128, 128, 2, 1}, {128, 256, 2, 1},
    {128, 128, 2, 1}, {256, 256, 2, 1}, {128, 128, 2, 1}};
inline int tile_m(int cfg) { return TILE_CFGS[cfg].bm; }
inline int tile_n(int cfg) { return TILE_CFGS[cfg].bn; }
inline int tile_nbat(int cfg) { return TILE_CFGS[cfg].nbat; }

}  // namespace ccsdt
