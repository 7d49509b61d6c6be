// Internal definitions shared by the kernels and the host runtime of the
// (T) library.  Not part of the public ABI (include/ccsdt.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccsdt {

// Packed operand rows are padded with zeros to a multiple of KPAD elements.
constexpr int KPAD = 32;
// Edge of the cubic virtual blocks the energy kernel walks (one block orbit
// per workgroup).
constexpr int EB = 16;
// Number of XCDs on MI355X; workgroups are dispatched round-robin over them.
constexpr int NXCD = 8;

enum Prec { P_FP64 = 0, P_FP32 = 1, P_BF16X3 = 2 };

inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// One occupied triple i<=j<=k of one problem, as seen by every kernel of a
// chunk.  All offsets count workgroups of the flattened launch grids.
struct Slot {
    int i, j, k, mult;        // triple and its multiplicity (6 or 3)
    int o, v, Kp, prob;       // sizes and problem index
    int tiles_m, tiles_n;     // ceil(v / tile edge) along m and n
    int nblk, pad_;           // energy blocks per dimension
    int a_begin, b_begin;     // first workgroup of this slot in pass A / pass B
    int e_begin, trip_index;  // first energy workgroup; index into e_trip
    int64_t part_begin;       // first partial-sum entry (2 doubles each)
    const void* gc;           // packed [p][x][y][Kp] operand of the problem
    const void* tc;           // packed [r][q][z][Kp] operand of the problem
    void* w;                  // W[a][b][c] of this slot (v^3 elements)
    const double* eps_o;
    const double* eps_v;
    const double* t1;
    const double* ovov;
};

// ---- launchers (defined in the .hip files) ---------------------------------
// Pack one problem's operands into the precision's layout (see pack.hip).
hipError_t launch_pack(int prec, int o, int v, int Kp, const double* vvvo, const double* t2,
                       const double* ovoo, void* gc, void* tc, hipStream_t s);
// Contraction pass A (pass=0) or B (pass=1) over the slots of a chunk.
hipError_t launch_contract(int prec, int tile_cfg, int pass, const Slot* d_slots, int nslot,
                           int total_wg, hipStream_t s);
// Energy partials over the block orbits of every slot.
hipError_t launch_energy(int prec, const Slot* d_slots, int nslot, int total_wg,
                         double* partials, hipStream_t s);
// Per-slot deterministic sum of partials into e_trip[trip_index].
hipError_t launch_slot_reduce(const Slot* d_slots, int nslot, int norb_max_unused,
                              const double* partials, double* e_trip, hipStream_t s);
// Per-problem deterministic sum of e_trip ranges into out[3*p].
hipError_t launch_final_reduce(const int* d_trip_begin, int nprob, const double* e_trip,
                               double* out, hipStream_t s);
// W (any precision) of one slot widened to float64.
hipError_t launch_widen_w(int prec, const void* w, int64_t n, double* out, hipStream_t s);

// Contraction tile configurations (workgroup tile BM x BN over the (row, col)
// plane of one batch index).  0-2: operands loaded straight from global
// memory into MFMA fragments, 2x2 waves.  3-5: operands staged through
// double-buffered LDS, 2x2 waves.
struct TileCfg { int bm, bn, lds; };
constexpr int NTILE_CFG = 6;
constexpr TileCfg TILE_CFGS[NTILE_CFG] = {
    {64, 64, 0}, {128, 64, 0}, {128, 128, 0}, {128, 128, 1}, {128, 256, 1}, {64, 128, 1}};
inline int tile_m(int cfg) { return TILE_CFGS[cfg].bm; }
inline int tile_n(int cfg) { return TILE_CFGS[cfg].bn; }

}  // namespace ccsdt
