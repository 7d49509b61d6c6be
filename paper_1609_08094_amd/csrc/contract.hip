// Connected triples quantity W (paper Sec. 2.2, eq. analytical_triples_ampl
// bracket, symmetrized by eq. symm_operator) on gfx950 MFMA.
//
// With the packed rows of pack.hip, X^xyz_pqr = <G[p][x][y], T[r][q][z]> and
//   W^abc_ijk = X^abc_ijk + X^acb_ikj + X^bac_jik + X^bca_jki + X^cab_kij + X^cba_kji.
// Each term is a batched NT product: one of the two G indices is a batch
// index, the other the MFMA row, and the T index the MFMA column.  Two
// orientations cover all six terms with three segments each:
//
//  pass A, batch a, tile (b,c):  W_A = <G_i[a][b],T_kj[c]> + <T_jk[b],G_i[a][c]> + <T_ji[b],G_k[c][a]>
//  pass B, batch b, tile (a,c):  W_B = <G_j[b][a],T_ki[c]> + <T_ik[a],G_j[b][c]> + <T_ij[a],G_k[c][b]>
//
// W = W_A + W_B.  The two passes are independent (one launch covers both),
// each writes its own buffer once, and the energy kernel adds the two when
// it stages W.  For a triple taken as (p, p, q), W_B[a][b][c] = W_A[b][a][c]:
// only pass A runs (Slot::npass = 1) and the energy kernel reads W_A twice.
// The three terms of a pass run as one K loop over three segments of length
// Kp.  W_A and W_B are FP64 for the FP64 path and FP32 otherwise, in the
// SB^3-blocked layout of common.hpp.
//
// MFMA shapes (all with a 16x16 output block; lane l holds four rows of
// column l%16: rows l/16 + 4r for the FP64 instruction, 4(l/16) + r for the
// FP32-accumulating ones, r < 4):
//   FP64    v_mfma_f64_16x16x4_f64     4 steps per 16-element chunk
//   FP32    v_mfma_f32_16x16x4_f32     4 steps per 16-element chunk
//   BF16X3  v_mfma_f32_16x16x32_bf16   hi*hi + hi*lo + lo*hi per 32-element chunk
// Within a chunk each lane owns a contiguous run of k; A and B use the same
// assignment, so the dot product covers every k exactly once.
#include "common.hpp"
#include "mfma.hpp"

namespace ccsdt {

// Row indices (in packed rows) of the operands of one segment.
struct SegRows {
    int64_t a0, aB, aM;  // A row = a0 + beta*aB + m*aM   (from G if aG else T)
    int64_t b0, bB, bN;  // B row = b0 + beta*bB + n*bN
    bool aG, bG;
};

__device__ __forceinline__ SegRows segment(int pass, int s, int i, int j, int k, int o, int v) {
    const int64_t V = v, V2 = (int64_t)v * v;
    auto trow = [&](int r, int q) { return ((int64_t)r * o + q) * V; };  // first row of T[r][q]
    SegRows g{};
    if (pass == 0) {  // batch a, row b, col c
        switch (s) {
            case 0: g = {i * V2, V, 1, trow(k, j), 0, 1, true, false}; break;   // G_i[a][b] . T_kj[c]
            case 1: g = {trow(j, k), 0, 1, i * V2, V, 1, false, true}; break;   // T_jk[b] . G_i[a][c]
            default: g = {trow(j, i), 0, 1, k * V2, 1, V, false, true}; break;  // T_ji[b] . G_k[c][a]
        }
    } else {  // batch b, row a, col c
        switch (s) {
            case 0: g = {j * V2, V, 1, trow(k, i), 0, 1, true, false}; break;   // G_j[b][a] . T_ki[c]
            case 1: g = {trow(i, k), 0, 1, j * V2, V, 1, false, true}; break;   // T_ik[a] . G_j[b][c]
            default: g = {trow(i, j), 0, 1, k * V2, 1, V, false, true}; break;  // T_ij[a] . G_k[c][b]
        }
    }
    return g;
}

constexpr int NSEG = 3;  // segments per pass

// Store a wave's accumulator blocks into W_A (pass A) or W_B (pass B).
template <class P, int WM, int WN>
__device__ __forceinline__ void store_tile(const Slot* S, int pass, int beta, int m0, int n0, int vm, int vn,
                                           int lane, typename P::Acc (&acc)[WM][WN]) {
    using Wt = typename P::W;
    const int v = S->v;
    const int nb = S->nbw;
    GLOBAL Wt* out = gpw(static_cast<Wt*>(S->w)) + (pass ? (int64_t)nb * nb * nb * (WB * WB * WB) : 0);
#pragma unroll
    for (int a = 0; a < WM; ++a) {
#pragma unroll
        for (int b = 0; b < WN; ++b) {
            if (a < vm && b < vn) {
                const int n = n0 + b * P::BS + (lane % P::BS);
#pragma unroll
                for (int r = 0; r < P::NACC; ++r) {
                    const int m = m0 + a * P::BS + P::out_row(lane, r);
                    if (m < v && n < v) {
                        // pass A: (a,b,c) = (beta, m, n); pass B: (m, beta, n)
                        const int64_t idx = pass ? w_index(m, beta, n, nb) : w_index(beta, m, n, nb);
                        out[idx] = (Wt)acc[a][b][r];
                    }
                }
            }
        }
    }
}

// Locate this workgroup's slot, pass, batch group and tile.  Within a slot
// the pass-A workgroups come first, then the pass-B ones.  A batch group is
// one batch index, or nbat consecutive ones for the batch-shared kernel.
__device__ __forceinline__ const Slot* find_slot(const Slot* slots, int nslot, int bid, int& pass, int& beta,
                                                 int& tmi, int& tni) {
    int lo = 0, hi = nslot - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (slots[mid].a_begin <= bid) lo = mid; else hi = mid - 1;
    }
    const Slot* S = slots + lo;
    const int tn = S->tiles_n;
    const int per_beta = S->tiles_m * tn;
    int local = bid - S->a_begin;
    const int per_pass = S->bgroups * per_beta;
    pass = local >= per_pass;
    local -= pass * per_pass;
    beta = local / per_beta;
    local -= beta * per_beta;
    tmi = local / tn;
    tni = local - tmi * tn;
    return S;
}

template <class P, int WM, int WN>
__global__ __launch_bounds__(256) void contract_kernel(const Slot* __restrict__ slots, int nslot, int total) {
    using E = typename P::E;
    using Wt = typename P::W;
    const int bid = xcd_remap(blockIdx.x, total);
    int pass, beta, tmi, tni;
    const Slot* S = find_slot(slots, nslot, bid, pass, beta, tmi, tni);
    const int v = S->v, o = S->o, Kp = S->Kp;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m0 = tmi * (32 * WM) + (wave >> 1) * (16 * WM);
    const int n0 = tni * (32 * WN) + (wave & 1) * (16 * WN);
    const int vm = min(WM, (v - m0 + 15) / 16);  // valid 16-row blocks of this wave
    const int vn = min(WN, (v - n0 + 15) / 16);
    if (m0 >= v || n0 >= v) return;  // no barrier in this kernel: idle waves may leave

    typename P::Acc acc[WM][WN];
#pragma unroll
    for (int a = 0; a < WM; ++a)
#pragma unroll
        for (int b = 0; b < WN; ++b) acc[a][b] = typename P::Acc{};

    const int64_t rl = (int64_t)Kp * P::UNITS;
    const E* G = static_cast<const E*>(S->gc);
    const E* T = static_cast<const E*>(S->tc);
    const int nseg = NSEG;
    const int nch = Kp / P::KCH;
    for (int s = 0; s < nseg; ++s) {
        const SegRows g = segment(pass, s, S->i, S->j, S->k, o, v);
        const E* pa[WM];
        const E* pb[WN];
#pragma unroll
        for (int a = 0; a < WM; ++a) {
            const int m = min(m0 + a * 16 + (lane & 15), v - 1);
            pa[a] = (g.aG ? G : T) + (g.a0 + beta * g.aB + m * g.aM) * rl;
        }
#pragma unroll
        for (int b = 0; b < WN; ++b) {
            const int n = min(n0 + b * 16 + (lane & 15), v - 1);
            pb[b] = (g.bG ? G : T) + (g.b0 + beta * g.bB + n * g.bN) * rl;
        }
        typename P::Frag fa[WM], fb[WN];
#pragma unroll
        for (int a = 0; a < WM; ++a) if (a < vm) P::load(fa[a], pa[a], 0, lane);
#pragma unroll
        for (int b = 0; b < WN; ++b) if (b < vn) P::load(fb[b], pb[b], 0, lane);
        for (int c = 0; c < nch; ++c) {
            typename P::Frag na[WM], nb[WN];
            if (c + 1 < nch) {
#pragma unroll
                for (int a = 0; a < WM; ++a) if (a < vm) P::load(na[a], pa[a], c + 1, lane);
#pragma unroll
                for (int b = 0; b < WN; ++b) if (b < vn) P::load(nb[b], pb[b], c + 1, lane);
            }
            mma_blocks<P, WM, WN, false>(acc, fa, fb, vm, vn);
#pragma unroll
            for (int a = 0; a < WM; ++a) fa[a] = na[a];
#pragma unroll
            for (int b = 0; b < WN; ++b) fb[b] = nb[b];
        }
    }

    store_tile<P, WM, WN>(S, pass, beta, m0, n0, vm, vn, lane, acc);
}

// LDS-staged variant.  Each workgroup (2x2 waves, wave tile WTM x WTN)
// streams its BM + BN operand rows through two LDS stages of ROWB bytes per
// row, one barrier per stage; the next stage is fetched into registers while
// the current one feeds the MFMAs.  A stage row holds 128 bytes of one
// operand row as eight 16-byte chunks.  For BF16X3 (hi/lo of k-group g) and
// FP64 (two halves of lane group g's 32 bytes) the first half goes to chunk
// g and the second to chunk 4 + g; FP32 keeps the global order (sub-step s,
// group g at chunk 4 s + g).  The chunk index is then XOR-ed with
// lds_swz(row).  With this layout, measured with the LDS bank-conflict
// counter over all XOR swizzles of this family, the fragment reads (16 rows
// x 4 lane groups) and the staging writes (8 rows x 8 chunks per wave) are
// free of bank conflicts.

template <int WTM, int WTN, int ROWB, int WGM = 2, int WGN = 2>
constexpr int lds_tile_bytes() { return 2 * (WGM * WTM + WGN * WTN) * ROWB; }

// Bounded pacing of the workgroups of one XCD (contract_lds_paced_kernel).
// Every PACE_PERIOD K stages a workgroup publishes how many stages it has
// completed (a store to its own 128-byte line: no shared read-modify-write)
// and then waits until every workgroup of its XCD has published at least
// `lag` stages fewer, or has completed all of its work.  Workgroups reading
// the same operand rows thus stay within a few stages of each other and find
// the rows in the XCD's L2.  The wait only orders timing: a spin that exceeds
// its bound switches pacing off for the workgroup, and no result depends on it.
constexpr int PACE_PERIOD = 4;
constexpr int PACE_SPIN_LIMIT = 4000;   // about 0.3 ms of s_sleep at the sustained clock
constexpr int PACE_STRIDE = 32;         // unsigned ints per published count (128 bytes)

struct Pacer {
    unsigned* mine;        // this workgroup's published count
    const unsigned* xcd;   // the XCD's counts, workgroup w at xcd[w * PACE_STRIDE]
    int done;              // stages completed by this workgroup
    int S;                 // stages per work item
    int per, rem, tlo;     // workgroups of the XCD; item counts tlo + 1 (first rem) or tlo
    int lag;
    bool on;
};

__device__ __forceinline__ void pace_step(Pacer& pc) {
    ++pc.done;
    if (!pc.on || pc.done % PACE_PERIOD != 0 || threadIdx.x >= 64) return;
    const int lane = threadIdx.x;
    if (lane == 0) __hip_atomic_store(pc.mine, (unsigned)pc.done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int c = pc.done - pc.lag;
    if (c <= 0) return;
    for (int spins = 0;; ++spins) {
        bool ok = true;
        for (int w = lane; w < pc.per; w += 64) {
            const int need = min(c, (pc.tlo + (w < pc.rem ? 1 : 0)) * pc.S);
            ok = ok && (int)__hip_atomic_load(pc.xcd + w * PACE_STRIDE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need;
        }
        if (__all(ok)) return;
        if (spins >= PACE_SPIN_LIMIT) {
            pc.on = false;
            return;
        }
        __builtin_amdgcn_s_sleep(2);
    }
}

// One LDS stage of a full wave tile (every block valid) with the next
// stage's NL global_load_lds requests spread over the MFMA stream, one after
// every MB * NB / NL blocks, instead of issued together before it: a burst
// of requests fills the vector-memory queue and stalls the wave's MFMA issue
// until it drains.  The fences keep the compiler from gathering the
// requests (and their address arithmetic) back into one place.
template <class P, int MB, int NB, int RS, int NL, class LD>
__device__ __forceinline__ void lds_stage_spread(typename P::Acc (&acc)[MB][NB], const char* As, const char* Bs, int g,
                                                 int sw, LD&& issue) {
    static_assert(P::NSUB == 1 && (MB * NB) % NL == 0, "one sub-step, loads spread evenly");
    constexpr int PER = MB * NB / NL;
    typename P::Frag fa[MB], fb[NB];
#pragma unroll
    for (int a = 0; a < MB; ++a) P::load_lds(fa[a], As + a * P::BS * RS, g, 0, sw);
#pragma unroll
    for (int b = 0; b < NB; ++b) P::load_lds(fb[b], Bs + b * P::BS * RS, g, 0, sw);
#pragma unroll
    for (int q = 0; q < MB * NB; ++q) {
        P::mma(acc[q / NB][q % NB], fa[q / NB], fb[q % NB]);
        if ((q + 1) % PER == 0) {
            __builtin_amdgcn_sched_barrier(0);
            issue((q + 1) / PER - 1);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

template <class P, int WTM, int WTN, int ROWB, bool DIRECT, int WGM = 2, int WGN = 2, bool PACE = false,
          bool SPREAD = false>
__device__ __forceinline__ void lds_tile(const Slot* __restrict__ slots, int nslot, int bid, char* lds,
                                         Pacer* pc = nullptr) {
    using E = typename P::E;
    constexpr int NT = 64 * WGM * WGN;   // WGM x WGN waves of WTM x WTN
    constexpr int BM = WGM * WTM, BN = WGN * WTN;
    constexpr int RS = ROWB;
    constexpr int ROWS = BM + BN;
    constexpr int TPR = ROWB / 16;
    constexpr int RPP = NT / TPR;
    constexpr int NP = ROWS / RPP;
    static_assert(ROWS % RPP == 0, "rows must split evenly over the threads");
    constexpr int BS = P::BS;
    constexpr int MB = WTM / BS, NB = WTN / BS;
    static_assert(ROWB == 128, "stage rows are eight 16-byte chunks");

    int pass, beta, tmi, tni;
    const Slot* S = find_slot(slots, nslot, bid, pass, beta, tmi, tni);
    const int v = S->v, o = S->o, Kp = S->Kp;
    const int mt0 = tmi * BM, nt0 = tni * BN;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wm = wave / WGN, wn = wave % WGN;
    const int m0 = mt0 + wm * WTM, n0 = nt0 + wn * WTN;
    const int vm = max(0, min(MB, (v - m0 + BS - 1) / BS));
    const int vn = max(0, min(NB, (v - n0 + BS - 1) / BS));

    const int64_t rowbytes = (int64_t)Kp * P::UNITS * sizeof(E);
    const int csteps = (int)(rowbytes / ROWB);
    const int nsteps = NSEG * csteps;
    const char* G = static_cast<const char*>(S->gc);
    const char* T = static_cast<const char*>(S->tc);
    const int lrow = threadIdx.x / TPR, lcol = (threadIdx.x % TPR) * 16;
    // LDS chunk of this thread's staging chunk (RPP keeps the swizzle bits)
    static_assert(RPP % (BS == 32 ? 32 : 8) == 0, "staging rows must keep the swizzle bits");
    const int gch = lcol >> 4;
    const int lch = P::SPLIT ? ((gch & 1) * 4 + (gch >> 1)) : gch;
    const int lcol_sw = (lch ^ lds_swz_bs<BS>(lrow)) * 16;
    // Direct staging (global_load_lds): lane l of a wave's p-th load writes the
    // 16 bytes at LDS row lrow + p RPP, chunk l % 8; it fetches the global chunk
    // that belongs there under the same permutation and swizzle.
    const int pch = (lane & 7) ^ lds_swz_bs<BS>(lrow);
    const int src_col = (P::SPLIT ? (((pch & 3) << 1) | (pch >> 2)) : pch) * 16;
    const int wave_row0 = (threadIdx.x >> 6) * (64 / TPR);

    // Byte offset of each of this thread's rows for the current segment,
    // relative to the segment's A or B operand array.
    int64_t roff[NP];
    u32x4 st[NP];
    typename P::Acc acc[MB][NB];
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = typename P::Acc{};

#define CCSDT_SET_PTRS(sg)                                                          \
    {                                                                               \
        const SegRows g_ = segment(pass, (sg), S->i, S->j, S->k, o, v);             \
        const int col_ = DIRECT ? src_col : lcol;                                   \
        baseA = g_.aG ? G : T;                                                      \
        baseB = g_.bG ? G : T;                                                      \
        _Pragma("unroll") for (int p = 0; p < NP; ++p) {                            \
            const int r = lrow + p * RPP;                                           \
            if (r < BM) {                                                           \
                const int m = min(mt0 + r, v - 1);                                  \
                roff[p] = (g_.a0 + beta * g_.aB + m * g_.aM) * rowbytes + col_;     \
            } else {                                                                \
                const int n = min(nt0 + r - BM, v - 1);                             \
                roff[p] = (g_.b0 + beta * g_.bB + n * g_.bN) * rowbytes + col_;     \
            }                                                                       \
        }                                                                           \
    }
#define CCSDT_GLOAD(c)                                                                         \
    _Pragma("unroll") for (int p = 0; p < NP; ++p) {                                           \
        const char* src = ((lrow + p * RPP) < BM ? baseA : baseB) + roff[p] + (int64_t)(c) * ROWB; \
        st[p] = *reinterpret_cast<const GLOBAL u32x4*>(gp(src));                               \
    }
#define CCSDT_GLOAD_DIRECT(c, buf)                                                             \
    _Pragma("unroll") for (int p = 0; p < NP; ++p) {                                           \
        const char* src = ((lrow + p * RPP) < BM ? baseA : baseB) + roff[p] + (int64_t)(c) * ROWB; \
        char* dst = lds + (buf) * (ROWS * RS) + (wave_row0 + p * RPP) * RS;                    \
        __builtin_amdgcn_global_load_lds((const GLOBAL void*)gp(src),                          \
                                         (__attribute__((address_space(3))) void*)dst, 16, 0, 0); \
    }
#define CCSDT_LSTORE(buf)                                                                      \
    {                                                                                          \
        char* dst_ = lds + (buf) * (ROWS * RS) + lrow * RS + lcol_sw;                          \
        _Pragma("unroll") for (int p = 0; p < NP; ++p)                                         \
            *reinterpret_cast<u32x4*>(dst_ + p * RPP * RS) = st[p];                            \
    }

    const char* baseA = G;
    const char* baseB = T;
    CCSDT_SET_PTRS(0);
    if constexpr (DIRECT) {
        CCSDT_GLOAD_DIRECT(0, 0);
    } else {
        CCSDT_GLOAD(0);
        CCSDT_LSTORE(0);
    }
    lds_dma_barrier();
    const bool active = vm > 0 && vn > 0;
    int sg_next = 0, c_next = 0;
    for (int step = 0; step < nsteps; ++step) {
        const int buf = step & 1;
        // Prefetch the next stage (the last step re-reads its own chunk, so the
        // loads and the LDS store below are unconditional: a branch around them
        // lets the compiler sink the loads past the MFMAs and expose their
        // latency on every stage).
        if (step + 1 < nsteps && ++c_next == csteps) {
            c_next = 0;
            ++sg_next;
            CCSDT_SET_PTRS(sg_next);
        }
        if constexpr (SPREAD && DIRECT && P::NSUB == 1) {
            if (vm == MB && vn == NB) {
                const char* As = lds + buf * (ROWS * RS) + (wm * WTM + (lane % BS)) * RS;
                const char* Bs = lds + buf * (ROWS * RS) + (BM + wn * WTN + (lane % BS)) * RS;
                const int cn = c_next;
                lds_stage_spread<P, MB, NB, RS, NP>(acc, As, Bs, lane / BS, lds_swz_bs<BS>(lane % BS), [&](int p) {
                    const char* src = ((lrow + p * RPP) < BM ? baseA : baseB) + roff[p] + (int64_t)cn * ROWB;
                    char* dst = lds + (buf ^ 1) * (ROWS * RS) + (wave_row0 + p * RPP) * RS;
                    __builtin_amdgcn_global_load_lds((const GLOBAL void*)gp(src),
                                                     (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
                });
                lds_dma_barrier();
                continue;
            }
        }
        if constexpr (DIRECT) {
            CCSDT_GLOAD_DIRECT(c_next, buf ^ 1);
        } else {
            CCSDT_GLOAD(c_next);
        }
        __builtin_amdgcn_sched_barrier(0);
        if (active) {
            const char* As = lds + buf * (ROWS * RS) + (wm * WTM + (lane % BS)) * RS;
            const char* Bs = lds + buf * (ROWS * RS) + (BM + wn * WTN + (lane % BS)) * RS;
            const int g = lane / BS;
            const int sw = lds_swz_bs<BS>(lane % BS);
            if (vm == MB && vn == NB)
                lds_stage<P, MB, NB, RS, true>(acc, As, Bs, g, sw, vm, vn);
            else
                lds_stage<P, MB, NB, RS, false>(acc, As, Bs, g, sw, vm, vn);
        }
        if constexpr (!DIRECT) CCSDT_LSTORE(buf ^ 1);
        if constexpr (PACE) pace_step(*pc);
        lds_dma_barrier();
    }
#undef CCSDT_SET_PTRS
#undef CCSDT_GLOAD
#undef CCSDT_GLOAD_DIRECT
#undef CCSDT_LSTORE
    if (active) store_tile<P, MB, NB>(S, pass, beta, m0, n0, vm, vn, lane, acc);
}

template <class P, int WTM, int WTN, int ROWB, int MINB, bool DIRECT>
__global__ __launch_bounds__(256, MINB) void contract_lds_kernel(const Slot* __restrict__ slots, int nslot,
                                                                  int total) {
    __shared__ __attribute__((aligned(16))) char lds[lds_tile_bytes<WTM, WTN, ROWB>()];
    lds_tile<P, WTM, WTN, ROWB, DIRECT>(slots, nslot, xcd_remap(blockIdx.x, total), lds);
}

// Configuration 6 with the next stage's requests spread over the MFMAs of
// the current one (lds_stage_spread) in full tiles.
template <class P>
__global__ __launch_bounds__(256, 2) void contract_lds_spread_kernel(const Slot* __restrict__ slots, int nslot,
                                                                      int total) {
    __shared__ __attribute__((aligned(16))) char lds[lds_tile_bytes<64, 64, 128>()];
    lds_tile<P, 64, 64, 128, true, 2, 2, false, true>(slots, nslot, xcd_remap(blockIdx.x, total), lds);
}

// Workgroups of WGM x WGN waves (more than 2 x 2): one staged copy of the
// shared rows serves more waves, so the rows of G of one batch index are
// read by fewer workgroups.
template <class P, int WTM, int WTN, int WGM, int WGN, int MINB>
__global__ __launch_bounds__(64 * WGM * WGN, MINB) void contract_lds_wide_kernel(const Slot* __restrict__ slots,
                                                                                  int nslot, int total) {
    __shared__ __attribute__((aligned(16))) char lds[lds_tile_bytes<WTM, WTN, 128, WGM, WGN>()];
    lds_tile<P, WTM, WTN, 128, true, WGM, WGN>(slots, nslot, xcd_remap(blockIdx.x, total), lds);
}

// Persistent form: gridDim.x (a multiple of NXCD) resident workgroups walk the
// work items.  Workgroup b runs on XCD b % NXCD and takes, within that XCD's
// contiguous range of logical items, every (gridDim.x / NXCD)-th item from
// position b / NXCD.  All items cost about the same, so the workgroups of an
// XCD start their t-th items together and read shared operand rows (the G
// rows of a batch index, the T rows of a segment) while they are still in
// that XCD's L2; one-item-per-workgroup launches drift apart and re-fetch them.
template <class P, int WTM, int WTN, int ROWB, int MINB, bool DIRECT>
__global__ __launch_bounds__(256, MINB) void contract_lds_persist_kernel(const Slot* __restrict__ slots, int nslot,
                                                                          int total) {
    __shared__ __attribute__((aligned(16))) char lds[lds_tile_bytes<WTM, WTN, ROWB>()];
    const int x = blockIdx.x % NXCD, lw = blockIdx.x / NXCD, per_xcd = gridDim.x / NXCD;
    const int q = total / NXCD, r = total % NXCD;
    const int begin = x * q + min(x, r), end = begin + q + (x < r ? 1 : 0);
    for (int id = begin + lw; id < end; id += per_xcd) lds_tile<P, WTM, WTN, ROWB, DIRECT>(slots, nslot, id, lds);
}

// Paced persistent form: the walk of contract_lds_persist_kernel with the
// workgroups of each XCD held within `lag` K stages of each other (Pacer).
// Pacing needs equal stage counts for all items (one Kp across the slots);
// otherwise it stays off.  `pace` holds one count per workgroup at a
// 128-byte stride, zero at launch.
template <class P, int WTM, int WTN, int MINB>
__global__ __launch_bounds__(256, MINB) void contract_lds_paced_kernel(const Slot* __restrict__ slots, int nslot,
                                                                        int total, unsigned* pace, int lag) {
    __shared__ __attribute__((aligned(16))) char lds[lds_tile_bytes<WTM, WTN, 128>()];
    const int x = blockIdx.x % NXCD, lw = blockIdx.x / NXCD, per_xcd = gridDim.x / NXCD;
    const int q = total / NXCD, r = total % NXCD;
    const int begin = x * q + min(x, r), end = begin + q + (x < r ? 1 : 0);
    const int Kp0 = slots[0].Kp;
    bool uniform = true;
    for (int s = 1; s < nslot; ++s) uniform = uniform && slots[s].Kp == Kp0;
    Pacer pc;
    pc.xcd = pace + (int64_t)x * per_xcd * PACE_STRIDE;
    pc.mine = pace + ((int64_t)x * per_xcd + lw) * PACE_STRIDE;
    pc.done = 0;
    pc.S = NSEG * (int)((int64_t)Kp0 * P::UNITS * sizeof(typename P::E) / 128);
    pc.per = per_xcd;
    pc.tlo = (end - begin) / per_xcd;
    pc.rem = (end - begin) % per_xcd;
    pc.lag = lag;
    pc.on = uniform && lag > 0;
    for (int id = begin + lw; id < end; id += per_xcd)
        lds_tile<P, WTM, WTN, 128, true, 2, 2, true>(slots, nslot, id, lds, &pc);
}

__global__ void pace_clear_kernel(unsigned* pace, int n) {
    for (int w = threadIdx.x; w < n; w += blockDim.x) pace[w * PACE_STRIDE] = 0u;
}

// Batch-shared variant.  In every segment exactly one operand depends on the
// batch index (rows of G) and the other does not (rows of T), so a
// workgroup that takes NBAT consecutive batch indices stages the shared
// operand once for all of them: per stage, 128 shared rows followed by 128
// batch-dependent rows per batch index, in the chunk order and swizzle of
// contract_lds_kernel, written straight from global memory (global_load_lds).
// Wave w computes the (WTM x WTN) sub-tile w % WPB of the 128 x 128 tile of
// batch index beta0 + w / WPB.
template <class P, int WTM, int WTN, int NBAT, int MINB>
__global__ __launch_bounds__(NBAT * (128 / WTM) * (128 / WTN) * 64, MINB) void contract_bat_kernel(
    const Slot* __restrict__ slots, int nslot, int total) {
    constexpr int BM = 128, BN = 128;
    constexpr int WPB = (BM / WTM) * (BN / WTN);
    constexpr int NT = 64 * NBAT * WPB;
    constexpr int RS = 128;
    constexpr int ROWS = 128 * (1 + NBAT);
    constexpr int TPR = RS / 16;
    constexpr int RPP = NT / TPR;
    constexpr int NP = ROWS / RPP;
    static_assert(ROWS % RPP == 0, "rows must split evenly over the threads");
    static_assert(RPP % 8 == 0, "staging rows must keep the swizzle bits");
    constexpr int MB = WTM / 16, NB = WTN / 16;
    __shared__ __attribute__((aligned(16))) char lds[2 * ROWS * RS];

    const int bid = xcd_remap(blockIdx.x, total);
    int pass, bgrp, tmi, tni;
    const Slot* S = find_slot(slots, nslot, bid, pass, bgrp, tmi, tni);
    const int v = S->v, o = S->o, Kp = S->Kp;
    const int mt0 = tmi * BM, nt0 = tni * BN;
    const int beta0 = bgrp * NBAT;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wb = wave / WPB, wsub = wave % WPB;
    const int wm = wsub / (BN / WTN), wn = wsub % (BN / WTN);
    const int beta = beta0 + wb;
    const int m0 = mt0 + wm * WTM, n0 = nt0 + wn * WTN;
    const int vm = beta < v ? max(0, min(MB, (v - m0 + 15) / 16)) : 0;
    const int vn = max(0, min(NB, (v - n0 + 15) / 16));

    const int64_t rowbytes = (int64_t)Kp * P::UNITS * sizeof(typename P::E);
    const int csteps = (int)(rowbytes / RS);
    const int nsteps = NSEG * csteps;
    const char* G = static_cast<const char*>(S->gc);
    const char* T = static_cast<const char*>(S->tc);
    const int lrow = threadIdx.x / TPR;
    const int pch = (lane & 7) ^ lds_swz(lrow);
    const int src_col = (P::SPLIT ? (((pch & 3) << 1) | (pch >> 2)) : pch) * 16;
    const int wave_row0 = wave * (64 / TPR);

    // Source of each of this thread's stage rows for the current segment.
    const char* rbase[NP];
    typename P::Acc acc[MB][NB];
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = typename P::Acc{};

    bool depA = true;  // segment's batch-dependent operand is A (rows) rather than B (cols)
    auto set_rows = [&](int sg) {
        const SegRows g = segment(pass, sg, S->i, S->j, S->k, o, v);
        depA = g.aB != 0;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int r = lrow + p * RPP;
            int64_t row;
            if (r < 128) {  // shared operand
                row = depA ? g.b0 + (int64_t)min(nt0 + r, v - 1) * g.bN : g.a0 + (int64_t)min(mt0 + r, v - 1) * g.aM;
            } else {
                const int bb = min(beta0 + (r - 128) / 128, v - 1), rr = (r - 128) % 128;
                row = depA ? g.a0 + bb * g.aB + (int64_t)min(mt0 + rr, v - 1) * g.aM
                           : g.b0 + bb * g.bB + (int64_t)min(nt0 + rr, v - 1) * g.bN;
            }
            const bool fromG = (r < 128) == !depA ? g.aG : g.bG;
            rbase[p] = (fromG ? G : T) + row * rowbytes + src_col;
        }
    };
    auto gload = [&](int c, int buf) {
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            char* dst = lds + buf * (ROWS * RS) + (wave_row0 + p * RPP) * RS;
            __builtin_amdgcn_global_load_lds((const GLOBAL void*)gp(rbase[p] + (int64_t)c * RS),
                                             (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
        }
    };

    set_rows(0);
    gload(0, 0);
    lds_dma_barrier();
    const bool active = vm > 0 && vn > 0;
    bool dep_cur = depA;
    int sg_next = 0, c_next = 0;
    for (int step = 0; step < nsteps; ++step) {
        const int buf = step & 1;
        const bool dep_this = dep_cur;
        if (step + 1 < nsteps && ++c_next == csteps) {
            c_next = 0;
            ++sg_next;
            set_rows(sg_next);
        }
        gload(c_next, buf ^ 1);
        dep_cur = depA;
        __builtin_amdgcn_sched_barrier(0);
        if (active) {
            const char* st = lds + buf * (ROWS * RS);
            const int arow = dep_this ? 128 * (1 + wb) + wm * WTM : wm * WTM;
            const int brow = dep_this ? wn * WTN : 128 * (1 + wb) + wn * WTN;
            const char* As = st + (arow + (lane & 15)) * RS;
            const char* Bs = st + (brow + (lane & 15)) * RS;
            const int g = lane >> 4;
            const int sw = lds_swz(lane & 15);
            if (vm == MB && vn == NB)
                lds_stage<P, MB, NB, RS, true>(acc, As, Bs, g, sw, vm, vn);
            else
                lds_stage<P, MB, NB, RS, false>(acc, As, Bs, g, sw, vm, vn);
        }
        lds_dma_barrier();
    }
    if (active) store_tile<P, MB, NB>(S, pass, beta, m0, n0, vm, vn, lane, acc);
}

// Fragments of one LDS stage for a wave's MB x NB blocks.
template <class P, int MB, int NB>
struct StageFrags {
    typename P::Frag a[P::NSUB][MB], b[P::NSUB][NB];
};

template <class P, int MB, int NB, int RS>
__device__ __forceinline__ void read_frags(StageFrags<P, MB, NB>& f, const char* As, const char* Bs, int g, int sw) {
#pragma unroll
    for (int sub = 0; sub < P::NSUB; ++sub) {
#pragma unroll
        for (int b = 0; b < NB; ++b) P::load_lds(f.b[sub][b], Bs + b * 16 * RS, g, sub, sw);
#pragma unroll
        for (int a = 0; a < MB; ++a) P::load_lds(f.a[sub][a], As + a * 16 * RS, g, sub, sw);
    }
}

// MFMAs of one stage from registers (cur) while the fragments of the next
// stage are read from LDS into nxt; the reads are spread over the MFMA
// stream (one fragment read per row of blocks) so that LDS latency hides
// behind matrix work.
template <class P, int MB, int NB, int RS, bool FULL>
__device__ __forceinline__ void mma_stage_overlap(typename P::Acc (&acc)[MB][NB], const StageFrags<P, MB, NB>& cur,
                                                  StageFrags<P, MB, NB>& nxt, const char* As, const char* Bs, int g,
                                                  int sw, int vm, int vn) {
#pragma unroll
    for (int sub = 0; sub < P::NSUB; ++sub) {
#pragma unroll
        for (int b = 0; b < NB; ++b) P::load_lds(nxt.b[sub][b], Bs + b * 16 * RS, g, sub, sw);
#pragma unroll
        for (int a = 0; a < MB; ++a) {
            P::load_lds(nxt.a[sub][a], As + a * 16 * RS, g, sub, sw);
#pragma unroll
            for (int b = 0; b < NB; ++b)
                if (FULL || (a < vm && b < vn)) P::mma(acc[a][b], cur.a[sub][a], cur.b[sub][b]);
        }
    }
}

// Batch-shared kernel with register-prefetched fragments.  Stage s of the K
// loop lives in LDS buffer s % 2; it is requested (global_load_lds) two
// steps before its MFMAs run, its fragments are read into registers during
// the step before, interleaved with that step's MFMAs, and the MFMAs of a
// step run from registers only.  One barrier per step (it waits for the
// wave's outstanding loads and LDS reads): after it, stage s + 1 has landed
// and every wave holds stage s in registers, so the request for stage s + 2
// may overwrite buffer s % 2.  Tiles, rows and swizzle as
// contract_bat_kernel.
template <class P, int WTM, int WTN, int NBAT, int MINB>
__global__ __launch_bounds__(NBAT * (128 / WTM) * (128 / WTN) * 64, MINB) void contract_pipe_kernel(
    const Slot* __restrict__ slots, int nslot, int total) {
    constexpr int BM = 128, BN = 128;
    constexpr int WPB = (BM / WTM) * (BN / WTN);
    constexpr int NT = 64 * NBAT * WPB;
    constexpr int RS = 128;
    constexpr int ROWS = 128 * (1 + NBAT);
    constexpr int TPR = RS / 16;
    constexpr int RPP = NT / TPR;
    constexpr int NP = ROWS / RPP;
    static_assert(ROWS % RPP == 0, "rows must split evenly over the threads");
    static_assert(RPP % 8 == 0, "staging rows must keep the swizzle bits");
    constexpr int MB = WTM / 16, NB = WTN / 16;
    __shared__ __attribute__((aligned(16))) char lds[2 * ROWS * RS];

    const int bid = xcd_remap(blockIdx.x, total);
    int pass, bgrp, tmi, tni;
    const Slot* S = find_slot(slots, nslot, bid, pass, bgrp, tmi, tni);
    const int v = S->v, o = S->o, Kp = S->Kp;
    const int mt0 = tmi * BM, nt0 = tni * BN;
    const int beta0 = bgrp * NBAT;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wb = wave / WPB, wsub = wave % WPB;
    const int wm = wsub / (BN / WTN), wn = wsub % (BN / WTN);
    const int beta = beta0 + wb;
    const int m0 = mt0 + wm * WTM, n0 = nt0 + wn * WTN;
    const int vm = beta < v ? max(0, min(MB, (v - m0 + 15) / 16)) : 0;
    const int vn = max(0, min(NB, (v - n0 + 15) / 16));

    const int64_t rowbytes = (int64_t)Kp * P::UNITS * sizeof(typename P::E);
    const int csteps = (int)(rowbytes / RS);
    const int nsteps = NSEG * csteps;
    const char* G = static_cast<const char*>(S->gc);
    const char* T = static_cast<const char*>(S->tc);
    const int lrow = threadIdx.x / TPR;
    const int pch = (lane & 7) ^ lds_swz(lrow);
    const int src_col = (P::SPLIT ? (((pch & 3) << 1) | (pch >> 2)) : pch) * 16;
    const int wave_row0 = wave * (64 / TPR);

    const char* rbase[NP];
    typename P::Acc acc[MB][NB];
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = typename P::Acc{};

    // In both passes the batch-dependent operand is A in segment 0 and B in
    // segments 1 and 2.
    auto set_rows = [&](int sg) {
        const SegRows g = segment(pass, sg, S->i, S->j, S->k, o, v);
        const bool depA = sg == 0;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int r = lrow + p * RPP;
            int64_t row;
            if (r < 128) {
                row = depA ? g.b0 + (int64_t)min(nt0 + r, v - 1) * g.bN : g.a0 + (int64_t)min(mt0 + r, v - 1) * g.aM;
            } else {
                const int bb = min(beta0 + (r - 128) / 128, v - 1), rr = (r - 128) % 128;
                row = depA ? g.a0 + bb * g.aB + (int64_t)min(mt0 + rr, v - 1) * g.aM
                           : g.b0 + bb * g.bB + (int64_t)min(nt0 + rr, v - 1) * g.bN;
            }
            const bool fromG = (r < 128) == !depA ? g.aG : g.bG;
            rbase[p] = (fromG ? G : T) + row * rowbytes + src_col;
        }
    };
    // Request the next stage (past the last one, the last chunk again) into buf.
    int ld_sg = 0, ld_c = -1;
    auto request = [&](int buf) {
        if (!(ld_sg == NSEG - 1 && ld_c == csteps - 1)) {
            if (++ld_c == csteps) {
                ld_c = 0;
                ++ld_sg;
                set_rows(ld_sg);
            }
        }
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            char* dst = lds + buf * (ROWS * RS) + (wave_row0 + p * RPP) * RS;
            __builtin_amdgcn_global_load_lds((const GLOBAL void*)gp(rbase[p] + (int64_t)ld_c * RS),
                                             (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
        }
    };
    const int g = lane >> 4;
    const int sw = lds_swz(lane & 15);
    // this wave's A / B fragment rows of stage `stage` in buffer `buf`
    auto a_ptr = [&](int stage, int buf) {
        const int arow = stage < csteps ? 128 * (1 + wb) + wm * WTM : wm * WTM;
        return lds + buf * (ROWS * RS) + (arow + (lane & 15)) * RS;
    };
    auto b_ptr = [&](int stage, int buf) {
        const int brow = stage < csteps ? wn * WTN : 128 * (1 + wb) + wn * WTN;
        return lds + buf * (ROWS * RS) + (brow + (lane & 15)) * RS;
    };

    set_rows(0);
    request(0);
    request(1);
    lds_dma_barrier();
    StageFrags<P, MB, NB> f0, f1;
    read_frags<P, MB, NB, RS>(f0, a_ptr(0, 0), b_ptr(0, 0), g, sw);
    const bool active = vm > 0 && vn > 0;
    const bool full = vm == MB && vn == NB;

    for (int step = 0; step < nsteps; step += 2) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int st = step + h;
            if (h == 1 && st >= nsteps) break;
            lds_dma_barrier();
            request(h);  // stage st + 2 into buffer st % 2 (= h)
            __builtin_amdgcn_sched_barrier(0);
            const int nst = min(st + 1, nsteps - 1);
            const char* As = a_ptr(nst, h ^ 1);
            const char* Bs = b_ptr(nst, h ^ 1);
            if (active) {
                if (full)
                    mma_stage_overlap<P, MB, NB, RS, true>(acc, h == 0 ? f0 : f1, h == 0 ? f1 : f0, As, Bs, g, sw,
                                                           vm, vn);
                else
                    mma_stage_overlap<P, MB, NB, RS, false>(acc, h == 0 ? f0 : f1, h == 0 ? f1 : f0, As, Bs, g, sw,
                                                            vm, vn);
            }
        }
    }
    if (active) store_tile<P, MB, NB>(S, pass, beta, m0, n0, vm, vn, lane, acc);
}

// Deep-ring variant of the batch-shared kernel: NSTAGE LDS stages, of which
// NSTAGE - 1 are in flight (global_load_lds) while one feeds the MFMAs, so
// that a stage is requested NSTAGE - 1 steps before it is used and HBM/L2
// latency hides behind that many steps of matrix work.  Per step: wait until
// only the NSTAGE - 2 most recent stages are outstanding (the vector-memory
// counter completes loads in issue order), barrier (the stage has landed for
// every wave, and every wave has finished with the previous stage's buffer),
// request the stage NSTAGE - 1 ahead into that buffer, then read fragments
// and run the MFMAs of the current stage.  Tiles, rows and swizzle as
// contract_bat_kernel.
template <int N>
__device__ __forceinline__ void ring_barrier() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    asm volatile("s_waitcnt vmcnt(%0)\n\ts_waitcnt lgkmcnt(0)\n\ts_barrier" ::"n"(N) : "memory");
}

template <class P, int WTM, int WTN, int NBAT, int NSTAGE, int MINB>
__global__ __launch_bounds__(NBAT * (128 / WTM) * (128 / WTN) * 64, MINB) void contract_ring_kernel(
    const Slot* __restrict__ slots, int nslot, int total) {
    constexpr int BM = 128, BN = 128;
    constexpr int WPB = (BM / WTM) * (BN / WTN);
    constexpr int NT = 64 * NBAT * WPB;
    constexpr int RS = 128;
    constexpr int ROWS = 128 * (1 + NBAT);
    constexpr int TPR = RS / 16;
    constexpr int RPP = NT / TPR;
    constexpr int NP = ROWS / RPP;
    static_assert(ROWS % RPP == 0, "rows must split evenly over the threads");
    static_assert(RPP % 8 == 0, "staging rows must keep the swizzle bits");
    static_assert(NSTAGE >= 3, "at least two stages in flight");
    constexpr int MB = WTM / 16, NB = WTN / 16;
    __shared__ __attribute__((aligned(16))) char lds[NSTAGE * ROWS * RS];

    const int bid = xcd_remap(blockIdx.x, total);
    int pass, bgrp, tmi, tni;
    const Slot* S = find_slot(slots, nslot, bid, pass, bgrp, tmi, tni);
    const int v = S->v, o = S->o, Kp = S->Kp;
    const int mt0 = tmi * BM, nt0 = tni * BN;
    const int beta0 = bgrp * NBAT;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wb = wave / WPB, wsub = wave % WPB;
    const int wm = wsub / (BN / WTN), wn = wsub % (BN / WTN);
    const int beta = beta0 + wb;
    const int m0 = mt0 + wm * WTM, n0 = nt0 + wn * WTN;
    const int vm = beta < v ? max(0, min(MB, (v - m0 + 15) / 16)) : 0;
    const int vn = max(0, min(NB, (v - n0 + 15) / 16));

    const int64_t rowbytes = (int64_t)Kp * P::UNITS * sizeof(typename P::E);
    const int csteps = (int)(rowbytes / RS);
    const int nsteps = NSEG * csteps;
    const char* G = static_cast<const char*>(S->gc);
    const char* T = static_cast<const char*>(S->tc);
    const int lrow = threadIdx.x / TPR;
    const int pch = (lane & 7) ^ lds_swz(lrow);
    const int src_col = (P::SPLIT ? (((pch & 3) << 1) | (pch >> 2)) : pch) * 16;
    const int wave_row0 = wave * (64 / TPR);

    const char* rbase[NP];
    typename P::Acc acc[MB][NB];
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = typename P::Acc{};

    // In both passes the batch-dependent operand is A in segment 0 and B in
    // segments 1 and 2.
    auto set_rows = [&](int sg) {
        const SegRows g = segment(pass, sg, S->i, S->j, S->k, o, v);
        const bool depA = sg == 0;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int r = lrow + p * RPP;
            int64_t row;
            if (r < 128) {
                row = depA ? g.b0 + (int64_t)min(nt0 + r, v - 1) * g.bN : g.a0 + (int64_t)min(mt0 + r, v - 1) * g.aM;
            } else {
                const int bb = min(beta0 + (r - 128) / 128, v - 1), rr = (r - 128) % 128;
                row = depA ? g.a0 + bb * g.aB + (int64_t)min(mt0 + rr, v - 1) * g.aM
                           : g.b0 + bb * g.bB + (int64_t)min(nt0 + rr, v - 1) * g.bN;
            }
            const bool fromG = (r < 128) == !depA ? g.aG : g.bG;
            rbase[p] = (fromG ? G : T) + row * rowbytes + src_col;
        }
    };
    // Request the next stage (past the last one, the last chunk again) into buf.
    int ld_sg = 0, ld_c = -1;
    auto request = [&](int buf) {
        if (!(ld_sg == NSEG - 1 && ld_c == csteps - 1)) {
            if (++ld_c == csteps) {
                ld_c = 0;
                ++ld_sg;
                set_rows(ld_sg);
            }
        }
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            char* dst = lds + buf * (ROWS * RS) + (wave_row0 + p * RPP) * RS;
            __builtin_amdgcn_global_load_lds((const GLOBAL void*)gp(rbase[p] + (int64_t)ld_c * RS),
                                             (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
        }
    };

    set_rows(0);
#pragma unroll
    for (int s = 0; s < NSTAGE - 1; ++s) request(s);
    const bool active = vm > 0 && vn > 0;
    const bool full = vm == MB && vn == NB;
    const int g = lane >> 4;
    const int sw = lds_swz(lane & 15);
    int buf = 0;                 // buffer of stage `step`
    int lbuf = NSTAGE - 1;       // buffer of stage step + NSTAGE - 1
    for (int step = 0; step < nsteps; ++step) {
        ring_barrier<(NSTAGE - 2) * NP>();
        request(lbuf);
        __builtin_amdgcn_sched_barrier(0);
        if (active) {
            const bool dep = step < csteps;
            const char* st = lds + buf * (ROWS * RS);
            const int arow = dep ? 128 * (1 + wb) + wm * WTM : wm * WTM;
            const int brow = dep ? wn * WTN : 128 * (1 + wb) + wn * WTN;
            const char* As = st + (arow + (lane & 15)) * RS;
            const char* Bs = st + (brow + (lane & 15)) * RS;
            constexpr bool ONE_WAVE_PER_SIMD = NT == 256;
            if constexpr (ONE_WAVE_PER_SIMD) {
                if (full)
                    lds_stage_pm<P, MB, NB, RS, true>(acc, As, Bs, g, sw, vm, vn);
                else
                    lds_stage_pm<P, MB, NB, RS, false>(acc, As, Bs, g, sw, vm, vn);
            } else {
                if (full)
                    lds_stage<P, MB, NB, RS, true>(acc, As, Bs, g, sw, vm, vn);
                else
                    lds_stage<P, MB, NB, RS, false>(acc, As, Bs, g, sw, vm, vn);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        buf = buf == NSTAGE - 1 ? 0 : buf + 1;
        lbuf = lbuf == NSTAGE - 1 ? 0 : lbuf + 1;
    }
    // drain the trailing requests before the workgroup's LDS is released
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    if (active) store_tile<P, MB, NB>(S, pass, beta, m0, n0, vm, vn, lane, acc);
}

// ---------------------------------------------------------------------------
// Large-tile kernel (32x32 MFMA blocks: BF16X3 and FP32).  A workgroup of
// four waves, one per SIMD, owns a 256 x 256 tile of the (row, col) plane of
// one batch index; each wave accumulates at most 4 x 4 blocks (128 x 128,
// 256 accumulator registers), so that a K stage of 128-byte rows feeds a
// wave with half the LDS bytes per MFMA of a 64 x 64 wave tile.  The rows
// of the tile (256 of A, 256 of B; 64 KB per stage) stream through two LDS
// stages with global_load_lds, in the chunk order and swizzle of
// contract_lds_kernel.  Per stage: the MFMAs of each sub-step run from
// registers while the fragments of the next sub-step are read from LDS; the
// one barrier of the stage sits before its last sub-step, whose MFMAs then
// overlap the reads of the next stage's first fragments and the
// global_load_lds of the stage after that into the buffer just released.
// One wave per SIMD has no other wave to hide a dependent MFMA behind, so
// the products are issued product by product across the wave's blocks.
// Edge tiles split their valid blocks over the four waves along the longer
// side instead of 2 x 2, so that no wave idles while another does a full
// tile's work; every wave runs the same loads and barriers.
constexpr int BIG_T = 256;   // workgroup tile edge
constexpr int BIG_W = 4;     // blocks per wave and dimension (at most)

template <class P, int RB, int CB>
__device__ __forceinline__ void big_mma(typename P::Acc (&acc)[BIG_W][BIG_W], const typename P::Frag (&fa)[BIG_W],
                                        const typename P::Frag (&fb)[BIG_W]) {
#pragma unroll
    for (int a = 0; a < RB; ++a)
#pragma unroll
        for (int b = 0; b < CB; ++b) P::template mma_t<0>(acc[a][b], fa[a], fb[b]);
#pragma unroll
    for (int a = 0; a < RB; ++a)
#pragma unroll
        for (int b = 0; b < CB; ++b) P::template mma_t<1>(acc[a][b], fa[a], fb[b]);
    if constexpr (P::NMMA > 2) {
#pragma unroll
        for (int a = 0; a < RB; ++a)
#pragma unroll
            for (int b = 0; b < CB; ++b) P::template mma_t<2>(acc[a][b], fa[a], fb[b]);
    }
    if constexpr (P::NMMA > 3) {
#pragma unroll
        for (int a = 0; a < RB; ++a)
#pragma unroll
            for (int b = 0; b < CB; ++b) P::template mma_t<3>(acc[a][b], fa[a], fb[b]);
    }
}

template <class P, int RB, int CB>
__device__ __forceinline__ void big_read(typename P::Frag (&fa)[BIG_W], typename P::Frag (&fb)[BIG_W],
                                         const char* As, const char* Bs, int g, int sub, int sw) {
#pragma unroll
    for (int a = 0; a < RB; ++a) P::load_lds(fa[a], As + a * P::BS * 128, g, sub, sw);
#pragma unroll
    for (int b = 0; b < CB; ++b) P::load_lds(fb[b], Bs + b * P::BS * 128, g, sub, sw);
}

// Spread NR LDS reads (and NV global loads) evenly over NM MFMAs in the
// schedule of one region.
template <int NM, int NR, int NV = 0, int I = 0>
__device__ __forceinline__ void big_interleave() {
    if constexpr (NR > 0 && I < NR) {
        constexpr int q = (NM * (I + 1)) / NR - (NM * I) / NR;
        constexpr int nv = (NV * (I + 1)) / NR - (NV * I) / NR;
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // one LDS read
        if constexpr (nv > 0) __builtin_amdgcn_sched_group_barrier(0x020, nv, 0);   // global loads
        if constexpr (q > 0) __builtin_amdgcn_sched_group_barrier(0x008, q, 0);   // q MFMAs
        big_interleave<NM, NR, NV, I + 1>();
    }
}

template <class P>
struct BigFrags {
    typename P::Frag a[BIG_W], b[BIG_W];
};

// The K loop of one wave over all stages of the tile (see above).  `gload`
// requests a stage into a buffer; As/Bs point at this wave's first A / B
// fragment row in buffer 0.
template <class P, int RB, int CB, class GL>
__device__ __forceinline__ void big_loop(typename P::Acc (&acc)[BIG_W][BIG_W], const char* As, const char* Bs,
                                         int g, int sw, int nsteps, GL&& gload) {
    constexpr int STAGE = 2 * BIG_T * 128;   // bytes of one LDS stage
    constexpr int NS = P::NSUB;
    constexpr int NM = P::NMMA * RB * CB;                    // MFMAs per sub-step
    constexpr int NR = (RB + CB) * (P::SPLIT ? 2 : 1);       // LDS reads per sub-step
    static_assert(NS % 2 == 0, "fragment buffers alternate per sub-step");
    BigFrags<P> f[2];
    if constexpr (RB > 0 && CB > 0) big_read<P, RB, CB>(f[0].a, f[0].b, As, Bs, g, 0, sw);
    for (int step = 0; step < nsteps; ++step) {
        const int off = (step & 1) * STAGE;
#pragma unroll
        for (int sub = 0; sub < NS - 1; ++sub) {
            if constexpr (RB > 0 && CB > 0) {
                big_read<P, RB, CB>(f[(sub + 1) & 1].a, f[(sub + 1) & 1].b, As + off, Bs + off, g, sub + 1, sw);
                big_mma<P, RB, CB>(acc, f[sub & 1].a, f[sub & 1].b);
                big_interleave<NM, NR>();
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        // stage step + 1 has landed for every wave and every wave is done
        // reading this stage's buffer
        asm volatile("s_waitcnt vmcnt(0)\n\ts_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
        if (step + 2 < nsteps) gload(step + 2, step & 1);
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (RB > 0 && CB > 0) {
            // next stage's first sub-step (stale data after the last stage; unused)
            big_read<P, RB, CB>(f[0].a, f[0].b, As + (STAGE - off), Bs + (STAGE - off), g, 0, sw);
            big_mma<P, RB, CB>(acc, f[1].a, f[1].b);
            big_interleave<NM, NR>();
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    asm volatile("s_waitcnt vmcnt(0)\n\ts_waitcnt lgkmcnt(0)" ::: "memory");
}

template <class P>
__global__ __launch_bounds__(256, 1) void contract_big_kernel(const Slot* __restrict__ slots, int nslot, int total) {
    static_assert(P::BS == 32, "32x32 MFMA blocks");
    constexpr int RS = 128;
    constexpr int ROWS = 2 * BIG_T;
    constexpr int NP = ROWS * (RS / 16) / 256;   // 16-byte loads per thread per stage
    constexpr int STAGE = ROWS * RS;
    __shared__ __attribute__((aligned(16))) char lds[2 * STAGE];

    const int bid = xcd_remap(blockIdx.x, total);
    int pass, beta, tmi, tni;
    const Slot* S = find_slot(slots, nslot, bid, pass, beta, tmi, tni);
    const int v = S->v, o = S->o, Kp = S->Kp;
    const int mt0 = tmi * BIG_T, nt0 = tni * BIG_T;
    const int mb = min(BIG_T / 32, (v - mt0 + 31) / 32), nb = min(BIG_T / 32, (v - nt0 + 31) / 32);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int r0, rb, c0, cb;
    if (mb > BIG_W && nb > BIG_W) {
        r0 = (wave >> 1) * BIG_W;
        rb = min(BIG_W, mb - r0);
        c0 = (wave & 1) * BIG_W;
        cb = min(BIG_W, nb - c0);
    } else if (mb >= nb) {
        const int per = (mb + 3) / 4;
        r0 = wave * per;
        rb = max(0, min(per, mb - r0));
        c0 = 0;
        cb = nb;
    } else {
        const int per = (nb + 3) / 4;
        c0 = wave * per;
        cb = max(0, min(per, nb - c0));
        r0 = 0;
        rb = mb;
    }

    const int64_t rowbytes = (int64_t)Kp * P::UNITS * sizeof(typename P::E);
    const int csteps = (int)(rowbytes / RS);
    const int nsteps = NSEG * csteps;
    const char* G = static_cast<const char*>(S->gc);
    const char* T = static_cast<const char*>(S->tc);
    const int lrow = threadIdx.x >> 3;                // 0..31; load p covers row lrow + 32 p
    const int pch = (lane & 7) ^ lds_swz_bs<32>(lrow);
    const int src_col = (P::SPLIT ? (((pch & 3) << 1) | (pch >> 2)) : pch) * 16;
    int64_t roff[NP];
    const char* baseA = G;
    const char* baseB = T;
    auto set_rows = [&](int sg) {
        const SegRows g = segment(pass, sg, S->i, S->j, S->k, o, v);
        baseA = g.aG ? G : T;
        baseB = g.bG ? G : T;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int r = lrow + 32 * p;
            if (r < BIG_T) {
                const int m = min(mt0 + r, v - 1);
                roff[p] = (g.a0 + beta * g.aB + m * g.aM) * rowbytes + src_col;
            } else {
                const int n = min(nt0 + r - BIG_T, v - 1);
                roff[p] = (g.b0 + beta * g.bB + n * g.bN) * rowbytes + src_col;
            }
        }
    };
    int ld_sg = 0, ld_c = 0;   // segment and chunk of the stage last requested
    auto issue = [&](int c, int buf) {
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const char* src = (p < NP / 2 ? baseA : baseB) + roff[p] + (int64_t)c * RS;
            char* dst = lds + buf * STAGE + (8 * wave + 32 * p) * RS;
            __builtin_amdgcn_global_load_lds((const GLOBAL void*)gp(src), (__attribute__((address_space(3))) void*)dst,
                                             16, 0, 0);
        }
    };
    // stages are requested in order: stage st is chunk st % csteps of segment st / csteps
    auto gload = [&](int st, int buf) {
        const int sg = st / csteps;
        if (sg != ld_sg) {
            ld_sg = sg;
            set_rows(sg);
        }
        ld_c = st - sg * csteps;
        issue(ld_c, buf);
    };
    static_assert(NP % 2 == 0 && BIG_T % 32 == 0, "A rows are the first half of the loads");

    typename P::Acc acc[BIG_W][BIG_W];
#pragma unroll
    for (int a = 0; a < BIG_W; ++a)
#pragma unroll
        for (int b = 0; b < BIG_W; ++b) acc[a][b] = typename P::Acc{};

    set_rows(0);
    issue(0, 0);
    if (nsteps > 1) {
        gload(1, 1);
        asm volatile("s_waitcnt vmcnt(%0)\n\ts_waitcnt lgkmcnt(0)\n\ts_barrier" ::"n"(NP) : "memory");
    } else {
        asm volatile("s_waitcnt vmcnt(0)\n\ts_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    }
    const int g = lane >> 5;
    const int sw = lds_swz_bs<32>(lane & 31);
    const char* As = lds + (r0 * 32 + (lane & 31)) * RS;
    const char* Bs = lds + (BIG_T + c0 * 32 + (lane & 31)) * RS;
#define CCSDT_BIG_CASE(R, C) \
    case R * 8 + C: big_loop<P, R, C>(acc, As, Bs, g, sw, nsteps, gload); break;
    switch ((rb > 0 && cb > 0) ? rb * 8 + cb : 0) {
        CCSDT_BIG_CASE(4, 4) CCSDT_BIG_CASE(4, 3) CCSDT_BIG_CASE(4, 2) CCSDT_BIG_CASE(4, 1)
        CCSDT_BIG_CASE(3, 4) CCSDT_BIG_CASE(3, 3) CCSDT_BIG_CASE(3, 2) CCSDT_BIG_CASE(3, 1)
        CCSDT_BIG_CASE(2, 4) CCSDT_BIG_CASE(2, 3) CCSDT_BIG_CASE(2, 2) CCSDT_BIG_CASE(2, 1)
        CCSDT_BIG_CASE(1, 4) CCSDT_BIG_CASE(1, 3) CCSDT_BIG_CASE(1, 2) CCSDT_BIG_CASE(1, 1)
        default: big_loop<P, 0, 0>(acc, As, Bs, g, sw, nsteps, gload); break;
    }
#undef CCSDT_BIG_CASE
    if (rb > 0 && cb > 0)
        store_tile<P, BIG_W, BIG_W>(S, pass, beta, mt0 + r0 * 32, nt0 + c0 * 32, rb, cb, lane, acc);
}

// Resident workgroups for the persistent kernels: `per_cu` per compute unit,
// rounded to a multiple of NXCD.
static int persist_grid(int per_cu) {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
            cus = n;
        else
            cus = 256;
    }
    return (cus * per_cu + NXCD - 1) / NXCD * NXCD;
}

static int pace_lag() {
    static int lag = -1;
    if (lag < 0) {
        const char* e = getenv("CCSDT_PACE_LAG");
        lag = e ? atoi(e) : 2;
        if (lag < 0) lag = 0;
    }
    return lag;
}

template <class P>
static hipError_t contract_impl(int cfg, const Slot* d_slots, int nslot, int total, unsigned* pace, hipStream_t s) {
    if (cfg == 24) {
        const int grid = persist_grid(2);
        if (!pace || (size_t)grid * PACE_STRIDE * sizeof(unsigned) > PACE_BYTES) return hipErrorInvalidValue;
        hipLaunchKernelGGL(pace_clear_kernel, dim3(1), dim3(256), 0, s, pace, grid);
        hipLaunchKernelGGL((contract_lds_paced_kernel<P, 64, 64, 2>), dim3(grid), dim3(256), 0, s, d_slots, nslot,
                           total, pace, pace_lag());
        return hipGetLastError();
    }
    switch (cfg) {
        case 0: hipLaunchKernelGGL((contract_kernel<P, 2, 2>), dim3(total), dim3(256), 0, s, d_slots, nslot, total); break;
        case 1: hipLaunchKernelGGL((contract_kernel<P, 4, 2>), dim3(total), dim3(256), 0, s, d_slots, nslot, total); break;
        case 2: hipLaunchKernelGGL((contract_kernel<P, 4, 4>), dim3(total), dim3(256), 0, s, d_slots, nslot, total); break;
        case 3: hipLaunchKernelGGL((contract_lds_kernel<P, 64, 64, 128, 2, false>), dim3(total), dim3(256), 0, s, d_slots, nslot, total); break;
        case 4: hipLaunchKernelGGL((contract_lds_kernel<P, 64, 128, 128, 1, false>), dim3(total), dim3(256), 0, s, d_slots, nslot, total); break;
        case 5: hipLaunchKernelGGL((contract_lds_kernel<P, 32, 64, 128, 2, false>), dim3(total), dim3(256), 0, s, d_slots, nslot, total); break;
        case 6: hipLaunchKernelGGL((contract_lds_kernel<P, 64, 64, 128, 2, true>), dim3(total), dim3(256), 0, s, d_slots, nslot, total); break;
        case 7: hipLaunchKernelGGL((contract_lds_kernel<P, 64, 128, 128, 1, true>), dim3(total), dim3(256), 0, s, d_slots, nslot, total); break;
        case 8: hipLaunchKernelGGL((contract_bat_kernel<P, 128, 64, 2, 1>), dim3(total), dim3(256), 0, s, d_slots, nslot, total); break;
        case 9: hipLaunchKernelGGL((contract_bat_kernel<P, 64, 64, 2, 1>), dim3(total), dim3(512), 0, s, d_slots, nslot, total); break;
        case 10: hipLaunchKernelGGL((contract_pipe_kernel<P, 128, 64, 2, 1>), dim3(total), dim3(256), 0, s, d_slots, nslot, total); break;
        case 11: hipLaunchKernelGGL((contract_pipe_kernel<P, 64, 64, 2, 1>), dim3(total), dim3(512), 0, s, d_slots, nslot, total); break;
        case 12: hipLaunchKernelGGL((contract_pipe_kernel<P, 64, 64, 1, 2>), dim3(total), dim3(256), 0, s, d_slots, nslot, total); break;
        case 13: hipLaunchKernelGGL((contract_ring_kernel<P, 64, 64, 2, 3, 1>), dim3(total), dim3(512), 0, s, d_slots, nslot, total); break;
        case 14: hipLaunchKernelGGL((contract_ring_kernel<P, 64, 64, 1, 4, 1>), dim3(total), dim3(256), 0, s, d_slots, nslot, total); break;
        case 15: hipLaunchKernelGGL((contract_ring_kernel<P, 128, 64, 2, 3, 1>), dim3(total), dim3(256), 0, s, d_slots, nslot, total); break;
        case 16: hipLaunchKernelGGL((contract_lds_persist_kernel<P, 64, 64, 128, 2, true>), dim3(persist_grid(2)), dim3(256), 0, s, d_slots, nslot, total); break;
        case 17: hipLaunchKernelGGL((contract_lds_kernel<P, 128, 128, 128, 1, true>), dim3(total), dim3(256), 0, s, d_slots, nslot, total); break;
        case 18: hipLaunchKernelGGL((contract_lds_kernel<P, 128, 64, 128, 1, true>), dim3(total), dim3(256), 0, s, d_slots, nslot, total); break;
        case 19: hipLaunchKernelGGL((contract_lds_wide_kernel<P, 64, 64, 4, 2, 2>), dim3(total), dim3(512), 0, s, d_slots, nslot, total); break;
        case 20: hipLaunchKernelGGL((contract_lds_wide_kernel<P, 64, 64, 2, 4, 2>), dim3(total), dim3(512), 0, s, d_slots, nslot, total); break;
        case 21: hipLaunchKernelGGL((contract_lds_kernel<P, 32, 64, 128, 3, true>), dim3(total), dim3(256), 0, s, d_slots, nslot, total); break;
        case 22: hipLaunchKernelGGL((contract_lds_kernel<typename Wide<P>::T, 64, 64, 128, 2, true>), dim3(total), dim3(256), 0, s, d_slots, nslot, total); break;
        case 23: hipLaunchKernelGGL((contract_lds_kernel<typename Wide<P>::T, 64, 128, 128, 1, true>), dim3(total), dim3(256), 0, s, d_slots, nslot, total); break;
        case 26: hipLaunchKernelGGL((contract_lds_spread_kernel<P>), dim3(total), dim3(256), 0, s, d_slots, nslot, total); break;
        case 25:
            if constexpr (Wide<P>::T::BS == 32)
                hipLaunchKernelGGL((contract_big_kernel<typename Wide<P>::T>), dim3(total), dim3(256), 0, s, d_slots, nslot, total);
            else
                return hipErrorInvalidValue;   // FP64 has no 32x32 MFMA: plans map 25 to 6
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_contract(int prec, int cfg, const Slot* d_slots, int nslot, int total, unsigned* pace,
                           hipStream_t s) {
    if (total <= 0) return hipSuccess;
    switch (prec) {
        case P_FP64: return contract_impl<PrecF64>(cfg, d_slots, nslot, total, pace, s);
        case P_FP32: return contract_impl<PrecF32>(cfg, d_slots, nslot, total, pace, s);
        case P_BF16X3: return contract_impl<PrecB3>(cfg, d_slots, nslot, total, pace, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ccsdt
