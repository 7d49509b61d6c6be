// Host runtime and C ABI of the (T) library (declarations in include/ccsdt.h).
//
// Work list (paper Sec. 3: restricted occupied loops collapsed into one loop
// of independent tasks, eq. tasks_ccsdpt): the triples i<=j<=k with a
// non-zero multiplicity.  Triples are processed in chunks whose W buffers fit
// the W budget; each chunk is three launches:
//   contraction (both passes)  ->  energy partials  ->  slot reduce
// after the operands of every problem have been packed once per call.  A
// final reduce sums the per-triple energies of each problem in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <random>
#include <string>
#include <vector>

#include "ccsdt.h"
#include "common.hpp"

using namespace ccsdt;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

enum { K_PACK = 0, K_CONTRACT = 1, K_ENERGY = 2, K_REDUCE = 3, K_ASSEMBLE = 4, K_MP2_GEMM = 5, K_MP2_ENERGY = 6,
       K_NCLASS = 7 };

size_t env_size(const char* name, size_t dflt) {
    const char* s = std::getenv(name);
    if (!s || !*s) return dflt;
    char* end = nullptr;
    unsigned long long v = std::strtoull(s, &end, 10);
    return (end && *end == 0) ? (size_t)v : dflt;
}

int env_int(const char* name, int dflt) {
    const char* s = std::getenv(name);
    if (!s || !*s) return dflt;
    return std::atoi(s);
}

}  // namespace

struct GraphEntry {
    bool valid = false;
    int prec = -1;
    uint64_t gen = 0;
    std::vector<ccsdt_problem> probs;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void* host = nullptr;      // pinned: slot table, triple ranges, problem table, results
    size_t host_bytes = 0;
    size_t layout_out = 0;     // byte offset of the result rows in ``host``
};

struct ccsdt_context {
    int device = 0;
    DevBuf gc, tc, w, part, etrip, slots, out, tripbeg, pdesc;
    uint64_t gen = 0;          // bumped whenever a device buffer is (re)allocated
    size_t cap = 0;            // CCSDT_MAX_DEVICE_BYTES (0 = none)
    size_t w_budget = 0;       // bytes of W per chunk
    double* host_out = nullptr;
    size_t host_out_bytes = 0;
    Slot* host_slots = nullptr;
    size_t host_slots_bytes = 0;
    int* host_tb = nullptr;
    size_t host_tb_bytes = 0;
    bool profile = false;
    int64_t prof_n[K_NCLASS] = {0};
    double prof_ms[K_NCLASS] = {0};
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<int> ev_class;
    std::map<std::pair<int, int>, int> plans;  // (precision, v bucket) -> tile configuration
    int forced_cfg = -1;                       // set by the autotuner while it measures
    GraphEntry graph;
    hipStream_t cap_stream = nullptr;          // private stream used only for graph capture
    int64_t n_captures = 0, n_replays = 0;
    // streaming of a host-resident vvvo: two device staging buffers, a copy
    // stream and the events that order copies and packs
    DevBuf stage;
    DevBuf pace;                               // per-XCD counters of the paced contraction
    size_t stage_budget = 0;                   // CCSDT_STAGE_BYTES: both staging buffers together
    hipStream_t copy_stream = nullptr;
    hipEvent_t ev_copy[2] = {nullptr, nullptr}, ev_pack[2] = {nullptr, nullptr}, ev_start = nullptr;
    int64_t streamed_bytes = 0;
    // test hooks, read at creation: CCSDT_FAIL_AT names a kernel class whose
    // next launch fails with CCSDT_EHIP instead of running; CCSDT_SHUFFLE
    // (a nonzero seed) shuffles the work list inside each tile plan
    int fail_at = -1;
    uint64_t shuffle = 0;
    GapDesc* host_desc = nullptr;
    size_t host_desc_bytes = 0;

    size_t allocated() const {
        return gc.bytes + tc.bytes + w.bytes + part.bytes + etrip.bytes + slots.bytes + out.bytes + tripbeg.bytes +
               pdesc.bytes + stage.bytes + pace.bytes;
    }
};

namespace {

int ensure(ccsdt_context* ctx, DevBuf& b, size_t bytes, const char* what) {
    if (bytes <= b.bytes) return CCSDT_OK;
    size_t others = ctx->allocated() - b.bytes;
    if (ctx->cap && others + bytes > ctx->cap)
        return fail(CCSDT_ENOMEM, std::string("workspace ") + what + " exceeds CCSDT_MAX_DEVICE_BYTES");
    if (b.p) {
        (void)hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
    }
    if (bytes == 0) return CCSDT_OK;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(CCSDT_ENOMEM, std::string("hipMalloc of ") + std::to_string(bytes) + " bytes for " + what +
                                      " failed: " + hipGetErrorString(e));
    }
    b.p = p;
    b.bytes = bytes;
    ++ctx->gen;
    return CCSDT_OK;
}

int ensure_host(void** p, size_t* have, size_t bytes) {
    if (bytes <= *have) return CCSDT_OK;
    if (*p) (void)hipHostFree(*p);
    *p = nullptr;
    *have = 0;
    hipError_t e = hipHostMalloc(p, bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(CCSDT_ENOMEM, "pinned host allocation failed");
    }
    *have = bytes;
    return CCSDT_OK;
}

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) {                                                               \
            (void)hipGetLastError();                                                          \
            return fail(CCSDT_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));       \
        }                                                                                     \
    } while (0)

#define CHK(expr)                  \
    do {                           \
        int rc_ = (expr);          \
        if (rc_ != CCSDT_OK) return rc_; \
    } while (0)

// ---- profiling -------------------------------------------------------------
int prof_begin(ccsdt_context* ctx, int cls, hipStream_t s) {
    if (!ctx->profile) return CCSDT_OK;
    while (ctx->ev_pool.size() < ctx->ev_used + 2) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        ctx->ev_pool.push_back(e);
    }
    HIPCHK(hipEventRecord(ctx->ev_pool[ctx->ev_used], s));
    ctx->ev_class.push_back(cls);
    return CCSDT_OK;
}

int prof_end(ccsdt_context* ctx, hipStream_t s) {
    if (!ctx->profile) return CCSDT_OK;
    HIPCHK(hipEventRecord(ctx->ev_pool[ctx->ev_used + 1], s));
    ctx->ev_used += 2;
    return CCSDT_OK;
}

void prof_start_call(ccsdt_context* ctx) {
    ctx->ev_class.clear();
    ctx->ev_used = 0;
}

int prof_collect(ccsdt_context* ctx) {
    if (!ctx->profile) return CCSDT_OK;
    for (size_t n = 0; n < ctx->ev_class.size(); ++n) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, ctx->ev_pool[2 * n], ctx->ev_pool[2 * n + 1]));
        ctx->prof_n[ctx->ev_class[n]] += 1;
        ctx->prof_ms[ctx->ev_class[n]] += ms;
    }
    ctx->ev_class.clear();
    ctx->ev_used = 0;
    return CCSDT_OK;
}

const char* const KERNEL_CLASS_NAMES[K_NCLASS] = {"pack", "contract", "energy", "reduce", "assemble", "mp2_gemm",
                                                   "mp2_energy"};

#define LAUNCH(cls, expr)                                                                         \
    do {                                                                                          \
        if (ctx->fail_at == (cls))                                                                \
            return fail(CCSDT_EHIP, std::string("injected failure (CCSDT_FAIL_AT) before a ") +  \
                                        KERNEL_CLASS_NAMES[cls] + " launch");                    \
        CHK(prof_begin(ctx, cls, s));                                                             \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) {                                                                   \
            (void)hipGetLastError();                                                              \
            return fail(CCSDT_EHIP, std::string("launch ") + #expr + ": " + hipGetErrorString(e_)); \
        }                                                                                         \
        CHK(prof_end(ctx, s));                                                                    \
    } while (0)

// ---- validation --------------------------------------------------------------
bool is_device_ptr(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t a;
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// Page-locked host memory (hipHostMalloc) that the device can copy from
// asynchronously.
bool is_pinned_host_ptr(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t a;
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeHost;
}

int check_problem(const ccsdt_problem* p, int idx, bool need_vvvo = true) {
    const std::string where = idx >= 0 ? " (problem " + std::to_string(idx) + ")" : "";
    if (!p) return fail(CCSDT_EINVAL, "null problem" + where);
    if (p->nocc < 1 || p->nvirt < 1) return fail(CCSDT_EINVAL, "nocc and nvirt must be >= 1" + where);
    // limits keep every flattened grid and slot offset inside int32
    if (p->nocc > 1024 || p->nvirt > 2048) return fail(CCSDT_EINVAL, "nocc > 1024 or nvirt > 2048" + where);
    const double* ptrs[7] = {p->eps_o, p->eps_v, p->t1, p->t2, p->vvvo, p->ovoo, p->ovov};
    const char* names[7] = {"eps_o", "eps_v", "t1", "t2", "vvvo", "ovoo", "ovov"};
    for (int n = 0; n < 7; ++n) {
        if (n == 4 && !need_vvvo) continue;
        if (!ptrs[n]) return fail(CCSDT_EINVAL, std::string("null pointer ") + names[n] + where);
        if (n == 4 && is_pinned_host_ptr(ptrs[n])) continue;   // streamed from host memory
        if (!is_device_ptr(ptrs[n]))
            return fail(CCSDT_EINVAL, std::string(names[n]) + " is not a device pointer" +
                                          (n == 4 ? " or pinned host memory" : "") + where);
    }
    return CCSDT_OK;
}

int check_gap(const ccsdt_problem* p, hipStream_t s, int idx) {
    std::vector<double> eo(p->nocc), ev(p->nvirt);
    HIPCHK(hipMemcpyAsync(eo.data(), p->eps_o, sizeof(double) * p->nocc, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(ev.data(), p->eps_v, sizeof(double) * p->nvirt, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double mo = -INFINITY, mv = INFINITY;
    for (double x : eo) {
        if (!std::isfinite(x)) return fail(CCSDT_EINVAL, "non-finite eps_o");
        mo = std::max(mo, x);
    }
    for (double x : ev) {
        if (!std::isfinite(x)) return fail(CCSDT_EINVAL, "non-finite eps_v");
        mv = std::min(mv, x);
    }
    if (!(mo < mv))
        return fail(CCSDT_EDENOM, "max(eps_o) >= min(eps_v): denominators must be negative" +
                                      (idx >= 0 ? " (problem " + std::to_string(idx) + ")" : std::string()));
    return CCSDT_OK;
}

// A context owns device memory of the device that was current when it was
// created; a call that launches work must run with that device current.
int check_ctx(ccsdt_context* ctx) {
    if (!ctx) return fail(CCSDT_EINVAL, "null context");
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev != ctx->device)
        return fail(CCSDT_EINVAL, "context belongs to device " + std::to_string(ctx->device) +
                                      ", but device " + std::to_string(dev) + " is current");
    return CCSDT_OK;
}

int check_prec(int prec) {
    if (prec != CCSDT_FP64 && prec != CCSDT_FP32 && prec != CCSDT_BF16X3)
        return fail(CCSDT_EUNSUPPORTED, "unknown precision " + std::to_string(prec));
    return CCSDT_OK;
}

size_t elem_bytes(int prec) { return prec == CCSDT_FP64 ? 8 : 4; }   // packed element (hi+lo = 4)
size_t w_bytes(int prec) { return prec == CCSDT_FP64 ? 8 : 4; }

// ---- plans ---------------------------------------------------------------------
// Tile plans are kept per (precision, v bucket); a bucket spans v in
// (2^(b-1), 2^b].  Without an autotuned entry the direct-to-LDS 128x128 tile
// is used for v >= 64 and the register-direct 64x64 tile below.
int v_bucket(int v) {
    int b = 0;
    while ((1 << b) < v) ++b;
    return b;
}

// The large-tile configuration (25) needs 32x32 MFMA blocks, which FP64
// lacks; FP64 runs configuration 6 in its place.
int cfg_for_prec(int prec, int cfg) { return (cfg == 25 && prec == CCSDT_FP64) ? 6 : cfg; }

int tile_cfg_for(const ccsdt_context* ctx, int prec, int v) {
    if (ctx->forced_cfg >= 0) return cfg_for_prec(prec, ctx->forced_cfg);
    int forced = env_int("CCSDT_TILE", -1);
    if (forced >= 0 && forced < NTILE_CFG) return cfg_for_prec(prec, forced);
    auto it = ctx->plans.find({prec, v_bucket(v)});
    if (it != ctx->plans.end()) return cfg_for_prec(prec, it->second);
    return v >= 64 ? 6 : 0;
}

struct ProbLayout {
    ccsdt_problem p;          // p.vvvo is null when G's particle part is DF-assembled
    const double* bvv;        // density-fitting factors (DF problems only)
    const double* bvo;
    int naux;
    bool vvvo_host;           // vvvo in pinned host memory: streamed through the staging ring
    int Kp;
    int cfg;
    size_t gc_off, tc_off;  // byte offsets in the pooled pack buffers
};

struct TripRef {
    int prob, i, j, k, mult, out_index;
};

struct Chunk {
    size_t first, n;  // slots [first, first + n)
    int totA, totE;   // contraction / energy workgroups
    int cfg;          // tile configuration (uniform inside a chunk)
};

// Everything a pipeline run needs besides the stream: problem layouts, the
// work list, its chunks and the slot table (host copy).
struct Plan {
    std::vector<ProbLayout> probs;
    std::vector<TripRef> trips;
    std::vector<Chunk> chunks;
    std::vector<Slot> slots;
    size_t n_out = 0;     // rows of the per-triple energy buffer
    bool one_per_chunk = false;
};

int multiplicity(int i, int j, int k) {
    if (i == j && j == k) return 0;
    if (i == j || j == k || i == k) return 3;
    return 6;
}

int prepare_streaming(ccsdt_context* ctx, const Plan& P);
bool is_pinned_host_ptr(const void* p);

// Host phase: tile choice, pooled pack offsets, chunking by the W budget,
// workspace allocation and the slot table.  Launches nothing.
int plan_pipeline(ccsdt_context* ctx, Plan& P, int prec) {
    for (auto& L : P.probs) L.vvvo_host = L.p.vvvo && is_pinned_host_ptr(L.p.vvvo);
    CHK(prepare_streaming(ctx, P));
    size_t gc_total = 0, tc_total = 0;
    const size_t es = elem_bytes(prec);
    for (auto& L : P.probs) {
        const int64_t o = L.p.nocc, v = L.p.nvirt;
        L.Kp = round_up((int)(o + v), KPAD);
        L.cfg = tile_cfg_for(ctx, prec, (int)v);
        L.gc_off = gc_total;
        L.tc_off = tc_total;
        gc_total += (size_t)(o * v * v * L.Kp) * es;
        tc_total += (size_t)(o * o * v * L.Kp) * es;
        gc_total = (gc_total + 255) / 256 * 256;
        tc_total = (tc_total + 255) / 256 * 256;
    }
    // triples of one tile configuration next to each other, so that chunks
    // (which break where the configuration changes) stay few
    if (ctx->shuffle) {
        // test hook: any order of the work list gives the same energies
        std::mt19937_64 rng(ctx->shuffle);
        std::shuffle(P.trips.begin(), P.trips.end(), rng);
    }
    std::stable_sort(P.trips.begin(), P.trips.end(), [&](const TripRef& x, const TripRef& y) {
        return P.probs[x.prob].cfg < P.probs[y.prob].cfg;
    });
    CHK(ensure(ctx, ctx->gc, gc_total, "packed G"));
    CHK(ensure(ctx, ctx->tc, tc_total, "packed T"));
    CHK(ensure(ctx, ctx->etrip, std::max<size_t>(P.n_out, 1) * 3 * sizeof(double), "per-triple energies"));

    const size_t wb = w_bytes(prec);
    auto w_of = [&](int v) {
        const size_t nb = (size_t)((v + WB - 1) / WB);
        return 2 * nb * nb * nb * WB * WB * WB * wb;   // W_A and W_B
    };
    size_t max_w = 0, max_part = 0;
    P.chunks.clear();
    for (size_t b = 0; b < P.trips.size();) {
        size_t e = b, wsum = 0, psum = 0;
        while (e < P.trips.size()) {
            const ProbLayout& L = P.probs[P.trips[e].prob];
            const int nb = (L.p.nvirt + WB - 1) / WB;
            const size_t wsz = w_of(L.p.nvirt);
            const size_t psz = (size_t)nb * (nb + 1) * (nb + 2) / 6 * 2 * sizeof(double);
            if (e > b && wsum + wsz > ctx->w_budget) break;
            if (e > b && L.cfg != P.probs[P.trips[b].prob].cfg) break;
            wsum += wsz;
            psum += psz;
            ++e;
            if (P.one_per_chunk) break;
        }
        P.chunks.push_back({b, e - b, 0, 0, P.probs[P.trips[b].prob].cfg});
        max_w = std::max(max_w, wsum);
        max_part = std::max(max_part, psum);
        b = e;
    }
    CHK(ensure(ctx, ctx->w, max_w, "W ring"));
    CHK(ensure(ctx, ctx->part, max_part, "energy partials"));
    CHK(ensure(ctx, ctx->slots, std::max<size_t>(P.trips.size(), 1) * sizeof(Slot), "slot table"));
    CHK(ensure(ctx, ctx->pace, PACE_BYTES, "pacing counters"));

    P.slots.assign(P.trips.size(), Slot{});
    for (auto& ch : P.chunks) {
        size_t woff = 0;
        int64_t poff = 0;
        for (size_t t = ch.first; t < ch.first + ch.n; ++t) {
            const TripRef& tr = P.trips[t];
            const ProbLayout& L = P.probs[tr.prob];
            const int v = L.p.nvirt;
            Slot& S = P.slots[t];
            std::memset(&S, 0, sizeof(Slot));
            S.i = tr.i; S.j = tr.j; S.k = tr.k; S.mult = tr.mult;
            // e_ijk is invariant under permutations of (i, j, k); a triple with
            // two equal indices is taken as (p, p, q), for which pass B is pass A
            // with a and b exchanged and is not run
            if (!P.one_per_chunk && tr.mult == 3) {
                if (tr.j == tr.k) { S.i = tr.j; S.j = tr.k; S.k = tr.i; }
                else if (tr.i == tr.k) { S.i = tr.i; S.j = tr.k; S.k = tr.j; }
            }
            S.o = L.p.nocc; S.v = v; S.Kp = L.Kp; S.prob = tr.prob;
            S.tiles_m = (v + tile_m(L.cfg) - 1) / tile_m(L.cfg);
            S.tiles_n = (v + tile_n(L.cfg) - 1) / tile_n(L.cfg);
            S.nbw = (v + WB - 1) / WB;
            const int norb = S.nbw * (S.nbw + 1) * (S.nbw + 2) / 6;
            S.bgroups = (v + tile_nbat(L.cfg) - 1) / tile_nbat(L.cfg);
            S.npass = (!P.one_per_chunk && S.i == S.j) ? 1 : 2;   // W of both passes for debug_w
            const int per = S.npass * S.bgroups * S.tiles_m * S.tiles_n;   // pass A then pass B
            S.a_begin = ch.totA; ch.totA += per;
            S.e_begin = ch.totE; ch.totE += norb;
            S.part_begin = poff; poff += norb;
            S.trip_index = tr.out_index;
            S.gc = static_cast<char*>(ctx->gc.p) + L.gc_off;
            S.tc = static_cast<char*>(ctx->tc.p) + L.tc_off;
            S.w = static_cast<char*>(ctx->w.p) + woff;
            woff += w_of(v);
            S.eps_o = L.p.eps_o; S.eps_v = L.p.eps_v; S.t1 = L.p.t1; S.ovov = L.p.ovov;
        }
    }
    return CCSDT_OK;
}

// Particle part of G from a host-resident (pinned) vvvo: chunks of whole
// rows y (v*v*o doubles each) are copied on the context's copy stream into
// two staging buffers in turn, and each is packed on stream s as soon as it
// has landed; a buffer is refilled only after the pack that read it.  The
// staging buffers are sized by CCSDT_STAGE_BYTES (both together, default
// 2 GiB, at least one row each).
// Rows per staging buffer for a problem streamed from host memory.
int stage_rows(const ccsdt_context* ctx, int o, int v) {
    const size_t row = (size_t)v * v * o * sizeof(double);
    return (int)std::max<size_t>(1, std::min<size_t>((size_t)v, ctx->stage_budget / 2 / row));
}

// Staging buffers, copy stream and events for host-resident vvvo (host phase).
int prepare_streaming(ccsdt_context* ctx, const Plan& P) {
    size_t need = 0;
    for (const auto& L : P.probs)
        if (L.vvvo_host)
            need = std::max(need, 2 * (size_t)stage_rows(ctx, L.p.nocc, L.p.nvirt) * L.p.nvirt * L.p.nvirt *
                                      L.p.nocc * sizeof(double));
    if (!need) return CCSDT_OK;
    CHK(ensure(ctx, ctx->stage, need, "staging buffers"));
    if (!ctx->copy_stream) HIPCHK(hipStreamCreateWithFlags(&ctx->copy_stream, hipStreamNonBlocking));
    for (int b = 0; b < 2; ++b) {
        if (!ctx->ev_copy[b]) HIPCHK(hipEventCreateWithFlags(&ctx->ev_copy[b], hipEventDisableTiming));
        if (!ctx->ev_pack[b]) HIPCHK(hipEventCreateWithFlags(&ctx->ev_pack[b], hipEventDisableTiming));
    }
    if (!ctx->ev_start) HIPCHK(hipEventCreateWithFlags(&ctx->ev_start, hipEventDisableTiming));
    return CCSDT_OK;
}

int stream_pack(ccsdt_context* ctx, const ProbLayout& L, int prec, char* g, hipStream_t s) {
    const int o = L.p.nocc, v = L.p.nvirt;
    const size_t row = (size_t)v * v * o * sizeof(double);
    const int ny = stage_rows(ctx, o, v);
    // the copies start after the work already queued on s
    HIPCHK(hipEventRecord(ctx->ev_start, s));
    HIPCHK(hipStreamWaitEvent(ctx->copy_stream, ctx->ev_start, 0));
    const char* host = reinterpret_cast<const char*>(L.p.vvvo);
    char* stage = static_cast<char*>(ctx->stage.p);
    int c = 0;
    for (int y0 = 0; y0 < v; y0 += ny, ++c) {
        const int n = std::min(ny, v - y0);
        const int b = c & 1;
        char* buf = stage + (size_t)b * ny * row;
        if (c >= 2) HIPCHK(hipStreamWaitEvent(ctx->copy_stream, ctx->ev_pack[b], 0));
        HIPCHK(hipMemcpyAsync(buf, host + (size_t)y0 * row, (size_t)n * row, hipMemcpyHostToDevice,
                              ctx->copy_stream));
        HIPCHK(hipEventRecord(ctx->ev_copy[b], ctx->copy_stream));
        HIPCHK(hipStreamWaitEvent(s, ctx->ev_copy[b], 0));
        LAUNCH(K_PACK, launch_pack_particle_chunk(prec, o, v, L.Kp, reinterpret_cast<const double*>(buf), y0, n, g, s));
        HIPCHK(hipEventRecord(ctx->ev_pack[b], s));
        ctx->streamed_bytes += (int64_t)((size_t)n * row);
    }
    return CCSDT_OK;
}

// Device phase: upload of the slot table (from pinned ``host_slots``), the
// packs and every chunk's launches, all on stream s.  Nothing here allocates
// or synchronizes, so the phase can be captured into a graph.  With debug_w
// the (single) triple's W is widened into it instead of the energy.
int enqueue_pipeline(ccsdt_context* ctx, const Plan& P, int prec, hipStream_t s, const Slot* host_slots,
                     double* debug_w) {
    if (!P.slots.empty())
        HIPCHK(hipMemcpyAsync(ctx->slots.p, host_slots, P.slots.size() * sizeof(Slot), hipMemcpyHostToDevice, s));
    for (const auto& L : P.probs) {
        char* g = static_cast<char*>(ctx->gc.p) + L.gc_off;
        char* t = static_cast<char*>(ctx->tc.p) + L.tc_off;
        const double* vvvo = L.p.vvvo;
        if (L.bvv)
            LAUNCH(K_ASSEMBLE, launch_assemble_df(prec, L.p.nocc, L.p.nvirt, L.naux, L.Kp, L.bvv, L.bvo, g, s));
        if (L.vvvo_host) {
            CHK(stream_pack(ctx, L, prec, g, s));
            vvvo = nullptr;
        }
        LAUNCH(K_PACK, launch_pack(prec, L.p.nocc, L.p.nvirt, L.Kp, vvvo, L.p.t2, L.p.ovoo, g, t, s));
    }
    const Slot* dslots = static_cast<const Slot*>(ctx->slots.p);
    double* part = static_cast<double*>(ctx->part.p);
    double* etrip = static_cast<double*>(ctx->etrip.p);
    for (const auto& ch : P.chunks) {
        const Slot* d = dslots + ch.first;
        const int n = (int)ch.n;
        LAUNCH(K_CONTRACT, launch_contract(prec, ch.cfg, d, n, ch.totA, static_cast<unsigned*>(ctx->pace.p), s));
        if (debug_w) {
            const Slot& S = P.slots[ch.first];
            LAUNCH(K_REDUCE, launch_widen_w(prec, S.w, S.v, debug_w, s));
            continue;
        }
        LAUNCH(K_ENERGY, launch_energy(prec, d, n, ch.totE, part, s));
        LAUNCH(K_REDUCE, launch_slot_reduce(d, n, part, etrip, s));
    }
    return CCSDT_OK;
}

// Plan + enqueue with the context's own pinned slot buffer (eager calls).
int run_pipeline(ccsdt_context* ctx, Plan& P, int prec, hipStream_t s, double* debug_w) {
    CHK(plan_pipeline(ctx, P, prec));
    const size_t n = std::max<size_t>(P.slots.size(), 1);
    CHK(ensure_host((void**)&ctx->host_slots, &ctx->host_slots_bytes, n * sizeof(Slot)));
    // the previous call's upload from this buffer finished before it returned
    if (!P.slots.empty()) std::memcpy(ctx->host_slots, P.slots.data(), P.slots.size() * sizeof(Slot));
    return enqueue_pipeline(ctx, P, prec, s, ctx->host_slots, debug_w);
}

// Work list of whole problems: every triple i<=j<=k with m != 0, problem by
// problem; trip_begin[p] .. trip_begin[p+1] are problem p's rows.
void whole_problem_plan(Plan& P, int nprob, const ccsdt_problem* probs, std::vector<int>& trip_begin) {
    P.probs.assign(nprob, ProbLayout{});
    P.trips.clear();
    trip_begin.assign(nprob + 1, 0);
    for (int p = 0; p < nprob; ++p) {
        P.probs[p].p = probs[p];
        P.probs[p].vvvo_host = is_pinned_host_ptr(probs[p].vvvo);
        const int o = probs[p].nocc;
        trip_begin[p] = (int)P.trips.size();
        for (int i = 0; i < o; ++i)
            for (int j = i; j < o; ++j)
                for (int k = j; k < o; ++k) {
                    const int m = multiplicity(i, j, k);
                    if (m) P.trips.push_back({p, i, j, k, m, (int)P.trips.size()});
                }
    }
    trip_begin[nprob] = (int)P.trips.size();
    P.n_out = P.trips.size();
}

// ---- captured graphs (batched submissions) ------------------------------------
void graph_reset(GraphEntry& G) {
    if (G.exec) (void)hipGraphExecDestroy(G.exec);
    if (G.graph) (void)hipGraphDestroy(G.graph);
    G.exec = nullptr;
    G.graph = nullptr;
    G.valid = false;
    G.probs.clear();
}

bool graph_matches(const ccsdt_context* ctx, int nprob, const ccsdt_problem* probs, int prec) {
    const GraphEntry& G = ctx->graph;
    return G.valid && G.prec == prec && G.gen == ctx->gen && (int)G.probs.size() == nprob &&
           std::memcmp(G.probs.data(), probs, sizeof(ccsdt_problem) * nprob) == 0;
}

// Pinned host block of a graph: slot table | trip_begin | gap descriptors | out.
struct GraphHostLayout {
    size_t slots_off, tb_off, desc_off, out_off, bytes;
};

GraphHostLayout graph_host_layout(size_t nslot, int nprob) {
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    GraphHostLayout h;
    h.slots_off = 0;
    h.tb_off = al(std::max<size_t>(nslot, 1) * sizeof(Slot));
    h.desc_off = h.tb_off + al(sizeof(int) * (nprob + 1));
    h.out_off = h.desc_off + al(sizeof(GapDesc) * nprob);
    h.bytes = h.out_off + al(sizeof(double) * 4 * nprob);
    return h;
}

// Device work of one batched submission: gap flags, the pipeline, the final
// per-problem reduce and the copy of (E, E4, E5, flag) rows to pinned memory.
int enqueue_batched(ccsdt_context* ctx, const Plan& P, int nprob, int prec, hipStream_t s, char* host,
                    const GraphHostLayout& h) {
    double* out = static_cast<double*>(ctx->out.p);
    HIPCHK(hipMemcpyAsync(ctx->pdesc.p, host + h.desc_off, sizeof(GapDesc) * nprob, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ctx->tripbeg.p, host + h.tb_off, sizeof(int) * (nprob + 1), hipMemcpyHostToDevice, s));
    LAUNCH(K_REDUCE, launch_gap_check(static_cast<const GapDesc*>(ctx->pdesc.p), nprob, out + 3 * nprob, s));
    CHK(enqueue_pipeline(ctx, P, prec, s, reinterpret_cast<const Slot*>(host + h.slots_off), nullptr));
    LAUNCH(K_REDUCE, launch_final_reduce(static_cast<const int*>(ctx->tripbeg.p), nprob,
                                         static_cast<const double*>(ctx->etrip.p), out, s));
    HIPCHK(hipMemcpyAsync(host + h.out_off, out, sizeof(double) * 4 * nprob, hipMemcpyDeviceToHost, s));
    return CCSDT_OK;
}

int capture_batched(ccsdt_context* ctx, const Plan& P, int nprob, int prec, char* host, const GraphHostLayout& h) {
    GraphEntry& G = ctx->graph;
    if (!ctx->cap_stream) HIPCHK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_batched(ctx, P, nprob, prec, ctx->cap_stream, host, h);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(ctx->cap_stream, &graph);
    if (rc != CCSDT_OK || e != hipSuccess) {
        (void)hipGetLastError();
        if (graph) (void)hipGraphDestroy(graph);
        return rc != CCSDT_OK ? rc : fail(CCSDT_EHIP, std::string("graph capture failed: ") + hipGetErrorString(e));
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        (void)hipGraphDestroy(graph);
        return fail(CCSDT_EHIP, std::string("graph instantiation failed: ") + hipGetErrorString(e));
    }
    G.graph = graph;
    G.exec = exec;
    return CCSDT_OK;
}

int check_flags(const double* flags, int nprob) {
    for (int p = 0; p < nprob; ++p) {
        const std::string where = nprob > 1 ? " (problem " + std::to_string(p) + ")" : std::string();
        if (flags[p] == 1.0) return fail(CCSDT_EINVAL, "non-finite orbital energy" + where);
        if (flags[p] != 0.0)
            return fail(CCSDT_EDENOM, "max(eps_o) >= min(eps_v): denominators must be negative" + where);
    }
    return CCSDT_OK;
}

// Batched submission through a captured graph.  The graph is rebuilt when
// the problem list, the precision or any workspace buffer (ctx->gen) changes,
// and replayed otherwise: a replay reads the inputs' current contents.
int energy_graph(ccsdt_context* ctx, int nprob, const ccsdt_problem* probs, int prec, hipStream_t s,
                 double* out_host) {
    GraphEntry& G = ctx->graph;
    if (!graph_matches(ctx, nprob, probs, prec)) {
        graph_reset(G);
        Plan P;
        std::vector<int> tb;
        whole_problem_plan(P, nprob, probs, tb);
        CHK(plan_pipeline(ctx, P, prec));
        CHK(ensure(ctx, ctx->tripbeg, sizeof(int) * (nprob + 1), "triple ranges"));
        CHK(ensure(ctx, ctx->out, sizeof(double) * 4 * nprob, "result"));
        CHK(ensure(ctx, ctx->pdesc, sizeof(GapDesc) * nprob, "problem table"));
        const GraphHostLayout h = graph_host_layout(P.slots.size(), nprob);
        CHK(ensure_host(&G.host, &G.host_bytes, h.bytes));
        char* host = static_cast<char*>(G.host);
        if (!P.slots.empty()) std::memcpy(host + h.slots_off, P.slots.data(), P.slots.size() * sizeof(Slot));
        std::memcpy(host + h.tb_off, tb.data(), sizeof(int) * (nprob + 1));
        GapDesc* desc = reinterpret_cast<GapDesc*>(host + h.desc_off);
        for (int p = 0; p < nprob; ++p) desc[p] = {probs[p].eps_o, probs[p].eps_v, probs[p].nocc, probs[p].nvirt};
        CHK(capture_batched(ctx, P, nprob, prec, host, h));
        G.layout_out = h.out_off;
        G.prec = prec;
        G.probs.assign(probs, probs + nprob);
        G.gen = ctx->gen;
        G.valid = true;
        ctx->n_captures++;
    }
    HIPCHK(hipGraphLaunch(G.exec, s));
    HIPCHK(hipStreamSynchronize(s));
    ctx->n_replays++;
    const double* res = reinterpret_cast<const double*>(static_cast<char*>(G.host) + G.layout_out);
    CHK(check_flags(res + 3 * nprob, nprob));
    std::memcpy(out_host, res, sizeof(double) * 3 * nprob);
    return CCSDT_OK;
}

// ---- autotuning ------------------------------------------------------------------
// Contraction time (ms) of tile configuration cfg on the given triples.
int time_cfg(ccsdt_context* ctx, const ccsdt_problem* prob, int prec, int cfg, const std::vector<TripRef>& trips,
             hipStream_t s, double* ms) {
    const bool was = ctx->profile;
    ctx->profile = true;
    ctx->forced_cfg = cfg;
    const int64_t n0 = ctx->prof_n[K_CONTRACT];
    const double t0 = ctx->prof_ms[K_CONTRACT];
    prof_start_call(ctx);
    Plan P;
    P.probs.assign(1, ProbLayout{});
    P.probs[0].p = *prob;
    P.trips = trips;
    P.n_out = trips.size();
    int rc = run_pipeline(ctx, P, prec, s, nullptr);
    if (rc == CCSDT_OK) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            rc = fail(CCSDT_EHIP, std::string("autotune: ") + hipGetErrorString(e));
        }
    }
    if (rc == CCSDT_OK) rc = prof_collect(ctx);
    *ms = ctx->prof_ms[K_CONTRACT] - t0;
    // the tuning launches are not part of the caller's profile
    ctx->prof_n[K_CONTRACT] = n0;
    ctx->prof_ms[K_CONTRACT] = t0;
    ctx->forced_cfg = -1;
    ctx->profile = was;
    return rc;
}

}  // namespace

extern "C" {

const char* ccsdt_last_error(void) { return g_err.c_str(); }

double ccsdt_flops(int nocc, int nvirt) {
    const double o = nocc, v = nvirt;
    return (o * o * o - o) * (2.0 * v * v * v * v + 2.0 * o * v * v * v);
}

int ccsdt_context_create(ccsdt_context** ctx_out) {
    if (!ctx_out) return fail(CCSDT_EINVAL, "null ctx_out");
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(CCSDT_EUNSUPPORTED, std::string("device is ") + prop.gcnArchName + ", not gfx950");
    auto* ctx = new (std::nothrow) ccsdt_context();
    if (!ctx) return fail(CCSDT_ENOMEM, "host allocation failed");
    ctx->device = dev;
    ctx->cap = env_size("CCSDT_MAX_DEVICE_BYTES", 0);
    ctx->w_budget = env_size("CCSDT_W_BYTES", (size_t)4 << 30);
    ctx->stage_budget = env_size("CCSDT_STAGE_BYTES", (size_t)2 << 30);
    if (const char* f = std::getenv("CCSDT_FAIL_AT"))
        for (int c = 0; c < K_NCLASS; ++c)
            if (std::strcmp(f, KERNEL_CLASS_NAMES[c]) == 0) ctx->fail_at = c;
    ctx->shuffle = env_size("CCSDT_SHUFFLE", 0);
    *ctx_out = ctx;
    return CCSDT_OK;
}

int ccsdt_context_destroy(ccsdt_context* ctx) {
    if (!ctx) return fail(CCSDT_EINVAL, "null context");
    graph_reset(ctx->graph);
    if (ctx->graph.host) (void)hipHostFree(ctx->graph.host);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->copy_stream) {
        (void)hipStreamSynchronize(ctx->copy_stream);
        (void)hipStreamDestroy(ctx->copy_stream);
    }
    for (hipEvent_t e : {ctx->ev_copy[0], ctx->ev_copy[1], ctx->ev_pack[0], ctx->ev_pack[1], ctx->ev_start})
        if (e) (void)hipEventDestroy(e);
    if (ctx->stage.p) (void)hipFree(ctx->stage.p);
    DevBuf* bufs[] = {&ctx->gc, &ctx->tc, &ctx->w, &ctx->part, &ctx->etrip, &ctx->slots, &ctx->out, &ctx->tripbeg,
                      &ctx->pdesc, &ctx->pace};
    for (DevBuf* b : bufs)
        if (b->p) (void)hipFree(b->p);
    if (ctx->host_out) (void)hipHostFree(ctx->host_out);
    if (ctx->host_slots) (void)hipHostFree(ctx->host_slots);
    if (ctx->host_tb) (void)hipHostFree(ctx->host_tb);
    if (ctx->host_desc) (void)hipHostFree(ctx->host_desc);
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    delete ctx;
    return CCSDT_OK;
}

int ccsdt_profile_enable(ccsdt_context* ctx, int on) {
    if (!ctx) return fail(CCSDT_EINVAL, "null context");
    ctx->profile = on != 0;
    return CCSDT_OK;
}

int ccsdt_profile_reset(ccsdt_context* ctx) {
    if (!ctx) return fail(CCSDT_EINVAL, "null context");
    for (int c = 0; c < K_NCLASS; ++c) {
        ctx->prof_n[c] = 0;
        ctx->prof_ms[c] = 0.0;
    }
    return CCSDT_OK;
}

int ccsdt_profile_get(ccsdt_context* ctx, int cls, int64_t* launches, double* total_ms) {
    if (!ctx || !launches || !total_ms) return fail(CCSDT_EINVAL, "null argument");
    if (cls < 0 || cls >= K_NCLASS) return fail(CCSDT_EINVAL, "kernel class out of range");
    *launches = ctx->prof_n[cls];
    *total_ms = ctx->prof_ms[cls];
    return CCSDT_OK;
}

// Eager E(T) of the problems in P (work list already built, trip_begin per
// problem): pipeline, final reduce, copy of (E, E4, E5) rows to out_host.
// The denominator check runs on the device with the pipeline (one flag per
// problem next to its result row), so the call synchronizes once, at the
// end; a failed check leaves the outputs untouched.
static int eager_energy(ccsdt_context* ctx, Plan& P, const std::vector<int>& tb, int prec, hipStream_t s,
                        double* out_host) {
    const int nprob = (int)P.probs.size();
    CHK(ensure(ctx, ctx->tripbeg, sizeof(int) * (nprob + 1), "triple ranges"));
    CHK(ensure(ctx, ctx->out, sizeof(double) * 4 * nprob, "result"));
    CHK(ensure(ctx, ctx->pdesc, sizeof(GapDesc) * nprob, "problem table"));
    CHK(ensure_host((void**)&ctx->host_tb, &ctx->host_tb_bytes, sizeof(int) * (nprob + 1)));
    CHK(ensure_host((void**)&ctx->host_out, &ctx->host_out_bytes, sizeof(double) * 4 * nprob));
    CHK(ensure_host((void**)&ctx->host_desc, &ctx->host_desc_bytes, sizeof(GapDesc) * nprob));
    // the previous call's uploads from these buffers finished before it returned
    for (int p = 0; p < nprob; ++p)
        ctx->host_desc[p] = {P.probs[p].p.eps_o, P.probs[p].p.eps_v, P.probs[p].p.nocc, P.probs[p].p.nvirt};
    double* out = static_cast<double*>(ctx->out.p);
    HIPCHK(hipMemcpyAsync(ctx->pdesc.p, ctx->host_desc, sizeof(GapDesc) * nprob, hipMemcpyHostToDevice, s));
    LAUNCH(K_REDUCE, launch_gap_check(static_cast<const GapDesc*>(ctx->pdesc.p), nprob, out + 3 * nprob, s));
    CHK(run_pipeline(ctx, P, prec, s, nullptr));
    std::memcpy(ctx->host_tb, tb.data(), sizeof(int) * (nprob + 1));
    HIPCHK(hipMemcpyAsync(ctx->tripbeg.p, ctx->host_tb, sizeof(int) * (nprob + 1), hipMemcpyHostToDevice, s));
    LAUNCH(K_REDUCE, launch_final_reduce(static_cast<const int*>(ctx->tripbeg.p), nprob,
                                         static_cast<const double*>(ctx->etrip.p), out, s));
    HIPCHK(hipMemcpyAsync(ctx->host_out, out, sizeof(double) * 4 * nprob, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    CHK(prof_collect(ctx));
    CHK(check_flags(ctx->host_out + 3 * nprob, nprob));
    std::memcpy(out_host, ctx->host_out, sizeof(double) * 3 * nprob);
    return CCSDT_OK;
}

static int energy_many(ccsdt_context* ctx, int nprob, const ccsdt_problem* probs, int prec, void* stream,
                       double* out_host) {
    CHK(check_ctx(ctx));
    if (!out_host) return fail(CCSDT_EINVAL, "null output");
    if (nprob < 1 || !probs) return fail(CCSDT_EINVAL, "no problems");
    CHK(check_prec(prec));
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int p = 0; p < nprob; ++p) CHK(check_problem(&probs[p], nprob > 1 ? p : -1));
    bool any_host = false;
    for (int p = 0; p < nprob; ++p) any_host = any_host || is_pinned_host_ptr(probs[p].vvvo);
    if (nprob > 1 && !ctx->profile && !any_host && env_int("CCSDT_GRAPH", 1) != 0)
        return energy_graph(ctx, nprob, probs, prec, s, out_host);

    prof_start_call(ctx);
    Plan P;
    std::vector<int> tb;
    whole_problem_plan(P, nprob, probs, tb);
    return eager_energy(ctx, P, tb, prec, s, out_host);
}

// Validates a DF problem and turns it into the common problem description
// (vvvo null) plus the factor pointers.
static int df_layout(const ccsdt_problem_df* d, ProbLayout& L) {
    if (!d) return fail(CCSDT_EINVAL, "null problem");
    ccsdt_problem p{d->nocc, d->nvirt, d->eps_o, d->eps_v, d->t1, d->t2, nullptr, d->ovoo, d->ovov};
    CHK(check_problem(&p, -1, false));
    if (d->naux < 1 || d->naux > 65536) return fail(CCSDT_EINVAL, "naux must be in 1..65536");
    if (!d->bvv || !d->bvo) return fail(CCSDT_EINVAL, "null pointer bvv or bvo");
    if (!is_device_ptr(d->bvv) || !is_device_ptr(d->bvo)) return fail(CCSDT_EINVAL, "bvv or bvo is not a device pointer");
    L = ProbLayout{};
    L.p = p;
    L.bvv = d->bvv;
    L.bvo = d->bvo;
    L.naux = d->naux;
    return CCSDT_OK;
}

int ccsdt_energy(ccsdt_context* ctx, const ccsdt_problem* prob, int precision, void* hip_stream, double* out_host) {
    if (!prob) return fail(CCSDT_EINVAL, "null problem");
    return energy_many(ctx, 1, prob, precision, hip_stream, out_host);
}

int ccsdt_energy_df(ccsdt_context* ctx, const ccsdt_problem_df* prob, int precision, void* hip_stream,
                    double* out_host) {
    CHK(check_ctx(ctx));
    if (!out_host) return fail(CCSDT_EINVAL, "null output");
    CHK(check_prec(precision));
    ProbLayout L;
    CHK(df_layout(prob, L));
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    prof_start_call(ctx);
    Plan P;
    std::vector<int> tb;
    whole_problem_plan(P, 1, &L.p, tb);
    P.probs[0] = L;
    return eager_energy(ctx, P, tb, precision, s, out_host);
}

int ccsdt_energy_batched(ccsdt_context* ctx, int nprob, const ccsdt_problem* probs_host, int precision,
                         void* hip_stream, double* out_host) {
    return energy_many(ctx, nprob, probs_host, precision, hip_stream, out_host);
}

int ccsdt_triples_energy(int nocc, int nvirt, const double* eps_o, const double* eps_v, const double* t1,
                         const double* t2, const double* vvvo, const double* ovoo, const double* ovov,
                         int precision, void* hip_stream, double* e_out) {
    if (!e_out) return fail(CCSDT_EINVAL, "null e_out");
    ccsdt_problem p{nocc, nvirt, eps_o, eps_v, t1, t2, vvvo, ovoo, ovov};
    ccsdt_context* ctx = nullptr;
    CHK(ccsdt_context_create(&ctx));
    double out[3];
    int rc = ccsdt_energy(ctx, &p, precision, hip_stream, out);
    std::string msg = g_err;
    ccsdt_context_destroy(ctx);
    if (rc != CCSDT_OK) return fail(rc, msg);
    *e_out = out[0];
    return CCSDT_OK;
}

// ---- allocation-free entry point ----------------------------------------------
// gfx950 check of a device, once per device.
static int noalloc_check_arch(int dev) {
    static std::mutex mu;
    static signed char state[64] = {};   // 0 unknown, 1 gfx950, -1 other
    if (dev < 0 || dev >= 64) return fail(CCSDT_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lock(mu);
    if (state[dev] == 0) {
        hipDeviceProp_t prop;
        HIPCHK(hipGetDeviceProperties(&prop, dev));
        state[dev] = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : -1;
    }
    if (state[dev] < 0) return fail(CCSDT_EUNSUPPORTED, "device is not gfx950");
    return CCSDT_OK;
}

static_assert(NOALLOC_SCRATCH_BYTES == CCSDT_NOALLOC_SCRATCH_BYTES, "workspace size of the header and the library");

int ccsdt_energy_noalloc(const ccsdt_problem* prob, int precision, void* hip_stream, double* out_dev) {
    if (!prob) return fail(CCSDT_EINVAL, "null problem");
    if (!out_dev) return fail(CCSDT_EINVAL, "null output");
    CHK(check_prec(precision));
    CHK(check_problem(prob, -1));
    if (is_pinned_host_ptr(prob->vvvo))
        return fail(CCSDT_EINVAL, "vvvo must be device memory for the allocation-free call");
    if (!is_device_ptr(out_dev)) return fail(CCSDT_EINVAL, "out_dev is not a device pointer");
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    CHK(noalloc_check_arch(dev));
    void* base = nullptr;
    {
        const hipError_t e = noalloc_scratch(dev, &base);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(CCSDT_EHIP, std::string("workspace symbol lookup failed: ") + hipGetErrorString(e));
        }
    }
    const int prec = precision;
    const int64_t o = prob->nocc, v = prob->nvirt;
    const int Kp = round_up((int)(o + v), KPAD);
    int cfg = env_int("CCSDT_TILE", -1);
    if (cfg < 0 || cfg >= NTILE_CFG || cfg == 24) cfg = v >= 64 ? 6 : 0;   // 24 needs its own counters
    cfg = cfg_for_prec(prec, cfg);
    const int64_t ntrip = o * (o + 1) * (o + 2) / 6 - o;
    const int nb = (int)((v + WB - 1) / WB);
    const int64_t norb = (int64_t)nb * (nb + 1) * (nb + 2) / 6;
    const int tiles_m = (int)((v + tile_m(cfg) - 1) / tile_m(cfg)), tiles_n = (int)((v + tile_n(cfg) - 1) / tile_n(cfg));
    const int bgroups = (int)((v + tile_nbat(cfg) - 1) / tile_nbat(cfg));
    const int64_t per_wg = 2 * (int64_t)bgroups * tiles_m * tiles_n;
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t es = elem_bytes(prec);
    const size_t slots_b = al((size_t)std::max<int64_t>(ntrip, 1) * sizeof(Slot));
    const size_t tb_b = al(2 * sizeof(int)), desc_b = al(sizeof(GapDesc)), flag_b = al(sizeof(double));
    const size_t etrip_b = al((size_t)std::max<int64_t>(ntrip, 1) * 3 * sizeof(double));
    const size_t gc_b = al((size_t)(o * v * v * Kp) * es), tc_b = al((size_t)(o * o * v * Kp) * es);
    const size_t w_per = al(2 * (size_t)nb * nb * nb * WB * WB * WB * w_bytes(prec));
    const size_t part_per = al((size_t)norb * 2 * sizeof(double));
    const size_t fixed = slots_b + tb_b + desc_b + flag_b + etrip_b + gc_b + tc_b;
    const size_t need_one = fixed + (ntrip > 0 ? w_per + part_per : 0);
    if (need_one > NOALLOC_SCRATCH_BYTES)
        return fail(CCSDT_EINVAL, "problem needs " + std::to_string(need_one) + " bytes of workspace; the "
                                  "allocation-free call has " + std::to_string(NOALLOC_SCRATCH_BYTES));
    int64_t chunk = ntrip > 0 ? (int64_t)((NOALLOC_SCRATCH_BYTES - fixed) / (w_per + part_per)) : 1;
    chunk = std::max<int64_t>(1, std::min<int64_t>(chunk, std::max<int64_t>(ntrip, 1)));
    // keep every flattened grid inside int32
    chunk = std::min<int64_t>(chunk, std::max<int64_t>(1, (INT32_MAX / 2) / std::max<int64_t>(per_wg, norb)));

    char* p = static_cast<char*>(base);
    Slot* slots = reinterpret_cast<Slot*>(p);           p += slots_b;
    int* tb = reinterpret_cast<int*>(p);                p += tb_b;
    GapDesc* desc = reinterpret_cast<GapDesc*>(p);      p += desc_b;
    double* flag = reinterpret_cast<double*>(p);        p += flag_b;
    double* etrip = reinterpret_cast<double*>(p);       p += etrip_b;
    char* gc = p;                                       p += gc_b;
    char* tc = p;                                       p += tc_b;
    double* part = reinterpret_cast<double*>(p);        p += (size_t)chunk * part_per;
    char* w = p;

    NoallocPlan np{};
    np.slots = slots; np.trip_begin = tb; np.desc = desc;
    np.ntrip = (int)ntrip; np.chunk = (int)chunk;
    np.o = (int)o; np.v = (int)v; np.Kp = Kp;
    np.tiles_m = tiles_m; np.tiles_n = tiles_n; np.nbw = nb; np.bgroups = bgroups;
    np.per_triple_wg = (int)per_wg; np.norb = (int)norb;
    np.gc = gc; np.tc = tc; np.w = w; np.w_bytes = w_per;
    np.eps_o = prob->eps_o; np.eps_v = prob->eps_v; np.t1 = prob->t1; np.ovov = prob->ovov;

    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    auto launched = [](hipError_t e, const char* what) {
        if (e == hipSuccess) return (int)CCSDT_OK;
        (void)hipGetLastError();
        return fail(CCSDT_EHIP, std::string("launch ") + what + ": " + hipGetErrorString(e));
    };
    CHK(launched(launch_noalloc_slots(np, s), "slot table"));
    CHK(launched(launch_gap_check(desc, 1, flag, s), "denominator check"));
    CHK(launched(launch_pack(prec, (int)o, (int)v, Kp, prob->vvvo, prob->t2, prob->ovoo, gc, tc, s), "pack"));
    for (int64_t c0 = 0; c0 < ntrip; c0 += chunk) {
        const int n = (int)std::min<int64_t>(chunk, ntrip - c0);
        const Slot* d = slots + c0;
        CHK(launched(launch_contract(prec, cfg, d, n, (int)(n * per_wg), nullptr, s), "contraction"));
        CHK(launched(launch_energy(prec, d, n, (int)(n * norb), part, s), "energy"));
        CHK(launched(launch_slot_reduce(d, n, part, etrip, s), "slot reduce"));
    }
    CHK(launched(launch_final_reduce(tb, 1, etrip, out_dev, s), "final reduce"));
    CHK(launched(launch_noalloc_finish(flag, out_dev, s), "finish"));
    return CCSDT_OK;
}

// Per-triple energies of one validated problem layout.
static int triple_energies_impl(ccsdt_context* ctx, const ProbLayout& L, int precision, int ntrip,
                                const int* ijk_host, void* hip_stream, double* out_host) {
    const int o = L.p.nocc;
    Plan P;
    std::vector<int> zero_rows;
    for (int t = 0; t < ntrip; ++t) {
        const int i = ijk_host[3 * t], j = ijk_host[3 * t + 1], k = ijk_host[3 * t + 2];
        if (!(0 <= i && i <= j && j <= k && k < o))
            return fail(CCSDT_EINVAL, "triple " + std::to_string(t) + " is not 0 <= i <= j <= k < nocc");
        const int m = multiplicity(i, j, k);
        if (m) P.trips.push_back({0, i, j, k, m, t});
        else zero_rows.push_back(t);
    }
    prof_start_call(ctx);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    CHK(check_gap(&L.p, s, -1));
    P.probs.assign(1, L);
    P.n_out = (size_t)ntrip;
    CHK(run_pipeline(ctx, P, precision, s, nullptr));
    CHK(ensure_host((void**)&ctx->host_out, &ctx->host_out_bytes, sizeof(double) * 3 * ntrip));
    HIPCHK(hipMemcpyAsync(ctx->host_out, ctx->etrip.p, sizeof(double) * 3 * ntrip, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    CHK(prof_collect(ctx));
    for (int t : zero_rows) ctx->host_out[3 * t] = ctx->host_out[3 * t + 1] = ctx->host_out[3 * t + 2] = 0.0;
    std::memcpy(out_host, ctx->host_out, sizeof(double) * 3 * ntrip);
    return CCSDT_OK;
}

int ccsdt_triple_energies(ccsdt_context* ctx, const ccsdt_problem* prob, int precision, int ntrip,
                          const int* ijk_host, void* hip_stream, double* out_host) {
    CHK(check_ctx(ctx));
    if (!out_host || !ijk_host) return fail(CCSDT_EINVAL, "null argument");
    if (ntrip < 1) return fail(CCSDT_EINVAL, "ntrip must be >= 1");
    CHK(check_prec(precision));
    CHK(check_problem(prob, -1));
    ProbLayout L{};
    L.p = *prob;
    L.vvvo_host = is_pinned_host_ptr(prob->vvvo);
    return triple_energies_impl(ctx, L, precision, ntrip, ijk_host, hip_stream, out_host);
}

int ccsdt_triple_energies_df(ccsdt_context* ctx, const ccsdt_problem_df* prob, int precision, int ntrip,
                             const int* ijk_host, void* hip_stream, double* out_host) {
    CHK(check_ctx(ctx));
    if (!out_host || !ijk_host) return fail(CCSDT_EINVAL, "null argument");
    if (ntrip < 1) return fail(CCSDT_EINVAL, "ntrip must be >= 1");
    CHK(check_prec(precision));
    ProbLayout L;
    CHK(df_layout(prob, L));
    return triple_energies_impl(ctx, L, precision, ntrip, ijk_host, hip_stream, out_host);
}

int ccsdt_debug_w(ccsdt_context* ctx, const ccsdt_problem* prob, int precision, int i, int j, int k,
                  void* hip_stream, double* w_host) {
    CHK(check_ctx(ctx));
    if (!w_host) return fail(CCSDT_EINVAL, "null w_host");
    CHK(check_prec(precision));
    CHK(check_problem(prob, -1));
    const int o = prob->nocc;
    if (!(0 <= i && i <= j && j <= k && k < o)) return fail(CCSDT_EINVAL, "need 0 <= i <= j <= k < nocc");
    prof_start_call(ctx);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int64_t v = prob->nvirt;
    Plan P;
    P.probs.assign(1, ProbLayout{});
    P.probs[0].p = *prob;
    P.trips = {{0, i, j, k, std::max(1, multiplicity(i, j, k)), 0}};
    P.n_out = 1;
    P.one_per_chunk = true;
    DevBuf tmp;
    const size_t bytes = (size_t)(v * v * v) * sizeof(double);
    hipError_t e = hipMalloc(&tmp.p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(CCSDT_ENOMEM, "hipMalloc for debug W failed");
    }
    int rc = run_pipeline(ctx, P, precision, s, static_cast<double*>(tmp.p));
    if (rc == CCSDT_OK) {
        e = hipMemcpyAsync(w_host, tmp.p, bytes, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            rc = fail(CCSDT_EHIP, std::string("copy of W failed: ") + hipGetErrorString(e));
        }
    } else {
        (void)hipStreamSynchronize(s);
        (void)hipGetLastError();
    }
    (void)hipFree(tmp.p);
    if (rc == CCSDT_OK) rc = prof_collect(ctx);
    return rc;
}

int ccsdt_autotune(ccsdt_context* ctx, const ccsdt_problem* prob, int precision, void* hip_stream, int* cfg_out) {
    CHK(check_ctx(ctx));
    CHK(check_prec(precision));
    CHK(check_problem(prob, -1));
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    CHK(check_gap(prob, s, -1));
    // up to four distinct triples (i<j<k) of the problem; two-equal triples
    // when nocc < 3
    const int o = prob->nocc;
    std::vector<TripRef> trips;
    for (int k = 2; k < o && trips.size() < 4; ++k) trips.push_back({0, 0, 1, k, 6, (int)trips.size()});
    for (int i = 0; i + 1 < o && trips.size() < 4; ++i) trips.push_back({0, i, i + 1, i + 1, 3, (int)trips.size()});
    if (trips.empty()) return fail(CCSDT_EINVAL, "nocc = 1 has no triples to time");
    int best = -1;
    double best_ms = 0.0;
    for (int cfg = 0; cfg < NTILE_CFG; ++cfg) {
        double ms = 0.0;
        CHK(time_cfg(ctx, prob, precision, cfg, trips, s, &ms));   // first run loads the kernel
        CHK(time_cfg(ctx, prob, precision, cfg, trips, s, &ms));
        if (best < 0 || ms < best_ms) {
            best = cfg;
            best_ms = ms;
        }
    }
    ctx->plans[{precision, v_bucket(prob->nvirt)}] = best;
    ++ctx->gen;   // captured graphs embed the tile choice
    if (cfg_out) *cfg_out = best;
    return CCSDT_OK;
}

int ccsdt_plan_get(ccsdt_context* ctx, int precision, int nvirt, int* cfg_out) {
    if (!ctx || !cfg_out) return fail(CCSDT_EINVAL, "null argument");
    CHK(check_prec(precision));
    if (nvirt < 1) return fail(CCSDT_EINVAL, "nvirt must be >= 1");
    *cfg_out = tile_cfg_for(ctx, precision, nvirt);
    return CCSDT_OK;
}

int ccsdt_plan_set(ccsdt_context* ctx, int precision, int nvirt, int cfg) {
    if (!ctx) return fail(CCSDT_EINVAL, "null context");
    CHK(check_prec(precision));
    if (nvirt < 1) return fail(CCSDT_EINVAL, "nvirt must be >= 1");
    if (cfg < -1 || cfg >= NTILE_CFG) return fail(CCSDT_EINVAL, "tile configuration out of range");
    if (cfg < 0) ctx->plans.erase({precision, v_bucket(nvirt)});
    else ctx->plans[{precision, v_bucket(nvirt)}] = cfg;
    ++ctx->gen;
    return CCSDT_OK;
}

int ccsdt_graph_stats(ccsdt_context* ctx, int64_t* captures, int64_t* replays) {
    if (!ctx || !captures || !replays) return fail(CCSDT_EINVAL, "null argument");
    *captures = ctx->n_captures;
    *replays = ctx->n_replays;
    return CCSDT_OK;
}

// ---- RI-MP2 -----------------------------------------------------------------------
// Workspace reuse: gc = packed coefficients, w = G_ij pair buffer, part =
// energy partials, slots = pair table (int2) followed by pair indices (int),
// etrip = pair energies, out = result.
static int mp2_check(const ccsdt_mp2_problem* p) {
    if (!p) return fail(CCSDT_EINVAL, "null problem");
    if (p->nocc < 1 || p->nvirt < 1 || p->naux < 1) return fail(CCSDT_EINVAL, "nocc, nvirt and naux must be >= 1");
    if (p->nocc > 1024 || p->nvirt > 8192 || p->naux > 65536)
        return fail(CCSDT_EINVAL, "nocc > 1024, nvirt > 8192 or naux > 65536");
    const double* ptrs[3] = {p->eps_o, p->eps_v, p->c_ov};
    const char* names[3] = {"eps_o", "eps_v", "c_ov"};
    for (int n = 0; n < 3; ++n) {
        if (!ptrs[n]) return fail(CCSDT_EINVAL, std::string("null pointer ") + names[n]);
        if (!is_device_ptr(ptrs[n])) return fail(CCSDT_EINVAL, std::string(names[n]) + " is not a device pointer");
    }
    return CCSDT_OK;
}

// Runs the pairs (i <= j) in ``pairs``; pair p's energy e_ij lands in
// etrip[p]; with ``total`` the weighted sum lands in out[0].
static int mp2_run(ccsdt_context* ctx, const ccsdt_mp2_problem* p, int prec, const std::vector<int2>& pairs,
                   bool total, hipStream_t s) {
    const int o = p->nocc, v = p->nvirt, naux = p->naux;
    const int Kq = round_up(naux, KPAD);
    const size_t es = elem_bytes(prec), wb = w_bytes(prec);
    const size_t np = pairs.size();
    const size_t per_slot = (size_t)v * v * wb;
    const size_t nc = std::max<size_t>(1, std::min(np, ctx->w_budget / per_slot));
    const int te = (v + 63) / 64;
    const size_t npt = (size_t)te * (te + 1) / 2;
    CHK(ensure(ctx, ctx->gc, (size_t)o * v * Kq * es, "packed coefficients"));
    CHK(ensure(ctx, ctx->w, nc * per_slot, "pair buffer"));
    CHK(ensure(ctx, ctx->part, nc * npt * sizeof(double), "energy partials"));
    const size_t tab = np * sizeof(int2) + np * sizeof(int);
    CHK(ensure(ctx, ctx->slots, tab, "pair table"));
    CHK(ensure(ctx, ctx->etrip, np * sizeof(double), "pair energies"));
    CHK(ensure(ctx, ctx->out, 4 * sizeof(double), "result"));
    CHK(ensure_host((void**)&ctx->host_slots, &ctx->host_slots_bytes, tab));
    char* h = reinterpret_cast<char*>(ctx->host_slots);
    std::memcpy(h, pairs.data(), np * sizeof(int2));
    int* hidx = reinterpret_cast<int*>(h + np * sizeof(int2));
    for (size_t q = 0; q < np; ++q) hidx[q] = (int)q;
    HIPCHK(hipMemcpyAsync(ctx->slots.p, h, tab, hipMemcpyHostToDevice, s));
    const int2* dpairs = static_cast<const int2*>(ctx->slots.p);
    const int* didx = reinterpret_cast<const int*>(static_cast<char*>(ctx->slots.p) + np * sizeof(int2));
    LAUNCH(K_PACK, launch_mp2_pack(prec, o, v, naux, Kq, p->c_ov, ctx->gc.p, s));
    for (size_t c0 = 0; c0 < np; c0 += nc) {
        const int n = (int)std::min(nc, np - c0);
        LAUNCH(K_MP2_GEMM, launch_mp2_gemm(prec, ctx->gc.p, dpairs + c0, n, v, Kq, ctx->w.p, s));
        LAUNCH(K_MP2_ENERGY, launch_mp2_energy(prec, ctx->w.p, dpairs + c0, n, p->eps_o, p->eps_v, v,
                                               static_cast<double*>(ctx->part.p), didx + c0,
                                               static_cast<double*>(ctx->etrip.p), s));
    }
    if (total)
        LAUNCH(K_REDUCE, launch_mp2_final(static_cast<const double*>(ctx->etrip.p), dpairs, (int)np,
                                          static_cast<double*>(ctx->out.p), s));
    return CCSDT_OK;
}

int ccsdt_rimp2_energy(ccsdt_context* ctx, const ccsdt_mp2_problem* prob, int precision, void* hip_stream,
                       double* e_out) {
    CHK(check_ctx(ctx));
    if (!e_out) return fail(CCSDT_EINVAL, "null output");
    CHK(check_prec(precision));
    CHK(mp2_check(prob));
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    prof_start_call(ctx);
    ccsdt_problem q{prob->nocc, prob->nvirt, prob->eps_o, prob->eps_v, nullptr, nullptr, nullptr, nullptr, nullptr};
    CHK(check_gap(&q, s, -1));
    std::vector<int2> pairs;
    for (int i = 0; i < prob->nocc; ++i)
        for (int j = i; j < prob->nocc; ++j) pairs.push_back(make_int2(i, j));
    CHK(mp2_run(ctx, prob, precision, pairs, true, s));
    CHK(ensure_host((void**)&ctx->host_out, &ctx->host_out_bytes, sizeof(double)));
    HIPCHK(hipMemcpyAsync(ctx->host_out, ctx->out.p, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    CHK(prof_collect(ctx));
    *e_out = ctx->host_out[0];
    return CCSDT_OK;
}

int ccsdt_rimp2_pair_energies(ccsdt_context* ctx, const ccsdt_mp2_problem* prob, int precision, int npair,
                              const int* ij_host, void* hip_stream, double* out_host) {
    CHK(check_ctx(ctx));
    if (!out_host || !ij_host) return fail(CCSDT_EINVAL, "null argument");
    if (npair < 1) return fail(CCSDT_EINVAL, "npair must be >= 1");
    CHK(check_prec(precision));
    CHK(mp2_check(prob));
    std::vector<int2> pairs;
    for (int q = 0; q < npair; ++q) {
        const int i = ij_host[2 * q], j = ij_host[2 * q + 1];
        if (!(0 <= i && i <= j && j < prob->nocc))
            return fail(CCSDT_EINVAL, "pair " + std::to_string(q) + " is not 0 <= i <= j < nocc");
        pairs.push_back(make_int2(i, j));
    }
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    prof_start_call(ctx);
    ccsdt_problem q{prob->nocc, prob->nvirt, prob->eps_o, prob->eps_v, nullptr, nullptr, nullptr, nullptr, nullptr};
    CHK(check_gap(&q, s, -1));
    CHK(mp2_run(ctx, prob, precision, pairs, false, s));
    CHK(ensure_host((void**)&ctx->host_out, &ctx->host_out_bytes, sizeof(double) * npair));
    HIPCHK(hipMemcpyAsync(ctx->host_out, ctx->etrip.p, sizeof(double) * npair, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    CHK(prof_collect(ctx));
    std::memcpy(out_host, ctx->host_out, sizeof(double) * npair);
    return CCSDT_OK;
}

double ccsdt_rimp2_flops(int nocc, int nvirt, int naux) {
    const double o = nocc, v = nvirt, q = naux;
    return o * (o + 1) / 2 * 2.0 * v * v * q;
}

}  // extern "C"
