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

enum { K_PACK = 0, K_CONTRACT = 1, K_ENERGY = 2, K_REDUCE = 3, K_NCLASS = 4 };

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
    void* host = nullptr;      // pinned copies of the slot table, triple ranges and problem table
    size_t host_bytes = 0;
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

    size_t allocated() const {
        return gc.bytes + tc.bytes + w.bytes + part.bytes + etrip.bytes + slots.bytes + out.bytes + tripbeg.bytes +
               pdesc.bytes;
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

#define LAUNCH(cls, expr)                                                                         \
    do {                                                                                          \
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

int check_problem(const ccsdt_problem* p, int idx) {
    const std::string where = idx >= 0 ? " (problem " + std::to_string(idx) + ")" : "";
    if (!p) return fail(CCSDT_EINVAL, "null problem" + where);
    if (p->nocc < 1 || p->nvirt < 1) return fail(CCSDT_EINVAL, "nocc and nvirt must be >= 1" + where);
    // limits keep every flattened grid and slot offset inside int32
    if (p->nocc > 1024 || p->nvirt > 2048) return fail(CCSDT_EINVAL, "nocc > 1024 or nvirt > 2048" + where);
    const double* ptrs[7] = {p->eps_o, p->eps_v, p->t1, p->t2, p->vvvo, p->ovoo, p->ovov};
    const char* names[7] = {"eps_o", "eps_v", "t1", "t2", "vvvo", "ovoo", "ovov"};
    for (int n = 0; n < 7; ++n) {
        if (!ptrs[n]) return fail(CCSDT_EINVAL, std::string("null pointer ") + names[n] + where);
        if (!is_device_ptr(ptrs[n]))
            return fail(CCSDT_EINVAL, std::string(names[n]) + " is not a device pointer" + where);
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

int check_prec(int prec) {
    if (prec != CCSDT_FP64 && prec != CCSDT_FP32 && prec != CCSDT_BF16X3)
        return fail(CCSDT_EUNSUPPORTED, "unknown precision " + std::to_string(prec));
    return CCSDT_OK;
}

size_t elem_bytes(int prec) { return prec == CCSDT_FP64 ? 8 : 4; }   // packed element (hi+lo = 4)
size_t w_bytes(int prec) { return prec == CCSDT_FP64 ? 8 : 4; }

// ---- plans ---------------------------------------------------------------------
int tile_cfg_for(int prec, int v) {
    int forced = env_int("CCSDT_TILE", -1);
    if (forced >= 0 && forced < NTILE_CFG) return forced;
    (void)prec;
    return v >= 64 ? 6 : 0;
}

struct ProbLayout {
    ccsdt_problem p;
    int Kp;
    int cfg;
    size_t gc_off, tc_off;  // byte offsets in the pooled pack buffers
};

struct TripRef {
    int prob, i, j, k, mult, out_index;
};

int multiplicity(int i, int j, int k) {
    if (i == j && j == k) return 0;
    if (i == j || j == k || i == k) return 3;
    return 6;
}

// Packs every problem, then runs the chunked pipeline over ``trips``, leaving
// (e, e4, e5) of trip t in e_trip[3*trips[t].out_index].  If debug_w is set,
// the W of the single triple is widened into it (v^3 doubles, device).
int run_pipeline(ccsdt_context* ctx, std::vector<ProbLayout>& probs, const std::vector<TripRef>& trips, int prec,
                 hipStream_t s, size_t n_out, double* debug_w) {
    // pack buffers
    size_t gc_total = 0, tc_total = 0;
    const size_t es = elem_bytes(prec);
    for (auto& L : probs) {
        const int64_t o = L.p.nocc, v = L.p.nvirt;
        L.Kp = round_up((int)(o + v), KPAD);
        L.cfg = tile_cfg_for(prec, (int)v);
        L.gc_off = gc_total;
        L.tc_off = tc_total;
        gc_total += (size_t)(o * v * v * L.Kp) * es;
        tc_total += (size_t)(o * o * v * L.Kp) * es;
        gc_total = (gc_total + 255) / 256 * 256;
        tc_total = (tc_total + 255) / 256 * 256;
    }
    CHK(ensure(ctx, ctx->gc, gc_total, "packed G"));
    CHK(ensure(ctx, ctx->tc, tc_total, "packed T"));
    for (auto& L : probs) {
        char* g = static_cast<char*>(ctx->gc.p) + L.gc_off;
        char* t = static_cast<char*>(ctx->tc.p) + L.tc_off;
        LAUNCH(K_PACK, launch_pack(prec, L.p.nocc, L.p.nvirt, L.Kp, L.p.vvvo, L.p.t2, L.p.ovoo, g, t, s));
    }
    CHK(ensure(ctx, ctx->etrip, std::max<size_t>(n_out, 1) * 3 * sizeof(double), "per-triple energies"));

    // chunking by W budget
    const size_t wb = w_bytes(prec);
    std::vector<std::pair<size_t, size_t>> chunks;  // [begin, end) into trips
    size_t max_w = 0, max_part = 0;
    {
        size_t b = 0;
        while (b < trips.size()) {
            size_t e = b, wsum = 0, psum = 0;
            while (e < trips.size()) {
                const int64_t v = probs[trips[e].prob].p.nvirt;
                const int nb = (int)((v + WB - 1) / WB);
                const size_t wsz = 2 * (size_t)nb * nb * nb * WB * WB * WB * wb;   // W_A and W_B
                const size_t psz = (size_t)nb * (nb + 1) * (nb + 2) / 6 * 2 * sizeof(double);
                if (e > b && wsum + wsz > ctx->w_budget) break;
                if (e > b && probs[trips[e].prob].cfg != probs[trips[b].prob].cfg) break;
                wsum += wsz;
                psum += psz;
                ++e;
                if (debug_w) break;
            }
            chunks.push_back({b, e});
            max_w = std::max(max_w, wsum);
            max_part = std::max(max_part, psum);
            b = e;
        }
    }
    CHK(ensure(ctx, ctx->w, max_w, "W ring"));
    CHK(ensure(ctx, ctx->part, max_part, "energy partials"));
    const size_t nslot_total = trips.size();
    CHK(ensure(ctx, ctx->slots, std::max<size_t>(nslot_total, 1) * sizeof(Slot), "slot table"));
    CHK(ensure_host((void**)&ctx->host_slots, &ctx->host_slots_bytes, std::max<size_t>(nslot_total, 1) * sizeof(Slot)));

    // slot descriptors of every chunk, uploaded once
    struct ChunkInfo { size_t first, n; int totA, totE; int cfgs; };
    std::vector<ChunkInfo> cinfo;
    for (auto& ch : chunks) {
        ChunkInfo ci{ch.first, ch.second - ch.first, 0, 0, -1};
        size_t woff = 0;
        int64_t poff = 0;
        for (size_t t = ch.first; t < ch.second; ++t) {
            const TripRef& tr = trips[t];
            const ProbLayout& L = probs[tr.prob];
            const int v = L.p.nvirt;
            Slot& S = ctx->host_slots[t];
            std::memset(&S, 0, sizeof(Slot));
            S.i = tr.i; S.j = tr.j; S.k = tr.k; S.mult = tr.mult;
            S.o = L.p.nocc; S.v = v; S.Kp = L.Kp; S.prob = tr.prob;
            S.tiles_m = (v + tile_m(L.cfg) - 1) / tile_m(L.cfg);
            S.tiles_n = (v + tile_n(L.cfg) - 1) / tile_n(L.cfg);
            S.nbw = (v + WB - 1) / WB;
            const int norb = S.nbw * (S.nbw + 1) * (S.nbw + 2) / 6;
            const int per = 2 * v * S.tiles_m * S.tiles_n;   // pass A then pass B
            S.a_begin = ci.totA; ci.totA += per;
            S.b_begin = S.a_begin;
            S.e_begin = ci.totE; ci.totE += norb;
            S.part_begin = poff; poff += norb;
            S.trip_index = tr.out_index;
            S.gc = static_cast<char*>(ctx->gc.p) + L.gc_off;
            S.tc = static_cast<char*>(ctx->tc.p) + L.tc_off;
            S.w = static_cast<char*>(ctx->w.p) + woff;
            woff += 2 * (size_t)S.nbw * S.nbw * S.nbw * WB * WB * WB * wb;
            S.eps_o = L.p.eps_o; S.eps_v = L.p.eps_v; S.t1 = L.p.t1; S.ovov = L.p.ovov;
            ci.cfgs = L.cfg;  // uniform inside a chunk (chunks break where it changes)
        }
        cinfo.push_back(ci);
    }
    HIPCHK(hipMemcpyAsync(ctx->slots.p, ctx->host_slots, nslot_total * sizeof(Slot), hipMemcpyHostToDevice, s));
    const Slot* dslots = static_cast<const Slot*>(ctx->slots.p);
    double* part = static_cast<double*>(ctx->part.p);
    double* etrip = static_cast<double*>(ctx->etrip.p);
    for (auto& ci : cinfo) {
        const Slot* d = dslots + ci.first;
        const int n = (int)ci.n;
        const int cfg = ci.cfgs;
        LAUNCH(K_CONTRACT, launch_contract(prec, cfg, d, n, ci.totA, s));
        if (debug_w) {
            const int v = ctx->host_slots[ci.first].v;
            LAUNCH(K_REDUCE, launch_widen_w(prec, ctx->host_slots[ci.first].w, v, debug_w, s));
            continue;
        }
        LAUNCH(K_ENERGY, launch_energy(prec, d, n, ci.totE, part, s));
        LAUNCH(K_REDUCE, launch_slot_reduce(d, n, 0, part, etrip, s));
    }
    return CCSDT_OK;
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
    *ctx_out = ctx;
    return CCSDT_OK;
}

int ccsdt_context_destroy(ccsdt_context* ctx) {
    if (!ctx) return fail(CCSDT_EINVAL, "null context");
    DevBuf* bufs[] = {&ctx->gc, &ctx->tc, &ctx->w, &ctx->part, &ctx->etrip, &ctx->slots, &ctx->out, &ctx->tripbeg};
    for (DevBuf* b : bufs)
        if (b->p) (void)hipFree(b->p);
    if (ctx->host_out) (void)hipHostFree(ctx->host_out);
    if (ctx->host_slots) (void)hipHostFree(ctx->host_slots);
    if (ctx->host_tb) (void)hipHostFree(ctx->host_tb);
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

static int energy_many(ccsdt_context* ctx, int nprob, const ccsdt_problem* probs, int prec, void* stream,
                       double* out_host) {
    if (!ctx) return fail(CCSDT_EINVAL, "null context");
    if (!out_host) return fail(CCSDT_EINVAL, "null output");
    if (nprob < 1 || !probs) return fail(CCSDT_EINVAL, "no problems");
    CHK(check_prec(prec));
    prof_start_call(ctx);
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<ProbLayout> L(nprob);
    std::vector<TripRef> trips;
    std::vector<int> tb(nprob + 1, 0);
    for (int p = 0; p < nprob; ++p) {
        CHK(check_problem(&probs[p], nprob > 1 ? p : -1));
        CHK(check_gap(&probs[p], s, nprob > 1 ? p : -1));
        L[p].p = probs[p];
        const int o = probs[p].nocc;
        tb[p] = (int)trips.size();
        for (int i = 0; i < o; ++i)
            for (int j = i; j < o; ++j)
                for (int k = j; k < o; ++k) {
                    const int m = multiplicity(i, j, k);
                    if (m) trips.push_back({p, i, j, k, m, (int)trips.size()});
                }
    }
    tb[nprob] = (int)trips.size();
    CHK(run_pipeline(ctx, L, trips, prec, s, trips.size(), nullptr));
    CHK(ensure(ctx, ctx->tripbeg, sizeof(int) * (nprob + 1), "triple ranges"));
    CHK(ensure(ctx, ctx->out, sizeof(double) * 3 * nprob, "result"));
    CHK(ensure_host((void**)&ctx->host_tb, &ctx->host_tb_bytes, sizeof(int) * (nprob + 1)));
    CHK(ensure_host((void**)&ctx->host_out, &ctx->host_out_bytes, sizeof(double) * 3 * nprob));
    std::memcpy(ctx->host_tb, tb.data(), sizeof(int) * (nprob + 1));
    HIPCHK(hipMemcpyAsync(ctx->tripbeg.p, ctx->host_tb, sizeof(int) * (nprob + 1), hipMemcpyHostToDevice, s));
    LAUNCH(K_REDUCE, launch_final_reduce(static_cast<const int*>(ctx->tripbeg.p), nprob,
                                         static_cast<const double*>(ctx->etrip.p), static_cast<double*>(ctx->out.p), s));
    HIPCHK(hipMemcpyAsync(ctx->host_out, ctx->out.p, sizeof(double) * 3 * nprob, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    CHK(prof_collect(ctx));
    std::memcpy(out_host, ctx->host_out, sizeof(double) * 3 * nprob);
    return CCSDT_OK;
}

int ccsdt_energy(ccsdt_context* ctx, const ccsdt_problem* prob, int precision, void* hip_stream, double* out_host) {
    if (!prob) return fail(CCSDT_EINVAL, "null problem");
    return energy_many(ctx, 1, prob, precision, hip_stream, out_host);
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

int ccsdt_triple_energies(ccsdt_context* ctx, const ccsdt_problem* prob, int precision, int ntrip,
                          const int* ijk_host, void* hip_stream, double* out_host) {
    if (!ctx) return fail(CCSDT_EINVAL, "null context");
    if (!out_host || !ijk_host) return fail(CCSDT_EINVAL, "null argument");
    if (ntrip < 1) return fail(CCSDT_EINVAL, "ntrip must be >= 1");
    CHK(check_prec(precision));
    CHK(check_problem(prob, -1));
    prof_start_call(ctx);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    CHK(check_gap(prob, s, -1));
    const int o = prob->nocc;
    std::vector<TripRef> trips;
    std::vector<int> zero_rows;
    for (int t = 0; t < ntrip; ++t) {
        const int i = ijk_host[3 * t], j = ijk_host[3 * t + 1], k = ijk_host[3 * t + 2];
        if (!(0 <= i && i <= j && j <= k && k < o))
            return fail(CCSDT_EINVAL, "triple " + std::to_string(t) + " is not 0 <= i <= j <= k < nocc");
        const int m = multiplicity(i, j, k);
        if (m) trips.push_back({0, i, j, k, m, t});
        else zero_rows.push_back(t);
    }
    std::vector<ProbLayout> L(1);
    L[0].p = *prob;
    CHK(run_pipeline(ctx, L, trips, precision, s, (size_t)ntrip, nullptr));
    CHK(ensure_host((void**)&ctx->host_out, &ctx->host_out_bytes, sizeof(double) * 3 * ntrip));
    HIPCHK(hipMemcpyAsync(ctx->host_out, ctx->etrip.p, sizeof(double) * 3 * ntrip, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    CHK(prof_collect(ctx));
    for (int t : zero_rows) ctx->host_out[3 * t] = ctx->host_out[3 * t + 1] = ctx->host_out[3 * t + 2] = 0.0;
    std::memcpy(out_host, ctx->host_out, sizeof(double) * 3 * ntrip);
    return CCSDT_OK;
}

int ccsdt_debug_w(ccsdt_context* ctx, const ccsdt_problem* prob, int precision, int i, int j, int k,
                  void* hip_stream, double* w_host) {
    if (!ctx) return fail(CCSDT_EINVAL, "null context");
    if (!w_host) return fail(CCSDT_EINVAL, "null w_host");
    CHK(check_prec(precision));
    CHK(check_problem(prob, -1));
    const int o = prob->nocc;
    if (!(0 <= i && i <= j && j <= k && k < o)) return fail(CCSDT_EINVAL, "need 0 <= i <= j <= k < nocc");
    prof_start_call(ctx);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int64_t v = prob->nvirt;
    std::vector<ProbLayout> L(1);
    L[0].p = *prob;
    std::vector<TripRef> trips{{0, i, j, k, std::max(1, multiplicity(i, j, k)), 0}};
    DevBuf tmp;
    const size_t bytes = (size_t)(v * v * v) * sizeof(double);
    hipError_t e = hipMalloc(&tmp.p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(CCSDT_ENOMEM, "hipMalloc for debug W failed");
    }
    int rc = run_pipeline(ctx, L, trips, precision, s, 1, static_cast<double*>(tmp.p));
    if (rc == CCSDT_OK) {
        e = hipMemcpyAsync(w_host, tmp.p, bytes, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            rc = fail(CCSDT_EHIP, std::string("copy of W failed: ") + hipGetErrorString(e));
        }
    }
    (void)hipFree(tmp.p);
    if (rc == CCSDT_OK) rc = prof_collect(ctx);
    return rc;
}

}  // extern "C"
