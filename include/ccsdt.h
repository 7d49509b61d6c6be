/*
 * ccsdt.h -- closed-shell CCSD(T) perturbative-triples energy on AMD MI355X
 * (gfx950), C ABI.
 *
 * The operation (Eriksen, arXiv:1609.08094, Sec. 2.2):
 *
 *   E(T) = E[4] + E[5]           (eq. piecuch_4th_and_5th_order)
 *
 * over canonical Hartree-Fock spatial orbitals, occupied i,j,k,l and virtual
 * a,b,c,d.  For every occupied triple the library forms the connected
 * quantity (eq. analytical_triples_ampl, symmetrized by eq. symm_operator)
 *
 *   W^abc_ijk = P^abc_ijk [ sum_d (bd|ai) t^cd_kj - sum_l (kc|jl) t^ab_il ]
 *
 * the disconnected numerator (eq. piecuch_z_coefficients)
 *
 *   Z^abc_ijk = t^a_i (jb|kc) + t^b_j (ia|kc) + t^c_k (ia|jb),   V = W + Z,
 *
 * and the denominator-weighted energy with the tilde combination of eq.
 * piecuch_tilde_quantity, evaluated over restricted triples i<=j<=k (Sec. 3,
 * task count eq. tasks_ccsdpt) in the equivalent symmetrized form
 *
 *   e_ijk = m_ijk/3 sum_abc W_abc [4V_abc + V_bca + V_cab - 2V_acb - 2V_bac - 2V_cba] / D_abc
 *   D_abc = e_i + e_j + e_k - e_a - e_b - e_c  (< 0),  m = 6 (i<j<k), 3 (two equal),
 *
 * E[4] is the same sum with V replaced by W and E[5] with V replaced by Z.
 * The sign convention of the denominator (negative D, so that E[4] <= 0) is
 * the reading of the paper this library follows.
 *
 * Inputs (all float64, C row-major, real orbitals, Mulliken notation (pq|rs)):
 *   eps_o[o]            occupied orbital energies
 *   eps_v[v]            virtual orbital energies
 *   t1[i][a]            = t^a_i                           (o*v)
 *   t2[i][j][a][b]      = t^ab_ij                         (o*o*v*v)
 *   vvvo[a][b][c][i]    = (ab|ci)                         (v*v*v*o)
 *   ovoo[i][a][j][k]    = (ia|jk)                         (o*v*o*o)
 *   ovov[i][a][j][b]    = (ia|jb)                         (o*v*o*v)
 * The elements read are exactly (bd|ai) = vvvo[b][d][a][i],
 * (kc|jl) = ovoo[k][c][j][l] and (jb|kc) = ovov[j][b][k][c]; no further
 * symmetry of the inputs is assumed.
 *
 * Entry points (names of the first draft of this interface in brackets):
 *   ccsdt_triples_energy          one problem, one-shot (own temporary context)
 *   ccsdt_energy                  one problem on a context, (E, E[4], E[5])
 *                                 [ccsdt_triples_energy_ctx]
 *   ccsdt_energy_batched          many problems on a context, one captured graph
 *                                 [ccsdt_triples_energy_batched; that draft had no
 *                                 context argument]
 *   ccsdt_triple_energies         per-triple partials of listed triples
 *                                 [ccsdt_triple_partials; here with the problem
 *                                 and precision passed again, not cached]
 *   ccsdt_debug_w                 W of one triple (problem, precision, stream
 *                                 added to the draft's signature)
 *   ccsdt_energy_noalloc          one problem, no allocation, result on the device
 *   ccsdt_energy_df, ccsdt_triple_energies_df   density-fitted (vv|vo)
 *   ccsdt_rimp2_energy, ccsdt_rimp2_pair_energies, ccsdt_rimp2_flops   RI-MP2
 *   ccsdt_autotune, ccsdt_plan_get, ccsdt_plan_set   tile plans
 *   ccsdt_graph_stats, ccsdt_profile_*, ccsdt_flops, ccsdt_last_error
 *
 * Memory and ownership: every input pointer is a DEVICE pointer (for example
 * the data pointer of a contiguous torch.float64 tensor on the HIP device),
 * except that vvvo, the largest block (o*v^3), may instead be page-locked
 * HOST memory (hipHostMalloc, or a torch tensor created with pin_memory):
 * the library then streams it in chunks of whole rows vvvo[y] through two
 * device staging buffers (CCSDT_STAGE_BYTES for both, default 2 GiB), the
 * copy of one chunk overlapping the packing of the previous one (Sec. 3:
 * tiles of the integrals staged from pinned host memory), and keeps only
 * the packed operand on the device.  Pageable host memory is rejected.
 * The caller owns the inputs; the library only reads them, during the call,
 * and never frees or retains them.  Outputs named *_host are host pointers.
 * Work runs on the HIP stream passed in (NULL = the default stream); every
 * call returns after its device work has finished.
 *
 * Precision: CCSDT_FP64 runs the contractions on FP64 MFMA; CCSDT_FP32 on
 * FP32 MFMA with FP32 accumulation (the paper's mixed-precision mode, Sec. 3:
 * single precision for the triples-amplitude products); CCSDT_BF16X3 splits
 * each operand x into hi = bf16(x), lo = bf16(x - hi) and accumulates
 * hi*hi + hi*lo + lo*hi on BF16 MFMA in FP32.  In every mode the
 * denominators, the t1 terms (from the caller's FP64 t1 and (jb|kc)) and
 * all energy sums are computed in FP64 (Sec. 4); in the FP32 and BF16X3
 * modes W is held in FP32.
 *
 * Errors: every function returns CCSDT_OK (0) or a negative status; on error
 * outputs are left untouched, nothing is leaked, no exception crosses the
 * ABI and the process is never aborted.  ccsdt_last_error() returns a
 * message describing the last non-zero status of the calling thread.
 */
#ifndef CCSDT_H
#define CCSDT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CCSDT_OK = 0,
    CCSDT_EINVAL = -1,        /* bad argument: null pointer, size < 1, overflow, bad index */
    CCSDT_ENOMEM = -2,        /* device allocation failed (or exceeded CCSDT_MAX_DEVICE_BYTES) */
    CCSDT_EHIP = -3,          /* a HIP runtime call failed */
    CCSDT_EUNSUPPORTED = -4,  /* unknown precision, or no gfx950 device */
    CCSDT_EDENOM = -5         /* max(eps_o) >= min(eps_v): a denominator is not negative */
};

typedef enum {
    CCSDT_FP64 = 0,
    CCSDT_FP32 = 1,
    CCSDT_BF16X3 = 2
} ccsdt_precision;

/* One (T) problem: sizes and device pointers to the seven input blocks,
 * laid out as described above. */
typedef struct ccsdt_problem {
    int nocc;
    int nvirt;
    const double* eps_o;
    const double* eps_v;
    const double* t1;
    const double* t2;
    const double* vvvo;
    const double* ovoo;
    const double* ovov;
} ccsdt_problem;

/* Opaque handle that keeps device workspace (packed operands, the W ring,
 * partial sums), the tile plan cache and captured graphs between calls.  A
 * context is bound to the device current at creation and must be used by
 * one thread at a time; a call that launches work while another device is
 * current fails with CCSDT_EINVAL. */
typedef struct ccsdt_context ccsdt_context;

int ccsdt_context_create(ccsdt_context** ctx_out);
int ccsdt_context_destroy(ccsdt_context* ctx);

/* E(T) of one problem (Sec. 2.2, eqs. piecuch_4th_and_5th_order through
 * piecuch_tilde_quantity, restricted triples of Sec. 3).
 * out_host[0] = E(T), out_host[1] = E[4], out_host[2] = E[5]  (Hartree). */
int ccsdt_energy(ccsdt_context* ctx, const ccsdt_problem* prob, int precision,
                 void* hip_stream, double* out_host);

/* One-shot convenience form of ccsdt_energy: creates and destroys a
 * temporary context; *e_out = E(T). */
int ccsdt_triples_energy(int nocc, int nvirt,
                         const double* eps_o, const double* eps_v,
                         const double* t1, const double* t2,
                         const double* vvvo, const double* ovoo, const double* ovov,
                         int precision, void* hip_stream, double* e_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that must not call hipMalloc): E(T) of one problem
 * as in ccsdt_energy, with no context, no device or pinned-host allocation
 * and no host synchronization.  Every workspace buffer (packed operands, W,
 * partial sums, the triple table) lives in one static device array of
 * CCSDT_NOALLOC_SCRATCH_BYTES per GPU, which the library holds until the
 * process ends.  Inputs as for ccsdt_energy, all in device memory (vvvo may
 * not be host memory here).  out_dev is a DEVICE pointer to 3 doubles that
 * receives (E(T), E[4], E[5]) when the stream reaches the end of the
 * enqueued work; the call itself only validates and enqueues.  If an orbital
 * energy is not finite or max(eps_o) >= min(eps_v), out_dev receives NaN
 * (the check runs on the device).  Tile configuration: the default of
 * ccsdt_energy (no tuned plans); both contraction passes run for every
 * triple, so results agree with ccsdt_energy to rounding, not bit for bit.
 * A problem whose workspace exceeds the array (packed operands
 * (o v^2 + o^2 v) roundup(o+v, 32) elements of 8 bytes in FP64 and 4
 * otherwise, plus the W of at least one triple, 2 ceil(v/16)^3 4096
 * elements) is rejected with CCSDT_EINVAL and a message giving the size it
 * needs.  All calls on one GPU share its array: calls that overlap on one
 * GPU (other streams, other threads) race and give wrong results; calls
 * ordered on one stream are safe. */
#define CCSDT_NOALLOC_SCRATCH_BYTES (256u << 20)
int ccsdt_energy_noalloc(const ccsdt_problem* prob, int precision, void* hip_stream,
                         double* out_dev);

/* Per-triple energies e_ijk (including the multiplicity m_ijk) of the
 * restricted triples listed in ijk_host[3*n] (each i<=j<=k< nocc; i=j=k
 * yields 0).  out_host[3*n] receives (e, e4, e5) per triple. */
int ccsdt_triple_energies(ccsdt_context* ctx, const ccsdt_problem* prob, int precision,
                          int ntrip, const int* ijk_host, void* hip_stream,
                          double* out_host);

/* W^abc_ijk (eq. analytical_triples_ampl bracket, symmetrized by eq.
 * symm_operator) of one triple i<=j<=k, copied to w_host[a][b][c] (v^3
 * doubles; widened from FP32 for the mixed precisions).  Test/debug aid. */
int ccsdt_debug_w(ccsdt_context* ctx, const ccsdt_problem* prob, int precision,
                  int i, int j, int k, void* hip_stream, double* w_host);

/* Many independent problems of uneven (nocc, nvirt) in one submission: the
 * triples of all problems form one work list (Sec. 3: the cycles of the
 * collapsed loop are independent), grouped by tile plan, and each
 * contraction launch takes triples of several problems at once.  The
 * submission runs as one captured HIP graph (see ccsdt_graph_stats).
 * out_host[3*p+0..2] = (E, E4, E5) of problem p.  A problem whose orbital
 * energies are not finite gives CCSDT_EINVAL, one with max(eps_o) >=
 * min(eps_v) CCSDT_EDENOM; both name the problem in ccsdt_last_error(). */
int ccsdt_energy_batched(ccsdt_context* ctx, int nprob, const ccsdt_problem* probs_host,
                         int precision, void* hip_stream, double* out_host);

/* Density-fitted form of a problem (paper Sec. 2.1, eq. eri_sym_decomp):
 * instead of the o*v^3 block vvvo, the caller passes the factors of
 *   (ab|ci) = sum_Q B^Q_ab B^Q_ci
 * with the auxiliary index fastest:
 *   bvv[a][b][Q] = B^Q_ab   (v*v*naux),   bvo[c][i][Q] = B^Q_ci   (v*o*naux).
 * The library assembles the (vv|vo) part of its packed operand on FP64
 * matrix cores (rounded to the working precision afterwards), so that
 * device memory holds B (C3: 5.5 GB) rather than vvvo (69 GB).  The other
 * fields mean what they mean in ccsdt_problem; 1 <= naux <= 65536. */
typedef struct ccsdt_problem_df {
    int nocc;
    int nvirt;
    int naux;
    const double* eps_o;
    const double* eps_v;
    const double* t1;
    const double* t2;
    const double* bvv;
    const double* bvo;
    const double* ovoo;
    const double* ovov;
} ccsdt_problem_df;

/* ccsdt_energy and ccsdt_triple_energies for a density-fitted problem. */
int ccsdt_energy_df(ccsdt_context* ctx, const ccsdt_problem_df* prob, int precision,
                    void* hip_stream, double* out_host);
int ccsdt_triple_energies_df(ccsdt_context* ctx, const ccsdt_problem_df* prob, int precision,
                             int ntrip, const int* ijk_host, void* hip_stream,
                             double* out_host);

/* ---- RI-MP2 (the paper's second kernel) --------------------------------
 * Closed-shell RI-MP2 correlation energy (Sec. 2.1, eq. mp2_energy with the
 * denominators of eq. e_orb_diff and the integrals of eq. eri_sym_decomp):
 *   E = - sum_ij sum_ab g_aibj (2 g_aibj - g_ajbi) / (e_a + e_b - e_i - e_j),
 *   g_aibj = sum_Q C^Q_ai C^Q_bj.
 * Input c_ov[i][a][Q] = C^Q_ai (o*v*naux float64, device, Q fastest): the
 * fitting coefficients of eq. fitting_coef, computed by the caller.
 * For each pair i <= j the library forms G_ij[a][b] = g_aibj as one matrix
 * product over Q (FP64 or FP32 MFMA; for CCSDT_BF16X3 the BF16 split with
 * all four products hi*hi + hi*lo + lo*hi + lo*lo, because the diagonal
 * g_aiai are sums of squares, on which dropping lo*lo is a one-signed bias;
 * the denominators and every sum in FP64) and
 * E = sum_i e_ii + 2 sum_{i<j} e_ij.
 * Limits: nocc <= 1024, nvirt <= 8192, naux <= 65536; CCSDT_EDENOM unless
 * max(eps_o) < min(eps_v). */
typedef struct ccsdt_mp2_problem {
    int nocc;
    int nvirt;
    int naux;
    const double* eps_o;
    const double* eps_v;
    const double* c_ov;
} ccsdt_mp2_problem;

/* *e_out = E_MP2 (Hartree). */
int ccsdt_rimp2_energy(ccsdt_context* ctx, const ccsdt_mp2_problem* prob, int precision,
                       void* hip_stream, double* e_out);
/* Pair energies e_ij = - sum_ab g_aibj (2 g_aibj - g_ajbi) / D for the npair
 * pairs ij_host[2*p], ij_host[2*p+1] (0 <= i <= j < nocc); out_host[npair]. */
int ccsdt_rimp2_pair_energies(ccsdt_context* ctx, const ccsdt_mp2_problem* prob, int precision,
                              int npair, const int* ij_host, void* hip_stream, double* out_host);
/* Flops of the pair products: o(o+1)/2 * 2 v^2 naux. */
double ccsdt_rimp2_flops(int nocc, int nvirt, int naux);

/* Tile plans.  The contraction kernel has NTILE = 25 tile configurations
 * (workgroup tile shape, operand staging through registers or LDS, direct
 * global-to-LDS loads, one or two batch indices per workgroup, fragment
 * prefetch, deep stage rings, persistent, paced persistent and eight-wave
 * workgroups, 16x16 or 32x32 MFMA output blocks), numbered 0..24.  The
 * context keeps one choice per (precision, nvirt bucket), a bucket spanning
 * nvirt in (2^(b-1), 2^b]; unset buckets use the built-in default.  The
 * environment variable CCSDT_TILE=<cfg> overrides every plan (testing aid);
 * CCSDT_PACE_LAG=<n> sets how many K stages the workgroups of one XCD may
 * drift apart in configuration 24 (default 2, 0 = unpaced), read once per
 * process.
 *
 * ccsdt_autotune times the contraction of every configuration on up to four
 * triples of ``prob`` (each twice, the second run counted) and stores the
 * fastest as the plan of prob's bucket; *cfg_out (may be NULL) receives it.
 * The timing launches do not count in the profile.  ccsdt_plan_get returns
 * the configuration a call with this nvirt would use; ccsdt_plan_set stores
 * one (cfg = -1 clears the bucket).  Changing a plan invalidates captured
 * graphs. */
int ccsdt_autotune(ccsdt_context* ctx, const ccsdt_problem* prob, int precision,
                   void* hip_stream, int* cfg_out);
int ccsdt_plan_get(ccsdt_context* ctx, int precision, int nvirt, int* cfg_out);
int ccsdt_plan_set(ccsdt_context* ctx, int precision, int nvirt, int cfg);

/* Graph reuse of ccsdt_energy_batched: with nprob > 1 and profiling off, the
 * whole submission (denominator check, packs, contractions, energies,
 * reductions and the result copy) is captured once into a HIP graph and
 * replayed while the problem list (sizes and pointers), the precision, the
 * plans and the context's workspace buffers stay the same.  A replay reads
 * the current contents of the inputs.  CCSDT_GRAPH=0 in the environment
 * disables capture.  ccsdt_graph_stats returns the number of captures and
 * replays since the context was created. */
int ccsdt_graph_stats(ccsdt_context* ctx, int64_t* captures, int64_t* replays);

/* Kernel timing: when enabled, every launch of each kernel class is bracketed
 * by HIP events on the launch stream, and ccsdt_profile_get returns the
 * number of launches and their summed duration (ms) since the last reset.
 * Classes: 0 pack, 1 contraction (both passes: the six permutation terms of
 * W for every triple of a chunk), 2 energy, 3 reductions, 4 DF assembly of
 * the (vv|vo) operand, 5 RI-MP2 pair products, 6 RI-MP2 pair energies. */
int ccsdt_profile_enable(ccsdt_context* ctx, int on);
int ccsdt_profile_get(ccsdt_context* ctx, int kernel_class, int64_t* launches,
                      double* total_ms);
int ccsdt_profile_reset(ccsdt_context* ctx);

/* Algorithmic flop count (o^3 - o)(2 v^4 + 2 o v^3) of the distinct
 * contractions under i<=j<=k symmetry, as a double. */
double ccsdt_flops(int nocc, int nvirt);

/* Message for the calling thread's last non-zero status ("" if none). */
const char* ccsdt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CCSDT_H */
