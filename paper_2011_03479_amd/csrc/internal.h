// Internal declarations shared by the library's translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/gempe.h"

// Device-side status bits (gempe_graph_s::status_dev and the embed status word).
enum : unsigned {
    kStatusNonFinite = 1u,    // a loss partial or a coordinate was NaN/Inf
    kStatusReserved = 2u,     // unused
    kStatusBadRowPtr = 4u,    // row_ptr not monotone / out of [0, nnz]
    kStatusBadCol = 8u,       // column id out of range or a self-loop
    kStatusUnsorted = 16u,    // a row not strictly ascending (duplicate or unsorted)
    kStatusAsymmetric = 32u,  // (i, j) present without (j, i)
    kStatusHashFull = 64u,    // hash insertion found no free slot (cannot happen at LF <= 0.5)
};

struct gempe_graph_s {
    int32_t n = 0;
    int64_t nnz = 0;     // directed entries, 2m
    int64_t m = 0;       // undirected edges
    int device = 0;
    int64_t *row_ptr = nullptr;  // device copy, int64[n+1]
    int32_t *col_idx = nullptr;  // device copy, int32[nnz]
    int32_t *coo_row = nullptr;  // device, row id of every CSR entry, int32[nnz]
    unsigned long long *hash = nullptr;  // device, open addressing, capacity hash_cap
    uint64_t hash_cap = 0;       // power of two >= 2m (>= 2)
    unsigned *status_dev = nullptr;  // device words: [0] graph validation, [1] counters
    void *mem = nullptr;         // the one device block holding all of the above (caller's workspace)
    bool server_owned = false;   // carved from a server's arena (released by the server)
};

// Host-side size checks shared by gempe_graph_create and the server's submit.
gempe_status gempe_graph_check_args(int32_t n, int64_t nnz, const void *row_ptr, const void *col_idx,
                                    const char *who);
// Bytes of the device block of a graph (CSR copy, row ids, hash, status words).
size_t gempe_graph_mem_bytes(int32_t n, int64_t nnz);
// Copies (kind: device or host source) and validates a CSR into `mem` (gempe_graph_mem_bytes
// bytes, 256-B aligned) and fills *g.  Synchronises `stream`.
gempe_status gempe_graph_build(int32_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col_idx,
                               hipMemcpyKind kind, void *mem, hipStream_t stream, gempe_graph_s *g);

// Empty slot marker of the edge hash (keys are (min << 32) | max with min < max < 2^31).
constexpr unsigned long long kHashEmpty = ~0ull;

// Kernel timing brackets (timing.hip); the classes are gempe.h's GEMPE_TK_*.
enum { kTkSweep = GEMPE_TK_SWEEP, kTkGram = GEMPE_TK_GRAM, kTkExact = GEMPE_TK_EXACT, kTkEdges = GEMPE_TK_EDGES,
       kTkFull = GEMPE_TK_FULL, kTkClasses = 5 };
bool gempe_timing_on();
void gempe_timing_begin(int cls, hipStream_t s);
void gempe_timing_end(int cls, hipStream_t s, int launches);
// Scoped bracket: events on `s` before and after the launches made while it lives.
struct TimedLaunches {
    int cls;
    hipStream_t s;
    int launches;
    bool on;
    TimedLaunches(int c, hipStream_t st, int nl = 1) : cls(c), s(st), launches(nl), on(gempe_timing_on()) {
        if (on) gempe_timing_begin(cls, s);
    }
    ~TimedLaunches() {
        if (on) gempe_timing_end(cls, s, launches);
    }
};

// Host-side checks of (n, d, params) shared by every call (api.hip).
gempe_status gempe_check_problem(int32_t n, int32_t d, const gempe_params *p, const char *who);

// Thread-local error text (api.hip).
void gempe_set_error(const std::string &msg);
gempe_status gempe_fail(gempe_status s, const std::string &msg);

#define GEMPE_HIP_TRY(expr)                                                            \
    do {                                                                               \
        hipError_t _e = (expr);                                                        \
        if (_e != hipSuccess)                                                          \
            return gempe_fail(GEMPE_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

// 64-bit finaliser of SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): a bijective mix
// so that linear probing sees well-spread home slots for structured (i, j) keys.
__host__ __device__ inline unsigned long long gempe_mix64(unsigned long long x) {
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ull;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebull;
    x ^= x >> 31;
    return x;
}

__host__ __device__ inline unsigned long long gempe_edge_key(int a, int b) {
    unsigned lo = (unsigned)(a < b ? a : b), hi = (unsigned)(a < b ? b : a);
    return ((unsigned long long)lo << 32) | hi;
}

// Device-side exact membership probe (linear probing; the table is at most half full, so
// an empty slot ends every search; the loop bound is a safety net only).
__device__ inline bool gempe_hash_contains(const unsigned long long *__restrict__ table,
                                           unsigned long long cap, unsigned long long key) {
    unsigned long long mask = cap - 1, s = gempe_mix64(key) & mask;
    for (unsigned long long probe = 0; probe < cap; ++probe) {
        unsigned long long v = table[s];
        if (v == key) return true;
        if (v == kHashEmpty) return false;
        s = (s + 1) & mask;
    }
    return false;
}

// ------------------------------------------------------------------------------------
// Workspace layout for the loss/gradient and step/embed calls.
// ------------------------------------------------------------------------------------
struct SweepPlan {
    int D = 0;          // padded compile-time dimension (1,2,3,4,8,16,32,64,128)
    int R = 1;          // rows per lane
    int W = 1;          // waves per workgroup sharing a column block
    int T = 64;         // super-tile edge (rows = columns) = 64 * R * W
    int nt = 0;         // tiles per side
    long long items = 0;  // upper-triangle super tiles nt (nt + 1) / 2
    long long grid = 0;   // workgroups launched (multiple of 8, >= items)
    int edge_blocks = 0;  // blocks of the exact edge pass
    long long partials = 0;  // float loss partials: items + edge_blocks
    // fused-iteration gradient descent (d <= 16, small n): one launch per iteration
    bool persist = false;
    long long nb64 = 0;        // 64-vertex blocks per side
    long long tiles64 = 0;     // upper-triangle 64x64 tiles
    long long units_sweep = 0, units_edge = 0, units = 0;  // work units per iteration
    long long iter_blocks = 0;  // workgroups per iteration: the units + one that sums the loss
    // BF16 Gram screen (precision GEMPE_BF16_GRAM): items = 64x64 upper tiles, D = padded
    // dimension of the exact pass over the flagged tiles
    bool bf16 = false;
    // one shard of the upper triangle (FP32 sweeps): items are then that shard's tiles
    int shard = 0, nshards = 1;
    // d = 16, 32, 64, 128 on the matrix cores (loss and gradient only): 64-row strips
    // against chunks of mfma_chunk column blocks of 64; the partial region holds
    // max(items, mfma_items) slots before the edge blocks' partials.  A BF16 plan at d = 16
    // keeps mfma false and fills the mfma_* fields for its all-dense evaluations (then
    // 2 mfma_items <= items, so the sweep's slots lie inside the list's cleared ones).
    bool mfma = false;
    int mfma_chunk = 8;
    long long mfma_items = 0, mfma_grid = 0;
};

// Tiles of shard s of G over nt strips (strips p and nt-1-p paired, pair p owned by shard
// p mod G); nt (nt + 1) / 2 when G == 1.
long long gempe_shard_items(int nt, int s, int G);

struct WsLayout {
    size_t counters = 0;  // 256 B: [0] int64 edge hits, [8] unsigned status, [16] FP64 loss
                          // scratch, [32] int flagged-tile count, [36] int all-dense flag,
                          // [40] int x 2 the route sample's flagged and sampled sub-tiles (BF16)
    size_t partials = 0;  // float[plan.partials]
    size_t gbuf = 0;      // float[n*d] gradient scratch for gempe_step/gempe_embed
    size_t zbuf = 0;      // float[n] weighted-majorization denominators z_i
    size_t xbuf = 0;      // float[n*d] embed: second slot of the double-buffered iterate
    size_t gring = 0;     // float[3*n*d] embed: three gradient slots
    size_t ppart = 0;     // float[2*plan.units] embed: double-buffered loss partials
    size_t red = 0;       // double[1024] first level of the FP64 loss reduction
    // BF16 Gram screen
    size_t xb = 0;        // bf16[n*d] rounded coordinates
    size_t nrm = 0;       // float[n] squared norms of the rounded coordinates
    size_t snorm = 0;     // float[n] norms of the coordinates
    size_t smax128 = 0;   // float[n/128] largest norm of every 128-vertex block
    size_t flags = 0;     // uint8[items] near flags of the 64x64 tiles
    size_t list = 0;      // int32[items] flagged tiles in order
    size_t dense = 0;     // uint8[items] per list slot: 1 = more near pairs than the sparse pass takes
    size_t chunks = 0;    // int32[tiles / 4096 + 1] compaction scratch
    size_t total = 0;
};

SweepPlan gempe_make_plan(const gempe_graph_s *g, int d, bool bf16);
// GEMPE_ERR_UNSUPPORTED when a launch of the plan would exceed HIP's grid limits.
gempe_status gempe_check_plan(const SweepPlan &p, const char *who);
WsLayout gempe_ws_layout(const gempe_graph_s *g, int d, const SweepPlan &plan);
// The part of the layout one FP32 loss/gradient evaluation with a caller-provided gradient
// uses: counters, loss partials and the first reduction level only.
WsLayout gempe_ws_layout_eval(const gempe_graph_s *g, int d, const SweepPlan &plan);

// Kernel launchers (sweep.hip).
struct PairParamsHost {
    float mu_s, inv_sigma, c_neg, c_pos;  // see gempe::PairParams
    float tk_scale, tk_off, slope_k, r_scale, w_scale, wk2;
    int table_full;
    int reverse;  // GEMPE_F_REVERSE_TILES: the FP32 sweeps take their tiles in reverse order
};
PairParamsHost gempe_pair_params(const gempe_params *p);

// Workspace pointers and threshold of the BF16 Gram screen (unused for FP32 plans).
struct GramCtx {
    void *xb = nullptr;
    float *nrm = nullptr, *snorm = nullptr, *smax128 = nullptr;
    unsigned char *flags = nullptr;
    int *list = nullptr, *count = nullptr;
    float theta0 = 0.0f;  // mu + near_k sigma
    unsigned char *dense = nullptr;
    int *chunks = nullptr;
    int *all_dense = nullptr;  // set by the sparse pass when the full matrix-core sweep takes every tile
    int *sample = nullptr;     // the route sample's flagged and sampled sub-tile counts (two ints)
};
GramCtx gempe_gram_ctx(const WsLayout &L, unsigned char *ws, const gempe_params *p);

hipError_t gempe_launch_loss_grad(const gempe_graph_s *g, int d, const SweepPlan &plan,
                                  const float *X, float *grad, float *row_loss, float *partials,
                                  unsigned char *counters, double *loss, int64_t *hits_out,
                                  const PairParamsHost &pp, hipStream_t s, bool clear_status,
                                  const GramCtx &gc, double *red, float *wm_z = nullptr);
// The d = 16 matrix-core sweep (sweep_mfma.hip): items of a plan with mfma_chunk, and the
// launch over pl.items items with pl.grid workgroups.
long long gempe_mfma_items(int n, int chunk);
// gate: the BF16 path's all-dense evaluation (runs only when *gate is set), else null.
hipError_t gempe_launch_sweep_mfma16(const SweepPlan &pl, const float *X, int n, float *G, float *partials,
                                     const PairParamsHost &pph, hipStream_t s, const int *gate = nullptr);
// The same for d = 32, 64, 128 (k_sweep_mfma_wide<d, gated>).
hipError_t gempe_launch_sweep_mfma_wide(const SweepPlan &pl, int d, const float *X, int n, float *G, float *partials,
                                        const PairParamsHost &pph, hipStream_t s, const int *gate = nullptr);
// The BF16 path's exact pass over its densely flagged tiles at d = 16, on the matrix cores.
hipError_t gempe_launch_sweep_mfma16_list(const SweepPlan &pl, const float *X, int n, const GramCtx &gc, float *G,
                                          float *partials, const PairParamsHost &pph, hipStream_t s);
// sample: null, or the route sample's counters (GramCtx::sample).  With them a sample of the
// tiles is screened first, and when more than half of it is flagged the screen and the flag
// compaction return at once (the full matrix-core sweep takes the evaluation).
hipError_t gempe_launch_gram_screen(const gempe_graph_s *g, int d, const float *X, void *Xb, float *nrm,
                                    float *snorm, float *smax128, unsigned char *flags, int *list, int *count,
                                    float theta0, int *chunk, hipStream_t s, int *sample = nullptr);
// Sparse exact pass over the flagged tiles (gram.hip); ex: 0 none, 1 row loss, 2 WM z.
// all_dense, when more than half of the tiles are flagged: 0 nothing special; 1 every
// flagged tile is marked dense for the dense pass without being recomputed here; 2 the full
// matrix-core sweep (d = 16, 32, 64, 128) takes every pair (the list's loss slots are cleared and
// *gc.all_dense is set, which the dense pass reads and skips).  *gc.all_dense is 0 otherwise.
// sample: the counters the screen was launched with (or null); when they show most sampled
// tiles flagged the pass only sets *gc.all_dense and the loss-slot count to full_items.
hipError_t gempe_launch_near_tiles(const gempe_graph_s *g, int d, const float *X, const GramCtx &gc,
                                   const PairParamsHost &pp, int ex, float *G, float *extra, float *partials,
                                   hipStream_t s, int all_dense = 0, const int *sample = nullptr,
                                   int full_items = 0);
hipError_t gempe_launch_axpy(float *X, const float *G, float eta, long long count, hipStream_t s);
hipError_t gempe_launch_wm_update(float *X, const float *G, const float *Z, int d, long long count, hipStream_t s);
// Continuous batching of fused iterations (sweep.hip): one table row per job.
size_t gempe_batch_entry_bytes();
void gempe_batch_entry_fill(void *dst, const gempe_graph_s *g, int d, const SweepPlan &plan, float *X,
                            int iters, float eta, double *loss_hist, const WsLayout &L, unsigned char *ws,
                            const PairParamsHost &pp, long long u0, int k0);
hipError_t gempe_batch_prepare(const gempe_graph_s *g, int d, const WsLayout &L, unsigned char *ws,
                               hipStream_t s);
hipError_t gempe_launch_iter_batch(int D, const void *table, int njobs, long long blocks, int tick,
                                   hipStream_t s);
hipError_t gempe_launch_embed_fused(const gempe_graph_s *g, int d, const SweepPlan &plan,
                                         float *X, int iters, float eta, double *loss_hist,
                                         const WsLayout &L, unsigned char *ws,
                                         const PairParamsHost &pp, hipStream_t s);

// Enqueues iterations [k_begin, k_end) of a run that is not fused (an evaluation of the loss
// and gradient followed by the step: X - eta G, or with wm the weighted-majorization update
// X - G / (2 z); k = iters is the final loss-only evaluation when loss_hist is given).  k = 0
// clears the status word.  Nothing is synchronised (api.hip).
hipError_t gempe_enqueue_embed_steps(const gempe_graph_s *g, int d, const SweepPlan &plan, const WsLayout &L,
                                     unsigned char *w, float *X, int iters, float eta, double *loss_hist,
                                     const gempe_params *p, hipStream_t stream, int k_begin, int k_end,
                                     bool wm = false);

// Distance histograms and the slope bisection (hist.hip).
size_t gempe_hist_partial_bytes(int n, int d, int nbins);
hipError_t gempe_launch_histogram(const gempe_graph_s *g, int d, const float *X, int nbins, float r2_max,
                                  unsigned long long *hist_all, unsigned long long *hist_edge, void *scratch,
                                  hipStream_t s);
hipError_t gempe_launch_box(const gempe_graph_s *g, int d, const float *X, int *box, hipStream_t s);
float gempe_box_code_to_float(int c);
double gempe_bisect_sigma(int nbins, double r2_max, const uint64_t *all, const uint64_t *edge, double mu,
                          double lo, double hi, int iters);

// Negative-sampled weighted majorization (sampled.hip).
size_t gempe_sampled_ws_bytes(const gempe_graph_s *g, int d);
hipError_t gempe_launch_sampled_step(const gempe_graph_s *g, int d, float *X, unsigned long long seed, int max_tries,
                                     int32_t *samples, double *loss, const PairParamsHost &pp, unsigned char *ws,
                                     bool clear_status, hipStream_t s);
unsigned *gempe_sampled_status(const gempe_graph_s *g, int d, unsigned char *ws);
