/*
 * gempe.h -- C ABI of the MI355X (gfx950) library for the all-pairs GEMPE coding cost.
 *
 * GEMPE (graph embedding by minimising the predictive entropy, Boehm and Plant) scores an
 * embedding x_1..x_n in R^d of a graph G = (V, E) by the number of bits needed to code
 * the upper triangle of the adjacency matrix when the probability that (i, j) is an edge
 * is a sigmoid of the distance delta_ij = |x_i - x_j| (Sec. II-B, Eq. 2):
 *
 *   s+(delta) = Phi(-(delta - mu)/sigma),  s-(delta) = Phi((delta - mu)/sigma)
 *   dl(i,j)   = -log2 s+(delta_ij) if (i,j) in E, -log2 s-(delta_ij) otherwise
 *   DL        = sum_{i<j} dl(i,j)  [bits],   PE = DL / N,  N = n(n-1)/2
 *
 * with Phi the standard normal CDF (1/2 -+ 1/2 erf(z) of the paper).  The library
 * evaluates DL and its gradient g_i = dDL/dx_i over ALL n(n-1)/2 vertex pairs (the
 * "non-sampling version" of Sec. III-C), at fixed mu and sigma, and runs fixed-step
 * gradient descent on it.  The contribution of a coincident pair (delta = 0) to the
 * gradient is 0, the convention Eq. 5 uses for s_ij.
 *
 * Conventions for every call:
 *   - Pointers are DEVICE pointers unless marked [host].  The caller owns all device
 *     memory, the graph's included (gempe_graph_workspace_bytes); the library allocates
 *     device memory only for a server's budget block (gempe_server_create).
 *   - Matrices are row-major: X and grad are n x d float32, vertex i at X + i*d.
 *   - Vertex ids are 0-based; col_idx is int32 (n < 2^31), row_ptr is int64.
 *   - No exceptions cross the ABI.  Every call returns a gempe_status; argument errors
 *     are detected synchronously on the host before anything is enqueued.
 *     gempe_last_error() returns a thread-local message describing the last failure.
 *   - Asynchronous calls enqueue work on `stream` (0 = the null stream) and return
 *     immediately; results are valid once the stream reaches them.
 *   - The hot-path calls allocate no device memory: scratch comes from a caller-provided
 *     workspace of at least gempe_workspace_bytes() bytes (256-byte aligned).
 *   - Calls on one graph handle may run concurrently on different streams only if they
 *     use disjoint workspaces and outputs.
 */
#ifndef GEMPE_H
#define GEMPE_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gempe_status {
    GEMPE_OK = 0,
    GEMPE_ERR_ARG = -1,          /* invalid argument (sizes, null pointers, parameters)   */
    GEMPE_ERR_GRAPH = -2,        /* CSR not a simple undirected graph (see graph_create)   */
    GEMPE_ERR_NOMEM = -3,        /* workspace too small, or a set-up allocation failed     */
    GEMPE_ERR_HIP = -4,          /* a HIP runtime call failed                              */
    GEMPE_ERR_NUMERIC = -5,      /* non-finite loss or coordinates detected on the device  */
    GEMPE_ERR_UNSUPPORTED = -6,  /* valid request the library does not implement           */
    GEMPE_ERR_TIMEOUT = -7       /* a wait exceeded its time limit (serving)               */
} gempe_status;

/* Arithmetic of the all-pairs sweep. */
typedef enum gempe_precision {
    GEMPE_FP32 = 0,      /* every pair in FP32 (1 <= d <= 128)                              */
    GEMPE_BF16_GRAM = 1  /* d >= 16, d % 16 == 0, n <= 4,194,240: distances screened by a BF16 MFMA Gram
                            tile with FP32 accumulation; edges and pairs whose screened
                            distance is below mu + near_k*sigma + margin are recomputed
                            exactly in FP32, the remaining far non-edges contribute 0 */
} gempe_precision;

/* Flags (gempe_params.flags). */
#define GEMPE_F_NONE 0u
/* A schedule perturbation, for determinism tests: the FP32 sweeps (d <= 128, the fused
 * gradient-descent iteration included) take their tiles in reverse order.  Every tile
 * still writes its loss partial to its own slot and the FP64 sum runs in slot order, so
 * the loss at a given X is bitwise the same as without the flag; the gradient differs
 * only by the order of its FP32 atomic additions (and the later iterates of gempe_embed by
 * what that rounding carries forward).  Ignored by the BF16 Gram path. */
#define GEMPE_F_REVERSE_TILES 1u

typedef struct gempe_params {
    double mu;          /* sigmoid position; the paper fixes mu = 1.5 (Sec. III-F)         */
    double sigma;       /* sigmoid slope, > 0; the paper starts from sigma = 1 (Fig. algo)  */
    int32_t precision;  /* gempe_precision                                                  */
    int32_t reserved0;  /* must be 0                                                        */
    double near_k;      /* BF16_GRAM only: exact-recompute cut-off in sigmas (default 9)    */
    uint32_t flags;     /* GEMPE_F_* (0 or GEMPE_F_REVERSE_TILES); other bits: GEMPE_ERR_ARG */
    uint32_t reserved1; /* must be 0                                                        */
} gempe_params;

/* Fills *p with mu = 1.5, sigma = 1, FP32, near_k = 9, no flags. [host] */
void gempe_params_default(gempe_params *p);

typedef struct gempe_graph_s *gempe_graph;

/* Bytes of device memory a graph handle needs for n vertices and nnz CSR entries (the
 * CSR copy, the row id of every entry, the exact edge hash and a few status words; a graph
 * of n = 1e6 vertices and m = 1e7 edges needs about 440 MB).  0 on invalid arguments. [host] */
size_t gempe_graph_workspace_bytes(int32_t n, int64_t nnz);

/*
 * Uploads and validates a graph (Sec. II-A: n vertices, m undirected, unweighted,
 * unlabeled edges) given as symmetric CSR on the device:
 *   row_ptr : int64[n+1], row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz
 *   col_idx : int32[nnz], nnz = 2m; each row sorted strictly ascending, no self-loops,
 *             every (i, j) present together with (j, i)
 *   ws      : device memory of ws_bytes >= gempe_graph_workspace_bytes(n, nnz), 256-byte
 *             aligned, owned by the caller; it holds the graph for the handle's lifetime
 *             and must stay valid until the last call using the handle has completed
 * The library copies the CSR into ws (the caller may free its CSR buffers after return)
 * and builds there an exact open-addressing hash of the m undirected edges (64-bit keys,
 * capacity the power of two >= 2m, load factor <= 0.5); it allocates no device memory.
 * Synchronous: returns after validation; GEMPE_ERR_GRAPH if the CSR violates any rule
 * above, GEMPE_ERR_NOMEM if ws_bytes is too small.  *out [host] receives the handle;
 * n >= 1, nnz >= 0.
 */
gempe_status gempe_graph_create(int32_t n, int64_t nnz, const int64_t *row_ptr,
                                const int32_t *col_idx, void *ws, size_t ws_bytes,
                                hipStream_t stream, gempe_graph *out);

/* Releases the host-side handle.  Makes no device call: the graph's memory is the caller's
 * workspace, which the caller frees once the work using the handle has completed. */
gempe_status gempe_graph_destroy(gempe_graph g);

int32_t gempe_graph_num_vertices(gempe_graph g); /* n, or -1 for a null handle */
int64_t gempe_graph_num_edges(gempe_graph g);    /* m (undirected), or -1      */

/*
 * Batch membership query against the exact edge hash: out[k] = 1 if {qi[k], qj[k]} is an
 * edge, else 0, for k < q.  qi, qj: int32[q] in [0, n) (out-of-range ids give 0);
 * out: uint8[q].  Asynchronous.
 */
gempe_status gempe_has_edge(gempe_graph g, int64_t q, const int32_t *qi, const int32_t *qj,
                            uint8_t *out, hipStream_t stream);

/* Bytes of workspace needed by gempe_loss_grad / gempe_step / gempe_embed for this
 * graph, dimension and parameters (0 on invalid arguments). [host] */
size_t gempe_workspace_bytes(gempe_graph g, int32_t d, const gempe_params *p);

/*
 * All-pairs loss and gradient at X (Eq. 2 at fixed mu, sigma; gradient of DL):
 *   X         : float32[n*d]                      (input)
 *   grad      : float32[n*d] or NULL              g_i = dDL/dx_i
 *   loss      : float64[1]                        DL in bits (PE = DL / N)
 *   edge_hits : int64[1] or NULL                  number of pairs i<j scored as edges;
 *                                                 equals m when membership is exact
 *   row_loss  : float32[n] or NULL                L_i = sum_{j != i} dl(i,j)
 *   ws        : workspace of ws_bytes >= gempe_workspace_bytes(g, d, p)
 * FP32 arithmetic per pair; the loss is summed in FP32 per tile and in FP64 across
 * tiles in a fixed order (deterministic).  The gradient is accumulated with FP32
 * atomics across tiles (order of summation varies between runs).  Asynchronous.
 */
gempe_status gempe_loss_grad(gempe_graph g, int32_t d, const float *X, float *grad, double *loss,
                             int64_t *edge_hits, float *row_loss, void *ws, size_t ws_bytes,
                             const gempe_params *p, hipStream_t stream);

/*
 * One device's share of gempe_loss_grad when the all-pairs sweep is split over several
 * devices (the block-wise division of the pair work, Sec. III-A, across devices instead of
 * cores; Eq. 2 summed over a subset of the pairs).  The upper triangle is cut into strips of
 * R = gempe_shard_rows(g, d, p) rows (pair i < j lies in strip floor(i / R)); with S strips,
 * strips q and S-1-q form strip pair min(q, S-1-q), and shard `shard` of `nshards` owns the
 * strip pairs p with p mod nshards == shard (equal pair counts up to one strip pair).
 *   grad, loss, edge_hits : as gempe_loss_grad, summed over the shard's pairs only; the
 *                           sums over all shards give gempe_loss_grad's values (to FP32
 *                           rounding; edge hits exactly)
 * FP32 only (GEMPE_ERR_UNSUPPORTED for BF16_GRAM); 0 <= shard < nshards.  Same workspace as
 * gempe_loss_grad.  Asynchronous.
 */
gempe_status gempe_loss_grad_shard(gempe_graph g, int32_t d, const float *X, float *grad, double *loss,
                                   int64_t *edge_hits, int32_t shard, int32_t nshards, void *ws,
                                   size_t ws_bytes, const gempe_params *p, hipStream_t stream);

/* The strip height R of gempe_loss_grad_shard's split for this graph, d and parameters
 * (0 on invalid arguments or BF16_GRAM). [host] */
int64_t gempe_shard_rows(gempe_graph g, int32_t d, const gempe_params *p);

/*
 * One fixed-step gradient-descent step X <- X - eta * grad DL(X), in place.
 *   loss_before : float64[1] or NULL, receives DL at the X on entry
 * eta > 0 and finite.  Asynchronous.
 */
gempe_status gempe_step(gempe_graph g, int32_t d, float *X, float eta, double *loss_before,
                        void *ws, size_t ws_bytes, const gempe_params *p, hipStream_t stream);

/*
 * iters steps of fixed-step gradient descent (the repeat loop of the paper's driver,
 * with the weighted-majorization update replaced by X <- X - eta * grad DL):
 *   X         : float32[n*d], initial coordinates in, final coordinates out
 *   loss_hist : float64[iters+1] or NULL; loss_hist[k] = DL(X_k), k = 0..iters
 *               (computing loss_hist[iters] costs one extra loss-only sweep)
 * For d <= 16 and at most 65,536 upper 64 x 64 tiles (n <= 23,000) every iteration is
 * ONE fused launch (the previous step applied on the fly, the sweep, the edge pass and
 * the FP64 loss of the previous iterate; the kernel boundary is the only global
 * synchronisation); otherwise each iteration is a loss/gradient evaluation followed by
 * the update.  Synchronises the stream once at the end to read the device status word:
 * returns GEMPE_ERR_NUMERIC if a non-finite loss appeared during the run.
 */
gempe_status gempe_embed(gempe_graph g, int32_t d, float *X, int32_t iters, float eta,
                         double *loss_hist, void *ws, size_t ws_bytes, const gempe_params *p,
                         hipStream_t stream);

/* ------------------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): gempe_loss_grad with the library's own
 * device scratch in place of the caller's workspace.
 * ------------------------------------------------------------------------------------ */
#define GEMPE_NOALLOC_SCRATCH_BYTES (32u << 20) /* per device, held until the process ends */

/* Scratch bytes gempe_loss_grad_noalloc needs for this problem: one float loss partial per
 * sweep tile and per edge block, plus 8.5 KiB of counters and reduction slots (n = 1e6 at
 * d = 16 needs about 8 MB; above about n = 190,000 at d > 16 it exceeds the array).  0 on
 * invalid arguments or BF16_GRAM. [host] */
size_t gempe_loss_grad_noalloc_bytes(gempe_graph g, int32_t d, const gempe_params *p);

/* gempe_loss_grad without a workspace argument: the same arguments otherwise (X, grad and
 * loss required), the same kernels and results, FP32 only.  Allocates nothing and calls no
 * allocating routine (unless gempe_timing_enable is on, whose brackets create HIP events):
 * its scratch is a file-scope device array of GEMPE_NOALLOC_SCRATCH_BYTES, one per device,
 * that every call on that device shares and that keeps the last call's contents (each call
 * clears what must start at zero).  Calls that overlap on one device race on the array:
 * the caller serialises them (one stream, or events).  GEMPE_ERR_NOMEM when
 * gempe_loss_grad_noalloc_bytes exceeds GEMPE_NOALLOC_SCRATCH_BYTES; GEMPE_ERR_UNSUPPORTED
 * for BF16_GRAM.  Asynchronous. */
gempe_status gempe_loss_grad_noalloc(gempe_graph g, int32_t d, const float *X, float *grad, double *loss,
                                     int64_t *edge_hits, float *row_loss, const gempe_params *p,
                                     hipStream_t stream);

/* ------------------------------------------------------------------------------------
 * Weighted majorization (Sec. II-C).  For each pair the parabola w_ij (delta - d_ij)^2 that
 * matches dl's slope and curvature at the current distance (Eqs. 3-4) has
 *   w_ij = dl''(delta_ij) / 2 = R (R + tau) / (2 sigma^2 ln 2),  R = phi(tau) / Phi(tau)
 * (the printed Eq. 3 carries a factor 2/(pi ln 2) where matching the curvature gives
 * 1/(pi ln 2); this library follows the derivation), and the update of Eq. 5,
 *   x_i <- y_i / z_i,  z_i = sum_{j != i} w_ij,
 * equals x_i - g_i / (2 z_i) with g the gradient of DL.  All w_ij > 0.
 * ------------------------------------------------------------------------------------ */

/* DL, gradient and z_i at X (z: float32[n], required; grad may be NULL).  Same arithmetic
 * and precision options as gempe_loss_grad; with GEMPE_BF16_GRAM the far non-edges the
 * screen skips add 0 to z (each would add < 7e-18).  Asynchronous. */
gempe_status gempe_wm_terms(gempe_graph g, int32_t d, const float *X, float *grad, float *z, double *loss,
                            void *ws, size_t ws_bytes, const gempe_params *p, hipStream_t stream);

/* One weighted-majorization step (Eq. 5) in place; loss_before (nullable) receives DL at the
 * X on entry.  A vertex with z_i <= 0 (every weight underflowed) keeps its coordinates.
 * Asynchronous. */
gempe_status gempe_wm_step(gempe_graph g, int32_t d, float *X, double *loss_before, void *ws, size_t ws_bytes,
                           const gempe_params *p, hipStream_t stream);

/* iters weighted-majorization steps at fixed mu, sigma (the loop the paper states for a
 * fixed sigmoid setting, Sec. II-C); loss_hist as in gempe_embed.  Synchronises once at the
 * end; GEMPE_ERR_NUMERIC if a non-finite loss appeared. */
gempe_status gempe_embed_wm(gempe_graph g, int32_t d, float *X, int32_t iters, double *loss_hist, void *ws,
                            size_t ws_bytes, const gempe_params *p, hipStream_t stream);

/* ------------------------------------------------------------------------------------
 * Slope optimisation (Sec. III-F).  mu stays fixed; sigma is chosen where d DL / d sigma = 0,
 * i.e. where F(sigma) = sum_{i<j} tau_ij R(tau_ij) vanishes (d tau / d sigma = -tau / sigma),
 * located by bisection on histograms of the pair distances kept separately for edges and
 * non-edges.  Histogram layout: nbins bins uniform in the squared distance on [0, r2_max);
 * a pair goes to bin floor(min(r2 * inv_w, nbins - 1)), inv_w = nbins / r2_max in single
 * precision, r2 the single-precision squared distance summed over the coordinates in order
 * with fused multiply-adds; a bin stands for the distance sqrt((b + 1/2) r2_max / nbins).
 * ------------------------------------------------------------------------------------ */

/* Workspace of gempe_distance_histogram (and the extra part gempe_embed_wm_sigma needs
 * beyond gempe_workspace_bytes); 0 on invalid arguments.  2 <= nbins <= 16384. [host] */
size_t gempe_histogram_workspace_bytes(gempe_graph g, int32_t d, int32_t nbins);

/* Counts of all unordered pairs (hist_all) and of the edges (hist_edge) per bin, uint64[nbins]
 * each, device.  Exact integer counts (deterministic).  Asynchronous. */
gempe_status gempe_distance_histogram(gempe_graph g, int32_t d, const float *X, int32_t nbins, float r2_max,
                                      uint64_t *hist_all, uint64_t *hist_edge, void *ws, size_t ws_bytes,
                                      hipStream_t stream);

/* *r2_max [host] = (squared diagonal of the coordinates' bounding box)(1 + 1e-5), an upper
 * bound of every pair's squared distance.  Synchronous; GEMPE_ERR_NUMERIC for non-finite
 * coordinates; ws >= 1024 bytes. */
gempe_status gempe_r2_bound(gempe_graph g, int32_t d, const float *X, float *r2_max, void *ws, size_t ws_bytes,
                            hipStream_t stream);

/* Bisection (200 geometric halvings of [sigma_lo, sigma_hi]) of F on the histograms
 * (host arrays); returns a bracket end when F does not change sign in it (the minimum of
 * Eq. 2 over that interval lies on its boundary). [host] */
gempe_status gempe_sigma_fit(int32_t nbins, float r2_max, const uint64_t *hist_all, const uint64_t *hist_edge,
                             double mu, double sigma_lo, double sigma_hi, double *sigma);

/* Weighted majorization with the slope refitted after every sigma_every steps (the loop of
 * Fig. algo: WM step, then histograms and sigma): *sigma [host] holds the initial slope and
 * receives the last one; loss_hist[k] = DL(X_k) at the slope step k used.  Workspace:
 * gempe_workspace_bytes + gempe_histogram_workspace_bytes.  Synchronises at every refit and
 * at the end (GEMPE_ERR_NUMERIC if a non-finite loss appeared). */
gempe_status gempe_embed_wm_sigma(gempe_graph g, int32_t d, float *X, int32_t iters, int32_t sigma_every,
                                  int32_t nbins, double *sigma, double *loss_hist, void *ws, size_t ws_bytes,
                                  const gempe_params *p, hipStream_t stream);

/* ------------------------------------------------------------------------------------
 * Negative sampling (Sec. III-C, Fig. algo): O(m) weighted-majorization steps.  Every edge
 * (i, j) takes part with its parabola, plus two sampled non-edges (i, g) and (j, h); Eq. 5 is
 * applied over that multiset of pairs (x_v <- x_v - g_v / (2 z_v) with g and z summed over the
 * pairs containing v; a vertex in no pair keeps its coordinates).  Draws: the paper's 32-bit
 * LCG s <- 1103515245 s + 1, one generator per sample seeded from the upper 32 bits of
 * SplitMix64(seed + 2 e + side) (e the CSR index of the entry (i, j) with i < j, side 0 for
 * g and 1 for h); the low 23 bits of s become the mantissa of f in [1, 2) and the candidate
 * is floor(f n - n) in single precision (multiply, then subtract; floor where the paper
 * rounds, so n itself cannot come out); a candidate equal to the vertex, outside [0, n) or
 * adjacent to it (exact edge hash) is rejected and the generator steps again, at most
 * max_tries (1..1024) draws, else the sample is dropped.  Pair arithmetic in FP32 (the
 * precision field is ignored).
 * ------------------------------------------------------------------------------------ */

/* Workspace of gempe_sampled_step / gempe_embed_sampled (0 on invalid arguments). [host] */
size_t gempe_sampled_workspace_bytes(gempe_graph g, int32_t d);

/* One sampled step in place.  samples: int32[2 nnz] or NULL; for the entry e with i < j,
 * samples[2e] = g and samples[2e + 1] = h (-1 when dropped), -1 for entries with i > j.
 * loss_sampled (nullable): dl summed over the pairs used, FP64.  Asynchronous. */
gempe_status gempe_sampled_step(gempe_graph g, int32_t d, float *X, uint64_t seed, int32_t max_tries,
                                int32_t *samples, double *loss_sampled, void *ws, size_t ws_bytes,
                                const gempe_params *p, hipStream_t stream);

/* iters sampled steps, step k drawing with seed + 2 nnz k; loss_hist: float64[iters] or NULL
 * (the sampled loss of each step's pairs at the X it started from).  Synchronises once at the
 * end; GEMPE_ERR_NUMERIC if a non-finite loss appeared. */
gempe_status gempe_embed_sampled(gempe_graph g, int32_t d, float *X, int32_t iters, uint64_t seed,
                                 int32_t max_tries, double *loss_hist, void *ws, size_t ws_bytes,
                                 const gempe_params *p, hipStream_t stream);

/* ------------------------------------------------------------------------------------
 * Serving: a request loop that runs many embedding jobs (each one gempe_embed-style
 * gradient-descent run on its own graph) on one GPU with continuous batching.
 *
 * The server owns one device block of `budget_bytes`; every admitted job's graph,
 * coordinates, loss history and workspace are carved from it (first fit), so the budget
 * is a hard bound and admission never calls the device allocator.  A job is admitted, in
 * order of arrival, as soon as its footprint fits; later jobs that fit may pass a job
 * that does not, until that job has waited 2 s.  Jobs with d <= 16, FP32 and at most
 * 65,536 upper 64 x 64 tiles advance together, one iteration per launch for all of them
 * (a job arriving while others run joins at the next launch); other jobs run their
 * iterations on separate streams, overlapping with those launches and with each other.
 * Results (final coordinates, loss history) are copied to the caller's host buffers when
 * a job finishes.  A job's result equals what gempe_embed computes for it alone, up to
 * the order of FP32 atomic additions in the gradient.  A job whose loss becomes
 * non-finite, or whose graph is invalid, fails alone.
 * ------------------------------------------------------------------------------------ */
typedef struct gempe_server_s *gempe_server;

enum { GEMPE_JOB_QUEUED = 0, GEMPE_JOB_RUNNING = 1, GEMPE_JOB_DONE = 2, GEMPE_JOB_FAILED = 3 };

typedef struct gempe_job_desc {
    int32_t n;               /* vertices, >= 2                                               */
    int32_t d;               /* embedding dimension, 1..128                                  */
    int64_t nnz;             /* CSR entries, 2m                                              */
    const int64_t *row_ptr;  /* [host] int64[n+1], rules of gempe_graph_create               */
    const int32_t *col_idx;  /* [host] int32[nnz]                                            */
    const float *X0;         /* [host] float32[n*d] initial coordinates                      */
    int32_t iters;           /* gradient-descent steps, >= 0                                 */
    float eta;               /* step size, finite and > 0                                    */
    gempe_params params;     /* as for gempe_embed                                           */
    double release_s;        /* arrival time in seconds after server creation; the job is
                                not admitted before it (earlier values mean "now")          */
    float *X_out;            /* [host] float32[n*d], final coordinates, written at DONE      */
    double *loss_hist;       /* [host] float64[iters+1] or NULL, DL(X_k), written at DONE    */
} gempe_job_desc;

typedef struct gempe_job_info {
    int32_t state;      /* GEMPE_JOB_*                                                       */
    int32_t status;     /* gempe_status of a failed job, GEMPE_OK otherwise                  */
    int32_t batched;    /* 1 if the job ran in the shared per-iteration launches             */
    int32_t reserved;
    double release_s;   /* arrival, admission and completion times, seconds after creation */
    double admit_s;
    double done_s;
    uint64_t footprint; /* bytes of the budget the job held while running                   */
} gempe_job_info;

typedef struct gempe_server_stats {
    int64_t submitted, admitted, done, failed, rejected;
    int64_t ticks;           /* shared per-iteration launches issued                         */
    int64_t peak_bytes;      /* high-water mark of the budget in use                         */
    int64_t max_concurrent;  /* most jobs on the device at once                              */
    int64_t budget_bytes;
    double pairs;            /* unordered vertex pairs x iterations of the finished jobs     */
} gempe_server_stats;

/* Bytes of the budget a job of this shape holds while it runs (0 on invalid arguments). */
size_t gempe_job_footprint(int32_t n, int64_t nnz, int32_t d, int32_t iters, const gempe_params *p);

/* Creates a server on the current device with a budget of budget_bytes (>= 4 KiB,
 * allocated at once: GEMPE_ERR_NOMEM if that fails) and at most max_jobs (1..4096) jobs
 * on the device at once.  Starts the scheduler thread. [host] */
gempe_status gempe_server_create(size_t budget_bytes, int32_t max_jobs, gempe_server *out);

/* Queues a job; copies the request's host arrays (they may be freed on return); X_out
 * and loss_hist must stay valid until the job is DONE or FAILED.  GEMPE_ERR_NOMEM (the
 * job is rejected) if its footprint exceeds the whole budget; argument errors as for
 * gempe_graph_create / gempe_embed; an invalid graph fails the job at admission. [host] */
gempe_status gempe_server_submit(gempe_server s, const gempe_job_desc *job, int64_t *job_id);

/* State of a job (GEMPE_ERR_ARG for an unknown id). [host] */
gempe_status gempe_server_query(gempe_server s, int64_t job_id, gempe_job_info *info);

/* Waits until the job is DONE or FAILED (job_id < 0: until every submitted job is), at
 * most timeout_s seconds (< 0: no limit); GEMPE_ERR_TIMEOUT when the limit passes. [host] */
gempe_status gempe_server_wait(gempe_server s, int64_t job_id, double timeout_s, gempe_job_info *info);

gempe_status gempe_server_get_stats(gempe_server s, gempe_server_stats *out); /* [host] */

/* Stops the scheduler, lets enqueued device work finish, marks unfinished jobs FAILED and
 * frees the server's memory. [host] */
gempe_status gempe_server_destroy(gempe_server s);

/* ------------------------------------------------------------------------------------
 * Kernel timing, for measurement.  While enabled, the library records a pair of HIP events
 * on the launch's own stream around the launches of each kernel class, so that the time
 * between them is those kernels' device time.  gempe_timing_read waits for the recorded
 * events of one class, returns the number of kernel launches they bracket and their summed
 * duration in milliseconds, and clears that class's record.  Enabling costs two event
 * records per bracket; disabled (the default), nothing is recorded.
 * ------------------------------------------------------------------------------------ */
enum {
    GEMPE_TK_SWEEP = 0,  /* the all-pairs FP32 sweep (one bracket per launch), or the fused
                            gradient-descent iteration (one bracket over the iterations of a
                            gempe_embed call, counted as that many launches)               */
    GEMPE_TK_GRAM = 1,   /* the BF16 MFMA Gram screen                                        */
    GEMPE_TK_EXACT = 2,  /* the exact FP32 passes over the BF16 screen's near tiles          */
    GEMPE_TK_EDGES = 3,  /* the exact edge correction over the CSR entries                  */
    GEMPE_TK_FULL = 4    /* the BF16 path's full FP32 matrix-core sweep: launched for plain
                            evaluations at d = 16 from n = 8,192 and at d = 32, 64, 128 from
                            n = 4,096; it evaluates every pair when more than half of the
                            tiles were flagged and returns at once otherwise               */
};

gempe_status gempe_timing_enable(int32_t on); /* [host] */
/* kclass: GEMPE_TK_*; *launches and *total_ms [host] receive the totals.  GEMPE_ERR_HIP if
 * an event failed.  [host] */
gempe_status gempe_timing_read(int32_t kclass, int64_t *launches, double *total_ms);

/* Static description of a status code. [host] */
const char *gempe_status_string(gempe_status s);

/* Thread-local description of the last error raised by a call on this thread. [host] */
const char *gempe_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GEMPE_H */
