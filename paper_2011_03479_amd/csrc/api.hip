// C ABI entry points: argument validation, workspace carving, launch sequencing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace {
thread_local std::string g_last_error;
}

void gempe_set_error(const std::string &msg) { g_last_error = msg; }

gempe_status gempe_fail(gempe_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

extern "C" const char *gempe_last_error(void) { return g_last_error.c_str(); }

extern "C" const char *gempe_status_string(gempe_status s) {
    switch (s) {
        case GEMPE_OK: return "ok";
        case GEMPE_ERR_ARG: return "invalid argument";
        case GEMPE_ERR_GRAPH: return "invalid graph";
        case GEMPE_ERR_NOMEM: return "insufficient memory or workspace";
        case GEMPE_ERR_HIP: return "HIP runtime error";
        case GEMPE_ERR_NUMERIC: return "non-finite value";
        case GEMPE_ERR_UNSUPPORTED: return "unsupported";
        case GEMPE_ERR_TIMEOUT: return "wait timed out";
    }
    return "unknown status";
}

extern "C" void gempe_params_default(gempe_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->mu = 1.5;
    p->sigma = 1.0;
    p->precision = GEMPE_FP32;
    p->near_k = 9.0;
    p->flags = GEMPE_F_NONE;
}

gempe_status gempe_check_problem(int32_t n, int32_t d, const gempe_params *p, const char *who) {
    std::string w(who);
    if (!p) return gempe_fail(GEMPE_ERR_ARG, w + ": null params");
    if (n < 2) return gempe_fail(GEMPE_ERR_ARG, w + ": the graph needs n >= 2 vertices");
    if (d < 1 || d > 128) return gempe_fail(GEMPE_ERR_ARG, w + ": d must be in [1, 128]");
    if (!(std::isfinite(p->mu) && std::isfinite(p->sigma) && p->sigma > 0.0))
        return gempe_fail(GEMPE_ERR_ARG, w + ": mu must be finite and sigma finite and > 0");
    if (p->reserved0 != 0 || p->reserved1 != 0)
        return gempe_fail(GEMPE_ERR_ARG, w + ": reserved fields must be 0");
    if ((p->flags & ~GEMPE_F_REVERSE_TILES) != 0u)
        return gempe_fail(GEMPE_ERR_ARG, w + ": unknown flag bits");
    if (p->precision == GEMPE_BF16_GRAM) {
        if (d < 16 || d % 16 != 0)
            return gempe_fail(GEMPE_ERR_ARG, w + ": BF16_GRAM needs d >= 16 and d % 16 == 0");
        if (!(std::isfinite(p->near_k) && p->near_k > 0.0))
            return gempe_fail(GEMPE_ERR_ARG, w + ": near_k must be finite and > 0");
        // the 64 x 64 tiles on or above the diagonal are indexed with 32-bit integers
        const long long nb64 = ((long long)n + 63) / 64;
        if (nb64 * (nb64 + 1) / 2 > 2147483647LL)
            return gempe_fail(GEMPE_ERR_ARG, w + ": BF16_GRAM supports n <= 4194240");
    }
    if (p->precision != GEMPE_FP32 && p->precision != GEMPE_BF16_GRAM)
        return gempe_fail(GEMPE_ERR_ARG, w + ": unknown precision");
    return GEMPE_OK;
}

namespace {

gempe_status check_common(gempe_graph g, int32_t d, const gempe_params *p, const char *who) {
    if (!g) return gempe_fail(GEMPE_ERR_ARG, std::string(who) + ": null graph handle");
    gempe_status st = gempe_check_problem(g->n, d, p, who);
    if (st != GEMPE_OK) return st;
    return gempe_check_plan(gempe_make_plan(g, d, p->precision == GEMPE_BF16_GRAM), who);
}

gempe_status check_ws(gempe_graph g, int32_t d, const void *ws, size_t ws_bytes, const WsLayout &L,
                      const char *who) {
    (void)g;
    (void)d;
    if (!ws) return gempe_fail(GEMPE_ERR_ARG, std::string(who) + ": null workspace");
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0)
        return gempe_fail(GEMPE_ERR_ARG, std::string(who) + ": workspace must be 256-byte aligned");
    if (ws_bytes < L.total)
        return gempe_fail(GEMPE_ERR_NOMEM, std::string(who) + ": workspace of " + std::to_string(ws_bytes) +
                                               " bytes, need " + std::to_string(L.total));
    return GEMPE_OK;
}

}  // namespace

extern "C" size_t gempe_workspace_bytes(gempe_graph g, int32_t d, const gempe_params *p) {
    gempe_status st = check_common(g, d, p, "workspace_bytes");
    if (st != GEMPE_OK) return 0;
    SweepPlan plan = gempe_make_plan(g, d, p->precision == GEMPE_BF16_GRAM);
    return gempe_ws_layout(g, d, plan).total;
}

extern "C" gempe_status gempe_loss_grad(gempe_graph g, int32_t d, const float *X, float *grad, double *loss,
                                        int64_t *edge_hits, float *row_loss, void *ws, size_t ws_bytes,
                                        const gempe_params *p, hipStream_t stream) {
    gempe_status st = check_common(g, d, p, "loss_grad");
    if (st != GEMPE_OK) return st;
    if (!X || !loss) return gempe_fail(GEMPE_ERR_ARG, "loss_grad: X and loss are required");
    SweepPlan plan = gempe_make_plan(g, d, p->precision == GEMPE_BF16_GRAM);
    WsLayout L = gempe_ws_layout(g, d, plan);
    if ((st = check_ws(g, d, ws, ws_bytes, L, "loss_grad")) != GEMPE_OK) return st;
    unsigned char *w = static_cast<unsigned char *>(ws);
    float *G = grad ? grad : reinterpret_cast<float *>(w + L.gbuf);
    GEMPE_HIP_TRY(gempe_launch_loss_grad(g, d, plan, X, G, row_loss, reinterpret_cast<float *>(w + L.partials),
                                         w + L.counters, loss, edge_hits, gempe_pair_params(p), stream, true,
                                         gempe_gram_ctx(L, w, p), reinterpret_cast<double *>(w + L.red)));
    return GEMPE_OK;
}

extern "C" int64_t gempe_shard_rows(gempe_graph g, int32_t d, const gempe_params *p) {
    if (check_common(g, d, p, "shard_rows") != GEMPE_OK) return 0;
    if (p->precision != GEMPE_FP32) {
        gempe_fail(GEMPE_ERR_UNSUPPORTED, "shard_rows: shards are FP32 only");
        return 0;
    }
    return gempe_make_plan(g, d, false).T;
}

extern "C" gempe_status gempe_loss_grad_shard(gempe_graph g, int32_t d, const float *X, float *grad, double *loss,
                                              int64_t *edge_hits, int32_t shard, int32_t nshards, void *ws,
                                              size_t ws_bytes, const gempe_params *p, hipStream_t stream) {
    gempe_status st = check_common(g, d, p, "loss_grad_shard");
    if (st != GEMPE_OK) return st;
    if (p->precision != GEMPE_FP32)
        return gempe_fail(GEMPE_ERR_UNSUPPORTED, "loss_grad_shard: shards are FP32 only");
    if (!X || !loss) return gempe_fail(GEMPE_ERR_ARG, "loss_grad_shard: X and loss are required");
    if (nshards < 1 || shard < 0 || shard >= nshards)
        return gempe_fail(GEMPE_ERR_ARG, "loss_grad_shard: need 0 <= shard < nshards");
    SweepPlan plan = gempe_make_plan(g, d, false);
    WsLayout L = gempe_ws_layout(g, d, plan);
    if ((st = check_ws(g, d, ws, ws_bytes, L, "loss_grad_shard")) != GEMPE_OK) return st;
    plan.shard = shard;
    plan.nshards = nshards;
    plan.items = gempe_shard_items(plan.nt, shard, nshards);
    plan.grid = std::max<long long>(1, (plan.items + 7) / 8) * 8;  // whole rounds over the 8 XCDs
    plan.partials = plan.items + plan.edge_blocks;
    unsigned char *w = static_cast<unsigned char *>(ws);
    float *G = grad ? grad : reinterpret_cast<float *>(w + L.gbuf);
    GEMPE_HIP_TRY(gempe_launch_loss_grad(g, d, plan, X, G, nullptr, reinterpret_cast<float *>(w + L.partials),
                                         w + L.counters, loss, edge_hits, gempe_pair_params(p), stream, true,
                                         gempe_gram_ctx(L, w, p), reinterpret_cast<double *>(w + L.red)));
    return GEMPE_OK;
}

extern "C" gempe_status gempe_step(gempe_graph g, int32_t d, float *X, float eta, double *loss_before, void *ws,
                                   size_t ws_bytes, const gempe_params *p, hipStream_t stream) {
    gempe_status st = check_common(g, d, p, "step");
    if (st != GEMPE_OK) return st;
    if (!X) return gempe_fail(GEMPE_ERR_ARG, "step: X is required");
    if (!(std::isfinite(eta) && eta > 0.0f)) return gempe_fail(GEMPE_ERR_ARG, "step: eta must be finite and > 0");
    SweepPlan plan = gempe_make_plan(g, d, p->precision == GEMPE_BF16_GRAM);
    WsLayout L = gempe_ws_layout(g, d, plan);
    if ((st = check_ws(g, d, ws, ws_bytes, L, "step")) != GEMPE_OK) return st;
    unsigned char *w = static_cast<unsigned char *>(ws);
    float *G = reinterpret_cast<float *>(w + L.gbuf);
    // the loss lands in the workspace when the caller does not want it
    double *lossp = loss_before ? loss_before : reinterpret_cast<double *>(w + L.counters + 16);
    GEMPE_HIP_TRY(gempe_launch_loss_grad(g, d, plan, X, G, nullptr, reinterpret_cast<float *>(w + L.partials),
                                         w + L.counters, lossp, nullptr, gempe_pair_params(p), stream, true,
                                         gempe_gram_ctx(L, w, p), reinterpret_cast<double *>(w + L.red)));
    GEMPE_HIP_TRY(gempe_launch_axpy(X, G, eta, (long long)g->n * d, stream));
    return GEMPE_OK;
}

hipError_t gempe_enqueue_embed_steps(const gempe_graph_s *g, int d, const SweepPlan &plan, const WsLayout &L,
                                     unsigned char *w, float *X, int iters, float eta, double *loss_hist,
                                     const gempe_params *p, hipStream_t stream, int k_begin, int k_end, bool wm) {
    float *G = reinterpret_cast<float *>(w + L.gbuf);
    float *Z = wm ? reinterpret_cast<float *>(w + L.zbuf) : nullptr;
    float *part = reinterpret_cast<float *>(w + L.partials);
    double *scratch_loss = reinterpret_cast<double *>(w + L.counters + 16);
    const PairParamsHost pp = gempe_pair_params(p);
    const GramCtx gc = gempe_gram_ctx(L, w, p);
    const long long nd = (long long)g->n * d;
    // the status word is cleared by the first sweep only, so it is sticky over the run
    for (int k = k_begin; k < k_end && k <= iters; ++k) {
        const bool last = (k == iters);
        if (last && !loss_hist) break;
        double *lossp = loss_hist ? loss_hist + k : scratch_loss;
        hipError_t e = gempe_launch_loss_grad(g, d, plan, X, G, nullptr, part, w + L.counters, lossp, nullptr, pp,
                                              stream, k == 0, gc, reinterpret_cast<double *>(w + L.red),
                                              last ? nullptr : Z);
        if (e != hipSuccess) return e;
        if (!last) {
            e = wm ? gempe_launch_wm_update(X, G, Z, d, nd, stream) : gempe_launch_axpy(X, G, eta, nd, stream);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

extern "C" gempe_status gempe_embed(gempe_graph g, int32_t d, float *X, int32_t iters, float eta,
                                    double *loss_hist, void *ws, size_t ws_bytes, const gempe_params *p,
                                    hipStream_t stream) {
    gempe_status st = check_common(g, d, p, "embed");
    if (st != GEMPE_OK) return st;
    if (!X) return gempe_fail(GEMPE_ERR_ARG, "embed: X is required");
    if (iters < 0) return gempe_fail(GEMPE_ERR_ARG, "embed: iters must be >= 0");
    if (!(std::isfinite(eta) && eta > 0.0f)) return gempe_fail(GEMPE_ERR_ARG, "embed: eta must be finite and > 0");
    SweepPlan plan = gempe_make_plan(g, d, p->precision == GEMPE_BF16_GRAM);
    WsLayout L = gempe_ws_layout(g, d, plan);
    if ((st = check_ws(g, d, ws, ws_bytes, L, "embed")) != GEMPE_OK) return st;
    unsigned char *w = static_cast<unsigned char *>(ws);
    unsigned *status_ws = reinterpret_cast<unsigned *>(w + L.counters + 8);
    const PairParamsHost pp = gempe_pair_params(p);
    if (iters == 0 && !loss_hist) return GEMPE_OK;
    if (plan.persist) {
        // one fused launch per iteration
        GEMPE_HIP_TRY(gempe_launch_embed_fused(g, d, plan, X, iters, eta, loss_hist, L, w, pp, stream));
    } else {
        GEMPE_HIP_TRY(
            gempe_enqueue_embed_steps(g, d, plan, L, w, X, iters, eta, loss_hist, p, stream, 0, iters + 1, false));
    }
    unsigned host_status = 0;
    GEMPE_HIP_TRY(hipMemcpyAsync(&host_status, status_ws, sizeof(unsigned), hipMemcpyDeviceToHost, stream));
    GEMPE_HIP_TRY(hipStreamSynchronize(stream));
    if (host_status & kStatusNonFinite) return gempe_fail(GEMPE_ERR_NUMERIC, "embed: non-finite loss");
    return GEMPE_OK;
}

// ------------------------------------------------------------------------------------
// Weighted majorization (Sec. II-C, Eqs. 3-5)
// ------------------------------------------------------------------------------------

extern "C" gempe_status gempe_wm_terms(gempe_graph g, int32_t d, const float *X, float *grad, float *z,
                                       double *loss, void *ws, size_t ws_bytes, const gempe_params *p,
                                       hipStream_t stream) {
    gempe_status st = check_common(g, d, p, "wm_terms");
    if (st != GEMPE_OK) return st;
    if (!X || !z || !loss) return gempe_fail(GEMPE_ERR_ARG, "wm_terms: X, z and loss are required");
    SweepPlan plan = gempe_make_plan(g, d, p->precision == GEMPE_BF16_GRAM);
    WsLayout L = gempe_ws_layout(g, d, plan);
    if ((st = check_ws(g, d, ws, ws_bytes, L, "wm_terms")) != GEMPE_OK) return st;
    unsigned char *w = static_cast<unsigned char *>(ws);
    float *G = grad ? grad : reinterpret_cast<float *>(w + L.gbuf);
    GEMPE_HIP_TRY(gempe_launch_loss_grad(g, d, plan, X, G, nullptr, reinterpret_cast<float *>(w + L.partials),
                                         w + L.counters, loss, nullptr, gempe_pair_params(p), stream, true,
                                         gempe_gram_ctx(L, w, p), reinterpret_cast<double *>(w + L.red), z));
    return GEMPE_OK;
}

extern "C" gempe_status gempe_wm_step(gempe_graph g, int32_t d, float *X, double *loss_before, void *ws,
                                      size_t ws_bytes, const gempe_params *p, hipStream_t stream) {
    gempe_status st = check_common(g, d, p, "wm_step");
    if (st != GEMPE_OK) return st;
    if (!X) return gempe_fail(GEMPE_ERR_ARG, "wm_step: X is required");
    SweepPlan plan = gempe_make_plan(g, d, p->precision == GEMPE_BF16_GRAM);
    WsLayout L = gempe_ws_layout(g, d, plan);
    if ((st = check_ws(g, d, ws, ws_bytes, L, "wm_step")) != GEMPE_OK) return st;
    unsigned char *w = static_cast<unsigned char *>(ws);
    float *G = reinterpret_cast<float *>(w + L.gbuf);
    float *Z = reinterpret_cast<float *>(w + L.zbuf);
    double *lossp = loss_before ? loss_before : reinterpret_cast<double *>(w + L.counters + 16);
    GEMPE_HIP_TRY(gempe_launch_loss_grad(g, d, plan, X, G, nullptr, reinterpret_cast<float *>(w + L.partials),
                                         w + L.counters, lossp, nullptr, gempe_pair_params(p), stream, true,
                                         gempe_gram_ctx(L, w, p), reinterpret_cast<double *>(w + L.red), Z));
    GEMPE_HIP_TRY(gempe_launch_wm_update(X, G, Z, d, (long long)g->n * d, stream));
    return GEMPE_OK;
}

extern "C" gempe_status gempe_embed_wm(gempe_graph g, int32_t d, float *X, int32_t iters, double *loss_hist,
                                       void *ws, size_t ws_bytes, const gempe_params *p, hipStream_t stream) {
    gempe_status st = check_common(g, d, p, "embed_wm");
    if (st != GEMPE_OK) return st;
    if (!X) return gempe_fail(GEMPE_ERR_ARG, "embed_wm: X is required");
    if (iters < 0) return gempe_fail(GEMPE_ERR_ARG, "embed_wm: iters must be >= 0");
    SweepPlan plan = gempe_make_plan(g, d, p->precision == GEMPE_BF16_GRAM);
    WsLayout L = gempe_ws_layout(g, d, plan);
    if ((st = check_ws(g, d, ws, ws_bytes, L, "embed_wm")) != GEMPE_OK) return st;
    if (iters == 0 && !loss_hist) return GEMPE_OK;
    unsigned char *w = static_cast<unsigned char *>(ws);
    unsigned *status_ws = reinterpret_cast<unsigned *>(w + L.counters + 8);
    GEMPE_HIP_TRY(gempe_enqueue_embed_steps(g, d, plan, L, w, X, iters, 1.0f, loss_hist, p, stream, 0, iters + 1, true));
    unsigned host_status = 0;
    GEMPE_HIP_TRY(hipMemcpyAsync(&host_status, status_ws, sizeof(unsigned), hipMemcpyDeviceToHost, stream));
    GEMPE_HIP_TRY(hipStreamSynchronize(stream));
    if (host_status & kStatusNonFinite) return gempe_fail(GEMPE_ERR_NUMERIC, "embed_wm: non-finite loss");
    return GEMPE_OK;
}

// ------------------------------------------------------------------------------------
// Slope optimisation (Sec. III-F)
// ------------------------------------------------------------------------------------

namespace {
constexpr int kSigmaIters = 200;
constexpr double kSigmaLo = 1e-3, kSigmaHi = 1e3;

gempe_status check_nbins(int32_t nbins, const char *who) {
    if (nbins < 2 || nbins > 16384)
        return gempe_fail(GEMPE_ERR_ARG, std::string(who) + ": nbins must be in [2, 16384]");
    return GEMPE_OK;
}

size_t hist_ws_bytes(const gempe_graph_s *g, int d, int nbins) {
    // partial histograms, then the two device histograms and the r2 word
    return ((gempe_hist_partial_bytes(g->n, d, nbins) + 255) & ~size_t(255)) + 2 * 8 * (size_t)nbins + 1024;
}
}  // namespace

extern "C" size_t gempe_histogram_workspace_bytes(gempe_graph g, int32_t d, int32_t nbins) {
    if (!g || d < 1 || d > 128 || nbins < 2 || nbins > 16384) return 0;
    return hist_ws_bytes(g, d, nbins);
}

extern "C" gempe_status gempe_distance_histogram(gempe_graph g, int32_t d, const float *X, int32_t nbins,
                                                 float r2_max, uint64_t *hist_all, uint64_t *hist_edge, void *ws,
                                                 size_t ws_bytes, hipStream_t stream) {
    if (!g) return gempe_fail(GEMPE_ERR_ARG, "distance_histogram: null graph handle");
    if (d < 1 || d > 128) return gempe_fail(GEMPE_ERR_ARG, "distance_histogram: d must be in [1, 128]");
    gempe_status st = check_nbins(nbins, "distance_histogram");
    if (st != GEMPE_OK) return st;
    if (!X || !hist_all || !hist_edge || !ws) return gempe_fail(GEMPE_ERR_ARG, "distance_histogram: null pointer");
    if (!(std::isfinite(r2_max) && r2_max > 0.0f))
        return gempe_fail(GEMPE_ERR_ARG, "distance_histogram: r2_max must be finite and > 0");
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0)
        return gempe_fail(GEMPE_ERR_ARG, "distance_histogram: workspace must be 256-byte aligned");
    if (ws_bytes < gempe_hist_partial_bytes(g->n, d, nbins))
        return gempe_fail(GEMPE_ERR_NOMEM, "distance_histogram: workspace too small");
    GEMPE_HIP_TRY(gempe_launch_histogram(g, d, X, nbins, r2_max, reinterpret_cast<unsigned long long *>(hist_all),
                                         reinterpret_cast<unsigned long long *>(hist_edge), ws, stream));
    return GEMPE_OK;
}

extern "C" gempe_status gempe_r2_bound(gempe_graph g, int32_t d, const float *X, float *r2_max, void *ws,
                                       size_t ws_bytes, hipStream_t stream) {
    if (!g || !X || !r2_max || !ws) return gempe_fail(GEMPE_ERR_ARG, "r2_bound: null argument");
    if (d < 1 || d > 128) return gempe_fail(GEMPE_ERR_ARG, "r2_bound: d must be in [1, 128]");
    if (ws_bytes < 2 * 4 * 128) return gempe_fail(GEMPE_ERR_NOMEM, "r2_bound: workspace too small");
    int *box = static_cast<int *>(ws);
    GEMPE_HIP_TRY(gempe_launch_box(g, d, X, box, stream));
    int codes[256];
    GEMPE_HIP_TRY(hipMemcpyAsync(codes, box, sizeof(int) * 2 * d, hipMemcpyDeviceToHost, stream));
    GEMPE_HIP_TRY(hipStreamSynchronize(stream));
    // every pair lies inside the bounding box, so its squared distance is below the squared
    // diagonal; the margin covers the single-precision rounding of the pairs' sums
    double diag2 = 0.0;
    for (int k = 0; k < d; ++k) {
        const double lo = gempe_box_code_to_float(codes[k]), hi = gempe_box_code_to_float(codes[d + k]);
        if (!std::isfinite(lo) || !std::isfinite(hi)) return gempe_fail(GEMPE_ERR_NUMERIC, "r2_bound: non-finite coordinates");
        diag2 += (hi - lo) * (hi - lo);
    }
    *r2_max = (float)(diag2 * (1.0 + 1e-5) + 1e-30);
    return GEMPE_OK;
}

extern "C" gempe_status gempe_sigma_fit(int32_t nbins, float r2_max, const uint64_t *hist_all,
                                        const uint64_t *hist_edge, double mu, double sigma_lo, double sigma_hi,
                                        double *sigma) {
    gempe_status st = check_nbins(nbins, "sigma_fit");
    if (st != GEMPE_OK) return st;
    if (!hist_all || !hist_edge || !sigma) return gempe_fail(GEMPE_ERR_ARG, "sigma_fit: null pointer");
    if (!(std::isfinite(r2_max) && r2_max > 0.0f) || !std::isfinite(mu))
        return gempe_fail(GEMPE_ERR_ARG, "sigma_fit: r2_max and mu must be finite, r2_max > 0");
    if (!(sigma_lo > 0.0 && sigma_hi > sigma_lo && std::isfinite(sigma_hi)))
        return gempe_fail(GEMPE_ERR_ARG, "sigma_fit: need 0 < sigma_lo < sigma_hi < inf");
    for (int b = 0; b < nbins; ++b)
        if (hist_edge[b] > hist_all[b]) return gempe_fail(GEMPE_ERR_ARG, "sigma_fit: an edge count exceeds its bin");
    *sigma = gempe_bisect_sigma(nbins, (double)r2_max, hist_all, hist_edge, mu, sigma_lo, sigma_hi, kSigmaIters);
    return GEMPE_OK;
}

extern "C" gempe_status gempe_embed_wm_sigma(gempe_graph g, int32_t d, float *X, int32_t iters,
                                             int32_t sigma_every, int32_t nbins, double *sigma, double *loss_hist,
                                             void *ws, size_t ws_bytes, const gempe_params *p, hipStream_t stream) {
    gempe_status st = check_common(g, d, p, "embed_wm_sigma");
    if (st != GEMPE_OK) return st;
    if (!X || !sigma) return gempe_fail(GEMPE_ERR_ARG, "embed_wm_sigma: X and sigma are required");
    if (iters < 0 || sigma_every < 1) return gempe_fail(GEMPE_ERR_ARG, "embed_wm_sigma: iters >= 0, sigma_every >= 1");
    if ((st = check_nbins(nbins, "embed_wm_sigma")) != GEMPE_OK) return st;
    if (!(std::isfinite(*sigma) && *sigma > 0.0))
        return gempe_fail(GEMPE_ERR_ARG, "embed_wm_sigma: the initial sigma must be finite and > 0");
    gempe_params q = *p;
    q.sigma = *sigma;
    SweepPlan plan = gempe_make_plan(g, d, q.precision == GEMPE_BF16_GRAM);
    WsLayout L = gempe_ws_layout(g, d, plan);
    WsLayout Lh = L;
    Lh.total = L.total + hist_ws_bytes(g, d, nbins);  // the histogram region follows the layout
    if ((st = check_ws(g, d, ws, ws_bytes, Lh, "embed_wm_sigma")) != GEMPE_OK) return st;
    unsigned char *w = static_cast<unsigned char *>(ws);
    unsigned char *hw = w + L.total;  // histogram region
    const size_t part = (gempe_hist_partial_bytes(g->n, d, nbins) + 255) & ~size_t(255);
    uint64_t *dev_all = reinterpret_cast<uint64_t *>(hw + part);
    uint64_t *dev_edge = dev_all + nbins;
    void *word = dev_edge + nbins;
    unsigned *status_ws = reinterpret_cast<unsigned *>(w + L.counters + 8);
    std::vector<uint64_t> h_all(nbins), h_edge(nbins);
    for (int k = 0; k <= iters; ++k) {
        if (k == iters && !loss_hist) break;
        GEMPE_HIP_TRY(gempe_enqueue_embed_steps(g, d, plan, L, w, X, iters, 1.0f, loss_hist, &q, stream, k, k + 1,
                                                true));
        if (k < iters && (k + 1) % sigma_every == 0) {
            // histograms of the new coordinates, then the slope where d DL / d sigma = 0
            float r2_max = 0.0f;
            if ((st = gempe_r2_bound(g, d, X, &r2_max, word, 1024, stream)) != GEMPE_OK) return st;
            GEMPE_HIP_TRY(gempe_launch_histogram(g, d, X, nbins, r2_max, reinterpret_cast<unsigned long long *>(dev_all),
                                                 reinterpret_cast<unsigned long long *>(dev_edge), hw, stream));
            GEMPE_HIP_TRY(hipMemcpyAsync(h_all.data(), dev_all, 8 * (size_t)nbins, hipMemcpyDeviceToHost, stream));
            GEMPE_HIP_TRY(hipMemcpyAsync(h_edge.data(), dev_edge, 8 * (size_t)nbins, hipMemcpyDeviceToHost, stream));
            GEMPE_HIP_TRY(hipStreamSynchronize(stream));
            q.sigma = gempe_bisect_sigma(nbins, (double)r2_max, h_all.data(), h_edge.data(), q.mu, kSigmaLo, kSigmaHi,
                                         kSigmaIters);
        }
    }
    *sigma = q.sigma;
    unsigned host_status = 0;
    GEMPE_HIP_TRY(hipMemcpyAsync(&host_status, status_ws, sizeof(unsigned), hipMemcpyDeviceToHost, stream));
    GEMPE_HIP_TRY(hipStreamSynchronize(stream));
    if (host_status & kStatusNonFinite) return gempe_fail(GEMPE_ERR_NUMERIC, "embed_wm_sigma: non-finite loss");
    return GEMPE_OK;
}

// ------------------------------------------------------------------------------------
// Negative sampling (Sec. III-C)
// ------------------------------------------------------------------------------------

extern "C" size_t gempe_sampled_workspace_bytes(gempe_graph g, int32_t d) {
    if (!g || d < 1 || d > 128) return 0;
    return gempe_sampled_ws_bytes(g, d);
}

namespace {
gempe_status check_sampled(gempe_graph g, int32_t d, float *X, int32_t max_tries, void *ws, size_t ws_bytes,
                           const gempe_params *p, const char *who) {
    gempe_status st = check_common(g, d, p, who);
    if (st != GEMPE_OK) return st;
    const std::string w(who);
    if (!X) return gempe_fail(GEMPE_ERR_ARG, w + ": X is required");
    if (max_tries < 1 || max_tries > 1024) return gempe_fail(GEMPE_ERR_ARG, w + ": max_tries must be in [1, 1024]");
    if (!ws) return gempe_fail(GEMPE_ERR_ARG, w + ": null workspace");
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0)
        return gempe_fail(GEMPE_ERR_ARG, w + ": workspace must be 256-byte aligned");
    if (ws_bytes < gempe_sampled_ws_bytes(g, d)) return gempe_fail(GEMPE_ERR_NOMEM, w + ": workspace too small");
    return GEMPE_OK;
}
}  // namespace

extern "C" gempe_status gempe_sampled_step(gempe_graph g, int32_t d, float *X, uint64_t seed, int32_t max_tries,
                                           int32_t *samples, double *loss_sampled, void *ws, size_t ws_bytes,
                                           const gempe_params *p, hipStream_t stream) {
    gempe_status st = check_sampled(g, d, X, max_tries, ws, ws_bytes, p, "sampled_step");
    if (st != GEMPE_OK) return st;
    GEMPE_HIP_TRY(gempe_launch_sampled_step(g, d, X, seed, max_tries, samples, loss_sampled, gempe_pair_params(p),
                                            static_cast<unsigned char *>(ws), true, stream));
    return GEMPE_OK;
}

extern "C" gempe_status gempe_embed_sampled(gempe_graph g, int32_t d, float *X, int32_t iters, uint64_t seed,
                                            int32_t max_tries, double *loss_hist, void *ws, size_t ws_bytes,
                                            const gempe_params *p, hipStream_t stream) {
    gempe_status st = check_sampled(g, d, X, max_tries, ws, ws_bytes, p, "embed_sampled");
    if (st != GEMPE_OK) return st;
    if (iters < 0) return gempe_fail(GEMPE_ERR_ARG, "embed_sampled: iters must be >= 0");
    unsigned char *w = static_cast<unsigned char *>(ws);
    const PairParamsHost pp = gempe_pair_params(p);
    // step k draws from seed + 2 nnz k, so no (step, entry, side) counter repeats
    for (int k = 0; k < iters; ++k)
        GEMPE_HIP_TRY(gempe_launch_sampled_step(g, d, X, seed + 2ull * (uint64_t)g->nnz * (uint64_t)k, max_tries,
                                                nullptr, loss_hist ? loss_hist + k : nullptr, pp, w, k == 0, stream));
    unsigned host_status = 0;
    GEMPE_HIP_TRY(hipMemcpyAsync(&host_status, gempe_sampled_status(g, d, w), sizeof(unsigned), hipMemcpyDeviceToHost,
                                 stream));
    GEMPE_HIP_TRY(hipStreamSynchronize(stream));
    if (host_status & kStatusNonFinite) return gempe_fail(GEMPE_ERR_NUMERIC, "embed_sampled: non-finite loss");
    return GEMPE_OK;
}

// ------------------------------------------------------------------------------------
// Loss and gradient without any allocation: the scratch of the evaluation (counters, loss
// partials, the first FP64 reduction level) lives in a file-scope device array instead of
// a caller workspace.  Every device the library runs on holds its own copy of the array
// until the process ends; host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device (the array's name is a host-side
// stand-in, not a device address).
// ------------------------------------------------------------------------------------

namespace {
constexpr size_t kScratchBytes = size_t(GEMPE_NOALLOC_SCRATCH_BYTES);
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of the scratch array, looked up once per device.
gempe_status scratch_for_current_device(unsigned char **out) {
    int dev = 0;
    GEMPE_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return gempe_fail(GEMPE_ERR_UNSUPPORTED, "loss_grad_noalloc: device id out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return gempe_fail(GEMPE_ERR_HIP, std::string("loss_grad_noalloc: hipGetSymbolAddress: ") +
                                                 hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = static_cast<unsigned char *>(g_scratch_ptr[dev]);
    return GEMPE_OK;
}

// The evaluation plan of the static-scratch entry point: the matrix-core sweep's one partial
// per item when that fits the array, else the vector sweep's fewer, larger tiles.
SweepPlan noalloc_plan(gempe_graph g, int32_t d) {
    SweepPlan plan = gempe_make_plan(g, d, false);
    if (plan.mfma && gempe_ws_layout_eval(g, d, plan).total > kScratchBytes) {
        plan.mfma = false;
        plan.partials = plan.items + plan.edge_blocks;
    }
    return plan;
}
}  // namespace

extern "C" size_t gempe_loss_grad_noalloc_bytes(gempe_graph g, int32_t d, const gempe_params *p) {
    if (check_common(g, d, p, "loss_grad_noalloc_bytes") != GEMPE_OK) return 0;
    if (p->precision != GEMPE_FP32) {
        gempe_fail(GEMPE_ERR_UNSUPPORTED, "loss_grad_noalloc_bytes: FP32 only");
        return 0;
    }
    return gempe_ws_layout_eval(g, d, noalloc_plan(g, d)).total;
}

extern "C" gempe_status gempe_loss_grad_noalloc(gempe_graph g, int32_t d, const float *X, float *grad, double *loss,
                                                int64_t *edge_hits, float *row_loss, const gempe_params *p,
                                                hipStream_t stream) {
    gempe_status st = check_common(g, d, p, "loss_grad_noalloc");
    if (st != GEMPE_OK) return st;
    if (p->precision != GEMPE_FP32)
        return gempe_fail(GEMPE_ERR_UNSUPPORTED, "loss_grad_noalloc: FP32 only (the BF16 screen needs a workspace)");
    if (!X || !grad || !loss) return gempe_fail(GEMPE_ERR_ARG, "loss_grad_noalloc: X, grad and loss are required");
    const SweepPlan plan = noalloc_plan(g, d);
    const WsLayout L = gempe_ws_layout_eval(g, d, plan);
    if (L.total > kScratchBytes)
        return gempe_fail(GEMPE_ERR_NOMEM, "loss_grad_noalloc: the evaluation needs " + std::to_string(L.total) +
                                               " bytes of scratch, the static array holds " +
                                               std::to_string(kScratchBytes));
    unsigned char *w = nullptr;
    if ((st = scratch_for_current_device(&w)) != GEMPE_OK) return st;
    // the counters are cleared by the evaluation's first kernel, every partial slot is
    // written by its tile or edge block, the reduction level by k_reduce1
    GEMPE_HIP_TRY(gempe_launch_loss_grad(g, d, plan, X, grad, row_loss, reinterpret_cast<float *>(w + L.partials),
                                         w + L.counters, loss, edge_hits, gempe_pair_params(p), stream, true,
                                         GramCtx(), reinterpret_cast<double *>(w + L.red)));
    return GEMPE_OK;
}
