// C ABI entry points: argument validation, workspace carving, launch sequencing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>

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
    if (p->reserved0 != 0 || p->reserved1 != 0 || p->flags != GEMPE_F_NONE)
        return gempe_fail(GEMPE_ERR_ARG, w + ": reserved fields and flags must be 0");
    if (p->precision == GEMPE_BF16_GRAM) {
        if (d < 16 || d % 16 != 0)
            return gempe_fail(GEMPE_ERR_ARG, w + ": BF16_GRAM needs d >= 16 and d % 16 == 0");
        if (!(std::isfinite(p->near_k) && p->near_k > 0.0))
            return gempe_fail(GEMPE_ERR_ARG, w + ": near_k must be finite and > 0");
    }
    if (p->precision != GEMPE_FP32 && p->precision != GEMPE_BF16_GRAM)
        return gempe_fail(GEMPE_ERR_ARG, w + ": unknown precision");
    return GEMPE_OK;
}

namespace {

gempe_status check_common(gempe_graph g, int32_t d, const gempe_params *p, const char *who) {
    if (!g) return gempe_fail(GEMPE_ERR_ARG, std::string(who) + ": null graph handle");
    return gempe_check_problem(g->n, d, p, who);
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
