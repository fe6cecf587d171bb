// gde_api.hip -- host runtime behind the C ABI of include/gde.h: argument
// validation, contexts, graphs, workspaces and the plain (one query) solver loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "gde_batch.h"
#include "gde_det.h"
#include "gde_global.h"
#include "gde_internal.h"
#include "gde_kernels.h"

namespace gde {

static thread_local std::string g_err;
static std::atomic<uint64_t> g_uid{1};
static std::mutex g_ctx_mu;
static std::vector<gde_ctx *> g_ctxs;  // live contexts, so a destroyed graph's workspaces are released

int fail(int status, const std::string &msg) {
    g_err = msg;
    return status;
}
int hip_fail(hipError_t e, const char *what) {
    g_err = std::string("HIP error ") + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ") in " + what;
    return GDE_ERR_DEVICE;
}

// ------------------------------------------------------------------ validation
static int validate_csr_host(int32_t n, int64_t nnz, const int32_t *rp, const int32_t *ci) {
    if (n <= 0) return fail(GDE_ERR_INVALID_ARG, "n must be > 0");
    if (nnz < 0 || nnz >= (int64_t)INT32_MAX) return fail(GDE_ERR_INVALID_ARG, "nnz must be in [0, 2^31-1)");
    if (!rp || (nnz > 0 && !ci)) return fail(GDE_ERR_INVALID_ARG, "null CSR pointer");
    if (rp[0] != 0) return fail(GDE_ERR_INVALID_ARG, "row_ptr[0] must be 0");
    if ((int64_t)rp[n] != nnz) return fail(GDE_ERR_INVALID_ARG, "row_ptr[n] must equal nnz");
    for (int32_t u = 0; u < n; u++) {
        if (rp[u + 1] < rp[u]) return fail(GDE_ERR_INVALID_ARG, "row_ptr must be non-decreasing");
        for (int32_t k = rp[u]; k < rp[u + 1]; k++) {
            if (ci[k] < 0 || ci[k] >= n) return fail(GDE_ERR_INVALID_ARG, "col_idx out of range");
            if (ci[k] == u) return fail(GDE_ERR_INVALID_ARG, "self-loops are not allowed");
        }
    }
    return GDE_OK;
}

static int validate_params(const gde_params *p) {
    if (!p) return fail(GDE_ERR_INVALID_ARG, "null params");
    if (p->kind < GDE_PPR || p->kind > GDE_SERIES) return fail(GDE_ERR_INVALID_ARG, "unknown kind");
    if (p->method != GDE_LOCAL_GD && p->method != GDE_LOCAL_CH && p->method != GDE_LOCAL_SOR)
        return fail(GDE_ERR_INVALID_ARG, "unknown method");
    if (p->method == GDE_LOCAL_SOR) {
        if (p->omega != 0.0 && !(p->omega > 0.0 && p->omega < 2.0))
            return fail(GDE_ERR_INVALID_ARG, "LocalSOR needs 0 < omega < 2 (0 means 1)");
        if (p->kind == GDE_HK || p->kind == GDE_SERIES)
            return fail(GDE_ERR_UNSUPPORTED, "LocalSOR covers PPR and Katz");
    }
    if (p->value_type != GDE_F32 && p->value_type != GDE_F64) return fail(GDE_ERR_INVALID_ARG, "unknown value_type");
    if (!(p->eps > 0.0) || !std::isfinite(p->eps)) return fail(GDE_ERR_INVALID_ARG, "eps must be finite and > 0");
    if (p->max_iters < 1) return fail(GDE_ERR_INVALID_ARG, "max_iters must be >= 1");
    if (p->kind != GDE_SERIES && p->c != nullptr)
        return fail(GDE_ERR_INVALID_ARG, "params.c is for GDE_SERIES only and must be NULL otherwise");
    if ((p->flags & GDE_SCATTER_BINNED) && (p->flags & GDE_SCATTER_ATOMIC))
        return fail(GDE_ERR_INVALID_ARG, "GDE_SCATTER_BINNED and GDE_SCATTER_ATOMIC exclude each other");
    if (p->flags & ~(GDE_KATZ_SUBTRACT_SEED | GDE_TRACE | GDE_RESULT_DEVICE | GDE_SCATTER_BINNED | GDE_SCATTER_ATOMIC |
                     GDE_DETERMINISTIC | GDE_SYM_NORM))
        return fail(GDE_ERR_INVALID_ARG, "unknown flag bits");
    if (p->flags & GDE_SYM_NORM) {
        if (p->kind == GDE_KATZ) return fail(GDE_ERR_INVALID_ARG, "GDE_SYM_NORM applies to the kinds with M = A D^-1");
        if (p->method == GDE_LOCAL_SOR || (p->flags & GDE_DETERMINISTIC))
            return fail(GDE_ERR_UNSUPPORTED, "GDE_SYM_NORM is provided for LocalGD, LocalCH and the level push");
    }
    switch (p->kind) {
    case GDE_PPR:
        if (!(p->alpha > 0.0 && p->alpha < 1.0)) return fail(GDE_ERR_INVALID_ARG, "PPR needs 0 < alpha < 1");
        break;
    case GDE_KATZ:
        if (!(p->beta > 0.0) || !std::isfinite(p->beta)) return fail(GDE_ERR_INVALID_ARG, "Katz needs beta > 0");
        if (!(p->lambda_bound > 0.0) || !std::isfinite(p->lambda_bound))
            return fail(GDE_ERR_INVALID_ARG, "Katz needs lambda_bound > 0 (an upper bound of lambda_max(A))");
        if (!(p->beta * p->lambda_bound < 1.0))
            return fail(GDE_ERR_INVALID_ARG, "Katz needs beta * lambda_bound < 1");
        break;
    case GDE_HK:
        if (!(p->tau >= 0.0) || !std::isfinite(p->tau)) return fail(GDE_ERR_INVALID_ARG, "HK needs tau >= 0");
        if (p->K < 0 || p->K > 256) return fail(GDE_ERR_INVALID_ARG, "HK needs 0 <= K <= 256");
        if (p->method == GDE_LOCAL_CH) return fail(GDE_ERR_UNSUPPORTED, "LocalCH is not defined for the heat kernel");
        break;
    case GDE_SERIES:
        if (p->K < 0 || p->K > 256) return fail(GDE_ERR_INVALID_ARG, "SERIES needs 0 <= K <= 256");
        if (!p->c) return fail(GDE_ERR_INVALID_ARG, "SERIES needs params.c (K + 1 coefficients)");
        for (int32_t k = 0; k <= p->K; k++)
            if (!(p->c[k] > 0.0) || !std::isfinite(p->c[k]))
                return fail(GDE_ERR_INVALID_ARG, "SERIES coefficients must be finite and > 0");
        if (p->method == GDE_LOCAL_CH) return fail(GDE_ERR_UNSUPPORTED, "LocalCH is not defined for SERIES");
        break;
    }
    return GDE_OK;
}

// seed check against host row pointers (degrees)
static int validate_seed(const gde_seed *s, int32_t n, const int32_t *rp_host) {
    if (!s || s->nnz <= 0 || !s->idx || !s->val) return fail(GDE_ERR_INVALID_ARG, "seed must have nnz > 0 entries");
    if (s->nnz > n) return fail(GDE_ERR_INVALID_ARG, "seed has more entries than nodes");
    for (int32_t i = 0; i < s->nnz; i++) {
        int32_t u = s->idx[i];
        if (u < 0 || u >= n) return fail(GDE_ERR_INVALID_ARG, "seed index out of range");
        if (i > 0 && u <= s->idx[i - 1]) return fail(GDE_ERR_INVALID_ARG, "seed indices must be strictly increasing");
        if (!(s->val[i] > 0.0) || !std::isfinite(s->val[i]))
            return fail(GDE_ERR_INVALID_ARG, "seed values must be finite and > 0");
    }
    for (int32_t i = 0; i < s->nnz; i++) {
        int32_t u = s->idx[i];
        if (rp_host[u + 1] == rp_host[u]) return fail(GDE_ERR_ISOLATED_SEED, "seed node has degree 0");
    }
    return GDE_OK;
}

static int validate_seed_deg(const gde_seed *s, int32_t n, const std::vector<int32_t> &deg) {
    if (!s || s->nnz <= 0 || !s->idx || !s->val) return fail(GDE_ERR_INVALID_ARG, "seed must have nnz > 0 entries");
    if (s->nnz > n) return fail(GDE_ERR_INVALID_ARG, "seed has more entries than nodes");
    for (int32_t i = 0; i < s->nnz; i++) {
        int32_t u = s->idx[i];
        if (u < 0 || u >= n) return fail(GDE_ERR_INVALID_ARG, "seed index out of range");
        if (i > 0 && u <= s->idx[i - 1]) return fail(GDE_ERR_INVALID_ARG, "seed indices must be strictly increasing");
        if (!(s->val[i] > 0.0) || !std::isfinite(s->val[i]))
            return fail(GDE_ERR_INVALID_ARG, "seed values must be finite and > 0");
    }
    for (int32_t i = 0; i < s->nnz; i++)
        if (deg[s->idx[i]] == 0) return fail(GDE_ERR_ISOLATED_SEED, "seed node has degree 0");
    return GDE_OK;
}

// ------------------------------------------------------------------ workspaces
struct GraphHost {
    std::vector<int32_t> row_ptr;  // host copy of the row pointers at creation
    std::vector<int32_t> deg;      // current degrees (seed validation); updated on edge insertions
};
static std::mutex g_graph_mu;
static std::vector<std::pair<const gde_graph *, GraphHost *>> g_graph_host;

static GraphHost *graph_host(const gde_graph *g) {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (auto &e : g_graph_host)
        if (e.first == g) return e.second;
    return nullptr;
}

static void ws_free(Workspace *w) {
    void *dev[] = {w->rd, w->rd2, w->x, w->bitmap, w->tbm, w->front[0], w->front[1], w->touched[0], w->touched[1],
                   w->touched[2], w->wl_node, w->wl_beg, w->wl_off, w->wl_sv, w->tile_start, w->delta, w->dstamp,
                   w->cstamp, w->blk, w->st, w->seed_idx, w->seed_val, w->out_idx, w->out_val, w->tr_size,
                   w->tr_vol, w->tr_nodes, w->lam_buf, w->bin_base, w->bin_cursor, w->bin_e, w->lvl_tab};
    for (void *p : dev)
        if (p) (void)hipFree(p);
    if (w->hst) (void)hipHostFree(w->hst);
    if (w->h_seed_idx) (void)hipHostFree(w->h_seed_idx);
    if (w->h_seed_val) (void)hipHostFree(w->h_seed_val);
    det_ws_free(w->det);
    glob_ws_free(w->glob);
    delete w;
}

#define WS_ALLOC(ptr, bytes)                                            \
    do {                                                                \
        hipError_t _e = hipMalloc((void **)&(ptr), (bytes));            \
        if (_e != hipSuccess) { ws_free(w); return hip_fail(_e, "hipMalloc(workspace)"); } \
        _e = hipMemsetAsync((ptr), 0, (bytes), s);                      \
        if (_e != hipSuccess) { ws_free(w); return hip_fail(_e, "hipMemsetAsync"); } \
    } while (0)

// Graph-dependent parts of a workspace: degrees in the residual planes, the
// push tile table and the bins (capacity nnz_cap, with headroom so that a graph
// growing by edge insertions keeps its buffers).  Called at creation and after
// the graph's CSR has been replaced.
static int ws_graph_state(Workspace *w, const gde_graph *g, hipStream_t s) {
    const int64_t n = w->n;
    const size_t vs = w->vsize;
    if (g->nnz > w->nnz_cap) {
        (void)hipFree(w->tile_start);
        (void)hipFree(w->bin_e);
        w->tile_start = nullptr;
        w->bin_e = nullptr;
        const int64_t cap = g->nnz + g->nnz / 8 + 65536;
        GDE_HIP(hipMalloc((void **)&w->tile_start, 4 * (size_t)(cap / kPushTile + 2)));
        if (w->bin_nranges > 0) {
            // in-volume of every range plus one LocalCH self-mark per node
            const size_t es = vs == 8 ? sizeof(BinEnt<double>) : sizeof(BinEnt<float>);
            GDE_HIP(hipMalloc(&w->bin_e, es * (size_t)(cap + n)));
        }
        w->nnz_cap = cap;
    }
    if (w->vtype == GDE_F64) launch_init_rd<double>(g->row_ptr, w->rd, g->n, s);
    else launch_init_rd<float>(g->row_ptr, w->rd, g->n, s);
    if (w->rd2) {
        if (w->vtype == GDE_F64) launch_init_rd<double>(g->row_ptr, w->rd2, g->n, s);
        else launch_init_rd<float>(g->row_ptr, w->rd2, g->n, s);
    }
    GDE_HIP(hipGetLastError());
    if (w->bin_nranges > 0) {
        const int64_t nr = w->bin_nranges;
        unsigned long long *cnt = nullptr;
        GDE_HIP(hipMalloc((void **)&cnt, 8 * nr));
        GDE_HIP(hipMemsetAsync(cnt, 0, 8 * nr, s));
        launch_bin_count(g->col_idx, g->nnz, w->bin_shift, (int)nr, cnt, s);
        std::vector<unsigned long long> h(nr);
        hipError_t e = hipMemcpyAsync(h.data(), cnt, 8 * nr, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        (void)hipFree(cnt);
        if (e != hipSuccess) return hip_fail(e, "bin counts");
        // a bin holds its range's in-volume (one update per CSR entry and iteration)
        // and one LocalCH self-mark per node of the range
        std::vector<long long> base(nr + 1, 0);
        for (int64_t r = 0; r < nr; r++) {
            const int64_t lo = r << w->bin_shift;
            const int64_t nodes = std::min<int64_t>((int64_t)1 << w->bin_shift, n - lo);
            base[r + 1] = base[r] + (long long)h[r] + (long long)nodes;
        }
        GDE_HIP(hipMemcpyAsync(w->bin_base, base.data(), 8 * (nr + 1), hipMemcpyHostToDevice, s));
        GDE_HIP(hipStreamSynchronize(s));
    }
    (void)n;
    return GDE_OK;
}

static int ws_create(gde_ctx *ctx, const gde_graph *g, int vtype, hipStream_t s, Workspace **out) {
    Workspace *w = new Workspace();
    w->g = g;
    w->guid = g->uid;
    w->vtype = vtype;
    w->n = g->n;
    w->vsize = vtype == GDE_F64 ? 8 : 4;
    const int64_t n = g->n;
    const size_t vs = w->vsize;
    WS_ALLOC(w->rd, 2 * vs * n);
    WS_ALLOC(w->x, vs * n);
    int64_t nwords = (n + 31) / 32;
    w->nblk = (nwords + kBlock - 1) / kBlock;
    WS_ALLOC(w->bitmap, 4 * nwords);
    WS_ALLOC(w->tbm, 4 * nwords);
    WS_ALLOC(w->blk, 4 * (w->nblk + 1));
    for (int i = 0; i < 2; i++) WS_ALLOC(w->front[i], 4 * n);
    WS_ALLOC(w->wl_node, 4 * n);
    WS_ALLOC(w->wl_beg, 4 * n);
    WS_ALLOC(w->wl_off, 4 * n);
    WS_ALLOC(w->wl_sv, vs * n);
    WS_ALLOC(w->st, sizeof(DevState));
    // host-coherent: the publication kernel writes it while the host polls it
    hipError_t e = hipHostMalloc((void **)&w->hst, sizeof(DevState) + 128, hipHostMallocCoherent);
    if (e == hipSuccess) {
        const size_t off = ((sizeof(DevState) + 63) / 64) * 64;
        w->hseq = (uint32_t *)((char *)w->hst + off);
        *w->hseq = 0u;
        w->seq = 0u;
        void *dp = nullptr;
        e = hipHostGetDevicePointer(&dp, w->hst, 0);
        if (e == hipSuccess && !dp) e = hipErrorInvalidValue;
        if (e == hipSuccess) {
            w->hst_dev = (DevState *)dp;
            w->hseq_dev = (uint32_t *)((char *)dp + off);
        }
    }
    if (e != hipSuccess) { ws_free(w); return hip_fail(e, "hipHostMalloc"); }
    // bins of the binned scatter: one per range of 2^S nodes, sized by the range's in-volume
    int shift = 0;
    while (((int64_t)vs << (shift + 1)) <= kBinLdsBytes) shift++;
    const int64_t nranges = (n + ((int64_t)1 << shift) - 1) >> shift;
    if (nranges <= kBinMaxRanges) {
        w->bin_shift = shift;
        w->bin_nranges = (int)nranges;
        WS_ALLOC(w->bin_base, 8 * (nranges + 1));
        WS_ALLOC(w->bin_cursor, 4 * nranges);
    }
    w->nnz_cap = -1;  // the graph state allocates tile table and bins
    int rc = ws_graph_state(w, g, s);
    if (rc) { ws_free(w); return rc; }
    (void)ctx;
    *out = w;
    return GDE_OK;
}

static int ws_ensure_hk(Workspace *w, const gde_graph *g, hipStream_t s) {
    const int64_t n = w->n;
    if (!w->rd2) {
        GDE_HIP(hipMalloc(&w->rd2, 2 * w->vsize * n));
        GDE_HIP(hipMemsetAsync(w->rd2, 0, 2 * w->vsize * n, s));
        if (w->vtype == GDE_F64) launch_init_rd<double>(g->row_ptr, w->rd2, g->n, s);
        else launch_init_rd<float>(g->row_ptr, w->rd2, g->n, s);
        GDE_HIP(hipGetLastError());
    }
    for (int i = 0; i < 3; i++)
        if (!w->touched[i]) {
            GDE_HIP(hipMalloc((void **)&w->touched[i], 4 * n));
        }
    if (!w->lvl_tab) GDE_HIP(hipMalloc((void **)&w->lvl_tab, 16 * (size_t)(kHkMaxLevels + 1)));
    return GDE_OK;
}

static int ws_ensure_ch(Workspace *w, hipStream_t s) {
    const int64_t n = w->n;
    if (!w->delta) {
        GDE_HIP(hipMalloc(&w->delta, w->vsize * n));
        GDE_HIP(hipMemsetAsync(w->delta, 0, w->vsize * n, s));
        GDE_HIP(hipMalloc((void **)&w->dstamp, 4 * n));
        GDE_HIP(hipMemsetAsync(w->dstamp, 0, 4 * n, s));
        GDE_HIP(hipMalloc((void **)&w->cstamp, 4 * n));
        GDE_HIP(hipMemsetAsync(w->cstamp, 0, 4 * n, s));
        w->stamp_base = 1;
    }
    return GDE_OK;
}

static int ws_ensure_seed(Workspace *w, int32_t nnz) {
    if (nnz <= w->seed_cap) return GDE_OK;
    int32_t cap = std::max<int32_t>(nnz, 64);
    if (w->seed_idx) { (void)hipFree(w->seed_idx); (void)hipFree(w->seed_val); }
    if (w->h_seed_idx) { (void)hipHostFree(w->h_seed_idx); (void)hipHostFree(w->h_seed_val); }
    w->seed_idx = nullptr; w->seed_val = nullptr; w->h_seed_idx = nullptr; w->h_seed_val = nullptr; w->seed_cap = 0;
    GDE_HIP(hipMalloc((void **)&w->seed_idx, 4 * (size_t)cap));
    GDE_HIP(hipMalloc((void **)&w->seed_val, 8 * (size_t)cap));
    GDE_HIP(hipHostMalloc((void **)&w->h_seed_idx, 4 * (size_t)cap, hipHostMallocDefault));
    GDE_HIP(hipHostMalloc((void **)&w->h_seed_val, 8 * (size_t)cap, hipHostMallocDefault));
    w->seed_cap = cap;
    return GDE_OK;
}

static int ws_ensure_out(Workspace *w, int64_t cap) {
    if (cap <= w->out_cap) return GDE_OK;
    if (w->out_idx) { (void)hipFree(w->out_idx); (void)hipFree(w->out_val); }
    w->out_idx = nullptr; w->out_val = nullptr; w->out_cap = 0;
    GDE_HIP(hipMalloc((void **)&w->out_idx, 4 * (size_t)cap));
    GDE_HIP(hipMalloc(&w->out_val, w->vsize * (size_t)cap));
    w->out_cap = cap;
    return GDE_OK;
}

static int ws_ensure_trace(Workspace *w, int64_t cap, int64_t ncap) {
    if (cap > w->tr_cap) {
        if (w->tr_size) { (void)hipFree(w->tr_size); (void)hipFree(w->tr_vol); }
        w->tr_size = w->tr_vol = nullptr; w->tr_cap = 0;
        GDE_HIP(hipMalloc((void **)&w->tr_size, 8 * (size_t)cap));
        GDE_HIP(hipMalloc((void **)&w->tr_vol, 8 * (size_t)cap));
        w->tr_cap = cap;
    }
    if (ncap > w->tr_nodes_cap) {
        if (w->tr_nodes) (void)hipFree(w->tr_nodes);
        w->tr_nodes = nullptr; w->tr_nodes_cap = 0;
        GDE_HIP(hipMalloc((void **)&w->tr_nodes, 4 * (size_t)ncap));
        w->tr_nodes_cap = ncap;
    }
    return GDE_OK;
}

int get_workspace(gde_ctx *ctx, const gde_graph *g, int vtype, hipStream_t s, Workspace **out) {
    for (Workspace *w : ctx->ws)
        if (w->guid == g->uid && w->vtype == vtype) { w->g = g; *out = w; return GDE_OK; }
    // keep a small number of workspaces per context
    while (ctx->ws.size() >= 4) {
        ws_free(ctx->ws.front());
        ctx->ws.erase(ctx->ws.begin());
    }
    Workspace *w = nullptr;
    int rc = ws_create(ctx, g, vtype, s, &w);
    if (rc) return rc;
    ctx->ws.push_back(w);
    *out = w;
    return GDE_OK;
}

void drop_workspaces_of(const gde_graph *g, gde_ctx *ctx) {
    for (size_t i = 0; i < ctx->ws.size();) {
        if (ctx->ws[i]->guid == g->uid) { ws_free(ctx->ws[i]); ctx->ws.erase(ctx->ws.begin() + i); }
        else i++;
    }
    drop_batch_workspaces_of(g, ctx);
}

// ------------------------------------------------------------------ kernel timing
int prof_mark(gde_ctx *ctx, hipStream_t s) {
    if (!ctx || !ctx->prof_on) return GDE_OK;
    if (ctx->ev_used == ctx->ev.size()) {
        hipEvent_t e;
        GDE_HIP(hipEventCreate(&e));
        ctx->ev.push_back(e);
    }
    GDE_HIP(hipEventRecord(ctx->ev[ctx->ev_used++], s));
    return GDE_OK;
}

// after the stream has been synchronised: fold the recorded pairs into the totals
int prof_collect(gde_ctx *ctx, int64_t edges, int64_t entries) {
    if (!ctx || !ctx->prof_on) return GDE_OK;
    for (size_t i = 0; i + 1 < ctx->ev_used; i += 2) {
        float ms = 0.f;
        GDE_HIP(hipEventElapsedTime(&ms, ctx->ev[i], ctx->ev[i + 1]));
        ctx->prof_ms += ms;
        ctx->prof_launches++;
    }
    ctx->ev_used = 0;
    ctx->prof_edges += edges;
    ctx->prof_entries += entries;
    return GDE_OK;
}

int prof_mark_batch(gde_ctx *ctx, hipStream_t s) {
    if (!ctx->prof_on) return GDE_OK;
    for (int i = 0; i < 2; i++)
        if (!ctx->ev_b[i]) GDE_HIP(hipEventCreate(&ctx->ev_b[i]));
    if (ctx->ev_b_used >= 2) ctx->ev_b_used = 0;
    GDE_HIP(hipEventRecord(ctx->ev_b[ctx->ev_b_used++], s));
    return GDE_OK;
}

// an event before or after one batched push launch
int prof_mark_batch_push(gde_ctx *ctx, hipStream_t s) {
    if (!ctx->prof_on) return GDE_OK;
    if (ctx->ev_bp_used == ctx->ev_bp.size()) {
        hipEvent_t e;
        GDE_HIP(hipEventCreate(&e));
        ctx->ev_bp.push_back(e);
    }
    GDE_HIP(hipEventRecord(ctx->ev_bp[ctx->ev_bp_used++], s));
    return GDE_OK;
}

int prof_collect_batch(gde_ctx *ctx, int64_t lane_edges, int64_t entries, int64_t rows, int64_t row_vol) {
    if (!ctx->prof_on) return GDE_OK;
    if (ctx->ev_b_used == 2) {
        float ms = 0.f;
        GDE_HIP(hipEventElapsedTime(&ms, ctx->ev_b[0], ctx->ev_b[1]));
        ctx->prof_b_ms += ms;
        ctx->prof_b_launches++;
        ctx->prof_b_lane_edges += lane_edges;
        ctx->prof_b_entries += entries;
        ctx->prof_b_rows += rows;
        ctx->prof_b_row_vol += row_vol;
    }
    for (size_t i = 0; i + 1 < ctx->ev_bp_used; i += 2) {
        float ms = 0.f;
        GDE_HIP(hipEventElapsedTime(&ms, ctx->ev_bp[i], ctx->ev_bp[i + 1]));
        ctx->prof_bp_ms += ms;
        ctx->prof_bp_launches++;
    }
    ctx->ev_b_used = 0;
    ctx->ev_bp_used = 0;
    return GDE_OK;
}

int gde_validate_query(const gde_graph *g, const gde_params *p, const gde_seed *s) {
    int rc = validate_params(p);
    if (rc) return rc;
    GraphHost *gh = graph_host(g);
    if (!gh) return fail(GDE_ERR_INVALID_ARG, "unknown graph handle");
    return validate_seed_deg(s, g->n, gh->deg);
}

static void register_graph(gde_graph *g, GraphHost *gh) {
    gh->deg.resize(g->n);
    for (int32_t u = 0; u < g->n; u++) gh->deg[u] = gh->row_ptr[u + 1] - gh->row_ptr[u];
    std::lock_guard<std::mutex> lk(g_graph_mu);
    g_graph_host.emplace_back(g, gh);
}

// a graph over device CSR arrays that the library takes ownership of (the server's private copy)
gde_graph *graph_wrap_device(gde_ctx *ctx, int32_t n, int64_t nnz, int32_t *rp, int32_t *ci) {
    gde_graph *g = new gde_graph();
    g->device = ctx->device;
    g->n = n;
    g->nnz = nnz;
    g->row_ptr = rp;
    g->col_idx = ci;
    g->owned = true;
    g->uid = g_uid++;
    GraphHost *gh = new GraphHost();
    gh->row_ptr.resize((size_t)n + 1);
    (void)hipMemcpy(gh->row_ptr.data(), rp, 4 * ((size_t)n + 1), hipMemcpyDeviceToHost);
    register_graph(g, gh);
    return g;
}

// swap in a rebuilt CSR (owned); degrees of the host copy grow by `inc` (directed sources)
int graph_replace_csr(gde_graph *g, int32_t *rp, int32_t *ci, int64_t nnz, const std::vector<int32_t> &inc) {
    if (g->owned) {
        (void)hipFree(g->row_ptr);
        (void)hipFree(g->col_idx);
    }
    g->row_ptr = rp;
    g->col_idx = ci;
    g->nnz = nnz;
    g->owned = true;
    GraphHost *gh = graph_host(g);
    if (gh)
        for (int32_t u : inc) gh->deg[u]++;
    return GDE_OK;
}

// swap in a rebuilt CSR (owned), and drop every context's workspaces of g
// (their tile tables, bins and degrees are stale); the host degrees follow
// through graph_add_degrees
int graph_set_csr(gde_graph *g, int32_t *rp, int32_t *ci, int64_t nnz) {
    {
        std::lock_guard<std::mutex> lk(g_ctx_mu);
        for (gde_ctx *c : g_ctxs) drop_workspaces_of(g, c);
    }
    if (g->owned) {
        (void)hipFree(g->row_ptr);
        (void)hipFree(g->col_idx);
    }
    g->row_ptr = rp;
    g->col_idx = ci;
    g->nnz = nnz;
    g->owned = true;
    return GDE_OK;
}

// the host degrees of `nodes` change by delta (an edge event at each); d_max
// stays an upper bound
void graph_add_degrees(gde_graph *g, const int32_t *nodes, int32_t k, int32_t delta) {
    GraphHost *gh = graph_host(g);
    if (!gh) return;
    for (int32_t i = 0; i < k; i++) {
        const int32_t d = gh->deg[nodes[i]] += delta;
        g->d_max = std::max(g->d_max, d);
    }
}

void plain_workspaces_drop(const gde_graph *g, gde_ctx *ctx) {
    for (size_t i = 0; i < ctx->ws.size();) {
        if (ctx->ws[i]->guid == g->uid) { ws_free(ctx->ws[i]); ctx->ws.erase(ctx->ws.begin() + i); }
        else i++;
    }
}

// after the CSR of g was replaced (same node count): update every workspace of g in place
int plain_workspaces_refresh(const gde_graph *g, gde_ctx *ctx, hipStream_t s) {
    for (size_t i = 0; i < ctx->ws.size(); i++)
        if (ctx->ws[i]->guid == g->uid) {
            const int rc = ws_graph_state(ctx->ws[i], g, s);
            if (rc) {
                plain_workspaces_drop(g, ctx);
                return rc;
            }
        }
    return GDE_OK;
}

// ------------------------------------------------------------------ the plain solver
static int push_grid(const gde_graph *g) {
    int64_t tiles = g->nnz / kPushTile + 1;
    return (int)std::min<int64_t>(std::max<int64_t>(tiles, 1), 512);
}
static int snap_grid(const gde_graph *g) {
    return (int)std::max<int64_t>(std::min<int64_t>((g->n + kSnapBlock - 1) / kSnapBlock, 512), 1);
}

// Makes the device state of w visible in w->hst: the publication kernel is
// enqueued after everything on s and the host polls its sequence number for a
// short while (the runtime's blocking wait resumes later than a polling host);
// a longer wait, or a stream that failed, falls back to the blocking wait.
static int sync_state(Workspace *w, hipStream_t s) {
    constexpr double kSpinSeconds = 2e-3;
    if (!w->hst_dev) {  // no host-coherent mirror: copy the state and wait for the stream
        GDE_HIP(hipMemcpyAsync(w->hst, w->st, sizeof(DevState), hipMemcpyDeviceToHost, s));
        GDE_HIP(hipStreamSynchronize(s));
        return GDE_OK;
    }
    const uint32_t want = ++w->seq;
    launch_publish(w->st, w->hst_dev, w->hseq_dev, want, s);
    GDE_HIP(hipGetLastError());
    const auto t0 = std::chrono::steady_clock::now();
    for (int k = 0;; k++) {
        if (__atomic_load_n(w->hseq, __ATOMIC_ACQUIRE) == want) return GDE_OK;
        if ((k & 255) == 255 &&
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > kSpinSeconds)
            break;
        __builtin_ia32_pause();
    }
    GDE_HIP(hipStreamSynchronize(s));
    if (__atomic_load_n(w->hseq, __ATOMIC_ACQUIRE) != want) return fail(GDE_ERR_DEVICE, "state publication missing");
    return GDE_OK;
}

// One plain solve on the workspace w.  ctx may be null (no kernel timing); a
// workspace whose buffers are all present (a view onto fixed device memory)
// makes the ws_ensure_* calls no-ops, and one without pinned mirrors reads the
// device state with a copy and a stream synchronisation.
template <typename V>
int solve_plain_ws(gde_ctx *ctx, const gde_graph *g, const gde_params *p, const gde_seed *sd, gde_result *res,
                   Workspace *w, hipStream_t s) {
    int rc = GDE_OK;
    const bool hk = p->kind == GDE_HK || p->kind == GDE_SERIES;  // the level push
    const bool ch = p->method == GDE_LOCAL_CH;
    // D^-1/2 A D^-1/2: seed scaled by sqrt(d), output by 1/sqrt(d) (the kernels read the degrees)
    const int32_t *sym_rp = (p->flags & GDE_SYM_NORM) ? g->row_ptr : nullptr;
    if (hk && (rc = ws_ensure_hk(w, g, s))) return rc;
    if (ch && (rc = ws_ensure_ch(w, s))) return rc;
    if ((rc = ws_ensure_seed(w, sd->nnz))) return rc;
    const bool trace = (p->flags & GDE_TRACE) != 0;
    long long tr_cap = 0, tr_ncap = 0;
    if (trace) {
        tr_cap = std::max<int64_t>(res->trace_capacity, 0);
        tr_ncap = res->trace_nodes ? std::max<int64_t>(res->trace_nodes_capacity, 0) : 0;
        if ((rc = ws_ensure_trace(w, std::max<long long>(tr_cap, 1), std::max<long long>(tr_ncap, 1)))) return rc;
    }
    long long *d_trs = trace && tr_cap > 0 ? (long long *)w->tr_size : nullptr;
    long long *d_trv = trace && tr_cap > 0 ? (long long *)w->tr_vol : nullptr;
    int32_t *d_trn = trace && tr_ncap > 0 ? w->tr_nodes : nullptr;

    // a small seed travels in the seed kernel's arguments; a larger one (or one
    // the Katz seed subtraction reads again) through the device seed buffers
    const bool sub_seed = p->kind == GDE_KATZ && (p->flags & GDE_KATZ_SUBTRACT_SEED);
    SeedInline inl{};
    const SeedInline *pinl = nullptr;
    if (sd->nnz <= kSeedInline && !sub_seed) {
        inl.n = sd->nnz;
        for (int32_t i = 0; i < sd->nnz; i++) {
            inl.idx[i] = sd->idx[i];
            inl.val[i] = sd->val[i];
        }
        pinl = &inl;
    } else if (w->h_seed_idx) {
        std::memcpy(w->h_seed_idx, sd->idx, 4 * (size_t)sd->nnz);
        std::memcpy(w->h_seed_val, sd->val, 8 * (size_t)sd->nnz);
        GDE_HIP(hipMemcpyAsync(w->seed_idx, w->h_seed_idx, 4 * (size_t)sd->nnz, hipMemcpyHostToDevice, s));
        GDE_HIP(hipMemcpyAsync(w->seed_val, w->h_seed_val, 8 * (size_t)sd->nnz, hipMemcpyHostToDevice, s));
    } else {  // no pinned staging: copy from the caller's arrays (the runtime stages pageable memory)
        GDE_HIP(hipMemcpyAsync(w->seed_idx, sd->idx, 4 * (size_t)sd->nnz, hipMemcpyHostToDevice, s));
        GDE_HIP(hipMemcpyAsync(w->seed_val, sd->val, 8 * (size_t)sd->nnz, hipMemcpyHostToDevice, s));
    }

    const int pgrid = push_grid(g), sgrid = snap_grid(g);
    BinArgs<V> bins{};
    if (w->bin_nranges > 0) {
        bins.shift = w->bin_shift;
        bins.nranges = w->bin_nranges;
        const long long nr = w->bin_nranges;
        const long long min_binned = std::max(kBinMinEdges, nr * nr / kBinRangeSqDiv);
        bins.min_edges = (p->flags & GDE_SCATTER_BINNED) ? 0 : min_binned;
        if ((p->flags & GDE_SCATTER_ATOMIC) || (nr < kBinMinRanges && !(p->flags & GDE_SCATTER_BINNED)))
            bins.nranges = 0;
        // PPR LocalGD: no iteration can reach the binning threshold when the whole
        // work bound vol(supp s) + ||s||_1 / (alpha eps) (Corollary 3.5) stays below
        // it; then neither the binned path nor the range-reduction launches are needed
        if (bins.nranges > 0 && !(p->flags & GDE_SCATTER_BINNED) && p->kind == GDE_PPR &&
            p->method == GDE_LOCAL_GD) {
            GraphHost *gh = graph_host(g);
            double bound = 0.0;
            for (int32_t i = 0; i < sd->nnz; i++)
                bound += (gh ? (double)gh->deg[sd->idx[i]] : (double)g->nnz) + sd->val[i] / (p->alpha * p->eps);
            if (bound < (double)min_binned) bins.nranges = 0;
        }
        bins.base = w->bin_base;
        bins.cursor = w->bin_cursor;
        bins.be = (BinEnt<V> *)w->bin_e;
    }
    SnapArgs a{};
    a.grid = sgrid;
    a.row_ptr = g->row_ptr;
    a.x = w->x;
    a.bitmap = w->bitmap;
    a.st = w->st;
    a.wl_node = w->wl_node;
    a.wl_beg = w->wl_beg;
    a.wl_off = w->wl_off;
    a.wl_sv = w->wl_sv;
    a.tile_start = w->tile_start;
    a.tr_nodes = d_trn;
    a.tr_cap = tr_ncap;
    a.cap = g->n;

    bool converged = false;
    int status = GDE_OK;
    if (p->flags & GDE_DETERMINISTIC) {
        // fixed-order iterations (pull instead of scatter), any kind and method
        if ((rc = det_run<V>(g, p, sd, w, pinl, d_trs, d_trv, d_trn, tr_cap, tr_ncap, s, &converged))) return rc;
    } else if (hk) {
        // ------------------------------------------------ heat kernel or SERIES, level by level
        const int K = p->K;
        const LevelSeries ls = level_series(p);
        const std::vector<double> &psi = ls.psi;
        // the single-workgroup kernel reads psi and the level ratios from the device table
        w->h_lvl.assign(2 * (size_t)(kHkMaxLevels + 1), 0.0);
        std::copy(ls.psi.begin(), ls.psi.end(), w->h_lvl.begin());
        std::copy(ls.ratio.begin(), ls.ratio.end(), w->h_lvl.begin() + kHkMaxLevels + 1);
        GDE_HIP(hipMemcpyAsync(w->lvl_tab, w->h_lvl.data(), 8 * w->h_lvl.size(), hipMemcpyHostToDevice, s));
        void *plane[2] = {w->rd, w->rd2};
        launch_seed_init<V>(w->rd, w->seed_idx, w->seed_val, pinl, sd->nnz, ls.c0, w->front[0], w->touched[0],
                            nullptr, 0, nullptr, w->st, s, sym_rp);
        auto eps_at = [&](int k) { return k >= K ? 0.0 : p->eps / ((double)(K + 1) * psi[k + 1]); };
        // level k on the grid-wide kernels: clean-up of k-1 and snapshot of k, then the push into k+1
        auto grid_level = [&](int k) -> int {
            a.rd = plane[k & 1];
            a.F = w->front[k & 1];
            a.cur = k & 1;
            const bool last = k == K;
            launch_snap_hk<V>(a, plane[(k + 1) & 1], (V)ls.ratio[k], last ? 1 : 0, 1,
                              k >= 1 ? w->touched[(k + 2) % 3] : nullptr, (k + 2) % 3, (k + 1) % 3,
                              k >= 1 ? psi[k - 1] : 0.0, k >= 1 ? (double)(K + 1) * psi[k - 1] : 0.0, s);
            int e = prof_mark(ctx, s);
            if (e) return e;
            launch_push<V>(1, pgrid, g->col_idx, plane[(k + 1) & 1], w->st, k & 1, w->wl_beg, w->wl_off, w->wl_sv,
                           w->tile_start, (V)eps_at(k), w->front[(k + 1) & 1], w->touched[(k + 1) % 3], (k + 1) % 3,
                           nullptr, 0, nullptr, d_trs, d_trv, tr_cap, last ? 0 : 1, g->n, (int32_t)g->nnz, bins, nullptr,
                           s);
            return prof_mark(ctx, s);
        };
        // small frontiers: one workgroup runs levels k .. (and the final clean-up)
        const bool small_ok = !(p->flags & GDE_SCATTER_BINNED);
        HkSmallArgs<V> ha{};
        ha.row_ptr = g->row_ptr;
        ha.col_idx = g->col_idx;
        ha.plane[0] = plane[0];
        ha.plane[1] = plane[1];
        ha.x = w->x;
        ha.bitmap = w->bitmap;
        ha.st = w->st;
        for (int i = 0; i < 2; i++) ha.front[i] = w->front[i];
        for (int i = 0; i < 3; i++) ha.touched[i] = w->touched[i];
        ha.wl_beg = w->wl_beg;
        ha.wl_off = w->wl_off;
        ha.wl_sv = w->wl_sv;
        ha.tile_start = w->tile_start;
        ha.tr_nodes = d_trn;
        ha.tr_ncap = tr_ncap;
        ha.tr_size = d_trs;
        ha.tr_vol = d_trv;
        ha.tr_cap = tr_cap;
        ha.lvl_tab = w->lvl_tab;
        ha.eps = p->eps;
        ha.K = K;
        ha.cap = g->n;
        ha.nnz = (int32_t)g->nnz;
        int k = 0;
        bool done = false;
        auto run_small_hk = [&]() -> int {
            ha.k0 = k;
            int e = prof_mark(ctx, s);
            if (e) return e;
            launch_small_hk<V>(ha, s);
            if ((e = prof_mark(ctx, s))) return e;
            GDE_HIP(hipGetLastError());
            if ((e = sync_state(w, s))) return e;
            k = w->hst->small_t;
            if (w->hst->small_phase == 2) {
                done = true;
            } else if (w->hst->small_phase == 1) {  // the snapshot of level k is done; its push is not
                if ((e = prof_mark(ctx, s))) return e;
                launch_push<V>(1, pgrid, g->col_idx, plane[(k + 1) & 1], w->st, k & 1, w->wl_beg, w->wl_off,
                               w->wl_sv, w->tile_start, (V)eps_at(k), w->front[(k + 1) & 1], w->touched[(k + 1) % 3],
                               (k + 1) % 3, nullptr, 0, nullptr, d_trs, d_trv, tr_cap, 1, g->n, (int32_t)g->nnz,
                               bins, nullptr, s);
                if ((e = prof_mark(ctx, s))) return e;
                k++;
            }
            return GDE_OK;
        };
        if (small_ok && (rc = run_small_hk())) return rc;
        // grid-wide levels: eight, then one synchronisation that hands a frontier
        // which has shrunk back to the single workgroup, then the rest back to
        // back (a synchronisation per chunk of levels measured slower than it saved)
        for (int pass = 0; pass < 2 && !done && k <= K; pass++) {
            const int end = pass == 0 && small_ok ? std::min(K + 1, k + 8) : K + 1;
            for (; k < end; k++)
                if ((rc = grid_level(k))) return rc;
            if (pass == 0 && small_ok && k <= K) {
                if ((rc = sync_state(w, s))) return rc;
                if (w->hst->fcount[k & 1] <= kSmallMaxNodes && w->hst->tcount[(k + 2) % 3] <= kSmallMaxEdges &&
                    (rc = run_small_hk()))
                    return rc;
            }
        }
        if (!done) {  // clean-up of the last level
            a.rd = plane[(K + 1) & 1];
            a.F = w->front[(K + 1) & 1];
            a.cur = (K + 1) & 1;
            launch_snap_hk<V>(a, plane[K & 1], (V)0, 1, 0, w->touched[K % 3], K % 3, -1, psi[K],
                              (double)(K + 1) * psi[K], s);
        }
        GDE_HIP(hipGetLastError());
        converged = true;
    } else {
        // ------------------------------------------------ PPR / Katz, LocalGD or LocalCH
        const bool ppr = p->kind == GDE_PPR;
        const double bscale = ppr ? p->alpha : 1.0;
        const V wscale = (V)(ppr ? 1.0 - p->alpha : p->beta);
        const int w_div_deg = ppr ? 1 : 0;
        const V eps_eff = (V)(ppr ? p->alpha * p->eps : p->eps);
        double sigma = 1.0, dlt = 0.0;
        int32_t base = 0;
        if (ch) {
            double mu, L;
            if (ppr) { mu = p->alpha; L = 2.0 - p->alpha; }
            else { mu = 1.0 - p->beta * p->lambda_bound; L = 1.0 + p->beta * p->lambda_bound; }
            sigma = (L + mu) / (L - mu);
            dlt = 1.0 / sigma;
            if (w->stamp_base > (1 << 30) - p->max_iters - 4) {
                GDE_HIP(hipMemsetAsync(w->dstamp, 0, 4 * (size_t)w->n, s));
                GDE_HIP(hipMemsetAsync(w->cstamp, 0, 4 * (size_t)w->n, s));
                w->stamp_base = 1;
            }
            base = w->stamp_base;
        }
        launch_seed_init<V>(w->rd, w->seed_idx, w->seed_val, pinl, sd->nnz, bscale, w->front[0], nullptr,
                            ch ? w->cstamp : nullptr, base, w->tbm, w->st, s, sym_rp);
        a.rd = w->rd;
        // LocalCH scalars (c_t, m_t) of iteration t: delta_{t+1} = 1 / (2 sigma - delta_t),
        // c_t = 2 sigma delta_{t+1}, m_t = delta_t delta_{t+1}; t = 0 is the forced first step
        std::vector<std::pair<V, V>> chs;
        auto ch_at = [&](int tt) {
            while ((int)chs.size() <= tt) {
                if (chs.empty()) {
                    chs.push_back({(V)1, (V)0});
                } else {
                    const double dnext = 1.0 / (2.0 * sigma - dlt);
                    chs.push_back({(V)(2.0 * sigma * dnext), (V)(dlt * dnext)});
                    dlt = dnext;
                }
            }
            return chs[tt];
        };
        int t = 0;
        const bool small_ok = !(p->flags & GDE_SCATTER_BINNED);
        SmallArgs<V> sa{};
        if (small_ok) {
            sa.row_ptr = g->row_ptr;
            sa.col_idx = g->col_idx;
            sa.rd = w->rd;
            sa.x = w->x;
            sa.bitmap = w->bitmap;
            sa.tbm = w->tbm;
            sa.st = w->st;
            sa.front0 = w->front[0];
            sa.front1 = w->front[1];
            sa.wl_node = w->wl_node;
            sa.wl_beg = w->wl_beg;
            sa.wl_off = w->wl_off;
            sa.wl_sv = w->wl_sv;
            sa.tile_start = w->tile_start;
            sa.tr_nodes = d_trn;
            sa.tr_ncap = tr_ncap;
            sa.tr_size = d_trs;
            sa.tr_vol = d_trv;
            sa.tr_cap = tr_cap;
            sa.wscale = wscale;
            sa.eps_eff = eps_eff;
            sa.w_div_deg = w_div_deg;
            sa.delta = w->delta;
            sa.dstamp = w->dstamp;
            sa.cstamp = w->cstamp;
            sa.stamp_base = base;
            sa.cap = g->n;
            sa.nnz = (int32_t)g->nnz;
        }
        // Small frontiers: one workgroup runs iterations t .. until the frontier
        // outgrows it, the solve converges or kSmallIters have run; then the host
        // reads where it stopped.  Used for the first iterations and again for the
        // tail, whenever a synchronisation finds the frontier small.
        auto run_small = [&]() -> int {
            sa.t0 = t;
            sa.t_end = std::min(p->max_iters, t + kSmallIters);
            if (ch)
                for (int k = t; k < sa.t_end; k++) {
                    const auto cm = ch_at(k);
                    sa.c_seq[k - t] = cm.first;
                    sa.m_seq[k - t] = cm.second;
                }
            int e = prof_mark(ctx, s);
            if (e) return e;
            launch_small<V>(sa, ch, s);
            if ((e = prof_mark(ctx, s))) return e;
            GDE_HIP(hipGetLastError());
            if ((e = sync_state(w, s))) return e;
            t = w->hst->small_t;
            if (w->hst->empty_seen || (!ch && w->hst->fcount[t & 1] == 0)) {
                converged = true;
            } else if (w->hst->small_phase == 1) {  // S_t is snapshot; its volume needs the grid-wide push
                if ((e = prof_mark(ctx, s))) return e;
                if (ch)
                    launch_push<V>(2, pgrid, g->col_idx, w->rd, w->st, t & 1, w->wl_beg, w->wl_off, w->wl_sv,
                                   w->tile_start, eps_eff, w->front[(t + 1) & 1], nullptr, 0, w->cstamp, base + t + 1,
                                   w->tbm, d_trs, d_trv, tr_cap, 1, g->n, (int32_t)g->nnz, bins, nullptr, s);
                else
                    launch_push<V>(0, pgrid, g->col_idx, w->rd, w->st, t & 1, w->wl_beg, w->wl_off, w->wl_sv,
                                   w->tile_start, eps_eff, w->front[(t + 1) & 1], nullptr, 0, nullptr, 0, w->tbm, d_trs,
                                   d_trv, tr_cap, 1, g->n, (int32_t)g->nnz, bins, nullptr, s);
                if ((e = prof_mark(ctx, s))) return e;
                t++;
            }
            return GDE_OK;
        };
        if (small_ok && (rc = run_small())) return rc;
        // grid-wide iterations in chunks between host synchronisations: 8, then
        // doubling up to 32 while the frontier stays large.  Inside a chunk the
        // range reduction of iteration t also takes the snapshot of t+1 (fused
        // into the reduction when t is binned, over the list otherwise), so an
        // iteration is two launches; the last reduction of a chunk does not, so
        // that every synchronisation sees an iteration boundary.
        FuseArgs<V> fz{};
        fz.row_ptr = g->row_ptr;
        fz.x = (V *)w->x;
        fz.bitmap = w->bitmap;
        fz.wl_node = w->wl_node;
        fz.wl_beg = w->wl_beg;
        fz.wl_off = w->wl_off;
        fz.wl_sv = (V *)w->wl_sv;
        fz.tile_start = w->tile_start;
        fz.tr_nodes = d_trn;
        fz.tr_cap = tr_ncap;
        fz.wscale = wscale;
        fz.w_div_deg = w_div_deg;
        fz.delta = (V *)w->delta;
        fz.dstamp = w->dstamp;
        fz.cap = g->n;
        int chunk = 8;
        while (!converged && t < p->max_iters) {
            int end = std::min(p->max_iters, t + chunk);
            bool taken = false;  // the range reduction of t-1 took the snapshot of t
            for (; t < end; t++) {
                a.F = w->front[t & 1];
                a.cur = t & 1;
                if (ch) {
                    const auto cm = ch_at(t);
                    const V c_t = cm.first, m_t = cm.second;
                    if (!taken)
                        launch_snap_ch<V>(a, wscale, w_div_deg, eps_eff, c_t, m_t, t == 0 ? 1 : 0, w->delta,
                                          w->dstamp, w->cstamp, base + t, w->front[(t + 1) & 1], s);
                    if ((rc = prof_mark(ctx, s))) return rc;
                    fz.on = t + 1 < end ? 1 : 0;
                    fz.c_next = ch_at(t + 1).first;
                    fz.m_next = ch_at(t + 1).second;
                    fz.list2 = w->front[t & 1];
                    launch_push<V>(2, pgrid, g->col_idx, w->rd, w->st, t & 1, w->wl_beg, w->wl_off, w->wl_sv,
                                   w->tile_start, eps_eff, w->front[(t + 1) & 1], nullptr, 0, w->cstamp, base + t + 1,
                                   w->tbm, d_trs, d_trv, tr_cap, 1, g->n, (int32_t)g->nnz, bins, &fz, s);
                    if ((rc = prof_mark(ctx, s))) return rc;
                } else {
                    if (!taken) launch_snap_gd<V>(a, wscale, w_div_deg, s);
                    if ((rc = prof_mark(ctx, s))) return rc;
                    fz.on = t + 1 < end ? 1 : 0;
                    launch_push<V>(0, pgrid, g->col_idx, w->rd, w->st, t & 1, w->wl_beg, w->wl_off, w->wl_sv,
                                   w->tile_start, eps_eff, w->front[(t + 1) & 1], nullptr, 0, nullptr, 0, w->tbm, d_trs,
                                   d_trv, tr_cap, 1, g->n, (int32_t)g->nnz, bins, &fz, s);
                    if ((rc = prof_mark(ctx, s))) return rc;
                }
                // a launched range reduction with fusion on takes the next snapshot,
                // binned (fused) or over the list (atomic iteration)
                taken = fz.on && bins.nranges > 0;
            }
            GDE_HIP(hipGetLastError());
            if ((rc = sync_state(w, s))) return rc;
            if (w->hst->empty_seen || (!ch && w->hst->fcount[t & 1] == 0)) { converged = true; break; }
            if (small_ok && t < p->max_iters && w->hst->fcount[t & 1] <= kSmallMaxNodes) {
                if ((rc = run_small())) return rc;
                chunk = 8;
            } else {
                chunk = std::min(chunk * 2, 32);
            }
        }
        if (!converged) {
            if (ch) {
                launch_ch_probe<V>(w->rd, w->front[t & 1], w->st, t & 1, eps_eff, g->n, s);
                GDE_HIP(hipGetLastError());
                if ((rc = sync_state(w, s))) return rc;
                converged = w->hst->probe == 0;
            } else {
                converged = w->hst->fcount[t & 1] == 0;
            }
        }
        if (ch) w->stamp_base += t + 2;
        launch_final_residual<V>(w->tbm, (w->n + 31) / 32, w->rd, w->st, ppr ? 1.0 / p->alpha : 1.0, s);
        if (p->kind == GDE_KATZ && (p->flags & GDE_KATZ_SUBTRACT_SEED))
            launch_subtract_seed<V>(w->x, w->seed_idx, w->seed_val, sd->nnz, s);
        GDE_HIP(hipGetLastError());
    }
    if (!converged) status = GDE_ERR_NOT_CONVERGED;

    // ------------------------------------------------ output (sorted by node id) and reset
    const int64_t nwords = (w->n + 31) / 32;
    const bool dev_out = (p->flags & GDE_RESULT_DEVICE) != 0;
    int64_t nnz = 0;
    bool fits = false;
    if (dev_out) {
        // device buffers: the output kernel itself checks |support| <= capacity
        // and writes nothing otherwise, so one synchronisation suffices
        const bool bufs = res->idx && res->val;
        launch_ex_count(w->bitmap, nwords, w->blk, w->nblk, s);
        launch_ex_scan(w->blk, w->nblk, w->st, s);
        launch_ex_emit<V>(w->bitmap, nwords, w->blk, w->nblk, w->x, bufs ? res->idx : nullptr,
                          bufs ? res->val : nullptr, bufs ? res->capacity : 0, w->st, s, sym_rp);
        GDE_HIP(hipGetLastError());
        if ((rc = sync_state(w, s))) return rc;
        nnz = w->hst->out_count;
        fits = bufs && nnz <= res->capacity;
    } else {
        // host buffers: the support size (from the output scan) decides the staging size
        launch_ex_count(w->bitmap, nwords, w->blk, w->nblk, s);
        launch_ex_scan(w->blk, w->nblk, w->st, s);
        GDE_HIP(hipGetLastError());
        if ((rc = sync_state(w, s))) return rc;
        nnz = w->hst->out_count;
        fits = nnz <= res->capacity && res->idx && res->val;
        int32_t *o_idx = nullptr;
        void *o_val = nullptr;
        if (fits) {
            if ((rc = ws_ensure_out(w, std::max<int64_t>(nnz, 1)))) return rc;
            o_idx = w->out_idx;
            o_val = w->out_val;
        }
        launch_ex_emit<V>(w->bitmap, nwords, w->blk, w->nblk, w->x, o_idx, o_val, fits ? nnz : 0, nullptr, s, sym_rp);
        GDE_HIP(hipGetLastError());
        if (fits && nnz > 0) {
            GDE_HIP(hipMemcpyAsync(res->idx, w->out_idx, 4 * (size_t)nnz, hipMemcpyDeviceToHost, s));
            GDE_HIP(hipMemcpyAsync(res->val, w->out_val, w->vsize * (size_t)nnz, hipMemcpyDeviceToHost, s));
        }
        // the caller's buffers may be pageable (filled by the runtime's staging),
        // so the final wait is the runtime's own
        GDE_HIP(hipMemcpyAsync(w->hst, w->st, sizeof(DevState), hipMemcpyDeviceToHost, s));
        GDE_HIP(hipStreamSynchronize(s));
    }
    const DevState &h = *w->hst;
    if (h.overflow) return fail(GDE_ERR_DEVICE, "internal list overflow (a frontier invariant was broken)");
    if ((rc = prof_collect(ctx, h.ops, h.pushes))) return rc;
    res->nnz = nnz;
    res->iters = h.iters;
    res->ops = h.ops;
    res->pushes = h.pushes;
    res->residual_l1 = h.res_l1;
    unsigned long long bits = h.res_dinf;
    double dinf;
    std::memcpy(&dinf, &bits, 8);
    res->residual_dinf = dinf;
    res->trace_len = h.iters;
    res->trace_nodes_len = h.pushes;
    if (trace) {
        int64_t m = std::min<int64_t>(h.iters, tr_cap);
        if (m > 0 && res->trace_size) GDE_HIP(hipMemcpy(res->trace_size, w->tr_size, 8 * m, hipMemcpyDeviceToHost));
        if (m > 0 && res->trace_vol) GDE_HIP(hipMemcpy(res->trace_vol, w->tr_vol, 8 * m, hipMemcpyDeviceToHost));
        int64_t mn = std::min<int64_t>(h.pushes, tr_ncap);
        if (mn > 0) GDE_HIP(hipMemcpy(res->trace_nodes, w->tr_nodes, 4 * mn, hipMemcpyDeviceToHost));
    }
    if (!fits) {
        res->status = GDE_ERR_CAPACITY;
        return fail(GDE_ERR_CAPACITY, "result capacity too small; result.nnz holds the size needed");
    }
    res->status = status;
    if (status == GDE_ERR_NOT_CONVERGED) return fail(status, "max_iters reached before S_t became empty");
    return GDE_OK;
}

template int solve_plain_ws<float>(gde_ctx *, const gde_graph *, const gde_params *, const gde_seed *, gde_result *,
                                   Workspace *, hipStream_t);
template int solve_plain_ws<double>(gde_ctx *, const gde_graph *, const gde_params *, const gde_seed *, gde_result *,
                                    Workspace *, hipStream_t);

template <typename V>
static int solve_plain(gde_ctx *ctx, const gde_graph *g, const gde_params *p, const gde_seed *sd, gde_result *res,
                       hipStream_t s) {
    Workspace *w = nullptr;
    int rc = get_workspace(ctx, g, p->value_type, s, &w);
    if (rc) return rc;
    return solve_plain_ws<V>(ctx, g, p, sd, res, w, s);
}

}  // namespace gde

using namespace gde;

extern "C" {

int gde_abi_version(void) { return GDE_ABI_VERSION; }

const char *gde_last_error(void) { return g_err.c_str(); }

int gde_ctx_create(int hip_device, gde_ctx **out) {
    if (!out) return fail(GDE_ERR_INVALID_ARG, "null out");
    int count = 0;
    GDE_HIP(hipGetDeviceCount(&count));
    if (hip_device < 0 || hip_device >= count) return fail(GDE_ERR_INVALID_ARG, "no such HIP device");
    GDE_HIP(hipSetDevice(hip_device));
    gde_ctx *c = new gde_ctx();
    c->device = hip_device;
    {
        std::lock_guard<std::mutex> lk(g_ctx_mu);
        g_ctxs.push_back(c);
    }
    *out = c;
    return GDE_OK;
}

int gde_ctx_destroy(gde_ctx *ctx) {
    if (!ctx) return fail(GDE_ERR_INVALID_ARG, "null ctx");
    {
        std::lock_guard<std::mutex> lk(g_ctx_mu);
        g_ctxs.erase(std::remove(g_ctxs.begin(), g_ctxs.end(), ctx), g_ctxs.end());
    }
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (Workspace *w : ctx->ws) ws_free(w);
    for (BatchWS *b : ctx->bws) batch_ws_free(b);
    for (hipEvent_t e : ctx->ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->ev_b)
        if (e) (void)hipEventDestroy(e);
    delete ctx;
    return GDE_OK;
}

int gde_ctx_profile(gde_ctx *ctx, int enable, gde_kernel_profile *out, int reset) {
    if (!ctx) return fail(GDE_ERR_INVALID_ARG, "null ctx");
    if (out) {
        out->launches = ctx->prof_launches;
        out->total_ms = ctx->prof_ms;
        out->edges = ctx->prof_edges;
        out->entries = ctx->prof_entries;
        out->batch_launches = ctx->prof_b_launches;
        out->batch_ms = ctx->prof_b_ms;
        out->batch_lane_edges = ctx->prof_b_lane_edges;
        out->batch_entries = ctx->prof_b_entries;
        out->batch_push_launches = ctx->prof_bp_launches;
        out->batch_push_ms = ctx->prof_bp_ms;
        out->batch_rows = ctx->prof_b_rows;
        out->batch_row_vol = ctx->prof_b_row_vol;
    }
    if (reset) {
        ctx->prof_launches = ctx->prof_edges = ctx->prof_entries = 0;
        ctx->prof_ms = 0.0;
        ctx->prof_b_launches = ctx->prof_b_lane_edges = ctx->prof_b_entries = 0;
        ctx->prof_b_ms = 0.0;
        ctx->prof_bp_launches = ctx->prof_b_rows = ctx->prof_b_row_vol = 0;
        ctx->prof_bp_ms = 0.0;
    }
    ctx->prof_on = enable != 0;
    ctx->ev_used = 0;
    return GDE_OK;
}

int gde_validate(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx, const gde_params *p,
                 const gde_seed *s) {
    int rc = validate_csr_host(n, nnz, row_ptr, col_idx);
    if (rc) return rc;
    if ((rc = validate_params(p))) return rc;
    return validate_seed(s, n, row_ptr);
}

int gde_graph_create(gde_ctx *ctx, int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                     uint32_t flags, hipStream_t stream, gde_graph **out) {
    if (!ctx || !out) return fail(GDE_ERR_INVALID_ARG, "null ctx or out");
    const bool host = (flags & GDE_HOST_PTRS) != 0, dev = (flags & GDE_DEVICE_PTRS) != 0;
    if (host == dev) return fail(GDE_ERR_INVALID_ARG, "exactly one of GDE_HOST_PTRS / GDE_DEVICE_PTRS");
    if ((flags & GDE_COPY) && (flags & GDE_BORROW)) return fail(GDE_ERR_INVALID_ARG, "GDE_COPY and GDE_BORROW");
    if (host && (flags & GDE_BORROW)) return fail(GDE_ERR_INVALID_ARG, "host pointers cannot be borrowed");
    if (n <= 0) return fail(GDE_ERR_INVALID_ARG, "n must be > 0");
    if (nnz < 0 || nnz >= (int64_t)INT32_MAX) return fail(GDE_ERR_INVALID_ARG, "nnz must be in [0, 2^31-1)");
    if (!row_ptr || (nnz > 0 && !col_idx)) return fail(GDE_ERR_INVALID_ARG, "null CSR pointer");
    GDE_HIP(hipSetDevice(ctx->device));
    GraphHost *gh = new GraphHost();
    gh->row_ptr.resize((size_t)n + 1);
    if (host) {
        int rc = validate_csr_host(n, nnz, row_ptr, col_idx);
        if (rc) { delete gh; return rc; }
        std::memcpy(gh->row_ptr.data(), row_ptr, 4 * ((size_t)n + 1));
    } else {
        hipError_t e = hipMemcpy(gh->row_ptr.data(), row_ptr, 4 * ((size_t)n + 1), hipMemcpyDeviceToHost);
        if (e != hipSuccess) { delete gh; return hip_fail(e, "hipMemcpy(row_ptr)"); }
        if (gh->row_ptr[0] != 0 || (int64_t)gh->row_ptr[n] != nnz) {
            delete gh;
            return fail(GDE_ERR_INVALID_ARG, "row_ptr must start at 0 and end at nnz");
        }
    }
    gde_graph *g = new gde_graph();
    g->device = ctx->device;
    g->n = n;
    g->nnz = nnz;
    g->uid = g_uid++;
    auto cleanup = [&](hipError_t e, const char *what) {
        if (g->owned) { (void)hipFree(g->row_ptr); (void)hipFree(g->col_idx); }
        delete g;
        delete gh;
        return hip_fail(e, what);
    };
    if (host || (flags & GDE_COPY) || !(flags & GDE_BORROW)) {
        hipError_t e = hipMalloc((void **)&g->row_ptr, 4 * ((size_t)n + 1));
        if (e != hipSuccess) return cleanup(e, "hipMalloc(row_ptr)");
        g->owned = true;
        e = hipMalloc((void **)&g->col_idx, 4 * (size_t)std::max<int64_t>(nnz, 1));
        if (e != hipSuccess) return cleanup(e, "hipMalloc(col_idx)");
        hipMemcpyKind kind = host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
        e = hipMemcpyAsync(g->row_ptr, row_ptr, 4 * ((size_t)n + 1), kind, stream);
        if (e == hipSuccess && nnz > 0) e = hipMemcpyAsync(g->col_idx, col_idx, 4 * (size_t)nnz, kind, stream);
        if (e != hipSuccess) return cleanup(e, "hipMemcpyAsync(csr)");
    } else {
        g->row_ptr = const_cast<int32_t *>(row_ptr);
        g->col_idx = const_cast<int32_t *>(col_idx);
    }
    // device-side structural check (covers device pointers; cheap for host ones)
    int32_t *chk = nullptr;
    hipError_t e = hipMalloc((void **)&chk, 8);
    if (e != hipSuccess) return cleanup(e, "hipMalloc(check)");
    e = hipMemsetAsync(chk, 0, 8, stream);
    if (e == hipSuccess) {
        launch_check_csr(g->row_ptr, g->col_idx, n, nnz, chk, chk + 1, stream);
        e = hipGetLastError();
    }
    int32_t hc[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(hc, chk, 8, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    (void)hipFree(chk);
    if (e != hipSuccess) return cleanup(e, "graph check");
    if (hc[0] != 0) {
        if (g->owned) { (void)hipFree(g->row_ptr); (void)hipFree(g->col_idx); }
        delete g;
        delete gh;
        return fail(GDE_ERR_INVALID_ARG, "malformed CSR (row_ptr order, col_idx range or self-loop)");
    }
    g->d_max = hc[1];
    register_graph(g, gh);
    *out = g;
    return GDE_OK;
}

int gde_graph_destroy(gde_graph *g) {
    if (!g) return fail(GDE_ERR_INVALID_ARG, "null graph");
    {
        std::lock_guard<std::mutex> lk(g_graph_mu);
        for (size_t i = 0; i < g_graph_host.size(); i++)
            if (g_graph_host[i].first == g) {
                delete g_graph_host[i].second;
                g_graph_host.erase(g_graph_host.begin() + i);
                break;
            }
    }
    (void)hipSetDevice(g->device);
    (void)hipDeviceSynchronize();
    {
        std::lock_guard<std::mutex> lk(g_ctx_mu);
        for (gde_ctx *c : g_ctxs) drop_workspaces_of(g, c);
    }
    if (g->owned) { (void)hipFree(g->row_ptr); (void)hipFree(g->col_idx); }
    delete g;
    return GDE_OK;
}

int gde_graph_info(const gde_graph *g, int32_t *n, int64_t *nnz) {
    if (!g) return fail(GDE_ERR_INVALID_ARG, "null graph");
    if (n) *n = g->n;
    if (nnz) *nnz = g->nnz;
    return GDE_OK;
}

int gde_graph_download(const gde_graph *g, int32_t *row_ptr, int32_t *col_idx) {
    if (!g) return fail(GDE_ERR_INVALID_ARG, "null graph");
    GDE_HIP(hipSetDevice(g->device));
    if (row_ptr) GDE_HIP(hipMemcpy(row_ptr, g->row_ptr, 4 * ((size_t)g->n + 1), hipMemcpyDeviceToHost));
    if (col_idx && g->nnz > 0) GDE_HIP(hipMemcpy(col_idx, g->col_idx, 4 * (size_t)g->nnz, hipMemcpyDeviceToHost));
    return GDE_OK;
}

int gde_graph_lambda_max(gde_ctx *ctx, gde_graph *g, int max_iters, double rtol, double *lower, double *upper,
                         hipStream_t s) {
    if (!ctx || !g || !lower || !upper) return fail(GDE_ERR_INVALID_ARG, "null argument");
    if (max_iters < 1 || !(rtol >= 0.0)) return fail(GDE_ERR_INVALID_ARG, "max_iters >= 1 and rtol >= 0");
    GDE_HIP(hipSetDevice(ctx->device));
    const int64_t n = g->n;
    double *buf = nullptr;
    GDE_HIP(hipMalloc((void **)&buf, 8 * (2 * (size_t)n + 4)));
    double *v = buf, *y = buf + n, *red = buf + 2 * n;
    double hred[4];
    double lo = 0.0, hi = 0.0;
    launch_fill_f64(v, n, 1.0, s);
    hipError_t e = hipSuccess;
    for (int it = 0; it < max_iters; it++) {
        e = hipMemsetAsync(red, 0, 32, s);
        if (e != hipSuccess) break;
        launch_lam_step(g->row_ptr, g->col_idx, v, y, g->n, red, s);
        launch_lam_scale(y, v, g->n, red, s);
        e = hipMemcpyAsync(hred, red, 32, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) break;
        double cw;
        std::memcpy(&cw, &hred[3], 8);
        lo = hred[0] / hred[1];
        hi = cw;
        if (hi - lo <= rtol * hi) break;
    }
    (void)hipFree(buf);
    if (e != hipSuccess) return hip_fail(e, "lambda_max");
    *lower = lo;
    *upper = hi;
    return GDE_OK;
}

int gde_solve(gde_ctx *ctx, const gde_graph *g, const gde_params *p, const gde_seed *s, gde_result *res,
              hipStream_t stream) {
    if (!ctx || !g || !res) return fail(GDE_ERR_INVALID_ARG, "null ctx, graph or result");
    int rc = validate_params(p);
    if (rc) { res->status = rc; return rc; }
    GraphHost *gh = graph_host(g);
    if (!gh) return fail(GDE_ERR_INVALID_ARG, "unknown graph handle");
    if ((rc = validate_seed_deg(s, g->n, gh->deg))) { res->status = rc; return rc; }
    if (res->capacity < 0) return fail(GDE_ERR_INVALID_ARG, "negative capacity");
    if (g->device != ctx->device) return fail(GDE_ERR_INVALID_ARG, "graph and context on different devices");
    GDE_HIP(hipSetDevice(ctx->device));
    if (p->method == GDE_LOCAL_SOR) return solve_fifo(ctx, g, 1, p, s, res, stream);
    if (p->value_type == GDE_F64) return solve_plain<double>(ctx, g, p, s, res, stream);
    return solve_plain<float>(ctx, g, p, s, res, stream);
}

int gde_solve_global(gde_ctx *ctx, const gde_graph *g, const gde_params *p, const gde_seed *s, gde_result *res,
                     hipStream_t stream) {
    if (!ctx || !g || !res) return fail(GDE_ERR_INVALID_ARG, "null ctx, graph or result");
    int rc = validate_params(p);
    if (rc) { res->status = rc; return rc; }
    if (p->kind == GDE_HK || p->kind == GDE_SERIES || p->method == GDE_LOCAL_SOR || (p->flags & GDE_SYM_NORM)) {
        res->status = GDE_ERR_UNSUPPORTED;
        return fail(GDE_ERR_UNSUPPORTED, "the global solvers are GD and Chebyshev for PPR and Katz (M = A D^-1)");
    }
    GraphHost *gh = graph_host(g);
    if (!gh) return fail(GDE_ERR_INVALID_ARG, "unknown graph handle");
    if ((rc = validate_seed_deg(s, g->n, gh->deg))) { res->status = rc; return rc; }
    if (res->capacity < 0) return fail(GDE_ERR_INVALID_ARG, "negative capacity");
    if (g->device != ctx->device) return fail(GDE_ERR_INVALID_ARG, "graph and context on different devices");
    GDE_HIP(hipSetDevice(ctx->device));
    return solve_global(ctx, g, p, s, res, stream);
}

}  // extern "C"
