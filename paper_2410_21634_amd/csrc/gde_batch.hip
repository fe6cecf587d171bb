// gde_batch.hip -- host side of gde_solve_batch: many LocalGD queries (PPR or
// Katz), or many level-push queries (heat kernel, series), solved together by
// the node-major lane kernels of gde_batch_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "gde_batch.h"
#include "gde_batch_kernels.h"
#include "gde_global.h"
#include "gde_internal.h"
#include "gde_kernels.h"

namespace gde {

// One reusable allocation per (graph, value type, lane count).  At rest every
// node-indexed array is zero; a batch leaves it zero again.
struct BatchWS {
    uint64_t guid = 0;
    uint32_t epoch = 0;  // touched-pair tag of the current solve (TM == epoch); 0 = never
    int vtype = 0, L = 0, Gcap = 0;
    int64_t n = 0, nwords = 0;
    size_t vs = 4;
    void *R = nullptr, *R2 = nullptr, *X = nullptr, *deg = nullptr, *col_deg = nullptr, *D = nullptr, *lane_eps = nullptr, *wl_sv = nullptr, *out_val = nullptr;
    uint32_t *NM = nullptr, *TM = nullptr, *PB = nullptr, *group_unconv = nullptr, *PM = nullptr;
    uint64_t *act[2] = {nullptr, nullptr}, *touched = nullptr, *touched2 = nullptr;
    int32_t *tdeg = nullptr, *tdeg2 = nullptr;  // batched solves: degrees beside the touched entries
    int32_t act_cap = 0, touch_cap = 0, wl_cap = 0;
    int64_t tile_cap = 0;
    int32_t *wl_node = nullptr, *wl_group = nullptr, *wl_beg = nullptr, *wl_c = nullptr, *tile_start = nullptr;
    long long *wl_off = nullptr;
    uint8_t *wl_lanes = nullptr;
    long long *lane_ops = nullptr, *lane_nnz = nullptr, *lane_out_off = nullptr;
    int32_t *lane_T = nullptr, *cnt = nullptr, *sub_flag = nullptr;
    double *lane_l1 = nullptr;
    unsigned long long *lane_dinf = nullptr;
    BatchDev *st = nullptr;
    int32_t *s_lane = nullptr, *s_node = nullptr;
    double *s_val = nullptr;
    int32_t s_cap = 0;
    int32_t *out_idx = nullptr;
    int64_t out_cap = 0;
    int nblk = 0;
    void **lane_dst = nullptr;  // [2 * Gcap * L]: per-lane output pointers (idx, then val) for device results
                                // (warm starts: the queries' rd, then x)
    void **warm_ptr = nullptr;  // [2 * Gcap * L]: warm starts: the queries' pushed, then touched bitmaps
    uint32_t *row_stamp = nullptr;  // [n], measurement only: distinct rows per round
    const int32_t *col_deg_of = nullptr;  // the col_idx that col_deg was built from
    int64_t col_deg_nnz = 0;
    uint32_t round = 0;
};

void batch_ws_free(BatchWS *w) {
    void *p[] = {w->R, w->R2, w->X, w->deg, w->col_deg, w->D, w->PM, w->lane_eps, w->wl_sv, w->out_val, w->NM, w->TM, w->PB, w->group_unconv,
                 w->act[0], w->act[1], w->touched, w->touched2, w->tdeg, w->tdeg2, w->wl_node, w->wl_group, w->wl_beg, w->wl_c, w->tile_start,
                 w->wl_off, w->wl_lanes, w->lane_ops, w->lane_nnz, w->lane_out_off, w->lane_T,
                 w->cnt, w->sub_flag, w->lane_l1, w->lane_dinf, w->st, w->s_lane, w->s_node, w->s_val, w->out_idx,
                 w->lane_dst, w->warm_ptr, w->row_stamp};
    for (void *q : p)
        if (q) (void)hipFree(q);
    delete w;
}

void drop_batch_workspaces_of(const gde_graph *g, gde_ctx *ctx) {
    for (size_t i = 0; i < ctx->bws.size();) {
        if (ctx->bws[i]->guid == g->uid) { batch_ws_free(ctx->bws[i]); ctx->bws.erase(ctx->bws.begin() + i); }
        else i++;
    }
}

int batch_workspaces_refresh(const gde_graph *g, gde_ctx *ctx, hipStream_t s) {
    for (BatchWS *b : ctx->bws) {
        if (b->guid != g->uid) continue;
        const hipError_t e = b->vtype == GDE_F64 ? batch_init_deg<double>(g->row_ptr, (double *)b->deg, g->n, s)
                                                 : batch_init_deg<float>(g->row_ptr, (float *)b->deg, g->n, s);
        if (e != hipSuccess) return hip_fail(e, "batch_init_deg");
        b->col_deg_of = nullptr;  // rebuilt from the new column array on the next solve
    }
    return GDE_OK;
}

struct DevBuf {  // device scratch released on every return path
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

struct Schedule {
    int lanes = 16;
    int blocks_per_cu = 0;  // 0: the occupancy limit
    int sort = 1;           // order queries by eps, then seed degree, before packing lanes
    int autotune = 0;       // choose lanes and blocks_per_cu by timing candidates (cached per context)
};

static int json_int(const char *js, const char *key, int dflt) {
    if (!js) return dflt;
    std::string k = std::string("\"") + key + "\"";
    const char *p = std::strstr(js, k.c_str());
    if (!p) return dflt;
    p = std::strchr(p + k.size(), ':');
    if (!p) return dflt;
    return (int)std::strtol(p + 1, nullptr, 10);
}

static int parse_schedule(const char *js, Schedule *sc) {
    sc->lanes = json_int(js, "lanes", 16);
    sc->blocks_per_cu = json_int(js, "blocks_per_cu", 0);
    sc->sort = json_int(js, "sort", 1);
    sc->autotune = json_int(js, "auto", 0);
    if (sc->lanes != 8 && sc->lanes != 16 && sc->lanes != 32)
        return fail(GDE_ERR_INVALID_ARG, "schedule.lanes must be 8, 16 or 32");
    if (sc->blocks_per_cu < 0 || sc->blocks_per_cu > 64) return fail(GDE_ERR_INVALID_ARG, "bad schedule.blocks_per_cu");
    // every iteration runs as one snapshot and one push launch; a single
    // cooperative launch for all iterations is not provided
    if (json_int(js, "persistent", 0)) return fail(GDE_ERR_UNSUPPORTED, "schedule.persistent is not provided");
    return GDE_OK;
}

#define BALLOC(ptr, bytes)                                                           \
    do {                                                                             \
        hipError_t _e = hipMalloc((void **)&(ptr), (size_t)(bytes));                 \
        if (_e != hipSuccess) { batch_ws_free(w); return hip_fail(_e, "hipMalloc(batch)"); } \
        _e = hipMemsetAsync((ptr), 0, (size_t)(bytes), s);                           \
        if (_e != hipSuccess) { batch_ws_free(w); return hip_fail(_e, "hipMemsetAsync(batch)"); } \
    } while (0)

static int batch_ws_get(gde_ctx *ctx, const gde_graph *g, int vtype, int L, int G, hipStream_t s, BatchWS **out) {
    for (size_t i = 0; i < ctx->bws.size(); i++) {
        BatchWS *b = ctx->bws[i];
        if (b->guid == g->uid && b->vtype == vtype && b->L == L && b->Gcap >= G) { *out = b; return GDE_OK; }
    }
    // one batch workspace per context: release the others first (they can be large)
    for (BatchWS *b : ctx->bws) batch_ws_free(b);
    ctx->bws.clear();
    BatchWS *w = new BatchWS();
    w->guid = g->uid;
    w->vtype = vtype;
    w->L = L;
    w->Gcap = G;
    w->n = g->n;
    w->nwords = (g->n + 31) / 32;
    w->vs = vtype == GDE_F64 ? 8 : 4;
    const int64_t n = g->n, GL = (int64_t)G * L;
    const int64_t pairs = n * (int64_t)G;
    // list capacities in (group, node) pairs; a batch whose lists outgrow them is
    // split in two by gde_solve_batch
    w->act_cap = (int32_t)std::min<int64_t>(pairs, 32000000);
    // work-list entries are counted in the top 24 bits of the packed reservation
    w->wl_cap = std::min<int32_t>(w->act_cap, (1 << 24) - 1);
    // touched entries: (lane, node) for batched solves, (group, node) for serving
    w->touch_cap = (int32_t)std::min<int64_t>(pairs * L, 320000000);
    w->tile_cap = 32000000;
    w->nblk = (int)((w->nwords + kBlock - 1) / kBlock);
    BALLOC(w->R, (size_t)n * GL * w->vs);
    BALLOC(w->X, (size_t)n * GL * w->vs);
    BALLOC(w->NM, (size_t)n * G * 4);
    BALLOC(w->TM, (size_t)n * G * 4);
    BALLOC(w->PB, (size_t)G * w->nwords * 4);
    BALLOC(w->deg, (size_t)n * w->vs);
    BALLOC(w->lane_eps, (size_t)GL * w->vs);
    BALLOC(w->act[0], (size_t)w->act_cap * 8);
    BALLOC(w->act[1], (size_t)w->act_cap * 8);
    BALLOC(w->touched, (size_t)w->touch_cap * 8);
    BALLOC(w->wl_node, (size_t)w->wl_cap * 4);
    BALLOC(w->wl_group, (size_t)w->wl_cap * 4);
    BALLOC(w->wl_beg, (size_t)w->wl_cap * 4);
    BALLOC(w->wl_c, (size_t)w->wl_cap * 4);
    BALLOC(w->wl_off, (size_t)w->wl_cap * 8);
    BALLOC(w->wl_lanes, (size_t)w->wl_cap * L);
    BALLOC(w->wl_sv, (size_t)w->wl_cap * L * w->vs);
    BALLOC(w->tile_start, (size_t)w->tile_cap * 4);
    BALLOC(w->lane_ops, (size_t)GL * kStatShards * 8);
    BALLOC(w->lane_l1, (size_t)GL * kStatShards * 8);
    BALLOC(w->lane_T, (size_t)GL * 4);
    BALLOC(w->lane_dinf, (size_t)GL * 8);
    BALLOC(w->lane_nnz, (size_t)GL * 8);
    BALLOC(w->lane_out_off, (size_t)GL * 8);
    BALLOC(w->sub_flag, (size_t)GL * 4);
    BALLOC(w->group_unconv, (size_t)G * 4);
    BALLOC(w->cnt, (size_t)GL * w->nblk * 4);
    BALLOC(w->st, sizeof(BatchDev));
    BALLOC(w->lane_dst, 2 * (size_t)GL * sizeof(void *));
    BALLOC(w->warm_ptr, 2 * (size_t)GL * sizeof(void *));
    hipError_t e = vtype == GDE_F64 ? batch_init_deg<double>(g->row_ptr, (double *)w->deg, g->n, s)
                                    : batch_init_deg<float>(g->row_ptr, (float *)w->deg, g->n, s);
    if (e != hipSuccess) { batch_ws_free(w); return hip_fail(e, "batch_init_deg"); }
    ctx->bws.push_back(w);
    *out = w;
    return GDE_OK;
}

// ---- access for the server (gde_server.hip)
int batch_ws_acquire(gde_ctx *ctx, const gde_graph *g, int vtype, int L, int G, hipStream_t s, BatchWS **out) {
    return batch_ws_get(ctx, g, vtype, L, G, s, out);
}

void batch_args_from_ws(BatchWS *w, const gde_graph *g, int G, BatchArgs<float> *a) {
    *a = BatchArgs<float>{};
    a->n = g->n;
    a->nnz = (int32_t)g->nnz;
    a->G = G;
    a->nwords = w->nwords;
    a->row_ptr = g->row_ptr;
    a->col_idx = g->col_idx;
    a->deg = (const float *)w->deg;
    a->R = (float *)w->R;
    a->X = (float *)w->X;
    a->NM = w->NM;
    a->TM = w->TM;
    a->PB = w->PB;
    a->act[0] = w->act[0];
    a->act[1] = w->act[1];
    a->act_cap = w->act_cap;
    a->touched = w->touched;
    a->touch_cap = w->touch_cap;
    a->wl_node = w->wl_node;
    a->wl_group = w->wl_group;
    a->wl_beg = w->wl_beg;
    a->wl_c = w->wl_c;
    a->wl_off = w->wl_off;
    a->wl_lanes = w->wl_lanes;
    a->wl_sv = (float *)w->wl_sv;
    a->wl_cap = w->wl_cap;
    a->tile_start = w->tile_start;
    a->tile_cap = w->tile_cap;
    a->lane_eps = (const float *)w->lane_eps;
    a->lane_ops = w->lane_ops;
    a->lane_T = w->lane_T;
    a->lane_l1 = w->lane_l1;
    a->lane_dinf = w->lane_dinf;
    a->group_unconv = w->group_unconv;
    a->st = w->st;
}

int32_t *batch_ws_touch_count(BatchWS *w) { return &w->st->tcount; }

void batch_ws_extract_buffers(BatchWS *w, int32_t **cnt, long long **lane_nnz, long long **lane_off) {
    *cnt = w->cnt;
    *lane_nnz = w->lane_nnz;
    *lane_off = w->lane_out_off;
}

// exchange one of the two active lists (or the touched list, which = 2) with a
// buffer of the same capacity: compaction writes into the spare and swaps it in
void batch_ws_swap_list(BatchWS *w, int which, uint64_t **spare) {
    uint64_t **slot = which == 2 ? &w->touched : &w->act[which];
    std::swap(*slot, *spare);
}

// Standing queries' state for a warm start (per query, device pointers): the
// residual-and-degree array, x, the pushed and touched bitmaps.
struct WarmState {
    void *const *rd;
    void *const *x;
    uint32_t *const *pushed;
    uint32_t *const *tbm;
};

template <typename V>
static int solve_batch_fused(gde_ctx *ctx, const gde_graph *g, int32_t B, const gde_params *p, const gde_seed *sd,
                             gde_result *res, const Schedule &sc, hipStream_t s, const WarmState *warm = nullptr) {
    const int L = sc.lanes;
    const int G = (B + L - 1) / L;
    const int vt = p[0].value_type;
    BatchWS *w = nullptr;
    int rc = batch_ws_get(ctx, g, vt, L, G, s, &w);
    if (rc) return rc;
    const bool ppr = p[0].kind == GDE_PPR;
    // level push (heat kernel, series): every lane runs the same levels, one per
    // iteration, on two residual planes (levels t and t + 1)
    const bool lvl = p[0].kind == GDE_HK || p[0].kind == GDE_SERIES;
    const int K = p[0].K;
    LevelSeries ls;
    if (lvl) {
        ls = level_series(&p[0]);
        if (!w->R2) {
            const size_t bytes = (size_t)g->n * (size_t)w->Gcap * L * w->vs;
            if (hipMalloc(&w->R2, bytes) != hipSuccess) {
                w->R2 = nullptr;
                (void)hipGetLastError();
                return fail(GDE_ERR_OOM, "no device memory for the second residual plane of the level push");
            }
            GDE_HIP(hipMemsetAsync(w->R2, 0, bytes, s));
        }
        if (!w->touched2) {
            if (hipMalloc((void **)&w->touched2, (size_t)w->touch_cap * 8) != hipSuccess ||
                hipMalloc((void **)&w->tdeg2, (size_t)w->touch_cap * 4) != hipSuccess) {
                (void)hipGetLastError();
                if (w->touched2) (void)hipFree(w->touched2);
                w->touched2 = nullptr;
                w->tdeg2 = nullptr;
                return fail(GDE_ERR_OOM, "no device memory for the odd levels' touched list");
            }
        }
    }

    // the destinations' degrees as a stream beside col_idx (batched solves only;
    // rebuilt if the graph's column array changed)
    if (!w->col_deg || w->col_deg_of != g->col_idx || w->col_deg_nnz != g->nnz) {
        if (w->col_deg && w->col_deg_nnz != g->nnz) {
            (void)hipFree(w->col_deg);
            w->col_deg = nullptr;
        }
        if (!w->col_deg && hipMalloc(&w->col_deg, (size_t)std::max<int64_t>(g->nnz, 1) * w->vs) != hipSuccess) {
            w->col_deg = nullptr;
            (void)hipGetLastError();
            return fail(GDE_ERR_OOM, "no device memory for the batch's column degrees");
        }
        GDE_HIP(batch_init_col_deg<V>(g->col_idx, (const V *)w->deg, (V *)w->col_deg, g->nnz, s));
        w->col_deg_of = g->col_idx;
        w->col_deg_nnz = g->nnz;
    }

    // LocalCH: the Delta plane and the previous-active masks, zero at rest
    const bool ch = p[0].method == GDE_LOCAL_CH;
    if (ch && !w->D) {
        const size_t dbytes = (size_t)g->n * (size_t)w->Gcap * L * w->vs, mbytes = (size_t)g->n * (size_t)w->Gcap * 4;
        if (hipMalloc(&w->D, dbytes) != hipSuccess || hipMalloc((void **)&w->PM, mbytes) != hipSuccess) {
            (void)hipGetLastError();
            if (w->D) (void)hipFree(w->D);
            w->D = nullptr;
            w->PM = nullptr;
            return fail(GDE_ERR_OOM, "no device memory for the LocalCH planes of the batch");
        }
        GDE_HIP(hipMemsetAsync(w->D, 0, dbytes, s));
        GDE_HIP(hipMemsetAsync(w->PM, 0, mbytes, s));
    }
    if (!w->tdeg && hipMalloc((void **)&w->tdeg, (size_t)w->touch_cap * 4) != hipSuccess) {
        w->tdeg = nullptr;
        (void)hipGetLastError();
        return fail(GDE_ERR_OOM, "no device memory for the touched entries' degrees");
    }

    // lane assignment: query order[j] occupies lane j (group j / L)
    std::vector<int32_t> order(B);
    std::iota(order.begin(), order.end(), 0);
    if (sc.sort) std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return p[a].eps < p[b].eps; });
    int64_t ns = 0;
    for (int32_t q = 0; q < B; q++) ns += sd[q].nnz;
    if (ns > w->s_cap) {
        if (w->s_lane) { (void)hipFree(w->s_lane); (void)hipFree(w->s_node); (void)hipFree(w->s_val); }
        w->s_lane = w->s_node = nullptr;
        w->s_val = nullptr;
        GDE_HIP(hipMalloc((void **)&w->s_lane, 4 * ns));
        GDE_HIP(hipMalloc((void **)&w->s_node, 4 * ns));
        GDE_HIP(hipMalloc((void **)&w->s_val, 8 * ns));
        w->s_cap = (int32_t)ns;
    }
    std::vector<int32_t> h_lane(ns), h_node(ns), h_flag((size_t)G * L, 0);
    std::vector<double> h_val(ns);
    std::vector<V> h_eps((size_t)G * L, (V)(sizeof(V) == 4 ? FLT_MAX : DBL_MAX));
    int64_t k = 0;
    for (int j = 0; j < B; j++) {
        const int q = order[j];
        for (int32_t i = 0; i < sd[q].nnz; i++, k++) {
            h_lane[k] = j;
            h_node[k] = sd[q].idx[i];
            h_val[k] = sd[q].val[i];
        }
        h_eps[j] = (V)(ppr ? p[q].alpha * p[q].eps : p[q].eps);  // level push: eps itself
        h_flag[j] = (!ppr && (p[q].flags & GDE_KATZ_SUBTRACT_SEED)) ? 1 : 0;
    }
    if (ns > 0) {
        GDE_HIP(hipMemcpyAsync(w->s_lane, h_lane.data(), 4 * ns, hipMemcpyHostToDevice, s));
        GDE_HIP(hipMemcpyAsync(w->s_node, h_node.data(), 4 * ns, hipMemcpyHostToDevice, s));
        GDE_HIP(hipMemcpyAsync(w->s_val, h_val.data(), 8 * ns, hipMemcpyHostToDevice, s));
    }
    // warm start: the queries' state pointers in lane order (rd, x, pushed, tbm)
    if (warm) {
        const size_t GLw = (size_t)G * L;
        std::vector<void *> qp(4 * GLw, nullptr);
        for (int j = 0; j < B; j++) {
            const int q = order[j];
            qp[j] = warm->rd[q];
            qp[GLw + j] = warm->x[q];
            qp[2 * GLw + j] = warm->pushed[q];
            qp[3 * GLw + j] = warm->tbm[q];
        }
        GDE_HIP(hipMemcpyAsync(w->lane_dst, qp.data(), sizeof(void *) * 2 * GLw, hipMemcpyHostToDevice, s));
        GDE_HIP(hipMemcpyAsync(w->warm_ptr, qp.data() + 2 * GLw, sizeof(void *) * 2 * GLw, hipMemcpyHostToDevice, s));
    }
    GDE_HIP(hipMemcpyAsync(w->lane_eps, h_eps.data(), sizeof(V) * h_eps.size(), hipMemcpyHostToDevice, s));
    GDE_HIP(hipMemcpyAsync(w->sub_flag, h_flag.data(), 4 * h_flag.size(), hipMemcpyHostToDevice, s));
    const size_t GL = (size_t)G * L;
    GDE_HIP(hipMemsetAsync(w->st, 0, sizeof(BatchDev), s));
    GDE_HIP(hipMemsetAsync(w->lane_ops, 0, GL * kStatShards * 8, s));
    GDE_HIP(hipMemsetAsync(w->lane_l1, 0, GL * kStatShards * 8, s));
    GDE_HIP(hipMemsetAsync(w->lane_T, 0, GL * 4, s));
    GDE_HIP(hipMemsetAsync(w->lane_dinf, 0, GL * 8, s));
    GDE_HIP(hipMemsetAsync(w->group_unconv, 0, (size_t)G * 4, s));

    BatchArgs<V> a{};
    a.n = g->n;
    a.nnz = (int32_t)g->nnz;
    a.G = G;
    a.nwords = w->nwords;
    a.row_ptr = g->row_ptr;
    a.col_idx = g->col_idx;
    a.deg = (const V *)w->deg;
    a.col_deg = (const V *)w->col_deg;
    a.R = (V *)w->R;
    a.X = (V *)w->X;
    a.NM = w->NM;
    a.TM = w->TM;
    // a new tag per solve marks the touched pairs, so the residual pass needs no
    // clearing writes; on wrap-around the flags are reset once
    if (++w->epoch == 0u) {
        GDE_HIP(hipMemsetAsync(w->TM, 0, (size_t)g->n * G * 4, s));
        w->epoch = 1u;
    }
    a.epoch = w->epoch;
    a.g_epoch = nullptr;
    a.PB = w->PB;
    a.act[0] = w->act[0];
    a.act[1] = w->act[1];
    a.act_cap = w->act_cap;
    a.touched = w->touched;
    a.touched2 = w->touched2;
    a.tdeg = w->tdeg;
    a.tdeg2 = w->tdeg2;
    a.touch_cap = w->touch_cap;
    a.wl_node = w->wl_node;
    a.wl_group = w->wl_group;
    a.wl_beg = w->wl_beg;
    a.wl_c = w->wl_c;
    a.wl_off = w->wl_off;
    a.wl_lanes = w->wl_lanes;
    a.wl_sv = (V *)w->wl_sv;
    a.wl_cap = w->wl_cap;
    a.tile_start = w->tile_start;
    a.tile_cap = w->tile_cap;
    a.lane_eps = (const V *)w->lane_eps;
    a.wscale = (V)(ppr ? 1.0 - p[0].alpha : p[0].beta);  // level push: set per level below
    a.w_div_deg = (ppr || lvl) ? 1 : 0;
    a.R2 = lvl ? (V *)w->R2 : nullptr;
    a.th_div = 0.0;
    a.no_push = 0;
    a.sym = (p[0].flags & GDE_SYM_NORM) ? 1 : 0;
    a.ch = ch ? 1 : 0;
    a.force = 0;
    a.probe = 0;
    a.sgn = warm ? 1 : 0;  // warm start: signed residuals, no forced S_0
    a.D = ch ? (V *)w->D : nullptr;
    a.PM = ch ? w->PM : nullptr;
    // LocalCH scalars (the plain solver's recurrence): t = 0 is the forced first
    // step h = r; then delta_{t+1} = 1 / (2 sigma - delta_t), c_t = 2 sigma delta_{t+1},
    // m_t = delta_t delta_{t+1}, with sigma = (L + mu) / (L - mu) from the kind's bounds
    double ch_sigma = 1.0, ch_dlt = 1.0;
    if (ch) {
        double mu, Lb;
        if (ppr) { mu = p[0].alpha; Lb = 2.0 - p[0].alpha; }
        else { mu = 1.0 - p[0].beta * p[0].lambda_bound; Lb = 1.0 + p[0].beta * p[0].lambda_bound; }
        ch_sigma = (Lb + mu) / (Lb - mu);
        ch_dlt = 1.0 / ch_sigma;
    }
    a.lane_ops = w->lane_ops;
    a.lane_T = w->lane_T;
    a.lane_l1 = w->lane_l1;
    a.lane_dinf = w->lane_dinf;
    a.group_unconv = w->group_unconv;
    a.tr_size = a.tr_vol = nullptr;
    a.tr_cap = 0;
    a.tr_nodes = nullptr;
    a.tr_noff = a.tr_ncap = nullptr;
    a.tr_ncount = nullptr;
    // optional trace (GDE_TRACE): per-lane |S_t|, vol(S_t) and the S_t lists
    bool trace = false;
    int32_t tr_cap = 0;
    std::vector<long long> h_noff(GL, 0), h_ncap(GL, 0);
    long long ntot = 0;
    for (int j = 0; j < B; j++) {
        const int q = order[j];
        if (!(p[q].flags & GDE_TRACE)) continue;
        trace = true;
        tr_cap = std::max<int32_t>(tr_cap, (int32_t)std::min<int64_t>(res[q].trace_capacity, 1 << 20));
        if (res[q].trace_nodes && res[q].trace_nodes_capacity > 0) {
            h_noff[j] = ntot;
            h_ncap[j] = res[q].trace_nodes_capacity;
            ntot += res[q].trace_nodes_capacity;
        }
    }
    DevBuf trbuf;
    if (trace) {
        tr_cap = std::max(tr_cap, 1);
        const size_t need = GL * (size_t)tr_cap * 16 + GL * 24 + (size_t)std::max<long long>(ntot, 1) * 4;
        GDE_HIP(hipMalloc(&trbuf.p, need));
        GDE_HIP(hipMemsetAsync(trbuf.p, 0, need, s));
        char *b = (char *)trbuf.p;
        a.tr_size = (long long *)b;
        a.tr_vol = a.tr_size + GL * tr_cap;
        a.tr_cap = tr_cap;
        long long *noff = a.tr_vol + GL * tr_cap;
        long long *ncap = noff + GL;
        a.tr_ncount = (unsigned long long *)(ncap + GL);
        a.tr_nodes = (int32_t *)(a.tr_ncount + GL);
        a.tr_noff = noff;
        a.tr_ncap = ncap;
        GDE_HIP(hipMemcpyAsync(noff, h_noff.data(), 8 * GL, hipMemcpyHostToDevice, s));
        GDE_HIP(hipMemcpyAsync(ncap, h_ncap.data(), 8 * GL, hipMemcpyHostToDevice, s));
    }
    a.st = w->st;
    a.max_iters = lvl ? K + 1 : p[0].max_iters;
    a.row_stamp = nullptr;
    if (ctx->prof_on) {  // measurement: count the distinct rows each round reads
        if (!w->row_stamp) {
            GDE_HIP(hipMalloc((void **)&w->row_stamp, 4 * (size_t)g->n));
            GDE_HIP(hipMemsetAsync(w->row_stamp, 0, 4 * (size_t)g->n, s));
            w->round = 0;
        }
        a.row_stamp = w->row_stamp;
    }

    if (warm)
        GDE_HIP(batch_warm_load<V>(L, a, (const void *const *)w->lane_dst,
                                   (const uint32_t *const *)(w->warm_ptr + GL), B, s));
    else
        GDE_HIP(batch_seed<V>(L, a, w->s_lane, w->s_node, w->s_val, (int32_t)ns,
                              lvl ? ls.c0 : ppr ? p[0].alpha : 1.0, s));
    int dev = 0;
    GDE_HIP(hipGetDevice(&dev));
    int cus = 0;
    GDE_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    int occ = 0;
    GDE_HIP(batch_occupancy<V>(L, &occ));
    int bpc = sc.blocks_per_cu > 0 ? std::min(sc.blocks_per_cu, occ) : occ;
    if (bpc < 1) return fail(GDE_ERR_DEVICE, "batched kernel does not fit on a compute unit");
    const int grid = bpc * cus;
    BatchDev hst{};
    if ((rc = prof_mark_batch(ctx, s))) return rc;
    int t = 0, chunk = 8;
    bool done = false;
    while (t < a.max_iters && !done) {
        int end = std::min(a.max_iters, t + chunk);
        for (; t < end; t++) {
            if (a.row_stamp && ++w->round == 0u) {  // tags wrapped: start the stamps afresh
                GDE_HIP(hipMemsetAsync(w->row_stamp, 0, 4 * (size_t)g->n, s));
                w->round = 1u;
            }
            a.round_tag = w->round;
            if (lvl) {  // level t: weight c_{t+1}/c_t, thresholds of level t + 1
                a.no_push = t >= K;
                a.wscale = (V)(t < K ? ls.ratio[t] : 0.0);
                a.th_div = t < K ? (double)(K + 1) * ls.psi[t + 1] : 1.0;
            }
            if (ch) {
                a.force = t == 0;
                if (t == 0) {
                    a.c_t = (V)1;
                    a.m_t = (V)0;
                } else {
                    const double dnext = 1.0 / (2.0 * ch_sigma - ch_dlt);
                    a.c_t = (V)(2.0 * ch_sigma * dnext);
                    a.m_t = (V)(ch_dlt * dnext);
                    ch_dlt = dnext;
                }
            }
            GDE_HIP(batch_launch<V>(1, L, a, grid, t, s));
            if ((rc = prof_mark_batch_push(ctx, s))) return rc;
            GDE_HIP(batch_launch<V>(2, L, a, grid, t, s));
            if ((rc = prof_mark_batch_push(ctx, s))) return rc;
            // what level t kept (below its thresholds) leaves the plane, weighted psi_t
            if (lvl) GDE_HIP(batch_harvest<V>(L, a, grid, t, ls.psi[t], (double)(K + 1) * ls.psi[t], s));
        }
        GDE_HIP(hipMemcpyAsync(&hst, w->st, sizeof(BatchDev), hipMemcpyDeviceToHost, s));
        GDE_HIP(hipStreamSynchronize(s));
        done = hst.acount[t & 1] == 0 || hst.ovf[0] || hst.ovf[1];
        chunk = std::min(chunk * 2, 32);
    }
    if (lvl && t <= K && !hst.ovf[0] && !hst.ovf[1]) {
        // no lane has an active node at level t, but push(t - 1) may have left
        // residual there
        GDE_HIP(batch_harvest<V>(L, a, grid, t, ls.psi[t], (double)(K + 1) * ls.psi[t], s));
    }
    if ((ch || warm) && t >= a.max_iters && hst.acount[t & 1] > 0 && !hst.ovf[0] && !hst.ovf[1]) {
        // LocalCH at the iteration cap: the list holds candidates; a snapshot that
        // changes nothing marks the lanes still active and clears the masks
        a.probe = 1;
        GDE_HIP(batch_launch<V>(1, L, a, grid, t, s));
        a.probe = 0;
    }
    if ((rc = prof_mark_batch(ctx, s))) return rc;
    const int final_parity = (ch || warm) ? -1 : (t & 1);
    if (hst.ovf[0] || hst.ovf[1]) {
        // the kernels stopped on a capacity limit: restore the rest state by brute force
        GDE_HIP(hipMemsetAsync(w->R, 0, (size_t)g->n * GL * w->vs, s));
        if (w->R2) GDE_HIP(hipMemsetAsync(w->R2, 0, (size_t)g->n * GL * w->vs, s));
        GDE_HIP(hipMemsetAsync(w->X, 0, (size_t)g->n * GL * w->vs, s));
        GDE_HIP(hipMemsetAsync(w->NM, 0, (size_t)g->n * G * 4, s));
        GDE_HIP(hipMemsetAsync(w->TM, 0, (size_t)g->n * G * 4, s));
        GDE_HIP(hipMemsetAsync(w->PB, 0, (size_t)G * w->nwords * 4, s));
        if (w->D) GDE_HIP(hipMemsetAsync(w->D, 0, (size_t)g->n * GL * w->vs, s));
        if (w->PM) GDE_HIP(hipMemsetAsync(w->PM, 0, (size_t)g->n * G * 4, s));
        GDE_HIP(hipStreamSynchronize(s));
        return fail(GDE_ERR_OOM, "batched work lists exceeded their capacity; split the batch");
    }
    // residual norms, unconverged lanes, Katz seed subtraction
    // warm start: the residuals go back to the queries before the pass clears them
    if (warm)
        GDE_HIP(batch_warm_store<V>(L, a, 0, w->lane_dst, (uint32_t *const *)(w->warm_ptr + GL), nullptr, nullptr, B,
                                    grid, s));
    // (the level push took its norms level by level and never hits a cap)
    const bool any_sub = std::any_of(h_flag.begin(), h_flag.end(), [](int32_t f) { return f != 0; });
    if (!lvl)
        GDE_HIP(batch_finish<V>(L, a, grid, ppr ? 1.0 / p[0].alpha : 1.0, final_parity, w->s_lane, w->s_node,
                                w->s_val, (int32_t)ns, any_sub ? w->sub_flag : nullptr, s));
    // extraction: counts per lane, then the sorted sparse outputs (warm start:
    // the lanes' x increments go into the queries' x instead)
    std::vector<long long> nnz(GL, 0), off(GL, 0);
    if (warm) {
        GDE_HIP(batch_warm_store<V>(L, a, 1, nullptr, nullptr, w->lane_dst + GL, (uint32_t *const *)w->warm_ptr, B,
                                    grid, s));
    } else {
        GDE_HIP(batch_extract<V>(L, a, 0, w->cnt, w->nblk, w->lane_nnz, nullptr, nullptr, nullptr, 0, s));
        std::fill(off.begin(), off.end(), -1);
        GDE_HIP(hipMemcpyAsync(nnz.data(), w->lane_nnz, 8 * GL, hipMemcpyDeviceToHost, s));
        GDE_HIP(hipStreamSynchronize(s));
        long long total = 0;
        for (int j = 0; j < B; j++) {
            const int q = order[j];
            if (nnz[j] <= res[q].capacity && res[q].idx && res[q].val) {
                off[j] = total;
                total += nnz[j];
            }
        }
        const bool dev_out = (p[0].flags & GDE_RESULT_DEVICE) != 0;
        if (dev_out) {
            // every lane's entries go straight to its query's device buffers
            std::vector<void *> dst(2 * (size_t)GL, nullptr);
            for (int j = 0; j < B; j++) {
                if (off[j] < 0) continue;
                dst[j] = res[order[j]].idx;
                dst[GL + j] = res[order[j]].val;
            }
            GDE_HIP(hipMemcpyAsync(w->lane_dst, dst.data(), sizeof(void *) * dst.size(), hipMemcpyHostToDevice, s));
            GDE_HIP(hipMemcpyAsync(w->lane_out_off, off.data(), 8 * GL, hipMemcpyHostToDevice, s));
            GDE_HIP(batch_extract<V>(L, a, 1, w->cnt, w->nblk, w->lane_nnz, w->lane_out_off, nullptr, nullptr, 1, s,
                                     nullptr, 0, (int32_t *const *)w->lane_dst, (V *const *)(w->lane_dst + GL)));
        } else {
            if (total > w->out_cap) {
                if (w->out_idx) { (void)hipFree(w->out_idx); (void)hipFree(w->out_val); }
                w->out_idx = nullptr;
                w->out_val = nullptr;
                w->out_cap = 0;
                GDE_HIP(hipMalloc((void **)&w->out_idx, 4 * (size_t)total));
                GDE_HIP(hipMalloc(&w->out_val, sizeof(V) * (size_t)total));
                w->out_cap = total;
            }
            GDE_HIP(hipMemcpyAsync(w->lane_out_off, off.data(), 8 * GL, hipMemcpyHostToDevice, s));
            GDE_HIP(batch_extract<V>(L, a, 1, w->cnt, w->nblk, w->lane_nnz, w->lane_out_off, w->out_idx,
                                     (V *)w->out_val, 1, s));
            for (int j = 0; j < B; j++) {
                const int q = order[j];
                if (off[j] < 0 || nnz[j] == 0) continue;
                GDE_HIP(hipMemcpyAsync(res[q].idx, w->out_idx + off[j], 4 * (size_t)nnz[j], hipMemcpyDeviceToHost, s));
                GDE_HIP(hipMemcpyAsync(res[q].val, (V *)w->out_val + off[j], sizeof(V) * (size_t)nnz[j],
                                       hipMemcpyDeviceToHost, s));
            }
        }
    }
    std::vector<long long> ops(GL * kStatShards);
    std::vector<double> l1(GL * kStatShards);
    std::vector<int32_t> T(GL);
    std::vector<unsigned long long> dinf(GL);
    std::vector<uint32_t> unconv(G);
    GDE_HIP(hipMemcpyAsync(ops.data(), w->lane_ops, 8 * ops.size(), hipMemcpyDeviceToHost, s));
    GDE_HIP(hipMemcpyAsync(l1.data(), w->lane_l1, 8 * l1.size(), hipMemcpyDeviceToHost, s));
    GDE_HIP(hipMemcpyAsync(T.data(), w->lane_T, 4 * T.size(), hipMemcpyDeviceToHost, s));
    GDE_HIP(hipMemcpyAsync(dinf.data(), w->lane_dinf, 8 * dinf.size(), hipMemcpyDeviceToHost, s));
    GDE_HIP(hipMemcpyAsync(unconv.data(), w->group_unconv, 4 * unconv.size(), hipMemcpyDeviceToHost, s));
    GDE_HIP(hipMemcpyAsync(&hst, w->st, sizeof(BatchDev), hipMemcpyDeviceToHost, s));
    GDE_HIP(hipStreamSynchronize(s));
    if ((rc = prof_collect_batch(ctx, hst.lane_edges, hst.entries, hst.rows, hst.row_vol))) return rc;
    std::vector<unsigned long long> ncount(trace ? GL : 0);
    if (trace) {
        GDE_HIP(hipMemcpy(ncount.data(), a.tr_ncount, 8 * GL, hipMemcpyDeviceToHost));
        for (int j = 0; j < B; j++) {
            const int q = order[j];
            if (!(p[q].flags & GDE_TRACE)) continue;
            const int64_t m = std::min<int64_t>(res[q].trace_capacity, tr_cap);
            if (m > 0 && res[q].trace_size)
                GDE_HIP(hipMemcpy(res[q].trace_size, a.tr_size + (size_t)j * tr_cap, 8 * m, hipMemcpyDeviceToHost));
            if (m > 0 && res[q].trace_vol)
                GDE_HIP(hipMemcpy(res[q].trace_vol, a.tr_vol + (size_t)j * tr_cap, 8 * m, hipMemcpyDeviceToHost));
            const int64_t mn = std::min<int64_t>((int64_t)ncount[j], h_ncap[j]);
            if (mn > 0)
                GDE_HIP(hipMemcpy(res[q].trace_nodes, a.tr_nodes + h_noff[j], 4 * mn, hipMemcpyDeviceToHost));
        }
    }
    int first = GDE_OK;
    for (int j = 0; j < B; j++) {
        const int q = order[j];
        gde_result &r = res[q];
        long long so = 0, sp = 0;
        double sl = 0.0;
        for (int sh = 0; sh < kStatShards; sh++) {
            const unsigned long long po = (unsigned long long)ops[(size_t)j * kStatShards + sh];
            so += (long long)(po & kOpsMask);
            sp += (long long)(po >> (64 - kPushBits));
            sl += l1[(size_t)j * kStatShards + sh];
        }
        r.nnz = nnz[j];
        r.iters = T[j];
        r.ops = so;
        r.pushes = sp;
        r.residual_l1 = sl;
        std::memcpy(&r.residual_dinf, &dinf[j], 8);
        r.trace_len = trace && (p[q].flags & GDE_TRACE) ? T[j] : 0;
        r.trace_nodes_len = trace && (p[q].flags & GDE_TRACE) ? (int64_t)ncount[j] : 0;
        if (off[j] < 0) r.status = GDE_ERR_CAPACITY;
        else if ((unconv[j / L] >> (j % L)) & 1u) r.status = GDE_ERR_NOT_CONVERGED;
        else r.status = GDE_OK;
        if (r.status != GDE_OK && first == GDE_OK) first = r.status;
    }
    if (first == GDE_ERR_CAPACITY) return fail(first, "a result capacity was too small (its nnz holds the size needed)");
    if (first == GDE_ERR_NOT_CONVERGED) return fail(first, "some queries reached max_iters");
    return GDE_OK;
}

}  // namespace gde

using namespace gde;

// Warm LocalGD re-solve of B standing queries (one kind and parameter) from
// their current state, all in one batch: see WarmState and the warm-start
// kernels.  res[i] receives iterations, work, residual norms and status.
int gde::batch_warm_resolve(gde_ctx *ctx, const gde_graph *g, int32_t B, const gde_params *p, void *const *rd,
                            void *const *x, uint32_t *const *pushed, uint32_t *const *tbm, gde_result *res,
                            hipStream_t s) {
    std::vector<gde_seed> sd((size_t)B, gde_seed{0, nullptr, nullptr});
    for (int32_t i = 0; i < B; i++) {
        res[i] = gde_result{};
        res[i].status = GDE_OK;
    }
    Schedule sc;
    sc.lanes = 16;
    sc.sort = 0;
    const WarmState ws{rd, x, pushed, tbm};
    return p[0].value_type == GDE_F64 ? solve_batch_fused<double>(ctx, g, B, p, sd.data(), res, sc, s, &ws)
                                      : solve_batch_fused<float>(ctx, g, B, p, sd.data(), res, sc, s, &ws);
}

// A batch whose work lists outgrow the workspace (GDE_ERR_OOM, state already
// restored) is solved as two halves, recursively, down to one lane group.
static int solve_batch_split(gde_ctx *ctx, const gde_graph *g, int32_t B, const gde_params *p, const gde_seed *s,
                             gde_result *res, const Schedule &sc, hipStream_t stream) {
    int rc = p[0].value_type == GDE_F64 ? solve_batch_fused<double>(ctx, g, B, p, s, res, sc, stream)
                                        : solve_batch_fused<float>(ctx, g, B, p, s, res, sc, stream);
    if (rc != GDE_ERR_OOM || B <= sc.lanes) return rc;
    const int32_t h = ((B / 2 + sc.lanes - 1) / sc.lanes) * sc.lanes;
    const int r1 = solve_batch_split(ctx, g, h, p, s, res, sc, stream);
    const int r2 = solve_batch_split(ctx, g, B - h, p + h, s + h, res + h, sc, stream);
    return r1 ? r1 : r2;
}

// "auto" schedule: the first batch of a (graph, kind, value type, size class)
// is solved twice with each candidate schedule, each run timed on the host
// around the whole call (workspace taken beforehand, so no candidate pays for
// an allocation); the candidate with the fastest run is kept in the context
// and used from then on.  The last run's results are returned (every run is a
// complete solve).
static int solve_batch_tuned(gde_ctx *ctx, const gde_graph *g, int32_t B, const gde_params *p, const gde_seed *s,
                             gde_result *res, const Schedule &sc, hipStream_t stream) {
    int bclass = 0;
    while ((1 << bclass) < B) bclass++;
    for (const gde_ctx::Tuned &t : ctx->tuned) {
        if (t.guid == g->uid && t.kind == p[0].kind && t.vtype == p[0].value_type && t.bclass == bclass) {
            Schedule c = sc;
            c.lanes = t.lanes;
            c.blocks_per_cu = t.bpc;
            return solve_batch_split(ctx, g, B, p, s, res, c, stream);
        }
    }
    static const int cand[][2] = {{8, 0}, {32, 0}, {16, 2}, {16, 0}};
    double best = 1e300;
    Schedule pick = sc;
    int rc = GDE_OK;
    for (const auto &cd : cand) {
        Schedule c = sc;
        c.lanes = cd[0];
        c.blocks_per_cu = cd[1];
        BatchWS *w = nullptr;
        if ((rc = batch_ws_get(ctx, g, p[0].value_type, c.lanes, (B + c.lanes - 1) / c.lanes, stream, &w))) return rc;
        GDE_HIP(hipStreamSynchronize(stream));
        for (int rep = 0; rep < 2; rep++) {
            const auto t0 = std::chrono::steady_clock::now();
            rc = solve_batch_split(ctx, g, B, p, s, res, c, stream);
            GDE_HIP(hipStreamSynchronize(stream));
            const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            if (rc != GDE_OK && rc != GDE_ERR_NOT_CONVERGED && rc != GDE_ERR_CAPACITY) return rc;
            if (dt < best) {
                best = dt;
                pick = c;
            }
        }
    }
    ctx->tuned.push_back(gde_ctx::Tuned{g->uid, p[0].kind, p[0].value_type, bclass, pick.lanes, pick.blocks_per_cu});
    return rc;
}

extern "C" {

int gde_batch_tuned(const gde_ctx *ctx, const gde_graph *g, int32_t kind, int32_t value_type, int32_t B,
                    int32_t *lanes, int32_t *blocks_per_cu) {
    if (!ctx || !g || !lanes || !blocks_per_cu || B < 1) return fail(GDE_ERR_INVALID_ARG, "null argument or B < 1");
    int bclass = 0;
    while ((1 << bclass) < B) bclass++;
    for (const gde_ctx::Tuned &t : ctx->tuned) {
        if (t.guid == g->uid && t.kind == kind && t.vtype == value_type && t.bclass == bclass) {
            *lanes = t.lanes;
            *blocks_per_cu = t.bpc;
            return GDE_OK;
        }
    }
    return fail(GDE_ERR_INVALID_ARG, "no schedule was chosen for this graph, kind, value type and batch size");
}

int gde_solve_batch(gde_ctx *ctx, const gde_graph *g, int32_t B, const gde_params *p, const gde_seed *s,
                    gde_result *res, const char *schedule_json, hipStream_t stream) {
    if (!ctx || !g || !p || !s || !res || B < 1) return fail(GDE_ERR_INVALID_ARG, "null argument or B < 1");
    Schedule sc;
    int rc = parse_schedule(schedule_json, &sc);
    if (rc) return rc;
    // validate everything on the host first
    for (int32_t i = 0; i < B; i++) {
        gde_seed one = s[i];
        gde_params pi = p[i];
        int v = gde_validate_query(g, &pi, &one);
        if (v) {
            for (int32_t j = 0; j < B; j++) res[j].status = j == i ? v : GDE_OK;
            return v;
        }
        if (res[i].capacity < 0) return fail(GDE_ERR_INVALID_ARG, "negative capacity");
    }
    // the fused kernels need one kind, LocalGD, one value type and shared kind
    // parameters (alpha, beta; tau and K; the series coefficients); anything
    // else is solved query by query (deterministic queries are solved one by
    // one in the fixed-order mode)
    auto same_kind_params = [](const gde_params &x, const gde_params &y) {
        if (x.kind != y.kind) return false;
        if (x.kind == GDE_PPR || x.kind == GDE_KATZ)
            return x.alpha == y.alpha && x.beta == y.beta && x.max_iters == y.max_iters &&
                   (x.method != GDE_LOCAL_CH || x.lambda_bound == y.lambda_bound);
        if (x.K != y.K) return false;
        if (x.kind == GDE_HK) return x.tau == y.tau;
        for (int32_t k = 0; k <= x.K; k++)
            if (x.c[k] != y.c[k]) return false;
        return true;
    };
    bool fused = (p[0].method == GDE_LOCAL_GD || p[0].method == GDE_LOCAL_CH) && !(p[0].flags & GDE_DETERMINISTIC);
    for (int32_t i = 1; i < B && fused; i++) {
        fused = same_kind_params(p[i], p[0]) && p[i].method == p[0].method && p[i].value_type == p[0].value_type &&
                !(p[i].flags & GDE_DETERMINISTIC) &&
                (p[i].flags & (GDE_RESULT_DEVICE | GDE_SYM_NORM)) == (p[0].flags & (GDE_RESULT_DEVICE | GDE_SYM_NORM));
    }
    GDE_HIP(hipSetDevice(ctx->device));
    // LocalSOR / APPR: every query in one wavefront of the same launch
    bool sor = true;
    for (int32_t i = 0; i < B && sor; i++)
        sor = p[i].method == GDE_LOCAL_SOR && p[i].value_type == p[0].value_type;
    if (sor) {
        for (int32_t i = 0; i < B; i++) res[i].status = GDE_OK;
        return solve_fifo(ctx, g, B, p, s, res, stream);
    }
    if (!fused) {
        int first = GDE_OK;
        for (int32_t i = 0; i < B; i++) {
            int r = gde_solve(ctx, g, &p[i], &s[i], &res[i], stream);
            res[i].status = r;
            if (r && !first) first = r;
        }
        return first;
    }
    if (sc.autotune) return solve_batch_tuned(ctx, g, B, p, s, res, sc, stream);
    return solve_batch_split(ctx, g, B, p, s, res, sc, stream);
}

}  // extern "C"
