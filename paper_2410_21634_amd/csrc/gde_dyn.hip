// gde_dyn.hip -- standing queries on a dynamic graph (Sec. 4, dynamic GDEs).
//
// A gde_dyn owns a private copy of a graph that changes by batches of edge
// insertions and deletions, and a set of standing PPR / Katz queries whose
// state (x, r) stays on the device between batches.  A batch is applied as
// (1) the Insert and Delete corrections of LocalGS(Dynamic) / LocalSOR(Dynamic)
// (Algorithms 2-5) in the generic form r = b - Q x: each undirected edge {a, c}
// is the directed event a -> c and then c -> a, inserts before deletes, and
// for PPR an event at a with current degree d moves D = x_a / d: insert
// x_a += D, r_a -= D, r_c += (1-alpha) D; delete x_a -= D, r_a += D,
// r_c -= (1-alpha) D (a node of degree 0 only adds (1-alpha) x_a to r_c on
// its first new edge); for Katz r_c += beta x_a or -= beta x_a; then (2) a
// warm LocalGD re-solve of every query from its corrected state (S_0 = the
// active nodes, residuals may be negative): the queries of one kind and
// parameter run together as the lanes of one batch (every touched lane a
// candidate, signed residuals), starting from and returning to the queries'
// own state.  A query's first solve runs the fixed-order iterations of the
// deterministic mode.  Everything in between stays resident: residuals,
// estimates, touched and pushed bitmaps, degrees.
//
// The corrections run one thread per node that has events, walking its events
// in their order (x_a and the degree change only by the node's own events, so
// D is exactly the sequential one); the additions into other nodes' residuals
// are atomic.  The graph is kept as a host adjacency (validation of events,
// CSR rebuild) and a device CSR that is replaced after each batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "gde_batch.h"
#include "gde_det.h"
#include "gde_device.h"
#include "gde_global.h"
#include "gde_kernels.h"

namespace gde {
gde_graph *graph_wrap_device(gde_ctx *ctx, int32_t n, int64_t nnz, int32_t *rp, int32_t *ci);
int graph_set_csr(gde_graph *g, int32_t *rp, int32_t *ci, int64_t nnz, const std::vector<int32_t> &deg);
}  // namespace gde

struct gde_dyn_query {
    gde_params p{};
    std::vector<int32_t> sidx;
    std::vector<double> sval;
    void *rd = nullptr;          // RD<V>[n]: residual and current degree
    void *x = nullptr;           // V[n]
    uint32_t *pushed = nullptr;  // nodes ever pushed
    uint32_t *tbm = nullptr;     // nodes whose residual may be nonzero
    int32_t iters = 0;           // of the last (re)solve
    int64_t ops = 0, pushes = 0;
    double res_l1 = 0.0, res_dinf = 0.0;
    int status = GDE_OK;
};

struct gde_dyn {
    gde_ctx *ctx = nullptr;
    // private context of the batched re-solves, not in the library's list of
    // contexts: its workspace survives the CSR replacements and is refreshed
    gde_ctx *bctx = nullptr;
    int vtype = GDE_F64;
    size_t vs = 8;
    int32_t n = 0;
    std::vector<std::vector<int32_t>> adj;  // sorted neighbour lists of the current graph
    gde_graph *g = nullptr;                 // the current version (owned device CSR)
    gde::Workspace view;                    // lists, counters, deterministic-mode buffers
    std::vector<gde_dyn_query *> q;
    hipStream_t s = nullptr;
    // event buffers (device): sources, their event ranges, targets and signs
    int32_t *ev_src = nullptr, *ev_off = nullptr, *ev_dst = nullptr, *ev_sign = nullptr;
    int64_t ev_cap = 0, src_cap = 0;
    int32_t *blk = nullptr;  // output compaction
    long long *total = nullptr;
    gde::DevState *h_st = nullptr;
    // the device CSR in two buffer sets (the graph points at one, the next
    // version is uploaded into the other) and its pinned host staging, so an
    // update allocates and frees nothing once the capacities suffice
    int32_t *d_rp[2] = {nullptr, nullptr}, *d_ci[2] = {nullptr, nullptr};
    int64_t d_ci_cap[2] = {0, 0};
    int cur = 0;
    int32_t *h_rp = nullptr, *h_ci = nullptr;
    int64_t h_ci_cap = 0;
};

namespace gde {

template <typename V>
__global__ void k_dyn_correct(const int32_t *__restrict__ src, const int32_t *__restrict__ off,
                              const int32_t *__restrict__ dst, const int32_t *__restrict__ sign, int32_t nsrc,
                              const int32_t *__restrict__ deg0, RD<V> *rd, V *x, uint32_t *tbm, int ppr, double param) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nsrc) return;
    const int32_t a = src[i];
    double xa = (double)x[a], ra = 0.0;
    int32_t d = deg0[i];
    for (int32_t e = off[i]; e < off[i + 1]; e++) {
        const int32_t c = dst[e];
        const int sg = sign[e];
        if (ppr) {
            if (d == 0) {  // first edge of an isolated node (an insert)
                atomicAdd(&rd[c].r, (V)((1.0 - param) * xa));
            } else {
                const double D = xa / (double)d;
                xa += sg * D;
                ra -= sg * D;
                atomicAdd(&rd[c].r, (V)(sg * (1.0 - param) * D));
            }
        } else {
            atomicAdd(&rd[c].r, (V)(sg * param * xa));
        }
        atomicOr(&tbm[c >> 5], 1u << (c & 31));
        d += sg;
    }
    x[a] = (V)xa;
    if (ra != 0.0) atomicAdd(&rd[a].r, (V)ra);
    rd[a].d = (V)d;
    atomicOr(&tbm[a >> 5], 1u << (a & 31));
}

template <typename V>
__global__ void k_dyn_seed(RD<V> *rd, uint32_t *tbm, const int32_t *__restrict__ idx, const double *__restrict__ val,
                           int32_t ns, double bscale) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ns) {
        const int32_t u = idx[i];
        rd[u].r = (V)(bscale * val[i]);
        atomicOr(&tbm[u >> 5], 1u << (u & 31));
    }
}

static void dyn_view_query(gde_dyn *dy, gde_dyn_query *q) {
    dy->view.rd = q->rd;
    dy->view.x = q->x;
    dy->view.bitmap = q->pushed;
    dy->view.tbm = q->tbm;
}

template <typename V>
static int dyn_resolve(gde_dyn *dy, gde_dyn_query *q, const int32_t *forced, int32_t nforced) {
    dyn_view_query(dy, q);
    int32_t T = 0;
    bool conv = false;
    int rc = det_warm<V>(dy->g, &q->p, &dy->view, dy->s, forced, nforced, &T, &conv);
    if (rc) return rc;
    GDE_HIP(hipMemcpyAsync(dy->h_st, dy->view.st, sizeof(DevState), hipMemcpyDeviceToHost, dy->s));
    GDE_HIP(hipStreamSynchronize(dy->s));
    q->iters = T;
    q->ops = dy->h_st->ops;
    q->pushes = dy->h_st->pushes;
    q->res_l1 = dy->h_st->res_l1;
    unsigned long long bits = dy->h_st->res_dinf;
    std::memcpy(&q->res_dinf, &bits, 8);
    q->status = conv ? GDE_OK : GDE_ERR_NOT_CONVERGED;
    return GDE_OK;
}

// the current adjacency as a CSR in the spare device buffer set (made the
// current one), staged through pinned host memory; returns its arrays
static int dyn_upload_csr(gde_dyn *dy, int32_t **rp_out, int32_t **ci_out, int64_t *nnz_out,
                          std::vector<int32_t> *deg) {
    const int32_t n = dy->n;
    if (!dy->h_rp) GDE_HIP(hipHostMalloc((void **)&dy->h_rp, 4 * ((size_t)n + 1), 0));
    int32_t *rp = dy->h_rp;
    rp[0] = 0;
    deg->assign((size_t)n, 0);
    for (int32_t u = 0; u < n; u++) {
        (*deg)[u] = (int32_t)dy->adj[u].size();
        rp[u + 1] = rp[u] + (*deg)[u];
    }
    const int64_t nnz = rp[n];
    const int64_t need = std::max<int64_t>(nnz, 1);
    if (need > dy->h_ci_cap) {
        if (dy->h_ci) (void)hipHostFree(dy->h_ci);
        dy->h_ci = nullptr;
        dy->h_ci_cap = 0;
        const int64_t cap = need + need / 8;  // room for growth
        GDE_HIP(hipHostMalloc((void **)&dy->h_ci, 4 * (size_t)cap, 0));
        dy->h_ci_cap = cap;
    }
    for (int32_t u = 0; u < n; u++) std::copy(dy->adj[u].begin(), dy->adj[u].end(), dy->h_ci + rp[u]);
    const int k = dy->d_rp[dy->cur] ? dy->cur ^ 1 : dy->cur;  // the set the graph does not use
    if (!dy->d_rp[k]) GDE_HIP(hipMalloc((void **)&dy->d_rp[k], 4 * ((size_t)n + 1)));
    if (need > dy->d_ci_cap[k]) {
        if (dy->d_ci[k]) (void)hipFree(dy->d_ci[k]);
        dy->d_ci[k] = nullptr;
        dy->d_ci_cap[k] = 0;
        const int64_t cap = need + need / 8;
        GDE_HIP(hipMalloc((void **)&dy->d_ci[k], 4 * (size_t)cap));
        dy->d_ci_cap[k] = cap;
    }
    GDE_HIP(hipMemcpyAsync(dy->d_rp[k], rp, 4 * ((size_t)n + 1), hipMemcpyHostToDevice, dy->s));
    GDE_HIP(hipMemcpyAsync(dy->d_ci[k], dy->h_ci, 4 * (size_t)need, hipMemcpyHostToDevice, dy->s));
    GDE_HIP(hipStreamSynchronize(dy->s));  // the staging is reused by the next update
    dy->cur = k;
    *rp_out = dy->d_rp[k];
    *ci_out = dy->d_ci[k];
    *nnz_out = nnz;
    return GDE_OK;
}

static void dyn_query_free(gde_dyn_query *q) {
    void *p[] = {q->rd, q->x, q->pushed, q->tbm};
    for (void *v : p)
        if (v) (void)hipFree(v);
    delete q;
}

}  // namespace gde

using namespace gde;

extern "C" {

int gde_dyn_create(gde_ctx *ctx, const gde_graph *g0, int32_t value_type, gde_dyn **out) {
    if (!ctx || !g0 || !out) return fail(GDE_ERR_INVALID_ARG, "null argument");
    if (value_type != GDE_F32 && value_type != GDE_F64) return fail(GDE_ERR_INVALID_ARG, "unknown value_type");
    if (g0->device != ctx->device) return fail(GDE_ERR_INVALID_ARG, "graph and context on different devices");
    GDE_HIP(hipSetDevice(ctx->device));
    const int32_t n = g0->n;
    std::vector<int32_t> rp((size_t)n + 1), ci((size_t)std::max<int64_t>(g0->nnz, 1));
    GDE_HIP(hipMemcpy(rp.data(), g0->row_ptr, 4 * ((size_t)n + 1), hipMemcpyDeviceToHost));
    if (g0->nnz > 0) GDE_HIP(hipMemcpy(ci.data(), g0->col_idx, 4 * (size_t)g0->nnz, hipMemcpyDeviceToHost));
    gde_dyn *dy = new gde_dyn();
    dy->ctx = ctx;
    dy->vtype = value_type;
    dy->vs = value_type == GDE_F64 ? 8 : 4;
    dy->n = n;
    dy->adj.resize(n);
    for (int32_t u = 0; u < n; u++) dy->adj[u].assign(ci.begin() + rp[u], ci.begin() + rp[u + 1]);
    int32_t *drp = nullptr, *dci = nullptr;
    int64_t nnz = 0;
    std::vector<int32_t> deg;
    int rc = dyn_upload_csr(dy, &drp, &dci, &nnz, &deg);
    if (rc) {
        gde_dyn_destroy(dy);
        return rc;
    }
    dy->g = graph_wrap_device(ctx, n, nnz, drp, dci);
    dy->g->owned = false;  // the buffer sets belong to the dynamic graph
    Workspace &w = dy->view;
    w.n = n;
    w.vtype = value_type;
    w.vsize = dy->vs;
    hipError_t e = hipSuccess;
    for (int i = 0; i < 2 && e == hipSuccess; i++) e = hipMalloc((void **)&w.front[i], 4 * (size_t)n);
    if (e == hipSuccess) e = hipMalloc((void **)&w.st, sizeof(DevState));
    if (e == hipSuccess) e = hipMalloc((void **)&dy->blk, 4 * (size_t)(dense_nblk(n) + 1));
    if (e == hipSuccess) e = hipMalloc((void **)&dy->total, 8);
    if (e == hipSuccess) e = hipHostMalloc((void **)&dy->h_st, sizeof(DevState), 0);
    if (e == hipSuccess) e = hipStreamCreate(&dy->s);
    if (e != hipSuccess) {
        gde_dyn_destroy(dy);
        return hip_fail(e, "dynamic graph buffers");
    }
    dy->bctx = new gde_ctx();
    dy->bctx->device = ctx->device;
    *out = dy;
    return GDE_OK;
}

const gde_graph *gde_dyn_graph(const gde_dyn *dy) { return dy ? dy->g : nullptr; }

int gde_dyn_add(gde_dyn *dy, const gde_params *p, const gde_seed *s, int32_t *qid) {
    if (!dy || !p || !s || !qid) return fail(GDE_ERR_INVALID_ARG, "null argument");
    int rc = gde_validate_query(dy->g, p, s);
    if (rc) return rc;
    if ((p->kind != GDE_PPR && p->kind != GDE_KATZ) || p->method != GDE_LOCAL_GD)
        return fail(GDE_ERR_UNSUPPORTED, "standing queries are PPR or Katz with LocalGD");
    if (p->value_type != dy->vtype) return fail(GDE_ERR_INVALID_ARG, "value_type differs from the dynamic graph's");
    if (p->flags & GDE_KATZ_SUBTRACT_SEED) return fail(GDE_ERR_UNSUPPORTED, "standing Katz queries keep x, not x - s");
    if (p->flags & GDE_SYM_NORM) return fail(GDE_ERR_UNSUPPORTED, "standing queries use M = A D^-1");
    GDE_HIP(hipSetDevice(dy->ctx->device));
    const int64_t n = dy->n;
    gde_dyn_query *q = new gde_dyn_query();
    q->p = *p;
    q->p.flags = 0;
    q->sidx.assign(s->idx, s->idx + s->nnz);
    q->sval.assign(s->val, s->val + s->nnz);
    const size_t words = ((size_t)n + 31) / 32;
    hipError_t e = hipMalloc(&q->rd, 2 * dy->vs * (size_t)n);
    if (e == hipSuccess) e = hipMalloc(&q->x, dy->vs * (size_t)n);
    if (e == hipSuccess) e = hipMalloc((void **)&q->pushed, 4 * words);
    if (e == hipSuccess) e = hipMalloc((void **)&q->tbm, 4 * words);
    if (e == hipSuccess) e = hipMemsetAsync(q->x, 0, dy->vs * (size_t)n, dy->s);
    if (e == hipSuccess) e = hipMemsetAsync(q->pushed, 0, 4 * words, dy->s);
    if (e == hipSuccess) e = hipMemsetAsync(q->tbm, 0, 4 * words, dy->s);
    if (e != hipSuccess) {
        dyn_query_free(q);
        return hip_fail(e, "standing query state");
    }
    int32_t *didx = nullptr;
    double *dval = nullptr;
    e = hipMalloc((void **)&didx, 4 * (size_t)s->nnz);
    if (e == hipSuccess) e = hipMalloc((void **)&dval, 8 * (size_t)s->nnz);
    if (e == hipSuccess) e = hipMemcpyAsync(didx, s->idx, 4 * (size_t)s->nnz, hipMemcpyHostToDevice, dy->s);
    if (e == hipSuccess) e = hipMemcpyAsync(dval, s->val, 8 * (size_t)s->nnz, hipMemcpyHostToDevice, dy->s);
    const double bscale = p->kind == GDE_PPR ? p->alpha : 1.0;
    if (dy->vtype == GDE_F64) {
        launch_init_rd<double>(dy->g->row_ptr, q->rd, dy->n, dy->s);
        hipLaunchKernelGGL(k_dyn_seed<double>, dim3((s->nnz + 255) / 256), dim3(256), 0, dy->s, (RD<double> *)q->rd,
                           q->tbm, didx, dval, s->nnz, bscale);
    } else {
        launch_init_rd<float>(dy->g->row_ptr, q->rd, dy->n, dy->s);
        hipLaunchKernelGGL(k_dyn_seed<float>, dim3((s->nnz + 255) / 256), dim3(256), 0, dy->s, (RD<float> *)q->rd,
                           q->tbm, didx, dval, s->nnz, bscale);
    }
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(dy->s);
    (void)hipFree(didx);
    (void)hipFree(dval);
    if (e != hipSuccess) {
        dyn_query_free(q);
        return hip_fail(e, "standing query seed");
    }
    // the first solve: S_0 = supp(s), forced (Definition 3.1)
    rc = dy->vtype == GDE_F64 ? dyn_resolve<double>(dy, q, q->sidx.data(), s->nnz)
                              : dyn_resolve<float>(dy, q, q->sidx.data(), s->nnz);
    if (rc) {
        dyn_query_free(q);
        return rc;
    }
    dy->q.push_back(q);
    *qid = (int32_t)dy->q.size() - 1;
    return GDE_OK;
}

int gde_dyn_update(gde_dyn *dy, int32_t k_ins, const int32_t *iu, const int32_t *iv, int32_t k_del,
                   const int32_t *du, const int32_t *dv) {
    if (!dy || k_ins < 0 || k_del < 0 || (k_ins > 0 && (!iu || !iv)) || (k_del > 0 && (!du || !dv)))
        return fail(GDE_ERR_INVALID_ARG, "bad event arrays");
    const int32_t n = dy->n;
    // validation against the current graph, before any change
    std::vector<std::pair<int32_t, int32_t>> ins, del;
    auto has = [&](int32_t a, int32_t b) { return std::binary_search(dy->adj[a].begin(), dy->adj[a].end(), b); };
    for (int32_t i = 0; i < k_ins; i++) {
        const int32_t a = iu[i], b = iv[i];
        if (a < 0 || a >= n || b < 0 || b >= n || a == b) return fail(GDE_ERR_INVALID_ARG, "bad inserted edge");
        if (has(a, b)) return fail(GDE_ERR_INVALID_ARG, "inserted edge already exists");
        ins.emplace_back(std::min(a, b), std::max(a, b));
    }
    for (int32_t i = 0; i < k_del; i++) {
        const int32_t a = du[i], b = dv[i];
        if (a < 0 || a >= n || b < 0 || b >= n || a == b) return fail(GDE_ERR_INVALID_ARG, "bad deleted edge");
        if (!has(a, b)) return fail(GDE_ERR_INVALID_ARG, "deleted edge does not exist");
        del.emplace_back(std::min(a, b), std::max(a, b));
    }
    {
        auto a2 = ins, b2 = del;
        std::sort(a2.begin(), a2.end());
        std::sort(b2.begin(), b2.end());
        if (std::adjacent_find(a2.begin(), a2.end()) != a2.end() || std::adjacent_find(b2.begin(), b2.end()) != b2.end())
            return fail(GDE_ERR_INVALID_ARG, "an edge appears twice in one batch");
    }
    GDE_HIP(hipSetDevice(dy->ctx->device));
    // directed events in order (inserts, then deletes; a -> c then c -> a), grouped by source
    struct Ev { int32_t a, c, sg; };
    std::vector<Ev> evs;
    evs.reserve(2 * ((size_t)k_ins + k_del));
    for (int32_t i = 0; i < k_ins; i++) { evs.push_back({iu[i], iv[i], 1}); evs.push_back({iv[i], iu[i], 1}); }
    for (int32_t i = 0; i < k_del; i++) { evs.push_back({du[i], dv[i], -1}); evs.push_back({dv[i], du[i], -1}); }
    std::stable_sort(evs.begin(), evs.end(), [](const Ev &x, const Ev &y) { return x.a < y.a; });
    std::vector<int32_t> src, off, dst, sgn, deg0;
    for (size_t i = 0; i < evs.size(); i++) {
        if (i == 0 || evs[i].a != evs[i - 1].a) {
            src.push_back(evs[i].a);
            off.push_back((int32_t)i);
            deg0.push_back((int32_t)dy->adj[evs[i].a].size());
        }
        dst.push_back(evs[i].c);
        sgn.push_back(evs[i].sg);
    }
    off.push_back((int32_t)evs.size());
    const int32_t nsrc = (int32_t)src.size();
    // the new graph
    for (auto &e : ins) {
        for (int dir = 0; dir < 2; dir++) {
            auto &v = dy->adj[dir ? e.second : e.first];
            v.insert(std::lower_bound(v.begin(), v.end(), dir ? e.first : e.second), dir ? e.first : e.second);
        }
    }
    for (auto &e : del) {
        for (int dir = 0; dir < 2; dir++) {
            auto &v = dy->adj[dir ? e.second : e.first];
            v.erase(std::lower_bound(v.begin(), v.end(), dir ? e.first : e.second));
        }
    }
    int32_t *drp = nullptr, *dci = nullptr;
    int64_t nnz = 0;
    std::vector<int32_t> deg;
    int rc = dyn_upload_csr(dy, &drp, &dci, &nnz, &deg);
    if (rc) return rc;
    graph_set_csr(dy->g, drp, dci, nnz, deg);
    dy->g->owned = false;  // the buffer sets belong to the dynamic graph
    if ((rc = batch_workspaces_refresh(dy->g, dy->bctx, dy->s))) return rc;
    if (nsrc == 0) return GDE_OK;
    // event buffers
    if ((int64_t)dst.size() > dy->ev_cap || nsrc + 1 > dy->src_cap) {
        void *p[] = {dy->ev_src, dy->ev_off, dy->ev_dst, dy->ev_sign};
        for (void *v : p)
            if (v) (void)hipFree(v);
        dy->ev_cap = std::max<int64_t>((int64_t)dst.size(), 1024);
        dy->src_cap = std::max<int64_t>(2 * (int64_t)(nsrc + 1), 1024);
        GDE_HIP(hipMalloc((void **)&dy->ev_src, 8 * (size_t)dy->src_cap));  // src, then deg0
        GDE_HIP(hipMalloc((void **)&dy->ev_off, 4 * (size_t)dy->src_cap));
        GDE_HIP(hipMalloc((void **)&dy->ev_dst, 4 * (size_t)dy->ev_cap));
        GDE_HIP(hipMalloc((void **)&dy->ev_sign, 4 * (size_t)dy->ev_cap));
    }
    int32_t *d_deg0 = dy->ev_src + dy->src_cap;
    GDE_HIP(hipMemcpyAsync(dy->ev_src, src.data(), 4 * (size_t)nsrc, hipMemcpyHostToDevice, dy->s));
    GDE_HIP(hipMemcpyAsync(d_deg0, deg0.data(), 4 * (size_t)nsrc, hipMemcpyHostToDevice, dy->s));
    GDE_HIP(hipMemcpyAsync(dy->ev_off, off.data(), 4 * (size_t)(nsrc + 1), hipMemcpyHostToDevice, dy->s));
    GDE_HIP(hipMemcpyAsync(dy->ev_dst, dst.data(), 4 * dst.size(), hipMemcpyHostToDevice, dy->s));
    GDE_HIP(hipMemcpyAsync(dy->ev_sign, sgn.data(), 4 * sgn.size(), hipMemcpyHostToDevice, dy->s));
    for (gde_dyn_query *q : dy->q) {
        const int ppr = q->p.kind == GDE_PPR;
        const double param = ppr ? q->p.alpha : q->p.beta;
        if (dy->vtype == GDE_F64)
            hipLaunchKernelGGL(k_dyn_correct<double>, dim3((nsrc + 255) / 256), dim3(256), 0, dy->s, dy->ev_src,
                               dy->ev_off, dy->ev_dst, dy->ev_sign, nsrc, d_deg0, (RD<double> *)q->rd,
                               (double *)q->x, q->tbm, ppr, param);
        else
            hipLaunchKernelGGL(k_dyn_correct<float>, dim3((nsrc + 255) / 256), dim3(256), 0, dy->s, dy->ev_src,
                               dy->ev_off, dy->ev_dst, dy->ev_sign, nsrc, d_deg0, (RD<float> *)q->rd,
                               (float *)q->x, q->tbm, ppr, param);
        GDE_HIP(hipGetLastError());
    }
    // the re-solves: one batch per kind and parameter
    std::vector<bool> done(dy->q.size(), false);
    for (size_t i = 0; i < dy->q.size(); i++) {
        if (done[i]) continue;
        const gde_params &pi = dy->q[i]->p;
        std::vector<size_t> grp;
        for (size_t j = i; j < dy->q.size(); j++) {
            const gde_params &pj = dy->q[j]->p;
            if (!done[j] && pj.kind == pi.kind && pj.alpha == pi.alpha && pj.beta == pi.beta &&
                pj.max_iters == pi.max_iters) {
                grp.push_back(j);
                done[j] = true;
            }
        }
        const int32_t B = (int32_t)grp.size();
        std::vector<gde_params> ps(B);
        std::vector<void *> rd(B), x(B);
        std::vector<uint32_t *> pushed(B), tbm(B);
        std::vector<gde_result> res(B);
        for (int32_t k = 0; k < B; k++) {
            gde_dyn_query *q = dy->q[grp[k]];
            ps[k] = q->p;
            rd[k] = q->rd;
            x[k] = q->x;
            pushed[k] = q->pushed;
            tbm[k] = q->tbm;
        }
        rc = batch_warm_resolve(dy->bctx, dy->g, B, ps.data(), rd.data(), x.data(), pushed.data(), tbm.data(),
                                res.data(), dy->s);
        if (rc && rc != GDE_ERR_NOT_CONVERGED) return rc;
        for (int32_t k = 0; k < B; k++) {
            gde_dyn_query *q = dy->q[grp[k]];
            q->iters = res[k].iters;
            q->ops = res[k].ops;
            q->pushes = res[k].pushes;
            q->res_l1 = res[k].residual_l1;
            q->res_dinf = res[k].residual_dinf;
            q->status = res[k].status;
        }
    }
    GDE_HIP(hipStreamSynchronize(dy->s));
    return GDE_OK;
}

int gde_dyn_read(gde_dyn *dy, int32_t qid, gde_result *res, uint32_t flags) {
    if (!dy || !res || qid < 0 || qid >= (int32_t)dy->q.size()) return fail(GDE_ERR_INVALID_ARG, "bad query id");
    if (res->capacity < 0) return fail(GDE_ERR_INVALID_ARG, "negative capacity");
    GDE_HIP(hipSetDevice(dy->ctx->device));
    gde_dyn_query *q = dy->q[qid];
    const int64_t n = dy->n, nblk = dense_nblk(n);
    if (dy->vtype == GDE_F64) launch_dense_count<double>((const double *)q->x, n, dy->blk, dy->s);
    else launch_dense_count<float>((const float *)q->x, n, dy->blk, dy->s);
    launch_dense_scan(dy->blk, nblk, dy->total, dy->s);
    GDE_HIP(hipGetLastError());
    long long nnz = 0;
    GDE_HIP(hipMemcpyAsync(&nnz, dy->total, 8, hipMemcpyDeviceToHost, dy->s));
    GDE_HIP(hipStreamSynchronize(dy->s));
    res->nnz = nnz;
    res->iters = q->iters;
    res->ops = q->ops;
    res->pushes = q->pushes;
    res->residual_l1 = q->res_l1;
    res->residual_dinf = q->res_dinf;
    res->trace_len = 0;
    res->trace_nodes_len = 0;
    if (!res->idx || !res->val || nnz > res->capacity) {
        res->status = GDE_ERR_CAPACITY;
        return fail(GDE_ERR_CAPACITY, "result capacity too small; result.nnz holds the size needed");
    }
    if (nnz > 0) {
        int32_t *oi = (int32_t *)res->idx;
        void *ov = res->val;
        void *stage = nullptr;
        if (!(flags & GDE_RESULT_DEVICE)) {
            GDE_HIP(hipMalloc(&stage, (4 + dy->vs) * (size_t)nnz));
            oi = (int32_t *)stage;
            ov = (char *)stage + 4 * (size_t)nnz;
        }
        if (dy->vtype == GDE_F64)
            launch_dense_emit<double>((const double *)q->x, n, dy->blk, oi, (double *)ov, dy->s);
        else
            launch_dense_emit<float>((const float *)q->x, n, dy->blk, oi, (float *)ov, dy->s);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess && stage) {
            e = hipMemcpyAsync(res->idx, oi, 4 * (size_t)nnz, hipMemcpyDeviceToHost, dy->s);
            if (e == hipSuccess) e = hipMemcpyAsync(res->val, ov, dy->vs * (size_t)nnz, hipMemcpyDeviceToHost, dy->s);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(dy->s);
        if (stage) (void)hipFree(stage);
        if (e != hipSuccess) return hip_fail(e, "standing query output");
    }
    res->status = q->status;
    return GDE_OK;
}

int gde_dyn_destroy(gde_dyn *dy) {
    if (!dy) return fail(GDE_ERR_INVALID_ARG, "null dynamic graph");
    (void)hipSetDevice(dy->ctx->device);
    if (dy->g) dy->g->owned = false;  // freed below with the buffer sets
    if (dy->s) (void)hipStreamSynchronize(dy->s);
    for (gde_dyn_query *q : dy->q) dyn_query_free(q);
    Workspace &w = dy->view;
    void *p[] = {w.front[0], w.front[1], w.st, dy->blk, dy->total, dy->ev_src, dy->ev_off, dy->ev_dst, dy->ev_sign};
    for (void *v : p)
        if (v) (void)hipFree(v);
    det_ws_free(w.det);
    if (dy->h_st) (void)hipHostFree(dy->h_st);
    if (dy->s) (void)hipStreamDestroy(dy->s);
    if (dy->bctx) gde_ctx_destroy(dy->bctx);
    if (dy->g) gde_graph_destroy(dy->g);
    for (int k = 0; k < 2; k++) {
        if (dy->d_rp[k]) (void)hipFree(dy->d_rp[k]);
        if (dy->d_ci[k]) (void)hipFree(dy->d_ci[k]);
    }
    if (dy->h_rp) (void)hipHostFree(dy->h_rp);
    if (dy->h_ci) (void)hipHostFree(dy->h_ci);
    delete dy;
    return GDE_OK;
}

}  // extern "C"
