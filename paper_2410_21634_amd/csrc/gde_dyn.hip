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
// parameter run together as the lanes of one batch (signed residuals: a lane
// whose |r| an update lifts across its threshold is a candidate, tested again
// by the snapshot), starting from and returning to the queries' own state.  A query's first solve runs the fixed-order iterations of the
// deterministic mode.  Everything in between stays resident: residuals,
// estimates, touched and pushed bitmaps, degrees.
//
// The graph lives on the device only, as a CSR with ascending rows in two
// buffer sets.  A batch becomes directed events keyed (source, delete flag,
// target) and radix-sorted on the device, so that each source's inserts come
// before its deletes, each group in target order.  One thread per event checks
// it against the current row (binary search: an insert must be absent, a
// delete present, no event twice) and records the target's position in the
// row.  The next version is then written into the spare set: new degrees, a
// scan for the row pointers, and one wavefront per row merging the old row
// (less its deleted entries) with its inserted targets.  The corrections run
// one thread per source, walking its events in key order (x_a and the degree
// change only by the node's own events, so D is exactly the sequential one);
// the additions into other nodes' residuals are atomic.
#include <hip/hip_runtime.h>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

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
int graph_set_csr(gde_graph *g, int32_t *rp, int32_t *ci, int64_t nnz);
void graph_add_degrees(gde_graph *g, const int32_t *nodes, int32_t k, int32_t delta);
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
    gde_graph *g = nullptr;                 // the current version (owned device CSR)
    gde::Workspace view;                    // lists, counters, deterministic-mode buffers
    std::vector<gde_dyn_query *> q;
    hipStream_t s = nullptr;
    // event buffers (device): keys as given and sorted, each event's position
    // in its source's row; pinned staging of the keys; sort / scan scratch
    uint64_t *ev_key = nullptr, *ev_sorted = nullptr, *h_key = nullptr;
    int32_t *ev_pos = nullptr;
    int64_t ev_cap = 0;
    void *tmp = nullptr;
    size_t tmp_bytes = 0;
    // per node: first sorted event of the node as a source (-1: none), its
    // insert and delete counts, its next degree; the check's error bits
    int32_t *nd_first = nullptr, *nd_ins = nullptr, *nd_del = nullptr, *nd_deg = nullptr, *d_err = nullptr;
    int32_t *h_err = nullptr;
    int32_t *blk = nullptr;  // output compaction
    long long *total = nullptr;
    gde::DevState *h_st = nullptr;
    // the device CSR in two buffer sets: the graph points at one, the next
    // version is written into the other
    int32_t *d_rp[2] = {nullptr, nullptr}, *d_ci[2] = {nullptr, nullptr};
    int64_t d_ci_cap[2] = {0, 0};
    int cur = 0;
};

namespace gde {

// an event key: the source in the high word, then the delete flag, then the target
__device__ __forceinline__ int32_t ev_src(uint64_t k) { return (int32_t)(k >> 32); }
__device__ __forceinline__ int32_t ev_dst(uint64_t k) { return (int32_t)(k & 0x7fffffffu); }
__device__ __forceinline__ bool ev_is_del(uint64_t k) { return ((k >> 31) & 1u) != 0u; }

// per sorted event: a repeat of the previous key, the test against the
// current row of its source (ascending, binary search) and the target's
// lower-bound position in that row; a source's first event records the
// source's event range
__global__ void k_dyn_check(const uint64_t *__restrict__ key, int32_t m, const int32_t *__restrict__ rp,
                            const int32_t *__restrict__ ci, int32_t *__restrict__ pos, int32_t *__restrict__ first,
                            int32_t *__restrict__ nins, int32_t *__restrict__ ndel, int32_t *err) {
    const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= m) return;
    const uint64_t k = key[i];
    const int32_t a = ev_src(k), c = ev_dst(k);
    const bool del = ev_is_del(k);
    const int32_t b = rp[a], e = rp[a + 1];
    int32_t lo = b, hi = e;
    while (lo < hi) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if (ci[mid] < c) lo = mid + 1;
        else hi = mid;
    }
    const bool found = lo < e && ci[lo] == c;
    const int bad = (!del && found ? 1 : 0) | (del && !found ? 2 : 0) | (i > 0 && key[i - 1] == k ? 4 : 0);
    pos[i] = lo - b;
    if (bad) atomicOr(err, bad);
    if (i == 0 || ev_src(key[i - 1]) != a) {
        int32_t ni = 0, nd = 0;
        for (int32_t j = i; j < m && ev_src(key[j]) == a; j++) {
            if (ev_is_del(key[j])) nd++;
            else ni++;
        }
        first[a] = i;
        nins[a] = ni;
        ndel[a] = nd;
    }
}

// the next degrees (the scan input) and the first row pointer
__global__ void k_dyn_degree(const int32_t *__restrict__ rp, const int32_t *__restrict__ first,
                             const int32_t *__restrict__ nins, const int32_t *__restrict__ ndel, int32_t n,
                             int32_t *__restrict__ deg, int32_t *__restrict__ new_rp) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u == 0) new_rp[0] = 0;
    if (u < n) deg[u] = rp[u + 1] - rp[u] + (first[u] >= 0 ? nins[u] - ndel[u] : 0);
}

// entries of the ascending list p[0, len) below v (strictly, or up to v inclusive)
__device__ __forceinline__ int32_t dyn_rank(const int32_t *p, int32_t len, int32_t v, bool incl) {
    int32_t lo = 0, hi = len;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (incl ? p[mid] <= v : p[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// one wavefront per row: a row without events is copied; otherwise old entry k
// (not deleted) lands after the k - (deletes before k) old ones kept and the
// inserts whose position is at most k, and insert j (targets ascending) with
// position p after the p - (deletes before p) old ones kept and j inserts
__global__ void __launch_bounds__(256) k_dyn_merge(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                   const int32_t *__restrict__ new_rp, int32_t *__restrict__ new_ci,
                                                   int32_t n, const uint64_t *__restrict__ key,
                                                   const int32_t *__restrict__ pos, const int32_t *__restrict__ first,
                                                   const int32_t *__restrict__ nins, const int32_t *__restrict__ ndel) {
    const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) / kWave);
    const int lane = (int)__lane_id();
    const int nwaves = (int)(gridDim.x * blockDim.x / kWave);
    for (int32_t u = wave; u < n; u += nwaves) {
        const int32_t b = rp[u], d0 = rp[u + 1] - b, nb = new_rp[u], f = first[u];
        if (f < 0) {
            for (int32_t k = lane; k < d0; k += kWave) new_ci[nb + k] = ci[b + k];
            continue;
        }
        const int32_t ni = nins[u], nd = ndel[u];
        const int32_t *ip = pos + f, *dp = pos + f + ni;
        for (int32_t k = lane; k < d0; k += kWave) {
            const int32_t db = dyn_rank(dp, nd, k, false);
            if (db < nd && dp[db] == k) continue;  // deleted
            new_ci[nb + k - db + dyn_rank(ip, ni, k, true)] = ci[b + k];
        }
        for (int32_t j = lane; j < ni; j += kWave) {
            const int32_t p = ip[j];
            new_ci[nb + p - dyn_rank(dp, nd, p, false) + j] = ev_dst(key[f + j]);
        }
    }
}

__global__ void k_dyn_reset(const uint64_t *__restrict__ key, int32_t m, int32_t *first) {
    const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < m) first[ev_src(key[i])] = -1;
}

// one thread per source (its first sorted event), degrees from the old rows
template <typename V>
__global__ void k_dyn_correct(const uint64_t *__restrict__ key, int32_t m, const int32_t *__restrict__ rp, RD<V> *rd,
                              V *x, uint32_t *tbm, int ppr, double param) {
    const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= m) return;
    const int32_t a = ev_src(key[i]);
    if (i > 0 && ev_src(key[i - 1]) == a) return;
    double xa = (double)x[a], ra = 0.0;
    int32_t d = rp[a + 1] - rp[a];
    for (int32_t e = i; e < m; e++) {
        const uint64_t k = key[e];
        if (ev_src(k) != a) break;
        const int32_t c = ev_dst(k);
        const int sg = ev_is_del(k) ? -1 : 1;
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

// buffer set k holds at least nnz column entries (12.5 % headroom on growth)
static int dyn_reserve_set(gde_dyn *dy, int k, int64_t nnz) {
    if (!dy->d_rp[k]) GDE_HIP(hipMalloc((void **)&dy->d_rp[k], 4 * ((size_t)dy->n + 1)));
    const int64_t need = std::max<int64_t>(nnz, 1);
    if (need > dy->d_ci_cap[k]) {
        if (dy->d_ci[k]) (void)hipFree(dy->d_ci[k]);
        dy->d_ci[k] = nullptr;
        dy->d_ci_cap[k] = 0;
        const int64_t cap = need + need / 8;
        GDE_HIP(hipMalloc((void **)&dy->d_ci[k], 4 * (size_t)cap));
        dy->d_ci_cap[k] = cap;
    }
    return GDE_OK;
}

// event buffers for m events, and sort / scan scratch for them (keys of
// end_bit bits) and for n nodes
static int dyn_reserve_events(gde_dyn *dy, int64_t m, int end_bit) {
    if (m > dy->ev_cap) {
        const int64_t cap = std::max<int64_t>(m + m / 4, 4096);
        if (dy->ev_key) (void)hipFree(dy->ev_key);
        if (dy->ev_sorted) (void)hipFree(dy->ev_sorted);
        if (dy->ev_pos) (void)hipFree(dy->ev_pos);
        if (dy->h_key) (void)hipHostFree(dy->h_key);
        dy->ev_key = dy->ev_sorted = dy->h_key = nullptr;
        dy->ev_pos = nullptr;
        dy->ev_cap = 0;
        GDE_HIP(hipMalloc((void **)&dy->ev_key, 8 * (size_t)cap));
        GDE_HIP(hipMalloc((void **)&dy->ev_sorted, 8 * (size_t)cap));
        GDE_HIP(hipMalloc((void **)&dy->ev_pos, 4 * (size_t)cap));
        GDE_HIP(hipHostMalloc((void **)&dy->h_key, 8 * (size_t)cap, 0));
        dy->ev_cap = cap;
    }
    size_t sort_bytes = 0, scan_bytes = 0;
    GDE_HIP(rocprim::radix_sort_keys(nullptr, sort_bytes, dy->ev_key, dy->ev_sorted, (size_t)m, 0, end_bit, dy->s));
    GDE_HIP(rocprim::inclusive_scan(nullptr, scan_bytes, dy->nd_deg, dy->d_rp[0], (size_t)dy->n,
                                    rocprim::plus<int32_t>(), dy->s));
    const size_t need = std::max(sort_bytes, scan_bytes);
    if (need > dy->tmp_bytes) {
        if (dy->tmp) (void)hipFree(dy->tmp);
        dy->tmp = nullptr;
        dy->tmp_bytes = 0;
        GDE_HIP(hipMalloc(&dy->tmp, need));
        dy->tmp_bytes = need;
    }
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
    for (int32_t u = 0; u < n; u++) std::sort(ci.begin() + rp[u], ci.begin() + rp[u + 1]);  // rows ascending
    gde_dyn *dy = new gde_dyn();
    dy->ctx = ctx;
    dy->vtype = value_type;
    dy->vs = value_type == GDE_F64 ? 8 : 4;
    dy->n = n;
    const int64_t nnz = g0->nnz;
    hipError_t e = hipStreamCreate(&dy->s);
    int rc = e == hipSuccess ? dyn_reserve_set(dy, 0, nnz) : hip_fail(e, "hipStreamCreate");
    if (!rc) {
        Workspace &w = dy->view;
        w.n = n;
        w.vtype = value_type;
        w.vsize = dy->vs;
        e = hipMemcpy(dy->d_rp[0], rp.data(), 4 * ((size_t)n + 1), hipMemcpyHostToDevice);
        if (e == hipSuccess && nnz > 0) e = hipMemcpy(dy->d_ci[0], ci.data(), 4 * (size_t)nnz, hipMemcpyHostToDevice);
        for (int i = 0; i < 2 && e == hipSuccess; i++) e = hipMalloc((void **)&w.front[i], 4 * (size_t)n);
        if (e == hipSuccess) e = hipMalloc((void **)&w.st, sizeof(DevState));
        if (e == hipSuccess) e = hipMalloc((void **)&dy->blk, 4 * (size_t)(dense_nblk(n) + 1));
        if (e == hipSuccess) e = hipMalloc((void **)&dy->total, 8);
        if (e == hipSuccess) e = hipHostMalloc((void **)&dy->h_st, sizeof(DevState), 0);
        int32_t **nd[] = {&dy->nd_first, &dy->nd_ins, &dy->nd_del, &dy->nd_deg};
        for (int32_t **a : nd)
            if (e == hipSuccess) e = hipMalloc((void **)a, 4 * (size_t)std::max(n, 1));
        if (e == hipSuccess) e = hipMalloc((void **)&dy->d_err, 4);
        if (e == hipSuccess) e = hipHostMalloc((void **)&dy->h_err, 4, 0);
        if (e == hipSuccess) e = hipMemset(dy->nd_first, 0xff, 4 * (size_t)std::max(n, 1));  // -1: no events
        if (e != hipSuccess) rc = hip_fail(e, "dynamic graph buffers");
    }
    if (!rc) rc = dyn_reserve_events(dy, 1, 64);
    if (rc) {
        gde_dyn_destroy(dy);
        return rc;
    }
    dy->cur = 0;
    dy->g = graph_wrap_device(ctx, n, nnz, dy->d_rp[0], dy->d_ci[0]);
    dy->g->owned = false;  // the buffer sets belong to the dynamic graph
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
    if ((int64_t)k_ins + k_del > (int64_t)INT32_MAX / 2) return fail(GDE_ERR_INVALID_ARG, "too many events");
    const int32_t n = dy->n;
    for (int32_t i = 0; i < k_ins; i++)
        if (iu[i] < 0 || iu[i] >= n || iv[i] < 0 || iv[i] >= n || iu[i] == iv[i])
            return fail(GDE_ERR_INVALID_ARG, "bad inserted edge");
    for (int32_t i = 0; i < k_del; i++)
        if (du[i] < 0 || du[i] >= n || dv[i] < 0 || dv[i] >= n || du[i] == dv[i])
            return fail(GDE_ERR_INVALID_ARG, "bad deleted edge");
    const int32_t m = 2 * (k_ins + k_del);
    if (m == 0) return GDE_OK;
    GDE_HIP(hipSetDevice(dy->ctx->device));
    int nbits = 1;
    while (nbits < 31 && ((int64_t)1 << nbits) < (int64_t)n) nbits++;
    int rc = dyn_reserve_events(dy, m, 32 + nbits);
    if (rc) return rc;
    // directed events keyed (source, delete flag, target): both directions of each edge
    uint64_t *hk = dy->h_key;
    auto key = [](int32_t a, int32_t c, uint64_t del) { return ((uint64_t)(uint32_t)a << 32) | (del << 31) | (uint32_t)c; };
    for (int32_t i = 0; i < k_ins; i++) {
        hk[2 * i] = key(iu[i], iv[i], 0);
        hk[2 * i + 1] = key(iv[i], iu[i], 0);
    }
    for (int32_t i = 0; i < k_del; i++) {
        hk[2 * (k_ins + i)] = key(du[i], dv[i], 1);
        hk[2 * (k_ins + i) + 1] = key(dv[i], du[i], 1);
    }
    const int32_t *rp = dy->d_rp[dy->cur], *ci = dy->d_ci[dy->cur];
    const unsigned eg = (unsigned)((m + 255) / 256);
    GDE_HIP(hipMemcpyAsync(dy->ev_key, hk, 8 * (size_t)m, hipMemcpyHostToDevice, dy->s));
    size_t tb = dy->tmp_bytes;
    GDE_HIP(rocprim::radix_sort_keys(dy->tmp, tb, dy->ev_key, dy->ev_sorted, (size_t)m, 0, 32 + nbits, dy->s));
    GDE_HIP(hipMemsetAsync(dy->d_err, 0, 4, dy->s));
    hipLaunchKernelGGL(k_dyn_check, dim3(eg), dim3(256), 0, dy->s, dy->ev_sorted, m, rp, ci, dy->ev_pos, dy->nd_first,
                       dy->nd_ins, dy->nd_del, dy->d_err);
    GDE_HIP(hipGetLastError());
    GDE_HIP(hipMemcpyAsync(dy->h_err, dy->d_err, 4, hipMemcpyDeviceToHost, dy->s));
    GDE_HIP(hipStreamSynchronize(dy->s));
    if (const int bad = *dy->h_err) {  // nothing changes: clear the per-node marks and report
        hipLaunchKernelGGL(k_dyn_reset, dim3(eg), dim3(256), 0, dy->s, dy->ev_sorted, m, dy->nd_first);
        GDE_HIP(hipGetLastError());
        GDE_HIP(hipStreamSynchronize(dy->s));
        return fail(GDE_ERR_INVALID_ARG, (bad & 1)   ? "inserted edge already exists"
                                         : (bad & 2) ? "deleted edge does not exist"
                                                     : "an edge appears twice in one batch");
    }
    // the next version in the spare buffer set
    const int k = dy->cur ^ 1;
    const int64_t nnz = dy->g->nnz + 2 * ((int64_t)k_ins - k_del);
    if ((rc = dyn_reserve_set(dy, k, nnz))) return rc;
    hipLaunchKernelGGL(k_dyn_degree, dim3((unsigned)(((int64_t)n + 255) / 256)), dim3(256), 0, dy->s, rp, dy->nd_first,
                       dy->nd_ins, dy->nd_del, n, dy->nd_deg, dy->d_rp[k]);
    GDE_HIP(hipGetLastError());
    tb = dy->tmp_bytes;
    GDE_HIP(rocprim::inclusive_scan(dy->tmp, tb, dy->nd_deg, dy->d_rp[k] + 1, (size_t)n, rocprim::plus<int32_t>(),
                                    dy->s));
    const unsigned mg = (unsigned)std::min<int64_t>(((int64_t)n + 3) / 4, 8192);  // 4 wavefronts per block
    hipLaunchKernelGGL(k_dyn_merge, dim3(std::max(mg, 1u)), dim3(256), 0, dy->s, rp, ci, dy->d_rp[k], dy->d_ci[k], n,
                       dy->ev_sorted, dy->ev_pos, dy->nd_first, dy->nd_ins, dy->nd_del);
    GDE_HIP(hipGetLastError());
    // the corrections, against the old degrees
    for (gde_dyn_query *q : dy->q) {
        const int ppr = q->p.kind == GDE_PPR;
        const double param = ppr ? q->p.alpha : q->p.beta;
        if (dy->vtype == GDE_F64)
            hipLaunchKernelGGL(k_dyn_correct<double>, dim3(eg), dim3(256), 0, dy->s, dy->ev_sorted, m, rp,
                               (RD<double> *)q->rd, (double *)q->x, q->tbm, ppr, param);
        else
            hipLaunchKernelGGL(k_dyn_correct<float>, dim3(eg), dim3(256), 0, dy->s, dy->ev_sorted, m, rp,
                               (RD<float> *)q->rd, (float *)q->x, q->tbm, ppr, param);
        GDE_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_dyn_reset, dim3(eg), dim3(256), 0, dy->s, dy->ev_sorted, m, dy->nd_first);
    GDE_HIP(hipGetLastError());
    // the graph switches to the new set (the old one stays intact until the next batch)
    dy->cur = k;
    graph_set_csr(dy->g, dy->d_rp[k], dy->d_ci[k], nnz);
    dy->g->owned = false;  // the buffer sets belong to the dynamic graph
    graph_add_degrees(dy->g, iu, k_ins, 1);
    graph_add_degrees(dy->g, iv, k_ins, 1);
    graph_add_degrees(dy->g, du, k_del, -1);
    graph_add_degrees(dy->g, dv, k_del, -1);
    if ((rc = batch_workspaces_refresh(dy->g, dy->bctx, dy->s))) return rc;
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
    void *p[] = {w.front[0], w.front[1], w.st, dy->blk, dy->total, dy->ev_key, dy->ev_sorted, dy->ev_pos, dy->tmp,
                 dy->nd_first, dy->nd_ins, dy->nd_del, dy->nd_deg, dy->d_err};
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
    if (dy->h_key) (void)hipHostFree(dy->h_key);
    if (dy->h_err) (void)hipHostFree(dy->h_err);
    delete dy;
    return GDE_OK;
}

}  // extern "C"
