// gde_global.hip -- the standard (global) counterparts of LocalGD and LocalCH.
//
// Table 2 and the eps sweep of Sec. 5 compare the local solvers with GD and
// Chebyshev iterations over the whole node set: S_t = V in every iteration,
// x <- x + h, r <- r - Q h with h = r (GD) or the Chebyshev combination of
// Sec. 3.3 (CH), until no node has |r_u| >= theta_u.  On the GPU each
// iteration is one sparse matrix-vector product over all rows, written as a
// pull: node w gathers z_u = W_u h_u over its neighbours (W_u = (1-alpha)/d_u
// for PPR, beta for Katz) and computes its own new residual, then its next
// update h and z_w for the following iteration.  That is one launch per
// iteration, a streaming pass over col_idx with the z gathers served by the
// caches, and no atomics on values.  x takes h at the start of the next
// iteration, so an update is applied only when the stop test has let the
// iteration run.
//
// The solver runs on its own copy of the graph with nodes relabelled by
// descending degree (made once per graph on the GPU).  On power-law graphs most
// CSR entries point at the high-degree nodes, so the gathers of z then fall on
// a short prefix of the array that the L2 caches hold; seeds are mapped in and
// x is mapped back to the caller's ids in the output pass.  Rows of at most
// kLongRow entries are summed by kLanesPerRow lanes each (strided loads, a
// fixed shuffle tree); the longer ones -- the first nlong rows after the
// relabelling -- get a workgroup each (fixed LDS tree).  The order of every sum is fixed, so
// two runs give bit-identical results.  The stop test counts active nodes per
// workgroup into one of three counter slots (iteration t reads slot t mod 3,
// writes t+1 mod 3, clears t+2 mod 3), and a launch whose iteration has no
// active node, or that follows such a launch, returns at once, so the host
// enqueues chunks of iterations and synchronises once per chunk.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "gde_batch.h"
#include "gde_device.h"
#include "gde_global.h"

namespace gde {

constexpr int kGlobBlock = 256;
constexpr int kLanesPerRow = 8;
constexpr int kRowsPerBlock = kGlobBlock / kLanesPerRow;
constexpr int kLongRow = 512;  // rows longer than this get a workgroup each

struct GlobCnt {            // counters of one iteration slot
    unsigned long long active;  // nodes with |r_u| >= theta_u after the iteration
    unsigned long long pad[7];
};

struct GlobWS {
    const gde_graph *g = nullptr;
    uint64_t guid = 0;
    int64_t n = 0, nnz = 0;
    size_t vs = 4;
    void *x = nullptr, *r = nullptr, *h = nullptr, *z[2] = {nullptr, nullptr};
    int32_t *rp = nullptr;         // the relabelled CSR: node v is the caller's node order[v]
    int32_t *ci = nullptr;
    int32_t *order = nullptr;      // [n] new id -> caller's id
    int32_t *inv = nullptr;        // [n] caller's id -> new id
    std::vector<int32_t> h_inv;    // host copy of inv (seed mapping)
    int32_t nlong = 0;             // rows longer than kLongRow: new ids [0, nlong)
    GlobCnt *cnt = nullptr;        // [3] slots
    int32_t *iters = nullptr;      // iterations that ran
    int32_t *blk = nullptr;        // output compaction: per-block counts, then offsets
    double *part = nullptr;        // norm partials: [nblk] l1, [nblk] max
    double *nrm = nullptr;         // [2]
    long long *total = nullptr;    // [1] support size
    int64_t nblk = 0;
    int32_t *seed_idx = nullptr;
    double *seed_val = nullptr;
    int32_t seed_cap = 0;
    void *h_buf = nullptr;         // pinned host mirror: counters and norms
};

void glob_ws_free(GlobWS *w) {
    if (!w) return;
    void *p[] = {w->x, w->r, w->h, w->z[0], w->z[1], w->rp, w->ci, w->order, w->inv, w->cnt, w->iters, w->blk,
                 w->part, w->nrm, w->total, w->seed_idx, w->seed_val};
    for (void *q : p)
        if (q) (void)hipFree(q);
    if (w->h_buf) (void)hipHostFree(w->h_buf);
    delete w;
}

template <typename V>
struct GlobArgs {
    int32_t n;
    const int32_t *row_ptr;
    const int32_t *col_idx;
    int32_t nlong;
    V *x, *r, *h;
    const V *z_cur;
    V *z_next;
    V wscale;     // (1 - alpha) (PPR, divided by d_u) or beta (Katz)
    int div_deg;  // PPR
    V eps_eff;    // theta_u = eps_eff * d_u
    GlobCnt *cnt;
    int32_t *iters;
};

// the per-node epilogue: apply h_t, new residual, next update and its scatter value
template <typename V>
__device__ __forceinline__ unsigned glob_node(const GlobArgs<V> &a, int32_t w, int32_t dw, V sum, int ch, V c, V m) {
    const V hw = a.h[w];
    a.x[w] = a.x[w] + hw;
    const V rn = a.r[w] - hw + sum;
    a.r[w] = rn;
    const V hn = ch ? c * rn + m * hw : rn;
    a.h[w] = hn;
    V zw = (V)0;
    if (dw > 0) zw = a.div_deg ? (a.wscale / (V)dw) * hn : a.wscale * hn;
    a.z_next[w] = zw;
    return (rn != (V)0 && fabs(rn) >= a.eps_eff * (V)dw) ? 1u : 0u;
}

template <typename V>
__global__ void __launch_bounds__(kGlobBlock) k_glob_step(GlobArgs<V> a, int t, V c, V m, int ch) {
    __shared__ V s_sum[kGlobBlock];
    __shared__ unsigned s_act[kGlobBlock / kWave];
    // stopped: an earlier launch returned here (iters stopped growing), or the
    // previous iteration left no active node.  Block 0 below moves iters to
    // t + 1 while other blocks of this launch read it, so they see t or t + 1.
    if (a.iters[0] < t || a.cnt[t % 3].active == 0ull) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.cnt[(t + 2) % 3].active = 0ull;
        a.iters[0] = t + 1;
    }
    unsigned act = 0u;
    if ((int)blockIdx.x < a.nlong) {
        // one long row per workgroup
        const int32_t w = (int32_t)blockIdx.x;
        const int32_t beg = a.row_ptr[w], end = a.row_ptr[w + 1];
        V sum = (V)0;
        for (int32_t e = beg + (int32_t)threadIdx.x; e < end; e += kGlobBlock) sum += a.z_cur[a.col_idx[e]];
        s_sum[threadIdx.x] = sum;
        __syncthreads();
        for (int off = kGlobBlock / 2; off > 0; off >>= 1) {
            if ((int)threadIdx.x < off) s_sum[threadIdx.x] = s_sum[threadIdx.x] + s_sum[threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0) act = glob_node(a, w, end - beg, s_sum[0], ch, c, m);
    } else {
        const int sub = (int)threadIdx.x / kLanesPerRow, sl = (int)threadIdx.x % kLanesPerRow;
        const int64_t w64 = a.nlong + (int64_t)((int)blockIdx.x - a.nlong) * kRowsPerBlock + sub;
        if (w64 < a.n) {
            const int32_t w = (int32_t)w64;
            const int32_t beg = a.row_ptr[w], end = a.row_ptr[w + 1];
            V sum = (V)0;
            for (int32_t e = beg + sl; e < end; e += kLanesPerRow) sum += a.z_cur[a.col_idx[e]];
#pragma unroll
            for (int off = kLanesPerRow / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off, kLanesPerRow);
            if (sl == 0) act = glob_node(a, w, end - beg, sum, ch, c, m);
        }
    }
    // active count: a wave sum, then one atomic per workgroup
    for (int off = kWave / 2; off > 0; off >>= 1) act += __shfl_xor(act, off);
    if (lane() == 0) s_act[threadIdx.x / kWave] = act;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tot = 0ull;
        for (int i = 0; i < kGlobBlock / kWave; i++) tot += s_act[i];
        if (tot) atomicAdd(&a.cnt[(t + 1) % 3].active, tot);
    }
}

// x = 0, r = b on the seeds and 0 elsewhere, h = r (the first update), z = W h;
// slot 0 says "run" (the first iteration is forced), slots 1 and 2 are cleared
template <typename V>
__global__ void k_glob_init(GlobArgs<V> a) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < a.n; u += (int64_t)gridDim.x * blockDim.x) {
        a.x[u] = (V)0;
        a.r[u] = (V)0;
        a.h[u] = (V)0;
        a.z_next[u] = (V)0;  // z of iteration 0 (the caller passes it as z_next here)
    }
    if (blockIdx.x == 0 && threadIdx.x < 3) {
        a.cnt[threadIdx.x].active = threadIdx.x == 0 ? 1ull : 0ull;
        if (threadIdx.x == 0) a.iters[0] = 0;
    }
}

template <typename V>
__global__ void k_glob_seed(GlobArgs<V> a, const int32_t *__restrict__ sidx, const double *__restrict__ sval,
                            int32_t ns, double bscale) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ns) {
        const int32_t u = sidx[i];
        const V b = (V)(bscale * sval[i]);
        a.r[u] = b;
        a.h[u] = b;
        const int32_t du = a.row_ptr[u + 1] - a.row_ptr[u];
        a.z_next[u] = a.div_deg ? (a.wscale / (V)du) * b : a.wscale * b;
    }
}

// residual norms over all nodes in a fixed shape: per-block partials, then one block
template <typename V>
__global__ void __launch_bounds__(kGlobBlock) k_glob_norm_part(const V *__restrict__ r, const int32_t *__restrict__ rp,
                                                                int64_t n, double rscale, double *part, int64_t nblk) {
    __shared__ double s_l1[kGlobBlock], s_mx[kGlobBlock];
    const int64_t u = blockIdx.x * (int64_t)kGlobBlock + threadIdx.x;
    double l1 = 0.0, mx = 0.0;
    if (u < n) {
        const double v = fabs((double)r[u]) * rscale;
        l1 = v;
        const double d = (double)(rp[u + 1] - rp[u]);
        if (d > 0.0) mx = v / d;
    }
    s_l1[threadIdx.x] = l1;
    s_mx[threadIdx.x] = mx;
    __syncthreads();
    for (int off = kGlobBlock / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            s_l1[threadIdx.x] = s_l1[threadIdx.x] + s_l1[threadIdx.x + off];
            s_mx[threadIdx.x] = fmax(s_mx[threadIdx.x], s_mx[threadIdx.x + off]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[blockIdx.x] = s_l1[0];
        part[nblk + blockIdx.x] = s_mx[0];
    }
}

__global__ void __launch_bounds__(kGlobBlock) k_glob_norm_final(const double *__restrict__ part, int64_t nblk,
                                                                 double *nrm) {
    __shared__ double s_l1[kGlobBlock], s_mx[kGlobBlock];
    double l1 = 0.0, mx = 0.0;
    for (int64_t j = threadIdx.x; j < nblk; j += kGlobBlock) {
        l1 = l1 + part[j];
        mx = fmax(mx, part[nblk + j]);
    }
    s_l1[threadIdx.x] = l1;
    s_mx[threadIdx.x] = mx;
    __syncthreads();
    for (int off = kGlobBlock / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            s_l1[threadIdx.x] = s_l1[threadIdx.x] + s_l1[threadIdx.x + off];
            s_mx[threadIdx.x] = fmax(s_mx[threadIdx.x], s_mx[threadIdx.x + off]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        nrm[0] = s_l1[0];
        nrm[1] = s_mx[0];
    }
}

// sparse output: the nodes with x_u != 0 in ascending order
// (x is read through inv when given: entry u of the output order is x[inv[u]])
template <typename V>
__global__ void __launch_bounds__(kGlobBlock) k_glob_count(const V *__restrict__ x, const int32_t *__restrict__ inv,
                                                            int64_t n, int32_t *blk) {
    __shared__ int s[kGlobBlock / kWave];
    const int64_t u = blockIdx.x * (int64_t)kGlobBlock + threadIdx.x;
    int c = (u < n && x[inv ? inv[u] : u] != (V)0) ? 1 : 0;
    for (int off = kWave / 2; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if (lane() == 0) s[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int i = 0; i < kGlobBlock / kWave; i++) tot += s[i];
        blk[blockIdx.x] = tot;
    }
}

__global__ void __launch_bounds__(1024) k_glob_scan(int32_t *blk, int64_t nblk, long long *total) {
    __shared__ long long s[1024];
    const int64_t per = (nblk + 1023) / 1024;
    const int64_t lo = threadIdx.x * per;
    const int64_t hi = lo + per < nblk ? lo + per : nblk;
    long long acc = 0;
    for (int64_t i = lo; i < hi; i++) acc += blk[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const long long y = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += y;
        __syncthreads();
    }
    long long run = s[threadIdx.x] - acc;
    for (int64_t i = lo; i < hi; i++) {
        const int32_t v = blk[i];
        blk[i] = (int32_t)run;
        run += v;
    }
    if (threadIdx.x == 1023) *total = s[1023];
}

template <typename V>
__global__ void __launch_bounds__(kGlobBlock) k_glob_emit(const V *__restrict__ x, const int32_t *__restrict__ inv,
                                                           int64_t n, const int32_t *__restrict__ blk,
                                                           int32_t *out_idx, V *out_val) {
    __shared__ int s_w[kGlobBlock / kWave];
    const int64_t u = blockIdx.x * (int64_t)kGlobBlock + threadIdx.x;
    const V v = u < n ? x[inv ? inv[u] : u] : (V)0;
    const bool nz = v != (V)0;
    const unsigned long long bal = __ballot(nz);
    const int before = __popcll(bal & lanemask_lt());
    if (lane() == 0) s_w[threadIdx.x / kWave] = __popcll(bal);
    __syncthreads();
    int off = blk[blockIdx.x];
    for (int i = 0; i < (int)threadIdx.x / kWave; i++) off += s_w[i];
    if (nz) {
        out_idx[off + before] = (int32_t)u;
        out_val[off + before] = v;
    }
}

// row v of the relabelled CSR = row order[v] of the caller's, columns mapped by inv
__global__ void __launch_bounds__(kGlobBlock) k_glob_relabel(const int32_t *__restrict__ rp,
                                                              const int32_t *__restrict__ ci,
                                                              const int32_t *__restrict__ order,
                                                              const int32_t *__restrict__ inv,
                                                              const int32_t *__restrict__ nrp, int32_t *nci, int32_t n) {
    const int64_t wid = (blockIdx.x * (int64_t)kGlobBlock + threadIdx.x) / kWave;
    const int64_t nw = (int64_t)gridDim.x * kGlobBlock / kWave;
    for (int64_t v = wid; v < n; v += nw) {
        const int32_t u = order[v];
        const int32_t beg = rp[u], len = rp[u + 1] - beg, dst = nrp[v];
        for (int32_t k = lane(); k < len; k += kWave) nci[dst + k] = inv[ci[beg + k]];
    }
}

// ------------------------------------------------------------------ host side
static int glob_ws_get(Workspace *w, const gde_graph *g, hipStream_t s, GlobWS **out) {
    if (w->glob && w->glob->guid == g->uid && w->glob->nnz == g->nnz) {
        *out = w->glob;
        return GDE_OK;
    }
    glob_ws_free(w->glob);
    w->glob = nullptr;
    GlobWS *q = new GlobWS();
    q->g = g;
    q->guid = g->uid;
    q->n = g->n;
    q->nnz = g->nnz;
    q->vs = w->vsize;
    q->nblk = (g->n + kGlobBlock - 1) / kGlobBlock;
    hipError_t e = hipSuccess;
    auto al = [&](void **p, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc(p, std::max<size_t>(bytes, 16));
    };
    al(&q->x, q->vs * q->n);
    al(&q->r, q->vs * q->n);
    al(&q->h, q->vs * q->n);
    al(&q->z[0], q->vs * q->n);
    al(&q->z[1], q->vs * q->n);
    al((void **)&q->cnt, 3 * sizeof(GlobCnt));
    al((void **)&q->iters, 64);
    al((void **)&q->blk, 4 * (size_t)(q->nblk + 1));
    al((void **)&q->part, 16 * (size_t)q->nblk);
    al((void **)&q->nrm, 16);
    al((void **)&q->total, 8);
    if (e == hipSuccess) e = hipHostMalloc(&q->h_buf, 4096, 0);
    // relabelling by descending degree (ties by id), from the host copy of the row pointers
    const int32_t n = g->n;
    std::vector<int32_t> rp((size_t)n + 1), order((size_t)n), nrp((size_t)n + 1);
    q->h_inv.assign((size_t)n, 0);
    if (e == hipSuccess) e = hipMemcpy(rp.data(), g->row_ptr, 4 * ((size_t)n + 1), hipMemcpyDeviceToHost);
    if (e == hipSuccess) {
        for (int32_t u = 0; u < n; u++) order[u] = u;
        std::stable_sort(order.begin(), order.end(),
                         [&](int32_t a2, int32_t b2) { return rp[a2 + 1] - rp[a2] > rp[b2 + 1] - rp[b2]; });
        nrp[0] = 0;
        q->nlong = 0;
        for (int32_t v = 0; v < n; v++) {
            const int32_t d = rp[order[v] + 1] - rp[order[v]];
            nrp[v + 1] = nrp[v] + d;
            q->h_inv[order[v]] = v;
            if (d > kLongRow) q->nlong = v + 1;
        }
        al((void **)&q->rp, 4 * ((size_t)n + 1));
        al((void **)&q->ci, 4 * (size_t)g->nnz);
        al((void **)&q->order, 4 * (size_t)n);
        al((void **)&q->inv, 4 * (size_t)n);
    }
    if (e == hipSuccess) e = hipMemcpy(q->rp, nrp.data(), 4 * ((size_t)n + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(q->order, order.data(), 4 * (size_t)n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(q->inv, q->h_inv.data(), 4 * (size_t)n, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_glob_relabel, dim3(8192), dim3(kGlobBlock), 0, s, g->row_ptr, g->col_idx, q->order,
                           q->inv, q->rp, q->ci, n);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        glob_ws_free(q);
        return hip_fail(e, "global solver workspace");
    }
    w->glob = q;
    *out = q;
    return GDE_OK;
}

template <typename V>
static int glob_run(gde_ctx *ctx, const gde_graph *g, const gde_params *p, const gde_seed *sd, gde_result *res,
                    hipStream_t s) {
    Workspace *w = nullptr;
    int rc = get_workspace(ctx, g, p->value_type, s, &w);
    if (rc) return rc;
    GlobWS *q = nullptr;
    if ((rc = glob_ws_get(w, g, s, &q))) return rc;
    if (sd->nnz > q->seed_cap) {
        if (q->seed_idx) { (void)hipFree(q->seed_idx); (void)hipFree(q->seed_val); }
        q->seed_idx = nullptr;
        q->seed_val = nullptr;
        q->seed_cap = 0;
        GDE_HIP(hipMalloc((void **)&q->seed_idx, 4 * (size_t)sd->nnz));
        GDE_HIP(hipMalloc((void **)&q->seed_val, 8 * (size_t)sd->nnz));
        q->seed_cap = sd->nnz;
    }
    std::vector<int32_t> sidx((size_t)sd->nnz);
    for (int32_t i = 0; i < sd->nnz; i++) sidx[i] = q->h_inv[sd->idx[i]];
    GDE_HIP(hipMemcpyAsync(q->seed_idx, sidx.data(), 4 * (size_t)sd->nnz, hipMemcpyHostToDevice, s));
    GDE_HIP(hipMemcpyAsync(q->seed_val, sd->val, 8 * (size_t)sd->nnz, hipMemcpyHostToDevice, s));

    const bool ppr = p->kind == GDE_PPR;
    const bool ch = p->method == GDE_LOCAL_CH;
    GlobArgs<V> a{};
    a.n = g->n;
    a.row_ptr = q->rp;
    a.col_idx = q->ci;
    a.nlong = q->nlong;
    a.x = (V *)q->x;
    a.r = (V *)q->r;
    a.h = (V *)q->h;
    a.wscale = (V)(ppr ? 1.0 - p->alpha : p->beta);
    a.div_deg = ppr ? 1 : 0;
    a.eps_eff = (V)(ppr ? p->alpha * p->eps : p->eps);
    a.cnt = q->cnt;
    a.iters = q->iters;
    const double bscale = ppr ? p->alpha : 1.0;
    a.z_cur = (const V *)q->z[1];
    a.z_next = (V *)q->z[0];
    hipLaunchKernelGGL(k_glob_init<V>, dim3((unsigned)std::min<int64_t>((g->n + 255) / 256, 8192)), dim3(256), 0, s,
                       a);
    hipLaunchKernelGGL(k_glob_seed<V>, dim3((sd->nnz + 255) / 256), dim3(256), 0, s, a, q->seed_idx, q->seed_val,
                       sd->nnz, bscale);
    GDE_HIP(hipGetLastError());

    // Chebyshev coefficients of iterations 1, 2, ... (iteration t's launch
    // computes the update of t + 1), as in the local solver
    double sigma = 1.0, dlt = 0.0;
    if (ch) {
        double mu, L;
        if (ppr) { mu = p->alpha; L = 2.0 - p->alpha; }
        else { mu = 1.0 - p->beta * p->lambda_bound; L = 1.0 + p->beta * p->lambda_bound; }
        sigma = (L + mu) / (L - mu);
        dlt = 1.0 / sigma;
    }
    const unsigned grid = (unsigned)(q->nlong + (g->n - q->nlong + kRowsPerBlock - 1) / kRowsPerBlock);
    int t = 0, chunk = 4;
    int32_t T = 0;
    bool converged = false;
    long long *hb = (long long *)q->h_buf;
    while (t < p->max_iters) {
        const int end = std::min(p->max_iters, t + chunk);
        if ((rc = prof_mark(ctx, s))) return rc;
        for (; t < end; t++) {
            double c = 1.0, m = 0.0;
            if (ch) {
                const double dnext = 1.0 / (2.0 * sigma - dlt);
                c = 2.0 * sigma * dnext;
                m = dlt * dnext;
                dlt = dnext;
            }
            a.z_cur = (const V *)q->z[t & 1];
            a.z_next = (V *)q->z[(t + 1) & 1];
            hipLaunchKernelGGL(k_glob_step<V>, dim3(grid), dim3(kGlobBlock), 0, s, a, t, (V)c, (V)m, ch ? 1 : 0);
        }
        if ((rc = prof_mark(ctx, s))) return rc;
        GDE_HIP(hipGetLastError());
        GDE_HIP(hipMemcpyAsync(hb, q->iters, 4, hipMemcpyDeviceToHost, s));
        GDE_HIP(hipMemcpyAsync(hb + 1, q->cnt, 3 * sizeof(GlobCnt), hipMemcpyDeviceToHost, s));
        GDE_HIP(hipStreamSynchronize(s));
        T = (int32_t)(*(int32_t *)hb);
        const GlobCnt *hc = (const GlobCnt *)(hb + 1);
        if (hc[T % 3].active == 0ull) { converged = true; break; }
        chunk = std::min(chunk * 2, 64);
    }
    if ((rc = prof_collect(ctx, (int64_t)T * g->nnz, (int64_t)T * g->n))) return rc;
    // residual norms and the sparse output
    hipLaunchKernelGGL(k_glob_norm_part<V>, dim3((unsigned)q->nblk), dim3(kGlobBlock), 0, s, (const V *)q->r,
                       q->rp, (int64_t)g->n, ppr ? 1.0 / p->alpha : 1.0, q->part, q->nblk);
    hipLaunchKernelGGL(k_glob_norm_final, dim3(1), dim3(kGlobBlock), 0, s, q->part, q->nblk, q->nrm);
    hipLaunchKernelGGL(k_glob_count<V>, dim3((unsigned)q->nblk), dim3(kGlobBlock), 0, s, (const V *)q->x, q->inv,
                       (int64_t)g->n, q->blk);
    hipLaunchKernelGGL(k_glob_scan, dim3(1), dim3(1024), 0, s, q->blk, q->nblk, q->total);
    GDE_HIP(hipGetLastError());
    GDE_HIP(hipMemcpyAsync(hb, q->total, 8, hipMemcpyDeviceToHost, s));
    GDE_HIP(hipMemcpyAsync(hb + 1, q->nrm, 16, hipMemcpyDeviceToHost, s));
    GDE_HIP(hipStreamSynchronize(s));
    const long long nnz = hb[0];
    double nrm[2];
    std::memcpy(nrm, hb + 1, 16);
    res->nnz = nnz;
    res->iters = T;
    res->ops = (int64_t)T * g->nnz;
    res->pushes = (int64_t)T * g->n;
    res->residual_l1 = nrm[0];
    res->residual_dinf = nrm[1];
    res->trace_len = T;
    res->trace_nodes_len = 0;
    if ((p->flags & GDE_TRACE) && res->trace_capacity > 0) {
        const int64_t mm = std::min<int64_t>(T, res->trace_capacity);
        for (int64_t i = 0; i < mm; i++) {
            if (res->trace_size) res->trace_size[i] = g->n;
            if (res->trace_vol) res->trace_vol[i] = g->nnz;
        }
    }
    const bool fits = res->idx && res->val && nnz <= res->capacity;
    if (!fits) {
        res->status = GDE_ERR_CAPACITY;
        return fail(GDE_ERR_CAPACITY, "result capacity too small; result.nnz holds the size needed");
    }
    if (nnz > 0) {
        if (p->flags & GDE_RESULT_DEVICE) {
            hipLaunchKernelGGL(k_glob_emit<V>, dim3((unsigned)q->nblk), dim3(kGlobBlock), 0, s, (const V *)q->x,
                               q->inv, (int64_t)g->n, q->blk, res->idx, (V *)res->val);
            GDE_HIP(hipGetLastError());
            GDE_HIP(hipStreamSynchronize(s));
        } else {
            // stage through the (free) z buffers: nnz <= n entries of each
            hipLaunchKernelGGL(k_glob_emit<V>, dim3((unsigned)q->nblk), dim3(kGlobBlock), 0, s, (const V *)q->x,
                               q->inv, (int64_t)g->n, q->blk, (int32_t *)q->z[0], (V *)q->z[1]);
            GDE_HIP(hipGetLastError());
            GDE_HIP(hipMemcpyAsync(res->idx, q->z[0], 4 * (size_t)nnz, hipMemcpyDeviceToHost, s));
            GDE_HIP(hipMemcpyAsync(res->val, q->z[1], q->vs * (size_t)nnz, hipMemcpyDeviceToHost, s));
            GDE_HIP(hipStreamSynchronize(s));
        }
    }
    res->status = converged ? GDE_OK : GDE_ERR_NOT_CONVERGED;
    if (!converged) return fail(GDE_ERR_NOT_CONVERGED, "max_iters reached before no node was active");
    return GDE_OK;
}

int64_t dense_nblk(int64_t n) { return (n + kGlobBlock - 1) / kGlobBlock; }

template <typename V>
void launch_dense_count(const V *x, int64_t n, int32_t *blk, hipStream_t s) {
    hipLaunchKernelGGL(k_glob_count<V>, dim3((unsigned)dense_nblk(n)), dim3(kGlobBlock), 0, s, x,
                       (const int32_t *)nullptr, n, blk);
}

void launch_dense_scan(int32_t *blk, int64_t nblk, long long *total, hipStream_t s) {
    hipLaunchKernelGGL(k_glob_scan, dim3(1), dim3(1024), 0, s, blk, nblk, total);
}

template <typename V>
void launch_dense_emit(const V *x, int64_t n, const int32_t *blk, int32_t *idx, V *val, hipStream_t s) {
    hipLaunchKernelGGL(k_glob_emit<V>, dim3((unsigned)dense_nblk(n)), dim3(kGlobBlock), 0, s, x,
                       (const int32_t *)nullptr, n, blk, idx, val);
}

template void launch_dense_count<float>(const float *, int64_t, int32_t *, hipStream_t);
template void launch_dense_count<double>(const double *, int64_t, int32_t *, hipStream_t);
template void launch_dense_emit<float>(const float *, int64_t, const int32_t *, int32_t *, float *, hipStream_t);
template void launch_dense_emit<double>(const double *, int64_t, const int32_t *, int32_t *, double *, hipStream_t);

int solve_global(gde_ctx *ctx, const gde_graph *g, const gde_params *p, const gde_seed *sd, gde_result *res,
                 hipStream_t s) {
    if (p->value_type == GDE_F64) return glob_run<double>(ctx, g, p, sd, res, s);
    return glob_run<float>(ctx, g, p, sd, res, s);
}

}  // namespace gde
