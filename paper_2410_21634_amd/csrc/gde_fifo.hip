// gde_fifo.hip -- LocalSOR (Eq. (7)) and APPR / AKatz (Algorithm 1, omega = 1)
// on the GPU: the sequential push, one query per wavefront.
//
// The paper's LocalSOR updates the nodes of S_t one after another, each with
// the residual left by the previous ones; with S_t taken from a FIFO queue
// this is the push of Algorithm 1 (APPR) generalised by omega.  A query's
// updates are inherently sequential, so a query is one wavefront: the popped
// node's scalar work runs on one lane, its row on all 64 (CSR order kept for
// the appends), and many queries run at once, one per wavefront.  Pop u;
// v = r_u; x_u += omega v; r_u -= omega v; r_w += (omega w_u) v for w in N(u)
// (w_u = (1-alpha)/d_u for PPR, beta for Katz); a neighbour that becomes
// active and is not queued joins the tail in CSR order, then u itself if it
// is still active.  Every operation is the sequential one, so in FP64 the
// result equals a sequential implementation of these steps bit for bit (FP
// contraction is off in this file).
//
// State is dense per slot (residual, estimate, queue ring of capacity n,
// touched list, a flag byte per node: queued / touched), each slot owned by
// one wavefront, so no atomics are needed.  The state is FP64 whatever the
// value type, which only sets the type of the returned x: a node is popped once
// per queue generation it is active in (hubs hundreds of times), so its
// residual and estimate take that many additions, and in FP32 their roundings
// add up past 1e-6 of the mass (measured: 1.16e-6 for Katz from a hub at
// omega 1.2, 22,930 pops); the kernel is bound by the latency of its dependent
// loads, not by bytes, so FP64 state costs nothing measurable.  Queries run in rounds of as many
// slots as the memory budget gives; after a round the outputs are compacted
// from the dense estimates (ascending ids) and the slots are reset through
// their touched lists.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "gde_batch.h"
#include "gde_device.h"
#include "gde_global.h"
#include "gde_internal.h"

namespace gde {

constexpr int kFifoBlock = 256;  // four wavefronts, four slots per workgroup
constexpr uint8_t kQueued = 1, kTouched = 2;

struct FifoQuery {
    double b;        // scale of the seed: alpha (PPR) or 1 (Katz)
    double w;        // (1 - alpha) (PPR, divided by d_u) or beta (Katz)
    double eps_eff;  // theta_u = eps_eff * d_u
    double omega;
    double rscale;   // reported residual scale: 1 / alpha (PPR) or 1
    int32_t ppr;
    int32_t pad;
    long long max_pops;
};

struct FifoStat {
    long long pops, ops, epochs, nt;
    double l1, dinf;
    int32_t status, pad;
};

struct FifoArgs {
    int32_t n;
    const int32_t *row_ptr, *col_idx;
    double *r, *x;     // [slots][n]
    uint8_t *fl;       // [slots][n]
    int32_t *q, *tl;   // [slots][n]
    int32_t nslots, q0, B;
    const FifoQuery *qp;            // [B]
    const long long *s_off;         // [B + 1] seed ranges
    const int32_t *s_idx;
    const double *s_val;
    FifoStat *stat;                 // [B]
};

__global__ void __launch_bounds__(kFifoBlock) k_fifo(FifoArgs a) {
    const int slot = (int)((blockIdx.x * (int64_t)kFifoBlock + threadIdx.x) / kWave);
    const int ln = lane();
    if (slot >= a.nslots) return;
    const int qi = a.q0 + slot;
    if (qi >= a.B) return;
    const int64_t n = a.n;
    double *r = a.r + (size_t)slot * n;
    double *x = a.x + (size_t)slot * n;
    uint8_t *fl = a.fl + (size_t)slot * n;
    int32_t *q = a.q + (size_t)slot * n;
    int32_t *tl = a.tl + (size_t)slot * n;
    const FifoQuery P = a.qp[qi];
    const long long s0 = a.s_off[qi], ns = a.s_off[qi + 1] - s0;
    // r = b on supp(s); the queue starts with supp(s) in index order
    for (long long i = ln; i < ns; i += kWave) {
        const int32_t u = a.s_idx[s0 + i];
        r[u] = P.b * a.s_val[s0 + i];
        fl[u] = kQueued | kTouched;
        q[i] = u;
        tl[i] = u;
    }
    __threadfence_block();
    long long head = 0, count = ns, nt = ns;
    long long pops = 0, ops = 0, epochs = 0, epoch_left = count;
    int status = GDE_OK;
    const double om = P.omega;
    // The next pop's node, row bounds and first 64 column ids are read while the
    // current pop runs: the queue entry is fixed once appended (appends go to
    // the tail of a ring of capacity n) and the CSR never changes, so only the
    // residuals and flags have to be read in order.
    bool have = false;
    int32_t nu = 0, nbeg = 0, nend = 0, nw = 0;
    while (count > 0) {
        if (pops >= P.max_pops) {
            status = GDE_ERR_NOT_CONVERGED;
            break;
        }
        if (epoch_left == 0) {
            epochs++;
            epoch_left = count;
        }
        const bool pre = have;
        int32_t u, beg, end;
        if (pre) {
            u = nu;
            beg = nbeg;
            end = nend;
        } else {
            u = q[head];
            beg = a.row_ptr[u];
            end = a.row_ptr[u + 1];
        }
        const int32_t w_first = nw;
        head = head + 1 == n ? 0 : head + 1;
        count--;
        epoch_left--;
        have = count > 0;  // the following pop is already in the queue
        if (have) nu = q[head];
        const int32_t du = end - beg;
        const double v = r[u];
        const double wu = P.ppr ? P.w / (double)du : P.w;
        const double coef = om * wu;
        double ru = 0.0;
        if (ln == 0) {
            x[u] = x[u] + om * v;
            ru = v - om * v;  // r[u] holds v: it is the residual just read
            r[u] = ru;
        }
        if (have) {
            nbeg = a.row_ptr[nu];
            nend = a.row_ptr[nu + 1];
        }
        for (int32_t base = beg; base < end; base += kWave) {
            const int32_t e = base + ln;
            const bool valid = e < end;
            int32_t w = 0;
            bool act = false, fresh = false;
            if (valid) {
                w = (pre && base == beg) ? w_first : a.col_idx[e];
                const double rw = r[w] + coef * v;
                r[w] = rw;
                const uint8_t f = fl[w];
                const int32_t dw = a.row_ptr[w + 1] - a.row_ptr[w];
                act = !(f & kQueued) && rw != 0.0 && fabs(rw) >= P.eps_eff * (double)dw;
                fresh = !(f & kTouched);
                if (act || fresh) fl[w] = (uint8_t)(f | kTouched | (act ? kQueued : 0));
            }
            const unsigned long long ma = __ballot(act), mt = __ballot(fresh);
            const unsigned long long below = lanemask_lt();
            if (act) {
                long long pos = head + count + __popcll(ma & below);
                if (pos >= n) pos -= n;
                q[pos] = w;
            }
            if (fresh) tl[nt + __popcll(mt & below)] = w;
            count += __popcll(ma);
            nt += __popcll(mt);
        }
        if (have) nw = nbeg + ln < nend ? a.col_idx[nbeg + ln] : 0;
        // u itself, after its row: no neighbour is u (simple graph), so its
        // residual is the ru lane 0 wrote and it is not queued (it was popped)
        int back = 0;
        if (ln == 0) {
            if (ru != 0.0 && fabs(ru) >= P.eps_eff * (double)du) {
                long long pos = head + count;
                if (pos >= n) pos -= n;
                q[pos] = u;
                fl[u] = (uint8_t)(kTouched | kQueued);
                back = 1;
            } else {
                fl[u] = kTouched;
            }
        }
        back = __shfl(back, 0);
        count += back;
        __threadfence_block();
        pops++;
        ops += du;
    }
    // residual norms over the touched nodes (reported scale), a fixed-shape reduction
    double l1 = 0.0, mx = 0.0;
    for (long long i = ln; i < nt; i += kWave) {
        const int32_t w = tl[i];
        const double av = fabs(r[w]) * P.rscale;
        l1 += av;
        const double d = (double)(a.row_ptr[w + 1] - a.row_ptr[w]);
        if (d > 0.0 && av / d > mx) mx = av / d;
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        l1 += __shfl_xor(l1, off);
        mx = fmax(mx, __shfl_xor(mx, off));
    }
    if (ln == 0) {
        FifoStat st;
        st.pops = pops;
        st.ops = ops;
        st.epochs = epochs + (pops > 0 ? 1 : 0);
        st.nt = nt;
        st.l1 = l1;
        st.dinf = mx;
        st.status = status;
        st.pad = 0;
        a.stat[qi] = st;
    }
}

// slot reset through the touched lists: one wavefront per slot
__global__ void __launch_bounds__(kFifoBlock) k_fifo_reset(FifoArgs a) {
    const int slot = (int)((blockIdx.x * (int64_t)kFifoBlock + threadIdx.x) / kWave);
    if (slot >= a.nslots || a.q0 + slot >= a.B) return;
    const long long nt = a.stat[a.q0 + slot].nt;
    const size_t off = (size_t)slot * a.n;
    for (long long i = lane(); i < nt; i += kWave) {
        const int32_t w = a.tl[off + i];
        a.r[off + w] = 0.0;
        a.x[off + w] = 0.0;
        a.fl[off + w] = 0;
    }
}

struct FifoWS {  // the buffers of one call
    void *r = nullptr, *x = nullptr;
    uint8_t *fl = nullptr;
    int32_t *q = nullptr, *tl = nullptr;
    int32_t *blk = nullptr;
    long long *total = nullptr;
    void *stage = nullptr;  // host results: values staged here (indices in the slot's free queue ring)
    void *xv = nullptr;     // FP32 results: the estimate rounded to the value type
};

__global__ void k_fifo_round(const double *__restrict__ x, float *xv, int64_t n) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x)
        xv[u] = (float)x[u];
}

template <typename V>
static int fifo_run(gde_ctx *ctx, const gde_graph *g, int32_t B, const gde_params *p, const gde_seed *sd,
                    gde_result *res, hipStream_t s) {
    const int64_t n = g->n;
    const size_t vs = sizeof(V);
    const size_t per_slot = (size_t)n * (8 + 8 + 1 + 4 + 4);
    // slots: every query at once when it fits in the budget, else rounds
    const size_t budget = (size_t)24 << 30;
    int32_t slots = (int32_t)std::max<int64_t>(1, std::min<int64_t>(B, (int64_t)(budget / std::max<size_t>(per_slot, 1))));
    FifoWS w;
    hipError_t e = hipMalloc(&w.r, 8 * (size_t)n * slots);
    if (e == hipSuccess) e = hipMalloc(&w.x, 8 * (size_t)n * slots);
    if (e == hipSuccess) e = hipMalloc((void **)&w.fl, (size_t)n * slots);
    if (e == hipSuccess) e = hipMalloc((void **)&w.q, 4 * (size_t)n * slots);
    if (e == hipSuccess) e = hipMalloc((void **)&w.tl, 4 * (size_t)n * slots);
    if (e == hipSuccess) e = hipMalloc((void **)&w.blk, 4 * (size_t)(dense_nblk(n) + 1));
    if (e == hipSuccess) e = hipMalloc((void **)&w.total, 8);
    bool host_out = false;
    for (int32_t i = 0; i < B; i++) host_out = host_out || !(p[i].flags & GDE_RESULT_DEVICE);
    if (e == hipSuccess && host_out) e = hipMalloc(&w.stage, vs * (size_t)std::max<int64_t>(n, 1));
    // FP32 results: the FP64 estimate is rounded into this buffer before compaction
    if (e == hipSuccess && vs == 4) e = hipMalloc(&w.xv, 4 * (size_t)std::max<int64_t>(n, 1));
    if (e == hipSuccess) e = hipMemsetAsync(w.r, 0, 8 * (size_t)n * slots, s);
    if (e == hipSuccess) e = hipMemsetAsync(w.x, 0, 8 * (size_t)n * slots, s);
    if (e == hipSuccess) e = hipMemsetAsync(w.fl, 0, (size_t)n * slots, s);
    // per-query parameters and seeds
    std::vector<FifoQuery> hq((size_t)B);
    std::vector<long long> hoff((size_t)B + 1, 0);
    for (int32_t i = 0; i < B; i++) {
        const bool ppr = p[i].kind == GDE_PPR;
        FifoQuery &fq = hq[i];
        fq.b = ppr ? p[i].alpha : 1.0;
        fq.w = ppr ? 1.0 - p[i].alpha : p[i].beta;
        fq.eps_eff = ppr ? p[i].alpha * p[i].eps : p[i].eps;
        fq.omega = p[i].omega == 0.0 ? 1.0 : p[i].omega;
        fq.rscale = ppr ? 1.0 / p[i].alpha : 1.0;
        fq.ppr = ppr ? 1 : 0;
        fq.pad = 0;
        fq.max_pops = (long long)std::max<int32_t>(p[i].max_iters, 1) * (long long)std::max<int64_t>(n, 1);
        hoff[i + 1] = hoff[i] + sd[i].nnz;
    }
    std::vector<int32_t> hidx((size_t)std::max<long long>(hoff[B], 1));
    std::vector<double> hval(hidx.size());
    for (int32_t i = 0; i < B; i++) {
        std::memcpy(hidx.data() + hoff[i], sd[i].idx, 4 * (size_t)sd[i].nnz);
        std::memcpy(hval.data() + hoff[i], sd[i].val, 8 * (size_t)sd[i].nnz);
    }
    FifoQuery *dq = nullptr;
    long long *doff = nullptr;
    int32_t *didx = nullptr;
    double *dval = nullptr;
    FifoStat *dst = nullptr;
    if (e == hipSuccess) e = hipMalloc((void **)&dq, sizeof(FifoQuery) * (size_t)B);
    if (e == hipSuccess) e = hipMalloc((void **)&doff, 8 * ((size_t)B + 1));
    if (e == hipSuccess) e = hipMalloc((void **)&didx, 4 * hidx.size());
    if (e == hipSuccess) e = hipMalloc((void **)&dval, 8 * hval.size());
    if (e == hipSuccess) e = hipMalloc((void **)&dst, sizeof(FifoStat) * (size_t)B);
    if (e == hipSuccess) e = hipMemcpyAsync(dq, hq.data(), sizeof(FifoQuery) * (size_t)B, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(doff, hoff.data(), 8 * ((size_t)B + 1), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(didx, hidx.data(), 4 * hidx.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dval, hval.data(), 8 * hval.size(), hipMemcpyHostToDevice, s);
    auto release = [&]() {
        void *ptrs[] = {w.r, w.x, w.fl, w.q, w.tl, w.blk, w.total, w.stage, w.xv, dq, doff, didx, dval, dst};
        for (void *v : ptrs)
            if (v) (void)hipFree(v);
    };
    if (e != hipSuccess) {
        release();
        return hip_fail(e, "LocalSOR workspace");
    }
    FifoArgs a{};
    a.n = (int32_t)n;
    a.row_ptr = g->row_ptr;
    a.col_idx = g->col_idx;
    a.r = (double *)w.r;
    a.x = (double *)w.x;
    a.fl = w.fl;
    a.q = w.q;
    a.tl = w.tl;
    a.nslots = slots;
    a.B = B;
    a.qp = dq;
    a.s_off = doff;
    a.s_idx = didx;
    a.s_val = dval;
    a.stat = dst;
    const unsigned grid = (unsigned)((slots * (int64_t)kWave + kFifoBlock - 1) / kFifoBlock);
    const int64_t nblk = dense_nblk(n);
    int first_err = GDE_OK;
    std::vector<FifoStat> hs((size_t)B);
    for (int32_t q0 = 0; q0 < B && first_err == GDE_OK; q0 += slots) {
        a.q0 = q0;
        if ((first_err = prof_mark(ctx, s))) break;
        hipLaunchKernelGGL(k_fifo, dim3(grid), dim3(kFifoBlock), 0, s, a);
        if ((first_err = prof_mark(ctx, s))) break;
        e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(hs.data() + q0, dst + q0, sizeof(FifoStat) * std::min(slots, B - q0),
                                                hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) { first_err = hip_fail(e, "LocalSOR kernel"); break; }
        // outputs, slot by slot: the nonzeros of the dense estimate in ascending order
        for (int32_t k = 0; k < slots && q0 + k < B && first_err == GDE_OK; k++) {
            const int32_t qi = q0 + k;
            const double *xk64 = (const double *)w.x + (size_t)k * n;
            const V *xk = (const V *)xk64;
            if (vs == 4) {
                hipLaunchKernelGGL(k_fifo_round, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256),
                                   0, s, xk64, (float *)w.xv, n);
                xk = (const V *)w.xv;
            }
            launch_dense_count<V>(xk, n, w.blk, s);
            launch_dense_scan(w.blk, nblk, w.total, s);
            long long nnz = 0;
            e = hipGetLastError();
            if (e == hipSuccess) e = hipMemcpyAsync(&nnz, w.total, 8, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) { first_err = hip_fail(e, "LocalSOR output"); break; }
            gde_result &rr = res[qi];
            const FifoStat &st = hs[qi];
            rr.nnz = nnz;
            rr.iters = (int32_t)st.epochs;
            rr.ops = st.ops;
            rr.pushes = st.pops;
            rr.residual_l1 = st.l1;
            rr.residual_dinf = st.dinf;
            rr.trace_len = 0;
            rr.trace_nodes_len = 0;
            if (!rr.idx || !rr.val || nnz > rr.capacity) {
                rr.status = GDE_ERR_CAPACITY;
                continue;
            }
            if (nnz > 0) {
                if (p[qi].flags & GDE_RESULT_DEVICE) {
                    launch_dense_emit<V>(xk, n, w.blk, (int32_t *)rr.idx, (V *)rr.val, s);
                    e = hipGetLastError();
                } else {
                    // indices staged in the slot's queue ring (free once its query is done)
                    int32_t *oi = w.q + (size_t)k * n;
                    launch_dense_emit<V>(xk, n, w.blk, oi, (V *)w.stage, s);
                    e = hipGetLastError();
                    if (e == hipSuccess) e = hipMemcpyAsync(rr.idx, oi, 4 * (size_t)nnz, hipMemcpyDeviceToHost, s);
                    if (e == hipSuccess)
                        e = hipMemcpyAsync(rr.val, w.stage, vs * (size_t)nnz, hipMemcpyDeviceToHost, s);
                    if (e == hipSuccess) e = hipStreamSynchronize(s);
                }
                if (e != hipSuccess) { first_err = hip_fail(e, "LocalSOR output"); break; }
            }
            rr.status = st.status;
        }
        if (first_err) break;
        hipLaunchKernelGGL(k_fifo_reset, dim3(grid), dim3(kFifoBlock), 0, s, a);
        e = hipGetLastError();
        if (e != hipSuccess) first_err = hip_fail(e, "LocalSOR reset");
    }
    if (first_err == GDE_OK) {
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) first_err = hip_fail(e, "LocalSOR");
    }
    if (first_err == GDE_OK) first_err = prof_collect(ctx, 0, 0);
    release();
    if (first_err) return first_err;
    int ret = GDE_OK;
    for (int32_t i = 0; i < B; i++)
        if (res[i].status != GDE_OK && ret == GDE_OK) ret = res[i].status;
    if (ret == GDE_ERR_CAPACITY) return fail(ret, "result capacity too small; result.nnz holds the size needed");
    if (ret == GDE_ERR_NOT_CONVERGED) return fail(ret, "the pop cap (max_iters * n) was reached");
    return ret;
}

int solve_fifo(gde_ctx *ctx, const gde_graph *g, int32_t B, const gde_params *p, const gde_seed *sd, gde_result *res,
               hipStream_t s) {
    if (p[0].value_type == GDE_F64) return fifo_run<double>(ctx, g, B, p, sd, res, s);
    return fifo_run<float>(ctx, g, B, p, sd, res, s);
}

}  // namespace gde
