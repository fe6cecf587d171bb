// gde_det.hip -- the deterministic mode of the plain solver (GDE_DETERMINISTIC).
//
// Every floating-point operation of an iteration happens in a fixed order, so
// two runs give bit-identical results.  The order is the sequential one of the
// local diffusion process read with the nodes of S_t in ascending id order
// (Eq. (9); Sec. 3.3 for LocalCH; the level push of Sec. 2 for the heat
// kernel): at every node w the updates arrive from the pushed nodes u in
// ascending u, and w's own change (r_w -= h_w) comes in at w's place in that
// order.  In FP64 this reproduces a sequential implementation of those steps
// bit for bit.
//
// An iteration is a pull instead of a scatter: a snapshot of S_t (values h_u,
// x_u += h_u), a marking pass over the rows of S_t that collects the nodes
// whose residual changes into a bitmap, and one wavefront per such node w
// that walks N(w) in CSR order (ascending, since rows are sorted), picks the
// members of S_t, and adds their contributions one after another.  No
// floating-point atomic is used anywhere; the residual norms are reduced in a
// fixed tree.  Bitmaps are compacted into ascending lists.  This mode is for
// checking and bisection, not speed: it reads every row of N(S_t) and
// synchronises with the host once per iteration.
//
// FP contraction is off in this file: a multiply and an add stay two
// roundings, as in the sequential reference arithmetic.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <vector>

#include "gde_det.h"
#include "gde_device.h"
#include "gde_kernels.h"

namespace gde {

constexpr int kDetBlock = 256;     // threads per workgroup of every kernel here
constexpr int kDetPullGrid = 4096; // workgroups of the pull (a wavefront per node, grid-stride)

struct DetWS {
    int64_t n = 0, nwords = 0, nblk = 0;
    void *sv[2] = {nullptr, nullptr};    // V[n]: h_u of the nodes of S_t (parity t & 1)
    uint32_t *sbm[2] = {nullptr, nullptr};  // S_t bitmaps by parity (S_{t-1}: LocalCH momentum support)
    uint32_t *ubm = nullptr;             // nodes whose residual changes in this iteration
    uint32_t *nbm = nullptr;             // S_{t+1} being found
    uint32_t *tbm2 = nullptr;            // heat kernel: touched bitmap of the odd levels
    int32_t *blk = nullptr;              // compaction: per-workgroup counts, then offsets
    double *part = nullptr;              // norm partials: [nblk] l1, then [nblk] max
    long long *cnt = nullptr;            // [0] list length of the last compaction, [1] S_{t+1} length
    double *nrm = nullptr;               // [2] reduced l1 and max
    long long *h_cnt = nullptr;          // pinned host mirror: [0..1] counts; doubles follow
};

void det_ws_free(DetWS *d) {
    if (!d) return;
    void *p[] = {d->sv[0], d->sv[1], d->sbm[0], d->sbm[1], d->ubm, d->nbm, d->tbm2, d->blk, d->part, d->cnt, d->nrm};
    for (void *q : p)
        if (q) (void)hipFree(q);
    if (d->h_cnt) (void)hipHostFree(d->h_cnt);
    delete d;
}

static int det_ws_get(Workspace *w, hipStream_t s, DetWS **out) {
    if (w->det) { *out = w->det; return GDE_OK; }
    DetWS *d = new DetWS();
    d->n = w->n;
    d->nwords = (w->n + 31) / 32;
    d->nblk = (d->nwords + kDetBlock - 1) / kDetBlock;
    auto al = [&](void **pp, size_t bytes) -> hipError_t {
        hipError_t e = hipMalloc(pp, bytes);
        if (e == hipSuccess) e = hipMemsetAsync(*pp, 0, bytes, s);
        return e;
    };
    hipError_t e = hipSuccess;
    for (int i = 0; i < 2 && e == hipSuccess; i++) e = al(&d->sv[i], w->vsize * (size_t)w->n);
    for (int i = 0; i < 2 && e == hipSuccess; i++) e = al((void **)&d->sbm[i], 4 * (size_t)d->nwords);
    if (e == hipSuccess) e = al((void **)&d->ubm, 4 * (size_t)d->nwords);
    if (e == hipSuccess) e = al((void **)&d->nbm, 4 * (size_t)d->nwords);
    if (e == hipSuccess) e = al((void **)&d->tbm2, 4 * (size_t)d->nwords);
    if (e == hipSuccess) e = al((void **)&d->blk, 4 * (size_t)(d->nblk + 1));
    if (e == hipSuccess) e = al((void **)&d->part, 16 * (size_t)d->nblk);
    if (e == hipSuccess) e = al((void **)&d->cnt, 32);
    if (e == hipSuccess) e = al((void **)&d->nrm, 16);
    if (e == hipSuccess) e = hipHostMalloc((void **)&d->h_cnt, 64, 0);
    if (e != hipSuccess) {
        det_ws_free(d);
        return hip_fail(e, "deterministic workspace");
    }
    w->det = d;
    *out = d;
    return GDE_OK;
}

__device__ __forceinline__ bool bm_test(const uint32_t *bm, int32_t u) { return (bm[u >> 5] >> (u & 31)) & 1u; }
__device__ __forceinline__ void bm_set(uint32_t *bm, int32_t u) {
    const uint32_t bit = 1u << (u & 31);
    if (!(bm[u >> 5] & bit)) atomicOr(&bm[u >> 5], bit);
}

// ------------------------------------------------------------------ bitmap -> ascending list
__global__ void __launch_bounds__(kDetBlock) k_det_bm_count(const uint32_t *__restrict__ bm, int64_t nwords,
                                                            int32_t *blk) {
    __shared__ int s[kDetBlock / kWave];
    const int64_t i = blockIdx.x * (int64_t)kDetBlock + threadIdx.x;
    int c = i < nwords ? __popc(bm[i]) : 0;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if (lane() == 0) s[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int a = 0;
        for (int k = 0; k < kDetBlock / kWave; k++) a += s[k];
        blk[blockIdx.x] = a;
    }
}

// one workgroup: exclusive scan of blk[0..nblk) in place, the total into *total
__global__ void __launch_bounds__(1024) k_det_bm_scan(int32_t *blk, int64_t nblk, long long *total) {
    __shared__ long long s[1024];
    const int64_t per = (nblk + 1023) / 1024;
    const int64_t lo = threadIdx.x * per;
    const int64_t hi = lo + per < nblk ? lo + per : nblk;
    long long a = 0;
    for (int64_t i = lo; i < hi; i++) a += blk[i];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const long long y = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += y;
        __syncthreads();
    }
    long long run = s[threadIdx.x] - a;
    for (int64_t i = lo; i < hi; i++) {
        const int32_t v = blk[i];
        blk[i] = (int32_t)run;
        run += v;
    }
    if (threadIdx.x == 1023) *total = s[1023];
}

// writes the set bits in ascending order at the scanned offsets and clears the words
__global__ void __launch_bounds__(kDetBlock) k_det_bm_emit(uint32_t *bm, int64_t nwords,
                                                           const int32_t *__restrict__ blk, int32_t *list) {
    __shared__ int s[kDetBlock];
    const int64_t i = blockIdx.x * (int64_t)kDetBlock + threadIdx.x;
    uint32_t m = i < nwords ? bm[i] : 0u;
    const int c = __popc(m);
    s[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < kDetBlock; off <<= 1) {
        const int y = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += y;
        __syncthreads();
    }
    int pos = blk[blockIdx.x] + s[threadIdx.x] - c;
    if (m) {
        bm[i] = 0u;
        while (m) {
            const int b = __ffs((int)m) - 1;
            m &= m - 1u;
            list[pos++] = (int32_t)(i * 32 + b);
        }
    }
}

// ------------------------------------------------------------------ snapshot of S_t
// mode 0: LocalGD / LocalCH (r untouched here; the pull applies r_u -= h_u),
// mode 1: heat-kernel level (r_k[u] = 0 now; the pull fills the next plane).
// h = r_u (LocalGD, first LocalCH step, heat kernel) or c r_u + m Delta_u with
// Delta_u = h_u of the previous iteration if u was in S_{t-1}, else 0.
template <typename V>
__global__ void __launch_bounds__(kDetBlock)
    k_det_snap(const int32_t *__restrict__ S, int64_t ns, RD<V> *rd, V *x, uint32_t *pushed, V *sv_cur,
               uint32_t *sbm_cur, const V *__restrict__ sv_prev, const uint32_t *__restrict__ sbm_prev, int use_ch,
               V c, V m, int mode, DevState *st, long long *tr_size, long long *tr_vol, int t, long long tr_cap,
               int32_t *tr_nodes, long long tr_ncap, long long node_base) {
    const int64_t i = blockIdx.x * (int64_t)kDetBlock + threadIdx.x;
    long long vol = 0, cnt = 0;
    if (i < ns) {
        const int32_t u = S[i];
        const RD<V> e = rd[u];
        V h = e.r;
        if (use_ch) {
            const V dlt = bm_test(sbm_prev, u) ? sv_prev[u] : (V)0;
            h = c * e.r + m * dlt;
        }
        sv_cur[u] = h;
        atomicOr(&sbm_cur[u >> 5], 1u << (u & 31));
        atomicOr(&pushed[u >> 5], 1u << (u & 31));
        x[u] = x[u] + h;
        if (mode == 1) rd[u].r = (V)0;
        vol = (long long)e.d;
        cnt = 1;
        if (tr_nodes && node_base + i < tr_ncap) tr_nodes[node_base + i] = u;
    }
    // integer totals: any order gives the same sums
    for (int off = kWave / 2; off > 0; off >>= 1) {
        vol += __shfl_xor(vol, off);
        cnt += __shfl_xor(cnt, off);
    }
    if (lane() == 0 && cnt > 0) {
        atomicAdd((unsigned long long *)&st->ops, (unsigned long long)vol);
        atomicAdd((unsigned long long *)&st->pushes, (unsigned long long)cnt);
        if (tr_size && t < tr_cap) {
            atomicAdd((unsigned long long *)&tr_size[t], (unsigned long long)cnt);
            atomicAdd((unsigned long long *)&tr_vol[t], (unsigned long long)vol);
        }
    }
}

// marks N(u) for every u in S_t in the update bitmap (and u itself when self)
// and in the touched bitmap; one wavefront per node of S_t
__global__ void __launch_bounds__(kDetBlock)
    k_det_mark(const int32_t *__restrict__ S, int64_t ns, const int32_t *__restrict__ row_ptr,
               const int32_t *__restrict__ col_idx, uint32_t *ubm, uint32_t *tbm, int self) {
    const int64_t wid = (blockIdx.x * (int64_t)kDetBlock + threadIdx.x) / kWave;
    const int64_t nw = (int64_t)gridDim.x * kDetBlock / kWave;
    for (int64_t i = wid; i < ns; i += nw) {
        const int32_t u = S[i];
        if (self && lane() == 0) bm_set(ubm, u);
        const int32_t beg = row_ptr[u], end = row_ptr[u + 1];
        for (int32_t e = beg + lane(); e < end; e += kWave) {
            const int32_t w = col_idx[e];
            bm_set(ubm, w);
            bm_set(tbm, w);
        }
    }
}

// ------------------------------------------------------------------ the pull
// One wavefront per node w of U (the nodes whose residual changes): walks N(w)
// in CSR order in chunks of 64, each lane computing the contribution of one
// neighbour u in S_t (PPR: ((1-alpha)/d_u) h_u; Katz: beta h_u; heat kernel:
// ((tau/(k+1)) h_u) / d_u), and then every lane adds the chunk's contributions
// to r_w one after another in ascending u, with w's own -h_w at its place.
// The new r_w is tested against its threshold (|r| >= eps_eff d_w, r != 0).
template <typename V>
__global__ void __launch_bounds__(kDetBlock)
    k_det_pull(const int32_t *__restrict__ U, const long long *__restrict__ nu_ptr,
               const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col_idx,
               const RD<V> *__restrict__ src, RD<V> *dst, const V *__restrict__ sv,
               const uint32_t *__restrict__ sbm, int mode, V wscale, int w_div_deg, V eps_eff, uint32_t *nbm) {
    const long long nu = *nu_ptr;
    const int64_t wid = (blockIdx.x * (int64_t)kDetBlock + threadIdx.x) / kWave;
    const int64_t nw = (int64_t)gridDim.x * kDetBlock / kWave;
    for (int64_t i = wid; i < nu; i += nw) {
        const int32_t w = U[i];
        const int32_t beg = row_ptr[w], end = row_ptr[w + 1];
        V r = dst[w].r;
        bool pending = mode == 0 && bm_test(sbm, w);
        const V hw = pending ? sv[w] : (V)0;
        for (int32_t base = beg; base < end; base += kWave) {
            const int32_t e = base + lane();
            const bool valid = e < end;
            const int32_t u = valid ? col_idx[e] : INT_MAX;
            const bool in = valid && bm_test(sbm, u);
            V cu = (V)0;
            if (in) {
                const V hu = sv[u];
                if (mode == 0) {
                    const V wu = w_div_deg ? wscale / src[u].d : wscale;
                    cu = wu * hu;
                } else {
                    cu = (wscale * hu) / src[u].d;
                }
            }
            const unsigned long long inm = __ballot(in);
            const unsigned long long gt = __ballot(valid && u > w);
            const int kself = (pending && gt) ? __ffsll((long long)gt) - 1 : kWave;
            unsigned long long lo = kself >= kWave ? inm : (inm & ((1ull << kself) - 1ull));
            unsigned long long hi = inm & ~lo;
            while (lo) {
                const int k = __ffsll((long long)lo) - 1;
                lo &= lo - 1ull;
                r = r + __shfl(cu, k);
            }
            if (kself < kWave) {
                r = r - hw;
                pending = false;
            }
            while (hi) {
                const int k = __ffsll((long long)hi) - 1;
                hi &= hi - 1ull;
                r = r + __shfl(cu, k);
            }
        }
        if (pending) r = r - hw;
        if (lane() == 0) {
            dst[w].r = r;
            if (r != (V)0 && fabs(r) >= eps_eff * dst[w].d) atomicOr(&nbm[w >> 5], 1u << (w & 31));
        }
    }
}

// ------------------------------------------------------------------ residual norms
// Over the nodes of a touched bitmap, in a fixed shape: each thread one word
// (its nodes in ascending order), a fixed tree per workgroup, then one
// workgroup over the partials.  The residuals and the bitmap are cleared.
template <typename V>
__global__ void __launch_bounds__(kDetBlock) k_det_norm_part(uint32_t *bm, int64_t nwords, RD<V> *rd, double rscale,
                                                             double *part, int64_t nblk, int clear) {
    __shared__ double s_l1[kDetBlock], s_mx[kDetBlock];
    const int64_t i = blockIdx.x * (int64_t)kDetBlock + threadIdx.x;
    double l1 = 0.0, mx = 0.0;
    if (i < nwords) {
        uint32_t m = bm[i];
        if (m) {
            if (clear) bm[i] = 0u;
            while (m) {
                const int b = __ffs((int)m) - 1;
                m &= m - 1u;
                const int64_t w = i * 32 + b;
                const RD<V> e = rd[w];
                if (clear) rd[w].r = (V)0;
                const double a = fabs((double)e.r) * rscale;
                l1 = l1 + a;
                const double dd = (double)e.d;
                if (dd > 0.0 && a / dd > mx) mx = a / dd;
            }
        }
    }
    s_l1[threadIdx.x] = l1;
    s_mx[threadIdx.x] = mx;
    __syncthreads();
    for (int off = kDetBlock / 2; off > 0; off >>= 1) {
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

__global__ void __launch_bounds__(kDetBlock) k_det_norm_final(const double *__restrict__ part, int64_t nblk,
                                                              double *nrm) {
    __shared__ double s_l1[kDetBlock], s_mx[kDetBlock];
    double l1 = 0.0, mx = 0.0;
    for (int64_t j = threadIdx.x; j < nblk; j += kDetBlock) {
        l1 = l1 + part[j];
        mx = fmax(mx, part[nblk + j]);
    }
    s_l1[threadIdx.x] = l1;
    s_mx[threadIdx.x] = mx;
    __syncthreads();
    for (int off = kDetBlock / 2; off > 0; off >>= 1) {
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

__global__ void k_det_finish(DevState *st, int32_t iters, const double *nrm, int from_nrm, double l1, double mx) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->iters = iters;
        const double a = from_nrm ? nrm[0] : l1;
        const double m = from_nrm ? nrm[1] : mx;
        st->res_l1 = a;
        st->res_dinf = (unsigned long long)__double_as_longlong(m);
    }
}

// ------------------------------------------------------------------ host driver
static inline unsigned grid_of(int64_t items, int per) { return (unsigned)std::max<int64_t>(1, (items + per - 1) / per); }

// bitmap -> ascending list; the length lands in d->cnt[slot]
static void det_compact(DetWS *d, uint32_t *bm, int32_t *list, int slot, hipStream_t s) {
    hipLaunchKernelGGL(k_det_bm_count, dim3((unsigned)d->nblk), dim3(kDetBlock), 0, s, bm, d->nwords, d->blk);
    hipLaunchKernelGGL(k_det_bm_scan, dim3(1), dim3(1024), 0, s, d->blk, d->nblk, d->cnt + slot);
    hipLaunchKernelGGL(k_det_bm_emit, dim3((unsigned)d->nblk), dim3(kDetBlock), 0, s, bm, d->nwords, d->blk, list);
}

template <typename V>
static void det_norms(DetWS *d, uint32_t *bm, void *rd, double rscale, hipStream_t s, int clear = 1) {
    hipLaunchKernelGGL(k_det_norm_part<V>, dim3((unsigned)d->nblk), dim3(kDetBlock), 0, s, bm, d->nwords,
                       (RD<V> *)rd, rscale, d->part, d->nblk, clear);
    hipLaunchKernelGGL(k_det_norm_final, dim3(1), dim3(kDetBlock), 0, s, d->part, d->nblk, d->nrm);
}

template <typename V>
static int det_gd_ch_loop(const gde_graph *g, const gde_params *p, Workspace *w, DetWS *d, long long ns,
                          long long *d_trs, long long *d_trv, int32_t *d_trn, long long tr_cap, long long tr_ncap,
                          hipStream_t s, int32_t *T_out, bool *converged);

template <typename V>
int det_run(const gde_graph *g, const gde_params *p, const gde_seed *sd, Workspace *w, const SeedInline *inl,
            long long *d_trs, long long *d_trv, int32_t *d_trn, long long tr_cap, long long tr_ncap, hipStream_t s,
            bool *converged) {
    DetWS *d = nullptr;
    int rc = det_ws_get(w, s, &d);
    if (rc) return rc;
    const size_t bmb = 4 * (size_t)d->nwords;
    int32_t *S = w->front[0];
    int32_t *U = w->front[1];
    const unsigned pull_grid = kDetPullGrid;
    long long ns = sd->nnz, base = 0;
    int32_t T = 0;
    *converged = false;
    GDE_HIP(hipMemsetAsync(d->sbm[0], 0, bmb, s));
    GDE_HIP(hipMemsetAsync(d->sbm[1], 0, bmb, s));
    // the snapshot adds each iteration's counts into the trace
    if (d_trs) GDE_HIP(hipMemsetAsync(d_trs, 0, 8 * (size_t)tr_cap, s));
    if (d_trv) GDE_HIP(hipMemsetAsync(d_trv, 0, 8 * (size_t)tr_cap, s));

    if (p->kind == GDE_HK || p->kind == GDE_SERIES) {
        const int K = p->K;
        const LevelSeries ls = level_series(p);
        const std::vector<double> &psi = ls.psi;
        void *plane[2] = {w->rd, w->rd2};
        uint32_t *tb[2] = {w->tbm, d->tbm2};
        launch_seed_init<V>(w->rd, w->seed_idx, w->seed_val, inl, sd->nnz, ls.c0, S, nullptr, nullptr, 0, tb[0],
                            w->st, s);
        double left_l1 = 0.0, left_dinf = 0.0;
        bool stopped = false;
        for (int k = 0; k <= K; k++) {
            if (stopped) ns = 0;
            const int cur = k & 1, nxt = cur ^ 1;
            long long ns_next = 0;
            if (ns > 0) {
                GDE_HIP(hipMemsetAsync(d->sbm[0], 0, bmb, s));
                hipLaunchKernelGGL(k_det_snap<V>, dim3(grid_of(ns, kDetBlock)), dim3(kDetBlock), 0, s, S, (int64_t)ns,
                                   (RD<V> *)plane[cur], (V *)w->x, w->bitmap, (V *)d->sv[0], d->sbm[0],
                                   (const V *)nullptr, (const uint32_t *)nullptr, 0, (V)0, (V)0, 1, w->st, d_trs,
                                   d_trv, T, tr_cap, d_trn, tr_ncap, base);
                if (k < K) {
                    hipLaunchKernelGGL(k_det_mark, dim3(grid_of(ns * kWave, kDetBlock)), dim3(kDetBlock), 0, s, S,
                                       (int64_t)ns, g->row_ptr, g->col_idx, d->ubm, tb[nxt], 0);
                    det_compact(d, d->ubm, U, 0, s);
                    const double eps_next = p->eps / ((double)(K + 1) * psi[k + 1]);
                    hipLaunchKernelGGL(k_det_pull<V>, dim3(pull_grid), dim3(kDetBlock), 0, s, U, d->cnt + 0,
                                       g->row_ptr, g->col_idx, (const RD<V> *)plane[cur], (RD<V> *)plane[nxt],
                                       (const V *)d->sv[0], d->sbm[0], 1, (V)ls.ratio[k], 1,
                                       (V)eps_next, d->nbm);
                    det_compact(d, d->nbm, S, 1, s);
                }
                GDE_HIP(hipGetLastError());
                T++;
                base += ns;
            } else {
                stopped = true;
            }
            // leftover of level k: psi_k ||r_k||_1 and (K+1) psi_k ||D^-1 r_k||_inf
            det_norms<V>(d, tb[cur], plane[cur], 1.0, s);
            GDE_HIP(hipGetLastError());
            GDE_HIP(hipMemcpyAsync(d->h_cnt, d->cnt, 16, hipMemcpyDeviceToHost, s));
            GDE_HIP(hipMemcpyAsync(d->h_cnt + 2, d->nrm, 16, hipMemcpyDeviceToHost, s));
            GDE_HIP(hipStreamSynchronize(s));
            double nv[2];
            std::memcpy(nv, d->h_cnt + 2, 16);
            left_l1 += psi[k] * nv[0];
            const double wd = (double)(K + 1) * psi[k] * nv[1];
            if (wd > left_dinf) left_dinf = wd;
            ns_next = (ns > 0 && k < K) ? d->h_cnt[1] : 0;
            if (ns > 0 && k == K) ns_next = 0;
            if (!stopped && ns_next == 0 && k < K) stopped = true;
            ns = ns_next;
        }
        hipLaunchKernelGGL(k_det_finish, dim3(1), dim3(1), 0, s, w->st, T, (const double *)nullptr, 0, left_l1,
                           left_dinf);
        GDE_HIP(hipGetLastError());
        *converged = true;
        return GDE_OK;
    }

    // PPR / Katz, LocalGD or LocalCH
    const bool ppr = p->kind == GDE_PPR;
    launch_seed_init<V>(w->rd, w->seed_idx, w->seed_val, inl, sd->nnz, ppr ? p->alpha : 1.0, S, nullptr, nullptr, 0,
                        w->tbm, w->st, s);
    if ((rc = det_gd_ch_loop<V>(g, p, w, d, ns, d_trs, d_trv, d_trn, tr_cap, tr_ncap, s, &T, converged))) return rc;
    det_norms<V>(d, w->tbm, w->rd, ppr ? 1.0 / p->alpha : 1.0, s);
    hipLaunchKernelGGL(k_det_finish, dim3(1), dim3(1), 0, s, w->st, T, (const double *)d->nrm, 1, 0.0, 0.0);
    if (p->kind == GDE_KATZ && (p->flags & GDE_KATZ_SUBTRACT_SEED))
        launch_subtract_seed<V>(w->x, w->seed_idx, w->seed_val, sd->nnz, s);
    GDE_HIP(hipGetLastError());
    // a run that stopped at the iteration cap leaves its S_{t+1} bits cleared by
    // the compaction; the S_t bitmaps are cleared at the next solve's start
    return GDE_OK;
}

// The LocalGD / LocalCH iterations from the ns nodes in w->front[0] (S_0), on
// w's residual/degree plane, estimate, pushed set and touched bitmap.
template <typename V>
static int det_gd_ch_loop(const gde_graph *g, const gde_params *p, Workspace *w, DetWS *d, long long ns,
                          long long *d_trs, long long *d_trv, int32_t *d_trn, long long tr_cap, long long tr_ncap,
                          hipStream_t s, int32_t *T_out, bool *converged) {
    const size_t bmb = 4 * (size_t)d->nwords;
    int32_t *S = w->front[0];
    int32_t *U = w->front[1];
    const unsigned pull_grid = kDetPullGrid;
    long long base = 0;
    int32_t T = 0;
    *converged = false;
    const bool ppr = p->kind == GDE_PPR;
    const bool ch = p->method == GDE_LOCAL_CH;
    const V wscale = (V)(ppr ? 1.0 - p->alpha : p->beta);
    const V eps_eff = (V)(ppr ? p->alpha * p->eps : p->eps);
    double sigma = 1.0, dlt = 0.0;
    if (ch) {
        double mu, L;
        if (ppr) { mu = p->alpha; L = 2.0 - p->alpha; }
        else { mu = 1.0 - p->beta * p->lambda_bound; L = 1.0 + p->beta * p->lambda_bound; }
        sigma = (L + mu) / (L - mu);
        dlt = 1.0 / sigma;
    }
    for (int t = 0;; t++) {
        if (ns == 0) { *converged = true; break; }
        if (t >= p->max_iters) break;
        const int cur = t & 1, prv = cur ^ 1;
        V c = (V)1, m = (V)0;
        if (ch && t > 0) {
            const double dnext = 1.0 / (2.0 * sigma - dlt);
            c = (V)(2.0 * sigma * dnext);
            m = (V)(dlt * dnext);
            dlt = dnext;
        }
        GDE_HIP(hipMemsetAsync(d->sbm[cur], 0, bmb, s));
        hipLaunchKernelGGL(k_det_snap<V>, dim3(grid_of(ns, kDetBlock)), dim3(kDetBlock), 0, s, S, (int64_t)ns,
                           (RD<V> *)w->rd, (V *)w->x, w->bitmap, (V *)d->sv[cur], d->sbm[cur], (const V *)d->sv[prv],
                           (const uint32_t *)d->sbm[prv], (ch && t > 0) ? 1 : 0, c, m, 0, w->st, d_trs, d_trv, t,
                           tr_cap, d_trn, tr_ncap, base);
        hipLaunchKernelGGL(k_det_mark, dim3(grid_of(ns * kWave, kDetBlock)), dim3(kDetBlock), 0, s, S, (int64_t)ns,
                           g->row_ptr, g->col_idx, d->ubm, w->tbm, 1);
        det_compact(d, d->ubm, U, 0, s);
        hipLaunchKernelGGL(k_det_pull<V>, dim3(pull_grid), dim3(kDetBlock), 0, s, U, d->cnt + 0, g->row_ptr,
                           g->col_idx, (const RD<V> *)w->rd, (RD<V> *)w->rd, (const V *)d->sv[cur], d->sbm[cur], 0,
                           wscale, ppr ? 1 : 0, eps_eff, d->nbm);
        det_compact(d, d->nbm, S, 1, s);
        GDE_HIP(hipGetLastError());
        GDE_HIP(hipMemcpyAsync(d->h_cnt, d->cnt, 16, hipMemcpyDeviceToHost, s));
        GDE_HIP(hipStreamSynchronize(s));
        T++;
        base += ns;
        ns = d->h_cnt[1];
    }
    *T_out = T;
    return GDE_OK;
}

// S_0 of a warm start: the nodes of the touched bitmap whose residual is active
template <typename V>
__global__ void __launch_bounds__(kDetBlock) k_det_select(const uint32_t *__restrict__ tbm, int64_t nwords,
                                                          const RD<V> *__restrict__ rd, V eps_eff, uint32_t *nbm) {
    const int64_t i = blockIdx.x * (int64_t)kDetBlock + threadIdx.x;
    if (i >= nwords) return;
    uint32_t m = tbm[i], out = 0u;
    while (m) {
        const int b = __ffs((int)m) - 1;
        m &= m - 1u;
        const RD<V> e = rd[i * 32 + b];
        if (e.r != (V)0 && fabs(e.r) >= eps_eff * e.d) out |= 1u << b;
    }
    nbm[i] = out;
}

template <typename V>
int det_warm(const gde_graph *g, const gde_params *p, Workspace *w, hipStream_t s, const int32_t *forced,
             int32_t nforced, int32_t *T, bool *converged) {
    DetWS *d = nullptr;
    int rc = det_ws_get(w, s, &d);
    if (rc) return rc;
    const bool ppr = p->kind == GDE_PPR;
    const V eps_eff = (V)(ppr ? p->alpha * p->eps : p->eps);
    const size_t bmb = 4 * (size_t)d->nwords;
    GDE_HIP(hipMemsetAsync(d->sbm[0], 0, bmb, s));
    GDE_HIP(hipMemsetAsync(d->sbm[1], 0, bmb, s));
    GDE_HIP(hipMemsetAsync(w->st, 0, sizeof(DevState), s));
    long long ns = 0;
    if (forced) {  // a given S_0 (ascending ids), e.g. supp(s) of a first solve (Definition 3.1)
        if (nforced > 0)
            GDE_HIP(hipMemcpyAsync(w->front[0], forced, 4 * (size_t)nforced, hipMemcpyHostToDevice, s));
        GDE_HIP(hipStreamSynchronize(s));
        ns = nforced;
    } else {
        hipLaunchKernelGGL(k_det_select<V>, dim3((unsigned)d->nblk), dim3(kDetBlock), 0, s, w->tbm, d->nwords,
                           (const RD<V> *)w->rd, eps_eff, d->nbm);
        det_compact(d, d->nbm, w->front[0], 1, s);
        GDE_HIP(hipGetLastError());
        GDE_HIP(hipMemcpyAsync(d->h_cnt, d->cnt, 16, hipMemcpyDeviceToHost, s));
        GDE_HIP(hipStreamSynchronize(s));
        ns = d->h_cnt[1];
    }
    if ((rc = det_gd_ch_loop<V>(g, p, w, d, ns, nullptr, nullptr, nullptr, 0, 0, s, T, converged))) return rc;
    det_norms<V>(d, w->tbm, w->rd, ppr ? 1.0 / p->alpha : 1.0, s, 0);
    hipLaunchKernelGGL(k_det_finish, dim3(1), dim3(1), 0, s, w->st, *T, (const double *)d->nrm, 1, 0.0, 0.0);
    GDE_HIP(hipGetLastError());
    return GDE_OK;
}

template int det_warm<float>(const gde_graph *, const gde_params *, Workspace *, hipStream_t, const int32_t *,
                             int32_t, int32_t *, bool *);
template int det_warm<double>(const gde_graph *, const gde_params *, Workspace *, hipStream_t, const int32_t *,
                              int32_t, int32_t *, bool *);

template int det_run<float>(const gde_graph *, const gde_params *, const gde_seed *, Workspace *, const SeedInline *,
                            long long *, long long *, int32_t *, long long, long long, hipStream_t, bool *);
template int det_run<double>(const gde_graph *, const gde_params *, const gde_seed *, Workspace *,
                             const SeedInline *, long long *, long long *, int32_t *, long long, long long, hipStream_t,
                             bool *);

}  // namespace gde
