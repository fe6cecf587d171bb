// gde_batch_kernels.hip -- batched LocalGD (PPR / Katz) for many queries at once.
//
// Queries are packed as lanes of node-major residual tiles: group g holds
// R[g][u][0..L) and X[g][u][0..L), so the L values of one node share a cache
// line.  Per iteration t (Eq. (9) for every lane, Definition 3.1):
//   snap : over the active (group, node) pairs, the lanes whose residual
//          crossed their own threshold are snapshot (v = r, r = 0, x += v) by
//          L threads per pair (one coalesced line access); each pair reserves
//          deg * c "lane-edges" (c = active lanes); the reservations of a
//          workgroup are summed and taken with one 64-bit atomic;
//   push : lane-edges are spread evenly over the grid in LDS-staged tiles; the
//          c threads of one edge update c residuals of the same line.  A
//          returned old value that crosses theta_lane * d_w sets the lane's bit
//          in the pair's next-mask; the first bit appends the pair to the next
//          active list.  A returned zero marks the pair as touched (the
//          residual clean-up at the end reads only touched pairs).  List
//          appends are aggregated per workgroup and tile (one counter atomic).
// Touched lists.  Batched solves (LT = true) record touched (lane, node)
// entries with no extra memory access: a snapshot leaves -0.0 where it took a
// residual, so a returned old value of +0.0 (bit pattern 0) means the lane has
// never held a residual in this solve, and each (lane, node) is listed exactly
// once (the seeds by the seed kernel).  The serving engine (LT = false) keeps
// per-group tags TM, because its groups change occupants between steps.
#include <hip/hip_runtime.h>

#include "gde_batch_kernels.h"
#include "gde_device.h"

namespace gde {

__device__ __forceinline__ int blane() { return (int)__lane_id(); }

__device__ __forceinline__ int bwave_append64(bool pred, int32_t *counter, uint64_t val, uint64_t *list, int32_t cap,
                                              int32_t *ovf) {
    unsigned long long mask = __ballot(pred);
    if (mask == 0ull) return -1;
    int leader = __ffsll((long long)mask) - 1;
    int base = 0;
    if (blane() == leader) base = atomicAdd(counter, (int)__popcll(mask));
    base = __shfl(base, leader);
    if (pred) {
        int s = base + (int)__popcll(mask & ((1ull << blane()) - 1ull));
        if (s < cap) list[s] = val;
        else *ovf = 1;
        return s;
    }
    return -1;
}

template <typename V>
__device__ __forceinline__ V batomic_take(V *p);
template <>
__device__ __forceinline__ float batomic_take<float>(float *p) { return atomicExch(p, 0.0f); }
template <>
__device__ __forceinline__ double batomic_take<double>(double *p) {
    return __longlong_as_double((long long)atomicExch((unsigned long long *)p, 0ull));
}

constexpr unsigned long long kLaneEdgeMask = (1ull << 40) - 1ull;

// ------------------------------------------------------------------ phase S
template <typename V>
__device__ __forceinline__ bool pos_zero(V v);
template <>
__device__ __forceinline__ bool pos_zero<float>(float v) { return __float_as_uint(v) == 0u; }
template <>
__device__ __forceinline__ bool pos_zero<double>(double v) { return __double_as_longlong(v) == 0ll; }

template <typename V, int L, bool LT>
__device__ void batch_snap(const BatchArgs<V> &a, int t, int bid, int nblocks) {
    BatchDev *st = a.st;
    const int cur = t & 1, nxt = cur ^ 1;
    const int nact = min(st->acount[cur], a.act_cap);
    V *Rs = (a.R2 && (t & 1)) ? a.R2 : a.R;  // the residual plane of this level
    if (bid == 0 && threadIdx.x == 0) {
        st->packed[nxt] = 0ull;
        st->acount[nxt] = 0;
        st->rowpack[nxt] = 0ull;
        // level push: push(t) lists the entries of level t + 1; that list last
        // held level t - 1, whose harvest has run
        if (a.R2) *(nxt ? &st->tcount2 : &st->tcount) = 0;
    }
    int32_t *ovf = &st->ovf[cur];
    if (nact > a.wl_cap) {  // one work-list entry per active pair: refuse rather than wrap
        if (bid == 0 && threadIdx.x == 0) *ovf = 1;
        return;
    }
    // one thread per active (group, node) pair for the masks and the reservation;
    // then the wavefront spreads its pairs' pushed lanes over its 64 lanes (a pair
    // has one active lane on a batch of unrelated queries and up to L on one of
    // overlapping queries, so neither a thread per pair nor a thread per lane
    // keeps the wavefront busy in both cases)
    constexpr uint32_t kAll = (L == 32) ? 0xffffffffu : ((1u << L) - 1u);
    __shared__ uint32_t s_pm[kBatchSnapBlock];  // candidate mode: the lanes that pass, per pair
    // workgroup-uniform trip count: every thread takes part in each reservation
    for (int bbase = bid * (int)blockDim.x; bbase < nact; bbase += nblocks * (int)blockDim.x) {
        const int i = bbase + (int)threadIdx.x;
        const bool valid = i < nact;
        int32_t g = 0, u = 0, beg = 0, deg = 0;
        uint32_t m = 0u, pm = 0u, prev = 0u;
        int mode = 0;
        if (valid) {
            const uint64_t p = a.act[cur][i];
            g = (int32_t)(p >> 32);
            u = (int32_t)(p & 0xffffffffull);
            uint32_t *nm = &a.NM[(size_t)u * a.G + g];
            m = *nm & kAll;
            *nm = 0u;  // each pair is listed once
            mode = a.g_mode ? a.g_mode[g] : ((a.w_div_deg ? 1 : 0) | ((a.ch && !a.force) || a.sgn ? 2 : 0));
            beg = a.row_ptr[u];
            deg = a.row_ptr[u + 1] - beg;
        }
        // candidate mode: the threshold decides, lane by lane, the wavefront's
        // candidate lanes spread over its 64 lanes as in the pushes below
        s_pm[threadIdx.x] = 0u;
        {
            const int cm = (valid && (mode & 2)) ? __popc(m) : 0;
            const int cincl = (int)wave_incl_scan64((unsigned long long)cm);
            const int ctotal = __shfl(cincl, kWave - 1);
            const int wbase = (int)threadIdx.x - blane();
            for (int tb = 0; tb < ctotal; tb += kWave) {  // uniform over the wavefront
                const int task = tb + blane();
                int src = 0;
#pragma unroll
                for (int step = kWave / 2; step > 0; step >>= 1)
                    if (__shfl(cincl, src + step - 1) <= task) src += step;
                const int k = task - __shfl(cincl - cm, src);
                const uint32_t msrc = (uint32_t)__shfl((int)m, src);
                const int32_t gs = __shfl(g, src), us = __shfl(u, src), ds = __shfl(deg, src);
                if (task >= ctotal) continue;
                uint32_t mm = msrc;
                for (int j = 0; j < k; j++) mm &= mm - 1u;
                const int l = __ffs((int)mm) - 1;
                const V r = Rs[((size_t)us * a.G + gs) * L + l];
                if (r != (V)0 && fabs(r) >= a.lane_eps[gs * L + l] * (V)ds) atomicOr(&s_pm[wbase + src], 1u << l);
            }
        }
        __syncthreads();
        if (valid) {
            pm = (mode & 2) ? s_pm[threadIdx.x] : m;
            if (a.probe) {  // LocalCH at the iteration cap: record active lanes, change nothing
                if (pm) atomicOr(&a.group_unconv[g], pm);
                pm = 0u;
            }
            if (a.ch) {  // the lanes active in t - 1 (their Delta counts), then those of t
                prev = a.PM[(size_t)u * a.G + g];
                a.PM[(size_t)u * a.G + g] = pm;
            }
            if (pm) atomicOr(&a.PB[(size_t)g * a.nwords + (u >> 5)], 1u << (u & 31));
        }
        const int c = __popc(pm);
        bool leader = valid && c > 0;
        if (a.row_stamp) {  // measurement: count each CSR row once per round (uniform branch)
            bool fresh_row = false;
            if (leader) fresh_row = atomicExch(&a.row_stamp[u], a.round_tag) != a.round_tag;
            block_reserve64(fresh_row ? ((1ull << 40) | (unsigned long long)deg) : 0ull, &st->rowpack[cur]);
        }
        const long long le = (leader && !a.no_push) ? (long long)deg * c : 0ll;
        const unsigned long long res =
            block_reserve64(leader ? ((1ull << 40) | (unsigned long long)le) : 0ull, &st->packed[cur]);
        const int slot0 = (int)(res >> 40);
        if (leader && slot0 >= a.wl_cap) {
            *ovf = 1;
            leader = false;
        }
        if (leader) {
            const long long off = (long long)(res & kLaneEdgeMask);
            a.wl_node[slot0] = u;
            a.wl_group[slot0] = g;
            a.wl_beg[slot0] = beg;
            a.wl_off[slot0] = off;
            a.wl_c[slot0] = c;
            const long long end = off + le;
            for (long long k = (off + kTile - 1) / kTile; k * kTile < end; k++) {
                if (k < a.tile_cap) a.tile_start[k] = slot0;
                else *ovf = 1;
            }
        }
        // the wavefront's pushed lanes as tasks 0 .. total-1, pair by pair
        const int cc = leader ? c : 0;
        const int incl = (int)wave_incl_scan64((unsigned long long)cc);
        const int excl = incl - cc;
        const int total = __shfl(incl, kWave - 1);
        const int shard = bid & (kStatShards - 1);
        for (int tb = 0; tb < total; tb += kWave) {  // uniform over the wavefront
            const int task = tb + blane();
            // the pair holding this task: the number of lanes whose count ends at or before it
            int src = 0;
#pragma unroll
            for (int step = kWave / 2; step > 0; step >>= 1)
                if (__shfl(incl, src + step - 1) <= task) src += step;
            const int k = task - __shfl(excl, src);
            const uint32_t pms = (uint32_t)__shfl((int)pm, src);
            const int slot = __shfl(slot0, src);
            const int32_t gs = __shfl(g, src), us = __shfl(u, src), ds = __shfl(deg, src);
            const int ms = __shfl(mode, src);
            const uint32_t prevs = (uint32_t)__shfl((int)prev, src);
            if (task >= total) continue;
            uint32_t mm = pms;  // its k-th active lane
            for (int j = 0; j < k; j++) mm &= mm - 1u;
            const int l = __ffs((int)mm) - 1;
            const size_t ri = ((size_t)us * a.G + gs) * L + l;
            V v;
            if (a.ch) {  // LocalCH: h = c_t r + m_t Delta (Delta of lanes active in t - 1)
                const V r = Rs[ri];
                const V h = a.force ? r : a.c_t * r + a.m_t * (((prevs >> l) & 1u) ? a.D[ri] : (V)0);
                const V rn = r - h;
                Rs[ri] = rn == (V)0 ? (V)-0.0 : rn;  // a zero keeps the touched mark
                a.X[ri] += h;
                a.D[ri] = h;
                v = h;
            } else {
                v = Rs[ri];
                Rs[ri] = LT ? (V)-0.0 : (V)0;  // -0.0: taken, already on the touched list
                a.X[ri] += v;
            }
            const V ws = a.g_wscale ? a.g_wscale[gs] : a.wscale;
            const V w = (ms & 1) ? ws / (V)ds : ws;
            a.wl_lanes[(size_t)slot * L + k] = (uint8_t)l;
            // level push: (c_{t+1} / c_t) v / d_u, in the order of the series' definition
            a.wl_sv[(size_t)slot * L + k] = a.R2 ? (ws * v) / (V)ds : w * v;
            const int lane_id = gs * L + l;
            atomicAdd((unsigned long long *)&a.lane_ops[(size_t)lane_id * kStatShards + shard],
                      (1ull << (64 - kPushBits)) | (unsigned long long)ds);
            if (a.lane_T[lane_id] < t + 1) atomicMax(&a.lane_T[lane_id], t + 1);
            if (a.tr_size && t < a.tr_cap) {
                atomicAdd((unsigned long long *)&a.tr_size[(size_t)lane_id * a.tr_cap + t], 1ull);
                atomicAdd((unsigned long long *)&a.tr_vol[(size_t)lane_id * a.tr_cap + t], (unsigned long long)ds);
            }
            if (a.tr_nodes) {
                // positions grow across iterations, so each S_t is one contiguous run
                const unsigned long long k2 = atomicAdd(&a.tr_ncount[lane_id], 1ull);
                if ((long long)k2 < a.tr_ncap[lane_id]) a.tr_nodes[a.tr_noff[lane_id] + (long long)k2] = us;
            }
        }
    }
}

// ------------------------------------------------------------------ phase P
template <typename V, int L, bool LT>
__device__ void batch_push(const BatchArgs<V> &a, int t, int bid, int nblocks) {
    __shared__ long long s_off[kTile + 1];
    __shared__ int32_t s_beg[kTile + 1];
    __shared__ int32_t s_c[kTile + 1];
    __shared__ int32_t s_g[kTile + 1];
    BatchDev *st = a.st;
    const int cur = t & 1, nxt = cur ^ 1;
    V *Rp = (a.R2 && !(t & 1)) ? a.R2 : a.R;  // the plane receiving the pushes
    const unsigned long long pk = st->packed[cur];
    const int count = min((int)(pk >> 40), a.wl_cap);
    const long long total = (long long)(pk & kLaneEdgeMask);
    int32_t *ovf = &st->ovf[cur];
    if (bid == 0 && threadIdx.x == 0 && count > 0) {
        st->lane_edges += total;
        st->entries += count;
        const unsigned long long rp = st->rowpack[cur];
        st->rows += (long long)(rp >> 40);
        st->row_vol += (long long)(rp & kLaneEdgeMask);
    }
    if (a.ch && count > 0) {
        // LocalCH: each pushed pair's residual changed, so its pushed lanes are
        // candidates of t + 1 (the snapshot cleared their masks)
        for (int b0 = bid * (int)blockDim.x; b0 < count; b0 += nblocks * (int)blockDim.x) {
            const int slot = b0 + (int)threadIdx.x;
            bool fresh = false;
            uint64_t pair = 0;
            if (slot < count) {
                const int c = a.wl_c[slot];
                uint32_t m = 0u;
                for (int k = 0; k < c; k++) m |= 1u << a.wl_lanes[(size_t)slot * L + k];
                const int32_t u = a.wl_node[slot], g = a.wl_group[slot];
                fresh = m && atomicOr(&a.NM[(size_t)u * a.G + g], m) == 0u;
                pair = ((uint64_t)(uint32_t)g << 32) | (uint32_t)u;
            }
            int sa = block_reserve(fresh ? 1 : 0, &st->acount[nxt]);
            if (fresh) {
                if (sa < a.act_cap) a.act[nxt][sa] = pair;
                else *ovf = 1;
            }
        }
    }
    const long long ntiles = min((total + kTile - 1) / kTile, (long long)a.tile_cap - 1);
    for (long long tile = bid; tile < ntiles; tile += nblocks) {
        const long long e0 = tile * kTile;
        const long long e1 = min(e0 + kTile, total);
        const int i0 = a.tile_start[tile];
        const int i1 = (tile + 1 < ntiles) ? a.tile_start[tile + 1] : count - 1;
        const int m = min(i1 - i0 + 1, kTile + 1);
        if (m <= 0 || i0 < 0 || i1 >= count) {
            if (threadIdx.x == 0) *ovf = 1;
            continue;
        }
        __syncthreads();
        for (int j = threadIdx.x; j < m; j += blockDim.x) {
            s_off[j] = a.wl_off[i0 + j];
            s_beg[j] = a.wl_beg[i0 + j];
            s_c[j] = a.wl_c[i0 + j];
            s_g[j] = a.wl_group[i0 + j];
        }
        __syncthreads();
        // kPer lane-edges per thread, strided by the workgroup size; their loads
        // and atomics are issued before any result is waited on
        constexpr int kPer = kTile / kBlock;
        int32_t gq[kPer], wq[kPer], lq[kPer];
        V dv[kPer], dq[kPer];
        bool hit[kPer], first[kPer];
#pragma unroll
        for (int q = 0; q < kPer; q++) {
            const long long e = e0 + (long long)q * kBlock + threadIdx.x;
            hit[q] = first[q] = false;
            gq[q] = 0;
            wq[q] = -1;
            lq[q] = 0;
            dv[q] = (V)0;
            dq[q] = (V)0;
            if (e < e1) {
                int lo = 0, hi = m - 1;
                while (lo < hi) {
                    int mid = (lo + hi + 1) >> 1;
                    if (s_off[mid] <= e) lo = mid; else hi = mid - 1;
                }
                const long long qq = e - s_off[lo];
                const int c = s_c[lo];
                if (c > 0) {
                    const long long edge = qq / c;
                    const int k = (int)(qq - edge * c);
                    const size_t slot = (size_t)(i0 + lo);
                    const int l = a.wl_lanes[slot * L + k];
                    const long long ci = (long long)s_beg[lo] + edge;
                    if (ci >= 0 && ci < a.nnz && l < L) {
                        gq[q] = s_g[lo];
                        wq[q] = a.col_idx[ci];
                        if (a.col_deg) dq[q] = a.col_deg[ci];
                        lq[q] = l;
                        dv[q] = a.wl_sv[slot * L + k];
                    } else {
                        *ovf = 1;
                    }
                }
            }
        }
        V old[kPer], th[kPer];
#pragma unroll
        for (int q = 0; q < kPer; q++) {
            th[q] = (V)0;
            if (wq[q] >= 0) {
                const V e = a.lane_eps[gq[q] * L + lq[q]];
                th[q] = (a.R2 ? (V)((double)e / a.th_div) : e) * (a.col_deg ? dq[q] : a.deg[wq[q]]);
            }
        }
#pragma unroll
        for (int q = 0; q < kPer; q++)
            old[q] = wq[q] >= 0 ? unsafeAtomicAdd(&Rp[((size_t)wq[q] * a.G + gq[q]) * L + lq[q]], dv[q]) : (V)0;
        int n_act = 0, n_touch = 0;
        bool new_act[kPer], new_touch[kPer];
#pragma unroll
        for (int q = 0; q < kPer; q++) {
            new_act[q] = new_touch[q] = false;
            if (wq[q] >= 0) {
                const V nw = old[q] + dv[q];
                // signed residuals (LocalCH, warm start, serving groups corrected for
                // inserted edges): |r| lifted across the threshold
                const bool sg = a.sgn || a.ch || (a.g_mode && (a.g_mode[gq[q]] & 2));
                hit[q] = sg ? (fabs(old[q]) < th[q] && fabs(nw) >= th[q]) : (old[q] < th[q] && nw >= th[q]);
                first[q] = LT ? (pos_zero(old[q]) && dv[q] != (V)0) : old[q] == (V)0;
                if (hit[q]) {
                    // (signed: a lane may be marked already, by its own push or a second
                    // crossing, so the mask is read before the atomic; a nonnegative
                    // residual crosses once per push and its lane is never marked)
                    uint32_t *nm = &a.NM[(size_t)wq[q] * a.G + gq[q]];
                    const uint32_t bit = 1u << lq[q];
                    new_act[q] = !(sg && (*nm & bit)) && atomicOr(nm, bit) == 0u;
                }
                if (LT) {
                    new_touch[q] = first[q];
                } else if (first[q]) {
                    uint32_t *tm = &a.TM[(size_t)wq[q] * a.G + gq[q]];
                    const uint32_t ep = a.g_epoch ? a.g_epoch[gq[q]] : a.epoch;
                    if (*tm != ep) new_touch[q] = atomicExch(tm, ep) != ep;
                }
            }
            n_act += new_act[q] ? 1 : 0;
            n_touch += new_touch[q] ? 1 : 0;
        }
        int sa = block_reserve(n_act, &st->acount[nxt]);
        const bool odd = a.R2 && !(t & 1);  // level push: entries of level t + 1 go to its parity's list
        uint64_t *tlist = odd ? a.touched2 : a.touched;
        int32_t *tdl = odd ? a.tdeg2 : a.tdeg;
        int stt = block_reserve(n_touch, odd ? &st->tcount2 : &st->tcount);
#pragma unroll
        for (int q = 0; q < kPer; q++) {
            const uint64_t pair = ((uint64_t)(uint32_t)gq[q] << 32) | (uint32_t)wq[q];
            if (new_act[q]) {
                if (sa < a.act_cap) a.act[nxt][sa] = pair;
                else *ovf = 1;
                sa++;
            }
            if (new_touch[q]) {
                // LT: the entry names the lane, (g * L + l) << 32 | node
                const uint64_t te = LT ? ((uint64_t)(uint32_t)(gq[q] * L + lq[q]) << 32) | (uint32_t)wq[q] : pair;
                if (stt < a.touch_cap) {
                    tlist[stt] = te;
                    // the node's degree beside the entry, for the norms at the end
                    if (LT && tdl) tdl[stt] = (int32_t)(a.col_deg ? dq[q] : a.deg[wq[q]]);
                }
                else *ovf = 1;
                stt++;
            }
        }
    }
}

// ------------------------------------------------------------------ launches
template <typename V, int L, bool LT>
__global__ void __launch_bounds__(kBatchSnapBlock) k_batch_snap(BatchArgs<V> a, int t) {
    batch_snap<V, L, LT>(a, t, blockIdx.x, gridDim.x);
}
template <typename V, int L, bool LT>
__global__ void __launch_bounds__(kBlock) k_batch_push(BatchArgs<V> a, int t) {
    batch_push<V, L, LT>(a, t, blockIdx.x, gridDim.x);
}

// r <- b for every lane's seeds; the (group, node) pairs of the seeds form S_0
// (forced, Definition 3.1) with their lanes' bits in the next-mask.  Each seed
// (lane, node) goes on the touched list (batched solves list lanes, see above).
template <typename V, int L>
__global__ void k_batch_seed(BatchArgs<V> a, const int32_t *__restrict__ s_lane, const int32_t *__restrict__ s_node,
                             const double *__restrict__ s_val, int32_t ns, double bscale) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    bool fresh = false;
    uint64_t pair = 0;
    if (i < ns) {
        const int lane_id = s_lane[i];
        const int g = lane_id / L, l = lane_id % L;
        const int32_t u = s_node[i];
        double sv = s_val[i];
        if (a.sym) sv = sv * sqrt((double)(a.row_ptr[u + 1] - a.row_ptr[u]));
        a.R[((size_t)u * a.G + g) * L + l] = (V)(bscale * sv);
        fresh = atomicOr(&a.NM[(size_t)u * a.G + g], 1u << l) == 0u;
        pair = ((uint64_t)(uint32_t)g << 32) | (uint32_t)u;
    }
    bwave_append64(fresh, &a.st->acount[0], pair, a.act[0], a.act_cap, &a.st->ovf[0]);
    const uint64_t te = i < ns ? ((uint64_t)(uint32_t)s_lane[i] << 32) | (uint32_t)s_node[i] : 0ull;
    const int sl = bwave_append64(i < ns, &a.st->tcount, te, a.touched, a.touch_cap, &a.st->ovf[0]);
    if (sl >= 0 && sl < a.touch_cap && a.tdeg) a.tdeg[sl] = a.row_ptr[s_node[i] + 1] - a.row_ptr[s_node[i]];
}

// Residual norms per lane over the touched (lane, node) entries (each listed
// once: read, reset to +0.0, one thread per entry), plus the lanes still active
// at the iteration cap.  With lds_lanes (G*L lanes fit in the dynamic LDS) a
// workgroup first sums its share per lane in LDS and adds each lane's total
// once at the end, instead of one global atomic per nonzero entry.
// Level push (lvl >= 0): the entries of level lvl only (its parity's list), on
// its plane, each |r| weighted rscale in the 1-norm and w_dinf * (|r| / d) in
// the max norm.
template <typename V, int L>
__global__ void __launch_bounds__(kBlock) k_batch_residual(BatchArgs<V> a, double rscale, int last, int lds_lanes,
                                                           int lvl, double w_dinf) {
    extern __shared__ __attribute__((aligned(16))) unsigned char s_res[];
    double *s_l1 = (double *)s_res;
    unsigned long long *s_dm = (unsigned long long *)(s_l1 + lds_lanes);
    BatchDev *st = a.st;
    int nt = min(st->tcount, a.touch_cap);
    V *R = a.R;
    const uint64_t *list = a.touched;
    const int32_t *dl = a.tdeg;
    if (lvl >= 0 && (lvl & 1)) {
        nt = min(st->tcount2, a.touch_cap);
        R = a.R2;
        list = a.touched2;
        dl = a.tdeg2;
    }
    for (int j = threadIdx.x; j < lds_lanes; j += blockDim.x) {
        s_l1[j] = 0.0;
        s_dm[j] = 0ull;
    }
    __syncthreads();
    // kU entries per thread and step: their list words, then their residuals,
    // are loaded before any is used (the loop is latency-bound otherwise)
    constexpr int kU = 4;
    const int stride = gridDim.x * blockDim.x;
    for (int base = blockIdx.x * blockDim.x * kU + threadIdx.x; base < nt; base += stride * kU) {
        uint64_t pr[kU];
        V val[kU];
        int32_t dd[kU];
#pragma unroll
        for (int q = 0; q < kU; q++) {
            const int i = base + q * (int)blockDim.x;
            pr[q] = i < nt ? list[i] : ~0ull;
            dd[q] = (i < nt && dl) ? dl[i] : 0;
        }
#pragma unroll
        for (int q = 0; q < kU; q++) {
            val[q] = (V)0;
            if (pr[q] != ~0ull) {
                const int32_t lane_id = (int32_t)(pr[q] >> 32), w = (int32_t)(pr[q] & 0xffffffffull);
                V *rp = &R[((size_t)w * a.G + lane_id / L) * L + lane_id % L];
                // LocalCH: a signed residual that cancelled to +0.0 is listed again when it
                // is touched next, so the value is taken by exchange (once) there
                val[q] = (a.ch || a.sgn) ? batomic_take<V>(rp) : *rp;
            }
        }
#pragma unroll
        for (int q = 0; q < kU; q++) {
            if (pr[q] == ~0ull) continue;
            const int32_t lane_id = (int32_t)(pr[q] >> 32), w = (int32_t)(pr[q] & 0xffffffffull);
            R[((size_t)w * a.G + lane_id / L) * L + lane_id % L] = (V)0;
            const double av = fabs((double)val[q]) * rscale;
            if (av > 0.0) {
                const double dw = dl ? (double)dd[q] : (double)a.deg[w];
                const double dm = lvl >= 0 ? w_dinf * (fabs((double)val[q]) / dw) : av / dw;
                const unsigned long long bits = (unsigned long long)__double_as_longlong(dm);
                if (lds_lanes) {
                    atomicAdd(&s_l1[lane_id], av);
                    if (s_dm[lane_id] < bits) atomicMax(&s_dm[lane_id], bits);
                } else {
                    atomicAdd(&a.lane_l1[(size_t)lane_id * kStatShards + (blockIdx.x & (kStatShards - 1))], av);
                    unsigned long long *dm = &a.lane_dinf[lane_id];
                    if (*dm < bits) atomicMax(dm, bits);
                }
            }
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < lds_lanes; j += blockDim.x) {
        if (s_l1[j] != 0.0) atomicAdd(&a.lane_l1[(size_t)j * kStatShards + (blockIdx.x & (kStatShards - 1))], s_l1[j]);
        if (s_dm[j] != 0ull && a.lane_dinf[j] < s_dm[j]) atomicMax(&a.lane_dinf[j], s_dm[j]);
    }
    // pairs left in the active list at the iteration cap: their lanes did not converge
    const int na = last >= 0 ? min(st->acount[last], a.act_cap) : 0;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < na; j += gridDim.x * blockDim.x) {
        const uint64_t p = a.act[last][j];
        const int32_t g = (int32_t)(p >> 32), u = (int32_t)(p & 0xffffffffull);
        uint32_t *nm = &a.NM[(size_t)u * a.G + g];
        const uint32_t m = *nm;
        *nm = 0u;
        if (m) atomicOr(&a.group_unconv[g], m);
    }
}

template <typename V, int L>
__global__ void k_batch_subtract_seed(BatchArgs<V> a, const int32_t *__restrict__ s_lane,
                                      const int32_t *__restrict__ s_node, const double *__restrict__ s_val, int32_t ns,
                                      const int32_t *__restrict__ lane_flag) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ns && lane_flag[s_lane[i]]) {
        const int g = s_lane[i] / L, l = s_lane[i] % L;
        a.X[((size_t)s_node[i] * a.G + g) * L + l] -= (V)s_val[i];
    }
}

// Extraction, per group: the pushed bitmap gives the nodes in ascending order;
// lane l's support is {u : X[g][u][l] != 0}.  count -> scan -> emit.
template <typename V, int L>
__global__ void __launch_bounds__(kBlock) k_batch_ex_count(BatchArgs<V> a, int32_t *cnt, int nblk,
                                                            const int32_t *__restrict__ gmap) {
    __shared__ int s[L];
    const int g = gmap ? gmap[blockIdx.y] : (int)blockIdx.y;
    const int64_t wi = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (threadIdx.x < L) s[threadIdx.x] = 0;
    __syncthreads();
    int my[L];
#pragma unroll
    for (int l = 0; l < L; l++) my[l] = 0;
    if (wi < a.nwords) {
        uint32_t word = a.PB[(size_t)g * a.nwords + wi];
        while (word) {
            const int b = __ffs(word) - 1;
            word &= word - 1u;
            const int64_t u = wi * 32 + b;
            const V *xr = a.X + ((size_t)u * a.G + g) * L;
#pragma unroll
            for (int l = 0; l < L; l++) my[l] += xr[l] != (V)0 ? 1 : 0;
        }
    }
#pragma unroll
    for (int l = 0; l < L; l++)
        if (my[l]) atomicAdd(&s[l], my[l]);
    __syncthreads();
    if (threadIdx.x < L) cnt[((size_t)g * L + threadIdx.x) * nblk + blockIdx.x] = s[threadIdx.x];
}

// one block per lane: exclusive scan over its blocks' counts, total into lane_nnz
__global__ void __launch_bounds__(256) k_batch_ex_scan(int32_t *cnt, int nblk, long long *lane_nnz, int L,
                                                       const int32_t *__restrict__ gmap) {
    __shared__ int s[256];
    __shared__ long long carry;
    const int lane_id = gmap ? gmap[blockIdx.x / L] * L + (int)(blockIdx.x % L) : (int)blockIdx.x;
    int32_t *c = cnt + (size_t)lane_id * nblk;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nblk; base += 256) {
        const int i = base + threadIdx.x;
        const int v = i < nblk ? c[i] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            int y = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0;
            __syncthreads();
            s[threadIdx.x] += y;
            __syncthreads();
        }
        if (i < nblk) c[i] = (int32_t)(carry + s[threadIdx.x] - v);
        __syncthreads();
        if (threadIdx.x == 255) carry += s[255];
        __syncthreads();
    }
    if (threadIdx.x == 0) lane_nnz[lane_id] = carry;
}

template <typename V, int L>
__global__ void __launch_bounds__(kBlock) k_batch_ex_emit(BatchArgs<V> a, const int32_t *__restrict__ cnt, int nblk,
                                                           const long long *__restrict__ lane_out_off,
                                                           int32_t *out_idx, V *out_val, int write,
                                                           const int32_t *__restrict__ gmap,
                                                           int32_t *const *__restrict__ lane_idx,
                                                           V *const *__restrict__ lane_val) {
    __shared__ int s[L][kBlock];
    const int g = gmap ? gmap[blockIdx.y] : (int)blockIdx.y;
    const int64_t wi = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    uint32_t word = wi < a.nwords ? a.PB[(size_t)g * a.nwords + wi] : 0u;
    int my[L];
#pragma unroll
    for (int l = 0; l < L; l++) my[l] = 0;
    {
        uint32_t wd = word;
        while (wd) {
            const int b = __ffs(wd) - 1;
            wd &= wd - 1u;
            const V *xr = a.X + ((size_t)(wi * 32 + b) * a.G + g) * L;
#pragma unroll
            for (int l = 0; l < L; l++) my[l] += xr[l] != (V)0 ? 1 : 0;
        }
    }
#pragma unroll
    for (int l = 0; l < L; l++) s[l][threadIdx.x] = my[l];
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        int y[L];
#pragma unroll
        for (int l = 0; l < L; l++) y[l] = (int)threadIdx.x >= off ? s[l][threadIdx.x - off] : 0;
        __syncthreads();
#pragma unroll
        for (int l = 0; l < L; l++) s[l][threadIdx.x] += y[l];
        __syncthreads();
    }
    if (word) {
        long long pos[L];
#pragma unroll
        for (int l = 0; l < L; l++)
            pos[l] = lane_out_off[g * L + l] + cnt[((size_t)g * L + l) * nblk + blockIdx.x] + s[l][threadIdx.x] - my[l];
        while (word) {
            const int b = __ffs(word) - 1;
            word &= word - 1u;
            const int32_t u = (int32_t)(wi * 32 + b);
            V *xr = a.X + ((size_t)u * a.G + g) * L;
#pragma unroll
            for (int l = 0; l < L; l++) {
                const V xv0 = xr[l];
                if (xv0 != (V)0) {
                    const long long lo = lane_out_off[g * L + l];
                    const V xv = a.sym ? (V)((double)xv0 / sqrt((double)(a.row_ptr[u + 1] - a.row_ptr[u]))) : xv0;
                    if (write && lo >= 0) {
                        if (lane_idx) {  // straight into the query's own buffers
                            lane_idx[g * L + l][pos[l] - lo] = u;
                            lane_val[g * L + l][pos[l] - lo] = xv;
                        } else {
                            out_idx[pos[l]] = u;
                            out_val[pos[l]] = xv;
                        }
                    }
                    pos[l]++;
                    xr[l] = (V)0;
                }
            }
        }
        a.PB[(size_t)g * a.nwords + wi] = 0u;
    }
}

// Warm start: one thread per (node, group) takes each lane's residual at the
// node when the node is in that query's touched bitmap (the only nodes where it
// can be nonzero); a nonzero one becomes a touched entry (its degree beside it)
// and the node a candidate of iteration 0.  The appends are wave-aggregated.
template <typename V, int L>
__global__ void __launch_bounds__(kBlock) k_batch_warm_load(BatchArgs<V> a, const RD<V> *const *__restrict__ q_rd,
                                                            const uint32_t *const *__restrict__ q_tbm, int B) {
    const int g = (int)blockIdx.y;
    const int64_t ui = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool in = ui < a.n;
    const int32_t u = in ? (int32_t)ui : 0;
    const int32_t dg = in && a.tdeg ? a.row_ptr[u + 1] - a.row_ptr[u] : 0;
    uint32_t mask = 0u;
    for (int l = 0; l < L; l++) {  // uniform over the wave: every lane takes part in the appends
        const int j = g * L + l;
        V r = (V)0;
        if (in && j < B && ((q_tbm[j][u >> 5] >> (u & 31)) & 1u)) r = q_rd[j][u].r;
        const bool nz = r != (V)0;
        if (nz) {
            a.R[((size_t)u * a.G + g) * L + l] = r;
            mask |= 1u << l;
        }
        const int te = bwave_append64(nz, &a.st->tcount, ((uint64_t)(uint32_t)j << 32) | (uint32_t)u, a.touched,
                                      a.touch_cap, &a.st->ovf[0]);
        if (nz && a.tdeg && te < a.touch_cap) a.tdeg[te] = dg;
    }
    const bool fresh = mask != 0u && atomicOr(&a.NM[(size_t)u * a.G + g], mask) == 0u;
    bwave_append64(fresh, &a.st->acount[0], ((uint64_t)(uint32_t)g << 32) | (uint32_t)u, a.act[0], a.act_cap,
                   &a.st->ovf[0]);
}

// stage 0 (before the residual pass): each touched entry's residual back into
// its query (and the node into the query's touched bitmap); the pass then reads
// and clears R as usual.  Stage 1 (the extraction): per group, every pushed
// node's lane increments added into the queries' x, which marks the node pushed.
template <typename V, int L>
__global__ void __launch_bounds__(kBlock) k_batch_warm_store_r(BatchArgs<V> a, RD<V> *const *__restrict__ q_rd,
                                                               uint32_t *const *__restrict__ q_tbm) {
    const int nt = min(a.st->tcount, a.touch_cap);
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < nt; i += gridDim.x * kBlock) {
        const uint64_t e = a.touched[i];
        const int32_t j = (int32_t)(e >> 32), u = (int32_t)(e & 0xffffffffull);
        const V v = a.R[((size_t)u * a.G + j / L) * L + j % L];
        q_rd[j][u].r = v == (V)0 ? (V)0 : v;  // -0.0 (taken) is stored as 0
        atomicOr(&q_tbm[j][u >> 5], 1u << (u & 31));
    }
}

// One thread per (pushed-bitmap word, lane): the L threads of a word sit in one
// wavefront (L divides 64), read the word together, and each owns its query's
// pushed-bitmap word, so no atomics are needed.
template <typename V, int L>
__global__ void __launch_bounds__(kBlock) k_batch_warm_store_x(BatchArgs<V> a, V *const *__restrict__ q_x,
                                                               uint32_t *const *__restrict__ q_pushed, int B) {
    static_assert(64 % L == 0, "the threads of one word must share a wavefront");
    const int g = (int)blockIdx.y;
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t wi = t / L;
    const int l = (int)(t % L), j = g * L + l;
    if (wi >= a.nwords) return;
    uint32_t *pw = a.PB + (size_t)g * a.nwords + wi;
    uint32_t word = *pw;
    if (!word) return;
    if (j < B) {
        V *__restrict__ qx = q_x[j];
        V *__restrict__ xb = a.X + (size_t)g * L + l;
        const size_t stride = (size_t)a.G * L;
        uint32_t pushed = 0u;
        for (uint32_t w = word; w; w &= w - 1u) {
            const int b = __ffs((int)w) - 1;
            const int32_t u = (int32_t)(wi * 32 + b);
            V *xp = xb + (size_t)u * stride;
            const V xv = *xp;
            if (xv == (V)0) continue;
            qx[u] = qx[u] + xv;
            *xp = (V)0;
            pushed |= 1u << b;
        }
        if (pushed) q_pushed[j][wi] |= pushed;
    }
    if (l == 0) *pw = 0u;
}

template <typename V>
__global__ void k_batch_init_deg(const int32_t *__restrict__ row_ptr, V *deg, int32_t n) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x)
        deg[u] = (V)(row_ptr[u + 1] - row_ptr[u]);
}

// ------------------------------------------------------------------ host-side launchers
template <typename V>
hipError_t batch_launch(int which, int L, const BatchArgs<V> &a, int grid, int t, hipStream_t s) {
    // per-group tags (serving) or lane entries (batched solves), see the touched lists above
    const bool lt = a.g_epoch == nullptr;
    const int sgrid = (grid * kBlock + kBatchSnapBlock - 1) / kBatchSnapBlock;
#define GDE_BL(LL)                                                                                       \
    case LL:                                                                                             \
        if (which == 1 && lt) hipLaunchKernelGGL((k_batch_snap<V, LL, true>), dim3(sgrid),                \
                                                 dim3(kBatchSnapBlock), 0, s, a, t);                      \
        else if (which == 1) hipLaunchKernelGGL((k_batch_snap<V, LL, false>), dim3(sgrid),                \
                                                dim3(kBatchSnapBlock), 0, s, a, t);                       \
        else if (lt) hipLaunchKernelGGL((k_batch_push<V, LL, true>), dim3(grid), dim3(kBlock), 0, s, a, t); \
        else hipLaunchKernelGGL((k_batch_push<V, LL, false>), dim3(grid), dim3(kBlock), 0, s, a, t);      \
        return hipGetLastError();
    switch (L) {
        GDE_BL(8)
        GDE_BL(16)
        GDE_BL(32)
    default:
        return hipErrorInvalidValue;
    }
#undef GDE_BL
}

template <typename V>
hipError_t batch_occupancy(int L, int *blocks_per_cu) {
    switch (L) {
    case 8: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_batch_push<V, 8, true>, kBlock, 0);
    case 16: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_batch_push<V, 16, true>, kBlock, 0);
    case 32: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_batch_push<V, 32, true>, kBlock, 0);
    default: return hipErrorInvalidValue;
    }
}

template <typename V>
hipError_t batch_seed(int L, const BatchArgs<V> &a, const int32_t *s_lane, const int32_t *s_node, const double *s_val,
                      int32_t ns, double bscale, hipStream_t s) {
    const int grid = (ns + 255) / 256;
    switch (L) {
    case 8: hipLaunchKernelGGL((k_batch_seed<V, 8>), dim3(grid), dim3(256), 0, s, a, s_lane, s_node, s_val, ns, bscale); break;
    case 16: hipLaunchKernelGGL((k_batch_seed<V, 16>), dim3(grid), dim3(256), 0, s, a, s_lane, s_node, s_val, ns, bscale); break;
    case 32: hipLaunchKernelGGL((k_batch_seed<V, 32>), dim3(grid), dim3(256), 0, s, a, s_lane, s_node, s_val, ns, bscale); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename V>
hipError_t batch_harvest(int L, const BatchArgs<V> &a, int grid, int t, double w_l1, double w_dinf, hipStream_t s) {
    const int lds_lanes = (int64_t)a.G * L <= kResLdsLanes ? a.G * L : 0;
    switch (L) {
    case 8: hipLaunchKernelGGL((k_batch_residual<V, 8>), dim3(grid), dim3(kBlock), 16 * (size_t)lds_lanes, s, a, w_l1, -1, lds_lanes, t, w_dinf); break;
    case 16: hipLaunchKernelGGL((k_batch_residual<V, 16>), dim3(grid), dim3(kBlock), 16 * (size_t)lds_lanes, s, a, w_l1, -1, lds_lanes, t, w_dinf); break;
    case 32: hipLaunchKernelGGL((k_batch_residual<V, 32>), dim3(grid), dim3(kBlock), 16 * (size_t)lds_lanes, s, a, w_l1, -1, lds_lanes, t, w_dinf); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename V>
hipError_t batch_finish(int L, const BatchArgs<V> &a, int grid, double rscale, int last, const int32_t *s_lane,
                        const int32_t *s_node, const double *s_val, int32_t ns, const int32_t *sub_flag,
                        hipStream_t s) {
    const int sg = (ns + 255) / 256;
    const int lds_lanes = (int64_t)a.G * L <= kResLdsLanes ? a.G * L : 0;
    switch (L) {
#define GDE_BF(LL)                                                                                             \
    case LL:                                                                                                   \
        hipLaunchKernelGGL((k_batch_residual<V, LL>), dim3(grid), dim3(kBlock), 16 * (size_t)lds_lanes, s, a,   \
                           rscale, last, lds_lanes, -1, 0.0);                                                  \
        if (sub_flag) hipLaunchKernelGGL((k_batch_subtract_seed<V, LL>), dim3(sg), dim3(256), 0, s, a, s_lane, \
                                         s_node, s_val, ns, sub_flag);                                         \
        break;
        GDE_BF(8)
        GDE_BF(16)
        GDE_BF(32)
#undef GDE_BF
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename V>
hipError_t batch_extract(int L, const BatchArgs<V> &a, int stage, int32_t *cnt, int nblk, long long *lane_nnz,
                         const long long *lane_out_off, int32_t *out_idx, V *out_val, int write, hipStream_t s,
                         const int32_t *gmap, int ngroups, int32_t *const *lane_idx, V *const *lane_val) {
    const int ng = gmap ? ngroups : a.G;
    if (ng <= 0) return hipSuccess;
    dim3 grid((unsigned)nblk, (unsigned)ng);
    switch (L) {
#define GDE_BE(LL)                                                                                                  \
    case LL:                                                                                                        \
        if (stage == 0) {                                                                                           \
            hipLaunchKernelGGL((k_batch_ex_count<V, LL>), grid, dim3(kBlock), 0, s, a, cnt, nblk, gmap);            \
            hipLaunchKernelGGL(k_batch_ex_scan, dim3((unsigned)(ng * LL)), dim3(256), 0, s, cnt, nblk, lane_nnz, LL,  \
                               gmap);                                                                               \
        } else {                                                                                                    \
            hipLaunchKernelGGL((k_batch_ex_emit<V, LL>), grid, dim3(kBlock), 0, s, a, cnt, nblk, lane_out_off,      \
                               out_idx, out_val, write, gmap, lane_idx, lane_val);                                  \
        }                                                                                                           \
        break;
        GDE_BE(8)
        GDE_BE(16)
        GDE_BE(32)
#undef GDE_BE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename V>
__global__ void k_batch_col_deg(const int32_t *__restrict__ col_idx, const V *__restrict__ deg, V *col_deg,
                                int64_t nnz) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x)
        col_deg[e] = deg[col_idx[e]];
}

template <typename V>
hipError_t batch_warm_load(int L, const BatchArgs<V> &a, const void *const *q_rd, const uint32_t *const *q_tbm, int B,
                           hipStream_t s) {
    const dim3 grid((unsigned)(((int64_t)a.n + kBlock - 1) / kBlock), (unsigned)a.G);
    const RD<V> *const *rd = (const RD<V> *const *)q_rd;
    switch (L) {
    case 8: hipLaunchKernelGGL((k_batch_warm_load<V, 8>), grid, dim3(kBlock), 0, s, a, rd, q_tbm, B); break;
    case 16: hipLaunchKernelGGL((k_batch_warm_load<V, 16>), grid, dim3(kBlock), 0, s, a, rd, q_tbm, B); break;
    case 32: hipLaunchKernelGGL((k_batch_warm_load<V, 32>), grid, dim3(kBlock), 0, s, a, rd, q_tbm, B); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename V>
hipError_t batch_warm_store(int L, const BatchArgs<V> &a, int stage, void *const *q_rd, uint32_t *const *q_tbm,
                            void *const *q_x, uint32_t *const *q_pushed, int B, int grid, hipStream_t s) {
    const dim3 gx((unsigned)((a.nwords * L + kBlock - 1) / kBlock), (unsigned)a.G);
    switch (L) {
#define GDE_BW(LL)                                                                                                   \
    case LL:                                                                                                         \
        if (stage == 0)                                                                                              \
            hipLaunchKernelGGL((k_batch_warm_store_r<V, LL>), dim3(grid), dim3(kBlock), 0, s, a, (RD<V> *const *)q_rd, \
                               q_tbm);                                                                               \
        else                                                                                                         \
            hipLaunchKernelGGL((k_batch_warm_store_x<V, LL>), gx, dim3(kBlock), 0, s, a, (V *const *)q_x, q_pushed, B); \
        break;
        GDE_BW(8)
        GDE_BW(16)
        GDE_BW(32)
#undef GDE_BW
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename V>
hipError_t batch_init_col_deg(const int32_t *col_idx, const V *deg, V *col_deg, int64_t nnz, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_col_deg<V>, dim3(8192), dim3(256), 0, s, col_idx, deg, col_deg, nnz);
    return hipGetLastError();
}

template <typename V>
hipError_t batch_init_deg(const int32_t *row_ptr, V *deg, int32_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_init_deg<V>, dim3(4096), dim3(256), 0, s, row_ptr, deg, n);
    return hipGetLastError();
}

#define GDE_BINST(V)                                                                                               \
    template hipError_t batch_launch<V>(int, int, const BatchArgs<V> &, int, int, hipStream_t);                    \
    template hipError_t batch_occupancy<V>(int, int *);                                                            \
    template hipError_t batch_harvest<V>(int, const BatchArgs<V> &, int, int, double, double, hipStream_t);        \
    template hipError_t batch_seed<V>(int, const BatchArgs<V> &, const int32_t *, const int32_t *, const double *, \
                                      int32_t, double, hipStream_t);                                               \
    template hipError_t batch_finish<V>(int, const BatchArgs<V> &, int, double, int, const int32_t *,              \
                                        const int32_t *, const double *, int32_t, const int32_t *, hipStream_t);   \
    template hipError_t batch_extract<V>(int, const BatchArgs<V> &, int, int32_t *, int, long long *,              \
                                         const long long *, int32_t *, V *, int, hipStream_t, const int32_t *,     \
                                         int, int32_t *const *, V *const *);                                       \
    template hipError_t batch_init_deg<V>(const int32_t *, V *, int32_t, hipStream_t);                            \
    template hipError_t batch_init_col_deg<V>(const int32_t *, const V *, V *, int64_t, hipStream_t);            \
    template hipError_t batch_warm_load<V>(int, const BatchArgs<V> &, const void *const *, const uint32_t *const *, \
                                           int, hipStream_t);                                                     \
    template hipError_t batch_warm_store<V>(int, const BatchArgs<V> &, int, void *const *, uint32_t *const *,      \
                                            void *const *, uint32_t *const *, int, int, hipStream_t);

GDE_BINST(float)
GDE_BINST(double)

}  // namespace gde
