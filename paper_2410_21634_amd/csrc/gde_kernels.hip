// gde_kernels.hip -- gfx950 kernels of the local diffusion process (Definition 3.1).
//
// One iteration t of LocalGD (Eq. (9)) is two launches:
//   snap : for every u in S_t take v_u = r_u (the synchronous snapshot), set
//          r_u = 0, x_u += v_u, and reserve a contiguous slice of the work list
//          and of the edge space with one 64-bit atomic per workgroup;
//   push : edge-balanced scatter r_w += W_u v_u over the CSR rows of S_t, tiles
//          of kPushTile edges staged through LDS; every returned old value is
//          tested against theta_w, and the unique add that lifts r_w over
//          theta_w appends w to S_{t+1} (workgroup-aggregated compaction).
// Because snap has already zeroed the residual of every u in S_t, the push only
// adds nonnegative mass, r_w is monotone during the launch and the crossing
// test fires exactly once for every node whose residual ends at or above its
// threshold: S_{t+1} is produced without scanning candidates.
//
// LocalCH (Sec. 3.3) has signed updates, so its push marks touched nodes as
// candidates (stamp de-duplication) and its snap applies the threshold.
// The heat kernel runs the same pair per Taylor level with the residual
// planes of level k and k+1 (the Kronecker block structure of the AHK push).
#include <hip/hip_runtime.h>

#include "gde_device.h"
#include "gde_internal.h"
#include "gde_kernels.h"

namespace gde {

// Workgroup-aggregated list append of v where pred; entries beyond cap are dropped and flagged.
__device__ __forceinline__ void block_list_append(bool pred, int32_t v, int32_t *counter, int32_t *list, int32_t cap,
                                                  DevState *st) {
    const int slot = block_reserve(pred ? 1 : 0, counter);
    if (pred) {
        if (slot < cap) list[slot] = v;
        else st->overflow = 1;
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    return v;
}

// block-wide sum and max of two doubles, folded into the device state
__device__ void block_fold_norms(double l1, double mx, DevState *st) {
    __shared__ double s_l1[kMaxWaves], s_mx[kMaxWaves];
    l1 = wave_sum(l1);
    mx = wave_max(mx);
    int w = threadIdx.x / kWave;
    if (lane() == 0) { s_l1[w] = l1; s_mx[w] = mx; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, m = 0.0;
        for (int i = 0; i < (int)(blockDim.x / kWave); i++) { a += s_l1[i]; m = fmax(m, s_mx[i]); }
        if (a != 0.0) atomicAdd(&st->res_l1, a);
        if (m > 0.0) atomicMax(&st->res_dinf, (unsigned long long)__double_as_longlong(m));
    }
}

template <typename V>
__device__ __forceinline__ V atomic_take(V *p);
template <>
__device__ __forceinline__ float atomic_take<float>(float *p) { return atomicExch(p, 0.0f); }
template <>
__device__ __forceinline__ double atomic_take<double>(double *p) {
    return __longlong_as_double((long long)atomicExch((unsigned long long *)p, 0ull));
}

// ------------------------------------------------------------------ setup
template <typename V>
__global__ void k_init_rd(const int32_t *__restrict__ row_ptr, RD<V> *rd, int32_t n) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
        RD<V> e;
        e.r = (V)0;
        e.d = (V)(row_ptr[u + 1] - row_ptr[u]);
        rd[u] = e;
    }
}

// r <- b on supp(s); S_0 = supp(s) (forced, Definition 3.1); counters reset.
// A seed of at most kSeedInline entries arrives in the kernel arguments (inl.n
// > 0) instead of device buffers, which saves two host-to-device copies.
// sym_rp (row pointers, or null): the propagation matrix D^-1/2 A D^-1/2, solved
// in the A D^-1 form from the source D^1/2 s (Sec. 3.3), so s_u is scaled by
// sqrt(d_u) here and x_u by 1/sqrt(d_u) on output.
template <typename V>
__global__ void k_seed_init(RD<V> *rd, const int32_t *__restrict__ sidx, const double *__restrict__ sval, int32_t nnz,
                            SeedInline inl, double bscale, int32_t *f0, int32_t *touched0, int32_t *cstamp,
                            int32_t stamp0, uint32_t *tbm, DevState *st, const int32_t *__restrict__ sym_rp) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nnz) {
        const int32_t u = inl.n ? inl.idx[i] : sidx[i];
        double sv = inl.n ? inl.val[i] : sval[i];
        if (sym_rp) sv = sv * sqrt((double)(sym_rp[u + 1] - sym_rp[u]));
        rd[u].r = (V)(bscale * sv);
        f0[i] = u;
        if (touched0) touched0[i] = u;
        if (cstamp) cstamp[u] = stamp0;
        if (tbm) atomicOr(&tbm[u >> 5], 1u << (u & 31));
    }
    if (i == 0) {
        st->packed[0] = st->packed[1] = 0ull;
        st->fcount[0] = nnz;
        st->fcount[1] = 0;
        st->tcount[0] = touched0 ? nnz : 0;
        st->tcount[1] = st->tcount[2] = 0;
        st->iters = 0;
        st->ops = st->pushes = 0;
        st->res_l1 = 0.0;
        st->res_dinf = 0ull;
        st->out_count = 0;
        st->empty_seen = 0;
        st->probe = 0;
        st->overflow = 0;
        st->fused_stamp = 0;
    }
}

// ------------------------------------------------------------------ snapshot (A2 + A5)
// List discipline per iteration t (cur = t & 1, nxt = cur ^ 1): snap(t) reads
// list[cur] and may append to list[nxt]; push(t) appends to list[nxt] and then
// empties list[cur].  list[nxt] was emptied by push(t-1) (or by seed_init).
// Shared tail of every snap kernel: record u in the pushed set, reserve work-list
// slots and edge offsets for the active lanes of the wave, write the entries.
template <typename V>
__device__ __forceinline__ void emit_entries(bool act, int32_t u, int32_t beg, int32_t deg, V sv, uint32_t *bitmap,
                                             DevState *st, int cur, int32_t *wl_node,
                                             int32_t *wl_beg, int32_t *wl_off, V *wl_sv, int32_t *tile_start,
                                             int32_t *tr_nodes, long long push_base, long long tr_cap, int32_t cap) {
    // the pushed set, counted by the output kernels (no return value needed)
    if (act) atomicOr(&bitmap[u >> 5], 1u << (u & 31));
    const unsigned long long mine = act ? ((1ull << 32) | (unsigned long long)(unsigned)deg) : 0ull;
    const unsigned long long res = block_reserve64(mine, &st->packed[cur]);
    if (act) {
        const int slot = (int)(res >> 32);
        if (slot >= cap) { st->overflow = 1; return; }
        const int off = (int)(res & 0xffffffffull);
        wl_node[slot] = u;
        wl_beg[slot] = beg;
        wl_off[slot] = off;
        wl_sv[slot] = sv;
        for (int k = (off + kPushTile - 1) / kPushTile; (long long)k * kPushTile < (long long)off + deg; k++)
            tile_start[k] = slot;
        if (tr_nodes && push_base + slot < tr_cap) tr_nodes[push_base + slot] = u;
    }
}

// LocalGD: v = r_u, r_u = 0, x_u += v, scatter value W_u v with
// W_u = wscale / d_u (PPR, wscale = 1 - alpha) or wscale (Katz, beta).
template <typename V>
__device__ void snap_gd(const int32_t *__restrict__ row_ptr, RD<V> *rd, V *x, uint32_t *bitmap,
                        const int32_t *__restrict__ F, DevState *st, int cur, int32_t *wl_node,
                        int32_t *wl_beg, int32_t *wl_off, V *wl_sv, int32_t *tile_start, V wscale, int w_div_deg,
                        int32_t *tr_nodes, long long tr_cap, int32_t cap, int bid, int nblocks) {
    const int nxt = cur ^ 1;
    const int n_f = min(st->fcount[cur], cap);
    const long long push_base = st->pushes;
    const int stride = nblocks * blockDim.x;
    for (int base = bid * blockDim.x; base < n_f; base += stride) {
        int i = base + threadIdx.x;
        bool act = i < n_f;
        int32_t u = 0, beg = 0, deg = 0;
        V sv = (V)0;
        if (act) {
            u = F[i];
            // every load before the first store: one round trip, not three
            const V v = rd[u].r;
            const V xo = x[u];
            const int32_t rp0 = row_ptr[u], rp1 = row_ptr[u + 1];
            rd[u].r = (V)0;
            x[u] = xo + v;
            beg = rp0;
            deg = rp1 - rp0;
            V w = w_div_deg ? wscale / (V)deg : wscale;
            sv = w * v;
        }
        emit_entries<V>(act, u, beg, deg, sv, bitmap, st, cur, wl_node, wl_beg, wl_off, wl_sv, tile_start,
                        tr_nodes, push_base, tr_cap, cap);
    }
}

template <typename V>
__global__ void __launch_bounds__(kSnapBlock) k_snap_gd(const int32_t *__restrict__ row_ptr, RD<V> *rd, V *x,
                                                     uint32_t *bitmap, const int32_t *__restrict__ F, DevState *st,
                                                     int cur, int32_t *wl_node, int32_t *wl_beg,
                                                     int32_t *wl_off, V *wl_sv, int32_t *tile_start, V wscale,
                                                     int w_div_deg, int32_t *tr_nodes, long long tr_cap, int32_t cap) {
    snap_gd<V>(row_ptr, rd, x, bitmap, F, st, cur, wl_node, wl_beg, wl_off, wl_sv, tile_start, wscale,
               w_div_deg, tr_nodes, tr_cap, cap, blockIdx.x, gridDim.x);
}

// Heat kernel, level k: snapshot of S_k from plane k (scatter value
// (tau/(k+1)) v / d_u, no edges at the last level), plus the clean-up of plane
// k-1: its leftover residuals are folded into the reported norms
// (psi_{k-1}-weighted) and the plane is zeroed for reuse by level k+1.
template <typename V>
__global__ void __launch_bounds__(kSnapBlock) k_snap_hk(const int32_t *__restrict__ row_ptr, RD<V> *plane, RD<V> *prev,
                                                     V *x, uint32_t *bitmap, const int32_t *__restrict__ F,
                                                     DevState *st, int cur, int32_t *wl_node,
                                                     int32_t *wl_beg, int32_t *wl_off, V *wl_sv,
                                                     int32_t *tile_start, V wmul, int last_level, int frontier_on,
                                                     const int32_t *__restrict__ prev_touched, int prev_tslot,
                                                     int next_tslot, double psi_prev, double wdinf_prev,
                                                     int32_t *tr_nodes, long long tr_cap, int32_t cap) {
    const int nxt = cur ^ 1;
    const int n_f = frontier_on ? min(st->fcount[cur], cap) : 0;
    const int n_c = prev_touched ? min(st->tcount[prev_tslot], cap) : 0;
    const long long push_base = st->pushes;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->packed[nxt] = 0ull;
        if (next_tslot >= 0) st->tcount[next_tslot] = 0;
    }
    const int stride = gridDim.x * blockDim.x;
    for (int base = blockIdx.x * blockDim.x; base < n_f; base += stride) {
        int i = base + threadIdx.x;
        bool act = i < n_f;
        int32_t u = 0, beg = 0, deg = 0;
        V sv = (V)0;
        if (act) {
            u = F[i];
            // every load before the first store: one round trip, not three
            const RD<V> e = plane[u];
            const V xo = x[u];
            const int32_t rp0 = row_ptr[u], rp1 = row_ptr[u + 1];
            plane[u].r = (V)0;
            x[u] = xo + e.r;
            beg = rp0;
            deg = rp1 - rp0;
            sv = last_level ? (V)0 : wmul * e.r / e.d;
        }
        emit_entries<V>(act, u, beg, deg, sv, bitmap, st, cur, wl_node, wl_beg, wl_off, wl_sv, tile_start,
                        tr_nodes, push_base, tr_cap, cap);
    }
    double l1 = 0.0, mx = 0.0;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n_c; j += stride) {
        int32_t w = prev_touched[j];
        V val = prev[w].r;
        prev[w].r = (V)0;
        double a = fabs((double)val);
        l1 += psi_prev * a;
        if (a > 0.0) mx = fmax(mx, wdinf_prev * a / (double)prev[w].d);
    }
    if (prev_touched) block_fold_norms(l1, mx, st);
}

// LocalCH: over the candidates C_t, S_t = {u : r_u != 0, |r_u| >= theta_u}
// (all of C_0 = supp(s) at t = 0); h_u = c_t r_u + m_t Delta_u with Delta_u
// the previous update if u was in S_{t-1}; x_u += h_u, r_u -= h_u, Delta_u = h_u.
template <typename V>
__device__ void snap_ch(const int32_t *__restrict__ row_ptr, RD<V> *rd, V *x, uint32_t *bitmap,
                        const int32_t *__restrict__ C, DevState *st, int cur, int32_t *wl_node,
                        int32_t *wl_beg, int32_t *wl_off, V *wl_sv, int32_t *tile_start, V wscale, int w_div_deg,
                        V eps_eff, V c_t, V m_t, int force, V *delta, int32_t *dstamp, int32_t *cstamp,
                        int32_t stamp_cur, int32_t *next_list, int32_t *tr_nodes, long long tr_cap, int32_t cap,
                        int bid, int nblocks) {
    const int nxt = cur ^ 1;
    // the range reduction of t-1 may have taken this snapshot already (binned
    // iteration with a fused reduction): then the candidate list is spent
    const bool fused = st->fused_stamp == stamp_cur;
    const int n_c = fused ? 0 : min(st->fcount[cur], cap);
    const long long push_base = st->pushes;
    const int stride = nblocks * blockDim.x;
    for (int base = bid * blockDim.x; base < n_c; base += stride) {
        int i = base + threadIdx.x;
        bool valid = i < n_c;
        bool act = false;
        int32_t u = 0, beg = 0, deg = 0;
        V sv = (V)0;
        if (valid) {
            u = C[i];
            RD<V> e = rd[u];
            act = force || (e.r != (V)0 && fabs(e.r) >= eps_eff * e.d);
            if (act) {
                // the node's other state in one round of loads (Delta is read even
                // when its stamp will say it is stale)
                const int32_t ds = dstamp[u];
                const V dl = delta[u];
                const V xo = x[u];
                const int32_t rp0 = row_ptr[u], rp1 = row_ptr[u + 1];
                V h = force ? e.r : c_t * e.r + m_t * (ds == stamp_cur - 1 ? dl : (V)0);
                x[u] = xo + h;
                rd[u].r = e.r - h;
                delta[u] = h;
                dstamp[u] = stamp_cur;
                beg = rp0;
                deg = rp1 - rp0;
                V w = w_div_deg ? wscale / (V)deg : wscale;
                sv = w * h;
            }
        }
        // u's own residual changed: it is a candidate of the next iteration.  u appears
        // once in C_t and only this iteration's push stamps stamp_cur + 1, later: a
        // plain store marks it
        const bool mark = act;
        if (act) cstamp[u] = stamp_cur + 1;
        block_list_append(mark, u, &st->fcount[nxt], next_list, cap, st);
        emit_entries<V>(act, u, beg, deg, sv, bitmap, st, cur, wl_node, wl_beg, wl_off, wl_sv, tile_start,
                        tr_nodes, push_base, tr_cap, cap);
    }
}

template <typename V>
__global__ void __launch_bounds__(kSnapBlock) k_snap_ch(const int32_t *__restrict__ row_ptr, RD<V> *rd, V *x,
                                                     uint32_t *bitmap, const int32_t *__restrict__ C, DevState *st,
                                                     int cur, int32_t *wl_node, int32_t *wl_beg,
                                                     int32_t *wl_off, V *wl_sv, int32_t *tile_start, V wscale,
                                                     int w_div_deg, V eps_eff, V c_t, V m_t, int force, V *delta,
                                                     int32_t *dstamp, int32_t *cstamp, int32_t stamp_cur,
                                                     int32_t *next_list, int32_t *tr_nodes, long long tr_cap,
                                                     int32_t cap) {
    snap_ch<V>(row_ptr, rd, x, bitmap, C, st, cur, wl_node, wl_beg, wl_off, wl_sv, tile_start, wscale,
               w_div_deg, eps_eff, c_t, m_t, force, delta, dstamp, cstamp, stamp_cur, next_list, tr_nodes, tr_cap, cap,
               blockIdx.x, gridDim.x);
}

// ------------------------------------------------------------------ push (A3 + A4)
// MODE 0: LocalGD / monotone residual -- returned old value, crossing test.
// MODE 1: heat kernel -- crossing test on plane k+1 and first-touch list.
// MODE 2: LocalCH -- signed add, candidate marking by stamp.
// A workgroup of kPushBlock threads takes one tile of kPushTile edges; each
// thread owns kPer edges strided by kPushBlock (coalesced col_idx reads) and
// issues their loads, then their atomics, before waiting on any of them.
// tbm (MODE 0 and 2): the set of nodes whose residual may be nonzero; a node is
// added when an add finds its residual at zero (MODE 0) or when it is first
// marked as a candidate in an iteration (MODE 2).
// Gather of one tile of M base tiles (M * kPushTile edges): the work-list
// entries of the tile staged in LDS, then for each of the thread's M edges
// (strided by kPushBlock) the entry by binary search and the destination from
// col_idx (w = -1 past the end).  Returns false, with the overflow flag set, on
// a broken work list.  Every thread of the workgroup calls it (it holds barriers).
template <typename V>
__device__ __forceinline__ bool gather_tile(int tile, int M, int nbase, int count, int total, int32_t cap,
                                            int32_t nnz, const int32_t *__restrict__ tile_start,
                                            const int32_t *__restrict__ wl_off, const int32_t *__restrict__ wl_beg,
                                            const V *__restrict__ wl_sv, const int32_t *__restrict__ col_idx,
                                            int32_t *s_off, int32_t *s_beg, V *s_sv, DevState *st,
                                            int32_t (&w)[kMacroTiles], V (&dv)[kMacroTiles],
                                            const int32_t *__restrict__ wl_node, int32_t (&su)[kMacroTiles]) {
#pragma unroll
    for (int q = 0; q < kMacroTiles; q++) {
        w[q] = -1;
        dv[q] = (V)0;
        su[q] = -1;
    }
    const int b0 = tile * M;
    const int e0 = b0 * kPushTile;
    const int e1 = min(e0 + M * kPushTile, total);
    const int i0 = tile_start[b0];
    const int i1 = (b0 + M < nbase) ? tile_start[b0 + M] : count - 1;
    const int m = min(i1 - i0 + 1, kMacroTiles * kPushTile + 1);
    if (m <= 0 || i0 < 0 || i1 >= cap) {  // a broken work list: never index with it
        if (threadIdx.x == 0) st->overflow = 1;
        return false;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < m; j += blockDim.x) {
        s_off[j] = wl_off[i0 + j];
        s_beg[j] = wl_beg[i0 + j];
        s_sv[j] = wl_sv[i0 + j];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kMacroTiles; q++) {
        const int e = e0 + q * kPushBlock + threadIdx.x;
        if (q < M && e < e1) {
            int lo = 0, hi = m - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_off[mid] <= e) lo = mid; else hi = mid - 1;
            }
            const int k = s_beg[lo] + (e - s_off[lo]);
            if (k >= 0 && k < nnz) {
                w[q] = col_idx[k];
                dv[q] = s_sv[lo];
            } else {
                st->overflow = 1;
            }
            // the first edge of an entry also names the entry's node (LocalCH self-marks)
            if (wl_node && e == s_off[lo]) su[q] = wl_node[i0 + lo];
        }
    }
    return true;
}

template <typename V, int MODE>
__device__ void push_edges(const int32_t *__restrict__ col_idx, RD<V> *dst, DevState *st, int cur,
                           const int32_t *__restrict__ wl_beg, const int32_t *__restrict__ wl_off,
                           const V *__restrict__ wl_sv, const int32_t *__restrict__ tile_start, V eps_eff,
                           int32_t *next_list, int32_t *touched, int tslot, int32_t *cstamp, int32_t stamp_next,
                           uint32_t *tbm, long long *tr_size, long long *tr_vol, long long tr_cap, int scatter,
                           int32_t cap, int32_t nnz, const BinArgs<V> &bins, const int32_t *wl_node, int self_marks,
                           int bid, int nblocks) {
    constexpr int kPer = kMacroTiles;  // edges per thread in a tile of kMacroTiles base tiles
    static_assert(kPushTile == kPushBlock, "a base tile holds one edge per thread");
    __shared__ int32_t s_off[kMacroTiles * kPushTile + 1];
    __shared__ int32_t s_beg[kMacroTiles * kPushTile + 1];
    __shared__ V s_sv[kMacroTiles * kPushTile + 1];
    extern __shared__ int32_t s_bin[];  // binned scatter: [nranges] counts, then [nranges] bases
    const int nxt = cur ^ 1;
    const unsigned long long pk = st->packed[cur];
    const int count = min((int)(pk >> 32), cap);
    const int total = (int)(pk & 0xffffffffull);
    // S_t (or C_t) has been consumed by the snapshot: its list becomes the
    // next-but-one append target, which the snapshot of t+1 may append to.  The
    // reservation counter of t+1 is cleared here (the snapshot of t+1 may run in
    // the range reduction of t, whose other workgroups still read the one of t).
    if (bid == 0 && threadIdx.x == 0) {
        st->fcount[cur] = 0;
        st->packed[nxt] = 0ull;
    }
    if (bid == 0 && threadIdx.x == 0 && count == 0) st->empty_seen = 1;
    if (bid == 0 && threadIdx.x == 0 && count > 0) {
        int it = st->iters;
        if (tr_size && it < tr_cap) {
            tr_size[it] = count;
            tr_vol[it] = total;
        }
        st->ops += total;
        st->pushes += count;
        st->iters = it + 1;
    }
    // tiles: kMacroTiles base tiles (kMacroTiles edges per thread, loads issued
    // together) for a large frontier, one base tile (one edge per thread, four
    // times as many workgroups) otherwise
    const int nbase = scatter ? (total + kPushTile - 1) / kPushTile : 0;
    const int M = (long long)total >= kMacroMinEdges ? kMacroTiles : 1;
    const int ntiles = (nbase + M - 1) / M;
    // large frontier: write the updates into the destination-range bins (summed
    // by k_reduce); small frontier: atomic scatter with the crossing test here
    const bool binned = bins.nranges > 0 && (long long)total >= bins.min_edges && scatter;
    int32_t *s_cnt = s_bin;
    int32_t *s_rbase = s_bin + bins.nranges;
    if (binned)
        for (int r = threadIdx.x; r < bins.nranges; r += blockDim.x) s_cnt[r] = 0;
    for (int tile = bid; tile < ntiles; tile += nblocks) {
        int32_t w[kPer], su[kPer];
        V dv[kPer];
        bool hit[kPer], first[kPer];
#pragma unroll
        for (int q = 0; q < kPer; q++) hit[q] = first[q] = false;
        const bool marks = MODE == 2 && binned && self_marks;
        if (!gather_tile<V>(tile, M, nbase, count, total, cap, nnz, tile_start, wl_off, wl_beg, wl_sv, col_idx,
                            s_off, s_beg, s_sv, st, w, dv, marks ? wl_node : nullptr, su))
            continue;
        if (binned) {
            // rank of each update inside its range for this tile (LDS), one global
            // reservation per nonempty range, then the writes; LocalCH with a fused
            // reduction also bins each node of S_t once, flagged, with value zero
            int rb[kPer], rk[kPer], sb[kPer], sk[kPer];
#pragma unroll
            for (int q = 0; q < kPer; q++) {
                rb[q] = sb[q] = -1;
                rk[q] = sk[q] = 0;
                if (w[q] >= 0 && (MODE == 2 || dv[q] != (V)0)) {
                    rb[q] = w[q] >> bins.shift;
                    rk[q] = atomicAdd(&s_cnt[rb[q]], 1);
                }
                if (su[q] >= 0) {
                    sb[q] = su[q] >> bins.shift;
                    sk[q] = atomicAdd(&s_cnt[sb[q]], 1);
                }
            }
            __syncthreads();
            for (int r = threadIdx.x; r < bins.nranges; r += blockDim.x) {
                const int c = s_cnt[r];
                if (c) {
                    s_rbase[r] = atomicAdd(&bins.cursor[r], c);
                    s_cnt[r] = 0;
                }
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < kPer; q++) {
                if (rb[q] >= 0) {
                    const long long pos = bins.base[rb[q]] + s_rbase[rb[q]] + rk[q];
                    if (pos < bins.base[rb[q] + 1]) {
                        BinEnt<V> e;
                        e.w = w[q];
                        e.v = dv[q];
                        bins.be[pos] = e;
                    } else {
                        st->overflow = 1;
                    }
                }
                if (sb[q] >= 0) {
                    const long long pos = bins.base[sb[q]] + s_rbase[sb[q]] + sk[q];
                    if (pos < bins.base[sb[q] + 1]) {
                        BinEnt<V> e;
                        e.w = (int32_t)((uint32_t)su[q] | kSelfMarkBit);
                        e.v = (V)0;
                        bins.be[pos] = e;
                    } else {
                        st->overflow = 1;
                    }
                }
            }
            continue;
        }
        if (MODE == 2) {
            // signed residuals: w is a candidate of t+1 when an update lifts |r_w|
            // across its threshold (every other node stays below it: the nodes of S_t
            // were made candidates by the snapshot), deduplicated by the stamp; a
            // first touch marks the touched bitmap
            V th[kPer], old[kPer];
#pragma unroll
            for (int q = 0; q < kPer; q++)  // d is read-only during the push
                th[q] = w[q] >= 0 ? eps_eff * dst[w[q]].d : (V)0;
#pragma unroll
            for (int q = 0; q < kPer; q++)
                old[q] = w[q] >= 0 ? unsafeAtomicAdd(&dst[w[q]].r, dv[q]) : (V)0;
#pragma unroll
            for (int q = 0; q < kPer; q++) {
                if (w[q] < 0) continue;
                const V nw = old[q] + dv[q];
                hit[q] = fabs(old[q]) < th[q] && fabs(nw) >= th[q] && cstamp[w[q]] != stamp_next &&
                         atomicExch(&cstamp[w[q]], stamp_next) != stamp_next;
                if (tbm && old[q] == (V)0 && dv[q] != (V)0) atomicOr(&tbm[w[q] >> 5], 1u << (w[q] & 31));
            }
        } else {
            V th[kPer], old[kPer];
#pragma unroll
            for (int q = 0; q < kPer; q++)  // d is read-only during the push
                th[q] = (w[q] >= 0 && dv[q] != (V)0) ? eps_eff * dst[w[q]].d : (V)0;
#pragma unroll
            for (int q = 0; q < kPer; q++)
                old[q] = (w[q] >= 0 && dv[q] != (V)0) ? unsafeAtomicAdd(&dst[w[q]].r, dv[q]) : (V)0;
#pragma unroll
            for (int q = 0; q < kPer; q++) {
                if (w[q] >= 0 && dv[q] != (V)0) {
                    hit[q] = (old[q] < th[q]) && (old[q] + dv[q] >= th[q]);
                    first[q] = old[q] == (V)0;
                    if (MODE == 0 && first[q] && tbm) atomicOr(&tbm[w[q] >> 5], 1u << (w[q] & 31));
                }
            }
        }
        int nh = 0;
#pragma unroll
        for (int q = 0; q < kPer; q++) nh += hit[q] ? 1 : 0;
        int slot = block_reserve(nh, &st->fcount[nxt]);
#pragma unroll
        for (int q = 0; q < kPer; q++)
            if (hit[q]) {
                if (slot < cap) next_list[slot] = w[q];
                else st->overflow = 1;
                slot++;
            }
        if (MODE == 1) {
            int nf = 0;
#pragma unroll
            for (int q = 0; q < kPer; q++) nf += first[q] ? 1 : 0;
            int ts = block_reserve(nf, &st->tcount[tslot]);
#pragma unroll
            for (int q = 0; q < kPer; q++)
                if (first[q]) {
                    if (ts < cap) touched[ts] = w[q];
                    else st->overflow = 1;
                    ts++;
                }
        }
    }
}

template <typename V, int MODE>
__global__ void __launch_bounds__(kPushBlock) k_push(const int32_t *__restrict__ col_idx, RD<V> *dst, DevState *st,
                                                      int cur, const int32_t *__restrict__ wl_beg,
                                                      const int32_t *__restrict__ wl_off, const V *__restrict__ wl_sv,
                                                      const int32_t *__restrict__ tile_start, V eps_eff,
                                                      int32_t *next_list, int32_t *touched, int tslot,
                                                      int32_t *cstamp, int32_t stamp_next, uint32_t *tbm,
                                                      long long *tr_size, long long *tr_vol, long long tr_cap,
                                                      int scatter, int32_t cap, int32_t nnz, BinArgs<V> bins,
                                                      const int32_t *wl_node, int self_marks) {
    push_edges<V, MODE>(col_idx, dst, st, cur, wl_beg, wl_off, wl_sv, tile_start, eps_eff, next_list, touched, tslot,
                        cstamp, stamp_next, tbm, tr_size, tr_vol, tr_cap, scatter, cap, nnz, bins, wl_node, self_marks,
                        blockIdx.x, gridDim.x);
}

// Small frontiers: iterations t0 .. t_end-1 of LocalGD (CH = false) or LocalCH
// run by ONE workgroup in one launch.  The frontier / candidate lists, the work
// list (row start, edge offset, scatter value) and every counter live in LDS;
// global memory is touched only for node state (r, d, x, Delta, stamps, the
// pushed and touched bitmaps), the CSR, and fire-and-forget copies of the next
// list that a grid-wide continuation reads.  Every access comes from this one
// workgroup, so a workgroup barrier (with its workgroup-scope fences) stands
// where a kernel boundary would be: the stores of the snapshot are ordered
// before the adds of the push, and the adds before the next snapshot, which
// reads r past L1 because atomics are performed in L2.  No device-scope fence
// (an L2 write-back on this part) is needed inside the loop.  The arithmetic
// and every decision are those of snap_gd / snap_ch followed by push_edges,
// iteration by iteration.
//
// The launch stops before the snapshot of t when the list of t exceeds
// kSmallMaxNodes (small_phase 0: the list is in global memory), after the
// snapshot when vol(S_t) exceeds kSmallMaxEdges (small_phase 1: the work list,
// its tile table and packed[t & 1] are written out for the grid-wide push of
// t), or when the iteration converges; small_t records where.
__device__ __forceinline__ unsigned long long block_excl_scan64(unsigned long long v, unsigned long long *total) {
    __shared__ unsigned long long s_w[kMaxWaves];
    __shared__ unsigned long long s_tot;
    const unsigned long long incl = wave_incl_scan64(v);
    const int wid = threadIdx.x / kWave;
    if (lane() == kWave - 1) s_w[wid] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tot = 0ull;
        for (int i = 0; i < (int)(blockDim.x / kWave); i++) {
            const unsigned long long x = s_w[i];
            s_w[i] = tot;
            tot += x;
        }
        s_tot = tot;
    }
    __syncthreads();
    const unsigned long long r = s_w[wid] + incl - v;
    *total = s_tot;
    __syncthreads();
    return r;
}

// Stages a touched-bitmap mark in LDS; a full stage marks at once instead.
__device__ __forceinline__ void small_mark_later(int32_t w, uint32_t *tbm, int32_t *pend, int *npend) {
    const int i = atomicAdd(npend, 1);
    if (i < kSmallPendMarks) pend[i] = w;
    else atomicOr(&tbm[w >> 5], 1u << (w & 31));
}

template <typename V, bool CH>
__global__ void __launch_bounds__(kSnapBlock) k_small(SmallArgs<V> a) {
    constexpr int kNodesPer = kSmallMaxNodes / kSnapBlock;  // list entries per thread in the snapshot
    constexpr int kEdgesPer = 4;                            // edges per thread and push round
    static_assert(kNodesPer * kSnapBlock == kSmallMaxNodes, "list entries must split evenly");
    __shared__ int32_t s_list[2][kSmallMaxNodes];
    __shared__ int32_t s_beg[kSmallMaxNodes];
    __shared__ int32_t s_off[kSmallMaxNodes + 1];
    __shared__ V s_sv[kSmallMaxNodes];
    __shared__ int s_cnt[2];
    __shared__ int s_ovf;
    // touched-bitmap marks of a push, issued after the fence that ends it (the
    // fence would otherwise wait for these memory-side atomics)
    __shared__ int32_t s_tpend[kSmallPendMarks];
    __shared__ int s_tpn;
    DevState *st = a.st;
    RD<V> *rd = (RD<V> *)a.rd;
    V *x = (V *)a.x;
    V *delta = (V *)a.delta;
    const int tid = threadIdx.x;
    // iteration counters: thread 0 keeps them and writes them back at the end
    int iters = 0;
    long long ops = 0, pushes = 0;
    if (tid == 0) {
        iters = st->iters;
        ops = st->ops;
        pushes = st->pushes;
        s_cnt[0] = st->fcount[0];
        s_cnt[1] = st->fcount[1];
        s_ovf = 0;
        s_tpn = 0;
    }
    __syncthreads();
    int t = a.t0;
    int phase = 0;
    bool empty_seen = false;
    {
        const int c0 = s_cnt[t & 1];
        const int32_t *F = (t & 1) ? a.front1 : a.front0;
        if (c0 <= kSmallMaxNodes)
            for (int i = tid; i < c0; i += blockDim.x) s_list[t & 1][i] = F[i];
    }
    __syncthreads();
    __shared__ long long s_push_base;
    for (; t < a.t_end; t++) {
        const int cur = t & 1, nxt = cur ^ 1;
        int32_t *Fn = nxt ? a.front1 : a.front0;
        const int n_f = s_cnt[cur];
        {
            const int np = min(s_tpn, kSmallPendMarks);
            for (int i = tid; i < np; i += blockDim.x)
                atomicOr(&a.tbm[s_tpend[i] >> 5], 1u << (s_tpend[i] & 31));
        }
        __syncthreads();
        if (tid == 0) s_tpn = 0;
        if (n_f > kSmallMaxNodes) break;
        if (tid == 0) s_push_base = pushes;
        // ---------------------------------------------------------- snapshot of t
        const V c_t = CH ? a.c_seq[t - a.t0] : (V)0;
        const V m_t = CH ? a.m_seq[t - a.t0] : (V)0;
        const bool force = CH && t == 0;
        const int32_t stamp_cur = a.stamp_base + t;
        int32_t u[kNodesPer], beg[kNodesPer], deg[kNodesPer];
        bool act[kNodesPer];
        V sv[kNodesPer];
        unsigned long long mine = 0ull;
#pragma unroll
        for (int k = 0; k < kNodesPer; k++) {
            const int i = tid * kNodesPer + k;
            act[k] = false;
            u[k] = 0;
            beg[k] = deg[k] = 0;
            sv[k] = (V)0;
            if (i < n_f) u[k] = s_list[cur][i];
        }
        // every load of the entries is issued before any is used
        RD<V> e[kNodesPer];
        V xo[kNodesPer], dl[kNodesPer];
        int32_t ds[kNodesPer], rp0[kNodesPer], rp1[kNodesPer];
#pragma unroll
        for (int k = 0; k < kNodesPer; k++) {
            const bool v = tid * kNodesPer + k < n_f;
            // r is updated by atomics, which are performed in L2: read it past L1
            e[k].r = v ? __hip_atomic_load(&rd[u[k]].r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : (V)0;
            e[k].d = v ? rd[u[k]].d : (V)0;
            xo[k] = v ? x[u[k]] : (V)0;
            rp0[k] = v ? a.row_ptr[u[k]] : 0;
            rp1[k] = v ? a.row_ptr[u[k] + 1] : 0;
            ds[k] = (CH && v) ? a.dstamp[u[k]] : 0;
            dl[k] = (CH && v) ? delta[u[k]] : (V)0;
        }
#pragma unroll
        for (int k = 0; k < kNodesPer; k++) {
            if (tid * kNodesPer + k >= n_f) continue;
            V h;
            if (CH) {
                act[k] = force || (e[k].r != (V)0 && fabs(e[k].r) >= a.eps_eff * e[k].d);
                if (!act[k]) continue;
                h = force ? e[k].r : c_t * e[k].r + m_t * (ds[k] == stamp_cur - 1 ? dl[k] : (V)0);
                rd[u[k]].r = e[k].r - h;
                delta[u[k]] = h;
                a.dstamp[u[k]] = stamp_cur;
                a.cstamp[u[k]] = stamp_cur + 1;  // u's residual changed: a candidate of t+1
            } else {
                act[k] = true;
                h = e[k].r;
                rd[u[k]].r = (V)0;
            }
            x[u[k]] = xo[k] + h;
            beg[k] = rp0[k];
            deg[k] = rp1[k] - rp0[k];
            const V w = a.w_div_deg ? a.wscale / (V)deg[k] : a.wscale;
            sv[k] = w * h;
            mine += (1ull << 32) | (unsigned long long)(unsigned)deg[k];
        }
        unsigned long long tot;
        const unsigned long long pre = block_excl_scan64(mine, &tot);
        const int count = (int)(tot >> 32);
        const int total = (int)(tot & 0xffffffffull);
        {
            int slot = (int)(pre >> 32);
            int off = (int)(pre & 0xffffffffull);
            const long long pb = s_push_base;
#pragma unroll
            for (int k = 0; k < kNodesPer; k++) {
                if (!act[k]) continue;
                s_beg[slot] = beg[k];
                s_off[slot] = off;
                s_sv[slot] = sv[k];
                if (a.tr_nodes && pb + slot < a.tr_ncap) a.tr_nodes[pb + slot] = u[k];
                if (CH) {  // self-mark into the candidates of t+1
                    const int c = atomicAdd(&s_cnt[nxt], 1);
                    if (c < kSmallMaxNodes) s_list[nxt][c] = u[k];
                    if (c < a.cap) Fn[c] = u[k];
                    else s_ovf = 1;
                }
                slot++;
                off += deg[k];
            }
        }
        if (tid == 0) s_off[count] = total;
        __syncthreads();
        // the pushed set (read only by the output kernels): marked after the fence
#pragma unroll
        for (int k = 0; k < kNodesPer; k++)
            if (act[k]) atomicOr(&a.bitmap[u[k] >> 5], 1u << (u[k] & 31));
        if (count > 0 && (long long)total > kSmallMaxEdges) {
            // hand the push of t to the grid-wide kernel: work list, tile table, counters
            for (int i = tid; i < count; i += blockDim.x) {
                const int off = s_off[i], d = s_off[i + 1] - off;
                a.wl_beg[i] = s_beg[i];
                a.wl_off[i] = off;
                ((V *)a.wl_sv)[i] = s_sv[i];
                for (int k = (off + kPushTile - 1) / kPushTile; (long long)k * kPushTile < (long long)off + d; k++)
                    a.tile_start[k] = i;
            }
            if (tid == 0) {
                st->packed[cur] = ((unsigned long long)count << 32) | (unsigned long long)(unsigned)total;
                st->packed[nxt] = 0ull;
            }
            phase = 1;
            break;
        }
        // ---------------------------------------------------------- push of t
        const int32_t stamp_next = stamp_cur + 1;
        for (int e0 = 0; e0 < total; e0 += kEdgesPer * (int)blockDim.x) {
            int32_t w[kEdgesPer];
            V dv[kEdgesPer];
#pragma unroll
            for (int q = 0; q < kEdgesPer; q++) {
                const int ee = e0 + q * (int)blockDim.x + tid;
                w[q] = -1;
                dv[q] = (V)0;
                if (ee < total) {
                    int lo = 0, hi = count - 1;
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (s_off[mid] <= ee) lo = mid; else hi = mid - 1;
                    }
                    const int kk = s_beg[lo] + (ee - s_off[lo]);
                    if (kk >= 0 && kk < a.nnz) {
                        w[q] = a.col_idx[kk];
                        dv[q] = s_sv[lo];
                    } else {
                        s_ovf = 1;
                    }
                }
            }
            bool hit[kEdgesPer];
            if (CH) {  // signed residuals: |r_w| lifted across the threshold (see k_push)
                V th[kEdgesPer], old[kEdgesPer];
#pragma unroll
                for (int q = 0; q < kEdgesPer; q++) th[q] = w[q] >= 0 ? a.eps_eff * rd[w[q]].d : (V)0;
#pragma unroll
                for (int q = 0; q < kEdgesPer; q++) old[q] = w[q] >= 0 ? unsafeAtomicAdd(&rd[w[q]].r, dv[q]) : (V)0;
#pragma unroll
                for (int q = 0; q < kEdgesPer; q++) {
                    hit[q] = false;
                    if (w[q] < 0) continue;
                    const V nw = old[q] + dv[q];
                    hit[q] = fabs(old[q]) < th[q] && fabs(nw) >= th[q] && a.cstamp[w[q]] != stamp_next &&
                             atomicExch(&a.cstamp[w[q]], stamp_next) != stamp_next;
                    if (old[q] == (V)0 && dv[q] != (V)0) small_mark_later(w[q], a.tbm, s_tpend, &s_tpn);
                }
            } else {
                V th[kEdgesPer], old[kEdgesPer];
#pragma unroll
                for (int q = 0; q < kEdgesPer; q++)
                    th[q] = (w[q] >= 0 && dv[q] != (V)0) ? a.eps_eff * rd[w[q]].d : (V)0;
#pragma unroll
                for (int q = 0; q < kEdgesPer; q++)
                    old[q] = (w[q] >= 0 && dv[q] != (V)0) ? unsafeAtomicAdd(&rd[w[q]].r, dv[q]) : (V)0;
#pragma unroll
                for (int q = 0; q < kEdgesPer; q++) {
                    hit[q] = false;
                    if (w[q] >= 0 && dv[q] != (V)0) {
                        hit[q] = (old[q] < th[q]) && (old[q] + dv[q] >= th[q]);
                        if (old[q] == (V)0) small_mark_later(w[q], a.tbm, s_tpend, &s_tpn);
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < kEdgesPer; q++)
                if (hit[q]) {
                    const int c = atomicAdd(&s_cnt[nxt], 1);
                    if (c < kSmallMaxNodes) s_list[nxt][c] = w[q];
                    if (c < a.cap) Fn[c] = w[q];
                    else s_ovf = 1;
                }
        }
        __syncthreads();
        if (tid == 0) {
            if (count > 0) {
                if (a.tr_size && iters < a.tr_cap) {
                    a.tr_size[iters] = count;
                    a.tr_vol[iters] = total;
                }
                ops += total;
                pushes += count;
                iters++;
            }
            s_cnt[cur] = 0;  // S_t consumed: the list becomes the append target of t+1
        }
        __syncthreads();
        if (count == 0) {  // S_t was empty: converged
            empty_seen = true;
            t++;
            break;
        }
        if (!CH && s_cnt[nxt] == 0) {  // LocalGD: S_{t+1} is empty
            t++;
            break;
        }
    }
    __syncthreads();
    {
        const int np = min(s_tpn, kSmallPendMarks);
        for (int i = tid; i < np; i += blockDim.x) atomicOr(&a.tbm[s_tpend[i] >> 5], 1u << (s_tpend[i] & 31));
    }
    if (tid == 0) {
        st->iters = iters;
        st->ops = ops;
        st->pushes = pushes;
        st->fcount[0] = s_cnt[0];
        st->fcount[1] = s_cnt[1];
        if (phase == 0) st->packed[0] = st->packed[1] = 0ull;
        if (empty_seen) st->empty_seen = 1;
        if (s_ovf) st->overflow = 1;
        st->small_t = t;
        st->small_phase = phase;
    }
}

template <typename V>
void launch_small(const SmallArgs<V> &a, bool ch, hipStream_t s) {
    if (ch) hipLaunchKernelGGL((k_small<V, true>), dim3(1), dim3(kSnapBlock), 0, s, a);
    else hipLaunchKernelGGL((k_small<V, false>), dim3(1), dim3(kSnapBlock), 0, s, a);
}

// Binned scatter, second half: workgroup r sums the updates of bin r into an
// LDS accumulator over its node range, then applies each touched node's total
// once: r_w += sum, with the tests of the atomic scatter (MODE 0/1: the
// crossing test, and first touch when the old residual was zero; MODE 2: w
// becomes a candidate of t+1 only if its final residual passes the threshold,
// since no later add of this iteration can change it).  Each node belongs to one range, so the updates of r_w,
// the stamps and the bitmap words of the range need no global atomics.  Every
// thread owns kRedPer consecutive nodes of the range; appends are aggregated
// per workgroup.  The bin cursor is reset for the next iteration.
template <typename V, int MODE>
__global__ void __launch_bounds__(kReduceBlock) k_reduce(BinArgs<V> bins, RD<V> *dst, DevState *st, int cur,
                                                          V eps_eff, int32_t *next_list, int32_t *touched, int tslot,
                                                          int32_t *cstamp, int32_t stamp_next, uint32_t *tbm,
                                                          int scatter, int32_t cap, int32_t n, FuseArgs<V> fz) {
    // 16-byte aligned: the FP64 accumulator takes 64-bit LDS atomics, which need natural alignment
    extern __shared__ __attribute__((aligned(16))) unsigned char s_red[];
    const int span_max = 1 << bins.shift;
    V *s_acc = (V *)s_red;
    uint32_t *s_bits = (uint32_t *)(s_acc + span_max);
    uint32_t *s_self = s_bits + span_max / 32;  // LocalCH fused: nodes of S_t (flagged bin entries)
    const int total = (int)(st->packed[cur] & 0xffffffffull);
    if (!(bins.nranges > 0 && (long long)total >= bins.min_edges && scatter)) {
        // an atomic iteration: with a fused reduction the snapshot of t+1 is taken
        // here over its list, so that no separate launch is needed
        if (MODE == 0 && fz.on)
            snap_gd<V>(fz.row_ptr, dst, fz.x, fz.bitmap, next_list, st, cur ^ 1, fz.wl_node, fz.wl_beg, fz.wl_off,
                       fz.wl_sv, fz.tile_start, fz.wscale, fz.w_div_deg, fz.tr_nodes, fz.tr_cap, fz.cap, blockIdx.x,
                       gridDim.x);
        if (MODE == 2 && fz.on)
            snap_ch<V>(fz.row_ptr, dst, fz.x, fz.bitmap, next_list, st, cur ^ 1, fz.wl_node, fz.wl_beg, fz.wl_off,
                       fz.wl_sv, fz.tile_start, fz.wscale, fz.w_div_deg, eps_eff, fz.c_next, fz.m_next, 0, fz.delta,
                       fz.dstamp, cstamp, stamp_next, fz.list2, fz.tr_nodes, fz.tr_cap, fz.cap, blockIdx.x,
                       gridDim.x);
        return;
    }
    const int r = blockIdx.x;
    const int lo = r << bins.shift;
    const int span = min(span_max, n - lo);
    // one thread reads the bin's cursor, hands it on through LDS and resets it
    // (a load by every thread could still be in flight at the reset)
    __shared__ int s_cnt0;
    if (threadIdx.x == 0) {
        s_cnt0 = bins.cursor[r];
        bins.cursor[r] = 0;
    }
    const long long b0 = bins.base[r];
    const long long avail = bins.base[r + 1] - b0;
    for (int j = threadIdx.x; j < span_max; j += blockDim.x) s_acc[j] = (V)0;
    for (int j = threadIdx.x; j < span_max / 32; j += blockDim.x) s_bits[j] = s_self[j] = 0u;
    __syncthreads();
    const int cnt = s_cnt0;
    const int m = (int)min((long long)cnt, avail);
    constexpr int kRedUnroll = 4;  // bin entries per thread and step, loaded before any LDS update
    for (int i0 = 0; i0 < m; i0 += kRedUnroll * (int)blockDim.x) {
        int jj[kRedUnroll];
        V vv[kRedUnroll];
        bool ok[kRedUnroll], self[kRedUnroll];
#pragma unroll
        for (int q = 0; q < kRedUnroll; q++) {
            const int i = i0 + q * (int)blockDim.x + (int)threadIdx.x;
            ok[q] = i < m;
            BinEnt<V> e{};
            if (ok[q]) e = bins.be[b0 + i];
            jj[q] = (int)((uint32_t)e.w & ~kSelfMarkBit) - lo;
            vv[q] = e.v;
            self[q] = MODE == 2 && ((uint32_t)e.w & kSelfMarkBit) != 0u;
        }
#pragma unroll
        for (int q = 0; q < kRedUnroll; q++) {
            if (!ok[q]) continue;
            if (jj[q] < 0 || jj[q] >= span) st->overflow = 1;
            else if (self[q]) atomicOr(&s_self[jj[q] >> 5], 1u << (jj[q] & 31));
            else atomicAdd(&s_acc[jj[q]], vv[q]);
        }
    }
    __syncthreads();
    // a node needs an update iff its binned sum is nonzero: the gathered values
    // are positive in MODE 0/1, and in MODE 2 a zero sum leaves r_w unchanged,
    // so w is neither newly nonzero nor a node whose test could change
    // nodes per thread: the range of kBinLdsBytes / sizeof(V) nodes over the workgroup
    constexpr int per = kBinLdsBytes / (int)sizeof(V) / kReduceBlock;
    static_assert(per >= 1 && per <= 32, "one hit bit per node of a thread");
    if (span_max != per * (int)blockDim.x) {  // the host sized the ranges differently: never index with it
        if (threadIdx.x == 0) st->overflow = 1;
        return;
    }
    const int j0 = (int)threadIdx.x * per;
    const bool fuse = MODE != 1 && fz.on;
    uint32_t hits = 0u, firsts = 0u, tmask = 0u;
    V hval[per];  // fused snapshot: the amount moved into x for each hit (v or h)
    // every load of the thread's nodes first (their stores would otherwise order
    // each node's loads after the previous node's stores), then the arithmetic
    V acc[per], xo[per], dl[per];
    RD<V> e[per];
    int32_t cs[per];
    bool need[per], in_s[per];
#pragma unroll
    for (int k = 0; k < per; k++) {
        const int j = j0 + k;
        hval[k] = (V)0;
        acc[k] = j < span ? s_acc[j] : (V)0;
        in_s[k] = MODE == 2 && fuse && j < span && ((s_self[j >> 5] >> (j & 31)) & 1u);
        need[k] = j < span && (acc[k] != (V)0 || in_s[k]);
        const int32_t w = lo + j;
        e[k] = need[k] ? dst[w] : RD<V>{};
        xo[k] = (need[k] && fuse) ? fz.x[w] : (V)0;
        dl[k] = in_s[k] ? fz.delta[w] : (V)0;
        cs[k] = (need[k] && MODE == 2 && !fuse) ? cstamp[w] : 0;
    }
#pragma unroll
    for (int k = 0; k < per; k++) {
        if (!need[k]) continue;
        if (acc[k] != (V)0) tmask |= 1u << k;
        const int32_t w = lo + j0 + k;
        if (MODE == 2 && fuse) {
            // every candidate of t+1 in the range is here (touched, or in S_t):
            // the snapshot of t+1 on its final residual, momentum for nodes of S_t
            const V nr = e[k].r + acc[k];
            if (nr != (V)0 && fabs(nr) >= eps_eff * e[k].d) {
                hits |= 1u << k;
                const V h = fz.c_next * nr + (in_s[k] ? fz.m_next * dl[k] : (V)0);
                hval[k] = h;
                dst[w].r = nr - h;
                fz.x[w] = xo[k] + h;
                fz.delta[w] = h;
                fz.dstamp[w] = stamp_next;
                cstamp[w] = stamp_next + 1;  // its residual changed again: a candidate of t+2
            } else if (acc[k] != (V)0) {
                dst[w].r = nr;
            }
        } else if (MODE == 2) {
            // the residual of w is final for this iteration: only an active w joins
            // the candidates of t+1 (nodes of S_t were added by the snapshot)
            const V nr = e[k].r + acc[k];
            dst[w].r = nr;
            if (nr != (V)0 && fabs(nr) >= eps_eff * e[k].d && cs[k] != stamp_next) {
                hits |= 1u << k;
                cstamp[w] = stamp_next;
            }
        } else {
            const V nw = e[k].r + acc[k];
            const V th = eps_eff * e[k].d;
            const bool hit = e[k].r < th && nw >= th;
            if (hit) hits |= 1u << k;
            if (e[k].r == (V)0) firsts |= 1u << k;
            if (hit && fuse) {  // snapshot of t+1: v = r_w, r_w = 0, x_w += v
                hval[k] = nw;
                dst[w].r = (V)0;
                fz.x[w] = xo[k] + nw;
            } else {
                dst[w].r = nw;
            }
        }
    }
    // the range's words of the touched-residual bitmap: every node with an update
    // (a superset of the first touches), one plain read-modify-write per word --
    // the words of a range belong to this workgroup alone
    if (MODE != 1 && tbm) {
        if (tmask) atomicOr(&s_bits[j0 >> 5], tmask << (j0 & 31));
        __syncthreads();
        for (int k = threadIdx.x; k < (span + 31) / 32; k += blockDim.x)
            if (s_bits[k]) tbm[(lo >> 5) + k] |= s_bits[k];
    }
    if (fuse) {
        if (MODE == 2 && blockIdx.x == 0 && threadIdx.x == 0) st->fused_stamp = stamp_next;
        // work-list entries of the hits (the list of t+1 is not needed for them)
        const long long push_base = st->pushes;
        int32_t begs[per], degs[per];
        unsigned long long mine = 0ull;
#pragma unroll
        for (int k = 0; k < per; k++) {
            begs[k] = degs[k] = 0;
            if (!((hits >> k) & 1u)) continue;
            const int32_t w = lo + j0 + k;
            begs[k] = fz.row_ptr[w];
            degs[k] = fz.row_ptr[w + 1] - begs[k];
            mine += (1ull << 32) | (unsigned long long)(unsigned)degs[k];
        }
        const unsigned long long res = block_reserve64(mine, &st->packed[cur ^ 1]);
        int slot = (int)(res >> 32);
        int off = (int)(res & 0xffffffffull);
#pragma unroll
        for (int k = 0; k < per; k++) {
            if (!((hits >> k) & 1u)) continue;
            const int32_t w = lo + j0 + k;
            if (slot >= fz.cap) {
                st->overflow = 1;
                continue;
            }
            const V wgt = fz.w_div_deg ? fz.wscale / (V)degs[k] : fz.wscale;
            fz.wl_node[slot] = w;
            fz.wl_beg[slot] = begs[k];
            fz.wl_off[slot] = off;
            fz.wl_sv[slot] = wgt * hval[k];
            for (int q = (off + kPushTile - 1) / kPushTile; (long long)q * kPushTile < (long long)off + degs[k]; q++)
                fz.tile_start[q] = slot;
            if (fz.tr_nodes && push_base + slot < fz.tr_cap) fz.tr_nodes[push_base + slot] = w;
            slot++;
            off += degs[k];
        }
        // the pushed set: the range's bitmap words belong to this workgroup, so the
        // hits are gathered in LDS and written with one plain OR per word
        __syncthreads();  // the touched-bitmap words have been read out of s_bits
        for (int q = threadIdx.x; q < span_max / 32; q += blockDim.x) s_bits[q] = 0u;
        __syncthreads();
        if (hits) atomicOr(&s_bits[j0 >> 5], hits << (j0 & 31));
        __syncthreads();
        for (int q = threadIdx.x; q < (span + 31) / 32; q += blockDim.x)
            if (s_bits[q]) fz.bitmap[(lo >> 5) + q] |= s_bits[q];
        if (MODE == 2) {  // the fused nodes are candidates of t+2
            int s2 = block_reserve(__popc(hits), &st->fcount[cur]);
            for (uint32_t hm = hits; hm; hm &= hm - 1u) {
                const int32_t w = lo + j0 + (__ffs((int)hm) - 1);
                if (s2 < cap) fz.list2[s2] = w;
                else st->overflow = 1;
                s2++;
            }
        }
        return;
    }
    int slot = block_reserve(__popc(hits), &st->fcount[cur ^ 1]);
    for (uint32_t h = hits; h; h &= h - 1u) {
        const int32_t w = lo + j0 + (__ffs((int)h) - 1);
        if (slot < cap) next_list[slot] = w;
        else st->overflow = 1;
        slot++;
    }
    if (MODE == 1) {
        int ts = block_reserve(__popc(firsts), &st->tcount[tslot]);
        for (uint32_t h = firsts; h; h &= h - 1u) {
            const int32_t w = lo + j0 + (__ffs((int)h) - 1);
            if (ts < cap) touched[ts] = w;
            else st->overflow = 1;
            ts++;
        }
    }
}

// In-volume of every destination range: the number of CSR entries whose
// column falls in it, the capacity of the range's bin (a node receives at
// most one update per entry of its column per iteration).
__global__ void __launch_bounds__(kBlock) k_bin_count(const int32_t *__restrict__ col_idx, long long nnz, int shift,
                                                       int nranges, unsigned long long *counts) {
    __shared__ int s_c[kBinMaxRanges];
    for (int r = threadIdx.x; r < nranges; r += blockDim.x) s_c[r] = 0;
    __syncthreads();
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nnz; e += (long long)gridDim.x * blockDim.x)
        atomicAdd(&s_c[col_idx[e] >> shift], 1);
    __syncthreads();
    for (int r = threadIdx.x; r < nranges; r += blockDim.x)
        if (s_c[r]) atomicAdd(&counts[r], (unsigned long long)s_c[r]);
}

// LocalCH at the iteration cap: is S_t empty?  (counts without updating)
template <typename V>
__global__ void k_ch_probe(const RD<V> *rd, const int32_t *__restrict__ C, DevState *st, int cur, V eps_eff,
                           int32_t cap) {
    const int n_c = min(st->fcount[cur], cap);
    int c = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_c; i += gridDim.x * blockDim.x) {
        RD<V> e = rd[C[i]];
        c += (e.r != (V)0 && fabs(e.r) >= eps_eff * e.d) ? 1 : 0;
    }
    if (c) atomicAdd(&st->probe, c);
}

// ------------------------------------------------------------------ finalisation (A6 + A7)
// Residual norms of LocalGD / LocalCH: r can be nonzero only on the nodes of the
// touched bitmap.  One thread per bitmap word reads and zeroes the residual of
// each set bit and clears the word, accumulating ||r~||_1 and ||D^-1 r~||_inf
// in FP64.  Cost O(n/32 + |touched|); every entry is handled by one thread.
template <typename V>
__global__ void __launch_bounds__(kBlock) k_final_residual(uint32_t *tbm, int64_t nwords, RD<V> *rd, DevState *st,
                                                            double rscale) {
    double l1 = 0.0, mx = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nwords;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t m = tbm[i];
        if (m == 0u) continue;
        tbm[i] = 0u;
        while (m) {
            const int b = __ffs((int)m) - 1;
            m &= m - 1u;
            const int64_t w = i * 32 + b;
            const RD<V> e = rd[w];
            rd[w].r = (V)0;
            const double a = fabs((double)e.r) * rscale;
            l1 += a;
            if (a > 0.0) mx = fmax(mx, a / (double)e.d);
        }
    }
    block_fold_norms(l1, mx, st);
}

// Katz centrality option: x <- x - s on supp(s).
template <typename V>
__global__ void k_subtract_seed(V *x, const int32_t *__restrict__ sidx, const double *__restrict__ sval, int nnz) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nnz) x[sidx[i]] -= (V)sval[i];
}

// Sparse output in ascending node order from the pushed-set bitmap:
// count -> scan -> emit; emit also restores x and the bitmap to zero.
__global__ void __launch_bounds__(kBlock) k_ex_count(const uint32_t *__restrict__ bm, int64_t nwords, int32_t *blk) {
    __shared__ int s[kBlock / kWave];
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int c = i < nwords ? __popc(bm[i]) : 0;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if (lane() == 0) s[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int a = 0;
        for (int k = 0; k < (int)(blockDim.x / kWave); k++) a += s[k];
        blk[blockIdx.x] = a;
    }
}

__global__ void __launch_bounds__(1024) k_ex_scan(int32_t *blk, int64_t nblk, DevState *st) {
    __shared__ int s[1024];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nblk; base += 1024) {
        int64_t i = base + threadIdx.x;
        int v = i < nblk ? blk[i] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            int y = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0;
            __syncthreads();
            s[threadIdx.x] += y;
            __syncthreads();
        }
        if (i < nblk) blk[i] = carry + s[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry += s[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) st->out_count = carry;
}

template <typename V>
__global__ void __launch_bounds__(kBlock) k_ex_emit(uint32_t *bm, int64_t nwords, const int32_t *__restrict__ blk,
                                                     V *x, int32_t *out_idx, V *out_val, int64_t cap,
                                                     const DevState *st, const int32_t *__restrict__ sym_rp) {
    __shared__ int s[kBlock];
    // with st: write only if the whole support fits (else nothing is written)
    if (st && (int64_t)st->out_count > cap) cap = 0;
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    uint32_t word = i < nwords ? bm[i] : 0u;
    int c = __popc(word);
    s[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        int y = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += y;
        __syncthreads();
    }
    if (word) {
        int64_t pos = blk[blockIdx.x] + s[threadIdx.x] - c;
        while (word) {
            int b = __ffs(word) - 1;
            word &= word - 1u;
            int32_t u = (int32_t)(i * 32 + b);
            if (out_idx && pos < cap) {
                out_idx[pos] = u;
                // D^-1/2 A D^-1/2: the A D^-1 solution scaled back (see k_seed_init)
                out_val[pos] = sym_rp ? (V)((double)x[u] / sqrt((double)(sym_rp[u + 1] - sym_rp[u]))) : x[u];
            }
            x[u] = (V)0;
            pos++;
        }
        bm[i] = 0u;
    }
}

// ------------------------------------------------------------------ graph preparation (A0)
__global__ void k_check_csr(const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col_idx, int32_t n,
                            int64_t nnz, int32_t *bad, int32_t *dmax) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
        int32_t b = row_ptr[u], e = row_ptr[u + 1];
        if (u == 0 && b != 0) atomicAdd(bad, 1);
        if (u == n - 1 && (int64_t)e != nnz) atomicAdd(bad, 1);
        if (e < b) { atomicAdd(bad, 1); continue; }
        atomicMax(dmax, e - b);
        for (int32_t k = b; k < e; k++) {
            int32_t w = col_idx[k];
            if (w < 0 || w >= n || w == (int32_t)u) { atomicAdd(bad, 1); break; }
        }
    }
}

// One power-iteration step on A + I: y = A v + v, with the Rayleigh terms
// v'Av, v'v, ||y||^2 and the Collatz-Wielandt ratio max (Av)_u / v_u.
__global__ void __launch_bounds__(kBlock) k_lam_step(const int32_t *__restrict__ row_ptr,
                                                      const int32_t *__restrict__ col_idx,
                                                      const double *__restrict__ v, double *y, int32_t n,
                                                      double *red) {
    __shared__ double s[3][kBlock / kWave];
    __shared__ double sm[kBlock / kWave];
    double a = 0.0, b = 0.0, c = 0.0, m = 0.0;
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int32_t k = row_ptr[u]; k < row_ptr[u + 1]; k++) acc += v[col_idx[k]];
        double vu = v[u];
        double yu = acc + vu;
        y[u] = yu;
        a += vu * acc;
        b += vu * vu;
        c += yu * yu;
        m = fmax(m, acc / vu);
    }
    a = wave_sum(a); b = wave_sum(b); c = wave_sum(c); m = wave_max(m);
    int w = threadIdx.x / kWave;
    if (lane() == 0) { s[0][w] = a; s[1][w] = b; s[2][w] = c; sm[w] = m; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t0 = 0, t1 = 0, t2 = 0, tm = 0;
        for (int i = 0; i < (int)(blockDim.x / kWave); i++) { t0 += s[0][i]; t1 += s[1][i]; t2 += s[2][i]; tm = fmax(tm, sm[i]); }
        atomicAdd(&red[0], t0);
        atomicAdd(&red[1], t1);
        atomicAdd(&red[2], t2);
        atomicMax((unsigned long long *)&red[3], (unsigned long long)__double_as_longlong(tm));
    }
}

__global__ void k_lam_scale(const double *__restrict__ y, double *v, int32_t n, const double *red) {
    double inv = rsqrt(red[2]);
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x)
        v[u] = y[u] * inv;
}

__global__ void k_fill_f64(double *v, int64_t n, double val) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x)
        v[u] = val;
}

// ------------------------------------------------------------------ launchers
// Publication of the solver state to host memory: every word of *st is copied
// into the host-coherent mirror, made visible at system scope, and then the
// sequence number is released; a host that reads the number reads the state.
__global__ void __launch_bounds__(64) k_publish(const DevState *__restrict__ st, DevState *out, uint32_t *seq,
                                                uint32_t val) {
    constexpr int kWords = (int)(sizeof(DevState) / 4);
    static_assert(kWords <= 64, "one wavefront copies the state");
    const int i = threadIdx.x;
    if (i < kWords) {
        ((uint32_t *)out)[i] = ((const uint32_t *)st)[i];
        __threadfence_system();
    }
    __syncthreads();
    if (i == 0) __hip_atomic_store(seq, val, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

void launch_publish(const DevState *st, DevState *out, uint32_t *seq, uint32_t val, hipStream_t s) {
    hipLaunchKernelGGL(k_publish, dim3(1), dim3(64), 0, s, st, out, seq, val);
}

static inline int grid_for(int64_t items, int block, int cap) {
    int64_t g = (items + block - 1) / block;
    if (g < 1) g = 1;
    return (int)(g > cap ? cap : g);
}

template <typename V>
void launch_init_rd(const int32_t *row_ptr, void *rd, int32_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_init_rd<V>, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, row_ptr, (RD<V> *)rd, n);
}

template <typename V>
void launch_seed_init(void *rd, const int32_t *sidx, const double *sval, const SeedInline *inl, int32_t nnz,
                      double bscale, int32_t *f0, int32_t *touched0, int32_t *cstamp, int32_t stamp0, uint32_t *tbm,
                      DevState *st, hipStream_t s, const int32_t *sym_rp) {
    SeedInline none{};
    hipLaunchKernelGGL(k_seed_init<V>, dim3(grid_for(nnz, 256, 65535)), dim3(256), 0, s, (RD<V> *)rd, sidx, sval, nnz,
                       inl ? *inl : none, bscale, f0, touched0, cstamp, stamp0, tbm, st, sym_rp);
}

template <typename V>
void launch_snap_gd(const SnapArgs &a, V wscale, int w_div_deg, hipStream_t s) {
    hipLaunchKernelGGL(k_snap_gd<V>, dim3(a.grid), dim3(kSnapBlock), 0, s, a.row_ptr, (RD<V> *)a.rd, (V *)a.x, a.bitmap,
                       a.F, a.st, a.cur, a.wl_node, a.wl_beg, a.wl_off, (V *)a.wl_sv, a.tile_start, wscale,
                       w_div_deg, a.tr_nodes, a.tr_cap, a.cap);
}

template <typename V>
void launch_snap_hk(const SnapArgs &a, void *prev, V wmul, int last_level, int frontier_on, const int32_t *prev_touched,
                    int prev_tslot, int next_tslot, double psi_prev, double wdinf_prev, hipStream_t s) {
    hipLaunchKernelGGL(k_snap_hk<V>, dim3(a.grid), dim3(kSnapBlock), 0, s, a.row_ptr, (RD<V> *)a.rd, (RD<V> *)prev,
                       (V *)a.x, a.bitmap, a.F, a.st, a.cur, a.wl_node, a.wl_beg, a.wl_off, (V *)a.wl_sv,
                       a.tile_start, wmul, last_level, frontier_on, prev_touched, prev_tslot, next_tslot, psi_prev,
                       wdinf_prev, a.tr_nodes, a.tr_cap, a.cap);
}

template <typename V>
void launch_snap_ch(const SnapArgs &a, V wscale, int w_div_deg, V eps_eff, V c_t, V m_t, int force, void *delta,
                    int32_t *dstamp, int32_t *cstamp, int32_t stamp_cur, int32_t *next_list, hipStream_t s) {
    hipLaunchKernelGGL(k_snap_ch<V>, dim3(a.grid), dim3(kSnapBlock), 0, s, a.row_ptr, (RD<V> *)a.rd, (V *)a.x, a.bitmap,
                       a.F, a.st, a.cur, a.wl_node, a.wl_beg, a.wl_off, (V *)a.wl_sv, a.tile_start, wscale,
                       w_div_deg, eps_eff, c_t, m_t, force, (V *)delta, dstamp, cstamp, stamp_cur, next_list,
                       a.tr_nodes, a.tr_cap, a.cap);
}

template <typename V>
void launch_push(int mode, int grid, const int32_t *col_idx, void *dst, DevState *st, int cur, const int32_t *wl_beg,
                 const int32_t *wl_off, const void *wl_sv, const int32_t *tile_start, V eps_eff, int32_t *next_list,
                 int32_t *touched, int tslot, int32_t *cstamp, int32_t stamp_next, uint32_t *tbm, long long *tr_size,
                 long long *tr_vol, long long tr_cap, int scatter, int32_t cap, int32_t nnz, const BinArgs<V> &bins,
                 const FuseArgs<V> *fz, hipStream_t s) {
    auto kern = mode == 0 ? k_push<V, 0> : mode == 1 ? k_push<V, 1> : k_push<V, 2>;
    const size_t dyn = 2 * sizeof(int32_t) * (size_t)bins.nranges;
    const int marks = (mode == 2 && fz && fz->on) ? 1 : 0;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kPushBlock), dyn, s, col_idx, (RD<V> *)dst, st, cur, wl_beg, wl_off,
                       (const V *)wl_sv, tile_start, eps_eff, next_list, touched, tslot, cstamp, stamp_next, tbm,
                       tr_size, tr_vol, tr_cap, scatter, cap, nnz, bins, fz ? fz->wl_node : nullptr, marks);
    if (bins.nranges > 0) {
        auto red = mode == 0 ? k_reduce<V, 0> : mode == 1 ? k_reduce<V, 1> : k_reduce<V, 2>;
        const size_t rdyn = sizeof(V) * ((size_t)1 << bins.shift) + 2 * sizeof(uint32_t) * (((size_t)1 << bins.shift) / 32);
        hipLaunchKernelGGL(red, dim3(bins.nranges), dim3(kReduceBlock), rdyn, s, bins, (RD<V> *)dst, st, cur, eps_eff,
                           next_list, touched, tslot, cstamp, stamp_next, tbm, scatter, cap, (int32_t)(cap),
                           fz ? *fz : FuseArgs<V>{});
    }
}

void launch_bin_count(const int32_t *col_idx, long long nnz, int shift, int nranges, unsigned long long *counts,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_bin_count, dim3(grid_for(nnz, kBlock, 2048)), dim3(kBlock), 0, s, col_idx, nnz, shift,
                       nranges, counts);
}

template <typename V>
void launch_final_residual(uint32_t *tbm, int64_t nwords, void *rd, DevState *st, double rscale, hipStream_t s) {
    hipLaunchKernelGGL(k_final_residual<V>, dim3(grid_for(nwords, kBlock, 2048)), dim3(kBlock), 0, s, tbm, nwords,
                       (RD<V> *)rd, st, rscale);
}

template <typename V>
void launch_subtract_seed(void *x, const int32_t *sidx, const double *sval, int nnz, hipStream_t s) {
    hipLaunchKernelGGL(k_subtract_seed<V>, dim3(grid_for(nnz, 256, 65535)), dim3(256), 0, s, (V *)x, sidx, sval, nnz);
}

template <typename V>
void launch_ch_probe(const void *rd, const int32_t *C, DevState *st, int cur, V eps_eff, int32_t cap, hipStream_t s) {
    hipLaunchKernelGGL(k_ch_probe<V>, dim3(256), dim3(256), 0, s, (const RD<V> *)rd, C, st, cur, eps_eff, cap);
}

void launch_ex_count(const uint32_t *bm, int64_t nwords, int32_t *blk, int64_t nblk, hipStream_t s) {
    hipLaunchKernelGGL(k_ex_count, dim3((unsigned)nblk), dim3(kBlock), 0, s, bm, nwords, blk);
}
void launch_ex_scan(int32_t *blk, int64_t nblk, DevState *st, hipStream_t s) {
    hipLaunchKernelGGL(k_ex_scan, dim3(1), dim3(1024), 0, s, blk, nblk, st);
}
template <typename V>
void launch_ex_emit(uint32_t *bm, int64_t nwords, const int32_t *blk, int64_t nblk, void *x, int32_t *out_idx,
                    void *out_val, int64_t cap, const DevState *st, hipStream_t s, const int32_t *sym_rp) {
    hipLaunchKernelGGL(k_ex_emit<V>, dim3((unsigned)nblk), dim3(kBlock), 0, s, bm, nwords, blk, (V *)x, out_idx,
                       (V *)out_val, cap, st, sym_rp);
}

void launch_check_csr(const int32_t *row_ptr, const int32_t *col_idx, int32_t n, int64_t nnz, int32_t *bad,
                      int32_t *dmax, hipStream_t s) {
    hipLaunchKernelGGL(k_check_csr, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, row_ptr, col_idx, n, nnz, bad,
                       dmax);
}
void launch_lam_step(const int32_t *row_ptr, const int32_t *col_idx, const double *v, double *y, int32_t n,
                     double *red, hipStream_t s) {
    hipLaunchKernelGGL(k_lam_step, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, s, row_ptr, col_idx, v, y, n,
                       red);
}
void launch_lam_scale(const double *y, double *v, int32_t n, const double *red, hipStream_t s) {
    hipLaunchKernelGGL(k_lam_scale, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, y, v, n, red);
}
void launch_fill_f64(double *v, int64_t n, double val, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, v, n, val);
}

#define GDE_INST(V)                                                                                               \
    template void launch_small<V>(const SmallArgs<V> &, bool, hipStream_t);                                       \
    template void launch_init_rd<V>(const int32_t *, void *, int32_t, hipStream_t);                               \
    template void launch_seed_init<V>(void *, const int32_t *, const double *, const SeedInline *, int32_t, double, int32_t *,        \
                                      int32_t *, int32_t *, int32_t, uint32_t *, DevState *, hipStream_t,         \
                                      const int32_t *);        \
    template void launch_snap_gd<V>(const SnapArgs &, V, int, hipStream_t);                                       \
    template void launch_snap_hk<V>(const SnapArgs &, void *, V, int, int, const int32_t *, int, int, double,    \
                                    double, hipStream_t);                                                         \
    template void launch_snap_ch<V>(const SnapArgs &, V, int, V, V, V, int, void *, int32_t *, int32_t *,        \
                                    int32_t, int32_t *, hipStream_t);                                             \
    template void launch_push<V>(int, int, const int32_t *, void *, DevState *, int, const int32_t *,            \
                                 const int32_t *, const void *, const int32_t *, V, int32_t *, int32_t *, int,    \
                                 int32_t *, int32_t, uint32_t *, long long *, long long *, long long, int,        \
                                 int32_t, int32_t, const BinArgs<V> &, const FuseArgs<V> *, hipStream_t);                              \
    template void launch_final_residual<V>(uint32_t *, int64_t, void *, DevState *, double, hipStream_t);         \
    template void launch_subtract_seed<V>(void *, const int32_t *, const double *, int, hipStream_t);             \
    template void launch_ch_probe<V>(const void *, const int32_t *, DevState *, int, V, int32_t, hipStream_t);     \
    template void launch_ex_emit<V>(uint32_t *, int64_t, const int32_t *, int64_t, void *, int32_t *, void *,   \
                                    int64_t, const DevState *, hipStream_t, const int32_t *);

GDE_INST(float)
GDE_INST(double)

}  // namespace gde
