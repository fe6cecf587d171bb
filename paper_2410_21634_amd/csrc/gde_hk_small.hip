// gde_hk_small.hip -- the heat-kernel level push (Sec. 2, "Heat Kernel": the AHK
// push on the Kronecker system, taken level by level) for small frontiers, run by
// ONE workgroup over consecutive levels in one launch.
//
// Level k holds the residual plane r_k (planes alternate between two RD<V>
// arrays, so plane k+1 is the plane of level k-1).  One level:
//   clean-up : the leftovers of level k-1 (its touched list) are folded into
//              the reported norms, weighted by psi_{k-1}, and their plane is
//              zeroed, since it becomes plane k+1;
//   snapshot : for u in S_k, x_u += r_k[u], r_k[u] = 0, scatter value
//              (c_{k+1}/c_k) r_k[u] / d_u (none at the last level K), which
//              for the heat kernel is (tau / (k+1)) r_k[u] / d_u;
//   push     : r_{k+1}[w] += value over the rows of S_k; the add that lifts
//              r_{k+1}[w] over eps d_w / ((K+1) psi_{k+1}) appends w to S_{k+1}
//              (crossing test, the plane only grows during the push), and the
//              add that finds r_{k+1}[w] at zero appends w to the touched list
//              of level k+1.
// These are the decisions of k_snap_hk and k_push<V, 1>.  Frontier lists, the
// work list and every counter live in LDS; the touched lists stay in global
// memory (with LDS counts), as do node state and the CSR.  All accesses come
// from this workgroup, so barriers (with their workgroup-scope fences) order
// the phases; residuals are read past L1 because atomics are performed in L2.
//
// The launch stops before level k when |S_k| exceeds kSmallMaxNodes or the
// touched list of level k-1 exceeds kSmallMaxEdges (small_phase 0: level k,
// clean-up included, is left to the grid-wide kernels), after the snapshot of
// k when vol(S_k) exceeds kSmallMaxEdges (small_phase 1: the work list of k is
// written out for the grid-wide push), or after the final clean-up of level K
// (small_phase 2: the solve is done).
#include <hip/hip_runtime.h>

#include "gde_device.h"
#include "gde_internal.h"
#include "gde_kernels.h"

namespace gde {

namespace {

__device__ __forceinline__ double hk_wave_sum(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ __forceinline__ double hk_wave_max(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    return v;
}

// Exclusive scan of a packed (count << 32 | amount) pair over the workgroup.
__device__ __forceinline__ unsigned long long hk_excl_scan64(unsigned long long v, unsigned long long *total) {
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

}  // namespace

template <typename V>
__global__ void __launch_bounds__(kSnapBlock) k_small_hk(HkSmallArgs<V> a) {
    constexpr int kNodesPer = kSmallMaxNodes / kSnapBlock;
    constexpr int kEdgesPer = 4;
    static_assert(kNodesPer * kSnapBlock == kSmallMaxNodes, "list entries must split evenly");
    __shared__ int32_t s_list[2][kSmallMaxNodes];
    __shared__ int32_t s_beg[kSmallMaxNodes];
    __shared__ int32_t s_off[kSmallMaxNodes + 1];
    __shared__ V s_sv[kSmallMaxNodes];
    __shared__ double s_psi[kHkMaxLevels + 1];
    __shared__ int s_fcnt[2], s_tcnt[3];
    __shared__ int s_ovf;
    __shared__ long long s_push_base;
    DevState *st = a.st;
    V *x = (V *)a.x;
    const int tid = threadIdx.x;
    const int K = a.K;
    // psi_k of the series, from the host's table
    for (int k = tid; k <= K; k += blockDim.x) s_psi[k] = a.lvl_tab[k];
    int iters = 0;
    long long ops = 0, pushes = 0;
    if (tid == 0) {
        iters = st->iters;
        ops = st->ops;
        pushes = st->pushes;
        s_fcnt[0] = st->fcount[0];
        s_fcnt[1] = st->fcount[1];
        for (int i = 0; i < 3; i++) s_tcnt[i] = st->tcount[i];
        s_ovf = 0;
    }
    __syncthreads();
    int k = a.k0;
    {
        const int c0 = s_fcnt[k & 1];
        const int32_t *F = a.front[k & 1];
        if (k <= K && c0 <= kSmallMaxNodes)
            for (int i = tid; i < c0; i += blockDim.x) s_list[k & 1][i] = F[i];
    }
    __syncthreads();
    double l1 = 0.0, mx = 0.0;
    int phase = 0;
    for (; k <= K + 1; k++) {
        const int cur = k & 1, nxt = cur ^ 1;
        const bool final_cleanup = k == K + 1;
        const int n_f = final_cleanup ? 0 : s_fcnt[cur];
        if (n_f > kSmallMaxNodes) break;
        // the clean-up of level k-1 walks its touched list: a long one goes to the grid too
        if (k >= 1 && (long long)s_tcnt[(k + 2) % 3] > kSmallMaxEdges) break;
        // ------------------------------------------------ clean-up of level k-1
        if (k >= 1) {
            RD<V> *prev = (RD<V> *)a.plane[nxt];
            const int ts = (k + 2) % 3;
            const int n_c = min(s_tcnt[ts], a.cap);
            const double psi_prev = s_psi[k - 1];
            const double wdinf_prev = (double)(K + 1) * psi_prev;
            const int32_t *T = a.touched[ts];
            for (int j = tid; j < n_c; j += blockDim.x) {
                const int32_t w = T[j];
                const V val = __hip_atomic_load(&prev[w].r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                prev[w].r = (V)0;
                const double av = fabs((double)val);
                l1 += psi_prev * av;
                if (av > 0.0) mx = fmax(mx, wdinf_prev * av / (double)prev[w].d);
            }
        }
        if (final_cleanup) {
            phase = 2;
            break;
        }
        // ------------------------------------------------ snapshot of level k
        const bool last = k == K;
        RD<V> *plane = (RD<V> *)a.plane[cur];
        RD<V> *nplane = (RD<V> *)a.plane[nxt];
        const V wmul = (V)a.lvl_tab[kHkMaxLevels + 1 + k];  // c_{k+1} / c_k
        if (tid == 0) {
            s_push_base = pushes;
            s_tcnt[(k + 1) % 3] = 0;  // the touched list of level k+1 starts empty
        }
        int32_t u[kNodesPer], beg[kNodesPer], deg[kNodesPer];
        V sv[kNodesPer];
        unsigned long long mine = 0ull;
#pragma unroll
        for (int q = 0; q < kNodesPer; q++) {
            const int i = tid * kNodesPer + q;
            u[q] = i < n_f ? s_list[cur][i] : -1;
            beg[q] = deg[q] = 0;
            sv[q] = (V)0;
        }
        V rv[kNodesPer], dv0[kNodesPer], xo[kNodesPer];
        int32_t rp0[kNodesPer], rp1[kNodesPer];
#pragma unroll
        for (int q = 0; q < kNodesPer; q++) {  // every load before any store
            const bool v = u[q] >= 0;
            rv[q] = v ? __hip_atomic_load(&plane[u[q]].r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : (V)0;
            dv0[q] = v ? plane[u[q]].d : (V)1;
            xo[q] = v ? x[u[q]] : (V)0;
            rp0[q] = v ? a.row_ptr[u[q]] : 0;
            rp1[q] = v ? a.row_ptr[u[q] + 1] : 0;
        }
#pragma unroll
        for (int q = 0; q < kNodesPer; q++) {
            if (u[q] < 0) continue;
            plane[u[q]].r = (V)0;
            x[u[q]] = xo[q] + rv[q];
            beg[q] = rp0[q];
            deg[q] = rp1[q] - rp0[q];
            sv[q] = last ? (V)0 : wmul * rv[q] / dv0[q];
            mine += (1ull << 32) | (unsigned long long)(unsigned)deg[q];
        }
        unsigned long long tot;
        const unsigned long long pre = hk_excl_scan64(mine, &tot);
        const int count = (int)(tot >> 32);
        const int total = (int)(tot & 0xffffffffull);
        {
            int slot = (int)(pre >> 32);
            int off = (int)(pre & 0xffffffffull);
            const long long pb = s_push_base;
#pragma unroll
            for (int q = 0; q < kNodesPer; q++) {
                if (u[q] < 0) continue;
                s_beg[slot] = beg[q];
                s_off[slot] = off;
                s_sv[slot] = sv[q];
                if (a.tr_nodes && pb + slot < a.tr_ncap) a.tr_nodes[pb + slot] = u[q];
                slot++;
                off += deg[q];
            }
        }
        if (tid == 0) s_off[count] = total;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kNodesPer; q++)  // the pushed set (read only by the output kernels)
            if (u[q] >= 0) atomicOr(&a.bitmap[u[q] >> 5], 1u << (u[q] & 31));
        if (!last && count > 0 && (long long)total > kSmallMaxEdges) {
            // hand the push of level k to the grid-wide kernel
            for (int i = tid; i < count; i += blockDim.x) {
                const int off = s_off[i], d = s_off[i + 1] - off;
                a.wl_beg[i] = s_beg[i];
                a.wl_off[i] = off;
                ((V *)a.wl_sv)[i] = s_sv[i];
                for (int q = (off + kPushTile - 1) / kPushTile; (long long)q * kPushTile < (long long)off + d; q++)
                    a.tile_start[q] = i;
            }
            if (tid == 0) {
                st->packed[cur] = ((unsigned long long)count << 32) | (unsigned long long)(unsigned)total;
                st->packed[nxt] = 0ull;
            }
            phase = 1;
            break;
        }
        // ------------------------------------------------ push of level k into level k+1
        if (!last) {
            const V eps_next = (V)(a.eps / ((double)(K + 1) * s_psi[k + 1]));
            int32_t *Fn = a.front[nxt];
            const int tsn = (k + 1) % 3;
            int32_t *Tn = a.touched[tsn];
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
                V th[kEdgesPer], old[kEdgesPer];
#pragma unroll
                for (int q = 0; q < kEdgesPer; q++)
                    th[q] = (w[q] >= 0 && dv[q] != (V)0) ? eps_next * nplane[w[q]].d : (V)0;
#pragma unroll
                for (int q = 0; q < kEdgesPer; q++)
                    old[q] = (w[q] >= 0 && dv[q] != (V)0) ? unsafeAtomicAdd(&nplane[w[q]].r, dv[q]) : (V)0;
#pragma unroll
                for (int q = 0; q < kEdgesPer; q++) {
                    if (w[q] < 0 || dv[q] == (V)0) continue;
                    if (old[q] < th[q] && old[q] + dv[q] >= th[q]) {
                        const int c = atomicAdd(&s_fcnt[nxt], 1);
                        if (c < kSmallMaxNodes) s_list[nxt][c] = w[q];
                        if (c < a.cap) Fn[c] = w[q];
                        else s_ovf = 1;
                    }
                    if (old[q] == (V)0) {
                        const int c = atomicAdd(&s_tcnt[tsn], 1);
                        if (c < a.cap) Tn[c] = w[q];
                        else s_ovf = 1;
                    }
                }
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
            s_fcnt[cur] = 0;  // S_k consumed: the list becomes the append target of level k+2
        }
        __syncthreads();
    }
    // norms of the levels cleaned here, one fold for the launch
    __shared__ double s_l1[kMaxWaves], s_mx[kMaxWaves];
    l1 = hk_wave_sum(l1);
    mx = hk_wave_max(mx);
    if (lane() == 0) {
        s_l1[tid / kWave] = l1;
        s_mx[tid / kWave] = mx;
    }
    __syncthreads();
    if (tid == 0) {
        double tl1 = 0.0, tmx = 0.0;
        for (int i = 0; i < (int)(blockDim.x / kWave); i++) {
            tl1 += s_l1[i];
            tmx = fmax(tmx, s_mx[i]);
        }
        if (tl1 != 0.0) atomicAdd(&st->res_l1, tl1);
        if (tmx > 0.0) atomicMax(&st->res_dinf, (unsigned long long)__double_as_longlong(tmx));
        st->iters = iters;
        st->ops = ops;
        st->pushes = pushes;
        st->fcount[0] = s_fcnt[0];
        st->fcount[1] = s_fcnt[1];
        for (int i = 0; i < 3; i++) st->tcount[i] = s_tcnt[i];
        if (phase != 1) st->packed[0] = st->packed[1] = 0ull;
        if (s_ovf) st->overflow = 1;
        st->small_t = k;
        st->small_phase = phase;
    }
}

template <typename V>
void launch_small_hk(const HkSmallArgs<V> &a, hipStream_t s) {
    hipLaunchKernelGGL(k_small_hk<V>, dim3(1), dim3(kSnapBlock), 0, s, a);
}

template void launch_small_hk<float>(const HkSmallArgs<float> &, hipStream_t);
template void launch_small_hk<double>(const HkSmallArgs<double> &, hipStream_t);

}  // namespace gde
