// gde_kernels.h -- host-side launch interface of the gfx950 kernels.
#pragma once

#include <cmath>
#include <vector>

#include "gde_internal.h"

namespace gde {

// Arguments common to the snapshot kernels (one iteration, one work list).
struct SnapArgs {
    int grid;
    const int32_t *row_ptr;
    void *rd;             // residual plane read and zeroed by the snapshot
    void *x;
    uint32_t *bitmap;
    const int32_t *F;     // S_t (GD, HK) or the candidates C_t (CH)
    DevState *st;
    int cur;
    int32_t *wl_node, *wl_beg, *wl_off;
    void *wl_sv;
    int32_t *tile_start;
    int32_t *tr_nodes;
    long long tr_cap;
    int32_t cap;          // capacity of every node list (n)
};

// The snapshot of t+1 taken inside the range reduction of a binned iteration t.
// LocalGD: every crossing (S_{t+1} is exactly the set of nodes that crossed).
// LocalCH: every candidate of t+1 (a node touched by the push of t, or a node of
// S_t, which the push marks in the bins with a zero-valued entry), so the
// separate snapshot of t+1 has nothing left to do.  Residuals are final in
// registers there and the node state is range-local.
template <typename V>
struct FuseArgs {
    int on;                      // 0: plain reduction (appends S_{t+1} / C_{t+1} to the list)
    const int32_t *row_ptr;
    V *x;
    uint32_t *bitmap;            // pushed set
    int32_t *wl_node, *wl_beg, *wl_off;
    V *wl_sv;
    int32_t *tile_start;
    int32_t *tr_nodes;
    long long tr_cap;
    V wscale;
    int w_div_deg;
    V c_next, m_next;            // LocalCH: c_{t+1}, m_{t+1}
    V *delta;
    int32_t *dstamp;
    int32_t *list2;              // LocalCH: candidates of t+2 (self-marks of S_{t+1})
    int32_t cap;
};

// Everything the single-workgroup iteration kernel needs (LocalGD or LocalCH).
template <typename V>
struct SmallArgs {
    const int32_t *row_ptr, *col_idx;
    void *rd, *x;
    uint32_t *bitmap, *tbm;
    DevState *st;
    int32_t *front0, *front1;
    int32_t *wl_node, *wl_beg, *wl_off;
    void *wl_sv;
    int32_t *tile_start;
    int32_t *tr_nodes;
    long long tr_ncap;
    long long *tr_size, *tr_vol;
    long long tr_cap;
    V wscale, eps_eff;
    int w_div_deg;
    void *delta;
    int32_t *dstamp, *cstamp;
    int32_t stamp_base;
    V c_seq[kSmallIters], m_seq[kSmallIters];  // LocalCH scalars of iterations t0 .. t0 + kSmallIters - 1
    int32_t cap, nnz;
    int t0, t_end;
};

template <typename V> void launch_small(const SmallArgs<V> &a, bool ch, hipStream_t s);

// The heat-kernel level push of small frontiers, one workgroup over consecutive
// levels k0 .. K (and the final clean-up).
template <typename V>
struct HkSmallArgs {
    const int32_t *row_ptr, *col_idx;
    void *plane[2];              // RD<V> planes: level k uses plane[k & 1]
    void *x;
    uint32_t *bitmap;
    DevState *st;
    int32_t *front[2];           // S_k in front[k & 1]
    int32_t *touched[3];         // nodes of level k with a nonzero residual in touched[k % 3]
    int32_t *wl_beg, *wl_off;
    void *wl_sv;
    int32_t *tile_start;
    int32_t *tr_nodes;
    long long tr_ncap;
    long long *tr_size, *tr_vol;
    long long tr_cap;
    const double *lvl_tab;       // device [2][kHkMaxLevels + 1]: psi_k, then the level ratios
    double eps;
    int K, k0;
    int32_t cap, nnz;
};

template <typename V> void launch_small_hk(const HkSmallArgs<V> &a, hipStream_t s);

// The series of a level-push query: c_0 (the scale of level 0), the level ratios
// c_{k+1}/c_k (ratio[k], k < K) and psi_k = sum_{j=k..K} c_j / c_k.  The heat
// kernel (c_k = e^-tau tau^k/k!) takes them from tau; GDE_SERIES from p->c.
struct LevelSeries {
    double c0 = 1.0;
    std::vector<double> ratio, psi;
};
inline LevelSeries level_series(const gde_params *p) {
    LevelSeries ls;
    const int K = p->K;
    ls.ratio.assign((size_t)K + 1, 0.0);
    ls.psi.assign((size_t)K + 1, 0.0);
    if (p->kind == GDE_SERIES) {
        ls.c0 = p->c[0];
        for (int k = 0; k <= K; k++) {
            double acc = 0.0;
            for (int j = k; j <= K; j++) acc += p->c[j] / p->c[k];
            ls.psi[k] = acc;
            if (k < K) ls.ratio[k] = p->c[k + 1] / p->c[k];
        }
    } else {
        const double tau = p->tau;
        ls.c0 = std::exp(-tau);
        for (int k = 0; k <= K; k++) {
            double acc = 0.0, term = 1.0;  // term = tau^{j-k} k!/j!
            for (int j = k; j <= K; j++) {
                if (j > k) term *= tau / (double)j;
                acc += term;
            }
            ls.psi[k] = acc;
            if (k < K) ls.ratio[k] = tau / (double)(k + 1);
        }
    }
    return ls;
}
void launch_publish(const DevState *st, DevState *out, uint32_t *seq, uint32_t val, hipStream_t s);

template <typename V> void launch_init_rd(const int32_t *row_ptr, void *rd, int32_t n, hipStream_t s);
// A seed small enough to travel in the kernel arguments.
constexpr int kSeedInline = 8;
struct SeedInline {
    int32_t n;  // 0: the seed is in the device buffers
    int32_t idx[kSeedInline];
    double val[kSeedInline];
};

template <typename V>
void launch_seed_init(void *rd, const int32_t *sidx, const double *sval, const SeedInline *inl, int32_t nnz,
                      double bscale, int32_t *f0,
                      int32_t *touched0, int32_t *cstamp, int32_t stamp0, uint32_t *tbm, DevState *st, hipStream_t s,
                      const int32_t *sym_rp = nullptr);
template <typename V> void launch_snap_gd(const SnapArgs &a, V wscale, int w_div_deg, hipStream_t s);
template <typename V>
void launch_snap_hk(const SnapArgs &a, void *prev, V wmul, int last_level, int frontier_on, const int32_t *prev_touched,
                    int prev_tslot, int next_tslot, double psi_prev, double wdinf_prev, hipStream_t s);
template <typename V>
void launch_snap_ch(const SnapArgs &a, V wscale, int w_div_deg, V eps_eff, V c_t, V m_t, int force, void *delta,
                    int32_t *dstamp, int32_t *cstamp, int32_t stamp_cur, int32_t *next_list, hipStream_t s);
template <typename V>
void launch_push(int mode, int grid, const int32_t *col_idx, void *dst, DevState *st, int cur, const int32_t *wl_beg,
                 const int32_t *wl_off, const void *wl_sv, const int32_t *tile_start, V eps_eff, int32_t *next_list,
                 int32_t *touched, int tslot, int32_t *cstamp, int32_t stamp_next, uint32_t *tbm, long long *tr_size,
                 long long *tr_vol, long long tr_cap, int scatter, int32_t cap, int32_t nnz, const BinArgs<V> &bins,
                 const FuseArgs<V> *fz, hipStream_t s);
void launch_bin_count(const int32_t *col_idx, long long nnz, int shift, int nranges, unsigned long long *counts,
                      hipStream_t s);
template <typename V>
void launch_final_residual(uint32_t *tbm, int64_t nwords, void *rd, DevState *st, double rscale, hipStream_t s);
template <typename V> void launch_subtract_seed(void *x, const int32_t *sidx, const double *sval, int nnz, hipStream_t s);
template <typename V>
void launch_ch_probe(const void *rd, const int32_t *C, DevState *st, int cur, V eps_eff, int32_t cap, hipStream_t s);
void launch_ex_count(const uint32_t *bm, int64_t nwords, int32_t *blk, int64_t nblk, hipStream_t s);
void launch_ex_scan(int32_t *blk, int64_t nblk, DevState *st, hipStream_t s);
template <typename V>
void launch_ex_emit(uint32_t *bm, int64_t nwords, const int32_t *blk, int64_t nblk, void *x, int32_t *out_idx,
                    void *out_val, int64_t cap, const DevState *st, hipStream_t s, const int32_t *sym_rp = nullptr);
void launch_check_csr(const int32_t *row_ptr, const int32_t *col_idx, int32_t n, int64_t nnz, int32_t *bad,
                      int32_t *dmax, hipStream_t s);
void launch_lam_step(const int32_t *row_ptr, const int32_t *col_idx, const double *v, double *y, int32_t n,
                     double *red, hipStream_t s);
void launch_lam_scale(const double *y, double *v, int32_t n, const double *red, hipStream_t s);
void launch_fill_f64(double *v, int64_t n, double val, hipStream_t s);

}  // namespace gde
