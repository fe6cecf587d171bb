// gde_batch_kernels.h -- device layout and launch interface of the batched solver.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "gde_internal.h"

namespace gde {

constexpr int kStatShards = 64;  // per-lane counters are sharded to spread atomics
// a lane's pushes and operations share one 64-bit counter per shard (one atomic
// per push): pushes in the top kPushBits bits, operations (sum of d_u) below
constexpr int kPushBits = 26;
constexpr unsigned long long kOpsMask = (1ull << (64 - kPushBits)) - 1ull;
constexpr int kResLdsLanes = 4096;  // lanes whose residual norms a workgroup can sum in LDS (64 KB)

struct BatchDev {
    unsigned long long packed[2];  // (entries << 40) | lane-edges of iteration parity
    int32_t acount[2];             // active (group, node) pairs
    int32_t tcount;                // touched pairs
    int32_t ovf[2];                // a capacity was exceeded during an iteration of this parity
                                   // (per parity, so the stop test after iteration t reads a
                                   // flag that no block can still be writing)
    int32_t pad0[2];
    long long lane_edges;          // sum over iterations of the lane-edges pushed
    long long entries;             // sum over iterations of the (group, node) entries
    // measurement only (row_stamp set): distinct rows pushed in iteration of
    // parity p, packed (rows << 40) | their volume, and the sums over iterations
    unsigned long long rowpack[2];
    long long rows;
    long long row_vol;
    int32_t tcount2;  // level push: entries of the odd levels' touched list (touched2)
};

// Everything a batch kernel needs.  Node-major layout: the L lanes of group g
// at node u live at ((u * G + g) * L + l), so all groups' values of a node
// share pages and each group's L values share a cache line.
template <typename V>
struct BatchArgs {
    int32_t n;
    int32_t nnz;
    int32_t G;
    int64_t nwords;  // pushed-bitmap words per group
    const int32_t *row_ptr;
    const int32_t *col_idx;
    const V *deg;
    const V *col_deg;  // optional [nnz]: deg[col_idx[e]], streamed beside col_idx instead of gathered
    V *R;
    V *X;
    uint32_t *NM;  // [n][G] lanes crossing their threshold this iteration
    uint32_t *TM;  // [n][G] pair touched: TM == the group's epoch (never 0), so no clearing pass
    uint32_t epoch;             // epoch of every group (batched solves)
    const uint32_t *g_epoch;    // optional [G] per-group epochs (serving); replaces epoch
    uint32_t *PB;  // [G][nwords] pushed bitmap
    uint64_t *act[2];
    int32_t act_cap;
    uint64_t *touched;
    uint64_t *touched2;  // level push: touched entries of odd levels (even levels use touched)
    int32_t *tdeg, *tdeg2;  // optional, parallel to touched / touched2: the entry node's degree
    int32_t touch_cap;
    int32_t *wl_node, *wl_group, *wl_beg, *wl_c;
    long long *wl_off;
    uint8_t *wl_lanes;
    V *wl_sv;
    int32_t wl_cap;
    int32_t *tile_start;
    int64_t tile_cap;
    const V *lane_eps;  // [G*L] eps_eff of each lane
    V wscale;
    int w_div_deg;
    // optional per-group overrides (serving mixes PPR and Katz groups in one launch):
    // g_wscale[g] replaces wscale; g_mode[g] bit 0 = divide by d_u (PPR), bit 1 =
    // candidate mode (signed residuals: lanes marked by |r| crossing the threshold, re-tested in the snapshot)
    const V *g_wscale;
    const int32_t *g_mode;
    long long *lane_ops;  // [G*L][kStatShards]: pushes and operations (kPushBits)
    int32_t *lane_T;                    // [G*L]
    double *lane_l1;                    // [G*L][kStatShards]
    unsigned long long *lane_dinf;      // [G*L]
    uint32_t *group_unconv;             // [G]
    long long *tr_size, *tr_vol;        // optional [G*L][tr_cap]
    int32_t tr_cap;
    int32_t *tr_nodes;                  // optional S_t lists: lane l writes at tr_noff[l] + k, k < tr_ncap[l]
    const long long *tr_noff, *tr_ncap;
    unsigned long long *tr_ncount;      // [G*L] entries recorded (may exceed the capacity)
    BatchDev *st;
    int32_t max_iters;
    // level push (heat kernel, series; null R2 = LocalGD): R holds the residual
    // of even levels, R2 of odd ones; snap(t) takes level t, push(t) adds into
    // level t + 1, whose threshold is (eps_lane / th_div) * d_u
    V *R2;
    double th_div;
    int32_t no_push;  // snap of the last level: x only, nothing pushed
    int32_t sym;      // M = D^-1/2 A D^-1/2: seeds scaled by sqrt(d), outputs by 1/sqrt(d)
    // LocalCH (ch != 0): every lane in iteration t applies h = c_t r + m_t Delta
    // (Delta kept only for lanes active in t - 1, PM), or h = r when force (t =
    // 0); residuals are signed: a lane whose |r| an update lifts across its
    // threshold is a candidate (NM), a pushed pair is a candidate of t + 1
    // itself, and the snapshot tests every candidate
    int32_t ch, force, probe;
    // warm start (standing queries): LocalGD steps with signed residuals: a lane
    // is a candidate when an update lifts |r| across its threshold, the snapshot
    // tests its candidates again (later updates may have lowered |r|), and the
    // final pass takes residuals by exchange (one that cancels to +0.0 is listed
    // again when it is touched next)
    int32_t sgn;
    V c_t, m_t;
    V *D;          // [n][G][L] Delta, the last update of each lane
    uint32_t *PM;  // [n][G] lanes active when the pair was last snapshot
    // measurement only: row_stamp[u] == round_tag once row u was counted in this
    // iteration (distinct CSR rows read per round, whatever the groups); null = off
    uint32_t *row_stamp;
    uint32_t round_tag;
};

// which: 1 snap(t), 2 push(t)
template <typename V> hipError_t batch_launch(int which, int L, const BatchArgs<V> &a, int grid, int t, hipStream_t s);
template <typename V> hipError_t batch_occupancy(int L, int *blocks_per_cu);
template <typename V>
hipError_t batch_seed(int L, const BatchArgs<V> &a, const int32_t *s_lane, const int32_t *s_node, const double *s_val,
                      int32_t ns, double bscale, hipStream_t s);
// level push: residual norms of level t over its touched entries (read, reset),
// weighted w_l1 = psi_t in the 1-norm and w_dinf = (K + 1) psi_t in the
// degree-scaled max norm
template <typename V>
hipError_t batch_harvest(int L, const BatchArgs<V> &a, int grid, int t, double w_l1, double w_dinf, hipStream_t s);
template <typename V>
hipError_t batch_finish(int L, const BatchArgs<V> &a, int grid, double rscale, int last, const int32_t *s_lane,
                        const int32_t *s_node, const double *s_val, int32_t ns, const int32_t *sub_flag,
                        hipStream_t s);
// gmap (optional): the ngroups groups to extract (all a.G groups when null)
template <typename V>
hipError_t batch_extract(int L, const BatchArgs<V> &a, int stage, int32_t *cnt, int nblk, long long *lane_nnz,
                         const long long *lane_out_off, int32_t *out_idx, V *out_val, int write, hipStream_t s,
                         const int32_t *gmap = nullptr, int ngroups = 0, int32_t *const *lane_idx = nullptr,
                         V *const *lane_val = nullptr);
template <typename V> hipError_t batch_init_deg(const int32_t *row_ptr, V *deg, int32_t n, hipStream_t s);
// warm start of B standing queries (lane j = query of lane j): load their residuals
// at the nodes of their touched bitmaps; afterwards store the residuals back
// (before the residual pass) and add the lanes' x into theirs (the extraction)
template <typename V>
hipError_t batch_warm_load(int L, const BatchArgs<V> &a, const void *const *q_rd, const uint32_t *const *q_tbm, int B,
                           hipStream_t s);
template <typename V>
hipError_t batch_warm_store(int L, const BatchArgs<V> &a, int stage, void *const *q_rd, uint32_t *const *q_tbm,
                            void *const *q_x, uint32_t *const *q_pushed, int B, int grid, hipStream_t s);
template <typename V>
hipError_t batch_init_col_deg(const int32_t *col_idx, const V *deg, V *col_deg, int64_t nnz, hipStream_t s);

}  // namespace gde
