// gde_internal.h -- data layout shared by the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "gde.h"

namespace gde {

constexpr int kWave = 64;      // CDNA wavefront width
constexpr int kBlock = 256;    // threads per workgroup of the batched and helper kernels
constexpr int kTile = 1024;    // lane-edges per batched push tile
constexpr int kMaxWaves = 16;  // wavefronts of the largest workgroup (1024 threads)
// Plain path.  Appends to the frontier lists and work-list reservations are
// aggregated per workgroup: a returning atomic on one shared counter costs
// about 11 ns on MI355X (measured), so one per 1024 threads instead of one per
// wavefront keeps the counters off the critical path.
constexpr int kSnapBlock = 1024;  // threads per snapshot workgroup
constexpr int kPushBlock = 1024;  // threads per push workgroup
constexpr int kPushTile = 1024;   // edges per push base tile (one per thread)
// A large frontier is pushed in tiles of kMacroTiles base tiles (kMacroTiles edges
// per thread, their loads issued together).
constexpr int kMacroTiles = 4;
constexpr long long kMacroMinEdges = 262144;
constexpr int kBatchSnapBlock = 1024;  // threads per batched snapshot workgroup
// Small frontiers: one workgroup runs consecutive iterations in one launch
// (workgroup barriers in place of kernel boundaries) while the frontier stays
// within these limits; larger frontiers hand over to the grid-wide kernels.
constexpr int kSmallIters = 32;             // iterations one single-workgroup launch may run
constexpr int kSmallMaxNodes = 4096;        // frontier / candidate list it accepts
constexpr long long kSmallMaxEdges = 16384; // frontier volume it accepts
constexpr int kSmallPendMarks = 8192;      // touched-bitmap marks it stages in LDS per push
constexpr int kHkMaxLevels = 256;          // largest heat-kernel truncation K
// Binned scatter for large frontiers: updates are written, grouped by
// destination range of 2^S nodes, into per-range bins and then summed in LDS
// by one workgroup per range (no global atomic per edge).
constexpr int kBinMaxRanges = 4096;     // ranges a graph may have for the binned scatter
constexpr int kBinLdsBytes = 16384;     // LDS accumulator bytes of one range (2^S values)
constexpr int kReduceBlock = 1024;      // threads per range-reduction workgroup
// The range reduction launches one workgroup per range, so a graph with more
// ranges needs a larger frontier before binning pays: the threshold is
// max(kBinMinEdges, ranges^2 / kBinRangeSqDiv) edges (measured: 8,192 on a
// 245-range graph, 128 to 512 edges per range on a 2,442-range graph).
constexpr long long kBinMinEdges = 8192;  // smallest frontier volume whose scatter is binned
constexpr long long kBinRangeSqDiv = 8;
// With fewer ranges the reduction runs on too few workgroups, the hub range (the
// lowest ids of a Chung-Lu graph) taking most entries: on a 10^4-node graph a
// solve took 1.55 ms binned against 0.68 ms atomic in FP32 (3 ranges), and
// 0.62 against 0.69 ms in FP64 (5 ranges)
constexpr long long kBinMinRanges = 4;
constexpr uint32_t kSelfMarkBit = 0x80000000u;  // a bin entry that marks a node of S_t (LocalCH)

// One binned update: destination node and value side by side, so that a tile's
// run of updates to one range is a single contiguous stream of 8-byte (FP32) or
// 16-byte (FP64) stores.
template <typename V>
struct alignas(sizeof(V) == 8 ? 16 : 8) BinEnt {
    int32_t w;
    V v;
};

// Device description of the bins of one workspace (value type V).
template <typename V>
struct BinArgs {
    int shift;               // S: range r holds nodes [r << S, (r + 1) << S)
    int nranges;             // 0: binning disabled for this graph
    long long min_edges;     // frontier volume from which the binned scatter runs
    const long long *base;   // [nranges + 1]: bin r occupies [base[r], base[r + 1])
    int32_t *cursor;         // [nranges]: entries written to bin r this iteration
    BinEnt<V> *be;           // the binned updates (destination node, value)
};

// Residual and degree of one node side by side, so that the atomic update of
// r_w and the read of d_w for the activation test hit the same cache line.
template <typename V>
struct alignas(2 * sizeof(V)) RD {
    V r;
    V d;
};

// Per-solve device counters.  Ping-pong slots are indexed by iteration parity.
struct DevState {
    unsigned long long packed[2];  // work-list reservation: (entries << 32) | edges
    int32_t fcount[2];             // frontier / candidate list lengths
    int32_t tcount[3];             // heat-kernel touched-list lengths (level mod 3)
    int32_t iters;                 // iterations with a nonempty active set
    int32_t pad0;
    long long ops;                 // sum vol(S_t)
    long long pushes;              // sum |S_t|
    double res_l1;                 // reported residual l1 norm
    unsigned long long res_dinf;   // bit pattern of the reported ||D^-1 r||_inf (>= 0)
    int32_t out_count;             // |union of S_t|: the pushed-set size found by the output scan
    int32_t empty_seen;            // an iteration found S_t empty (converged)
    int32_t probe;                 // LocalCH: active candidates at the iteration cap
    int32_t overflow;              // a list append found its capacity exhausted (invariant broken)
    int32_t small_t;               // single-workgroup launch: next iteration to run
    int32_t small_phase;           // 1: the snapshot of iteration small_t is done, its push is not
    int32_t fused_stamp;           // LocalCH: the range reduction took the snapshot of the iteration with this stamp
};

struct DetWS;   // buffers of the deterministic mode (gde_det.hip)
struct GlobWS;  // buffers of the global solvers (gde_global.hip)

// Solver workspace for one (graph, value type).  All node-indexed arrays are
// dense over n; between solves every entry is back at its rest value (zero),
// restored by the finalisation kernels, so a solve costs O(work), not O(n).
struct Workspace {
    const gde_graph *g = nullptr;
    uint64_t guid = 0;             // uid of the graph it was built for
    int vtype = 0;
    int64_t n = 0;
    size_t vsize = 0;
    void *rd = nullptr;            // RD<V>[n]  (residual plane 0 + degree)
    void *rd2 = nullptr;           // RD<V>[n]  heat-kernel plane 1 (lazily)
    void *x = nullptr;             // V[n]
    uint32_t *bitmap = nullptr;    // pushed set, ceil(n/32) words
    uint32_t *tbm = nullptr;       // nodes whose residual may be nonzero (LocalGD / LocalCH), ceil(n/32) words
    int32_t *front[2] = {nullptr, nullptr};
    int32_t *touched[3] = {nullptr, nullptr, nullptr};
    int32_t *wl_node = nullptr, *wl_beg = nullptr, *wl_off = nullptr;
    void *wl_sv = nullptr;
    int32_t *tile_start = nullptr;
    void *delta = nullptr;         // LocalCH previous update
    int32_t *dstamp = nullptr, *cstamp = nullptr;
    int32_t stamp_base = 1;
    int32_t *blk = nullptr;        // extraction block sums
    int64_t nblk = 0;
    DevState *st = nullptr;        // device
    DevState *hst = nullptr;       // pinned, host-coherent mirror of st
    uint32_t *hseq = nullptr;      // in the same allocation: sequence number of the last publication
    DevState *hst_dev = nullptr;   // device address of hst (for the publication kernel)
    uint32_t *hseq_dev = nullptr;  // device address of hseq
    uint32_t seq = 0;              // last sequence number asked for
    int32_t *seed_idx = nullptr;   // device staging for seeds
    double *seed_val = nullptr;
    int32_t seed_cap = 0;
    int32_t *h_seed_idx = nullptr; // pinned staging
    double *h_seed_val = nullptr;
    int32_t *out_idx = nullptr;    // device staging of the sparse output
    void *out_val = nullptr;
    int64_t out_cap = 0;
    int64_t *tr_size = nullptr, *tr_vol = nullptr;
    int64_t tr_cap = 0;
    int32_t *tr_nodes = nullptr;
    int64_t tr_nodes_cap = 0;
    double *lam_buf = nullptr;     // power-iteration vectors and reductions
    // binned scatter (graphs with at most kBinMaxRanges ranges)
    int bin_shift = 0;
    int bin_nranges = 0;
    long long *bin_base = nullptr; // device [nranges + 1]
    int32_t *bin_cursor = nullptr; // device [nranges], zero between iterations
    void *bin_e = nullptr;         // device [nnz_cap] BinEnt<V> entries
    int64_t nnz_cap = 0;           // CSR entries the tile table and bins can hold
    double *lvl_tab = nullptr;     // level push: device [2][kHkMaxLevels + 1], psi then level ratios
    std::vector<double> h_lvl;     // its host copy for the current solve
    DetWS *det = nullptr;          // deterministic mode, lazily
    GlobWS *glob = nullptr;        // global solvers, lazily
};

struct BatchWS;
void batch_ws_free(BatchWS *w);

}  // namespace gde

struct gde_graph {
    int device = 0;
    int32_t n = 0;
    int64_t nnz = 0;
    int32_t *row_ptr = nullptr;
    int32_t *col_idx = nullptr;
    bool owned = false;
    uint64_t uid = 0;
    int32_t d_max = 0;
};

struct gde_ctx {
    int device = 0;
    std::vector<gde::Workspace *> ws;
    // push-kernel timing (gde_ctx_profile)
    bool prof_on = false;
    std::vector<hipEvent_t> ev;   // pairs: [2i] before, [2i+1] after launch i of the current solve
    size_t ev_used = 0;
    int64_t prof_launches = 0, prof_edges = 0, prof_entries = 0;
    double prof_ms = 0.0;
    int64_t prof_b_launches = 0, prof_b_lane_edges = 0, prof_b_entries = 0;
    double prof_b_ms = 0.0;
    std::vector<gde::BatchWS *> bws;  // batched-solver workspaces
    // schedules chosen by gde_solve_batch's "auto" mode, per (graph, kind, value
    // type, batch size class): lanes and blocks per CU
    struct Tuned {
        uint64_t guid;
        int32_t kind, vtype, bclass, lanes, bpc;
    };
    std::vector<Tuned> tuned;
    hipEvent_t ev_b[2] = {nullptr, nullptr};
    int ev_b_used = 0;
    // batched push launches: event pairs of the current solve, and their totals
    std::vector<hipEvent_t> ev_bp;
    size_t ev_bp_used = 0;
    int64_t prof_bp_launches = 0, prof_b_rows = 0, prof_b_row_vol = 0;
    double prof_bp_ms = 0.0;
};

namespace gde {
// error reporting (thread-local message)
int fail(int status, const std::string &msg);
int hip_fail(hipError_t e, const char *what);
}  // namespace gde

#define GDE_HIP(call)                                               \
    do {                                                            \
        hipError_t _e = (call);                                     \
        if (_e != hipSuccess) return ::gde::hip_fail(_e, #call);    \
    } while (0)
