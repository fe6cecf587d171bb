// gde_server.hip -- continuous-batching server for diffusion queries on a
// dynamic graph.
//
// Queries wait in a FIFO queue.  PPR and Katz queries are packed, oldest
// first and kind by kind, into groups of L lanes of the node-major batched
// solver (gde_batch_kernels.hip).  A group is admitted as soon as a group
// slot is free (memory admission: at most max_groups slots, sized when the
// server is created), so new queries start while earlier groups are still
// iterating.  One engine step runs iters_per_step LocalGD iterations of every
// busy group in the same launches.  A group whose lanes have all converged (or
// that reached max_iters) is harvested: residual norms, sorted sparse outputs,
// completions, and its slot is free again.  Heat-kernel queries run through the
// plain level-push solver on the server's stream between engine steps.
//
// Edge insertions are applied between engine steps.  The device CSR is
// rebuilt with the new edges (O(nnz) at memory speed).  In-flight lanes keep
// their (x, r) and receive the corrections that keep r = b - Q x exact on the
// new graph:
//   PPR : the Insert correction of the dynamic GDE (Sec. 4, Algorithm 3), applied
//         to both directions of every new edge.  With k new edges at u and old
//         degree d0: r_w += (1-alpha) x_u / d0 for each new neighbour w,
//         r_u -= k x_u / d0, x_u *= (d0 + k) / d0.
//   Katz: Q = I - beta A gains -beta on (u,v) and (v,u): r_u += beta x_v, r_v += beta x_u.
// The residuals can now be negative, so the affected groups continue in
// candidate mode: the corrected pairs are candidates, a lane whose |r| an update
// lifts across its threshold becomes one, and the snapshot re-tests them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <mutex>
#include <shared_mutex>
#include <thread>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <set>
#include <string>
#include <unordered_set>
#include <vector>

#include "gde_batch.h"
#include "gde_batch_kernels.h"
#include "gde_device.h"
#include "gde_internal.h"
#include "gde_kernels.h"

namespace gde {

// ------------------------------------------------------------------ device helpers
// per (group) count of active pairs; pairs of dropped groups are removed (and
// their lanes flagged as unconverged), the rest compacted into `out`
__global__ void __launch_bounds__(kSnapBlock) k_srv_active(const uint64_t *__restrict__ in, const int32_t *cnt_in,
                                                            uint64_t *out, int32_t *cnt_out, int32_t cap, int32_t G,
                                                            const int32_t *__restrict__ drop, int32_t *group_active,
                                                            uint32_t *NM, uint32_t *unconv) {
    const int n_in = min(*cnt_in, cap);
    const int stride = gridDim.x * blockDim.x;
    for (int base = blockIdx.x * blockDim.x; base < n_in; base += stride) {  // workgroup-uniform trip count
        const int i = base + (int)threadIdx.x;
        bool keep = false;
        uint64_t p = 0;
        if (i < n_in) {
            p = in[i];
            const int32_t g = (int32_t)(p >> 32), u = (int32_t)(p & 0xffffffffull);
            if (drop[g]) {
                uint32_t *nm = &NM[(size_t)u * G + g];
                const uint32_t m = *nm;
                *nm = 0u;
                if (m) atomicOr(&unconv[g], m);
            } else {
                keep = true;
                if (group_active[g] == 0) group_active[g] = 1;  // a flag: any writer stores 1
            }
        }
        const int s = block_reserve(keep ? 1 : 0, cnt_out);
        if (keep && s < cap) out[s] = p;
    }
}

// residual norms of the harvested groups over their touched pairs (each read and
// zeroed once); the other groups' pairs are kept (compacted into `out`)
template <int L>
__global__ void __launch_bounds__(kBlock) k_srv_residual(const uint64_t *__restrict__ in, const int32_t *cnt_in,
                                                          uint64_t *out, int32_t *cnt_out, int32_t cap, int32_t G,
                                                          const int32_t *__restrict__ harvest, float *R, uint32_t *TM,
                                                          const float *__restrict__ deg,
                                                          const float *__restrict__ rscale, double *lane_l1,
                                                          unsigned long long *lane_dinf, int lds_lanes) {
    // per-lane partial norms in LDS (G*L lanes when they fit), one global add per lane and workgroup
    extern __shared__ __attribute__((aligned(16))) unsigned char s_res[];
    double *s_l1 = (double *)s_res;
    unsigned long long *s_dm = (unsigned long long *)(s_l1 + lds_lanes);
    constexpr int PPW = kWave / L;
    const int lane = (int)__lane_id();
    const int sub = lane / L, l = lane % L;
    const int n_in = min(*cnt_in, cap);
    const int wpb = (int)blockDim.x / kWave;
    for (int j = threadIdx.x; j < lds_lanes; j += blockDim.x) {
        s_l1[j] = 0.0;
        s_dm[j] = 0ull;
    }
    __syncthreads();
    for (int bbase = blockIdx.x * wpb * PPW; bbase < n_in; bbase += gridDim.x * wpb * PPW) {
        const int i = bbase + ((int)threadIdx.x / kWave) * PPW + sub;
        bool keep = false;
        uint64_t p = 0;
        if (i < n_in) {
            p = in[i];
            const int32_t g = (int32_t)(p >> 32), w = (int32_t)(p & 0xffffffffull);
            if (harvest[g]) {
                const size_t ri = ((size_t)w * G + g) * L + l;
                const float val = R[ri];
                R[ri] = 0.0f;
                const double av = fabs((double)val) * (double)rscale[g];
                if (av > 0.0) {
                    const int lane_id = g * L + l;
                    const unsigned long long bits = (unsigned long long)__double_as_longlong(av / (double)deg[w]);
                    if (lds_lanes) {
                        atomicAdd(&s_l1[lane_id], av);
                        if (s_dm[lane_id] < bits) atomicMax(&s_dm[lane_id], bits);
                    } else {
                        atomicAdd(&lane_l1[(size_t)lane_id * kStatShards + (blockIdx.x & (kStatShards - 1))], av);
                        if (lane_dinf[lane_id] < bits) atomicMax(&lane_dinf[lane_id], bits);
                    }
                }
            } else {
                keep = l == 0;
            }
        }
        const int s = block_reserve(keep ? 1 : 0, cnt_out);
        if (keep && s < cap) out[s] = p;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < lds_lanes; j += blockDim.x) {
        if (s_l1[j] != 0.0) atomicAdd(&lane_l1[(size_t)j * kStatShards + (blockIdx.x & (kStatShards - 1))], s_l1[j]);
        if (s_dm[j] != 0ull && lane_dinf[j] < s_dm[j]) atomicMax(&lane_dinf[j], s_dm[j]);
    }
}

// r <- b for the seeds of newly admitted lanes; (group, node) pairs join the active list
__global__ void k_srv_seed(float *R, uint32_t *NM, int32_t G, int L, const int32_t *__restrict__ s_lane,
                           const int32_t *__restrict__ s_node, const float *__restrict__ s_b, int32_t ns,
                           uint64_t *act, int32_t *acount, int32_t cap) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ns) {
        const int g = s_lane[i] / L, l = s_lane[i] % L;
        const int32_t u = s_node[i];
        R[((size_t)u * G + g) * L + l] = s_b[i];
        if (atomicOr(&NM[(size_t)u * G + g], 1u << l) == 0u) {
            const int s = atomicAdd(acount, 1);
            if (s < cap) act[s] = ((uint64_t)(uint32_t)g << 32) | (uint32_t)u;
        }
    }
}

// ---- CSR rebuild with a batch of new undirected edges (given as directed pairs e = (src, dst))
// flag[e] = 1 if the edge is already present in row src[e] (one wave per candidate)
__global__ void k_srv_present(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                              const int32_t *__restrict__ src, const int32_t *__restrict__ dst, int32_t m,
                              int32_t *flag) {
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int lane = (int)__lane_id();
    const int nwaves = gridDim.x * blockDim.x / kWave;
    for (int e = wave; e < m; e += nwaves) {
        const int32_t u = src[e], v = dst[e];
        bool hit = false;
        for (int32_t k = rp[u] + lane; k < rp[u + 1]; k += kWave) hit = hit || ci[k] == v;
        const unsigned long long b = __ballot(hit);
        if (lane == 0) flag[e] = b != 0ull;
    }
}

__global__ void k_srv_degrees(const int32_t *__restrict__ rp, int32_t n, int32_t *deg) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x)
        deg[u] = rp[u + 1] - rp[u];
}

__global__ void k_srv_count_new(const int32_t *__restrict__ src, int32_t m, int32_t *add) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) atomicAdd(&add[src[i]], 1);
}

// block-level inclusive sums of (old degree + added) -> partial row pointers
__global__ void __launch_bounds__(256) k_srv_scan_blocks(const int32_t *__restrict__ rp, const int32_t *__restrict__ add,
                                                         int32_t n, int32_t *newrp, int32_t *bsum) {
    __shared__ int s[256];
    const int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int v = u < n ? (rp[u + 1] - rp[u]) + add[u] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int y = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += y;
        __syncthreads();
    }
    if (u < n) newrp[u + 1] = s[threadIdx.x];
    if (threadIdx.x == 255) bsum[blockIdx.x] = s[255];
}

__global__ void __launch_bounds__(1024) k_srv_scan_sums(int32_t *bsum, int32_t nb) {
    __shared__ int s[1024];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nb; base += 1024) {
        const int i = base + threadIdx.x;
        const int v = i < nb ? bsum[i] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int y = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0;
            __syncthreads();
            s[threadIdx.x] += y;
            __syncthreads();
        }
        if (i < nb) bsum[i] = carry + s[threadIdx.x] - v;  // exclusive
        __syncthreads();
        if (threadIdx.x == 1023) carry += s[1023];
        __syncthreads();
    }
}

__global__ void k_srv_scan_add(int32_t *newrp, const int32_t *__restrict__ bsum, int32_t n) {
    const int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (u < n) newrp[u + 1] += bsum[blockIdx.x];
    if (u == 0) newrp[0] = 0;
}

// copy the old rows, then append the new edges after them
__global__ void k_srv_copy_rows(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                const int32_t *__restrict__ newrp, int32_t *newci, int32_t n, int32_t *cursor) {
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int lane = (int)__lane_id();
    const int nwaves = gridDim.x * blockDim.x / kWave;
    for (int u = wave; u < n; u += nwaves) {
        const int32_t b = rp[u], e = rp[u + 1], nb = newrp[u];
        for (int k = b + lane; k < e; k += kWave) newci[nb + (k - b)] = ci[k];
        if (lane == 0) cursor[u] = nb + (e - b);
    }
}

__global__ void k_srv_append(const int32_t *__restrict__ src, const int32_t *__restrict__ dst, int32_t m,
                             int32_t *newci, int32_t *cursor) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) newci[atomicAdd(&cursor[src[i]], 1)] = dst[i];
}

// in-flight corrections, per directed new edge (u -> w) and lane of a busy group
__global__ void k_srv_correct_edges(const int32_t *__restrict__ src, const int32_t *__restrict__ dst, int32_t m,
                                    const int32_t *__restrict__ old_deg, int32_t G, int L,
                                    const int32_t *__restrict__ busy_kind, const float *__restrict__ gparam, float *R,
                                    const float *__restrict__ X) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)m * G * L;
    if (idx >= total) return;
    const int e = (int)(idx / ((int64_t)G * L));
    const int gl = (int)(idx % ((int64_t)G * L));
    const int g = gl / L, l = gl % L;
    const int kind = busy_kind[g];  // -1 idle, GDE_PPR, GDE_KATZ
    if (kind < 0) return;
    const int32_t u = src[e], w = dst[e];
    if (kind == GDE_PPR) {
        const float xu = X[((size_t)u * G + g) * L + l];
        if (xu != 0.0f) atomicAdd(&R[((size_t)w * G + g) * L + l], (1.0f - gparam[g]) * xu / (float)old_deg[u]);
    } else {
        // directed event u -> w contributes beta x_w to r_u (its mirror w -> u gives beta x_u to r_w)
        const float xw = X[((size_t)w * G + g) * L + l];
        if (xw != 0.0f) atomicAdd(&R[((size_t)u * G + g) * L + l], gparam[g] * xw);
    }
}

// per node with k new edges: PPR r_u -= k x_u / d0, x_u *= (d0 + k) / d0; then every
// changed pair is marked touched and, with all its lanes, a candidate of the next snapshot
__global__ void k_srv_correct_nodes(const int32_t *__restrict__ nodes, int32_t nn, const int32_t *__restrict__ add,
                                    const int32_t *__restrict__ old_deg, int32_t G, int L,
                                    const int32_t *__restrict__ busy_kind, float *R, float *X, uint32_t *NM,
                                    uint32_t *TM, const uint32_t *__restrict__ g_epoch, uint64_t *act,
                                    int32_t *acount, int32_t act_cap, uint64_t *touched, int32_t *tcount,
                                    int32_t touch_cap) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)nn * G) return;
    const int j = (int)(idx / G), g = (int)(idx % G);
    const int kind = busy_kind[g];
    if (kind < 0) return;
    const int32_t u = nodes[j];
    if (kind == GDE_PPR) {
        const float d0 = (float)old_deg[u], k = (float)add[u];
        for (int l = 0; l < L; l++) {
            const size_t ri = ((size_t)u * G + g) * L + l;
            const float xu = X[ri];
            if (xu != 0.0f) {
                R[ri] -= k * xu / d0;  // this node's own lanes: no concurrent writer in this kernel
                X[ri] = xu * (d0 + k) / d0;
            }
        }
    }
    const uint32_t all = (L == 32) ? 0xffffffffu : ((1u << L) - 1u);
    if (atomicOr(&NM[(size_t)u * G + g], all) == 0u) {
        const int s = atomicAdd(acount, 1);
        if (s < act_cap) act[s] = ((uint64_t)(uint32_t)g << 32) | (uint32_t)u;
    }
    if (atomicExch(&TM[(size_t)u * G + g], g_epoch[g]) != g_epoch[g]) {
        const int s = atomicAdd(tcount, 1);
        if (s < touch_cap) touched[s] = ((uint64_t)(uint32_t)g << 32) | (uint32_t)u;
    }
}

// ------------------------------------------------------------------ host side
static double now_s(const std::chrono::steady_clock::time_point &t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

struct SReq {
    uint64_t ticket = 0;
    gde_params p{};
    std::vector<int32_t> idx;
    std::vector<double> val;
    std::vector<double> coef;  // GDE_SERIES: the server's copy of p.c
    double t_sub = 0.0;
};

struct SGroup {
    bool busy = false;
    int kind = -1;
    double param = 0.0;  // alpha (PPR) or beta (Katz)
    uint32_t epoch = 0;  // touched-pair tag of the group's current occupants
    int start_t = 0;
    int max_iters = 0;
    bool cand = false;
    std::vector<SReq> lanes;
};

// Heat-kernel queries are solved by the plain level-push solver on worker
// threads, each with a private context (its own dense workspace) and stream,
// so that several run at once beside the batched groups.
// Three workers plus the engine stream keep the server within the four
// hardware queues a process gets, so the engine never shares a queue.
constexpr int kHkWorkers = 3;

struct HkWorker {
    gde_ctx *ctx = nullptr;
    hipStream_t s = nullptr;
    std::thread th;
    std::vector<int32_t> idx;
    std::vector<float> val;
};

struct HkDone {
    gde_completion c{};
    std::vector<int32_t> idx;
    std::vector<float> val;
};

}  // namespace gde

struct gde_server {
    gde_ctx *user_ctx = nullptr;
    gde_ctx *ctx = nullptr;  // private context: the server's workspaces
    gde_graph *g = nullptr;  // private, rebuilt on insertions
    hipStream_t s = nullptr;
    gde_server_cfg cfg{};
    int L = 16, G = 8;
    int t = 0;  // global iteration counter (list parity)
    uint64_t next_ticket = 1;
    std::chrono::steady_clock::time_point t0;
    // pending PPR / Katz queries, one FIFO per (kind, alpha or beta): a free group
    // takes the key whose head is the oldest and fills its lanes from that FIFO
    std::map<std::pair<int, double>, std::deque<gde::SReq>> pending;
    int64_t n_pending = 0;
    std::vector<gde::SGroup> groups;
    std::vector<std::pair<int32_t, int32_t>> inserts;
    std::vector<gde_completion> done;
    std::vector<std::vector<int32_t>> done_idx;
    std::vector<std::vector<float>> done_val;
    size_t done_read = 0;
    gde::BatchWS *w = nullptr;
    // device scratch for the server
    int32_t *d_drop = nullptr, *d_gactive = nullptr, *d_kind = nullptr, *d_mode = nullptr, *d_cnt = nullptr;
    float *d_gws = nullptr, *d_gparam = nullptr, *d_rscale = nullptr;
    uint32_t *d_gepoch = nullptr;  // [G] touched-pair tags
    uint32_t epoch_next = 1;
    uint64_t *d_act_tmp = nullptr;    // compaction target of the active list (capacity act_cap)
    uint64_t *d_touch_tmp = nullptr;  // compaction target of the touched list (capacity touch_cap)
    float *d_seed_b = nullptr;
    int32_t *d_seed_lane = nullptr, *d_seed_node = nullptr;
    int32_t seed_cap = 0;
    int32_t *d_out_idx = nullptr;
    float *d_out_val = nullptr;
    int64_t out_cap = 0;
    int64_t inserted_edges = 0;
    // insertion buffers, kept across batches: the CSR being built next (spare)
    // and the node-sized and batch-sized scratch
    int32_t *spare_rp = nullptr, *spare_ci = nullptr;
    int64_t spare_ci_cap = 0, cur_ci_cap = 0;
    int32_t *t_add = nullptr, *t_olddeg = nullptr, *t_cursor = nullptr, *t_bsum = nullptr;
    int32_t *t_src = nullptr, *t_dst = nullptr, *t_flag = nullptr;
    int64_t t_cap = 0;
    // heat-kernel workers: a queue of queries, their completions, and a lock that
    // solves hold shared and graph rebuilds hold exclusive
    std::vector<gde::HkWorker *> hk_w;
    std::mutex hk_mu;
    std::condition_variable hk_cv;       // workers wait for a query or for stop
    std::condition_variable hk_done_cv;  // poll waits for a completion
    std::deque<gde::SReq> hk_queue;
    std::vector<gde::HkDone> hk_done;
    int64_t hk_running = 0;
    bool hk_stop = false;
    bool hk_gate = false;                // a rebuild waits: workers start no new solve
    int hk_err = 0;                      // a worker's solve failed with a device error
    std::shared_mutex graph_mu;
    // the step enqueued by srv_step_launch and not yet finished
    bool step_open = false;
    std::vector<int32_t> step_drop;
};

namespace gde {

// internal access to the batch workspace layout (gde_batch.hip)
int batch_ws_acquire(gde_ctx *ctx, const gde_graph *g, int vtype, int L, int G, hipStream_t s, BatchWS **out);
void batch_args_from_ws(BatchWS *w, const gde_graph *g, int G, BatchArgs<float> *a);
int32_t *batch_ws_touch_count(BatchWS *w);
void plain_workspaces_drop(const gde_graph *g, gde_ctx *ctx);
int plain_workspaces_refresh(const gde_graph *g, gde_ctx *ctx, hipStream_t s);
gde_graph *graph_wrap_device(gde_ctx *ctx, int32_t n, int64_t nnz, int32_t *rp, int32_t *ci);
int graph_replace_csr(gde_graph *g, int32_t *rp, int32_t *ci, int64_t nnz, const std::vector<int32_t> &inc);

static int srv_args(gde_server *sv, BatchArgs<float> *a) {
    batch_args_from_ws(sv->w, sv->g, sv->G, a);
    a->g_wscale = sv->d_gws;
    a->g_epoch = sv->d_gepoch;
    a->g_mode = sv->d_mode;
    a->max_iters = 1 << 30;
    return GDE_OK;
}

static int srv_upload_group_params(gde_server *sv) {
    std::vector<int32_t> kind(sv->G, -1), mode(sv->G, 0);
    std::vector<float> ws(sv->G, 0.f), prm(sv->G, 0.f), rsc(sv->G, 1.f);
    std::vector<uint32_t> ep(sv->G, 0u);
    for (int gi = 0; gi < sv->G; gi++) {
        const SGroup &gr = sv->groups[gi];
        if (!gr.busy) continue;
        kind[gi] = gr.kind;
        ep[gi] = gr.epoch;
        prm[gi] = (float)gr.param;
        ws[gi] = (float)(gr.kind == GDE_PPR ? 1.0 - gr.param : gr.param);
        mode[gi] = (gr.kind == GDE_PPR ? 1 : 0) | (gr.cand ? 2 : 0);
        rsc[gi] = (float)(gr.kind == GDE_PPR ? 1.0 / gr.param : 1.0);
    }
    GDE_HIP(hipMemcpyAsync(sv->d_kind, kind.data(), 4 * sv->G, hipMemcpyHostToDevice, sv->s));
    GDE_HIP(hipMemcpyAsync(sv->d_mode, mode.data(), 4 * sv->G, hipMemcpyHostToDevice, sv->s));
    GDE_HIP(hipMemcpyAsync(sv->d_gws, ws.data(), 4 * sv->G, hipMemcpyHostToDevice, sv->s));
    GDE_HIP(hipMemcpyAsync(sv->d_gparam, prm.data(), 4 * sv->G, hipMemcpyHostToDevice, sv->s));
    GDE_HIP(hipMemcpyAsync(sv->d_rscale, rsc.data(), 4 * sv->G, hipMemcpyHostToDevice, sv->s));
    GDE_HIP(hipMemcpyAsync(sv->d_gepoch, ep.data(), 4 * sv->G, hipMemcpyHostToDevice, sv->s));
    return GDE_OK;
}

// fill free group slots from the queue (oldest first, one kind and parameter per group)
static int srv_admit(gde_server *sv) {
    std::vector<int32_t> s_lane, s_node;
    std::vector<float> s_b;
    std::vector<float> eps_upd;
    std::vector<int> admitted;
    for (int gi = 0; gi < sv->G && sv->n_pending > 0; gi++) {
        SGroup &gr = sv->groups[gi];
        if (gr.busy) continue;
        // the oldest pending request decides the group's kind and parameter
        auto best = sv->pending.end();
        for (auto qt = sv->pending.begin(); qt != sv->pending.end(); ++qt)
            if (best == sv->pending.end() || qt->second.front().ticket < best->second.front().ticket) best = qt;
        if (best == sv->pending.end()) break;
        std::deque<SReq> &q = best->second;
        gr = SGroup();
        gr.busy = true;
        // a fresh tag: pairs the previous occupants touched read as untouched
        if (sv->epoch_next == 0u) {
            BatchArgs<float> ta{};
            batch_args_from_ws(sv->w, sv->g, sv->G, &ta);
            GDE_HIP(hipMemsetAsync(ta.TM, 0, (size_t)sv->g->n * sv->G * 4, sv->s));
            sv->epoch_next = 1u;
        }
        gr.epoch = sv->epoch_next++;
        gr.kind = best->first.first;
        gr.param = best->first.second;
        gr.start_t = sv->t;
        gr.max_iters = 0;
        while (!q.empty() && (int)gr.lanes.size() < sv->L) {
            gr.max_iters = std::max(gr.max_iters, q.front().p.max_iters);
            gr.lanes.push_back(std::move(q.front()));
            q.pop_front();
            sv->n_pending--;
        }
        if (q.empty()) sv->pending.erase(best);
        admitted.push_back(gi);
        for (int l = 0; l < (int)gr.lanes.size(); l++) {
            const SReq &r = gr.lanes[l];
            const double bsc = gr.kind == GDE_PPR ? gr.param : 1.0;
            for (size_t k = 0; k < r.idx.size(); k++) {
                s_lane.push_back(gi * sv->L + l);
                s_node.push_back(r.idx[k]);
                s_b.push_back((float)(bsc * r.val[k]));
            }
        }
    }
    if (admitted.empty()) return GDE_OK;
    BatchArgs<float> a{};
    srv_args(sv, &a);
    // lane thresholds and per-lane statistics of the admitted groups
    std::vector<float> eps((size_t)sv->G * sv->L);
    GDE_HIP(hipMemcpyAsync(eps.data(), a.lane_eps, 4 * eps.size(), hipMemcpyDeviceToHost, sv->s));
    GDE_HIP(hipStreamSynchronize(sv->s));
    for (int gi : admitted) {
        const SGroup &gr = sv->groups[gi];
        for (int l = 0; l < sv->L; l++) {
            const size_t j = (size_t)gi * sv->L + l;
            if (l < (int)gr.lanes.size()) {
                const gde_params &p = gr.lanes[l].p;
                eps[j] = (float)(gr.kind == GDE_PPR ? p.alpha * p.eps : p.eps);
            } else {
                eps[j] = 3.0e38f;  // an empty lane never activates
            }
        }
        const size_t lo = (size_t)gi * sv->L;
        GDE_HIP(hipMemsetAsync(a.lane_ops + lo * kStatShards, 0, 8 * sv->L * kStatShards, sv->s));
        GDE_HIP(hipMemsetAsync(a.lane_l1 + lo * kStatShards, 0, 8 * sv->L * kStatShards, sv->s));
        GDE_HIP(hipMemsetAsync(a.lane_T + lo, 0, 4 * sv->L, sv->s));
        GDE_HIP(hipMemsetAsync(a.lane_dinf + lo, 0, 8 * sv->L, sv->s));
        GDE_HIP(hipMemsetAsync(a.group_unconv + gi, 0, 4, sv->s));
    }
    GDE_HIP(hipMemcpyAsync((void *)a.lane_eps, eps.data(), 4 * eps.size(), hipMemcpyHostToDevice, sv->s));
    int rc = srv_upload_group_params(sv);
    if (rc) return rc;
    const int32_t ns = (int32_t)s_lane.size();
    if (ns > sv->seed_cap) {
        if (sv->d_seed_lane) { (void)hipFree(sv->d_seed_lane); (void)hipFree(sv->d_seed_node); (void)hipFree(sv->d_seed_b); }
        GDE_HIP(hipMalloc((void **)&sv->d_seed_lane, 4 * (size_t)ns));
        GDE_HIP(hipMalloc((void **)&sv->d_seed_node, 4 * (size_t)ns));
        GDE_HIP(hipMalloc((void **)&sv->d_seed_b, 4 * (size_t)ns));
        sv->seed_cap = ns;
    }
    GDE_HIP(hipMemcpyAsync(sv->d_seed_lane, s_lane.data(), 4 * (size_t)ns, hipMemcpyHostToDevice, sv->s));
    GDE_HIP(hipMemcpyAsync(sv->d_seed_node, s_node.data(), 4 * (size_t)ns, hipMemcpyHostToDevice, sv->s));
    GDE_HIP(hipMemcpyAsync(sv->d_seed_b, s_b.data(), 4 * (size_t)ns, hipMemcpyHostToDevice, sv->s));
    const int cur = sv->t & 1;
    if (ns > 0) {
        hipLaunchKernelGGL(k_srv_seed, dim3((ns + 255) / 256), dim3(256), 0, sv->s, a.R, a.NM, sv->G, sv->L,
                           sv->d_seed_lane, sv->d_seed_node, sv->d_seed_b, ns, a.act[cur], &a.st->acount[cur],
                           a.act_cap);
        GDE_HIP(hipGetLastError());
    }
    // The seeds' pairs are not put on the touched list here: every lane's first
    // snapshot is forced (S_0 = supp(s)) and takes the whole seed residual, so a
    // seed pair holds a nonzero residual later only if a push reaches it, and
    // that push marks it as touched.
    return GDE_OK;
}

// harvest the groups flagged in `hv`: residual norms, sorted outputs, completions
static int srv_harvest(gde_server *sv, const std::vector<int> &hv_groups, const std::vector<int32_t> &hv_flag) {
    if (hv_groups.empty()) return GDE_OK;
    BatchWS *w = sv->w;
    BatchArgs<float> a{};
    srv_args(sv, &a);
    const int G = sv->G, L = sv->L;
    GDE_HIP(hipMemcpyAsync(sv->d_drop, hv_flag.data(), 4 * G, hipMemcpyHostToDevice, sv->s));
    // residual over the touched pairs of the harvested groups; keep the rest
    int32_t *tcnt = batch_ws_touch_count(w);
    GDE_HIP(hipMemsetAsync(sv->d_cnt, 0, 4, sv->s));
    const int grid = 1024;
    const int lds_lanes = G * L <= kResLdsLanes ? G * L : 0;
    const size_t dyn = 16 * (size_t)lds_lanes;
    switch (L) {
    case 8: hipLaunchKernelGGL(k_srv_residual<8>, dim3(grid), dim3(kBlock), dyn, sv->s, a.touched, tcnt, sv->d_touch_tmp, sv->d_cnt, a.touch_cap, G, sv->d_drop, a.R, a.TM, a.deg, sv->d_rscale, a.lane_l1, a.lane_dinf, lds_lanes); break;
    case 16: hipLaunchKernelGGL(k_srv_residual<16>, dim3(grid), dim3(kBlock), dyn, sv->s, a.touched, tcnt, sv->d_touch_tmp, sv->d_cnt, a.touch_cap, G, sv->d_drop, a.R, a.TM, a.deg, sv->d_rscale, a.lane_l1, a.lane_dinf, lds_lanes); break;
    default: hipLaunchKernelGGL(k_srv_residual<32>, dim3(grid), dim3(kBlock), dyn, sv->s, a.touched, tcnt, sv->d_touch_tmp, sv->d_cnt, a.touch_cap, G, sv->d_drop, a.R, a.TM, a.deg, sv->d_rscale, a.lane_l1, a.lane_dinf, lds_lanes); break;
    }
    GDE_HIP(hipGetLastError());
    // the compacted list becomes the touched list
    batch_ws_swap_list(w, 2, &sv->d_touch_tmp);
    GDE_HIP(hipMemcpyAsync(tcnt, sv->d_cnt, 4, hipMemcpyDeviceToDevice, sv->s));
    srv_args(sv, &a);
    // extraction of the harvested groups
    int32_t *gmap = sv->d_gactive;  // reuse as the group map
    GDE_HIP(hipMemcpyAsync(gmap, hv_groups.data(), 4 * hv_groups.size(), hipMemcpyHostToDevice, sv->s));
    const int ng = (int)hv_groups.size();
    int nblk = (int)((a.nwords + kBlock - 1) / kBlock);
    long long *lane_nnz = nullptr, *lane_off = nullptr;
    int32_t *cnt = nullptr;
    batch_ws_extract_buffers(w, &cnt, &lane_nnz, &lane_off);
    GDE_HIP(batch_extract<float>(L, a, 0, cnt, nblk, lane_nnz, nullptr, nullptr, nullptr, 0, sv->s, gmap, ng));
    std::vector<long long> nnz((size_t)G * L), off((size_t)G * L, -1);
    GDE_HIP(hipMemcpyAsync(nnz.data(), lane_nnz, 8 * nnz.size(), hipMemcpyDeviceToHost, sv->s));
    GDE_HIP(hipStreamSynchronize(sv->s));
    long long total = 0;
    const long long rcap = std::max<int32_t>(sv->cfg.result_capacity, 1);
    for (int gi : hv_groups)
        for (int l = 0; l < (int)sv->groups[gi].lanes.size(); l++) {
            const size_t j = (size_t)gi * L + l;
            if (nnz[j] <= rcap) { off[j] = total; total += nnz[j]; }
        }
    if (total > sv->out_cap) {
        if (sv->d_out_idx) { (void)hipFree(sv->d_out_idx); (void)hipFree(sv->d_out_val); }
        sv->d_out_idx = nullptr; sv->d_out_val = nullptr; sv->out_cap = 0;
        GDE_HIP(hipMalloc((void **)&sv->d_out_idx, 4 * (size_t)std::max<long long>(total, 1)));
        GDE_HIP(hipMalloc((void **)&sv->d_out_val, 4 * (size_t)std::max<long long>(total, 1)));
        sv->out_cap = total;
    }
    GDE_HIP(hipMemcpyAsync(lane_off, off.data(), 8 * off.size(), hipMemcpyHostToDevice, sv->s));
    GDE_HIP(batch_extract<float>(L, a, 1, cnt, nblk, lane_nnz, lane_off, sv->d_out_idx, sv->d_out_val, 1, sv->s, gmap, ng));
    std::vector<int32_t> h_idx(total);
    std::vector<float> h_val(total);
    if (total > 0) {
        GDE_HIP(hipMemcpyAsync(h_idx.data(), sv->d_out_idx, 4 * total, hipMemcpyDeviceToHost, sv->s));
        GDE_HIP(hipMemcpyAsync(h_val.data(), sv->d_out_val, 4 * total, hipMemcpyDeviceToHost, sv->s));
    }
    const size_t GL = (size_t)G * L;
    std::vector<double> l1(GL * kStatShards);
    std::vector<int32_t> T(GL);
    std::vector<unsigned long long> dinf(GL);
    std::vector<uint32_t> unconv(G);
    GDE_HIP(hipMemcpyAsync(l1.data(), a.lane_l1, 8 * l1.size(), hipMemcpyDeviceToHost, sv->s));
    GDE_HIP(hipMemcpyAsync(T.data(), a.lane_T, 4 * T.size(), hipMemcpyDeviceToHost, sv->s));
    GDE_HIP(hipMemcpyAsync(dinf.data(), a.lane_dinf, 8 * dinf.size(), hipMemcpyDeviceToHost, sv->s));
    GDE_HIP(hipMemcpyAsync(unconv.data(), a.group_unconv, 4 * unconv.size(), hipMemcpyDeviceToHost, sv->s));
    GDE_HIP(hipStreamSynchronize(sv->s));
    const double now = now_s(sv->t0);
    for (int gi : hv_groups) {
        SGroup &gr = sv->groups[gi];
        for (int l = 0; l < (int)gr.lanes.size(); l++) {
            const size_t j = (size_t)gi * L + l;
            gde_completion c{};
            c.ticket = gr.lanes[l].ticket;
            c.submit_time_s = gr.lanes[l].t_sub;
            c.done_time_s = now;
            c.iters = std::max(0, T[j] - gr.start_t);
            double sl = 0.0;
            for (int sh = 0; sh < kStatShards; sh++) sl += l1[j * kStatShards + sh];
            c.residual_l1 = sl;
            std::memcpy(&c.residual_dinf, &dinf[j], 8);
            std::vector<int32_t> ii;
            std::vector<float> vv;
            if (off[j] >= 0) {
                ii.assign(h_idx.begin() + off[j], h_idx.begin() + off[j] + nnz[j]);
                vv.assign(h_val.begin() + off[j], h_val.begin() + off[j] + nnz[j]);
                c.status = ((unconv[gi] >> l) & 1u) ? GDE_ERR_NOT_CONVERGED : GDE_OK;
            } else {
                c.status = GDE_ERR_CAPACITY;
            }
            c.nnz = off[j] >= 0 ? nnz[j] : 0;
            sv->done.push_back(c);
            sv->done_idx.push_back(std::move(ii));
            sv->done_val.push_back(std::move(vv));
        }
        gr = SGroup();
    }
    return srv_upload_group_params(sv);
}

// one engine step: iters_per_step iterations of every busy group, then harvest
// Enqueue iters_per_step batched iterations and the per-group activity count
// on the server's stream without waiting for them; srv_step_finish reads the
// result.  Heat-kernel solves run on their own stream in between.
static int srv_step_launch(gde_server *sv) {
    bool any = false;
    for (const SGroup &gr : sv->groups) any = any || gr.busy;
    if (!any) return GDE_OK;
    BatchArgs<float> a{};
    srv_args(sv, &a);
    int dev = 0, cus = 0, occ = 0;
    GDE_HIP(hipGetDevice(&dev));
    GDE_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    GDE_HIP(batch_occupancy<float>(sv->L, &occ));
    const int grid = std::max(1, occ) * cus;
    for (int k = 0; k < std::max(1, sv->cfg.iters_per_step); k++, sv->t++) {
        GDE_HIP(batch_launch<float>(1, sv->L, a, grid, sv->t, sv->s));
        GDE_HIP(batch_launch<float>(2, sv->L, a, grid, sv->t, sv->s));
    }
    // per-group active pairs; groups over their iteration cap are dropped
    std::vector<int32_t> &drop = sv->step_drop;
    drop.assign(sv->G, 0);
    for (int gi = 0; gi < sv->G; gi++)
        if (sv->groups[gi].busy && sv->t - sv->groups[gi].start_t >= sv->groups[gi].max_iters) drop[gi] = 1;
    const int cur = sv->t & 1;
    GDE_HIP(hipMemcpyAsync(sv->d_drop, drop.data(), 4 * sv->G, hipMemcpyHostToDevice, sv->s));
    GDE_HIP(hipMemsetAsync(sv->d_gactive, 0, 4 * sv->G, sv->s));
    GDE_HIP(hipMemsetAsync(sv->d_cnt, 0, 4, sv->s));
    hipLaunchKernelGGL(k_srv_active, dim3(512), dim3(kSnapBlock), 0, sv->s, a.act[cur], &a.st->acount[cur], sv->d_act_tmp,
                       sv->d_cnt, a.act_cap, sv->G, sv->d_drop, sv->d_gactive, a.NM, a.group_unconv);
    GDE_HIP(hipGetLastError());
    batch_ws_swap_list(sv->w, cur, &sv->d_act_tmp);
    GDE_HIP(hipMemcpyAsync(&a.st->acount[cur], sv->d_cnt, 4, hipMemcpyDeviceToDevice, sv->s));
    sv->step_open = true;
    return GDE_OK;
}

// Wait for the enqueued step and harvest the groups that converged or reached
// their iteration cap.
static int srv_step_finish(gde_server *sv) {
    if (!sv->step_open) return GDE_OK;
    sv->step_open = false;
    BatchArgs<float> a{};
    srv_args(sv, &a);
    std::vector<int32_t> gact(sv->G);
    BatchDev hst{};
    GDE_HIP(hipMemcpyAsync(gact.data(), sv->d_gactive, 4 * sv->G, hipMemcpyDeviceToHost, sv->s));
    GDE_HIP(hipMemcpyAsync(&hst, a.st, sizeof(BatchDev), hipMemcpyDeviceToHost, sv->s));
    GDE_HIP(hipStreamSynchronize(sv->s));
    if (hst.ovf[0] || hst.ovf[1]) return fail(GDE_ERR_OOM, "server work lists exceeded their capacity");
    const std::vector<int32_t> &drop = sv->step_drop;
    std::vector<int> hv;
    std::vector<int32_t> flag(sv->G, 0);
    for (int gi = 0; gi < sv->G; gi++)
        if (sv->groups[gi].busy && (gact[gi] == 0 || drop[gi])) { hv.push_back(gi); flag[gi] = 1; }
    return srv_harvest(sv, hv, flag);
}

// One heat-kernel worker: takes the oldest queued query, solves it on its own
// context and stream while holding the graph lock shared, and queues the
// completion for the next poll.
static void hk_worker_main(gde_server *sv, HkWorker *wk) {
    (void)hipSetDevice(wk->ctx->device);
    const int64_t cap = std::max<int32_t>(sv->cfg.result_capacity, 1);
    for (;;) {
        SReq q;
        {
            std::unique_lock<std::mutex> lk(sv->hk_mu);
            sv->hk_cv.wait(lk, [&] { return sv->hk_stop || (!sv->hk_queue.empty() && !sv->hk_gate); });
            if (sv->hk_stop) return;
            q = std::move(sv->hk_queue.front());
            sv->hk_queue.pop_front();
            sv->hk_running++;
        }
        HkDone d;
        {
            std::shared_lock<std::shared_mutex> gl(sv->graph_mu);
            gde_seed sd{(int32_t)q.idx.size(), q.idx.data(), q.val.data()};
            gde_params p = q.p;
            if (p.kind == GDE_SERIES) p.c = q.coef.data();
            p.value_type = GDE_F32;
            p.flags &= ~(uint32_t)(GDE_RESULT_DEVICE | GDE_TRACE);
            gde_result r{};
            r.capacity = cap;
            r.idx = wk->idx.data();
            r.val = wk->val.data();
            const int rc = gde_solve(wk->ctx, sv->g, &p, &sd, &r, wk->s);
            // nothing of this solve may still run when a rebuild takes the lock
            const hipError_t e = hipStreamSynchronize(wk->s);
            d.c.ticket = q.ticket;
            d.c.submit_time_s = q.t_sub;
            d.c.status = (rc == GDE_OK && e != hipSuccess) ? GDE_ERR_DEVICE : rc;
            d.c.iters = r.iters;
            d.c.residual_l1 = r.residual_l1;
            d.c.residual_dinf = r.residual_dinf;
            d.c.nnz = (d.c.status == GDE_OK || d.c.status == GDE_ERR_NOT_CONVERGED) ? r.nnz : 0;
            d.idx.assign(wk->idx.begin(), wk->idx.begin() + d.c.nnz);
            d.val.assign(wk->val.begin(), wk->val.begin() + d.c.nnz);
        }
        {
            std::lock_guard<std::mutex> lk(sv->hk_mu);
            if (d.c.status == GDE_ERR_DEVICE) sv->hk_err = GDE_ERR_DEVICE;
            sv->hk_done.push_back(std::move(d));
            sv->hk_running--;
        }
        sv->hk_done_cv.notify_all();
    }
}

// Move finished heat-kernel queries to the completions.  When this poll found
// nothing else to do and heat-kernel queries are still running, wait briefly
// for one of them.
static int srv_hk_collect(gde_server *sv, bool idle) {
    std::unique_lock<std::mutex> lk(sv->hk_mu);
    if (idle && sv->done.empty() && sv->hk_done.empty() && (sv->hk_running > 0 || !sv->hk_queue.empty()))
        sv->hk_done_cv.wait_for(lk, std::chrono::milliseconds(2), [&] { return !sv->hk_done.empty(); });
    const double t = now_s(sv->t0);
    for (HkDone &d : sv->hk_done) {
        d.c.done_time_s = t;
        sv->done.push_back(d.c);
        sv->done_idx.push_back(std::move(d.idx));
        sv->done_val.push_back(std::move(d.val));
    }
    sv->hk_done.clear();
    return sv->hk_err;
}

// apply the queued insertions: rebuild the CSR, correct in-flight lanes
static int srv_apply_inserts(gde_server *sv) {
    if (sv->inserts.empty()) return GDE_OK;
    // Heat-kernel solves read the CSR and the plain workspaces that this
    // rebuilds.  The gate keeps workers from starting new solves meanwhile (the
    // shared mutex alone may keep admitting readers ahead of this writer).
    struct Gate {
        gde_server *sv;
        explicit Gate(gde_server *v) : sv(v) {
            std::lock_guard<std::mutex> lk(sv->hk_mu);
            sv->hk_gate = true;
        }
        ~Gate() {
            {
                std::lock_guard<std::mutex> lk(sv->hk_mu);
                sv->hk_gate = false;
            }
            sv->hk_cv.notify_all();
        }
    } gate(sv);
    std::unique_lock<std::shared_mutex> gl(sv->graph_mu);
    // host: drop self-loops and repeats within the batch, keep canonical pairs
    std::set<std::pair<int32_t, int32_t>> uniq;
    for (auto &e : sv->inserts)
        if (e.first != e.second) uniq.insert({std::min(e.first, e.second), std::max(e.first, e.second)});
    sv->inserts.clear();
    // drop edges already present (checked on the device, one wave per candidate)
    std::vector<int32_t> src, dst;
    {
        std::vector<int32_t> cu, cv;
        for (const auto &e : uniq) { cu.push_back(e.first); cv.push_back(e.second); }
        const int32_t mc = (int32_t)cu.size();
        if (2 * (int64_t)mc > sv->t_cap) {  // batch-sized scratch, grown geometrically
            (void)hipFree(sv->t_src); (void)hipFree(sv->t_dst); (void)hipFree(sv->t_flag);
            sv->t_src = sv->t_dst = sv->t_flag = nullptr;
            const int64_t c = std::max<int64_t>(2 * (int64_t)mc, 2 * sv->t_cap);
            GDE_HIP(hipMalloc((void **)&sv->t_src, 4 * (size_t)c));
            GDE_HIP(hipMalloc((void **)&sv->t_dst, 4 * (size_t)c));
            GDE_HIP(hipMalloc((void **)&sv->t_flag, 4 * (size_t)c));
            sv->t_cap = c;
        }
        int32_t *du = sv->t_src, *dv = sv->t_dst, *fl = sv->t_flag;
        GDE_HIP(hipMemcpyAsync(du, cu.data(), 4 * (size_t)mc, hipMemcpyHostToDevice, sv->s));
        GDE_HIP(hipMemcpyAsync(dv, cv.data(), 4 * (size_t)mc, hipMemcpyHostToDevice, sv->s));
        hipLaunchKernelGGL(k_srv_present, dim3(1024), dim3(256), 0, sv->s, sv->g->row_ptr, sv->g->col_idx, du, dv, mc,
                           fl);
        std::vector<int32_t> hf(mc);
        GDE_HIP(hipMemcpyAsync(hf.data(), fl, 4 * (size_t)mc, hipMemcpyDeviceToHost, sv->s));
        GDE_HIP(hipStreamSynchronize(sv->s));
        for (int32_t i = 0; i < mc; i++) {
            if (hf[i]) continue;
            src.push_back(cu[i]); dst.push_back(cv[i]);
            src.push_back(cv[i]); dst.push_back(cu[i]);
        }
    }
    const int32_t m = (int32_t)src.size();
    if (m == 0) return GDE_OK;
    const int32_t n = sv->g->n;
    const int64_t new_nnz = sv->g->nnz + m;
    if (new_nnz >= (int64_t)INT32_MAX) return fail(GDE_ERR_OOM, "graph would exceed 2^31 entries");
    const int nb = (n + 255) / 256;
    if (!sv->t_add) {  // node-sized scratch, allocated once
        GDE_HIP(hipMalloc((void **)&sv->t_add, 4 * (size_t)n));
        GDE_HIP(hipMalloc((void **)&sv->t_olddeg, 4 * (size_t)n));
        GDE_HIP(hipMalloc((void **)&sv->t_cursor, 4 * (size_t)n));
        GDE_HIP(hipMalloc((void **)&sv->t_bsum, 4 * (size_t)nb));
        GDE_HIP(hipMalloc((void **)&sv->spare_rp, 4 * ((size_t)n + 1)));
    }
    if (sv->spare_ci_cap < new_nnz) {  // the next CSR, with room for later batches
        (void)hipFree(sv->spare_ci);
        sv->spare_ci = nullptr;
        const int64_t c = std::min<int64_t>(new_nnz + new_nnz / 8 + 65536, (int64_t)INT32_MAX);
        GDE_HIP(hipMalloc((void **)&sv->spare_ci, 4 * (size_t)c));
        sv->spare_ci_cap = c;
    }
    if (m > sv->t_cap) {
        (void)hipFree(sv->t_src); (void)hipFree(sv->t_dst); (void)hipFree(sv->t_flag);
        sv->t_src = sv->t_dst = sv->t_flag = nullptr;
        GDE_HIP(hipMalloc((void **)&sv->t_src, 4 * (size_t)m));
        GDE_HIP(hipMalloc((void **)&sv->t_dst, 4 * (size_t)m));
        GDE_HIP(hipMalloc((void **)&sv->t_flag, 4 * (size_t)m));
        sv->t_cap = m;
    }
    int32_t *d_src = sv->t_src, *d_dst = sv->t_dst, *add = sv->t_add, *newrp = sv->spare_rp, *newci = sv->spare_ci,
            *cursor = sv->t_cursor, *bsum = sv->t_bsum, *olddeg = sv->t_olddeg, *nodes = sv->t_flag;
    GDE_HIP(hipMemcpyAsync(d_src, src.data(), 4 * (size_t)m, hipMemcpyHostToDevice, sv->s));
    GDE_HIP(hipMemcpyAsync(d_dst, dst.data(), 4 * (size_t)m, hipMemcpyHostToDevice, sv->s));
    GDE_HIP(hipMemsetAsync(add, 0, 4 * (size_t)n, sv->s));
    hipLaunchKernelGGL(k_srv_count_new, dim3((m + 255) / 256), dim3(256), 0, sv->s, d_src, m, add);
    hipLaunchKernelGGL(k_srv_scan_blocks, dim3(nb), dim3(256), 0, sv->s, sv->g->row_ptr, add, n, newrp, bsum);
    hipLaunchKernelGGL(k_srv_scan_sums, dim3(1), dim3(1024), 0, sv->s, bsum, nb);
    hipLaunchKernelGGL(k_srv_scan_add, dim3(nb), dim3(256), 0, sv->s, newrp, bsum, n);
    hipLaunchKernelGGL(k_srv_copy_rows, dim3(4096), dim3(256), 0, sv->s, sv->g->row_ptr, sv->g->col_idx, newrp, newci,
                       n, cursor);
    hipLaunchKernelGGL(k_srv_append, dim3((m + 255) / 256), dim3(256), 0, sv->s, d_src, d_dst, m, newci, cursor);
    GDE_HIP(hipGetLastError());
    // old degrees for the corrections (from the old row pointers)
    hipLaunchKernelGGL(k_srv_degrees, dim3(4096), dim3(256), 0, sv->s, sv->g->row_ptr, n, olddeg);
    // in-flight corrections (the X / R of idle lanes are zero, so they are untouched)
    BatchArgs<float> a{};
    srv_args(sv, &a);
    std::vector<int32_t> hnodes(src);
    std::sort(hnodes.begin(), hnodes.end());
    hnodes.erase(std::unique(hnodes.begin(), hnodes.end()), hnodes.end());
    GDE_HIP(hipMemcpyAsync(nodes, hnodes.data(), 4 * hnodes.size(), hipMemcpyHostToDevice, sv->s));
    bool any_busy = false;
    for (SGroup &gr : sv->groups)
        if (gr.busy) { gr.cand = true; any_busy = true; }
    if (any_busy) {
        int rc = srv_upload_group_params(sv);
        if (rc) return rc;
        const int64_t tot = (int64_t)m * sv->G * sv->L;
        hipLaunchKernelGGL(k_srv_correct_edges, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, sv->s, d_src, d_dst,
                           m, olddeg, sv->G, sv->L, sv->d_kind, sv->d_gparam, a.R, a.X);
        const int64_t tn = (int64_t)hnodes.size() * sv->G;
        const int cur = sv->t & 1;
        int32_t *tcnt = batch_ws_touch_count(sv->w);
        hipLaunchKernelGGL(k_srv_correct_nodes, dim3((unsigned)((tn + 255) / 256)), dim3(256), 0, sv->s, nodes,
                           (int32_t)hnodes.size(), add, olddeg, sv->G, sv->L, sv->d_kind, a.R, a.X, a.NM, a.TM, sv->d_gepoch,
                           a.act[cur], &a.st->acount[cur], a.act_cap, a.touched, tcnt, a.touch_cap);
        GDE_HIP(hipGetLastError());
    }
    GDE_HIP(hipStreamSynchronize(sv->s));
    // swap in the new CSR (the old one becomes the spare); degree-dependent state follows
    int32_t *old_rp = sv->g->row_ptr, *old_ci = sv->g->col_idx;
    const int64_t old_cap = sv->cur_ci_cap > 0 ? sv->cur_ci_cap : sv->g->nnz;
    sv->g->owned = false;  // keep the old arrays: they are reused for the next batch
    int rc = graph_replace_csr(sv->g, newrp, newci, new_nnz, src);
    if (rc) return rc;
    sv->cur_ci_cap = sv->spare_ci_cap;
    sv->spare_rp = old_rp;
    sv->spare_ci = old_ci;
    sv->spare_ci_cap = old_cap;
    if ((rc = plain_workspaces_refresh(sv->g, sv->ctx, sv->s))) return rc;
    for (HkWorker *wk : sv->hk_w)
        if ((rc = plain_workspaces_refresh(sv->g, wk->ctx, sv->s))) return rc;
    GDE_HIP(batch_init_deg<float>(sv->g->row_ptr, (float *)a.deg, n, sv->s));
    GDE_HIP(hipStreamSynchronize(sv->s));
    sv->inserted_edges += m / 2;
    return GDE_OK;
}

}  // namespace gde

using namespace gde;

extern "C" {

int gde_server_create(gde_ctx *ctx, const gde_graph *g, const gde_server_cfg *cfg, gde_server **out) {
    if (!ctx || !g || !cfg || !out) return fail(GDE_ERR_INVALID_ARG, "null argument");
    if (cfg->lanes_per_group != 8 && cfg->lanes_per_group != 16 && cfg->lanes_per_group != 32)
        return fail(GDE_ERR_INVALID_ARG, "lanes_per_group must be 8, 16 or 32");
    if (cfg->max_groups < 1 || cfg->max_groups > 4096) return fail(GDE_ERR_INVALID_ARG, "max_groups in [1, 4096]");
    if (cfg->iters_per_step < 1 || cfg->queue_capacity < 1 || cfg->result_capacity < 1)
        return fail(GDE_ERR_INVALID_ARG, "iters_per_step, queue_capacity and result_capacity must be >= 1");
    if (cfg->value_type != GDE_F32) return fail(GDE_ERR_UNSUPPORTED, "the server computes in FP32");
    GDE_HIP(hipSetDevice(ctx->device));
    gde_server *sv = new gde_server();
    sv->user_ctx = ctx;
    sv->cfg = *cfg;
    sv->L = cfg->lanes_per_group;
    sv->G = cfg->max_groups;
    sv->t0 = std::chrono::steady_clock::now();
    sv->groups.resize(sv->G);
    auto bail = [&](int rc) {
        gde_server_destroy(sv);
        return rc;
    };
    hipError_t e = hipStreamCreateWithFlags(&sv->s, hipStreamNonBlocking);
    if (e != hipSuccess) { delete sv; return hip_fail(e, "hipStreamCreate"); }
    sv->ctx = new gde_ctx();
    sv->ctx->device = ctx->device;
    // private copy of the graph (the server rebuilds it on insertions)
    int32_t *rp = nullptr, *ci = nullptr;
    e = hipMalloc((void **)&rp, 4 * ((size_t)g->n + 1));
    if (e == hipSuccess) e = hipMalloc((void **)&ci, 4 * (size_t)std::max<int64_t>(g->nnz, 1));
    if (e == hipSuccess) e = hipMemcpyAsync(rp, g->row_ptr, 4 * ((size_t)g->n + 1), hipMemcpyDeviceToDevice, sv->s);
    if (e == hipSuccess && g->nnz) e = hipMemcpyAsync(ci, g->col_idx, 4 * (size_t)g->nnz, hipMemcpyDeviceToDevice, sv->s);
    if (e == hipSuccess) e = hipStreamSynchronize(sv->s);
    if (e != hipSuccess) { if (rp) (void)hipFree(rp); if (ci) (void)hipFree(ci); return bail(hip_fail(e, "graph copy")); }
    sv->g = graph_wrap_device(sv->ctx, g->n, g->nnz, rp, ci);
    int rc = batch_ws_acquire(sv->ctx, sv->g, GDE_F32, sv->L, sv->G, sv->s, &sv->w);
    if (rc) return bail(rc);
    BatchArgs<float> a{};
    batch_args_from_ws(sv->w, sv->g, sv->G, &a);
    e = hipMalloc((void **)&sv->d_act_tmp, 8 * (size_t)a.act_cap);
    if (e == hipSuccess) e = hipMalloc((void **)&sv->d_touch_tmp, 8 * (size_t)a.touch_cap);
    if (e == hipSuccess) e = hipMalloc((void **)&sv->d_drop, 4 * (size_t)sv->G);
    if (e == hipSuccess) e = hipMalloc((void **)&sv->d_gactive, 4 * (size_t)sv->G);
    if (e == hipSuccess) e = hipMalloc((void **)&sv->d_kind, 4 * (size_t)sv->G);
    if (e == hipSuccess) e = hipMalloc((void **)&sv->d_mode, 4 * (size_t)sv->G);
    if (e == hipSuccess) e = hipMalloc((void **)&sv->d_cnt, 4);
    if (e == hipSuccess) e = hipMalloc((void **)&sv->d_gws, 4 * (size_t)sv->G);
    if (e == hipSuccess) e = hipMalloc((void **)&sv->d_gparam, 4 * (size_t)sv->G);
    if (e == hipSuccess) e = hipMalloc((void **)&sv->d_rscale, 4 * (size_t)sv->G);
    if (e == hipSuccess) e = hipMalloc((void **)&sv->d_gepoch, 4 * (size_t)sv->G);
    if (e == hipSuccess) e = hipMemset(sv->d_gepoch, 0, 4 * (size_t)sv->G);
    if (e == hipSuccess) e = hipMemsetAsync(a.st, 0, sizeof(BatchDev), sv->s);
    if (e != hipSuccess) return bail(hip_fail(e, "server buffers"));
    rc = srv_upload_group_params(sv);
    if (rc) return bail(rc);
    e = hipStreamSynchronize(sv->s);
    if (e != hipSuccess) return bail(hip_fail(e, "server init"));
    for (int i = 0; i < kHkWorkers; i++) {
        HkWorker *wk = new HkWorker();
        sv->hk_w.push_back(wk);
        wk->ctx = new gde_ctx();
        wk->ctx->device = ctx->device;
        e = hipStreamCreateWithFlags(&wk->s, hipStreamNonBlocking);
        if (e != hipSuccess) { wk->s = nullptr; return bail(hip_fail(e, "hipStreamCreate")); }
        const size_t cap = (size_t)std::max<int32_t>(cfg->result_capacity, 1);
        wk->idx.resize(cap);
        wk->val.resize(cap);
        wk->th = std::thread(hk_worker_main, sv, wk);
    }
    *out = sv;
    return GDE_OK;
}

int gde_server_submit(gde_server *sv, const gde_params *p, const gde_seed *s, uint64_t *ticket) {
    if (!sv || !p || !s || !ticket) return fail(GDE_ERR_INVALID_ARG, "null argument");
    int rc = gde_validate_query(sv->g, p, s);
    if (rc) return rc;
    if (p->method != GDE_LOCAL_GD) return fail(GDE_ERR_UNSUPPORTED, "the server runs LocalGD");
    if (p->flags & (GDE_DETERMINISTIC | GDE_SYM_NORM))
        return fail(GDE_ERR_UNSUPPORTED, "the deterministic mode and GDE_SYM_NORM are provided by gde_solve, not by "
                                         "the server");
    std::unique_lock<std::mutex> lk(sv->hk_mu);
    if (sv->n_pending + (int64_t)sv->hk_queue.size() >= sv->cfg.queue_capacity)
        return fail(GDE_ERR_BUSY, "server queue is full");
    const bool level = p->kind == GDE_HK || p->kind == GDE_SERIES;  // level-push workers
    if (!level) lk.unlock();
    SReq r;
    r.ticket = sv->next_ticket++;
    r.p = *p;
    if (p->kind == GDE_SERIES) {
        r.coef.assign(p->c, p->c + p->K + 1);
        r.p.c = nullptr;  // set to the copy when a worker takes the query
    }
    r.idx.assign(s->idx, s->idx + s->nnz);
    r.val.assign(s->val, s->val + s->nnz);
    r.t_sub = now_s(sv->t0);
    *ticket = r.ticket;
    if (level) {
        sv->hk_queue.push_back(std::move(r));
        lk.unlock();
        sv->hk_cv.notify_one();
        return GDE_OK;
    }
    sv->pending[{p->kind, p->kind == GDE_PPR ? p->alpha : p->beta}].push_back(std::move(r));
    sv->n_pending++;
    return GDE_OK;
}

int gde_server_poll(gde_server *sv, gde_completion *out, int32_t cap, int32_t *n_out) {
    if (!sv || !n_out || (cap > 0 && !out)) return fail(GDE_ERR_INVALID_ARG, "null argument");
    GDE_HIP(hipSetDevice(sv->ctx->device));
    // completions handed out by the previous poll are released now
    if (sv->done_read > 0) {
        sv->done.erase(sv->done.begin(), sv->done.begin() + sv->done_read);
        sv->done_idx.erase(sv->done_idx.begin(), sv->done_idx.begin() + sv->done_read);
        sv->done_val.erase(sv->done_val.begin(), sv->done_val.begin() + sv->done_read);
        sv->done_read = 0;
    }
    int rc = srv_apply_inserts(sv);
    if (rc) return rc;
    if ((rc = srv_admit(sv))) return rc;
    if ((rc = srv_step_launch(sv))) return rc;
    const bool stepped = sv->step_open;
    if ((rc = srv_step_finish(sv))) return rc;
    if ((rc = srv_hk_collect(sv, !stepped))) return fail(rc, "a heat-kernel solve failed on the device");
    const int32_t k = (int32_t)std::min<size_t>(sv->done.size(), (size_t)std::max(cap, 0));
    for (int32_t i = 0; i < k; i++) {
        out[i] = sv->done[i];
        out[i].idx = sv->done_idx[i].data();
        out[i].val = sv->done_val[i].data();
    }
    sv->done_read = (size_t)k;
    *n_out = k;
    return GDE_OK;
}

int gde_server_insert_edges(gde_server *sv, int32_t k, const int32_t *u, const int32_t *v) {
    if (!sv || k < 0 || (k > 0 && (!u || !v))) return fail(GDE_ERR_INVALID_ARG, "null argument");
    for (int32_t i = 0; i < k; i++)
        if (u[i] < 0 || u[i] >= sv->g->n || v[i] < 0 || v[i] >= sv->g->n)
            return fail(GDE_ERR_INVALID_ARG, "edge endpoint out of range");
    if (sv->cfg.max_insert_edges > 0 && sv->inserted_edges + (int64_t)sv->inserts.size() + k > sv->cfg.max_insert_edges)
        return fail(GDE_ERR_OOM, "max_insert_edges reached");
    for (int32_t i = 0; i < k; i++) sv->inserts.emplace_back(u[i], v[i]);
    return GDE_OK;
}

int gde_server_destroy(gde_server *sv) {
    if (!sv) return fail(GDE_ERR_INVALID_ARG, "null server");
    {
        std::lock_guard<std::mutex> lk(sv->hk_mu);
        sv->hk_stop = true;
    }
    sv->hk_cv.notify_all();
    for (HkWorker *wk : sv->hk_w) {
        if (wk->th.joinable()) wk->th.join();
        if (wk->s) (void)hipStreamDestroy(wk->s);
        if (wk->ctx) gde_ctx_destroy(wk->ctx);
        delete wk;
    }
    sv->hk_w.clear();
    if (sv->s) (void)hipStreamSynchronize(sv->s);
    void *p[] = {sv->d_drop, sv->d_gactive, sv->d_kind, sv->d_mode, sv->d_cnt, sv->d_gws, sv->d_gparam, sv->d_rscale, sv->d_gepoch,
                 sv->d_act_tmp, sv->d_touch_tmp, sv->d_seed_b, sv->d_seed_lane, sv->d_seed_node, sv->d_out_idx, sv->d_out_val,
                 sv->spare_rp, sv->spare_ci, sv->t_add, sv->t_olddeg, sv->t_cursor, sv->t_bsum, sv->t_src, sv->t_dst,
                 sv->t_flag};
    for (void *q : p)
        if (q) (void)hipFree(q);
    if (sv->ctx) gde_ctx_destroy(sv->ctx);
    if (sv->g) gde_graph_destroy(sv->g);
    if (sv->s) (void)hipStreamDestroy(sv->s);
    delete sv;
    return GDE_OK;
}

}  // extern "C"
