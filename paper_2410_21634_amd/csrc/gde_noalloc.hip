// gde_noalloc.hip -- gde_solve_noalloc: the plain solver on fixed device memory.
//
// For callers that cannot allocate device memory during a call (serving loops
// that forbid it, code between captures, harnesses without an allocator).  The
// solver's workspace -- residual/degree planes, estimate, bitmaps, frontier
// and work lists, push tile table, LocalCH and heat-kernel extras, the device
// counters and the seed copy -- is carved from one file-scope device array of
// GDE_NOALLOC_SCRATCH_BYTES.  Its device address is looked up once per device with
// hipGetSymbolAddress (the array's name is a host-side stand-in in host code)
// and only that address is used afterwards.
//
// Every call clears the part of the array it uses and rebuilds the degree
// planes from the caller's CSR, so calls may alternate graphs and sizes.  All
// calls on one device share the array: calls that overlap in time on one GPU
// (two host threads, or two streams) race on it and give undefined results.
//
// The iterations are those of gde_solve (Eq. (9); Sec. 3.3; the level push of
// Sec. 2) with its small-frontier single-workgroup launches and the atomic
// scatter; the binned scatter, whose bins scale with nnz, is not used.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>

#include "gde_batch.h"
#include "gde_internal.h"
#include "gde_kernels.h"

namespace gde {

template <typename V>
int solve_plain_ws(gde_ctx *ctx, const gde_graph *g, const gde_params *p, const gde_seed *sd, gde_result *res,
                   Workspace *w, hipStream_t s);

// the fixed workspace: GDE_NOALLOC_SCRATCH_BYTES per device, for the life of the process
static __device__ __align__(256) unsigned char scratch[GDE_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
constexpr int32_t kNoallocSeedCap = 4096;  // seed entries the array holds
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// device address of this device's array (the device is current)
int scratch_address(int dev, unsigned char **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(GDE_ERR_INVALID_ARG, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(GDE_ERR_DEVICE, "hipGetSymbolAddress(scratch) gave a null address");
        g_ptr[dev] = ptr;
    }
    *out = (unsigned char *)g_ptr[dev];
    return GDE_OK;
}

// bump allocation of 256-byte aligned pieces; with base == nullptr it only sizes
struct Carve {
    unsigned char *base;
    size_t used = 0;
    template <typename T>
    void take(T **p, size_t bytes) {
        used = (used + 255) & ~(size_t)255;
        *p = base ? (T *)(base + used) : nullptr;
        used += bytes;
    }
};

// lays out every buffer the plain solve of (g, p, nseed) touches
void layout(Carve &c, Workspace *w, const gde_graph *g, const gde_params *p, int32_t nseed) {
    const int64_t n = g->n;
    const size_t vs = w->vsize;
    const int64_t nwords = (n + 31) / 32;
    w->nblk = (nwords + kBlock - 1) / kBlock;
    c.take(&w->st, sizeof(DevState));
    c.take(&w->rd, 2 * vs * n);
    c.take(&w->x, vs * n);
    c.take(&w->bitmap, 4 * nwords);
    c.take(&w->tbm, 4 * nwords);
    c.take(&w->blk, 4 * (w->nblk + 1));
    for (int i = 0; i < 2; i++) c.take(&w->front[i], 4 * n);
    c.take(&w->wl_node, 4 * n);
    c.take(&w->wl_beg, 4 * n);
    c.take(&w->wl_off, 4 * n);
    c.take(&w->wl_sv, vs * n);
    c.take(&w->tile_start, 4 * (size_t)(g->nnz / kPushTile + 2));
    if (p->kind == GDE_HK || p->kind == GDE_SERIES) {
        c.take(&w->rd2, 2 * vs * n);
        for (int i = 0; i < 3; i++) c.take(&w->touched[i], 4 * n);
        c.take(&w->lvl_tab, 16 * (size_t)(kHkMaxLevels + 1));
    }
    if (p->method == GDE_LOCAL_CH) {
        c.take(&w->delta, vs * n);
        c.take(&w->dstamp, 4 * n);
        c.take(&w->cstamp, 4 * n);
    }
    const bool sub_seed = p->kind == GDE_KATZ && (p->flags & GDE_KATZ_SUBTRACT_SEED);
    if (nseed > kSeedInline || sub_seed) {
        c.take(&w->seed_idx, 4 * (size_t)nseed);
        c.take(&w->seed_val, 8 * (size_t)nseed);
        w->seed_cap = nseed;
    } else {
        w->seed_cap = kSeedInline;  // the seed travels in the kernel arguments
    }
}

__global__ void k_zero_words(uint4 *p, size_t n16) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

}  // namespace

}  // namespace gde

using namespace gde;

extern "C" size_t gde_solve_noalloc_bytes(const gde_graph *g, const gde_params *p, const gde_seed *s) {
    if (!g || !p || !s) return 0;
    Workspace w;
    w.n = g->n;
    w.vsize = p->value_type == GDE_F64 ? 8 : 4;
    Carve c{nullptr};
    layout(c, &w, g, p, s->nnz);
    return (c.used + 255) & ~(size_t)255;
}

extern "C" int gde_solve_noalloc(const gde_graph *g, const gde_params *p, const gde_seed *s, gde_result *res,
                                 hipStream_t stream) {
    if (!g || !p || !s || !res) return fail(GDE_ERR_INVALID_ARG, "null graph, params, seed or result");
    int rc = gde_validate_query(g, p, s);
    if (rc) { res->status = rc; return rc; }
    if (res->capacity < 0) return fail(GDE_ERR_INVALID_ARG, "negative capacity");
    if (!(p->flags & GDE_RESULT_DEVICE))
        return fail(GDE_ERR_INVALID_ARG, "gde_solve_noalloc writes device results only (set GDE_RESULT_DEVICE)");
    if (p->method == GDE_LOCAL_SOR) return fail(GDE_ERR_UNSUPPORTED, "gde_solve_noalloc runs LocalGD and LocalCH");
    if (p->flags & (GDE_TRACE | GDE_DETERMINISTIC | GDE_SCATTER_BINNED | GDE_SYM_NORM))
        return fail(GDE_ERR_UNSUPPORTED,
                    "gde_solve_noalloc provides no trace, deterministic mode, binned scatter or GDE_SYM_NORM");
    if (s->nnz > kNoallocSeedCap) return fail(GDE_ERR_INVALID_ARG, "gde_solve_noalloc takes at most 4096 seed entries");
    const size_t need = gde_solve_noalloc_bytes(g, p, s);
    if (need > (size_t)GDE_NOALLOC_SCRATCH_BYTES)
        return fail(GDE_ERR_OOM, "gde_solve_noalloc: this graph needs " + std::to_string(need) +
                                     " bytes of workspace; the fixed array holds " +
                                     std::to_string((size_t)GDE_NOALLOC_SCRATCH_BYTES));
    GDE_HIP(hipSetDevice(g->device));
    unsigned char *base = nullptr;
    if ((rc = scratch_address(g->device, &base))) return rc;

    Workspace w;
    w.g = g;
    w.guid = g->uid;
    w.vtype = p->value_type;
    w.n = g->n;
    w.vsize = p->value_type == GDE_F64 ? 8 : 4;
    Carve c{base};
    layout(c, &w, g, p, s->nnz);
    w.nnz_cap = g->nnz;
    w.bin_nranges = 0;     // atomic scatter only
    DevState host_state{};  // device counters are read back with a copy (no pinned mirror)
    w.hst = &host_state;
    w.hst_dev = nullptr;

    // rest state: everything zero, then the degrees of the residual planes
    const size_t n16 = (c.used + 15) / 16;
    const unsigned grid = (unsigned)std::min<size_t>((n16 + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zero_words, dim3(std::max(grid, 1u)), dim3(256), 0, stream, (uint4 *)base, n16);
    if (w.vtype == GDE_F64) {
        launch_init_rd<double>(g->row_ptr, w.rd, g->n, stream);
        if (w.rd2) launch_init_rd<double>(g->row_ptr, w.rd2, g->n, stream);
    } else {
        launch_init_rd<float>(g->row_ptr, w.rd, g->n, stream);
        if (w.rd2) launch_init_rd<float>(g->row_ptr, w.rd2, g->n, stream);
    }
    GDE_HIP(hipGetLastError());
    gde_params q = *p;
    q.flags |= GDE_SCATTER_ATOMIC;
    if (w.vtype == GDE_F64) return solve_plain_ws<double>(nullptr, g, &q, s, res, &w, stream);
    return solve_plain_ws<float>(nullptr, g, &q, s, res, &w, stream);
}
