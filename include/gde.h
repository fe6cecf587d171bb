/*
 * gde.h -- C ABI of the MI355X (gfx950) local graph-diffusion solver library.
 *
 * The library computes approximate graph diffusion vectors
 *     f = sum_k c_k M^k s                       (Eq. (1), Table 1)
 * for Personalized PageRank, Katz and the heat kernel with the local diffusion
 * process of Definition 3.1: starting from x = 0, r = b, S_0 = supp(s), each
 * iteration updates the estimate x and the residual r = b - Q x on the active
 * set S_t = {u : |r_u| >= theta_u} only, until S_t is empty.
 *
 *   PPR  : Q = I - (1-alpha) A D^-1, b = alpha s   (Eq. (2)); theta_u = alpha*eps*d_u
 *   Katz : Q = I - beta A,           b = s         (Eq. (3)); theta_u = eps*d_u
 *   HK   : Taylor truncation f_K = sum_{k<=K} e^-tau tau^k/k! (A D^-1)^k s, solved
 *          level by level on the Kronecker system of the AHK push (Sec. 2);
 *          level-k threshold eps*d_u/((K+1) psi_k), psi_k = sum_{j=k..K} tau^(j-k) k!/j!.
 *   SERIES : any truncated series f_K = sum_{k<=K} c_k (A D^-1)^k s with given
 *          c_k > 0 (Eq. (1), Table 1), by the same level push with ratio
 *          c_{k+1}/c_k and psi_k = sum_{j=k..K} c_j/c_k.
 *
 * Methods: LocalGD (Eq. (9): x += r_S, r -= Q r_S) and LocalCH (Sec. 3.3,
 * Chebyshev update restricted to S_t).  The heat kernel and SERIES always use
 * the level push.
 *
 * Conventions shared by every entry point
 *   - All sizes and indices are int32 node ids / int64 counts; the graph is a
 *     simple undirected graph stored as a symmetric CSR (row_ptr[n+1],
 *     col_idx[nnz], nnz = 2|E| < 2^31, no self-loops).
 *   - Every call returns a gde_status.  No exception crosses the ABI.  All
 *     argument validation runs on the host before any device work, so a
 *     rejected call leaves the device untouched.  gde_last_error() gives a
 *     thread-local text for the last non-OK status.
 *   - Device work is enqueued on the hipStream_t passed in (NULL = the
 *     default stream).  gde_solve and gde_solve_batch return with their
 *     outputs final (they synchronise that stream).
 *   - A gde_ctx is used by one host thread at a time.  A gde_graph is
 *     immutable and may be shared by contexts on the same device.
 *   - Inputs are borrowed for the duration of the call; results are written
 *     only into caller-owned buffers.  Every *_create has a matching *_destroy.
 */
#ifndef GDE_H
#define GDE_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GDE_ABI_VERSION 2

typedef enum gde_status {
    GDE_OK = 0,
    GDE_ERR_INVALID_ARG = 1,   /* null pointer, malformed CSR, parameter out of range (see gde_params) */
    GDE_ERR_ISOLATED_SEED = 2, /* some u in supp(s) has d_u = 0: D^-1 is undefined there */
    GDE_ERR_CAPACITY = 3,      /* result buffer too small: result.nnz holds the size needed, nothing written */
    GDE_ERR_NOT_CONVERGED = 4, /* max_iters reached; the result is valid and its residual is reported */
    GDE_ERR_OOM = 5,           /* device or host allocation failed */
    GDE_ERR_BUSY = 6,          /* server admission refused and its queue is full */
    GDE_ERR_DEVICE = 7,        /* a HIP call failed; gde_last_error() has the HIP message */
    GDE_ERR_UNSUPPORTED = 8    /* valid but not provided (LocalCH for the heat kernel) */
} gde_status;

typedef enum gde_kind { GDE_PPR = 0, GDE_KATZ = 1, GDE_HK = 2, GDE_SERIES = 3 } gde_kind;
typedef enum gde_method { GDE_LOCAL_GD = 0, GDE_LOCAL_CH = 1, GDE_LOCAL_SOR = 2 } gde_method;
typedef enum gde_value_type { GDE_F32 = 0, GDE_F64 = 1 } gde_value_type;

/* gde_graph_create flags */
#define GDE_HOST_PTRS 0x1u   /* row_ptr / col_idx are host pointers (always copied) */
#define GDE_DEVICE_PTRS 0x2u /* row_ptr / col_idx are device pointers on the context's device */
#define GDE_COPY 0x4u        /* the library keeps its own device copy */
#define GDE_BORROW 0x8u      /* device pointers are used in place; they must outlive the graph */

/* gde_params.flags */
#define GDE_KATZ_SUBTRACT_SEED 0x1u /* Katz: return x - s, the centrality ((I - beta A)^-1 - I) s */
#define GDE_TRACE 0x2u              /* record |S_t|, vol(S_t) and the S_t lists into the result */
#define GDE_RESULT_DEVICE 0x4u      /* result idx / val are device pointers (else host) */
/* Scatter strategy of the plain solver (gde_solve).  By default small frontiers
 * run in one workgroup (several iterations per launch); larger ones run on the
 * whole device, where an iteration whose frontier volume reaches a fixed
 * threshold writes its updates into destination-range bins that are summed in
 * on-chip memory, and smaller ones use one atomic add per edge.  All compute the
 * same iteration (Eq. (9)); only the order of floating-point additions differs.
 * Setting both is INVALID_ARG. */
#define GDE_SCATTER_BINNED 0x8u     /* bin every iteration's scatter (no single-workgroup launches) */
#define GDE_SCATTER_ATOMIC 0x10u    /* never bin: one atomic add per edge */
/* Deterministic mode (for checking and A/B bisection, not speed).  The same
 * iterations (Eq. (9); Sec. 3.3; the level push of Sec. 2) with every
 * floating-point operation in a fixed order: at each node the updates of an
 * iteration are added one after another in ascending order of the pushed node
 * they come from, the node's own change at its place in that order -- a
 * sequential reading of the iteration with S_t taken in ascending ids.  No
 * floating-point atomics; residual norms are reduced in a fixed tree.  Two runs
 * give bit-identical x, residual norms and traces; in FP64, x equals a
 * sequential implementation of those steps bit for bit.  It overrides the
 * scatter flags.  gde_solve_batch honours it by solving each query in this mode;
 * the server rejects it (GDE_ERR_UNSUPPORTED). */
#define GDE_DETERMINISTIC 0x20u
/* PPR, HK and GDE_SERIES: propagation matrix M = D^-1/2 A D^-1/2 (APPNP in
 * Table 1) in place of A D^-1.  Since (D^-1/2 A D^-1/2)^k = D^-1/2 (A D^-1)^k
 * D^1/2, the call solves the A D^-1 form from the source D^1/2 s and returns
 * x_u / sqrt(d_u) (the symmetrisation of Sec. 3.3).  The stop rule, T, the
 * operation counts and the residual norms are those of the A D^-1 form with
 * source D^1/2 s, so |f_u - x_u| <= eps sqrt(d_u) (PPR LocalGD).  gde_solve and
 * gde_solve_batch; Katz gives GDE_ERR_INVALID_ARG, LocalSOR, the deterministic
 * mode, gde_solve_global, gde_solve_noalloc, the server and standing queries
 * give GDE_ERR_UNSUPPORTED. */
#define GDE_SYM_NORM 0x40u

typedef struct gde_ctx gde_ctx;
typedef struct gde_graph gde_graph;
typedef struct gde_server gde_server;

/*
 * One diffusion query.
 *   kind, method     : gde_kind, gde_method (LocalCH or LocalSOR with HK or SERIES ->
 *                      GDE_ERR_UNSUPPORTED).  GDE_LOCAL_SOR is the sequential push of
 *                      Eq. (7) / Algorithm 1 (APPR and AKatz at omega = 1): a FIFO queue
 *                      starting with supp(s) in index order; pop u, v = r_u,
 *                      x_u += omega v, r_u -= omega v, r_w += omega w_u v on N(u), and
 *                      every active node that is not queued joins the tail (the
 *                      neighbours in CSR order, then u).  Each query runs in one
 *                      wavefront; gde_solve_batch runs many at once.  Its "iterations"
 *                      are the queue generations (the t of Eq. (7)), pushes the pops.
 *   value_type       : GDE_F32 or GDE_F64 -- the type of x and r on the device
 *   alpha            : PPR damping, 0 < alpha < 1
 *   beta             : Katz weight, beta > 0 and beta * lambda_bound < 1
 *   tau, K           : heat-kernel temperature (tau >= 0) and truncation (0 <= K <= 256);
 *                      K is also the truncation of GDE_SERIES
 *   eps              : tolerance, finite and > 0 (stop iff max_u |r~_u|/d_u < eps)
 *   lambda_bound     : an upper bound of the spectral radius of A (Katz).  It is
 *                      required for Katz (validation of beta) and is the
 *                      Chebyshev bound of Katz-LocalCH: mu = 1 - beta*lambda,
 *                      L = 1 + beta*lambda.  gde_graph_lambda_max provides one.
 *   c                : GDE_SERIES only (NULL for every other kind): K + 1 coefficients
 *                      c_0 .. c_K in host memory, each finite and > 0; the call
 *                      solves f_K = sum_k c_k (A D^-1)^k s (Eq. (1), Table 1) by the
 *                      heat kernel's level push with level ratio c_{k+1}/c_k and
 *                      level thresholds eps d_u / ((K+1) psi_k), psi_k = sum_{j>=k}
 *                      c_j / c_k.  The heat kernel is c_k = e^-tau tau^k / k!;
 *                      alpha (1-alpha)^k is the truncated PPR series.  LocalGD only.
 *   max_iters        : iteration cap (>= 1); reaching it gives GDE_ERR_NOT_CONVERGED
 *   flags            : GDE_KATZ_SUBTRACT_SEED | GDE_TRACE | GDE_RESULT_DEVICE |
 *                      GDE_SCATTER_BINNED | GDE_SCATTER_ATOMIC | GDE_DETERMINISTIC
 */
typedef struct gde_params {
    int32_t kind;
    int32_t method;
    int32_t value_type;
    int32_t K;
    double alpha;
    double beta;
    double tau;
    double eps;
    double lambda_bound;
    const double *c;
    int32_t max_iters;
    uint32_t flags;
    double omega;  /* GDE_LOCAL_SOR: relaxation, 0 < omega < 2; 0 means 1 (APPR / AKatz) */
} gde_params;

/* Sparse source vector s in host memory: idx strictly increasing node ids,
 * val finite and > 0 (Theorem 3.4 assumes s >= 0). */
typedef struct gde_seed {
    int32_t nnz;
    const int32_t *idx;
    const double *val;
} gde_seed;

/*
 * Caller-allocated result.
 * In : capacity          -- entries available in idx / val
 *      idx               -- int32[capacity], node ids of supp(x), written ascending
 *      val               -- float[] or double[] (per value_type) x values
 *                           (host pointers unless GDE_RESULT_DEVICE)
 *      trace_capacity    -- entries of trace_size / trace_vol (host int64), may be 0
 *      trace_nodes_capacity, trace_nodes -- host int32 buffer for the concatenated
 *                           S_t lists (GDE_TRACE), may be 0 / NULL
 * Out: nnz               -- |supp(x)| (on GDE_ERR_CAPACITY: the capacity needed)
 *      residual_l1       -- ||r~||_1 in the reported scale (PPR: r/alpha; HK:
 *                           sum_k psi_k ||leftover_k||_1, which equals ||f_K - x||_1)
 *      residual_dinf     -- ||D^-1 r~||_inf (HK: max_k (K+1) psi_k ||D^-1 leftover_k||_inf);
 *                           below eps when the process has converged
 *      iters             -- T, the number of iterations with a nonempty S_t
 *      ops               -- sum_t vol(S_t), the paper's operation count (Definition 3.1)
 *      pushes            -- sum_t |S_t|
 *      status            -- the gde_status of the call
 *      trace_len         -- T (entries written: min(T, trace_capacity))
 *      trace_nodes_len   -- sum_t |S_t| (entries written: min(that, capacity))
 */
typedef struct gde_result {
    int64_t capacity;
    int32_t *idx;
    void *val;
    int64_t trace_capacity;
    int64_t *trace_size;
    int64_t *trace_vol;
    int64_t trace_nodes_capacity;
    int32_t *trace_nodes;
    int64_t nnz;
    double residual_l1;
    double residual_dinf;
    int32_t iters;
    int32_t status;
    int64_t ops;
    int64_t pushes;
    int64_t trace_len;
    int64_t trace_nodes_len;
} gde_result;

/* ABI version (GDE_ABI_VERSION). */
int gde_abi_version(void);

/* Thread-local text describing the last non-OK status returned on this thread. */
const char *gde_last_error(void);

/* Context bound to HIP device `hip_device`; owns the solver workspaces. */
int gde_ctx_create(int hip_device, gde_ctx **out);
int gde_ctx_destroy(gde_ctx *ctx);

/*
 * Upload (or borrow) a CSR graph.  Host pointers are validated on the host
 * (monotone row_ptr starting at 0 and ending at nnz, col_idx in range, no
 * self-loops); device pointers are validated by a device check before use.
 * With GDE_DEVICE_PTRS | GDE_BORROW the arrays are used in place.
 */
int gde_graph_create(gde_ctx *ctx, int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                     uint32_t flags, hipStream_t stream, gde_graph **out);
int gde_graph_destroy(gde_graph *g);

/*
 * The graph's node and entry counts, and a synchronous copy of its CSR into
 * caller-owned host arrays (row_ptr: n + 1 entries, col_idx: nnz entries;
 * either may be NULL to skip it).  The current version of a dynamic graph
 * (gde_dyn_graph) has ascending rows.  Errors: GDE_ERR_INVALID_ARG for a null
 * graph, GDE_ERR_DEVICE if the copy fails.
 */
int gde_graph_info(const gde_graph *g, int32_t *n, int64_t *nnz);
int gde_graph_download(const gde_graph *g, int32_t *row_ptr, int32_t *col_idx);

/*
 * Bounds of lambda_max(A) by power iteration on A + I from the all-ones vector
 * (a global O(nnz) pass per iteration; graph preparation, not part of a solve):
 * lower = Rayleigh quotient v'Av / v'v, upper = max_u (Av)_u / v_u
 * (Collatz-Wielandt; a certified bound for nonnegative A and v > 0).  Stops
 * when (upper - lower) <= rtol * upper or after max_iters iterations.
 */
int gde_graph_lambda_max(gde_ctx *ctx, gde_graph *g, int max_iters, double rtol, double *lower, double *upper,
                         hipStream_t stream);

/*
 * Kernel timing for measurement.  While enabled, every launch of the push
 * (residual scatter) kernel of the plain solver and every launch of the
 * batched solver's kernel in this context is bracketed by HIP events on the
 * solve's stream; the totals accumulate until read.  `out` may be NULL.
 *   launches, total_ms  -- push launches and their summed event time
 *   edges, entries      -- CSR entries they traversed (sum vol(S_t)) and sum |S_t|
 *   batch_launches, batch_ms -- batched-solver kernel launches and their time
 *   batch_lane_edges    -- (edge, query) updates the batched kernel applied
 *   batch_entries       -- (group, node) work entries it processed
 *   batch_push_launches, batch_push_ms -- the batched push (scatter) launches
 *                          alone, each bracketed by its own event pair
 *   batch_rows, batch_row_vol -- distinct CSR rows the batched rounds read (a
 *                          row pushed by several queries in one round counts
 *                          once) and their summed degree
 * reset != 0 clears the totals after reading.
 */
typedef struct gde_kernel_profile {
    int64_t launches;
    double total_ms;
    int64_t edges;
    int64_t entries;
    int64_t batch_launches;
    double batch_ms;
    int64_t batch_lane_edges;
    int64_t batch_entries;
    int64_t batch_push_launches;
    double batch_push_ms;
    int64_t batch_rows;
    int64_t batch_row_vol;
} gde_kernel_profile;
int gde_ctx_profile(gde_ctx *ctx, int enable, gde_kernel_profile *out, int reset);

/* Host-only validation of one query against a host CSR (no device work; usable without a GPU). */
int gde_validate(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx, const gde_params *p,
                 const gde_seed *s);

/* One query (Definition 3.1 with the method of p).  See gde_result. */
int gde_solve(gde_ctx *ctx, const gde_graph *g, const gde_params *p, const gde_seed *s, gde_result *res,
              hipStream_t stream);

/*
 * The standard (global) counterparts of LocalGD and LocalCH that Table 2 and
 * the eps sweep of Sec. 5 compare the local solvers against: the same update
 * with S_t = V, every node, in every iteration -- GD (h = r) or Chebyshev
 * (p->method = GDE_LOCAL_CH: the Sec. 3.3 recurrence over all nodes) -- until
 * no node has |r_u| >= theta_u (the first iteration always runs).  Each
 * iteration is one pass over the whole CSR (a sparse matrix-vector product), so
 * res.ops = T * nnz and res.pushes = T * n.  PPR and Katz only (the heat
 * kernel gives GDE_ERR_UNSUPPORTED).  Arguments, result layout, flags
 * (GDE_RESULT_DEVICE, GDE_TRACE: |S_t| = n, vol(S_t) = nnz) and errors as
 * gde_solve; every sum runs in a fixed order, so results are bit-identical
 * from run to run (GDE_DETERMINISTIC changes nothing here).
 */
int gde_solve_global(gde_ctx *ctx, const gde_graph *g, const gde_params *p, const gde_seed *s, gde_result *res,
                     hipStream_t stream);

/*
 * gde_solve without any allocation, for callers that cannot allocate device
 * or pinned host memory during a call (serving loops or harnesses that forbid
 * it, code run between stream captures).  It runs the iterations of gde_solve
 * (small frontiers in one workgroup, larger ones with one atomic add per edge;
 * never the binned scatter) on a workspace carved from one fixed device array
 * of GDE_NOALLOC_SCRATCH_BYTES that the library holds on every device it runs
 * on until the process ends; no hipMalloc, hipFree or allocating library call
 * is made.  The device counters are read back with stream synchronisations.
 *   g      : a graph from gde_graph_create (its CSR is read; its host degree
 *            copy validates the seed)
 *   p      : as gde_solve, with GDE_RESULT_DEVICE required (res idx / val are
 *            device pointers); GDE_TRACE, GDE_DETERMINISTIC and
 *            GDE_SCATTER_BINNED give GDE_ERR_UNSUPPORTED
 *   s      : host seed, at most 4096 entries (else GDE_ERR_INVALID_ARG)
 *   res    : as gde_solve
 * A graph and query whose workspace (gde_solve_noalloc_bytes) exceeds the
 * array give GDE_ERR_OOM before any device work: at 64 MiB that is about
 * 1.2 M nodes for FP32 PPR/Katz LocalGD, 0.5 M nodes for FP64 heat kernel.
 * Each call clears the part of the array it uses and rebuilds the degree
 * planes from g (O(n) device work), so calls may alternate graphs.  All calls
 * on one device share the array: calls that overlap in time on one GPU (from
 * two threads or on two streams) race and give undefined results.
 */
#define GDE_NOALLOC_SCRATCH_BYTES (64ull * 1024ull * 1024ull)
int gde_solve_noalloc(const gde_graph *g, const gde_params *p, const gde_seed *s, gde_result *res,
                      hipStream_t stream);
/* Bytes of the fixed array gde_solve_noalloc would use for (g, p, s); 0 on a null argument. */
size_t gde_solve_noalloc_bytes(const gde_graph *g, const gde_params *p, const gde_seed *s);

/*
 * B independent queries on one graph solved together, every iteration of all
 * of them in the same launches: seeds are packed into lanes of node-major
 * residual tiles, so a CSR row that several queries push in the same round is
 * read once.  Queries may differ in eps; they must share kind, method
 * (LocalGD or LocalCH), value type and kind parameters (alpha, beta, and
 * lambda_bound for Katz LocalCH; tau and K; the series coefficients).  PPR and
 * Katz run the LocalGD (Eq. (9)) or LocalCH (Sec. 3.3) iterations, every lane
 * with its own residuals and, for LocalCH, its own momentum term; the heat
 * kernel and GDE_SERIES run the level push, level t of every lane in
 * iteration t.  A batch of GDE_LOCAL_SOR queries runs one query per wavefront
 * (the sequential push of Eq. (7)); any other mix is solved query by query.
 * schedule_json: NULL = the default schedule (16 lanes, full occupancy), else
 * a JSON object {"lanes":L,"blocks_per_cu":G,"sort":0|1,"auto":0|1}.  With
 * "auto":1 the first batch of a (graph, kind, value type, power-of-two size
 * class) is solved twice per candidate schedule (8, 32 and 16 lanes, 16 lanes
 * at two blocks per CU) and timed; the candidate of the fastest run is kept in
 * the context for later calls, and the results of the last run (a complete
 * solve) are returned.
 * Every iteration is one snapshot and one push launch; "persistent":1 (a
 * single launch for all iterations) is not provided and gives
 * GDE_ERR_UNSUPPORTED.
 * res[i].status holds each query's own status; the call returns the first
 * non-OK status, or GDE_OK.
 */
int gde_solve_batch(gde_ctx *ctx, const gde_graph *g, int32_t B, const gde_params *p, const gde_seed *s,
                    gde_result *res, const char *schedule_json, hipStream_t stream);

/* The schedule the "auto" mode of gde_solve_batch chose in ctx for batches of
 * B queries of this kind and value type on g: *lanes and *blocks_per_cu (0 =
 * the occupancy limit).  GDE_ERR_INVALID_ARG when none was chosen yet or an
 * argument is null.  Host only. */
int gde_batch_tuned(const gde_ctx *ctx, const gde_graph *g, int32_t kind, int32_t value_type, int32_t B,
                    int32_t *lanes, int32_t *blocks_per_cu);

/* ------------------------------------------------ standing queries on a dynamic graph */
/*
 * Dynamic GDEs (Sec. 4): a private copy of a graph that changes by batches of
 * edge insertions and deletions, and standing PPR / Katz LocalGD queries whose
 * estimate x and residual r stay on the device between batches.  Each batch is
 * applied to every query as the Insert / Delete corrections of
 * LocalGS(Dynamic) and LocalSOR(Dynamic) (Algorithms 2-5) in the generic form
 * r = b - Q x -- each undirected edge {a, c} as the directed events a -> c and
 * c -> a, each source taking its inserts and then its deletes, targets
 * ascending within each; for PPR an event at a of current degree d
 * moves D = x_a / d (insert: x_a += D, r_a -= D, r_c += (1-alpha) D; delete:
 * the opposite signs; the first edge of a degree-0 node only adds (1-alpha) x_a
 * to r_c); for Katz r_c +/-= beta x_a -- followed by a warm LocalGD re-solve
 * from the corrected state: S_0 = {u : |r_u| >= theta_u, r_u != 0}, residuals
 * may be negative.  The queries of one kind and parameter are re-solved
 * together as the lanes of one batch (the scatter path: additions are atomic,
 * so FP summation order varies between runs).  The first solve of a query
 * starts from x = 0, r = b with S_0 = supp(s) forced (Definition 3.1), in the
 * fixed-order iterations of GDE_DETERMINISTIC.  The graph stays on the device:
 * a batch's events are sorted and checked there and the next version is
 * merged from the current one.
 *
 * gde_dyn_create : copies g0 (device CSR, rows sorted ascending) as version 0;
 *                  value_type GDE_F32 or GDE_F64 for every query of this object.
 * gde_dyn_graph  : the current version, usable with gde_solve / gde_solve_global
 *                  (e.g. to compare with a solve from scratch); valid until the
 *                  next gde_dyn_update or gde_dyn_destroy.
 * gde_dyn_add    : a new standing query (PPR or Katz, LocalGD, p->value_type as
 *                  the object's; GDE_KATZ_SUBTRACT_SEED unsupported), solved at
 *                  once on the current version; *qid receives its id.
 * gde_dyn_update : k_ins edges (iu[i], iv[i]) to insert -- each new, no
 *                  self-loops -- and k_del existing edges (du[i], dv[i]) to
 *                  delete; no edge twice in one batch.  All events are validated
 *                  before anything changes (GDE_ERR_INVALID_ARG).  Then every
 *                  query is corrected and re-solved.  Host arrays, borrowed.
 * gde_dyn_read   : query qid's current x (sorted sparse, nonzero entries) into
 *                  res (device buffers if flags has GDE_RESULT_DEVICE, else host),
 *                  with iters / ops / pushes / residual norms of its last
 *                  (re)solve.  GDE_ERR_CAPACITY as gde_solve.
 * A gde_dyn is used by one host thread at a time; its work runs on its own
 * stream and every call returns with it finished.
 */
typedef struct gde_dyn gde_dyn;
int gde_dyn_create(gde_ctx *ctx, const gde_graph *g0, int32_t value_type, gde_dyn **out);
const gde_graph *gde_dyn_graph(const gde_dyn *dy);
int gde_dyn_add(gde_dyn *dy, const gde_params *p, const gde_seed *s, int32_t *qid);
int gde_dyn_update(gde_dyn *dy, int32_t k_ins, const int32_t *iu, const int32_t *iv, int32_t k_del,
                   const int32_t *du, const int32_t *dv);
int gde_dyn_read(gde_dyn *dy, int32_t qid, gde_result *res, uint32_t flags);
int gde_dyn_destroy(gde_dyn *dy);

/* ---------------------------------------------------------------- serving */
typedef struct gde_server_cfg {
    int32_t lanes_per_group;   /* queries per node-major residual tile (8, 16 or 32) */
    int32_t max_groups;        /* tiles per kind resident at once (memory admission) */
    int32_t iters_per_step;    /* local iterations per engine step */
    int32_t queue_capacity;    /* pending queries beyond which submit returns GDE_ERR_BUSY */
    int32_t value_type;        /* GDE_F32 */
    int32_t result_capacity;   /* max |supp(x)| kept per completed query */
    int64_t max_insert_edges;  /* capacity of the dynamic edge store */
} gde_server_cfg;

typedef struct gde_completion {
    uint64_t ticket;
    int32_t status;
    int32_t iters;
    int64_t nnz;         /* entries in idx / val (host memory owned by the server until the next poll) */
    const int32_t *idx;
    const float *val;
    double residual_l1;
    double residual_dinf;
    double submit_time_s; /* server clock at submit */
    double done_time_s;   /* server clock when the completion was harvested */
} gde_completion;

/* A continuous-batching server on a private dynamic copy of the graph.
 * PPR and Katz queries (LocalGD) advance in node-major lane groups on the
 * server's stream; heat-kernel queries are solved one each by the plain
 * level-push solver on three worker threads, each with its own context and
 * stream, and always on one graph version (a rebuild waits for running
 * solves).  The handle is used by one thread at a time. */
int gde_server_create(gde_ctx *ctx, const gde_graph *g, const gde_server_cfg *cfg, gde_server **out);
/* Enqueue a query (non-blocking); *ticket identifies its completion. */
int gde_server_submit(gde_server *sv, const gde_params *p, const gde_seed *s, uint64_t *ticket);
/* Apply queued insertions, admit, run one engine step and return up to cap
 * completions.  With no group in flight and heat-kernel queries running it
 * waits up to 2 ms for one of them; with nothing in flight it returns at once. */
int gde_server_poll(gde_server *sv, gde_completion *out, int32_t cap, int32_t *n_out);
/* Insert k undirected edges (u[i], v[i]); applied between engine steps, with the
 * warm-start corrections of the dynamic GDE (Sec. 4) to every in-flight query. */
int gde_server_insert_edges(gde_server *sv, int32_t k, const int32_t *u, const int32_t *v);
int gde_server_destroy(gde_server *sv);

#ifdef __cplusplus
}
#endif
#endif /* GDE_H */
