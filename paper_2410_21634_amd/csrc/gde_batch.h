// gde_batch.h -- host interface shared by the plain solver, the batched solver and the server.
#pragma once

#include "gde_internal.h"

namespace gde {
int get_workspace(gde_ctx *ctx, const gde_graph *g, int vtype, hipStream_t s, Workspace **out);
void drop_workspaces_of(const gde_graph *g, gde_ctx *ctx);
void drop_batch_workspaces_of(const gde_graph *g, gde_ctx *ctx);
// after g's CSR was replaced (same n): recompute the degrees the batch workspaces of ctx hold
int batch_workspaces_refresh(const gde_graph *g, gde_ctx *ctx, hipStream_t s);
// warm LocalGD re-solve of B standing queries (PPR or Katz, one kind and
// parameter) from their device state (per query: RD<V> array, x, pushed and
// touched bitmaps), as one batch; res[i]: iters, ops, pushes, norms, status
int batch_warm_resolve(gde_ctx *ctx, const gde_graph *g, int32_t B, const gde_params *p, void *const *rd,
                       void *const *x, uint32_t *const *pushed, uint32_t *const *tbm, gde_result *res,
                       hipStream_t s);
// push-kernel timing helpers (no-ops unless profiling is enabled on ctx)
int prof_mark(gde_ctx *ctx, hipStream_t s);
int prof_collect(gde_ctx *ctx, int64_t edges, int64_t entries);
int prof_mark_batch(gde_ctx *ctx, hipStream_t s);
int prof_mark_batch_push(gde_ctx *ctx, hipStream_t s);
int prof_collect_batch(gde_ctx *ctx, int64_t lane_edges, int64_t entries, int64_t rows, int64_t row_vol);
struct BatchWS;
void batch_ws_extract_buffers(BatchWS *w, int32_t **cnt, long long **lane_nnz, long long **lane_off);
void batch_ws_swap_list(BatchWS *w, int which, uint64_t **spare);
// host validation of one query against a graph (parameters, seed, isolated seeds)
int gde_validate_query(const gde_graph *g, const gde_params *p, const gde_seed *s);
}  // namespace gde
