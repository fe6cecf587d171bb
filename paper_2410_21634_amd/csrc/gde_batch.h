// gde_batch.h -- host interface shared by the plain solver, the batched solver and the server.
#pragma once

#include "gde_internal.h"

namespace gde {
int get_workspace(gde_ctx *ctx, const gde_graph *g, int vtype, hipStream_t s, Workspace **out);
void drop_workspaces_of(const gde_graph *g, gde_ctx *ctx);
// push-kernel timing helpers (no-ops unless profiling is enabled on ctx)
int prof_mark(gde_ctx *ctx, hipStream_t s);
int prof_collect(gde_ctx *ctx, int64_t edges, int64_t entries);
}  // namespace gde
