// gde_batch.h -- host interface shared by the plain solver, the batched solver and the server.
#pragma once

#include "gde_internal.h"

namespace gde {
int get_workspace(gde_ctx *ctx, const gde_graph *g, int vtype, hipStream_t s, Workspace **out);
void drop_workspaces_of(const gde_graph *g, gde_ctx *ctx);
}  // namespace gde
