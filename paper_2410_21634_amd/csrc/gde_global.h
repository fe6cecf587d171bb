// gde_global.h -- the global GD / Chebyshev solvers (gde_global.hip).
#pragma once

#include "gde_internal.h"

namespace gde {

// One query with S_t = V in every iteration (GD or CH by p->method); results
// as gde_solve (sorted sparse x, residual norms, T, ops = T nnz).
int solve_global(gde_ctx *ctx, const gde_graph *g, const gde_params *p, const gde_seed *sd, gde_result *res,
                 hipStream_t s);

void glob_ws_free(GlobWS *w);

}  // namespace gde
