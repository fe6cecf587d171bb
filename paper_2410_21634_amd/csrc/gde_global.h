// gde_global.h -- the global GD / Chebyshev solvers (gde_global.hip).
#pragma once

#include "gde_internal.h"

namespace gde {

// One query with S_t = V in every iteration (GD or CH by p->method); results
// as gde_solve (sorted sparse x, residual norms, T, ops = T nnz).
int solve_global(gde_ctx *ctx, const gde_graph *g, const gde_params *p, const gde_seed *sd, gde_result *res,
                 hipStream_t s);

void glob_ws_free(GlobWS *w);

// LocalSOR / APPR (the FIFO push, gde_fifo.hip): B queries, one wavefront each;
// every p[i] has method GDE_LOCAL_SOR and the same value type.
int solve_fifo(gde_ctx *ctx, const gde_graph *g, int32_t B, const gde_params *p, const gde_seed *sd, gde_result *res,
               hipStream_t s);

// Sparse form of a dense device vector (ascending ids of its nonzeros):
// per-block counts into blk[dense_nblk(n) + 1], an exclusive scan with the total,
// then the emission of (id, value) pairs at the scanned offsets.
int64_t dense_nblk(int64_t n);
template <typename V> void launch_dense_count(const V *x, int64_t n, int32_t *blk, hipStream_t s);
void launch_dense_scan(int32_t *blk, int64_t nblk, long long *total, hipStream_t s);
template <typename V>
void launch_dense_emit(const V *x, int64_t n, const int32_t *blk, int32_t *idx, V *val, hipStream_t s);

}  // namespace gde
