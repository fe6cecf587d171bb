// gde_det.h -- the deterministic mode of the plain solver (gde_det.hip).
#pragma once

#include "gde_internal.h"
#include "gde_kernels.h"

namespace gde {

// Runs the iterations of one query in the deterministic order (see gde_det.hip)
// on the workspace w, leaving w's device state (iters, ops, pushes, residual
// norms) and the pushed-set bitmap / x for the caller's output extraction.
template <typename V>
int det_run(const gde_graph *g, const gde_params *p, const gde_seed *sd, Workspace *w, const SeedInline *inl,
            long long *d_trs, long long *d_trv, int32_t *d_trn, long long tr_cap, long long tr_ncap, hipStream_t s,
            bool *converged);

// LocalGD continued from the state in w (residual/degree plane, estimate, pushed
// set, touched bitmap), the re-solve after edge events: S_0 = the active nodes
// of the touched set, or the host list `forced` when given (a first solve's
// supp(s)); signed residuals allowed; the state is left in place (residuals and
// bitmaps are not cleared).  w->st holds the ops, pushes and residual norms.
template <typename V>
int det_warm(const gde_graph *g, const gde_params *p, Workspace *w, hipStream_t s, const int32_t *forced,
             int32_t nforced, int32_t *T, bool *converged);

void det_ws_free(DetWS *d);

}  // namespace gde
