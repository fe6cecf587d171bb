// gde_batch.hip -- batched solver and continuous-batching server (in progress).
#include <hip/hip_runtime.h>

#include "gde_batch.h"
#include "gde_internal.h"

using namespace gde;

extern "C" {

int gde_solve_batch(gde_ctx *ctx, const gde_graph *g, int32_t B, const gde_params *p, const gde_seed *s,
                    gde_result *res, const char *schedule_json, hipStream_t stream) {
    (void)schedule_json;
    if (!ctx || !g || !p || !s || !res || B < 0) return fail(GDE_ERR_INVALID_ARG, "null argument");
    int first = GDE_OK;
    for (int32_t i = 0; i < B; i++) {
        int rc = gde_solve(ctx, g, &p[i], &s[i], &res[i], stream);
        res[i].status = rc;
        if (rc && !first) first = rc;
    }
    return first;
}

int gde_server_create(gde_ctx *, const gde_graph *, const gde_server_cfg *, gde_server **) {
    return fail(GDE_ERR_UNSUPPORTED, "server not built");
}
int gde_server_submit(gde_server *, const gde_params *, const gde_seed *, uint64_t *) {
    return fail(GDE_ERR_UNSUPPORTED, "server not built");
}
int gde_server_poll(gde_server *, gde_completion *, int32_t, int32_t *) {
    return fail(GDE_ERR_UNSUPPORTED, "server not built");
}
int gde_server_insert_edges(gde_server *, int32_t, const int32_t *, const int32_t *) {
    return fail(GDE_ERR_UNSUPPORTED, "server not built");
}
int gde_server_destroy(gde_server *) { return fail(GDE_ERR_UNSUPPORTED, "server not built"); }

}  // extern "C"
