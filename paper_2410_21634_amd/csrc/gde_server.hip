// gde_server.hip -- continuous-batching server (not yet provided).
#include <hip/hip_runtime.h>

#include "gde_batch.h"
#include "gde_internal.h"

using namespace gde;

extern "C" {

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
