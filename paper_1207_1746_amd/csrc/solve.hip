// gscl_solve: placeholder until the solver driver lands.
#include "api_internal.h"

extern "C" size_t gscl_solve_workspace_bytes(const gscl_solve_desc*, const gscl_grid*, int) { return 0; }
extern "C" int gscl_solve(gscl_ctx*, const gscl_solve_desc*, gscl_grid* const*, const gscl_grid* const*, int,
                          const gscl_grid* const*, int, void*, size_t, gscl_solve_stats*) {
    return gscl_fail(GSCL_ERR_UNSUPPORTED, "gscl_solve not built yet");
}
extern "C" int gscl_batch_create(gscl_ctx*, const gscl_batch_desc*, gscl_batch**) {
    return gscl_fail(GSCL_ERR_UNSUPPORTED, "batch not built yet");
}
extern "C" size_t gscl_batch_footprint(const gscl_batch*, const int64_t*) { return 0; }
extern "C" int gscl_batch_admit(gscl_batch*, gscl_grid*, const gscl_grid*, double, int*) {
    return gscl_fail(GSCL_ERR_UNSUPPORTED, "batch not built yet");
}
extern "C" int gscl_batch_step(gscl_batch*) { return gscl_fail(GSCL_ERR_UNSUPPORTED, "batch not built yet"); }
extern "C" int gscl_batch_poll(gscl_batch*, int*, int, int*) { return gscl_fail(GSCL_ERR_UNSUPPORTED, "batch not built yet"); }
extern "C" int gscl_batch_retire(gscl_batch*, int, gscl_slot_stats*) { return gscl_fail(GSCL_ERR_UNSUPPORTED, "batch not built yet"); }
extern "C" int gscl_batch_destroy(gscl_batch*) { return gscl_fail(GSCL_ERR_UNSUPPORTED, "batch not built yet"); }
