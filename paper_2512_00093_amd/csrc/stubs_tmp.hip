// temporary: batch and serve entry points (replaced by batch.hip / serve.hip)
#include "../../include/ranmar.h"
extern "C" {
int ranmar_batch_create(uint64_t, uint64_t, uint64_t, ranmar_batch**) { return RANMAR_EINVAL; }
int ranmar_batch_run(ranmar_batch*, const ranmar_request*, uint64_t, void*) { return RANMAR_EINVAL; }
int ranmar_run_unbatched(const ranmar_request*, uint64_t, void*) { return RANMAR_EINVAL; }
int ranmar_batch_destroy(ranmar_batch*) { return RANMAR_EINVAL; }
int ranmar_serve_create(void*, uint64_t, const ranmar_serve_cfg*, ranmar_server**) { return RANMAR_EINVAL; }
int ranmar_serve_submit(ranmar_server*, int32_t, ranmar_u128, uint64_t, int, uint64_t, uint64_t*) { return RANMAR_EINVAL; }
int ranmar_serve_poll(ranmar_server*, uint64_t, int*) { return RANMAR_EINVAL; }
int ranmar_serve_wait(ranmar_server*, uint64_t, int64_t) { return RANMAR_EINVAL; }
int ranmar_serve_result(ranmar_server*, uint64_t, const void**, uint64_t*) { return RANMAR_EINVAL; }
int ranmar_serve_release(ranmar_server*, uint64_t) { return RANMAR_EINVAL; }
int ranmar_serve_stats_get(ranmar_server*, ranmar_serve_stats*) { return RANMAR_EINVAL; }
int ranmar_serve_destroy(ranmar_server*) { return RANMAR_EINVAL; }
}
