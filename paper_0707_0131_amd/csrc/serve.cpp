// Serving scheduler (placeholder until the continuous-batching loop lands).
#include "engine.h"

extern "C" {
int eigcg_server_create(uint64_t, eigcg_server** out) { if (out) *out = nullptr; return EIGCG_EINVAL; }
int eigcg_server_add(eigcg_server*, eigcg_ctx*, int32_t*) { return EIGCG_EINVAL; }
int eigcg_submit(eigcg_server*, int32_t, const void*, void*, double, uint64_t*) { return EIGCG_EINVAL; }
int eigcg_poll(eigcg_server*, uint64_t, eigcg_stats*) { return EIGCG_EINVAL; }
int eigcg_server_drain(eigcg_server*) { return EIGCG_EINVAL; }
int eigcg_server_destroy(eigcg_server*) { return EIGCG_EINVAL; }
}
