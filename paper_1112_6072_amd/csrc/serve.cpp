// Serving loop of libhperm (continuous batching of permanent requests).
#include "ctx.h"

namespace hp {
struct Serving {};
void serve_shutdown(hperm_ctx *) {}
}  // namespace hp

extern "C" {

hperm_status hperm_serve_start(hperm_ctx *c, int32_t, size_t) {
    return hp::set_error(c, HPERM_E_INVALID, "serving is not available in this build");
}
hperm_status hperm_serve_stop(hperm_ctx *c) {
    return hp::set_error(c, HPERM_E_INVALID, "serving is not available in this build");
}
hperm_status hperm_submit(hperm_ctx *c, int32_t, const int32_t *, const int32_t *, const uint32_t *,
                          uint64_t *) {
    return hp::set_error(c, HPERM_E_INVALID, "serving is not available in this build");
}
hperm_status hperm_poll(hperm_ctx *c, uint64_t, hperm_result *) {
    return hp::set_error(c, HPERM_E_INVALID, "serving is not available in this build");
}
hperm_status hperm_wait(hperm_ctx *c, uint64_t, double, hperm_result *) {
    return hp::set_error(c, HPERM_E_INVALID, "serving is not available in this build");
}
hperm_status hperm_cancel(hperm_ctx *c, uint64_t) {
    return hp::set_error(c, HPERM_E_INVALID, "serving is not available in this build");
}

}  // extern "C"
