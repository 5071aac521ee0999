// Serving loop (placeholder until the continuous-batching server lands).
#include <errno.h>

#include "runtime.h"

struct devirt_server {
    int unused;
};

extern "C" int devirt_server_start(devirt_ctx *, const devirt_server_cfg *, devirt_server **out) {
    if (out) *out = nullptr;
    return dv_fail(-ENOSYS, "the serving loop is not available in this build");
}
extern "C" int devirt_server_submit(devirt_server *, const devirt_request *, uint32_t, uint32_t *) {
    return dv_fail(-ENOSYS, "the serving loop is not available in this build");
}
extern "C" int devirt_server_poll(devirt_server *, devirt_completion *, uint32_t, uint32_t *) {
    return dv_fail(-ENOSYS, "the serving loop is not available in this build");
}
extern "C" int devirt_server_drain(devirt_server *) {
    return dv_fail(-ENOSYS, "the serving loop is not available in this build");
}
extern "C" int devirt_server_stop(devirt_server *) {
    return dv_fail(-ENOSYS, "the serving loop is not available in this build");
}
