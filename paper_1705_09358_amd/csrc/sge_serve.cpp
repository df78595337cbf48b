// Serving: resident targets, queries admitted as slots and memory allow.
#include "sge_ctx.h"

using namespace sge;

namespace sge {
struct Server {};
void ServerDeleter::operator()(Server *s) const { delete s; }
}  // namespace sge

extern "C" {

__attribute__((visibility("hidden"))) void sge_serve_shutdown_internal(sge_ctx *c) {
    if (c) c->server.reset();
}

sge_status sge_serve_start(sge_ctx *c, uint32_t, uint64_t) {
    return fail(c, SGE_E_INVAL, "serving is not available in this build");
}
sge_status sge_serve_submit(sge_ctx *c, const sge_job *, uint64_t *) {
    return fail(c, SGE_E_INVAL, "server not started");
}
sge_status sge_serve_poll(sge_ctx *c, uint64_t, sge_result *) {
    return fail(c, SGE_E_HANDLE, "server not started");
}
sge_status sge_serve_stop(sge_ctx *c) {
    if (!c) return SGE_E_INVAL;
    c->server.reset();
    return SGE_OK;
}

}  // extern "C"
