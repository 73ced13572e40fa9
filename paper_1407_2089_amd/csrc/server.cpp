// Serving loop (vr_submit / vr_poll / vr_release).
#include "lib.h"

namespace vr {

vr_status server_submit(vr_ctx*, const vr_render_req*, uint64_t*) {
    return fail(VR_ERR_UNSUPPORTED, "serving is not available in this build");
}
vr_status server_poll(vr_ctx*, uint64_t, vr_ticket_info*) {
    return fail(VR_ERR_NOT_FOUND, "unknown ticket");
}
vr_status server_release(vr_ctx*, uint64_t) { return fail(VR_ERR_NOT_FOUND, "unknown ticket"); }
vr_status server_stop(vr_ctx*) { return VR_OK; }

}  // namespace vr

using namespace vr;

extern "C" {
vr_status vr_submit(vr_ctx* ctx, const vr_render_req* req, uint64_t* ticket) {
    if (!ctx) return fail(VR_ERR_INVALID_ARG, "context is NULL");
    if (!ticket) return fail(VR_ERR_INVALID_ARG, "ticket is NULL");
    vr_status st = check_request(ctx, req);
    if (st != VR_OK) return st;
    return server_submit(ctx, req, ticket);
}
vr_status vr_poll(vr_ctx* ctx, uint64_t ticket, vr_ticket_info* info) {
    if (!ctx) return fail(VR_ERR_INVALID_ARG, "context is NULL");
    if (!info) return fail(VR_ERR_INVALID_ARG, "info is NULL");
    return server_poll(ctx, ticket, info);
}
vr_status vr_release(vr_ctx* ctx, uint64_t ticket) {
    if (!ctx) return fail(VR_ERR_INVALID_ARG, "context is NULL");
    return server_release(ctx, ticket);
}
}
