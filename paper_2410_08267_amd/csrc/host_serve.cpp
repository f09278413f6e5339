// Batched solve and the continuous-batching serving loop.
#include <hip/hip_runtime.h>

#include "nh_context.h"

namespace nh {
void serve_shutdown(nh_context *ctx) { (void)ctx; }
}  // namespace nh

using namespace nh;

extern "C" {

int nh_serve_set_budget(nh_context *ctx, size_t bytes)
{
    (void)bytes;
    return set_err(ctx, NH_EINVAL, "serving: not built yet");
}

int nh_submit(nh_context *ctx, const nh_request *req, uint64_t *ticket)
{
    (void)req; (void)ticket;
    return set_err(ctx, NH_EINVAL, "serving: not built yet");
}

int nh_poll(nh_context *ctx, uint64_t ticket, double *out, nh_stats *stats)
{
    (void)ticket; (void)out; (void)stats;
    return set_err(ctx, NH_EINVAL, "serving: not built yet");
}

int nh_cancel(nh_context *ctx, uint64_t ticket)
{
    (void)ticket;
    return set_err(ctx, NH_EINVAL, "serving: not built yet");
}

}  // extern "C"
