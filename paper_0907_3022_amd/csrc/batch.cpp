// Batched propagation of many independent ribbons (placeholder until the
// batched kernels land).
#include <string>

#include "internal.h"

namespace chebtd {
int fail(Ctx *c, int code, const std::string &msg);
struct BatchState {};
void batch_destroy(Ctx *c)
{
    delete c->batch;
    c->batch = nullptr;
}
}  // namespace chebtd

using namespace chebtd;
struct chebtd_ctx : public Ctx {};

extern "C" {
int chebtd_batch_create(chebtd_ctx *ctx, int, const chebtd_sys_desc *, double, double, double)
{
    return fail(ctx, CHEBTD_E_STATE, "batched propagation is not available yet");
}
int chebtd_batch_set_schedule(chebtd_ctx *ctx, int, int, int, int)
{
    return fail(ctx, CHEBTD_E_STATE, "batched propagation is not available yet");
}
int chebtd_batch_autotune(chebtd_ctx *ctx, const char *, int *)
{
    return fail(ctx, CHEBTD_E_STATE, "batched propagation is not available yet");
}
int chebtd_batch_propagate(chebtd_ctx *ctx, int64_t, unsigned)
{
    return fail(ctx, CHEBTD_E_STATE, "batched propagation is not available yet");
}
int chebtd_batch_info(const chebtd_ctx *ctx, int *, int *)
{
    return fail(const_cast<chebtd_ctx *>(ctx), CHEBTD_E_STATE, "batched propagation is not available yet");
}
}
