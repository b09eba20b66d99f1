#include "common.hpp"
namespace rk {
rocket_status sp_prepare(rocket_ctx *ctx, const rocket_items *, int64_t, hipStream_t) { return fail(ctx, ROCKET_E_UNSUPPORTED, "sparse not built yet"); }
rocket_status sp_compare(rocket_ctx *ctx, float *, uint32_t *, hipStream_t) { return fail(ctx, ROCKET_E_UNSUPPORTED, "sparse not built yet"); }
}
