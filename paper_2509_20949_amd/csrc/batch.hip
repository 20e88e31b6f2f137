// batch.hip -- batched replicas and the serving loop (filled in below).
#include "../../include/smcx.h"
#include "ctx.h"

using namespace smcx;

extern "C" {
smcx_status smcx_batch_create(int32_t, const smcx_desc*, const uint8_t* const*, const int32_t* const*,
                              const double*, smcx_batch** out)
{
    if (out) *out = nullptr;
    return fail_global(SMCX_E_UNSUPPORTED, "not built yet");
}
smcx_status smcx_batch_run(smcx_batch*, const int32_t*) { return SMCX_E_UNSUPPORTED; }
smcx_status smcx_batch_run_unbatched(smcx_batch*, const int32_t*) { return SMCX_E_UNSUPPORTED; }
smcx_status smcx_batch_ctx(smcx_batch*, int32_t, smcx_ctx**) { return SMCX_E_UNSUPPORTED; }
smcx_status smcx_batch_set_temperature(smcx_batch*, int32_t, double) { return SMCX_E_UNSUPPORTED; }
smcx_status smcx_batch_exchange(smcx_batch*, const int32_t*, const int32_t*, int32_t, uint64_t, uint64_t, int32_t*)
{
    return SMCX_E_UNSUPPORTED;
}
smcx_status smcx_batch_synchronize(smcx_batch*) { return SMCX_E_UNSUPPORTED; }
void smcx_batch_destroy(smcx_batch*) {}
smcx_status smcx_server_create(size_t, int32_t, int32_t, smcx_server** out)
{
    if (out) *out = nullptr;
    return SMCX_E_UNSUPPORTED;
}
smcx_status smcx_server_submit(smcx_server*, const smcx_desc*, const uint8_t*, const int32_t*, double, int32_t,
                               uint64_t*)
{
    return SMCX_E_UNSUPPORTED;
}
smcx_status smcx_server_step(smcx_server*, int32_t*, int32_t*, int32_t*) { return SMCX_E_UNSUPPORTED; }
smcx_status smcx_server_poll(smcx_server*, uint64_t, int32_t*) { return SMCX_E_UNSUPPORTED; }
smcx_status smcx_server_result(smcx_server*, uint64_t, int64_t*, uint64_t*, uint8_t*, size_t)
{
    return SMCX_E_UNSUPPORTED;
}
size_t smcx_server_footprint(const smcx_desc*) { return 0; }
void smcx_server_destroy(smcx_server*) {}
const char* smcx_server_last_error(const smcx_server*) { return ""; }
}
