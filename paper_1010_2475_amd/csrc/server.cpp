// Serving entry points (placeholder until the batching server lands).
#include "api_internal.hpp"

extern "C" {
mmvm_status mmvm_server_create(size_t, int32_t, mmvm_server** out)
{
    if (out) *out = nullptr;
    return MMVM_EINVAL;
}
mmvm_status mmvm_submit(mmvm_server*, const mmvm_problem*, double, double, int64_t, const double*, const double*,
                        mmvm_precision, uint64_t*)
{
    return MMVM_EINVAL;
}
mmvm_status mmvm_poll(mmvm_server*, uint64_t, double*, double*, mmvm_stats*) { return MMVM_ENOTFOUND; }
mmvm_status mmvm_server_drain(mmvm_server*) { return MMVM_EINVAL; }
mmvm_status mmvm_server_destroy(mmvm_server*) { return MMVM_OK; }
}
