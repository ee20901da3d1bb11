// Serving loop (continuous batching under a device-memory budget).
#include "msf_internal.hpp"

using namespace msf;

extern "C" {

msf_status msf_server_create(msf_ctx *, size_t, msf_server **)
{
    set_error("server not available");
    return MSF_EINVAL;
}
void msf_server_destroy(msf_server *) {}
msf_status msf_server_submit(msf_server *, int32_t, int64_t, const int32_t *, const void *,
                             msf_wtype, uint64_t *)
{
    return MSF_EINVAL;
}
msf_status msf_server_poll(msf_server *, uint64_t, int *) { return MSF_EINVAL; }
msf_status msf_server_latency(msf_server *, uint64_t, double *) { return MSF_EINVAL; }
msf_status msf_server_result(msf_server *, uint64_t, int32_t *, int64_t *, msf_total *)
{
    return MSF_EINVAL;
}

}  // extern "C"
