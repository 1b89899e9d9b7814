// placeholder, replaced by the server implementation
#include "sip_runtime.h"
extern "C" {
sip_status sip_server_create(const sip_server_config *, sip_server *) { return sipk::set_error(SIP_EINVAL, "server not built"); }
sip_status sip_batch_submit(sip_server, const sip_request *, uint64_t *) { return SIP_EINVAL; }
sip_status sip_batch_poll(sip_server, uint64_t, int32_t, sip_result *) { return SIP_EINVAL; }
sip_status sip_server_release(sip_server, uint64_t) { return SIP_EINVAL; }
sip_status sip_server_stats(sip_server, uint64_t *) { return SIP_EINVAL; }
sip_status sip_server_destroy(sip_server) { return SIP_EINVAL; }
}
