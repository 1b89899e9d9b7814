// Host-only helpers of the SIP library: error reporting (sip_last_error,
// sip_status_str in include/sip.h).
#include "sip_host.h"

#include <cstdarg>
#include <cstdio>

namespace sipk {

thread_local std::string g_last_error;

sip_status set_error(sip_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

}  // namespace sipk

extern "C" {

const char *sip_last_error(void) { return sipk::g_last_error.c_str(); }

const char *sip_status_str(sip_status st)
{
    switch (st) {
    case SIP_OK: return "SIP_OK";
    case SIP_PENDING: return "SIP_PENDING";
    case SIP_EINVAL: return "SIP_EINVAL";
    case SIP_ENOMEM: return "SIP_ENOMEM";
    case SIP_EBREAKDOWN: return "SIP_EBREAKDOWN";
    case SIP_ENOTCONV: return "SIP_ENOTCONV";
    case SIP_EDEVICE: return "SIP_EDEVICE";
    case SIP_EBUSY: return "SIP_EBUSY";
    case SIP_ECANCELLED: return "SIP_ECANCELLED";
    }
    return "SIP_UNKNOWN";
}

}  // extern "C"
