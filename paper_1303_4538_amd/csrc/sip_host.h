// Host-only helpers shared by every part of the SIP library: the calling
// thread's last error.  No device code and no HIP header, so that the parts
// built on it (the request scheduler) also build with a plain C++ compiler.
#pragma once
#include "../../include/sip.h"

#include <string>

namespace sipk {

extern thread_local std::string g_last_error;
// Records the message for sip_last_error() and returns st.
sip_status set_error(sip_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

}  // namespace sipk
