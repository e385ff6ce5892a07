// Error reporting shared by the library's translation units: the message
// becomes this thread's turpy_last_error() and the status is returned.
#pragma once
#include "turpy.h"

namespace turpy {
turpy_status report(turpy_status st, const char* fmt, ...);
}  // namespace turpy
