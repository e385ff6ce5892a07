// Host helpers shared by the library's translation units.
#pragma once
#include <string>

#include "turpy.h"

namespace turpy {
// Error reporting: the message becomes this thread's turpy_last_error() and
// the status is returned.
turpy_status report(turpy_status st, const char* fmt, ...);
// The tuning-cache keys of a plan's column pass and synthesis as one string
// (equal strings: the same keys).
std::string tune_signature(const turpy_plan* pl);
}  // namespace turpy
