// Host helpers shared by the library's translation units.
#pragma once
#include <cstdarg>
#include <cstdint>
#include <string>

#include "turpy.h"

namespace turpy {
// Error reporting: the message becomes this thread's turpy_last_error() and
// the status is returned.
turpy_status report(turpy_status st, const char* fmt, ...);
turpy_status vreport(turpy_status st, const char* fmt, va_list ap);
// turpy_plan_create's checks of a path descriptor and the plan flags.
turpy_status validate_path(const turpy_path* p, uint32_t flags);
// The tuning-cache keys of a plan's column pass and synthesis as one string
// (equal strings: the same keys).
std::string tune_signature(const turpy_plan* pl);
}  // namespace turpy
