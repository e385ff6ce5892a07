// Host-only part of the library: the thread's error message and the
// validation of path descriptors.  Plain C++ (no HIP), so that it also builds
// with the host compiler and its sanitizers.
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "report.hpp"
#include "turpy.h"

namespace {

thread_local std::string g_last_error;

bool pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

}  // namespace

turpy_status turpy::vreport(turpy_status st, const char* fmt, va_list ap) {
  char buf[512];
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  g_last_error = buf;
  return st;
}

turpy_status turpy::report(turpy_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  const turpy_status r = vreport(st, fmt, ap);
  va_end(ap);
  return r;
}

// A path descriptor as turpy_plan_create accepts it (Sec. 2.1 inputs; the
// sampling limit of Eq. 7), checked before anything touches the GPU.
turpy_status turpy::validate_path(const turpy_path* p, uint32_t flags) {
  if (!p) return report(TURPY_E_INVALID, "plan_create: NULL argument");
  if (flags & ~(TURPY_ALLOW_ALIASING | TURPY_SCREEN_CHECKPOINTS | TURPY_CHECK_FINITE))
    return report(TURPY_E_INVALID, "plan_create: unknown flags 0x%x", flags);
  if (!pow2(p->n)) return report(TURPY_E_INVALID, "plan_create: n=%d is not a power of two", p->n);
  if (p->n < 16 || p->n > 2048) return report(TURPY_E_UNSUPPORTED, "plan_create: n=%d outside 16..2048", p->n);
  if (p->num_screens < 0) return report(TURPY_E_INVALID, "plan_create: num_screens < 0");
  if (p->num_screens > (1 << 20)) return report(TURPY_E_UNSUPPORTED, "plan_create: num_screens too large");
  if (!(p->dx > 0) || !std::isfinite(p->dx)) return report(TURPY_E_INVALID, "plan_create: dx must be > 0");
  if (!(p->wavelength > 0) || !std::isfinite(p->wavelength))
    return report(TURPY_E_INVALID, "plan_create: wavelength must be > 0");
  if (!(p->n0 > 0) || !std::isfinite(p->n0)) return report(TURPY_E_INVALID, "plan_create: n0 must be > 0");
  if (!p->dz) return report(TURPY_E_INVALID, "plan_create: dz is NULL");
  if (p->num_screens > 0 && !p->cn2dz) return report(TURPY_E_INVALID, "plan_create: cn2dz is NULL");
  if (p->sh_levels < 0 || p->sh_levels > 3)
    return report(TURPY_E_UNSUPPORTED, "plan_create: sh_levels=%d outside 0..3", p->sh_levels);
  if (p->tf_kind != TURPY_TF_FRESNEL && p->tf_kind != TURPY_TF_ANGULAR_SPECTRUM)
    return report(TURPY_E_INVALID, "plan_create: unknown tf_kind %d", p->tf_kind);
  if (p->inner_scale_conv != 0 && p->inner_scale_conv != 1)
    return report(TURPY_E_INVALID, "plan_create: inner_scale_conv must be 0 or 1");
  if (p->realizations < 1 || p->realizations > (int64_t(1) << 31))
    return report(TURPY_E_INVALID, "plan_create: realizations=%lld out of range", (long long)p->realizations);
  if (std::isnan(p->l0) || std::isnan(p->L0)) return report(TURPY_E_INVALID, "plan_create: l0/L0 is NaN");
  if (p->psd_alpha != 0.0 && !(p->psd_alpha > 2.0 && p->psd_alpha < 6.0))
    return report(TURPY_E_INVALID, "plan_create: psd_alpha=%g outside (2, 6) (0 selects 11/3)", p->psd_alpha);
  const int M = p->num_screens, n = p->n;
  const double limit = n * p->dx * p->dx * p->n0 / p->wavelength;  // Eq. 7 at the Nyquist frequency
  for (int i = 0; i <= M; ++i) {
    const double d = p->dz[i];
    if (!(d >= 0) || !std::isfinite(d)) return report(TURPY_E_INVALID, "plan_create: dz[%d] must be >= 0", i);
    if (i > 0 && i < M && d == 0)
      return report(TURPY_E_UNSUPPORTED, "plan_create: dz[%d] = 0 between two screens (merge them)", i);
    if (d > limit && !(flags & TURPY_ALLOW_ALIASING))
      return report(TURPY_E_ALIASING, "plan_create: dz[%d] = %g m exceeds the sampling limit N dx^2 n0/lambda = %g m",
                    i, d, limit);
  }
  for (int i = 0; i < M; ++i)
    if (!(p->cn2dz[i] >= 0) || !std::isfinite(p->cn2dz[i]))
      return report(TURPY_E_INVALID, "plan_create: cn2dz[%d] must be >= 0", i);
  return TURPY_OK;
}

extern "C" const char* turpy_last_error(void) { return g_last_error.c_str(); }
