// Internal interface of the host runtime shared by its translation units
// (api.hip: the entry points; group.cpp: grouped launches of uneven
// batches): the plan, the workspace layout, the kernel-argument builders, the
// launch wrapper with per-kernel timing and failure injection, and HIP error
// reporting.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "layout.hpp"
#include "report.hpp"
#include "turpy.h"

namespace turpy {

// Launch-failure injection (turpy_debug_fail_launch): launches left before
// the one that fails, 0 when disarmed; g_injected marks a failure that came
// from it, for the message.
extern std::atomic<int64_t> g_fail_countdown;
extern thread_local bool g_injected;

// TURPY_E_HIP with the HIP error (or the injected failure) after `where`.
turpy_status hip_fail(hipError_t e, const char* where);

#define TURPY_HIP(call, where)                 \
  do {                                         \
    hipError_t e_ = (call);                    \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

#define TURPY_HIP_E(call)            \
  do {                               \
    hipError_t e_ = (call);          \
    if (e_ != hipSuccess) return e_; \
  } while (0)

constexpr double kPi = 3.14159265358979323846;
constexpr double kLog2e = 1.4426950408889634;
constexpr size_t kAlign = 256;

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
inline bool pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

// exp(2 pi i rev) with exact range reduction of rev in FP64.
inline float2 phasor(double rev) {
  rev -= std::rint(rev);
  return make_float2(static_cast<float>(std::cos(2.0 * kPi * rev)), static_cast<float>(std::sin(2.0 * kPi * rev)));
}

inline int signed_bin(int k, int n) { return k < n / 2 ? k : k - n; }

// Per-kernel event timing (turpy_profile).
struct EventPair {
  hipEvent_t start, stop;
};
struct Profiler {
  bool on = false;
  std::string only;  // time only this family when non-empty
  std::map<std::string, std::vector<EventPair>> live;
  std::vector<EventPair> pool;
  EventPair take() {
    if (!pool.empty()) {
      EventPair e = pool.back();
      pool.pop_back();
      return e;
    }
    EventPair e{};
    (void)hipEventCreate(&e.start);
    (void)hipEventCreate(&e.stop);
    return e;
  }
  void recycle() {
    for (auto& kv : live)
      for (auto& e : kv.second) pool.push_back(e);
    live.clear();
  }
};
extern Profiler g_prof;

// Launch `fn` (returning hipError_t) bracketed by events when profiling is on.
template <class Fn>
hipError_t timed(const char* family, hipStream_t st, Fn&& fn) {
  if (g_fail_countdown.load(std::memory_order_relaxed) > 0 && g_fail_countdown.fetch_sub(1) == 1) {
    g_injected = true;
    return hipErrorUnknown;
  }
  if (!g_prof.on || (!g_prof.only.empty() && g_prof.only != family)) return fn();
  EventPair e = g_prof.take();
  (void)hipEventRecord(e.start, st);
  const hipError_t r = fn();
  (void)hipEventRecord(e.stop, st);
  g_prof.live[family].push_back(e);
  return r;
}

}  // namespace turpy

// A plan (turpy_plan_create): the path, its FP64-generated device tables and
// its launch choices.
struct turpy_plan {
  int device = 0;
  int n = 0, M = 0, sh_levels = 0, tf_kind = 0, conv = 0;
  int64_t R = 0, P = 0;
  double dx = 0, wavelength = 0, n0 = 1, l0 = 0, L0 = 0, df = 0;
  std::vector<double> dz, cn2dz;
  // per-screen synthesis constants
  std::vector<float> amp_rev;   // sqrt(0.023) r0^(-5/6) df / (2 pi)
  std::vector<float> amp_rad;   // sqrt(0.023) r0^(-5/6) df
  float df2 = 0, inner = 0, f02 = 0, qexp = 11.0f / 12.0f;
  double alpha = 11.0 / 3.0;
  float2 sh_mean_fac[3] = {};
  // device tables (owned)
  float2* d_tw = nullptr;        // [N]
  float2* d_row = nullptr;       // [M+1][N] h_i[k]
  float2* d_col = nullptr;       // [M+1][N] h_i[k] / N
  // angular spectrum: H_as / H_fresnel as a function of q = k0^2 + k1^2 (signed
  // bins), one table of N^2/2 + 1 entries per distinct distance
  float2* d_as = nullptr;
  std::vector<int> as_index;     // [M+1] table of each step
  float2* d_sh_phasor = nullptr; // [3][N]
  float* d_sh_amp = nullptr;     // [M][3][2]
  float* d_amp_rad = nullptr;    // [M]
  const uint32_t* d_t = nullptr; // bound device time step (turpy_plan_bind_time), or NULL
  float* d_moments = nullptr;    // bound moment sums [4][N][N] (turpy_plan_bind_moments), or NULL
  // TURPY_CHECK_FINITE: non-finite count on the device and its pinned host copy
  unsigned long long* d_nonfinite = nullptr;
  unsigned long long* h_nonfinite = nullptr;
  // strip widths of the column pass and the synthesis (0: built-in choice for n)
  int col_width = 0, synth_width = 0;
  // second-pass radix of their transforms (0: the default plan) and the
  // occupancy hints of the forward and adjoint screen row passes (0: default)
  int col_radix = 0, synth_radix = 0, row_waves = 0, row_waves_bwd = 0;
  // strip width and radix of the synthesis with the AR step fused (0: built-in)
  int ar_width = 0, ar_radix = 0;
  bool screen_ck = false;        // TURPY_SCREEN_CHECKPOINTS: checkpoints keep the screens' column halves
  std::string arch;              // device architecture (tuning-cache key)

  size_t plane_bytes() const { return static_cast<size_t>(n) * n * sizeof(float2); }
  size_t off_sh() const { return turpy::align_up(static_cast<size_t>(P) * plane_bytes()); }
  size_t off_src() const {
    return off_sh() + turpy::align_up(sh_levels > 0 ? static_cast<size_t>(P) * (M > 0 ? M : 1) * 32 * sizeof(float2) : 0);
  }
  size_t off_gbuf() const { return off_src() + turpy::align_up(plane_bytes()); }
  size_t ws_forward() const { return off_gbuf(); }
  size_t ws_backward() const { return off_gbuf() + turpy::align_up(static_cast<size_t>(R) * plane_bytes()); }
  // reversible adjoint: also the rebuilt forward field and its value at the current screen
  size_t off_ubuf() const { return ws_backward(); }
  size_t ws_reversible() const { return ws_backward() + 2 * turpy::align_up(static_cast<size_t>(R) * plane_bytes()); }
  // tuning: the scratch planes (synthesis) and the R-plane buffer (column pass)
  size_t ws_tune() const { return ws_reversible(); }
};

namespace turpy {

// A call's workspace, carved by the offsets of the plan.
struct Ws {
  float2* scratch;
  float2* sh;
  float2* src;
  float2* gbuf;
  // column halves of the screens kept with the checkpoints (plans created with
  // TURPY_SCREEN_CHECKPOINTS): [M][P][N][N], or NULL to use `scratch`
  float2* screens = nullptr;
  size_t screen_stride = 0;
  float2* screen(int s) const { return screens ? screens + static_cast<size_t>(s) * screen_stride : scratch; }
};

inline Ws carve(const turpy_plan* pl, void* ws) {
  char* b = static_cast<char*>(ws);
  return Ws{reinterpret_cast<float2*>(b), reinterpret_cast<float2*>(b + pl->off_sh()),
            reinterpret_cast<float2*>(b + pl->off_src()), reinterpret_cast<float2*>(b + pl->off_gbuf())};
}

inline void key_of(uint64_t seed, uint32_t* k0, uint32_t* k1) {
  *k0 = static_cast<uint32_t>(seed & 0xFFFFFFFFu);
  *k1 = static_cast<uint32_t>(seed >> 32);
}

inline RowArgs base_row(const turpy_plan* pl) {
  RowArgs a{};
  a.tw = pl->d_tw;
  a.waves = pl->row_waves;
  a.R = pl->R;
  a.scale = 1.0f;
  a.M = pl->M;
  a.sh_phasor = pl->d_sh_phasor;
  a.sh_scale = 1.0f;
  return a;
}

inline const char* row_family(const RowArgs& a) {
  if (a.screen_mode == ROW_NO_SCREEN) return "row_plain";
  return a.backward ? "row_bwd" : "row_fwd";
}

inline ColArgs col_args(const turpy_plan* pl, int step, const float2* in, int64_t in_stride, float2* out, int64_t R,
                 bool adjoint) {
  ColArgs c{};
  c.tw = pl->d_tw;
  c.in = in;
  c.in_stride = in_stride;
  c.out = out;
  c.R = R;
  c.table = pl->d_col + static_cast<size_t>(step) * pl->n;
  c.conj_table = adjoint ? 1 : 0;
  c.width = pl->col_width;
  c.radix = pl->col_radix;
  c.angular = pl->tf_kind == TURPY_TF_ANGULAR_SPECTRUM ? 1 : 0;
  if (c.angular) {
    if (pl->d_as)
      c.as_table = pl->d_as + static_cast<size_t>(pl->as_index[step]) * (static_cast<size_t>(pl->n) * pl->n / 2 + 1);
    const double k = 2.0 * kPi * pl->n0 / pl->wavelength;
    const double w2 = (2.0 * kPi * pl->df) * (2.0 * kPi * pl->df);
    c.as_b = static_cast<float>(w2 / (k * k));
    c.as_c = static_cast<float>(-pl->dz[step] * w2 * w2 / (4.0 * kPi * k * k * k));
  }
  return c;
}

// An AR step fused into the synthesis (turpy_evolve_propagate).
struct EvolveStep {
  double alpha, sx, sy;
};

inline SynthArgs synth_args(const turpy_plan* pl, uint64_t seed, uint32_t t, int s, const float2* spectra, const Ws& w,
                     const EvolveStep* ev = nullptr) {
  SynthArgs a{};
  a.tw = pl->d_tw;
  a.scratch = w.screen(s);
  a.P = pl->P;
  key_of(seed, &a.key0, &a.key1);
  a.t = t;
  a.t_dev = pl->d_t;
  a.screen = static_cast<uint32_t>(s);
  a.tag = TAG_MAIN;
  a.amp = pl->amp_rev[s];
  a.df2 = pl->df2;
  a.inner = pl->inner;
  a.f02 = pl->f02;
  a.q = pl->qexp;
  a.spectra = spectra;
  a.M = pl->M;
  a.width = ev ? pl->ar_width : pl->synth_width;
  a.radix = ev ? pl->ar_radix : pl->synth_radix;
  if (ev) {
    a.evolve = 1;
    a.state = const_cast<float2*>(spectra);
    a.ar_tag = TAG_AR;
    a.alpha_f = static_cast<float>(ev->alpha);
    a.blend = static_cast<float>(std::sqrt(1.0 - ev->alpha * ev->alpha));
    a.sx = ev->sx;
    a.sy = ev->sy;
    a.amp_rad = pl->amp_rad[s];
  }
  return a;
}

// Arguments of the subharmonic kernel: fresh coefficients of every pair and screen.
inline ShArgs sh_args(const turpy_plan* pl, uint64_t seed, uint32_t t, float2* sh) {
  ShArgs a{};
  a.sh = sh;
  a.P = pl->P;
  a.M = pl->M;
  a.levels = pl->sh_levels;
  a.n = pl->n;
  key_of(seed, &a.key0, &a.key1);
  a.t = t;
  a.t_dev = pl->d_t;
  a.tag = TAG_SH;
  a.amp = pl->d_sh_amp;
  a.scale = 1.0f;
  for (int i = 0; i < 3; ++i) a.mean_fac[i] = pl->sh_mean_fac[i];
  return a;
}

// The subharmonic block of an AR state: after the pair spectra.
inline float2* state_sh(const turpy_plan* pl, const void* spectra) {
  return const_cast<float2*>(static_cast<const float2*>(spectra)) +
         static_cast<size_t>(pl->P) * pl->M * pl->n * pl->n;
}

// Fill the screen fields of a row pass for screen s.
inline turpy_status screen_fields(const turpy_plan* pl, int32_t src, const void* screens_or_spectra, const Ws& w,
                                  int s, RowArgs* a) {
  a->screen = s;
  if (src == TURPY_SCREENS_MATERIALIZED) {
    a->screen_mode = ROW_MATERIALIZED;
    a->screens = static_cast<const float*>(screens_or_spectra);
  } else {
    a->screen_mode = ROW_SCRATCH;
    a->scratch = w.screen(s);
    a->sh_levels = pl->sh_levels;
    if (src == TURPY_SCREENS_SYNTH) {
      a->sh = w.sh;
      a->sh_scale = 1.0f;
    } else {  // the AR state's subharmonic block, in radians
      a->sh = state_sh(pl, screens_or_spectra);
      a->sh_scale = static_cast<float>(1.0 / (2.0 * kPi));
    }
  }
  return TURPY_OK;
}

}  // namespace turpy
