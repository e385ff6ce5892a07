// Host runtime of the C ABI declared in include/turpy.h: validation, plans
// with FP64-generated tables, workspace layout and the pass schedule of each
// entry point.  Every kernel is enqueued on the caller's stream; nothing here
// synchronises except plan creation / destruction (table upload / free), the
// tuner and the output checks of TURPY_CHECK_FINITE plans.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "runtime.hpp"
#include "turpy.h"

using namespace turpy;

std::atomic<int64_t> turpy::g_fail_countdown{0};
thread_local bool turpy::g_injected = false;
turpy::Profiler turpy::g_prof;

namespace {

turpy_status fail(turpy_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  const turpy_status r = turpy::vreport(st, fmt, ap);
  va_end(ap);
  return r;
}

}  // namespace

turpy_status turpy::hip_fail(hipError_t e, const char* where) {
  if (g_injected) {
    g_injected = false;
    return fail(TURPY_E_HIP, "%s: launch failure injected by turpy_debug_fail_launch", where);
  }
  return fail(TURPY_E_HIP, "%s: %s", where, hipGetErrorString(e));
}

namespace {

// Device scratch of turpy_propagate_static: one array per GPU the library
// runs on, held until the process ends.  Host code never uses the name
// `scratch` as an address: turpy_plan_create looks up each device's copy with
// hipGetSymbolAddress once, and the kernels get that pointer.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;  // device -> address of its `scratch`

// Record the current device's scratch address (set-up time, once per device).
hipError_t register_static_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr.count(device)) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

void* static_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  return it == g_scratch_ptr.end() ? nullptr : it->second;
}

}  // namespace

namespace {
void apply_cached_widths(turpy_plan* pl);
std::string device_arch(int device);
}  // namespace

extern "C" {

const char* turpy_version(void) { return "turpy-mi355x 0.1 (gfx950)"; }

turpy_status turpy_plan_create(turpy_plan** out, const turpy_path* p, uint32_t flags) {
  if (!out || !p) return fail(TURPY_E_INVALID, "plan_create: NULL argument");
  *out = nullptr;
  if (turpy_status s_ = turpy::validate_path(p, flags)) return s_;
  const int M = p->num_screens, n = p->n;

  turpy_plan* pl = new turpy_plan();
  (void)hipGetDevice(&pl->device);
  pl->n = n;
  pl->M = M;
  pl->sh_levels = p->sh_levels;
  pl->tf_kind = p->tf_kind;
  pl->conv = p->inner_scale_conv;
  pl->R = p->realizations;
  pl->P = (p->realizations + 1) / 2;
  pl->screen_ck = (flags & TURPY_SCREEN_CHECKPOINTS) != 0;
  pl->dx = p->dx;
  pl->wavelength = p->wavelength;
  pl->n0 = p->n0;
  pl->l0 = p->l0;
  pl->L0 = p->L0;
  pl->df = 1.0 / (n * p->dx);
  pl->alpha = p->psd_alpha != 0.0 ? p->psd_alpha : 11.0 / 3.0;
  pl->qexp = static_cast<float>(pl->alpha / 4.0);
  pl->dz.assign(p->dz, p->dz + M + 1);
  if (M > 0) pl->cn2dz.assign(p->cn2dz, p->cn2dz + M);

  // PSD constants (Eq. S17, frequencies in cycles/m)
  const double df = pl->df;
  double fm2 = 0.0;  // 0: no inner-scale cutoff
  if (p->l0 > 0) {
    const double fm = p->inner_scale_conv == 1 ? 5.92 / (2.0 * kPi * p->l0) : 1.0 / p->l0;
    fm2 = fm * fm;
  }
  const double f0 = (std::isfinite(p->L0) && p->L0 > 0) ? 1.0 / p->L0 : 0.0;
  pl->df2 = static_cast<float>(df * df);
  pl->inner = fm2 > 0 ? static_cast<float>(kLog2e / (2.0 * fm2)) : 0.0f;
  pl->f02 = static_cast<float>(f0 * f0);
  const double k = 2.0 * kPi * p->n0 / p->wavelength;
  const double alpha = pl->alpha;
  auto psd = [&](double f2, double r0inv53) {  // W(f^2) of Eq. S17 (power law alpha)
    const double inner = fm2 > 0 ? std::exp(-f2 / fm2) : 1.0;
    return 0.023 * r0inv53 * inner / std::pow(f2 + f0 * f0, alpha / 2.0);
  };
  std::vector<float> sh_amp(static_cast<size_t>(std::max(M, 1)) * 6, 0.0f);
  for (int s = 0; s < M; ++s) {
    // Eq. S18: r0 = (0.423 k^2 cn2dz)^(-3/5); r0^(-5/3) = 0.423 k^2 cn2dz
    const double r0inv53 = 0.423 * k * k * p->cn2dz[s];
    const double a = std::sqrt(0.023 * r0inv53) * df;  // sqrt(0.023) r0^(-5/6) df
    pl->amp_rad.push_back(static_cast<float>(a));
    pl->amp_rev.push_back(static_cast<float>(a / (2.0 * kPi)));
    for (int lv = 0; lv < 3; ++lv) {
      const double dfp = df / std::pow(3.0, lv + 1);
      for (int d = 0; d < 2; ++d) {
        const double f2 = (d + 1) * dfp * dfp;
        sh_amp[(static_cast<size_t>(s) * 3 + lv) * 2 + d] =
            static_cast<float>(std::sqrt(psd(f2, r0inv53)) * dfp / (2.0 * kPi));
      }
    }
  }

  // FP64-generated tables
  std::vector<float2> tw(n), row(static_cast<size_t>(M + 1) * n), col(static_cast<size_t>(M + 1) * n),
      shp(static_cast<size_t>(3) * n);
  for (int i = 0; i < n; ++i) tw[i] = phasor(-static_cast<double>(i) / n);
  for (int s = 0; s <= M; ++s) {
    // h(k) = exp(-i pi (lambda/n0) dz f_k^2): revolutions -(lambda/n0) dz df^2 k^2 / 2
    const double a = (p->wavelength / p->n0) * pl->dz[s] * df * df * 0.5;
    for (int kk = 0; kk < n; ++kk) {
      const double kh = signed_bin(kk, n);
      const float2 h = phasor(-a * kh * kh);
      row[static_cast<size_t>(s) * n + kk] = h;
      col[static_cast<size_t>(s) * n + kk] = make_float2(h.x / n, h.y / n);
    }
  }
  for (int lv = 0; lv < 3; ++lv) {
    const double scale = 1.0 / (static_cast<double>(n) * std::pow(3.0, lv + 1));
    double mr = 0, mi = 0;
    for (int i = 0; i < n; ++i) {
      const double rev = (i - n / 2) * scale;
      shp[static_cast<size_t>(lv) * n + i] = phasor(rev);
      mr += std::cos(2.0 * kPi * rev);
      mi += std::sin(2.0 * kPi * rev);
    }
    pl->sh_mean_fac[lv] = make_float2(static_cast<float>(mr / n), static_cast<float>(mi / n));
  }
  // Angular-spectrum correction (Sec. 2.1, R1): H_as / H_fresnel at
  // kappa^2 = (2 pi df)^2 q, in FP64 with exact range reduction:
  //   propagating (kappa < k): exp(-i dz kappa^4 / (2k (s + k)^2)), s = sqrt(k^2 - kappa^2)
  //   evanescent: exp(-dz sqrt(kappa^2 - k^2)) exp(i dz (kappa^2 / (2k) - k))
  std::vector<float2> as;
  // the grid corner kappa^2 = 2 (pi/dx)^2 against k^2: tables only where bins are evanescent
  const bool evanescent = 2.0 * (kPi / pl->dx) * (kPi / pl->dx) >= 0.999 * k * k;
  if (pl->tf_kind == TURPY_TF_ANGULAR_SPECTRUM && evanescent) {
    const size_t qn = static_cast<size_t>(n) * n / 2 + 1;
    std::vector<double> distinct;
    for (int s = 0; s <= M; ++s) {
      int idx = -1;
      for (size_t d = 0; d < distinct.size(); ++d)
        if (distinct[d] == pl->dz[s]) idx = static_cast<int>(d);
      if (idx < 0) {
        idx = static_cast<int>(distinct.size());
        distinct.push_back(pl->dz[s]);
      }
      pl->as_index.push_back(idx);
    }
    as.resize(distinct.size() * qn);
    const double w2 = (2.0 * kPi * df) * (2.0 * kPi * df);
    for (size_t d = 0; d < distinct.size(); ++d) {
      const double dz = distinct[d];
      for (size_t q = 0; q < qn; ++q) {
        const double kap2 = w2 * static_cast<double>(q);
        float2 v;
        if (kap2 < k * k) {
          const double sp = std::sqrt(k * k - kap2) + k;
          v = phasor(-dz * kap2 * kap2 / (2.0 * k * sp * sp) / (2.0 * kPi));
        } else {
          const double decay = dz * std::sqrt(kap2 - k * k);
          const double mag = decay > 745.0 ? 0.0 : std::exp(-decay);
          const float2 ph = phasor(dz * (kap2 / (2.0 * k) - k) / (2.0 * kPi));
          v = make_float2(static_cast<float>(mag * ph.x), static_cast<float>(mag * ph.y));
        }
        as[d * qn + q] = v;
      }
    }
  }
  auto upload = [&](auto** dst, const void* src, size_t bytes) -> hipError_t {
    hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), bytes);
    if (e != hipSuccess) return e;
    return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
  };
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = upload(&pl->d_tw, tw.data(), tw.size() * sizeof(float2));
  if (e == hipSuccess) e = upload(&pl->d_row, row.data(), row.size() * sizeof(float2));
  if (e == hipSuccess) e = upload(&pl->d_col, col.data(), col.size() * sizeof(float2));
  if (e == hipSuccess && !as.empty()) e = upload(&pl->d_as, as.data(), as.size() * sizeof(float2));
  if (e == hipSuccess) e = upload(&pl->d_sh_phasor, shp.data(), shp.size() * sizeof(float2));
  if (e == hipSuccess) e = upload(&pl->d_sh_amp, sh_amp.data(), sh_amp.size() * sizeof(float));
  std::vector<float> amp_rad = pl->amp_rad;
  if (amp_rad.empty()) amp_rad.push_back(0.0f);
  if (e == hipSuccess) e = upload(&pl->d_amp_rad, amp_rad.data(), amp_rad.size() * sizeof(float));
  if (e == hipSuccess && (flags & TURPY_CHECK_FINITE)) {
    e = hipMalloc(reinterpret_cast<void**>(&pl->d_nonfinite), sizeof(unsigned long long));
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&pl->h_nonfinite), sizeof(unsigned long long));
  }
  if (e != hipSuccess) {
    turpy_plan_destroy(pl);
    return hip_fail(e, "plan_create: table upload");
  }
  e = register_static_scratch(pl->device);
  if (e != hipSuccess) {
    turpy_plan_destroy(pl);
    return hip_fail(e, "plan_create: scratch address of turpy_propagate_static");
  }
  pl->arch = device_arch(pl->device);
  apply_cached_widths(pl);
  *out = pl;
  return TURPY_OK;
}

turpy_status turpy_plan_destroy(turpy_plan* pl) {
  if (!pl) return TURPY_OK;
  (void)hipFree(pl->d_tw);
  (void)hipFree(pl->d_row);
  (void)hipFree(pl->d_col);
  (void)hipFree(pl->d_as);
  (void)hipFree(pl->d_sh_phasor);
  (void)hipFree(pl->d_sh_amp);
  (void)hipFree(pl->d_amp_rad);
  (void)hipFree(pl->d_nonfinite);
  if (pl->h_nonfinite) (void)hipHostFree(pl->h_nonfinite);
  delete pl;
  return TURPY_OK;
}

turpy_status turpy_checkpoint_size(const turpy_plan* pl, size_t* bytes) {
  if (!pl || !bytes) return fail(TURPY_E_INVALID, "checkpoint_size: NULL argument");
  const size_t plane = static_cast<size_t>(pl->n) * pl->n * sizeof(float2);
  *bytes = static_cast<size_t>(pl->R) * pl->M * plane + (pl->screen_ck ? static_cast<size_t>(pl->M) * pl->P * plane : 0);
  return TURPY_OK;
}

turpy_status turpy_workspace_size(const turpy_plan* pl, int32_t op, size_t* bytes) {
  if (!pl || !bytes) return fail(TURPY_E_INVALID, "workspace_size: NULL argument");
  switch (op) {
    case TURPY_OP_SCREEN_GENERATE:
    case TURPY_OP_PROPAGATE: *bytes = pl->ws_forward(); return TURPY_OK;
    case TURPY_OP_PROPAGATE_BACKWARD: *bytes = pl->ws_backward(); return TURPY_OK;
    case TURPY_OP_EVOLVE: *bytes = 0; return TURPY_OK;
    case TURPY_OP_PROPAGATE_BACKWARD_REVERSIBLE: *bytes = pl->ws_reversible(); return TURPY_OK;
    case TURPY_OP_TUNE: *bytes = pl->ws_tune(); return TURPY_OK;
    default: return fail(TURPY_E_INVALID, "workspace_size: unknown op %d", op);
  }
}

}  // extern "C"

namespace {

// With TURPY_SCREEN_CHECKPOINTS and a checkpoint buffer, the screens' column
// halves live after the checkpointed fields: the forward pass writes them
// there and the adjoint reads them instead of synthesising them again.
void keep_screens(const turpy_plan* pl, void* checkpoints, int32_t src, Ws* w) {
  if (!pl->screen_ck || !checkpoints || src == TURPY_SCREENS_MATERIALIZED || pl->M == 0) return;
  const size_t plane = static_cast<size_t>(pl->n) * pl->n;
  w->screens = static_cast<float2*>(checkpoints) + static_cast<size_t>(pl->R) * pl->M * plane;
  w->screen_stride = static_cast<size_t>(pl->P) * plane;
}

turpy_status check_t(int64_t t) {
  if (t < 0 || t > 0xFFFFFFFFll) return fail(TURPY_E_INVALID, "time step t=%lld out of range", (long long)t);
  return TURPY_OK;
}

hipError_t enqueue_screen_col(const turpy_plan* pl, uint64_t seed, uint32_t t, int s, const float2* spectra,
                              const Ws& w, hipStream_t st, const EvolveStep* ev = nullptr) {
  const SynthArgs a = synth_args(pl, seed, t, s, spectra, w, ev);
  return timed("synth", st, [&] { return launch_synth(pl->n, a, st); });
}

// Column pass of distance `step` over all realizations; with synth_screen >= 0
// the column half of that screen's synthesis follows it into ws.scratch.
hipError_t enqueue_col(const turpy_plan* pl, int step, const float2* in, int64_t in_stride, float2* out,
                       bool adjoint, int synth_screen, uint64_t seed, uint32_t t, const float2* spectra,
                       const Ws& w, hipStream_t st, const EvolveStep* ev = nullptr) {
  const ColArgs c = col_args(pl, step, in, in_stride, out, pl->R, adjoint);
  TURPY_HIP_E(timed("col", st, [&] { return launch_col(pl->n, c, st); }));
  if (synth_screen >= 0) return enqueue_screen_col(pl, seed, t, synth_screen, spectra, w, st, ev);
  return hipSuccess;
}

// Fresh subharmonic coefficients of every pair and screen (revolutions) into ws.sh.
hipError_t enqueue_sh(const turpy_plan* pl, uint64_t seed, uint32_t t, const Ws& w, hipStream_t st) {
  const ShArgs a = sh_args(pl, seed, t, w.sh);
  return timed("sh", st, [&] { return launch_sh(a, st); });
}

turpy_status check_src(const turpy_plan* pl, int32_t src, const void* screens_or_spectra) {
  if (src != TURPY_SCREENS_SYNTH && src != TURPY_SCREENS_MATERIALIZED && src != TURPY_SCREENS_SPECTRA)
    return fail(TURPY_E_INVALID, "unknown screen source %d", src);
  if (src != TURPY_SCREENS_SYNTH && pl->M > 0 && !screens_or_spectra)
    return fail(TURPY_E_INVALID, "screen source %d needs a screens/spectra pointer", src);
  return TURPY_OK;
}

turpy_status check_device(const turpy_plan* pl) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != pl->device)
    return fail(TURPY_E_INVALID, "plan was created on device %d but device %d is current", pl->device, dev);
  return TURPY_OK;
}

constexpr int64_t kRecvChunks = 16;

// TURPY_CHECK_FINITE: its checks synchronise, so a checked call refuses a
// capturing stream before it enqueues anything.
turpy_status check_capture(const turpy_plan* pl, hipStream_t st, const char* where) {
  if (!pl->d_nonfinite) return TURPY_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  TURPY_HIP(hipStreamIsCapturing(st, &cs), where);
  if (cs != hipStreamCaptureStatusNone)
    return fail(TURPY_E_INVALID, "%s: a TURPY_CHECK_FINITE plan synchronises; not on a capturing stream", where);
  return TURPY_OK;
}

// One output of a call: `floats` FP32 words at p (complex values count two).
struct Output {
  const void* p;
  int64_t floats;
  const char* name;
};

// TURPY_CHECK_FINITE: count the NaN and infinite values of each output, wait
// for the count, and report the first output that has any.
turpy_status check_outputs(const turpy_plan* pl, hipStream_t st, const char* where, std::initializer_list<Output> outs) {
  if (!pl->d_nonfinite) return TURPY_OK;
  for (const Output& o : outs) {
    if (!o.p || o.floats <= 0) continue;
    TURPY_HIP(timed("nonfinite", st, [&] {
                return launch_nonfinite(static_cast<const float*>(o.p), o.floats, pl->d_nonfinite, st);
              }),
              where);
    TURPY_HIP(hipMemcpyAsync(pl->h_nonfinite, pl->d_nonfinite, sizeof(unsigned long long), hipMemcpyDeviceToHost, st),
              where);
    TURPY_HIP(hipStreamSynchronize(st), where);
    if (*pl->h_nonfinite)
      return fail(TURPY_E_NONFINITE, "%s: %llu non-finite values in %s", where, *pl->h_nonfinite, o.name);
  }
  return TURPY_OK;
}

turpy_status check_receiver_shape(int32_t n, int64_t batch) {
  if (!pow2(n)) return fail(TURPY_E_INVALID, "receiver: n=%d is not a power of two", n);
  if (n < 16 || n > 2048) return fail(TURPY_E_UNSUPPORTED, "receiver: n=%d outside 16..2048", n);
  if (batch < 1 || batch > (int64_t(1) << 31)) return fail(TURPY_E_INVALID, "receiver: batch out of range");
  return TURPY_OK;
}

size_t receiver_ws(int32_t n, int64_t batch) {
  const size_t plane = static_cast<size_t>(n) * n;
  const int64_t chunks = batch < kRecvChunks ? batch : kRecvChunks;
  return 2 * align_up(batch * plane * sizeof(float2)) + align_up(chunks * plane * sizeof(float));
}

// Process-wide FP64-generated twiddle tables per (device, N) for the plan-less
// receiver calls, built by turpy_receiver_setup (a set-up call: it allocates
// and uploads synchronously); the stream-ordered calls only look them up.
std::mutex g_tw_mutex;
std::map<std::pair<int, int>, float2*> g_tw_cache;

turpy_status twiddles_for(int n, const float2** out) {
  int dev = 0;
  TURPY_HIP(hipGetDevice(&dev), "twiddle table");
  std::lock_guard<std::mutex> lock(g_tw_mutex);
  auto it = g_tw_cache.find({dev, n});
  if (it == g_tw_cache.end())
    return fail(TURPY_E_INVALID, "receiver: no tables for n=%d on device %d (call turpy_receiver_setup first)", n,
                dev);
  *out = it->second;
  return TURPY_OK;
}

// The end of the adjoint for a source shared by every realization, on the
// one plane `sum` that already holds the gradients summed over realizations
// (row-spectral when `spectral`): the diffraction before screen 0 is the same
// linear map for every realization, so it runs once, on the sum (column pass
// with conj h_0, then the adjoint of the source row transform into grad_u_in).
// Without that diffraction the sum was written to grad_u_in directly.
turpy_status adjoint_shared_tail(const turpy_plan* pl, float2* sum, bool spectral, float2* grad_u_in, hipStream_t st) {
  if (!spectral) return TURPY_OK;
  const int64_t plane = static_cast<int64_t>(pl->n) * pl->n;
  const ColArgs c = col_args(pl, 0, sum, plane, sum, 1, true);
  TURPY_HIP(timed("col", st, [&] { return launch_col(pl->n, c, st); }), "propagate_backward: shared column pass");
  RowArgs a = base_row(pl);
  a.in = sum;
  a.in_stride = plane;
  a.out = grad_u_in;
  a.R = 1;
  a.in_spectral = 1;
  a.pre = pl->d_row;
  a.conj_tables = 1;
  TURPY_HIP(timed(row_family(a), st, [&] { return launch_row(pl->n, a, 1, st); }),
            "propagate_backward: shared last row pass");
  return TURPY_OK;
}

}  // namespace

extern "C" {

turpy_status turpy_screen_generate(turpy_plan* pl, uint64_t seed, int64_t t, float* screens, void* ws,
                                   size_t ws_bytes, void* stream) {
  if (!pl || !screens) return fail(TURPY_E_INVALID, "screen_generate: NULL argument");
  if (turpy_status st = check_t(t)) return st;
  if (turpy_status st = check_device(pl)) return st;
  if (pl->M == 0) return TURPY_OK;
  if (!ws || ws_bytes < pl->ws_forward())
    return fail(TURPY_E_WORKSPACE, "screen_generate: workspace %zu < %zu bytes", ws_bytes, pl->ws_forward());
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (turpy_status s_ = check_capture(pl, st, "screen_generate")) return s_;
  const Ws w = carve(pl, ws);
  if (pl->sh_levels > 0) TURPY_HIP(enqueue_sh(pl, seed, static_cast<uint32_t>(t), w, st), "screen_generate: sh");
  for (int s = 0; s < pl->M; ++s) {
    TURPY_HIP(enqueue_screen_col(pl, seed, static_cast<uint32_t>(t), s, nullptr, w, st), "screen_generate: col");
    RowArgs a = base_row(pl);
    screen_fields(pl, TURPY_SCREENS_SYNTH, nullptr, w, s, &a);
    a.screen_mode = ROW_SCRATCH;
    a.in = nullptr;  // no field: the row kernel only emits the phases
    a.phase_out = screens;
    TURPY_HIP(timed(row_family(a), st, [&] { return launch_row(pl->n, a, pl->P, st); }), "screen_generate: row");
  }
  return check_outputs(pl, st, "screen_generate",
                       {{screens, pl->R * pl->M * static_cast<int64_t>(pl->n) * pl->n, "screens"}});
}

}  // extern "C"

namespace {

// turpy_propagate; with `ev`, every screen's synthesis first takes the AR step
// of its stored spectra (turpy_evolve_propagate).
turpy_status propagate_impl(turpy_plan* pl, uint64_t seed, int64_t t, const void* u_in, int64_t u_in_stride,
                            int32_t src, const void* screens_or_spectra, void* u_out, void* checkpoints, void* ws,
                            size_t ws_bytes, void* stream, const EvolveStep* ev) {
  if (!pl || !u_in || !u_out) return fail(TURPY_E_INVALID, "propagate: NULL argument");
  if (turpy_status s_ = check_t(t)) return s_;
  if (turpy_status s_ = check_device(pl)) return s_;
  if (turpy_status s_ = check_src(pl, src, screens_or_spectra)) return s_;
  const int64_t plane = static_cast<int64_t>(pl->n) * pl->n;
  if (u_in_stride != 0 && u_in_stride != plane)
    return fail(TURPY_E_INVALID, "propagate: u_in_stride must be 0 or N*N");
  if (u_in_stride == 0 && u_in == u_out && pl->R > 1)
    return fail(TURPY_E_INVALID, "propagate: a shared source cannot alias u_out");
  if (!ws || ws_bytes < pl->ws_forward())
    return fail(TURPY_E_WORKSPACE, "propagate: workspace %zu < %zu bytes", ws_bytes, pl->ws_forward());
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (turpy_status s_ = check_capture(pl, st, "propagate")) return s_;
  Ws w = carve(pl, ws);
  keep_screens(pl, checkpoints, src, &w);
  const int n = pl->n, M = pl->M;
  const float inv_n = 1.0f / n;
  const float2* uin = static_cast<const float2*>(u_in);
  float2* uout = static_cast<float2*>(u_out);
  const float2* spectra = src == TURPY_SCREENS_SPECTRA ? static_cast<const float2*>(screens_or_spectra) : nullptr;

  if (src == TURPY_SCREENS_SYNTH && pl->sh_levels > 0 && M > 0)
    TURPY_HIP(enqueue_sh(pl, seed, static_cast<uint32_t>(t), w, st), "propagate: sh");

  const float2* cur = uin;
  int64_t cur_stride = u_in_stride;
  bool spectral = false;
  const bool synth = src != TURPY_SCREENS_MATERIALIZED;
  const uint32_t tt = static_cast<uint32_t>(t);
  bool scratch_ready = false;  // the scratch plane holds the next row pass's screen
  if (pl->dz[0] > 0) {
    // row transform of the source (x h_0(k1)), then the first column pass
    RowArgs a = base_row(pl);
    a.in = uin;
    a.in_stride = u_in_stride;
    a.out_spectral = 1;
    a.post = pl->d_row;
    float2* dst = uout;
    int64_t rows_r = pl->R;
    if (u_in_stride == 0) {
      dst = w.src;
      rows_r = 1;
    }
    a.out = dst;
    a.R = rows_r;
    TURPY_HIP(timed(row_family(a), st, [&] { return launch_row(n, a, (rows_r + 1) / 2, st); }),
              "propagate: source row transform");
    if (u_in_stride == 0) {
      // Shared source: the diffraction before the first screen is the same for
      // every realization, so it runs once, in place on the source plane, and
      // the first screen pass reads that plane for all of them.
      const ColArgs c = col_args(pl, 0, w.src, 0, w.src, 1, false);
      TURPY_HIP(timed("col", st, [&] { return launch_col(n, c, st); }), "propagate: column pass 0");
      cur = w.src;
      cur_stride = 0;
    } else {
      const int syn = synth && M > 0 ? 0 : -1;
      TURPY_HIP(enqueue_col(pl, 0, dst, plane, uout, false, syn, seed, tt, spectra, w, st, ev),
                "propagate: column pass 0");
      scratch_ready = syn >= 0;
      cur = uout;
      cur_stride = plane;
    }
    spectral = true;
  }
  for (int s = 0; s < M; ++s) {
    if (synth && !scratch_ready)
      TURPY_HIP(enqueue_screen_col(pl, seed, tt, s, spectra, w, st, ev), "propagate: screen col");
    const bool out_spec = pl->dz[s + 1] > 0;
    RowArgs a = base_row(pl);
    a.in = cur;
    a.in_stride = cur_stride;
    a.out = uout;
    a.in_spectral = spectral ? 1 : 0;
    a.out_spectral = out_spec ? 1 : 0;
    a.post = out_spec ? pl->d_row + static_cast<size_t>(s + 1) * n : nullptr;
    a.scale = spectral ? inv_n : 1.0f;
    screen_fields(pl, src, screens_or_spectra, w, s, &a);
    a.ckpt_out = static_cast<float2*>(checkpoints);
    TURPY_HIP(timed(row_family(a), st, [&] { return launch_row(n, a, pl->P, st); }), "propagate: row pass");
    cur = uout;
    cur_stride = plane;
    spectral = out_spec;
    scratch_ready = false;
    if (out_spec) {
      const int syn = synth && s + 1 < M ? s + 1 : -1;
      TURPY_HIP(enqueue_col(pl, s + 1, uout, plane, uout, false, syn, seed, tt, spectra, w, st, ev),
                "propagate: column pass");
      scratch_ready = syn >= 0;
    }
  }
  if (spectral) {
    RowArgs a = base_row(pl);
    a.in = cur;  // the shared source plane when there are no screens
    a.in_stride = cur_stride;
    a.out = uout;
    a.in_spectral = 1;
    a.scale = inv_n;
    if (pl->d_moments)
      TURPY_HIP(timed("row_moments", st, [&] { return launch_row_moments(n, a, pl->d_moments, st); }),
                "propagate: final row pass with moments");
    else
      TURPY_HIP(timed(row_family(a), st, [&] { return launch_row(n, a, pl->P, st); }), "propagate: final row pass");
  } else {
    if (M == 0)
      TURPY_HIP(timed("copy", st, [&] { return launch_copy(uin, u_in_stride, uout, plane, pl->R, st); }),
                "propagate: copy");
    if (pl->d_moments) {
      // the output comes from a screen row pass or a copy: the sums read it back
      StatsArgs a{};
      a.u = uout;
      a.batch = pl->R;
      a.n = n;
      a.moments = pl->d_moments;
      TURPY_HIP(timed("stats", st, [&] { return launch_stats(a, st); }), "propagate: moments");
    }
  }
  const int64_t fields = 2 * pl->R * plane;
  return check_outputs(pl, st, "propagate",
                       {{u_out, fields, "u_out"},
                        {checkpoints, fields * M, "checkpoints"},
                        {ev ? screens_or_spectra : nullptr, 2 * pl->P * M * plane, "the AR state"},
                        {pl->d_moments, 4 * plane, "the bound moments"}});
}

}  // namespace

extern "C" {

turpy_status turpy_propagate(turpy_plan* pl, uint64_t seed, int64_t t, const void* u_in, int64_t u_in_stride,
                             int32_t src, const void* screens_or_spectra, void* u_out, void* checkpoints, void* ws,
                             size_t ws_bytes, void* stream) {
  return propagate_impl(pl, seed, t, u_in, u_in_stride, src, screens_or_spectra, u_out, checkpoints, ws, ws_bytes,
                        stream, nullptr);
}

turpy_status turpy_evolve_propagate(turpy_plan* pl, uint64_t seed, int64_t t, double alpha, double shift_x,
                                    double shift_y, void* state, const void* u_in, int64_t u_in_stride, void* u_out,
                                    void* checkpoints, void* ws, size_t ws_bytes, void* stream) {
  if (!pl || !state) return fail(TURPY_E_INVALID, "evolve_propagate: NULL argument");
  if (turpy_status s_ = check_t(t)) return s_;
  if (t < 1) return fail(TURPY_E_INVALID, "evolve_propagate: t must be >= 1 (t = 0 initialises with turpy_evolve)");
  if (!(alpha >= 0.0 && alpha <= 1.0)) return fail(TURPY_E_INVALID, "evolve_propagate: alpha must be in [0, 1]");
  if (!std::isfinite(shift_x) || !std::isfinite(shift_y))
    return fail(TURPY_E_INVALID, "evolve_propagate: non-finite shift");
  if (turpy_status s_ = check_device(pl)) return s_;
  if (!u_in || !u_out) return fail(TURPY_E_INVALID, "evolve_propagate: NULL argument");
  if (!ws || ws_bytes < pl->ws_forward())
    return fail(TURPY_E_WORKSPACE, "evolve_propagate: workspace %zu < %zu bytes", ws_bytes, pl->ws_forward());
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (turpy_status s_ = check_capture(pl, st, "evolve_propagate")) return s_;
  if (pl->sh_levels > 0 && pl->M > 0) {
    // the subharmonic coefficients: the same translation and blend at their frequencies
    ShArgs b = sh_args(pl, seed, static_cast<uint32_t>(t), state_sh(pl, state));
    b.scale = static_cast<float>(2.0 * kPi);
    b.ar = 1;
    b.tag = TAG_AR_SH;
    b.alpha = alpha;
    b.sx = shift_x;
    b.sy = shift_y;
    TURPY_HIP(timed("sh", st, [&] { return launch_sh(b, st); }), "evolve_propagate: subharmonics");
  }
  const EvolveStep ev{alpha, shift_x, shift_y};
  return propagate_impl(pl, seed, t, u_in, u_in_stride, TURPY_SCREENS_SPECTRA, state, u_out, checkpoints, ws,
                        ws_bytes, stream, pl->M > 0 ? &ev : nullptr);
}

turpy_status turpy_propagate_static(turpy_plan* pl, uint64_t seed, int64_t t, const void* u_in,
                                    int64_t u_in_stride, int32_t src, const void* screens_or_spectra, void* u_out,
                                    void* checkpoints, void* stream) {
  if (!pl) return fail(TURPY_E_INVALID, "propagate_static: NULL plan");
  if (turpy_status s_ = check_device(pl)) return s_;
  const size_t need = pl->ws_forward();
  if (need > kStaticScratchBytes)
    return fail(TURPY_E_WORKSPACE,
                "propagate_static: the plan needs %zu bytes of scratch, beyond the %zu of the static array "
                "(use turpy_propagate with a workspace)", need, kStaticScratchBytes);
  void* ptr = static_scratch(pl->device);
  if (!ptr) return fail(TURPY_E_INVALID, "propagate_static: no scratch address for device %d", pl->device);
  return turpy_propagate(pl, seed, t, u_in, u_in_stride, src, screens_or_spectra, u_out, checkpoints, ptr,
                         kStaticScratchBytes, stream);
}

static turpy_status backward_checkpointed(turpy_plan* pl, uint64_t seed, int64_t t, const void* grad_u_out,
                                          const void* checkpoints, int32_t src, const void* screens_or_spectra,
                                          void* grad_u_in, int64_t grad_u_in_stride, float* grad_screens, void* ws,
                                          size_t ws_bytes, void* stream) {
  if (!pl || !grad_u_out) return fail(TURPY_E_INVALID, "propagate_backward: NULL argument");
  if (turpy_status s_ = check_t(t)) return s_;
  if (turpy_status s_ = check_device(pl)) return s_;
  if (turpy_status s_ = check_src(pl, src, screens_or_spectra)) return s_;
  const int n = pl->n, M = pl->M;
  const int64_t plane = static_cast<int64_t>(n) * n;
  if (grad_u_in_stride != 0 && grad_u_in_stride != plane)
    return fail(TURPY_E_INVALID, "propagate_backward: grad_u_in_stride must be 0 or N*N");
  if (M > 0 && !checkpoints) return fail(TURPY_E_INVALID, "propagate_backward: checkpoints are required");
  if (!ws || ws_bytes < pl->ws_backward())
    return fail(TURPY_E_WORKSPACE, "propagate_backward: workspace %zu < %zu bytes", ws_bytes, pl->ws_backward());
  hipStream_t st = static_cast<hipStream_t>(stream);
  Ws w = carve(pl, ws);
  keep_screens(pl, const_cast<void*>(checkpoints), src, &w);
  const bool stored = w.screens != nullptr;  // the forward pass kept the screens' column halves
  const float inv_n = 1.0f / n;
  // a shared source receives the sum over realizations: the realizations'
  // gradients are carried in the workspace up to screen 0 and summed there
  const bool shared = grad_u_in && grad_u_in_stride == 0;
  float2* g = grad_u_in && !shared ? static_cast<float2*>(grad_u_in) : w.gbuf;
  const float2* gout = static_cast<const float2*>(grad_u_out);
  const float2* spectra = src == TURPY_SCREENS_SPECTRA ? static_cast<const float2*>(screens_or_spectra) : nullptr;

  if (shared && M == 0) {
    // no screen: the sum of the output gradients goes through the one diffraction
    float2* dst = pl->dz[0] > 0 ? w.src : static_cast<float2*>(grad_u_in);
    TURPY_HIP(timed("sum", st, [&] { return launch_sum_planes(gout, pl->R, plane, dst, st); }),
              "propagate_backward: sum over realizations");
    if (pl->dz[0] > 0) {
      RowArgs a = base_row(pl);  // adjoint of the final (1/N) inverse row transform
      a.in = w.src;
      a.in_stride = plane;
      a.out = w.src;
      a.R = 1;
      a.out_spectral = 1;
      a.scale = inv_n;
      TURPY_HIP(timed(row_family(a), st, [&] { return launch_row(n, a, 1, st); }),
                "propagate_backward: first row pass");
    }
    return adjoint_shared_tail(pl, w.src, pl->dz[0] > 0, static_cast<float2*>(grad_u_in), st);
  }

  if (src == TURPY_SCREENS_SYNTH && pl->sh_levels > 0 && M > 0)
    TURPY_HIP(enqueue_sh(pl, seed, static_cast<uint32_t>(t), w, st), "propagate_backward: sh");

  const float2* cur = gout;
  bool spectral = false;
  const bool synth = src != TURPY_SCREENS_MATERIALIZED && !stored;
  const uint32_t tt = static_cast<uint32_t>(t);
  bool scratch_ready = false;
  if (pl->dz[M] > 0) {
    RowArgs a = base_row(pl);  // adjoint of the final (1/N) inverse row transform
    a.in = gout;
    a.in_stride = plane;
    a.out = g;
    a.out_spectral = 1;
    a.scale = inv_n;
    TURPY_HIP(timed(row_family(a), st, [&] { return launch_row(n, a, pl->P, st); }),
              "propagate_backward: first row pass");
    const int syn = synth && M > 0 ? M - 1 : -1;
    TURPY_HIP(enqueue_col(pl, M, g, plane, g, true, syn, seed, tt, spectra, w, st),
              "propagate_backward: column pass");
    scratch_ready = syn >= 0;
    cur = g;
    spectral = true;
  }
  for (int s = M - 1; s >= 0; --s) {
    if (synth && !scratch_ready)
      TURPY_HIP(enqueue_screen_col(pl, seed, tt, s, spectra, w, st), "propagate_backward: screen col");
    const bool out_spec = pl->dz[s] > 0;
    RowArgs a = base_row(pl);
    a.in = cur;
    a.in_stride = plane;
    a.out = g;
    a.in_spectral = spectral ? 1 : 0;
    a.pre = spectral ? pl->d_row + static_cast<size_t>(s + 1) * n : nullptr;
    a.conj_tables = 1;
    a.out_spectral = out_spec ? 1 : 0;
    a.scale = out_spec ? inv_n : 1.0f;
    screen_fields(pl, src, screens_or_spectra, w, s, &a);
    a.backward = 1;
    a.waves = pl->row_waves_bwd;
    a.ckpt_in = static_cast<const float2*>(checkpoints);
    a.grad_screens = grad_screens;
    TURPY_HIP(timed(row_family(a), st, [&] { return launch_row(n, a, pl->P, st); }),
              "propagate_backward: row pass");
    cur = g;
    spectral = out_spec;
    scratch_ready = false;
    if (s == 0 && shared) {
      float2* dst = spectral ? w.src : static_cast<float2*>(grad_u_in);
      TURPY_HIP(timed("sum", st, [&] { return launch_sum_planes(g, pl->R, plane, dst, st); }),
                "propagate_backward: sum over realizations");
      return adjoint_shared_tail(pl, w.src, spectral, static_cast<float2*>(grad_u_in), st);
    }
    if (out_spec) {
      const int syn = synth && s > 0 ? s - 1 : -1;
      TURPY_HIP(enqueue_col(pl, s, g, plane, g, true, syn, seed, tt, spectra, w, st),
                "propagate_backward: column pass");
      scratch_ready = syn >= 0;
    }
  }
  if (spectral) {
    RowArgs a = base_row(pl);  // adjoint of the source row transform: conj h_0, unnormalised inverse
    a.in = g;
    a.in_stride = plane;
    a.out = g;
    a.in_spectral = 1;
    a.pre = pl->d_row;
    a.conj_tables = 1;
    TURPY_HIP(timed(row_family(a), st, [&] { return launch_row(n, a, pl->P, st); }), "propagate_backward: last row pass");
  } else if (M == 0) {
    TURPY_HIP(timed("copy", st, [&] { return launch_copy(gout, plane, g, plane, pl->R, st); }), "propagate_backward: copy");
  }
  return TURPY_OK;
}

static turpy_status backward_reversible(turpy_plan* pl, uint64_t seed, int64_t t, const void* grad_u_out,
                                        const void* u_out, int32_t src, const void* screens_or_spectra,
                                        void* grad_u_in, int64_t grad_u_in_stride, float* grad_screens, void* ws,
                                        size_t ws_bytes, void* stream) {
  if (!pl || !grad_u_out) return fail(TURPY_E_INVALID, "propagate_backward_reversible: NULL argument");
  if (turpy_status s_ = check_t(t)) return s_;
  if (turpy_status s_ = check_device(pl)) return s_;
  if (turpy_status s_ = check_src(pl, src, screens_or_spectra)) return s_;
  const int n = pl->n, M = pl->M;
  const int64_t plane = static_cast<int64_t>(n) * n;
  if (grad_u_in_stride != 0 && grad_u_in_stride != plane)
    return fail(TURPY_E_INVALID, "propagate_backward_reversible: grad_u_in_stride must be 0 or N*N");
  if (M == 0)  // nothing to rebuild: the plain adjoint needs no checkpoints
    return turpy_propagate_backward(pl, seed, t, grad_u_out, nullptr, src, screens_or_spectra, grad_u_in,
                                    grad_u_in_stride, grad_screens, ws, ws_bytes, stream);
  if (pl->d_as)
    // evanescent bins (|H| < 1): the conjugate step damps them again instead
    // of undoing the forward step, so the fields cannot be rebuilt
    return fail(TURPY_E_UNSUPPORTED,
                "propagate_backward_reversible: the angular-spectrum transfer function of this grid has evanescent "
                "bins, so the path is not unitary; use turpy_propagate_backward with checkpoints");
  if (!u_out) return fail(TURPY_E_INVALID, "propagate_backward_reversible: u_out is required");
  if (!ws || ws_bytes < pl->ws_reversible())
    return fail(TURPY_E_WORKSPACE, "propagate_backward_reversible: workspace %zu < %zu bytes", ws_bytes,
                pl->ws_reversible());
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Ws w = carve(pl, ws);
  const float inv_n = 1.0f / n;
  const bool shared = grad_u_in && grad_u_in_stride == 0;
  float2* g = grad_u_in && !shared ? static_cast<float2*>(grad_u_in) : w.gbuf;
  float2* ub = reinterpret_cast<float2*>(static_cast<char*>(ws) + pl->off_ubuf());
  float2* wb = ub + static_cast<size_t>(pl->R) * plane;
  const float2* gout = static_cast<const float2*>(grad_u_out);
  const float2* uo = static_cast<const float2*>(u_out);
  const float2* spectra = src == TURPY_SCREENS_SPECTRA ? static_cast<const float2*>(screens_or_spectra) : nullptr;
  const bool synth = src != TURPY_SCREENS_MATERIALIZED;
  const uint32_t tt = static_cast<uint32_t>(t);

  if (src == TURPY_SCREENS_SYNTH && pl->sh_levels > 0)
    TURPY_HIP(enqueue_sh(pl, seed, tt, w, st), "propagate_backward_reversible: sh");

  // The adjoint chain applied to u_out runs the forward chain backwards (each
  // step is unitary): right before exp(-i phi_s) of screen s it holds the
  // forward field after screen s, which the gradient of that screen needs.
  const float2* gc = gout;
  const float2* uc = uo;
  bool spectral = false;
  if (pl->dz[M] > 0) {
    for (int chain = 0; chain < 2; ++chain) {
      RowArgs a = base_row(pl);  // adjoint of the final (1/N) inverse row transform
      a.in = chain == 0 ? gout : uo;
      a.in_stride = plane;
      a.out = chain == 0 ? g : ub;
      a.out_spectral = 1;
      a.scale = inv_n;
      TURPY_HIP(timed(row_family(a), st, [&] { return launch_row(n, a, pl->P, st); }),
                "propagate_backward_reversible: first row pass");
      TURPY_HIP(enqueue_col(pl, M, a.out, plane, a.out, true, -1, seed, tt, spectra, w, st),
                "propagate_backward_reversible: column pass");
    }
    gc = g;
    uc = ub;
    spectral = true;
  }
  for (int s = M - 1; s >= 0; --s) {
    if (synth) TURPY_HIP(enqueue_screen_col(pl, seed, tt, s, spectra, w, st), "propagate_backward_reversible: screen");
    const bool out_spec = pl->dz[s] > 0;
    for (int chain = 1; chain >= 0; --chain) {  // the field first, then the gradient that reads it
      RowArgs a = base_row(pl);
      a.in = chain == 0 ? gc : uc;
      a.in_stride = plane;
      a.out = chain == 0 ? g : ub;
      a.in_spectral = spectral ? 1 : 0;
      a.pre = spectral ? pl->d_row + static_cast<size_t>(s + 1) * n : nullptr;
      a.conj_tables = 1;
      // the field's own continuation past screen 0 is never read
      const bool cont = out_spec && (chain == 0 || s > 0);
      a.out_spectral = cont ? 1 : 0;
      a.scale = cont ? inv_n : 1.0f;
      screen_fields(pl, src, screens_or_spectra, w, s, &a);
      a.backward = 1;
      a.waves = pl->row_waves_bwd;
    a.waves = pl->row_waves_bwd;
      a.ckpt_single = 1;
      if (chain == 1) {
        a.ckpt_out = wb;
      } else {
        a.ckpt_in = wb;
        a.grad_screens = grad_screens;
      }
      TURPY_HIP(timed(row_family(a), st, [&] { return launch_row(n, a, pl->P, st); }),
                "propagate_backward_reversible: row pass");
      if (chain == 0 && s == 0 && shared) {
        float2* dst = out_spec ? w.src : static_cast<float2*>(grad_u_in);
        TURPY_HIP(timed("sum", st, [&] { return launch_sum_planes(g, pl->R, plane, dst, st); }),
                  "propagate_backward_reversible: sum over realizations");
        return adjoint_shared_tail(pl, w.src, out_spec, static_cast<float2*>(grad_u_in), st);
      }
      if (cont)
        TURPY_HIP(enqueue_col(pl, s, a.out, plane, a.out, true, -1, seed, tt, spectra, w, st),
                  "propagate_backward_reversible: column pass");
    }
    gc = g;
    uc = ub;
    spectral = out_spec;
  }
  if (spectral) {
    RowArgs a = base_row(pl);  // adjoint of the source row transform: conj h_0, unnormalised inverse
    a.in = g;
    a.in_stride = plane;
    a.out = g;
    a.in_spectral = 1;
    a.pre = pl->d_row;
    a.conj_tables = 1;
    TURPY_HIP(timed(row_family(a), st, [&] { return launch_row(n, a, pl->P, st); }),
              "propagate_backward_reversible: last row pass");
  }
  return TURPY_OK;
}

// TURPY_CHECK_FINITE around an adjoint: no capturing stream, then the
// gradients checked.
extern "C++" template <class Body>
static turpy_status checked_backward(turpy_plan* pl, void* stream, const char* where, void* grad_u_in,
                                     int64_t grad_u_in_stride, float* grad_screens, Body&& body) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (pl)
    if (turpy_status s_ = check_capture(pl, st, where)) return s_;
  if (turpy_status s_ = body()) return s_;
  const int64_t plane = static_cast<int64_t>(pl->n) * pl->n;
  return check_outputs(pl, st, where,
                       {{grad_u_in, 2 * (grad_u_in_stride ? pl->R : 1) * plane, "grad_u_in"},
                        {grad_screens, pl->R * pl->M * plane, "grad_screens"}});
}

turpy_status turpy_propagate_backward(turpy_plan* pl, uint64_t seed, int64_t t, const void* grad_u_out,
                                      const void* checkpoints, int32_t src, const void* screens_or_spectra,
                                      void* grad_u_in, int64_t grad_u_in_stride, float* grad_screens, void* ws,
                                      size_t ws_bytes, void* stream) {
  return checked_backward(pl, stream, "propagate_backward", grad_u_in, grad_u_in_stride, grad_screens, [&] {
    return backward_checkpointed(pl, seed, t, grad_u_out, checkpoints, src, screens_or_spectra, grad_u_in,
                                 grad_u_in_stride, grad_screens, ws, ws_bytes, stream);
  });
}

turpy_status turpy_propagate_backward_reversible(turpy_plan* pl, uint64_t seed, int64_t t, const void* grad_u_out,
                                                 const void* u_out, int32_t src, const void* screens_or_spectra,
                                                 void* grad_u_in, int64_t grad_u_in_stride, float* grad_screens,
                                                 void* ws, size_t ws_bytes, void* stream) {
  return checked_backward(pl, stream, "propagate_backward_reversible", grad_u_in, grad_u_in_stride, grad_screens,
                          [&] {
                            return backward_reversible(pl, seed, t, grad_u_out, u_out, src, screens_or_spectra,
                                                       grad_u_in, grad_u_in_stride, grad_screens, ws, ws_bytes,
                                                       stream);
                          });
}

turpy_status turpy_evolve(turpy_plan* pl, uint64_t seed, int64_t t, double alpha, double shift_x, double shift_y,
                          void* spectra, void* ws, size_t ws_bytes, void* stream) {
  (void)ws;
  (void)ws_bytes;
  if (!pl || !spectra) return fail(TURPY_E_INVALID, "evolve: NULL argument");
  if (turpy_status s_ = check_t(t)) return s_;
  if (turpy_status s_ = check_device(pl)) return s_;
  if (!(alpha >= 0.0 && alpha <= 1.0)) return fail(TURPY_E_INVALID, "evolve: alpha must be in [0, 1]");
  if (!std::isfinite(shift_x) || !std::isfinite(shift_y)) return fail(TURPY_E_INVALID, "evolve: non-finite shift");
  if (pl->M == 0) return TURPY_OK;
  EvolveArgs a{};
  a.spectra = static_cast<float2*>(spectra);
  a.P = pl->P;
  a.M = pl->M;
  a.n = pl->n;
  key_of(seed, &a.key0, &a.key1);
  a.t = static_cast<uint32_t>(t);
  a.t_dev = pl->d_t;
  a.init = t == 0 ? 1 : 0;
  a.tag = t == 0 ? TAG_MAIN : TAG_AR;
  a.alpha_f = static_cast<float>(alpha);
  a.blend = static_cast<float>(std::sqrt(1.0 - alpha * alpha));
  a.log2n = 0;
  while ((1 << a.log2n) < pl->n) ++a.log2n;
  a.sx = shift_x;
  a.sy = shift_y;
  a.amp = pl->d_amp_rad;
  a.df2 = pl->df2;
  a.inner = pl->inner;
  a.f02 = pl->f02;
  a.q = pl->qexp;
  hipStream_t st = static_cast<hipStream_t>(stream);
  TURPY_HIP(timed("evolve", st, [&] { return launch_evolve(a, st); }), "evolve");
  if (pl->sh_levels > 0) {
    // the subharmonic coefficients after the spectra: fresh at t = 0 (the
    // static ones), else the same translation and blend at their frequencies
    ShArgs b = sh_args(pl, seed, static_cast<uint32_t>(t), state_sh(pl, spectra));
    b.scale = static_cast<float>(2.0 * kPi);
    b.ar = t == 0 ? 0 : 1;
    b.tag = t == 0 ? TAG_SH : TAG_AR_SH;
    b.alpha = alpha;
    b.sx = shift_x;
    b.sy = shift_y;
    TURPY_HIP(timed("sh", st, [&] { return launch_sh(b, st); }), "evolve: subharmonics");
  }
  return TURPY_OK;
}

turpy_status turpy_noise(int32_t n, int64_t pairs, uint64_t seed, int64_t t, int32_t tag, int32_t screen, void* out,
                         void* stream) {
  if (!pow2(n) || n < 2 || n > 65536) return fail(TURPY_E_INVALID, "noise: n=%d is not a power of two in 2..65536", n);
  if (pairs < 0 || pairs > 0xFFFFFFFFll) return fail(TURPY_E_INVALID, "noise: pairs out of range");
  if (tag < 1 || tag > 15) return fail(TURPY_E_INVALID, "noise: tag must be in 1..15");
  if (screen < 0 || screen >= (1 << 28)) return fail(TURPY_E_INVALID, "noise: screen out of range");
  if (turpy_status st = check_t(t)) return st;
  if (pairs == 0) return TURPY_OK;
  if (!out) return fail(TURPY_E_INVALID, "noise: out is NULL");
  NoiseArgs a{};
  a.out = static_cast<float2*>(out);
  a.pairs = pairs;
  a.n = n;
  key_of(seed, &a.key0, &a.key1);
  a.t = static_cast<uint32_t>(t);
  a.tag = static_cast<uint32_t>(tag);
  a.screen = static_cast<uint32_t>(screen);
  hipStream_t st = static_cast<hipStream_t>(stream);
  TURPY_HIP(timed("noise", st, [&] { return launch_noise(a, st); }), "noise");
  return TURPY_OK;
}

turpy_status turpy_plan_bind_time(turpy_plan* pl, const void* dev_t) {
  if (!pl) return fail(TURPY_E_INVALID, "plan_bind_time: NULL plan");
  if (reinterpret_cast<uintptr_t>(dev_t) % 4 != 0) return fail(TURPY_E_INVALID, "plan_bind_time: misaligned");
  pl->d_t = static_cast<const uint32_t*>(dev_t);
  return TURPY_OK;
}

turpy_status turpy_plan_bind_moments(turpy_plan* pl, float* moments) {
  if (!pl) return fail(TURPY_E_INVALID, "plan_bind_moments: NULL plan");
  pl->d_moments = moments;
  return TURPY_OK;
}

turpy_status turpy_state_size(const turpy_plan* pl, size_t* bytes) {
  if (!pl || !bytes) return fail(TURPY_E_INVALID, "state_size: NULL argument");
  const size_t spectra = static_cast<size_t>(pl->P) * pl->M * pl->n * pl->n * sizeof(float2);
  *bytes = spectra + (pl->sh_levels > 0 ? static_cast<size_t>(pl->P) * pl->M * 32 * sizeof(float2) : 0);
  return TURPY_OK;
}

turpy_status turpy_stats(int32_t n, double dx, int64_t batch, const void* u, float* moments, int64_t count,
                         int32_t finalize, const float* weight, double power_fraction, float* si_map, double* summary,
                         void* stream) {
  if (n < 1 || n > 65536) return fail(TURPY_E_INVALID, "stats: n=%d out of range", n);
  if (!moments) return fail(TURPY_E_INVALID, "stats: moments is NULL");
  if (batch < 0) return fail(TURPY_E_INVALID, "stats: batch < 0");
  if (!(power_fraction >= 0.0 && power_fraction <= 1.0))
    return fail(TURPY_E_INVALID, "stats: power_fraction must be in [0, 1]");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (batch > 0) {
    if (!u) return fail(TURPY_E_INVALID, "stats: u is NULL");
    StatsArgs a{static_cast<const float2*>(u), batch, n, moments};
    TURPY_HIP(timed("stats", st, [&] { return launch_stats(a, st); }), "stats: accumulate");
  }
  if (finalize) {
    if (!summary) return fail(TURPY_E_INVALID, "stats: summary is NULL");
    if (count < 1) return fail(TURPY_E_INVALID, "stats: count must be >= 1 to finalize");
    if (!(dx > 0)) return fail(TURPY_E_INVALID, "stats: dx must be > 0");
    FinalizeArgs a{moments, n, dx, static_cast<double>(count), si_map, summary, weight, power_fraction};
    TURPY_HIP(timed("finalize", st, [&] { return launch_finalize(a, st); }), "stats: finalize");
  }
  return TURPY_OK;
}

turpy_status turpy_profile(int32_t enable) {
  g_prof.recycle();
  g_prof.on = enable != 0;
  return TURPY_OK;
}

turpy_status turpy_profile_only(const char* family) {
  g_prof.only = family ? family : "";
  return TURPY_OK;
}

turpy_status turpy_debug_fail_launch(int64_t k) {
  if (k < 0) return fail(TURPY_E_INVALID, "debug_fail_launch: k < 0");
  g_injected = false;
  g_fail_countdown.store(k);
  return TURPY_OK;
}

turpy_status turpy_profile_read(const char* family, int64_t* launches, double* total_ms) {
  if (!family || !launches || !total_ms) return fail(TURPY_E_INVALID, "profile_read: NULL argument");
  *launches = 0;
  *total_ms = 0.0;
  auto it = g_prof.live.find(family);
  if (it == g_prof.live.end()) return TURPY_OK;
  for (auto& e : it->second) {
    TURPY_HIP(hipEventSynchronize(e.stop), "profile_read");
    float ms = 0.0f;
    TURPY_HIP(hipEventElapsedTime(&ms, e.start, e.stop), "profile_read");
    *total_ms += ms;
    ++*launches;
  }
  return TURPY_OK;
}

turpy_status turpy_receiver_setup(int32_t n) {
  if (turpy_status st = check_receiver_shape(n, 1)) return st;
  int dev = 0;
  TURPY_HIP(hipGetDevice(&dev), "receiver_setup");
  std::lock_guard<std::mutex> lock(g_tw_mutex);
  if (g_tw_cache.count({dev, n})) return TURPY_OK;
  std::vector<float2> tw(n);
  for (int i = 0; i < n; ++i) tw[i] = phasor(-static_cast<double>(i) / n);
  float2* d = nullptr;
  TURPY_HIP(hipMalloc(&d, n * sizeof(float2)), "receiver_setup: twiddle table");
  const hipError_t e = hipMemcpy(d, tw.data(), n * sizeof(float2), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return hip_fail(e, "receiver_setup: twiddle table");
  }
  g_tw_cache[{dev, n}] = d;
  return TURPY_OK;
}

turpy_status turpy_receiver_workspace_size(int32_t n, int64_t batch, size_t* bytes) {
  if (!bytes) return fail(TURPY_E_INVALID, "receiver_workspace_size: NULL argument");
  if (turpy_status st = check_receiver_shape(n, batch)) return st;
  *bytes = receiver_ws(n, batch);
  return TURPY_OK;
}

turpy_status turpy_receiver(int32_t n, double dx, double aperture_diameter, int64_t batch, const void* u,
                            const float* theta1, const float* theta2, void* u_out, void* ws, size_t ws_bytes,
                            void* stream) {
  (void)ws;
  (void)ws_bytes;
  if (turpy_status st = check_receiver_shape(n, batch)) return st;
  if (!u || !theta1 || !theta2 || !u_out) return fail(TURPY_E_INVALID, "receiver: NULL argument");
  if (!(dx > 0) || !(aperture_diameter > 0)) return fail(TURPY_E_INVALID, "receiver: dx and diameter must be > 0");
  if (u == u_out) return fail(TURPY_E_INVALID, "receiver: u and u_out must not alias");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const float2* tw = nullptr;
  if (turpy_status e = twiddles_for(n, &tw)) return e;
  RecvArgs a{};
  a.tw = tw;
  a.n = n;
  a.batch = batch;
  a.dx = dx;
  a.radius2 = 0.25 * aperture_diameter * aperture_diameter;
  a.theta1 = theta1;
  a.theta2 = theta2;
  a.u = static_cast<const float2*>(u);
  a.out = static_cast<float2*>(u_out);
  TURPY_HIP(timed("recv_row", st, [&] { return launch_recv_row_in(a, st); }), "receiver: row pass");
  a.in = a.out;
  TURPY_HIP(timed("recv_col", st, [&] { return launch_recv_col(a, st); }), "receiver: column pass");
  RowArgs r{};
  r.tw = tw;
  r.in = a.out;
  r.in_stride = static_cast<int64_t>(n) * n;
  r.out = a.out;
  r.R = batch;
  r.in_spectral = 1;
  r.scale = 1.0f / n;
  TURPY_HIP(timed("row_plain", st, [&] { return launch_row(n, r, (batch + 1) / 2, st); }), "receiver: last row pass");
  return TURPY_OK;
}

turpy_status turpy_receiver_backward(int32_t n, double dx, double aperture_diameter, int64_t batch, const void* u,
                                     const float* theta1, const float* theta2, const void* grad_out, void* grad_u,
                                     float* grad_theta1, float* grad_theta2, void* ws, size_t ws_bytes,
                                     void* stream) {
  if (turpy_status st = check_receiver_shape(n, batch)) return st;
  if (!u || !theta1 || !theta2 || !grad_out) return fail(TURPY_E_INVALID, "receiver_backward: NULL argument");
  if (!(dx > 0) || !(aperture_diameter > 0))
    return fail(TURPY_E_INVALID, "receiver_backward: dx and diameter must be > 0");
  const size_t need = receiver_ws(n, batch);
  if (!ws || ws_bytes < need)
    return fail(TURPY_E_WORKSPACE, "receiver_backward: workspace %zu < %zu bytes", ws_bytes, need);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const float2* tw = nullptr;
  if (turpy_status e = twiddles_for(n, &tw)) return e;
  const size_t plane = static_cast<size_t>(n) * n;
  char* base = static_cast<char*>(ws);
  float2* gbuf = reinterpret_cast<float2*>(base);
  float2* xbuf = reinterpret_cast<float2*>(base + align_up(batch * plane * sizeof(float2)));
  float* part = reinterpret_cast<float*>(base + 2 * align_up(batch * plane * sizeof(float2)));
  // G = row FFT of grad_out
  RowArgs r{};
  r.tw = tw;
  r.in = static_cast<const float2*>(grad_out);
  r.in_stride = static_cast<int64_t>(plane);
  r.out = gbuf;
  r.R = batch;
  r.out_spectral = 1;
  r.scale = 1.0f;
  TURPY_HIP(timed("row_plain", st, [&] { return launch_row(n, r, (batch + 1) / 2, st); }),
            "receiver_backward: row FFT of the gradient");
  RecvArgs a{};
  a.tw = tw;
  a.n = n;
  a.batch = batch;
  a.dx = dx;
  a.radius2 = 0.25 * aperture_diameter * aperture_diameter;
  a.theta1 = theta1;
  a.theta2 = theta2;
  a.u = static_cast<const float2*>(u);
  a.out = xbuf;
  a.chunks = static_cast<int>(batch < kRecvChunks ? batch : kRecvChunks);
  a.partial = part;
  TURPY_HIP(timed("recv_row", st, [&] { return launch_recv_row_in(a, st); }), "receiver_backward: U1 row FFT");
  a.in = xbuf;
  a.in2 = gbuf;
  a.out = gbuf;
  TURPY_HIP(timed("recv_col_grad", st, [&] { return launch_recv_col_grad(a, st); }),
            "receiver_backward: column pass");
  if (grad_theta2)
    TURPY_HIP(timed("recv_reduce", st, [&] { return launch_recv_reduce(a, grad_theta2, 1, st); }),
              "receiver_backward: theta2 reduce");
  a.in = gbuf;
  a.out = static_cast<float2*>(grad_u);
  TURPY_HIP(timed("recv_row_grad", st, [&] { return launch_recv_row_grad(a, st); }), "receiver_backward: row pass");
  if (grad_theta1)
    TURPY_HIP(timed("recv_reduce", st, [&] { return launch_recv_reduce(a, grad_theta1, 0, st); }),
              "receiver_backward: theta1 reduce");
  return TURPY_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Launch-configuration tuning and its process-wide cache.
// ---------------------------------------------------------------------------
namespace {

constexpr int kWidths[3] = {4, 8, 16};

// Second-pass radices built per grid size for the column pass and the
// synthesis (0 = the default plan, min(16, N/16)).
bool radix_built_rt(int n, int r) {
  return r == 0 || ((n == 512 || n == 1024) && (r == 8 || r == 4)) || (n == 2048 && r == 8);
}
// Occupancy hints built for the screen row passes.
bool waves_built_rt(int n, int w) { return w == 3 || (n >= 256 && (w == 2 || w == 4)); }

bool is_row_kernel(int k) { return k == TURPY_TUNE_ROW_FWD || k == TURPY_TUNE_ROW_BWD; }

struct TuneKey {
  std::string arch;
  int kernel, n, batch_class;
  bool operator<(const TuneKey& o) const {
    if (arch != o.arch) return arch < o.arch;
    if (kernel != o.kernel) return kernel < o.kernel;
    if (n != o.n) return n < o.n;
    return batch_class < o.batch_class;
  }
};

std::mutex g_tune_mu;
std::map<TuneKey, turpy_tune_entry> g_tune;

int bit_length(int64_t v) {
  int b = 0;
  for (; v > 0; v >>= 1) ++b;
  return b;
}

std::string device_arch(int device) {
  static std::mutex mu;
  static std::map<int, std::string> known;
  std::lock_guard<std::mutex> lock(mu);
  auto it = known.find(device);
  if (it != known.end()) return it->second;
  hipDeviceProp_t prop;
  std::string a = "unknown";
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
    a = prop.gcnArchName;
    const size_t colon = a.find(':');
    if (colon != std::string::npos) a.resize(colon);
  }
  known[device] = a;
  return a;
}

int col_kernel_id(const turpy_plan* pl) {
  if (pl->tf_kind != TURPY_TF_ANGULAR_SPECTRUM) return TURPY_TUNE_COL_FRESNEL;
  return pl->d_as ? TURPY_TUNE_COL_AS_TABLE : TURPY_TUNE_COL_ANGULAR;
}

TuneKey col_key(const turpy_plan* pl) { return TuneKey{pl->arch, col_kernel_id(pl), pl->n, bit_length(pl->R)}; }
TuneKey synth_key(const turpy_plan* pl) { return TuneKey{pl->arch, TURPY_TUNE_SYNTH, pl->n, bit_length(pl->P)}; }
TuneKey row_key(const turpy_plan* pl, int kernel) { return TuneKey{pl->arch, kernel, pl->n, bit_length(pl->P)}; }
TuneKey ar_key(const turpy_plan* pl) { return TuneKey{pl->arch, TURPY_TUNE_SYNTH_AR, pl->n, bit_length(pl->P)}; }

bool cached(const TuneKey& k, turpy_tune_entry* e) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_tune.find(k);
  if (it == g_tune.end()) return false;
  *e = it->second;
  return true;
}

void store(const turpy_tune_entry& e) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune[TuneKey{std::string(e.arch), e.kernel, e.n, e.batch_class}] = e;
}

// Apply the cached choices for every key of the plan.
void apply_cached_widths(turpy_plan* pl) {
  turpy_tune_entry e{};
  if (cached(col_key(pl), &e)) {
    pl->col_width = e.width;
    pl->col_radix = e.radix;
  }
  if (cached(synth_key(pl), &e)) {
    pl->synth_width = e.width;
    pl->synth_radix = e.radix;
  }
  if (cached(ar_key(pl), &e)) {
    pl->ar_width = e.width;
    pl->ar_radix = e.radix;
  }
  if (cached(row_key(pl, TURPY_TUNE_ROW_FWD), &e)) pl->row_waves = e.waves;
  if (cached(row_key(pl, TURPY_TUNE_ROW_BWD), &e)) pl->row_waves_bwd = e.waves;
}

struct LaunchChoice {
  int width, radix, waves;
};

// Microseconds per launch of `launch(choice)` for every choice: one launch,
// then three loops of about 2 ms, minimum per launch.
template <class Launch>
turpy_status time_choices(const std::vector<LaunchChoice>& choices, hipStream_t st, std::vector<float>* us,
                          Launch&& launch) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  us->assign(choices.size(), 0.0f);
  for (size_t i = 0; e == hipSuccess && i < choices.size(); ++i) {
    float ms = 0.0f;
    e = hipEventRecord(e0, st);
    if (e == hipSuccess) e = launch(choices[i]);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    const int reps = std::min(50, std::max(2, static_cast<int>(2.0f / std::max(ms, 1e-3f))));
    float best = 0.0f;
    for (int rep = 0; e == hipSuccess && rep < 3; ++rep) {
      e = hipEventRecord(e0, st);
      for (int k = 0; e == hipSuccess && k < reps; ++k) e = launch(choices[i]);
      if (e == hipSuccess) e = hipEventRecord(e1, st);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      const float per = 1000.0f * ms / reps;
      if (e == hipSuccess && (rep == 0 || per < best)) best = per;
    }
    (*us)[i] = best;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return e == hipSuccess ? TURPY_OK : hip_fail(e, "plan_tune: timed launch");
}

// Measure `choices`, keep the fastest under `key`; `dflt` is the built-in
// choice (its time is kept beside the winner's).
template <class Launch>
turpy_status tune_key(const TuneKey& key, const std::vector<LaunchChoice>& choices, const LaunchChoice& dflt,
                      hipStream_t st, Launch&& launch) {
  std::vector<float> us;
  if (turpy_status s = time_choices(choices, st, &us, launch)) return s;
  size_t best = 0;
  float us_default = 0.0f;
  for (size_t i = 0; i < choices.size(); ++i) {
    if (us[i] < us[best]) best = i;
    const LaunchChoice& c = choices[i];
    if (c.width == dflt.width && c.radix == dflt.radix && c.waves == dflt.waves) us_default = us[i];
  }
  turpy_tune_entry e{};
  std::snprintf(e.arch, sizeof(e.arch), "%s", key.arch.c_str());
  e.kernel = key.kernel;
  e.n = key.n;
  e.batch_class = key.batch_class;
  e.width = choices[best].width;
  e.radix = choices[best].radix;
  e.waves = choices[best].waves;
  e.configs = static_cast<int32_t>(choices.size());
  e.us = us[best];
  e.us_default = us_default;
  store(e);
  return TURPY_OK;
}

std::vector<LaunchChoice> strip_choices(int n) {
  std::vector<LaunchChoice> out;
  for (int k : kWidths)
    for (int r : {0, 8, 4})
      if (strip_fits_rt(n, k) && radix_built_rt(n, r)) out.push_back({k, r, 0});
  return out;
}

std::vector<LaunchChoice> wave_choices(int n) {
  std::vector<LaunchChoice> out;
  for (int w : {3, 2, 4})
    if (waves_built_rt(n, w)) out.push_back({0, 0, w});
  return out;
}

}  // namespace

std::string turpy::tune_signature(const turpy_plan* pl) {
  const TuneKey c = col_key(pl), s = synth_key(pl);
  char buf[96];
  std::snprintf(buf, sizeof(buf), "%s/%d/%d/%d/%d/%d", c.arch.c_str(), c.kernel, c.n, c.batch_class,
                pl->M > 0 ? s.batch_class : 0, pl->M > 0 ? 1 : 0);
  return buf;
}

extern "C" {

turpy_status turpy_plan_tune(turpy_plan* pl, uint32_t flags, void* ws, size_t ws_bytes, void* stream,
                             int32_t* col_width, int32_t* synth_width) {
  if (!pl) return fail(TURPY_E_INVALID, "plan_tune: NULL plan");
  if (!ws || ws_bytes < pl->ws_tune())
    return fail(TURPY_E_WORKSPACE, "plan_tune: workspace %zu < %zu bytes", ws_bytes, pl->ws_tune());
  if (turpy_status s_ = check_device(pl)) return s_;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  TURPY_HIP(hipStreamIsCapturing(st, &cap), "plan_tune: stream state");
  if (cap != hipStreamCaptureStatusNone) return fail(TURPY_E_INVALID, "plan_tune: the stream is capturing");
  const bool force = (flags & TURPY_TUNE_FORCE) != 0;
  const TuneKey ck = col_key(pl), sk = synth_key(pl);
  const TuneKey rf = row_key(pl, TURPY_TUNE_ROW_FWD), rb = row_key(pl, TURPY_TUNE_ROW_BWD);
  turpy_tune_entry e{};
  const bool screens = pl->M > 0;
  const bool need_col = force || !cached(ck, &e);
  const bool need_synth = screens && (force || !cached(sk, &e));
  const TuneKey ak = ar_key(pl);
  const bool need_ar = screens && (force || !cached(ak, &e));
  const bool need_rf = screens && (force || !cached(rf, &e));
  const bool need_rb = screens && (force || !cached(rb, &e));
  if (need_col || need_synth || need_ar || need_rf || need_rb)
    TURPY_HIP(hipMemsetAsync(ws, 0, pl->ws_tune(), st), "plan_tune: clear workspace");
  const Ws wsp = carve(pl, ws);
  const int n = pl->n;
  const int64_t plane = static_cast<int64_t>(n) * n;
  if (need_col) {
    ColArgs c = col_args(pl, 0, wsp.gbuf, plane, wsp.gbuf, pl->R, false);
    if (turpy_status s = tune_key(ck, strip_choices(n), {default_col_width(n), 0, 0}, st, [&](const LaunchChoice& k) {
          c.width = k.width;
          c.radix = k.radix;
          return launch_col(n, c, st);
        }))
      return s;
  }
  if (need_synth) {
    SynthArgs a = synth_args(pl, 0, 0, 0, nullptr, wsp);
    a.t_dev = nullptr;
    if (turpy_status s = tune_key(sk, strip_choices(n), {default_synth_width(n), 0, 0}, st,
                                  [&](const LaunchChoice& k) {
                                    a.width = k.width;
                                    a.radix = k.radix;
                                    return launch_synth(n, a, st);
                                  }))
      return s;
  }
  if (need_ar) {
    // the AR step of screen 0 on a state of one screen per pair (pair j at
    // plane j), alternating between two such states (the R-plane buffer and
    // the buffer after it): as in a step over M screens, the state a launch
    // reads is not the one the launch before it left in the last-level cache
    const EvolveStep ev{0.99, 0.5, 0.25};
    float2* second = reinterpret_cast<float2*>(static_cast<char*>(ws) + pl->off_ubuf());
    SynthArgs a = synth_args(pl, 0, 1, 0, wsp.gbuf, wsp, &ev);
    a.t_dev = nullptr;
    a.M = 1;
    bool flip = false;
    if (turpy_status s = tune_key(ak, strip_choices(n), {default_synth_width(n), 0, 0}, st,
                                  [&](const LaunchChoice& k) {
                                    a.width = k.width;
                                    a.radix = k.radix;
                                    flip = !flip;
                                    a.state = flip ? second : wsp.gbuf;
                                    return launch_synth(n, a, st);
                                  }))
      return s;
  }
  if (need_rf || need_rb) {
    // screen 0's row pass on the workspace planes: a forward one without
    // checkpoints, an adjoint one reading a one-screen checkpoint
    float2* ub = reinterpret_cast<float2*>(static_cast<char*>(ws) + pl->off_ubuf());
    RowArgs a = base_row(pl);
    a.in = wsp.gbuf;
    a.in_stride = plane;
    a.out = wsp.gbuf;
    a.in_spectral = 1;
    a.out_spectral = 1;
    a.scale = 1.0f / n;
    a.M = 1;
    screen_fields(pl, TURPY_SCREENS_SYNTH, nullptr, wsp, 0, &a);
    a.screen = 0;
    if (need_rf) {
      a.post = pl->d_row + n;
      if (turpy_status s = tune_key(rf, wave_choices(n), {0, 0, 3}, st, [&](const LaunchChoice& k) {
            a.waves = k.waves;
            return launch_row(n, a, pl->P, st);
          }))
        return s;
    }
    if (need_rb) {
      a.post = nullptr;
      a.pre = pl->d_row + n;
      a.conj_tables = 1;
      a.backward = 1;
      a.ckpt_single = 1;
      a.ckpt_in = ub;
      a.grad_screens = reinterpret_cast<float*>(ub + static_cast<size_t>(pl->R) * plane);
      if (turpy_status s = tune_key(rb, wave_choices(n), {0, 0, 3}, st, [&](const LaunchChoice& k) {
            a.waves = k.waves;
            return launch_row(n, a, pl->P, st);
          }))
        return s;
    }
  }
  apply_cached_widths(pl);
  return turpy_plan_widths(pl, col_width, synth_width);
}

turpy_status turpy_plan_widths(const turpy_plan* pl, int32_t* col_width, int32_t* synth_width) {
  if (!pl) return fail(TURPY_E_INVALID, "plan_widths: NULL plan");
  if (col_width) *col_width = pl->col_width ? pl->col_width : default_col_width(pl->n);
  if (synth_width) *synth_width = pl->synth_width ? pl->synth_width : default_synth_width(pl->n);
  return TURPY_OK;
}

turpy_status turpy_plan_set_widths(turpy_plan* pl, int32_t col_width, int32_t synth_width) {
  if (!pl) return fail(TURPY_E_INVALID, "plan_set_widths: NULL plan");
  for (int32_t k : {col_width, synth_width})
    if (k != 0 && !strip_fits_rt(pl->n, k))
      return fail(TURPY_E_INVALID, "plan_set_widths: %d columns per block is not built for n=%d", k, pl->n);
  pl->col_width = col_width;
  pl->synth_width = synth_width;
  return TURPY_OK;
}

turpy_status turpy_plan_config(const turpy_plan* pl, turpy_launch_config* out) {
  if (!pl || !out) return fail(TURPY_E_INVALID, "plan_config: NULL argument");
  out->col_width = pl->col_width ? pl->col_width : default_col_width(pl->n);
  out->col_radix = pl->col_radix;
  out->synth_width = pl->synth_width ? pl->synth_width : default_synth_width(pl->n);
  out->synth_radix = pl->synth_radix;
  out->row_waves = pl->row_waves ? pl->row_waves : 3;
  out->row_waves_bwd = pl->row_waves_bwd ? pl->row_waves_bwd : 3;
  out->ar_width = pl->ar_width ? pl->ar_width : default_synth_width(pl->n);
  out->ar_radix = pl->ar_radix;
  return TURPY_OK;
}

turpy_status turpy_plan_set_config(turpy_plan* pl, const turpy_launch_config* c) {
  if (!pl || !c) return fail(TURPY_E_INVALID, "plan_set_config: NULL argument");
  const int n = pl->n;
  for (int32_t k : {c->col_width, c->synth_width, c->ar_width})
    if (k != 0 && !strip_fits_rt(n, k))
      return fail(TURPY_E_INVALID, "plan_set_config: %d columns per block is not built for n=%d", k, n);
  for (int32_t r : {c->col_radix, c->synth_radix, c->ar_radix})
    if (!radix_built_rt(n, r)) return fail(TURPY_E_INVALID, "plan_set_config: radix %d is not built for n=%d", r, n);
  for (int32_t w : {c->row_waves, c->row_waves_bwd})
    if (w != 0 && !waves_built_rt(n, w))
      return fail(TURPY_E_INVALID, "plan_set_config: %d waves per SIMD is not built for n=%d", w, n);
  pl->col_width = c->col_width;
  pl->col_radix = c->col_radix;
  pl->synth_width = c->synth_width;
  pl->synth_radix = c->synth_radix;
  pl->row_waves = c->row_waves;
  pl->row_waves_bwd = c->row_waves_bwd;
  pl->ar_width = c->ar_width;
  pl->ar_radix = c->ar_radix;
  return TURPY_OK;
}

turpy_status turpy_tune_cache_get(turpy_tune_entry* entries, int32_t capacity, int32_t* count) {
  if (!count || capacity < 0 || (capacity > 0 && !entries))
    return fail(TURPY_E_INVALID, "tune_cache_get: NULL argument or negative capacity");
  std::lock_guard<std::mutex> lock(g_tune_mu);
  int32_t i = 0;
  for (const auto& kv : g_tune) {
    if (i < capacity) entries[i] = kv.second;
    ++i;
  }
  *count = i;
  return TURPY_OK;
}

turpy_status turpy_tune_cache_put(const turpy_tune_entry* entries, int32_t count) {
  if (count < 0 || (count > 0 && !entries)) return fail(TURPY_E_INVALID, "tune_cache_put: NULL entries");
  for (int32_t i = 0; i < count; ++i) {
    const turpy_tune_entry& e = entries[i];
    if (e.kernel < TURPY_TUNE_COL_FRESNEL || e.kernel > TURPY_TUNE_SYNTH_AR)
      return fail(TURPY_E_INVALID, "tune_cache_put: entry %d has unknown kernel %d", i, e.kernel);
    if (e.n < 16 || e.n > 2048 || !pow2(e.n))
      return fail(TURPY_E_INVALID, "tune_cache_put: entry %d: n=%d is not built", i, e.n);
    if (is_row_kernel(e.kernel)) {
      if (e.width != 0 || e.radix != 0 || !waves_built_rt(e.n, e.waves))
        return fail(TURPY_E_INVALID, "tune_cache_put: entry %d: waves %d is not built for n=%d (row kernels take "
                    "waves only)", i, e.waves, e.n);
    } else {
      if (!strip_fits_rt(e.n, e.width))
        return fail(TURPY_E_INVALID, "tune_cache_put: entry %d: width %d is not built for n=%d", i, e.width, e.n);
      if (!radix_built_rt(e.n, e.radix) || e.waves != 0)
        return fail(TURPY_E_INVALID, "tune_cache_put: entry %d: radix %d / waves %d is not built for n=%d", i,
                    e.radix, e.waves, e.n);
    }
    if (e.batch_class < 1 || e.batch_class > 63)
      return fail(TURPY_E_INVALID, "tune_cache_put: entry %d has batch class %d", i, e.batch_class);
    if (strnlen(e.arch, sizeof(e.arch)) == sizeof(e.arch))
      return fail(TURPY_E_INVALID, "tune_cache_put: entry %d: arch is not NUL-terminated", i);
    store(e);
  }
  return TURPY_OK;
}

turpy_status turpy_tune_cache_clear(void) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune.clear();
  return TURPY_OK;
}

}  // extern "C"
