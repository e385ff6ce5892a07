// gfx950 kernels of the split-step turbulence path.
//
// Field layout: complex64 [R][N][N], row-major (i0 = y, i1 = x).  Between the
// passes of a propagation the field lives in the "row-spectral" domain: each
// row has been transformed along x.  One step of Eq. 1 is then two passes:
//   column pass: FFT along y, multiply by the separable chirp h(k0)/N (and the
//                angular-spectrum correction), inverse FFT along y;
//   row pass:    inverse FFT along x (1/N folded into the next multiply),
//                multiply by exp(i phi) of the screen, forward FFT along x and
//                multiply by the next distance's chirp h(k1).
// Each pass reads and writes the field once.  The screen of a realization pair
// is synthesised in two halves that follow the same split: the column half
// (noise, PSD weighting, inverse FFT along y) writes one complex scratch plane
// per pair; the row pass finishes it (inverse FFT along x, subharmonics,
// piston) right before the modulation, so the real screens never touch HBM.
//
// Strided accesses are written (p + t)[T * m]: one address per row or column
// for the thread, then compile-time offsets per element (the index form
// p[t + T * m] made the compiler build a 64-bit address per element).
#include <algorithm>

#include "fft.hpp"
#include "kernels.hpp"
#include "layout.hpp"

namespace turpy {

namespace {

// PSD weighting of Eq. S16/S17 at integer radius^2 q (in bins):
// amp * exp(-f^2/(2 fm^2)) * (f^2 + f0^2)^(-alpha/4), f^2 = q df^2; zero at DC
// (alpha = 11/3 for Eq. S17; other media per App. B Table S1).
__device__ __forceinline__ float psd_amp(int q, float amp, float df2, float inner, float f02, float qexp) {
  if (q == 0) return 0.0f;
  const float f2 = static_cast<float>(q) * df2;
  const float l2 = -f2 * inner - qexp * __builtin_amdgcn_logf(f2 + f02);
  return amp * __builtin_amdgcn_exp2f(l2);
}

__device__ __forceinline__ int signed_bin(int k, int n) { return k < (n >> 1) ? k : k - n; }

// The noise time step of a launch: its argument, or, for plans bound to a
// device-resident time step (graph replays), the value there when it runs.
template <class Args>
__device__ __forceinline__ uint32_t time_step(const Args& a) {
  return a.t_dev ? *a.t_dev : a.t;
}

// A field row in the strided layout, v[m] = p[T m]: with the non-temporal
// policy (NT) when each realization reads its own row, plain when all of them
// read one shared source plane (its rows are then re-read from L2).
template <bool NT, int T>
__device__ __forceinline__ void load_field_row(float2 (&v)[kE], const float2* p, bool shared) {
  if (shared) {
#pragma unroll
    for (int m = 0; m < kE; ++m) v[m] = p[T * m];
  } else {
#pragma unroll
    for (int m = 0; m < kE; ++m) v[m] = ld_s<NT>(p + T * m);
  }
}

// ---------------------------------------------------------------------------
// Row pass.
// ---------------------------------------------------------------------------
template <int N, int SCREEN, bool BWD>
__device__ __forceinline__ void row_pass_body(const RowArgs& a) {
  constexpr int T = N / kE;
  constexpr int G = row_groups<N>();
  constexpr bool WV = T <= 64;  // each row's transform lives in one wavefront
  __shared__ float2 smem[G * RowLds::words(N)];
  TURPY_LDS_INIT(smem);
  const int g = threadIdx.x / T;
  const int t = threadIdx.x % T;
  const int i0 = blockIdx.x * G + g;
  const int64_t j = blockIdx.y;
  const RowLds lds{smem + g * RowLds::words(N)};
  __shared__ float2 tw_lds[N];
  const float2* tw = stage_twiddles<N>(tw_lds, a.tw);
  const size_t plane = static_cast<size_t>(N) * N;
  const size_t row_off = static_cast<size_t>(i0) * N;

  float pa[kE], pb[kE];  // screen phase (revolutions) for realizations 2j and 2j+1
  if constexpr (SCREEN == ROW_SCRATCH) {
    float2 z[kE];
    const float2* src = a.scratch + j * plane + row_off;
#pragma unroll
    for (int m = 0; m < kE; ++m) z[m] = (src + t)[T * m];
    fft<N, kE, true, WV>(z, lds, t, tw);
    if (a.sh_levels > 0) {
      const float2* c = a.sh + (static_cast<size_t>(j) * a.M + a.screen) * 32;
      const float2 mean = c_scale(c[24], a.sh_scale);
#pragma unroll
      for (int m = 0; m < kE; ++m) z[m] = c_sub(z[m], mean);
      for (int p = 0; p < a.sh_levels; ++p) {
        const float2* cp = c + 8 * p;
        const float2* ph = a.sh_phasor + static_cast<size_t>(p) * N;
        const float2 ey = ph[i0];
        const float2 eyc = make_float2(ey.x, -ey.y);
        // offsets (m, n): 0 (-1,-1) 1 (-1,0) 2 (-1,1) 3 (0,-1) 4 (0,1) 5 (1,-1) 6 (1,0) 7 (1,1)
        const float2 dm = c_scale(c_add(c_add(c_mul(cp[0], eyc), cp[3]), c_mul(cp[5], ey)), a.sh_scale);
        const float2 d0 = c_scale(c_add(c_mul(cp[1], eyc), c_mul(cp[6], ey)), a.sh_scale);
        const float2 dp = c_scale(c_add(c_add(c_mul(cp[2], eyc), cp[4]), c_mul(cp[7], ey)), a.sh_scale);
        const float2 sa = c_add(dp, dm);
        const float2 sb = c_sub(dp, dm);
#pragma unroll
        for (int m = 0; m < kE; ++m) {
          const float2 ex = (ph + t)[T * m];
          z[m].x += d0.x + sa.x * ex.x - sb.y * ex.y;
          z[m].y += d0.y + sa.y * ex.x + sb.x * ex.y;
        }
      }
    }
#pragma unroll
    for (int m = 0; m < kE; ++m) {
      pa[m] = z[m].x;
      pb[m] = z[m].y;
    }
  } else if constexpr (SCREEN == ROW_MATERIALIZED) {
    constexpr float inv2pi = 0.15915494309189535f;
    const int64_t ra = 2 * j, rb = 2 * j + 1;
    const float* sa = a.screens + (static_cast<size_t>(ra) * a.M + a.screen) * plane + row_off;
#pragma unroll
    for (int m = 0; m < kE; ++m) pa[m] = (sa + t)[T * m] * inv2pi;
    if (rb < a.R) {
      const float* sb = a.screens + (static_cast<size_t>(rb) * a.M + a.screen) * plane + row_off;
#pragma unroll
      for (int m = 0; m < kE; ++m) pb[m] = (sb + t)[T * m] * inv2pi;
    }
  }

  if (SCREEN != ROW_NO_SCREEN && a.phase_out) {
    constexpr float two_pi = 6.283185307179586f;
    for (int b = 0; b < 2; ++b) {
      const int64_t r = 2 * j + b;
      if (r >= a.R) break;
      float* dst = a.phase_out + (static_cast<size_t>(r) * a.M + a.screen) * plane + row_off;
      const float* ph = b ? pb : pa;
#pragma unroll
      for (int m = 0; m < kE; ++m) (dst + t)[T * m] = ph[m] * two_pi;
    }
  }
  if (!a.in) return;  // uniform over the block

  for (int b = 0; b < 2; ++b) {
    const int64_t r = 2 * j + b;
    if (r >= a.R) break;  // uniform over the block
    float2 x[kE];
    const float2* src = a.in + r * a.in_stride + row_off;
#pragma unroll
    for (int m = 0; m < kE; ++m) x[m] = (src + t)[T * m];
    if (a.in_spectral) {
      if (a.pre) {
#pragma unroll
        for (int m = 0; m < kE; ++m) {
          const float2 h = (a.pre + t)[T * m];
          x[m] = a.conj_tables ? c_mulc(x[m], h) : c_mul(x[m], h);
        }
      }
      fft<N, kE, true, WV>(x, lds, t, tw);
    }
    const float* ph = b ? pb : pa;
    if constexpr (SCREEN != ROW_NO_SCREEN) {
      const size_t ck = (static_cast<size_t>(r) * a.M + a.screen) * plane + row_off;
      const size_t cw = a.ckpt_single ? static_cast<size_t>(r) * plane + row_off : ck;
      if constexpr (!BWD) {
#pragma unroll
        for (int m = 0; m < kE; ++m) {
          float s, c;
          sincos_rev(ph[m], &s, &c);
          x[m] = c_mul(x[m], make_float2(c * a.scale, s * a.scale));
        }
        if (a.ckpt_out) {
#pragma unroll
          for (int m = 0; m < kE; ++m) st_s<true>(a.ckpt_out + cw + t + T * m, x[m]);
        }
      } else {
        if (a.ckpt_out) {  // the forward field at this screen, rebuilt by the adjoint chain
#pragma unroll
          for (int m = 0; m < kE; ++m) (a.ckpt_out + cw + t)[T * m] = x[m];
        }
        if (a.grad_screens) {
#pragma unroll
          for (int m = 0; m < kE; ++m) {
            const float2 w = (a.ckpt_in + cw + t)[T * m];
            st_f<true>(a.grad_screens + ck + t + T * m, w.x * x[m].y - w.y * x[m].x);  // Im(conj(W) g)
          }
        }
#pragma unroll
        for (int m = 0; m < kE; ++m) {
          float s, c;
          sincos_rev(ph[m], &s, &c);
          x[m] = c_mul(x[m], make_float2(c * a.scale, -s * a.scale));
        }
      }
    } else {
      if (a.scale != 1.0f) {
#pragma unroll
        for (int m = 0; m < kE; ++m) x[m] = c_scale(x[m], a.scale);
      }
    }
    if (a.out_spectral) {
      fft<N, kE, false, WV>(x, lds, t, tw);
      if (a.post) {
#pragma unroll
        for (int m = 0; m < kE; ++m) {
          const float2 h = (a.post + t)[T * m];
          x[m] = a.conj_tables ? c_mulc(x[m], h) : c_mul(x[m], h);
        }
      }
    }
    float2* dst = a.out + r * plane + row_off;
#pragma unroll
    for (int m = 0; m < kE; ++m) (dst + t)[T * m] = x[m];
  }
}

template <int N, int SCREEN, bool BWD>
__global__ __launch_bounds__(row_block<N>()) void row_pass_kernel(RowArgs a) { row_pass_body<N, SCREEN, BWD>(a); }

// ---------------------------------------------------------------------------
// Row pass with a screen, split over the two realizations of a pair.  Half A
// (realization 2j) finishes the screen row: inverse FFT of the scratch row,
// subharmonics and piston, keeps Re z and hands Im z to half B through LDS.
// Half B (realization 2j+1) meanwhile loads and inverse-transforms its own
// field row.  Then both modulate (or, backward, form dL/dphi and apply the
// conjugate phase) and transform forward.  Both halves pass the same barrier
// sequence: a half with no transform at a stage runs idle_fft.
// ---------------------------------------------------------------------------
template <int N, int SCREEN, bool BWD>
__device__ __forceinline__ void row_pair_body(const RowArgs& a) {
  constexpr int T = N / kE;
  constexpr int G = pair_rows<N>();
  constexpr int HALF = G * T;
  constexpr bool WV = T <= 64;  // each row's transform lives in one wavefront
  __shared__ float2 smem[2 * G * RowLds::words(N)];
  TURPY_LDS_INIT(smem);
  const int role = threadIdx.x / HALF;
  const int g = (threadIdx.x % HALF) / T;
  const int t = threadIdx.x % T;
  const int i0 = blockIdx.x * G + g;
  const int64_t j = blockIdx.y;
  const bool has_b = 2 * j + 1 < a.R;
  const int64_t r = (role == 1 && has_b) ? 2 * j + 1 : 2 * j;
  const bool writes = role == 0 || has_b;
  const RowLds lds{smem + (role * G + g) * RowLds::words(N)};
  float* handoff = reinterpret_cast<float*>(smem + (G + g) * RowLds::words(N));  // half B's buffer
  __shared__ float2 tw_lds[N];
  const float2* tw = stage_twiddles<N>(tw_lds, a.tw);
  const size_t plane = static_cast<size_t>(N) * N;
  const size_t row_off = static_cast<size_t>(i0) * N;
  const bool in_spec = a.in_spectral != 0, out_spec = a.out_spectral != 0;

  float ph[kE];
  float2 x[kE];
  float2 y[kE];  // half A's field row, fetched with its screen row (scratch mode)
  // adjoint: the checkpointed forward field of this row, fetched before the
  // transform that precedes its use in the screen gradient
  float2 wck[kE];
  const bool want_ck = BWD && a.grad_screens && writes;
  const size_t ck_row = (static_cast<size_t>(r) * a.M + a.screen) * plane + row_off;
  const size_t cw_row = a.ckpt_single ? static_cast<size_t>(r) * plane + row_off : ck_row;
  auto fetch_ckpt = [&]() {
    if constexpr (BWD) {
      if (want_ck) {
#pragma unroll
        for (int m = 0; m < kE; ++m) wck[m] = ld_s<true>(a.ckpt_in + cw_row + t + T * m);
      }
    }
  };
  // stage 1: A -> screen row (scratch) or its phases (materialised); B -> its field row
  if (role == 0) {
    if constexpr (SCREEN == ROW_SCRATCH) {
      const float2* src = a.scratch + j * plane + row_off;
#pragma unroll
      for (int m = 0; m < kE; ++m) x[m] = ld_s<true>(src + t + T * m);
      {
        const float2* fa = a.in + r * a.in_stride + row_off;
        load_field_row<true, T>(y, fa + t, a.in_stride == 0);
      }
      fft<N, kE, true, WV>(x, lds, t, tw);
    } else {
      constexpr float inv2pi = 0.15915494309189535f;
      const float* sa = a.screens + (static_cast<size_t>(r) * a.M + a.screen) * plane + row_off;
#pragma unroll
      for (int m = 0; m < kE; ++m) ph[m] = (sa + t)[T * m] * inv2pi;
      if (in_spec) idle_fft<N, WV>();
    }
  } else {
    const float2* src = a.in + r * a.in_stride + row_off;
    load_field_row<true, T>(x, src + t, a.in_stride == 0);
    fetch_ckpt();
    if (in_spec) {
      if (a.pre) {
#pragma unroll
        for (int m = 0; m < kE; ++m) {
          const float2 h = (a.pre + t)[T * m];
          x[m] = a.conj_tables ? c_mulc(x[m], h) : c_mul(x[m], h);
        }
      }
      fft<N, kE, true, WV>(x, lds, t, tw);
    } else if (SCREEN == ROW_SCRATCH) {
      idle_fft<N, WV>();
    }
  }
  // stage 2: phases of both halves.  The hand-off goes through half B's
  // exchange buffer: half B must be done with its stage-1 transform first.
  if constexpr (SCREEN == ROW_SCRATCH) {
    __syncthreads();
    if (role == 0) {
      if (a.sh_levels > 0) {
        const float2* c = a.sh + (static_cast<size_t>(j) * a.M + a.screen) * 32;
        const float2 mean = c_scale(c[24], a.sh_scale);
#pragma unroll
        for (int m = 0; m < kE; ++m) x[m] = c_sub(x[m], mean);
        for (int p = 0; p < a.sh_levels; ++p) {
          const float2* cp = c + 8 * p;
          const float2* phs = a.sh_phasor + static_cast<size_t>(p) * N;
          const float2 ey = phs[i0];
          const float2 eyc = make_float2(ey.x, -ey.y);
          // offsets (m, n): 0 (-1,-1) 1 (-1,0) 2 (-1,1) 3 (0,-1) 4 (0,1) 5 (1,-1) 6 (1,0) 7 (1,1)
          const float2 dm = c_scale(c_add(c_add(c_mul(cp[0], eyc), cp[3]), c_mul(cp[5], ey)), a.sh_scale);
          const float2 d0 = c_scale(c_add(c_mul(cp[1], eyc), c_mul(cp[6], ey)), a.sh_scale);
          const float2 dp = c_scale(c_add(c_add(c_mul(cp[2], eyc), cp[4]), c_mul(cp[7], ey)), a.sh_scale);
          const float2 sa = c_add(dp, dm);
          const float2 sb = c_sub(dp, dm);
#pragma unroll
          for (int m = 0; m < kE; ++m) {
            const float2 ex = (phs + t)[T * m];
            x[m].x += d0.x + sa.x * ex.x - sb.y * ex.y;
            x[m].y += d0.y + sa.y * ex.x + sb.x * ex.y;
          }
        }
      }
#pragma unroll
      for (int m = 0; m < kE; ++m) {
        ph[m] = x[m].x;
        (handoff + t)[T * m] = x[m].y;
      }
    }
    __syncthreads();
    if (role == 1) {
#pragma unroll
      for (int m = 0; m < kE; ++m) ph[m] = (handoff + t)[T * m];
    }
    __syncthreads();
  } else {
    if (role == 1) {
      constexpr float inv2pi = 0.15915494309189535f;
      const float* sb = a.screens + (static_cast<size_t>(r) * a.M + a.screen) * plane + row_off;
#pragma unroll
      for (int m = 0; m < kE; ++m) ph[m] = (sb + t)[T * m] * inv2pi;
    }
  }

  // the pointwise step of Eq. 1 (or its adjoint) and the forward transform
  auto finish = [&]() {
    const size_t ck = ck_row, cw = cw_row;
    if constexpr (!BWD) {
#pragma unroll
      for (int m = 0; m < kE; ++m) {
        float s, c;
        sincos_rev(ph[m], &s, &c);
        x[m] = c_mul(x[m], make_float2(c * a.scale, s * a.scale));
      }
      if (a.ckpt_out && writes) {
#pragma unroll
        for (int m = 0; m < kE; ++m) st_s<true>(a.ckpt_out + cw + t + T * m, x[m]);
      }
    } else {
      if (a.ckpt_out && writes) {  // the forward field at this screen, rebuilt by the adjoint chain
#pragma unroll
        for (int m = 0; m < kE; ++m) (a.ckpt_out + cw + t)[T * m] = x[m];
      }
      if (want_ck) {
#pragma unroll
        for (int m = 0; m < kE; ++m) {
          const float2 w = wck[m];
          st_f<true>(a.grad_screens + ck + t + T * m, w.x * x[m].y - w.y * x[m].x);  // Im(conj(W) g)
        }
      }
#pragma unroll
      for (int m = 0; m < kE; ++m) {
        float s, c;
        sincos_rev(ph[m], &s, &c);
        x[m] = c_mul(x[m], make_float2(c * a.scale, -s * a.scale));
      }
    }
    if (out_spec) {
      fft<N, kE, false, WV>(x, lds, t, tw);
      if (a.post) {
#pragma unroll
        for (int m = 0; m < kE; ++m) {
          const float2 h = (a.post + t)[T * m];
          x[m] = a.conj_tables ? c_mulc(x[m], h) : c_mul(x[m], h);
        }
      }
    }
    if (writes) {
      float2* dst = a.out + r * static_cast<int64_t>(plane) + row_off;
#pragma unroll
      for (int m = 0; m < kE; ++m) (dst + t)[T * m] = x[m];
    }
  };

  // stage 3: A loads / inverse-transforms its field; B finishes
  if (role == 0) {
    if (SCREEN == ROW_SCRATCH) {
#pragma unroll
      for (int m = 0; m < kE; ++m) x[m] = y[m];
    } else {
      const float2* src = a.in + r * a.in_stride + row_off;
      load_field_row<true, T>(x, src + t, a.in_stride == 0);
    }
    fetch_ckpt();
    if (in_spec) {
      if (a.pre) {
#pragma unroll
        for (int m = 0; m < kE; ++m) {
          const float2 h = (a.pre + t)[T * m];
          x[m] = a.conj_tables ? c_mulc(x[m], h) : c_mul(x[m], h);
        }
      }
      fft<N, kE, true, WV>(x, lds, t, tw);
    } else if (out_spec) {
      idle_fft<N, WV>();
    }
  } else {
    finish();
    if (in_spec && !out_spec) idle_fft<N, WV>();
  }
  // stage 4: A finishes
  if (role == 0) {
    finish();
  } else if (out_spec) {
    idle_fft<N, WV>();
  }
}

template <int N, int SCREEN, bool BWD, int W>
__global__ __launch_bounds__(pair_block<N>()) __attribute__((amdgpu_waves_per_eu(W, 0)))
void row_pair_kernel(RowArgs a) { row_pair_body<N, SCREEN, BWD>(a); }

// ---------------------------------------------------------------------------
// Forward row pass over a realization pair with synthesised screens and no
// checkpoint output, relay schedule.  A block holds two workers (whole waves)
// and two row groups of pair j: group 0 = rows [i0, i0 + G), group 1 = rows
// [i0 + G, i0 + 2G).  Each group needs five transforms: the inverse transform
// of its screen rows (S), the inverse transforms of the field rows of
// realizations 2j and 2j+1 (A, B), and their forward transforms after the
// pointwise step (A', B'), which need S.  Worker 0 draws S of group 0,
// worker 1 S of group 1, and five stages keep both workers busy (the pair
// schedule above leaves one half idle in its last stage):
//   stage 0: w0 S0    w1 B0
//   stage 1: w0 A0    w1 B0'   (Im S0 handed from w0 to w1 through LDS)
//   stage 2: w0 A0'   w1 S1
//   stage 3: w0 B1    w1 A1
//   stage 4: w0 B1'   w1 A1'   (Im S1 handed from w1 to w0)
// Each worker fetches an A row together with the screen row before it.  Two
// block barriers order the hand-offs.  Where the transforms use block
// barriers a stage whose two transforms differ in kind passes the same
// barriers on both sides (idle_fft).
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ void row_relay_body(const RowArgs& a) {
  constexpr int T = N / kE;
  constexpr int G = relay_rows<N>();
  constexpr int HALF = G * T;
  constexpr bool WV = T <= 64;  // each row's transform lives in one wavefront
  static_assert(HALF % 64 == 0 && 2 * G <= N, "a relay worker is whole waves over half the block's rows");
  __shared__ float2 smem[2 * G * RowLds::words(N)];
  TURPY_LDS_INIT(smem);
  __shared__ float handoff_rows[G * N];
  TURPY_LDS_INIT(handoff_rows);
  __shared__ float2 tw_lds[N];
  const int w = threadIdx.x / HALF;
  const int g = (threadIdx.x % HALF) / T;
  const int t = threadIdx.x % T;
  const int64_t j = blockIdx.y;
  const bool has_b = 2 * j + 1 < a.R;
  const int64_t ra = 2 * j, rb = has_b ? 2 * j + 1 : 2 * j;  // a missing B reads A's rows, writes nothing
  const int row0 = blockIdx.x * 2 * G + g;  // this thread's row in group 0
  const int row1 = row0 + G;                // and in group 1
  const RowLds lds{smem + (w * G + g) * RowLds::words(N)};
  float* hand = handoff_rows + g * N + t;
  const float2* tw = stage_twiddles<N>(tw_lds, a.tw);
  const size_t plane = static_cast<size_t>(N) * N;
  const bool in_spec = a.in_spectral != 0, out_spec = a.out_spectral != 0;
  const bool both = in_spec || out_spec;

  float ph[kE];
  float2 x[kE], y[kE];
  auto load_field = [&](float2 (&v)[kE], int64_t r, int row) {
    const float2* src = a.in + r * a.in_stride + static_cast<size_t>(row) * N + t;
    load_field_row<true, T>(v, src, a.in_stride == 0);
  };
  // x (a loaded field row) to real space; slot: the other worker transforms
  // in this stage
  auto inverse = [&](bool slot) {
    if (in_spec) {
      fft<N, kE, true, WV>(x, lds, t, tw);
    } else if (slot) {
      idle_fft<N, WV>();
    }
  };
  auto load_screen = [&](int row) {
    const float2* src = a.scratch + j * plane + static_cast<size_t>(row) * N + t;
#pragma unroll
    for (int m = 0; m < kE; ++m) x[m] = ld_s<true>(src + T * m);
  };
  // screen row of pair j: inverse row transform of the scratch row, the
  // subharmonics and the piston of Eq. 2-3; Re into ph, Im into the hand-off
  auto screen = [&](int row) {
    fft<N, kE, true, WV>(x, lds, t, tw);
    if (a.sh_levels > 0) {
      const float2* c = a.sh + (static_cast<size_t>(j) * a.M + a.screen) * 32;
      const float2 mean = c_scale(c[24], a.sh_scale);
#pragma unroll
      for (int m = 0; m < kE; ++m) x[m] = c_sub(x[m], mean);
      for (int p = 0; p < a.sh_levels; ++p) {
        const float2* cp = c + 8 * p;
        const float2* phs = a.sh_phasor + static_cast<size_t>(p) * N;
        const float2 ey = phs[row];
        const float2 eyc = make_float2(ey.x, -ey.y);
        // offsets (m, n): 0 (-1,-1) 1 (-1,0) 2 (-1,1) 3 (0,-1) 4 (0,1) 5 (1,-1) 6 (1,0) 7 (1,1)
        const float2 dm = c_scale(c_add(c_add(c_mul(cp[0], eyc), cp[3]), c_mul(cp[5], ey)), a.sh_scale);
        const float2 d0 = c_scale(c_add(c_mul(cp[1], eyc), c_mul(cp[6], ey)), a.sh_scale);
        const float2 dp = c_scale(c_add(c_add(c_mul(cp[2], eyc), cp[4]), c_mul(cp[7], ey)), a.sh_scale);
        const float2 sa = c_add(dp, dm);
        const float2 sb = c_sub(dp, dm);
#pragma unroll
        for (int m = 0; m < kE; ++m) {
          const float2 ex = (phs + t)[T * m];
          x[m].x += d0.x + sa.x * ex.x - sb.y * ex.y;
          x[m].y += d0.y + sa.y * ex.x + sb.x * ex.y;
        }
      }
    }
#pragma unroll
    for (int m = 0; m < kE; ++m) {
      ph[m] = x[m].x;
      hand[T * m] = x[m].y;
    }
  };
  // the pointwise step of Eq. 1, the forward transform and the store of
  // realization r's row
  auto finish = [&](int64_t r, int row, bool writes, bool slot) {
#pragma unroll
    for (int m = 0; m < kE; ++m) {
      float s, c;
      sincos_rev(ph[m], &s, &c);
      x[m] = c_mul(x[m], make_float2(c * a.scale, s * a.scale));
    }
    if (out_spec) {
      fft<N, kE, false, WV>(x, lds, t, tw);
      if (a.post) {
#pragma unroll
        for (int m = 0; m < kE; ++m) x[m] = c_mul(x[m], (a.post + t)[T * m]);
      }
    } else if (slot) {
      idle_fft<N, WV>();
    }
    if (writes) {
      float2* dst = a.out + r * static_cast<int64_t>(plane) + static_cast<size_t>(row) * N + t;
#pragma unroll
      for (int m = 0; m < kE; ++m) dst[T * m] = x[m];
    }
  };

  if (w == 0) {
    load_screen(row0);                  // stage 0: S0, with A0's field row
    load_field(y, ra, row0);
    screen(row0);
  } else {
    load_field(x, rb, row0);            // stage 0: B0
    inverse(true);
  }
  __syncthreads();  // Im S0 in the hand-off
  if (w == 0) {
#pragma unroll
    for (int m = 0; m < kE; ++m) x[m] = y[m];
    inverse(both);                      // stage 1: A0
    finish(ra, row0, true, true);       // stage 2: A0'
    load_field(x, rb, row1);            // stage 3: B1
    inverse(false);
  } else {
#pragma unroll
    for (int m = 0; m < kE; ++m) ph[m] = hand[T * m];
    finish(rb, row0, has_b, both);      // stage 1: B0'
    load_screen(row1);                  // stage 2: S1, with A1's field row
    load_field(y, ra, row1);
    screen(row1);
#pragma unroll
    for (int m = 0; m < kE; ++m) x[m] = y[m];
    inverse(false);                     // stage 3: A1
  }
  __syncthreads();  // Im S1 in the hand-off
  if (w == 0) {
#pragma unroll
    for (int m = 0; m < kE; ++m) ph[m] = hand[T * m];
    finish(rb, row1, has_b, false);     // stage 4: B1'
  } else {
    finish(ra, row1, true, false);      // stage 4: A1'
  }
}

template <int N, int W>
__global__ __launch_bounds__(relay_block<N>()) __attribute__((amdgpu_waves_per_eu(W, 0)))
void row_relay_kernel(RowArgs a) { row_relay_body<N>(a); }

// ---------------------------------------------------------------------------
// Column pass: FFT along y, x h(k0)/N (x angular-spectrum correction), IFFT.
// ---------------------------------------------------------------------------
// Transfer-function modes of the column pass: Fresnel chirp only, or the
// angular-spectrum correction H_as / H_fresnel on top of it (Sec. 2.1).
constexpr int TF_FRESNEL_ONLY = 0;
constexpr int TF_AS_FP32 = 1;   // every bin propagates: the small angle in FP32
constexpr int TF_AS_TABLE = 2;  // evanescent bins present: the plan's FP64 radial table

// Correction of bin (k0, k1), a function of q = k0^2 + k1^2 (signed bins).
// FP32 form: -dz kappa^4 / (2k (s + k)^2), s = sqrt(k^2 - kappa^2), written as
// C q^2 / (1 + sqrt(1 - B q))^2 revolutions with kappa^2 = (2 pi df)^2 q,
// B = (2 pi df)^2 / k^2, C = -dz (2 pi df)^4 / (4 pi k^3); well conditioned
// (no cancellation) for every propagating bin.
template <int MODE>
__device__ __forceinline__ float2 angular_correction(const ColArgs& a, int k0, int k1, int n) {
  const int kx = signed_bin(k1, n), ky = signed_bin(k0, n);
  const int q = kx * kx + ky * ky;
  if constexpr (MODE == TF_AS_TABLE) {
    return a.as_table[q];
  } else {
    const float qf = static_cast<float>(q);
    const float r = 1.0f + __builtin_amdgcn_sqrtf(1.0f - qf * a.as_b);
    const float rev = a.as_c * qf * qf * __builtin_amdgcn_rcpf(r * r);
    float sn, cs;
    sincos_rev(rev, &sn, &cs);
    return make_float2(cs, sn);
  }
}

template <int N, int ANGULAR, int K, int R2SEL>
__device__ __forceinline__ void col_pass_body(const ColArgs& a) {
  constexpr int T = N / kE;
  constexpr int STRIPS = N / K;
  __shared__ float2 smem[ColLds<K>::words(N)];
  TURPY_LDS_INIT(smem);
  int strip;
  int64_t r;
  col_tile(blockIdx.x, gridDim.x, STRIPS, a.R, &strip, &r);
  const int c = threadIdx.x % K;
  const int t = threadIdx.x / K;
  const int k1 = strip * K + c;
  const ColLds<K> lds{smem, c};
  __shared__ float2 tw_lds[N];
  __shared__ float2 h_lds[N];
  TURPY_LDS_INIT(h_lds);
  for (int i = threadIdx.x; i < N; i += blockDim.x) h_lds[i] = a.table[i];
  const float2* chirp = h_lds;
  const float2* tw = stage_twiddles<N>(tw_lds, a.tw);
  const float2* src = a.in + r * a.in_stride + k1;
  float2 x[kE];
#pragma unroll
  for (int m = 0; m < kE; ++m) x[m] = (src + static_cast<size_t>(t) * N)[static_cast<size_t>(T * m) * N];
  fft<N, kE, false, false, R2SEL>(x, lds, t, tw);
#pragma unroll
  for (int m = 0; m < kE; ++m) {
    const int k0 = t + T * m;
    float2 h = chirp[k0];
    if constexpr (ANGULAR != TF_FRESNEL_ONLY) h = c_mul(h, angular_correction<ANGULAR>(a, k0, k1, N));
    x[m] = a.conj_table ? c_mulc(x[m], h) : c_mul(x[m], h);
  }
  fft<N, kE, true, false, R2SEL>(x, lds, t, tw);
  float2* dst = a.out + r * static_cast<int64_t>(N) * N + k1;
#pragma unroll
  for (int m = 0; m < kE; ++m) (dst + static_cast<size_t>(t) * N)[static_cast<size_t>(T * m) * N] = x[m];
}

template <int N, int ANGULAR, int K, int R2SEL>
__global__ __launch_bounds__(K * (N / kE))
void col_pass_kernel(ColArgs a) { col_pass_body<N, ANGULAR, K, R2SEL>(a); }

// ---------------------------------------------------------------------------
// Column half of the screen synthesis: noise x PSD weight (Eq. S16/S17), or a
// stored spectrum, then the unnormalised inverse transform along y.
// ---------------------------------------------------------------------------
template <int N, int K, int R2SEL>
__device__ __forceinline__ void synth_col_body(const SynthArgs& a) {
  constexpr int T = N / kE;
  constexpr int STRIPS = N / K;
  __shared__ float2 smem[ColLds<K>::words(N)];
  TURPY_LDS_INIT(smem);
  const uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
  const int strip = b % STRIPS;
  const int64_t j = b / STRIPS;
  const int c = threadIdx.x % K;
  const int t = threadIdx.x / K;
  const int k1 = strip * K + c;
  const ColLds<K> lds{smem, c};
  __shared__ float2 tw_lds[N];
  const float2* tw = stage_twiddles<N>(tw_lds, a.tw);
  float2 x[kE];
  if (a.evolve) {
    // Eq. 4 (translation by exp(-2 pi i (kx sx + ky sy)/N), the phase reduced
    // in FP64) then Eq. 5 (alpha blend with fresh innovations), bin pairs
    // (k0, k1), (k0 + N/2, k1) sharing one Philox block; DC kept at zero
    constexpr float inv2pi = 0.15915494309189535f;
    float2* st = a.state + (static_cast<size_t>(j) * a.M + a.screen) * N * N + k1 + static_cast<size_t>(t) * N;
    const int kx = signed_bin(k1, N);
    const double inv_n = 1.0 / N;
    float2 old[kE];
#pragma unroll
    for (int m = 0; m < kE; ++m) old[m] = st[static_cast<size_t>(T * m) * N];
#pragma unroll
    for (int m = 0; m < kE / 2; ++m) {
      const int k0 = t + T * m;  // < N/2
      const uint32_t e = static_cast<uint32_t>(k0) * N + k1;
      const uint4 v = philox4x32_10(noise_counter(e, time_step(a), static_cast<uint32_t>(j), a.ar_tag, a.screen),
                                    a.key0, a.key1);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int kk0 = k0 + h * (N / 2);
        const int ky = signed_bin(kk0, N);
        const float w = psd_amp(ky * ky + kx * kx, a.amp_rad, a.df2, a.inner, a.f02, a.q);
        const float2 nc = h == 0 ? box_muller(v.x, v.y) : box_muller(v.z, v.w);
        double rev = -(static_cast<double>(kx) * a.sx + static_cast<double>(ky) * a.sy) * inv_n;
        rev -= rint(rev);
        float sn, cs;
        sincos_rev(static_cast<float>(rev), &sn, &cs);
        float2 out = c_add(c_scale(c_mul(old[m + h * (kE / 2)], make_float2(cs, sn)), a.alpha_f),
                           c_scale(nc, a.blend * w));
        if (kk0 == 0 && k1 == 0) out = make_float2(0.0f, 0.0f);
        x[m + h * (kE / 2)] = out;
      }
    }
#pragma unroll
    for (int m = 0; m < kE; ++m) {
      // read back one time step later: non-temporal where a strip row is a
      // whole 128-byte line (16 columns)
      st_s<(K >= 16)>(st + static_cast<size_t>(T * m) * N, x[m]);
      x[m] = c_scale(x[m], inv2pi);
    }
  } else if (a.spectra) {
    constexpr float inv2pi = 0.15915494309189535f;
    const float2* src = a.spectra + (static_cast<size_t>(j) * a.M + a.screen) * N * N + k1;
#pragma unroll
    for (int m = 0; m < kE; ++m)
      x[m] = c_scale((src + static_cast<size_t>(t) * N)[static_cast<size_t>(T * m) * N], inv2pi);
  } else {
    const int kx = signed_bin(k1, N);
#pragma unroll
    for (int m = 0; m < kE / 2; ++m) {
      const int k0 = t + T * m;  // < N/2
      const uint32_t e = static_cast<uint32_t>(k0) * N + k1;
      const uint4 v = philox4x32_10(noise_counter(e, time_step(a), static_cast<uint32_t>(j), a.tag, a.screen), a.key0,
                                    a.key1);
      const int ky_lo = k0;             // signed bin of k0 (< N/2)
      const int ky_hi = k0 - N / 2;     // signed bin of k0 + N/2
      const float w_lo = psd_amp(ky_lo * ky_lo + kx * kx, a.amp, a.df2, a.inner, a.f02, a.q);
      const float w_hi = psd_amp(ky_hi * ky_hi + kx * kx, a.amp, a.df2, a.inner, a.f02, a.q);
      x[m] = c_scale(box_muller(v.x, v.y), w_lo);
      x[m + kE / 2] = c_scale(box_muller(v.z, v.w), w_hi);
    }
  }
  fft<N, kE, true, false, R2SEL>(x, lds, t, tw);
  float2* dst = a.scratch + j * static_cast<int64_t>(N) * N + k1;
#pragma unroll
  for (int m = 0; m < kE; ++m) (dst + static_cast<size_t>(t) * N)[static_cast<size_t>(T * m) * N] = x[m];
}

template <int N, int K, int R2SEL>
__global__ __launch_bounds__(K * (N / kE))
void synth_col_kernel(SynthArgs a) { synth_col_body<N, K, R2SEL>(a); }

// ---------------------------------------------------------------------------
// Subharmonic coefficients of Eq. 2 for every (pair, screen), and their mean.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void sh_body(const ShArgs& a) {
  __shared__ float2 coef[24];
  TURPY_LDS_INIT(coef);
  const int64_t j = blockIdx.x;
  const int s = blockIdx.y;
  const int l = threadIdx.x;
  float2* out = a.sh + (static_cast<size_t>(j) * a.M + s) * 32;
  if (l < 4 * a.levels) {
    const int p = l / 4;
    const uint4 v = philox4x32_10(noise_counter(static_cast<uint32_t>(l), time_step(a), static_cast<uint32_t>(j), a.tag,
                                                static_cast<uint32_t>(s)),
                                  a.key0, a.key1);
    const float* amp = a.amp + (static_cast<size_t>(s) * 3 + p) * 2;
    for (int h = 0; h < 2; ++h) {
      const int q = 2 * (l % 4) + h;
      // offset (m, n) of point q: 0 (-1,-1) 1 (-1,0) 2 (-1,1) 3 (0,-1) 4 (0,1) 5 (1,-1) 6 (1,0) 7 (1,1)
      const int m = q < 3 ? -1 : (q < 5 ? 0 : 1);
      const int nn = q < 3 ? q - 1 : (q == 3 ? -1 : (q == 4 ? 1 : q - 6));
      const bool diag = m != 0 && nn != 0;
      float2 c = c_scale(h == 0 ? box_muller(v.x, v.y) : box_muller(v.z, v.w), amp[diag ? 1 : 0] * a.scale);
      if (a.ar) {
        // Eq. 4 at (n df_p, m df_p): exp(-2 pi i (n sx + m sy) / (3^p N)), then Eq. 5
        double rev = -(nn * a.sx + m * a.sy) / (a.n * (p == 0 ? 3.0 : (p == 1 ? 9.0 : 27.0)));
        rev -= rint(rev);
        float sn, cs;
        sincos_rev(static_cast<float>(rev), &sn, &cs);
        const float2 old = out[8 * p + q];
        c = c_add(c_scale(c_mul(old, make_float2(cs, sn)), static_cast<float>(a.alpha)),
                  c_scale(c, static_cast<float>(sqrt(1.0 - a.alpha * a.alpha))));
      }
      coef[8 * p + q] = c;
    }
  }
  __syncthreads();
  if (l < 24) out[l] = l < 8 * a.levels ? coef[l] : make_float2(0.0f, 0.0f);
  if (l == 0) {
    float2 mean = make_float2(0.0f, 0.0f);
    for (int p = 0; p < a.levels; ++p) {
      const float2 e1 = a.mean_fac[p];
      const float2 em = make_float2(e1.x, -e1.y);
      const float2 one = make_float2(1.0f, 0.0f);
      int q = 0;
      for (int mm = -1; mm <= 1; ++mm)
        for (int nn = -1; nn <= 1; ++nn) {
          if (mm == 0 && nn == 0) continue;
          const float2 fy = mm < 0 ? em : (mm > 0 ? e1 : one);
          const float2 fx = nn < 0 ? em : (nn > 0 ? e1 : one);
          mean = c_add(mean, c_mul(coef[8 * p + q], c_mul(fy, fx)));
          ++q;
        }
    }
    out[24] = mean;
  }
}

__global__ __launch_bounds__(64) void sh_kernel(ShArgs a) { sh_body(a); }

// ---------------------------------------------------------------------------
// Spectrum evolution (Eq. 4 then Eq. 5), elementwise on bin pairs (k0, k1),
// (k0 + N/2, k1) that share one Philox block.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void evolve_kernel(EvolveArgs a) {
  const int n = a.n;
  const int64_t half = static_cast<int64_t>(n / 2) * n;  // a power of two
  const int64_t total = a.P * a.M * half;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int64_t js = idx >> (2 * a.log2n - 1);
  const int64_t rem = idx & (half - 1);
  const int k0 = static_cast<int>(rem >> a.log2n);
  const int k1 = static_cast<int>(rem & (n - 1));
  int64_t j;
  int s;
  if (js <= 0xFFFFFFFFll) {  // 32-bit division where it suffices
    const uint32_t js32 = static_cast<uint32_t>(js), m32 = static_cast<uint32_t>(a.M);
    j = js32 / m32;
    s = static_cast<int>(js32 - static_cast<uint32_t>(j) * m32);
  } else {
    j = js / a.M;
    s = static_cast<int>(js - j * a.M);
  }
  const uint4 v = philox4x32_10(
      noise_counter(static_cast<uint32_t>(rem), time_step(a), static_cast<uint32_t>(j), a.tag, static_cast<uint32_t>(s)),
      a.key0, a.key1);
  float2* base = a.spectra + js * static_cast<int64_t>(n) * n;
  const float amp = a.amp[s];
  const int kx = signed_bin(k1, n);
  const double inv_n = 1.0 / n;  // exact: n is a power of two
  for (int h = 0; h < 2; ++h) {
    const int kk0 = k0 + h * (n / 2);
    const int ky = signed_bin(kk0, n);
    const float w = psd_amp(ky * ky + kx * kx, amp, a.df2, a.inner, a.f02, a.q);
    const float2 nc = h == 0 ? box_muller(v.x, v.y) : box_muller(v.z, v.w);
    float2* p = base + static_cast<int64_t>(kk0) * n + k1;
    float2 out;
    if (a.init) {
      out = c_scale(nc, w);
    } else {
      double rev = -(static_cast<double>(kx) * a.sx + static_cast<double>(ky) * a.sy) * inv_n;
      rev -= rint(rev);
      float sn, cs;
      sincos_rev(static_cast<float>(rev), &sn, &cs);
      out = c_add(c_scale(c_mul(*p, make_float2(cs, sn)), a.alpha_f), c_scale(nc, a.blend * w));
    }
    if (kk0 == 0 && k1 == 0) out = make_float2(0.0f, 0.0f);
    *p = out;
  }
}

// ---------------------------------------------------------------------------
// Ensemble moments: Kahan-compensated sums of I and I^2 per pixel.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void stats_kernel(StatsArgs a) {
  const int64_t np = static_cast<int64_t>(a.n) * a.n;
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= np) return;
  float s1 = a.moments[p], c1 = a.moments[np + p];
  float s2 = a.moments[2 * np + p], c2 = a.moments[3 * np + p];
  const int C = moment_chunks(a.n);
  for (int c = 0; c < C; ++c) {
    const int64_t lo = c * a.batch / C, hi = (c + 1) * a.batch / C;
    if (lo == hi) continue;
    float ps1 = 0.0f, pc1 = 0.0f, ps2 = 0.0f, pc2 = 0.0f;
    // U loads in flight per thread; the sums stay in realization order
    constexpr int U = 16;
    int64_t b = lo;
    for (; b + U <= hi; b += U) {
      float2 u[U];
#pragma unroll
      for (int q = 0; q < U; ++q) u[q] = ld_s<true>(a.u + (b + q) * np + p);
#pragma unroll
      for (int q = 0; q < U; ++q) moment_add(ps1, pc1, ps2, pc2, u[q]);
    }
    for (; b < hi; ++b) moment_add(ps1, pc1, ps2, pc2, ld_s<true>(a.u + b * np + p));
    kahan_join(s1, c1, ps1, pc1);
    kahan_join(s2, c2, ps2, pc2);
  }
  a.moments[p] = s1;
  a.moments[np + p] = c1;
  a.moments[2 * np + p] = s2;
  a.moments[3 * np + p] = c2;
}

// ---------------------------------------------------------------------------
// Final row pass with the ensemble moments (Sec. 3.3).  The inverse row
// transform of each realization's spectral row is the output field: it is
// stored and, still in registers, added into the per-pixel moment sums, so
// the output planes are not read a second time.  A block is one row by C
// chunks of realizations (moment_chunks): thread group c transforms the
// realizations of chunk c in order into sums of its own, and the chunk sums
// are joined into the stored ones in chunk order through LDS.  The field is
// the plain final row pass's and the sums are the stats kernel's, bit for
// bit.  Groups past the end of their chunk transform a valid row and keep
// nothing, so every group passes the same barriers.
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(moment_chunks(N) * (N / kE)) void row_moments_kernel(RowArgs a, float* moments) {
  constexpr int T = N / kE;
  constexpr int C = moment_chunks(N);
  constexpr bool WV = T <= 64;  // each row's transform lives in one wavefront
  static_assert(2 * N <= 2 * RowLds::words(N), "a chunk's partial sums fit in its transform's LDS");
  __shared__ float2 smem[C * RowLds::words(N)];
  TURPY_LDS_INIT(smem);
  __shared__ float2 tw_lds[N];
  const int c = threadIdx.x / T;
  const int t = threadIdx.x % T;
  const RowLds lds{smem + c * RowLds::words(N)};
  const float2* tw = stage_twiddles<N>(tw_lds, a.tw);
  const size_t plane = static_cast<size_t>(N) * N;
  const size_t row_off = static_cast<size_t>(blockIdx.x) * N;
  const int64_t lo = c * a.R / C, hi = (c + 1) * a.R / C;
  const int64_t iters = (a.R + C - 1) / C;

  float s1[kE], c1[kE], s2[kE], c2[kE];
#pragma unroll
  for (int m = 0; m < kE; ++m) s1[m] = c1[m] = s2[m] = c2[m] = 0.0f;
  for (int64_t i = 0; i < iters; ++i) {
    const int64_t r = lo + i;
    const bool live = r < hi;
    const float2* src = a.in + (live ? r : a.R - 1) * a.in_stride + row_off;
    float2 x[kE];
#pragma unroll
    for (int m = 0; m < kE; ++m) x[m] = (src + t)[T * m];
    fft<N, kE, true, WV>(x, lds, t, tw);
    if (a.scale != 1.0f) {
#pragma unroll
      for (int m = 0; m < kE; ++m) x[m] = c_scale(x[m], a.scale);
    }
    if (live) {
      float2* dst = a.out + r * plane + row_off;
#pragma unroll
      for (int m = 0; m < kE; ++m) (dst + t)[T * m] = x[m];
#pragma unroll
      for (int m = 0; m < kE; ++m) moment_add(s1[m], c1[m], s2[m], c2[m], x[m]);
    }
  }

  // non-empty chunks, bit q for chunk q (C <= 64)
  uint64_t filled = 0;
  for (int q = 0; q < C; ++q)
    if (q * a.R / C != (q + 1) * a.R / C) filled |= uint64_t(1) << q;
  float* part = reinterpret_cast<float*>(smem);  // [C][2][N]: one moment's s and c per chunk
  for (int k = 0; k < 2; ++k) {
    __syncthreads();  // the transforms' (or the last round's) LDS reads are done
#pragma unroll
    for (int m = 0; m < kE; ++m) {
      part[(2 * c) * N + t + T * m] = k ? s2[m] : s1[m];
      part[(2 * c + 1) * N + t + T * m] = k ? c2[m] : c1[m];
    }
    __syncthreads();
    for (int p = threadIdx.x; p < N; p += C * T) {
      float* ms = moments + static_cast<size_t>(2 * k) * plane + row_off + p;
      float s = ms[0], cc = ms[plane];
      for (int q = 0; q < C; ++q)
        if (filled >> q & 1) kahan_join(s, cc, part[(2 * q) * N + p], part[(2 * q + 1) * N + p]);
      ms[0] = s;
      ms[plane] = cc;
    }
  }
}

// ---------------------------------------------------------------------------
// Output check of TURPY_CHECK_FINITE plans: the number of NaN and infinite
// values among `count` floats, added to *counter (cleared first by the
// one-thread kernel before it).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1) void clear_counter_kernel(unsigned long long* counter) { *counter = 0; }

__global__ __launch_bounds__(256) void nonfinite_kernel(const float* x, int64_t count, unsigned long long* counter) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  unsigned bad = 0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += stride)
    bad += __builtin_isfinite(x[i]) ? 0u : 1u;
  for (int off = 32; off > 0; off >>= 1) bad += __shfl_xor(bad, off);
  if ((threadIdx.x & 63) == 0 && bad) atomicAdd(counter, static_cast<unsigned long long>(bad));
}

template <int NT>
__device__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

template <int NT>
__device__ double block_max(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Mean intensity of pixel p from the compensated sums, rounded to FP32: the
// quantity the power-cutoff region of Sec. 4.1 is decided on.
__device__ __forceinline__ float mean_intensity(const FinalizeArgs& a, int64_t p, int64_t np) {
  return static_cast<float>((static_cast<double>(a.moments[p]) - a.moments[np + p]) / a.count);
}

__global__ __launch_bounds__(1024) void finalize_kernel(FinalizeArgs a) {
  constexpr int NT = 1024;
  __shared__ double red[NT];
  TURPY_LDS_INIT(red);
  const int n = a.n;
  const int64_t np = static_cast<int64_t>(n) * n;
  double m1_sum = 0, r2m1 = 0, m1_max = 0, m1f_sum = 0;
  for (int64_t p = threadIdx.x; p < np; p += NT) {
    const int i0 = static_cast<int>(p / n), i1 = static_cast<int>(p % n);
    const double m1 = (static_cast<double>(a.moments[p]) - a.moments[np + p]) / a.count;
    const double m2 = (static_cast<double>(a.moments[2 * np + p]) - a.moments[3 * np + p]) / a.count;
    if (a.si_map) a.si_map[p] = static_cast<float>(m2 / (m1 * m1) - 1.0);
    const double x = (i1 - n / 2) * a.dx, y = (i0 - n / 2) * a.dx;
    m1_sum += m1;
    r2m1 += (x * x + y * y) * m1;
    m1_max = fmax(m1_max, m1);
    m1f_sum += mean_intensity(a, p, np);
  }
  m1_sum = block_sum<NT>(m1_sum, red);
  r2m1 = block_sum<NT>(r2m1, red);
  m1_max = block_max<NT>(m1_max, red);
  m1f_sum = block_sum<NT>(m1f_sum, red);
  // Power-cutoff region (Sec. 4.1): the largest threshold t whose pixels
  // m1 >= t hold power_fraction of the total, by bisection over the ordered
  // bit patterns of non-negative FP32 values (exact after 32 halvings).
  uint32_t thr_bits = 0;
  if (a.power_fraction > 0) {
    const double target = a.power_fraction * m1f_sum;
    uint32_t lo = 0, hi = 0x7F800000u;  // S(lo) >= target; hi: +inf, above every finite m1
    while (hi - lo > 1u) {
      const uint32_t mid = lo + (hi - lo) / 2u;
      const float t = __uint_as_float(mid);
      double s = 0;
      for (int64_t p = threadIdx.x; p < np; p += NT) {
        const float m = mean_intensity(a, p, np);
        if (m >= t) s += m;
      }
      s = block_sum<NT>(s, red);
      if (s >= target) lo = mid; else hi = mid;
    }
    thr_bits = lo;
  }
  const float thr = __uint_as_float(thr_bits);
  double si_sum = 0, w_sum = 0;
  for (int64_t p = threadIdx.x; p < np; p += NT) {
    bool in;
    if (a.power_fraction > 0) {
      in = mean_intensity(a, p, np) >= thr;
    } else {
      const int i0 = static_cast<int>(p / n), i1 = static_cast<int>(p % n);
      in = abs(i0 - n / 2) < n / 4 && abs(i1 - n / 2) < n / 4;
    }
    if (in) {
      const double m1 = (static_cast<double>(a.moments[p]) - a.moments[np + p]) / a.count;
      const double m2 = (static_cast<double>(a.moments[2 * np + p]) - a.moments[3 * np + p]) / a.count;
      const double w = a.weight ? static_cast<double>(a.weight[p]) : 1.0;
      si_sum += w * (m2 / (m1 * m1) - 1.0);
      w_sum += w;
    }
  }
  si_sum = block_sum<NT>(si_sum, red);
  w_sum = block_sum<NT>(w_sum, red);
  const double cut = exp(-2.0) * m1_max;
  double s0 = 0, sx = 0, sxx = 0, sy = 0, sxy = 0;
  for (int64_t p = threadIdx.x; p < np; p += NT) {
    const double m1 = (static_cast<double>(a.moments[p]) - a.moments[np + p]) / a.count;
    if (m1 >= cut && m1 > 0) {
      const int i0 = static_cast<int>(p / n), i1 = static_cast<int>(p % n);
      const double x = (i1 - n / 2) * a.dx, y = (i0 - n / 2) * a.dx;
      const double r2 = x * x + y * y, l = log(m1);
      s0 += 1;
      sx += r2;
      sxx += r2 * r2;
      sy += l;
      sxy += r2 * l;
    }
  }
  s0 = block_sum<NT>(s0, red);
  sx = block_sum<NT>(sx, red);
  sxx = block_sum<NT>(sxx, red);
  sy = block_sum<NT>(sy, red);
  sxy = block_sum<NT>(sxy, red);
  if (threadIdx.x == 0) {
    const double den = s0 * sxx - sx * sx;
    const double slope = den != 0 ? (s0 * sxy - sx * sy) / den : 0.0;
    a.summary[0] = w_sum != 0 ? si_sum / w_sum : 0.0;
    a.summary[1] = m1_sum > 0 ? sqrt(2.0 * r2m1 / m1_sum) : 0.0;
    a.summary[2] = slope < 0 ? sqrt(-2.0 / slope) : __builtin_huge_val();
    a.summary[3] = a.count;
    a.summary[4] = si_sum;
    a.summary[5] = w_sum;
    a.summary[6] = a.power_fraction > 0 ? static_cast<double>(thr) : 0.0;
    a.summary[7] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// The complex normals of a spectrum on their own (Eq. S16's N_c, with the
// counter layout of the synthesis): one Philox block per bin pair (k0, k1),
// (k0 + N/2, k1) of pair j.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void noise_kernel(NoiseArgs a) {
  const int n = a.n;
  const int64_t half = static_cast<int64_t>(n / 2) * n;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= a.pairs * half) return;
  const int64_t j = idx / half;
  const uint32_t e = static_cast<uint32_t>(idx - j * half);  // k0 * N + k1, k0 < N/2
  const uint4 v = philox4x32_10(noise_counter(e, a.t, static_cast<uint32_t>(j), a.tag, a.screen), a.key0, a.key1);
  float2* out = a.out + j * static_cast<int64_t>(n) * n;
  out[e] = box_muller(v.x, v.y);
  out[e + half] = box_muller(v.z, v.w);
}

// ---------------------------------------------------------------------------
// Sum of R planes into one (the gradient of a source shared by every
// realization): each thread owns one element and adds the planes in order with
// Kahan compensation, sixteen non-temporal loads in flight.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void sum_planes_kernel(const float2* in, int64_t R, int64_t count, float2* out) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= count) return;
  float2 s = make_float2(0.0f, 0.0f), c = make_float2(0.0f, 0.0f);
  auto add = [&](float2 v) {
    const float yx = v.x - c.x, yy = v.y - c.y;
    const float tx = s.x + yx, ty = s.y + yy;
    c.x = (tx - s.x) - yx;
    c.y = (ty - s.y) - yy;
    s.x = tx;
    s.y = ty;
  };
  constexpr int U = 16;
  int64_t r = 0;
  for (; r + U <= R; r += U) {
    float2 v[U];
#pragma unroll
    for (int q = 0; q < U; ++q) v[q] = ld_s<true>(in + (r + q) * count + p);
#pragma unroll
    for (int q = 0; q < U; ++q) add(v[q]);
  }
  for (; r < R; ++r) add(ld_s<true>(in + r * count + p));
  out[p] = s;
}

__global__ __launch_bounds__(256) void copy_kernel(const float2* in, int64_t in_stride, float2* out,
                                                   int64_t count, int64_t R) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= count * R) return;
  const int64_t r = idx / count, p = idx % count;
  out[idx] = in[r * in_stride + p];
}

// Occupancy hints of the screen row passes (minimum waves per SIMD the
// register allocation must allow): 3 by default; the tuner also times 2 and 4
// for N >= 256.
constexpr int kRowWaves = 3;
constexpr bool row_waves_built(int n, int w) { return w == kRowWaves || (n >= 256 && (w == 2 || w == 4)); }

// A forward screen pass of a single realization where the relay schedule is
// not built (N > 1024): the pair schedule would leave half of every block
// transforming rows nobody keeps, so one group of threads per row takes it
// (serving mix: the 252 instances at N = 2048 274 -> 213 ms forward; all 4096
// forward + adjoint with checkpoints 3.11 -> 2.94 s).  At N <= 1024 the relay
// schedule stays, and in the adjoint the pair schedule (one group per row
// measured 3.11 -> 3.28 s there).
template <int N>
constexpr bool solo_forward(int64_t R, int backward, const void* ckpt) {
  (void)ckpt;
  return N > 1024 && R == 1 && !backward;
}

// The relay kernel for forward passes with synthesised screens and no
// checkpoint output, where its workers are whole waves and it keeps three
// waves per SIMD (N <= 1024); false: not launched.  With checkpoint writes
// and in the adjoint the pair schedule measured as fast or faster.
// A hint not built for N launches the default one (the host refuses such
// choices before they reach a plan).
template <int N, int W>
void relay_launch_w(const RowArgs& a, int64_t pairs, hipStream_t s) {
  constexpr int WB = row_waves_built(N, W) ? W : kRowWaves;
  const dim3 grid(N / (2 * relay_rows<N>()), static_cast<uint32_t>(pairs));
  hipLaunchKernelGGL((row_relay_kernel<N, WB>), grid, dim3(relay_block<N>()), 0, s, a);
}

template <int N>
bool relay_launch(const RowArgs& a, int64_t pairs, hipStream_t s) {
  if constexpr (!relay_fits<N>() || N > 1024) {
    return false;
  } else {
    if (a.screen_mode != ROW_SCRATCH || a.backward || a.conj_tables || a.ckpt_out || a.pre) return false;
    switch (a.waves ? a.waves : kRowWaves) {
      case 2: relay_launch_w<N, 2>(a, pairs, s); break;
      case 4: relay_launch_w<N, 4>(a, pairs, s); break;
      default: relay_launch_w<N, kRowWaves>(a, pairs, s); break;
    }
    return true;
  }
}

template <int N, int SCREEN, bool BWD, int W>
void pair_launch_w(const RowArgs& a, int64_t pairs, hipStream_t s) {
  constexpr int WB = row_waves_built(N, W) && SCREEN == ROW_SCRATCH ? W : kRowWaves;
  constexpr int GP = pair_rows<N>();
  const dim3 pgrid(N / GP, static_cast<uint32_t>(pairs));
  hipLaunchKernelGGL((row_pair_kernel<N, SCREEN, BWD, WB>), pgrid, dim3(pair_block<N>()), 0, s, a);
}

template <int N, int SCREEN, bool BWD>
void pair_launch(const RowArgs& a, int64_t pairs, hipStream_t s) {
  const int w = SCREEN == ROW_SCRATCH && a.waves ? a.waves : kRowWaves;
  if (w == 2) pair_launch_w<N, SCREEN, BWD, 2>(a, pairs, s);
  else if (w == 4) pair_launch_w<N, SCREEN, BWD, 4>(a, pairs, s);
  else pair_launch_w<N, SCREEN, BWD, kRowWaves>(a, pairs, s);
}

template <int N>
hipError_t row_launch(const RowArgs& a, int64_t pairs, hipStream_t s) {
  constexpr int G = row_groups<N>();
  dim3 grid(N / G, static_cast<uint32_t>(pairs));
  dim3 block(row_block<N>());
  if (a.screen_mode == ROW_NO_SCREEN)
    hipLaunchKernelGGL((row_pass_kernel<N, ROW_NO_SCREEN, false>), grid, block, 0, s, a);
  else if (a.phase_out || (pair_rows<N>() * (N / kE)) % 64 != 0 || solo_forward<N>(a.R, a.backward, a.ckpt_out)) {
    // screen output, grids too small for the two halves to sit in separate
    // waves, or a single realization on the pair schedule
    if (a.screen_mode == ROW_SCRATCH && !a.backward)
      hipLaunchKernelGGL((row_pass_kernel<N, ROW_SCRATCH, false>), grid, block, 0, s, a);
    else if (a.screen_mode == ROW_SCRATCH)
      hipLaunchKernelGGL((row_pass_kernel<N, ROW_SCRATCH, true>), grid, block, 0, s, a);
    else if (!a.backward)
      hipLaunchKernelGGL((row_pass_kernel<N, ROW_MATERIALIZED, false>), grid, block, 0, s, a);
    else
      hipLaunchKernelGGL((row_pass_kernel<N, ROW_MATERIALIZED, true>), grid, block, 0, s, a);
  } else if (relay_launch<N>(a, pairs, s)) {
    // synthesised screens on the relay schedule
  } else {
    if (a.screen_mode == ROW_SCRATCH && !a.backward) pair_launch<N, ROW_SCRATCH, false>(a, pairs, s);
    else if (a.screen_mode == ROW_SCRATCH) pair_launch<N, ROW_SCRATCH, true>(a, pairs, s);
    else if (!a.backward) pair_launch<N, ROW_MATERIALIZED, false>(a, pairs, s);
    else pair_launch<N, ROW_MATERIALIZED, true>(a, pairs, s);
  }
  return hipGetLastError();
}

// Second-pass radices built for the column pass and the synthesis: the
// default plan, and for N = 512..2048 the alternatives the tuner times.
constexpr bool radix_built(int n, int r2) {
  return r2 == 0 || ((n == 512 || n == 1024) && (r2 == 8 || r2 == 4)) || (n == 2048 && r2 == 8);
}

template <int N, int K, int R2SEL>
hipError_t col_launch_kr(const ColArgs& a, hipStream_t s) {
  if constexpr (!strip_fits<N, K>() || !radix_built(N, R2SEL)) {
    return hipErrorInvalidValue;
  } else {
    const uint64_t blocks = static_cast<uint64_t>(N / K) * a.R;
    const dim3 grid(static_cast<uint32_t>(blocks)), block(K * (N / kE));
    if (!a.angular)
      hipLaunchKernelGGL((col_pass_kernel<N, TF_FRESNEL_ONLY, K, R2SEL>), grid, block, 0, s, a);
    else if (a.as_table)
      hipLaunchKernelGGL((col_pass_kernel<N, TF_AS_TABLE, K, R2SEL>), grid, block, 0, s, a);
    else
      hipLaunchKernelGGL((col_pass_kernel<N, TF_AS_FP32, K, R2SEL>), grid, block, 0, s, a);
    return hipGetLastError();
  }
}

template <int N, int K>
hipError_t col_launch_k(const ColArgs& a, hipStream_t s) {
  switch (a.radix) {
    case 0: return col_launch_kr<N, K, 0>(a, s);
    case 4: return col_launch_kr<N, K, 4>(a, s);
    case 8: return col_launch_kr<N, K, 8>(a, s);
    default: return hipErrorInvalidValue;
  }
}

// Strip width a.width (4, 8 or 16 columns per block), or the built-in choice
// for N when a.width is 0; second-pass radix a.radix (0: the default plan).
template <int N>
hipError_t col_launch(const ColArgs& a, hipStream_t s) {
  switch (a.width ? a.width : col_width<N>()) {
    case 4: return col_launch_k<N, 4>(a, s);
    case 8: return col_launch_k<N, 8>(a, s);
    case 16: return col_launch_k<N, 16>(a, s);
    default: return hipErrorInvalidValue;
  }
}

template <int N, int K, int R2SEL>
hipError_t synth_launch_kr(const SynthArgs& a, hipStream_t s) {
  if constexpr (!strip_fits<N, K>() || !radix_built(N, R2SEL)) {
    return hipErrorInvalidValue;
  } else {
    const uint64_t blocks = static_cast<uint64_t>(N / K) * a.P;
    hipLaunchKernelGGL((synth_col_kernel<N, K, R2SEL>), dim3(static_cast<uint32_t>(blocks)), dim3(K * (N / kE)), 0, s,
                       a);
    return hipGetLastError();
  }
}

template <int N, int K>
hipError_t synth_launch_k(const SynthArgs& a, hipStream_t s) {
  switch (a.radix) {
    case 0: return synth_launch_kr<N, K, 0>(a, s);
    case 4: return synth_launch_kr<N, K, 4>(a, s);
    case 8: return synth_launch_kr<N, K, 8>(a, s);
    default: return hipErrorInvalidValue;
  }
}

template <int N>
hipError_t synth_launch(const SynthArgs& a, hipStream_t s) {
  switch (a.width ? a.width : synth_width<N>()) {
    case 4: return synth_launch_k<N, 4>(a, s);
    case 8: return synth_launch_k<N, 8>(a, s);
    case 16: return synth_launch_k<N, 16>(a, s);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// Grouped launches (uneven batches): the kernels above over many instances,
// each block taking its instance's record and adding the call's bases.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ T* rebase(char* base, T* off) {
  return reinterpret_cast<T*>(base + reinterpret_cast<uintptr_t>(off));
}
template <class T>
__device__ __forceinline__ const T* rebase(const char* base, const T* off) {
  return reinterpret_cast<const T*>(base + reinterpret_cast<uintptr_t>(off));
}

// The instance's key: the call's seed plus the seed offset in the record.
__device__ __forceinline__ void group_key(const GroupCall& g, uint32_t* k0, uint32_t* k1) {
  const uint64_t s = g.seed + ((static_cast<uint64_t>(*k1) << 32) | *k0);
  *k0 = static_cast<uint32_t>(s);
  *k1 = static_cast<uint32_t>(s >> 32);
}

__device__ __forceinline__ RowArgs row_record(const RowArgs* tab, uint32_t i, const GroupCall& g) {
  RowArgs a = tab[i];
  const char* ws = g.ws;
  a.in = rebase(g.in, a.in);
  a.out = rebase(g.out, a.out);
  a.scratch = rebase(ws, a.scratch);
  a.sh = rebase(ws, a.sh);
  a.ckpt_out = g.ck ? rebase(g.ck, a.ckpt_out) : nullptr;
  return a;
}

// The adjoint's screen passes read the checkpoints and write dL/dphi.
__device__ __forceinline__ RowArgs row_record_bwd(const RowArgs* tab, uint32_t i, const GroupCall& g) {
  RowArgs a = tab[i];
  const char* ws = g.ws;
  const char* ck = g.ck;
  a.in = rebase(g.in, a.in);
  a.out = rebase(g.out, a.out);
  a.scratch = rebase(ws, a.scratch);
  a.sh = rebase(ws, a.sh);
  a.ckpt_out = nullptr;
  a.ckpt_in = rebase(ck, a.ckpt_in);
  a.grad_screens = g.gs ? rebase(g.gs, a.grad_screens) : nullptr;
  return a;
}

template <int N, int SCREEN>
__global__ __launch_bounds__(row_block<N>()) void row_pass_group_kernel(const RowArgs* tab, GroupCall g) {
  row_pass_body<N, SCREEN, false>(row_record(tab, blockIdx.z, g));
}

template <int N>
__global__ __launch_bounds__(row_block<N>()) void row_pass_group_bwd_kernel(const RowArgs* tab, GroupCall g) {
  row_pass_body<N, ROW_SCRATCH, true>(row_record_bwd(tab, blockIdx.z, g));
}

template <int N>
__global__ __launch_bounds__(pair_block<N>()) __attribute__((amdgpu_waves_per_eu(kRowWaves, 0)))
void row_pair_group_bwd_kernel(const RowArgs* tab, GroupCall g) {
  row_pair_body<N, ROW_SCRATCH, true>(row_record_bwd(tab, blockIdx.z, g));
}

template <int N>
__global__ __launch_bounds__(pair_block<N>()) __attribute__((amdgpu_waves_per_eu(kRowWaves, 0)))
void row_pair_group_kernel(const RowArgs* tab, GroupCall g) {
  row_pair_body<N, ROW_SCRATCH, false>(row_record(tab, blockIdx.z, g));
}

template <int N>
__global__ __launch_bounds__(relay_block<N>()) __attribute__((amdgpu_waves_per_eu(kRowWaves, 0)))
void row_relay_group_kernel(const RowArgs* tab, GroupCall g) {
  row_relay_body<N>(row_record(tab, blockIdx.z, g));
}

template <int N, int ANGULAR, int R2SEL>
__global__ __launch_bounds__(col_width<N>() * (N / kE)) void col_pass_group_kernel(const ColArgs* tab, GroupCall g) {
  ColArgs a = tab[blockIdx.y];
  a.in = rebase(g.in, a.in);
  a.out = rebase(g.out, a.out);
  col_pass_body<N, ANGULAR, col_width<N>(), R2SEL>(a);
}

template <int N, int R2SEL>
__global__ __launch_bounds__(synth_width<N>() * (N / kE)) void synth_group_kernel(const SynthArgs* tab, GroupCall g) {
  SynthArgs a = tab[blockIdx.y];
  a.scratch = rebase(g.ws, a.scratch);
  group_key(g, &a.key0, &a.key1);
  a.t = g.t;
  a.t_dev = g.t_dev;
  synth_col_body<N, synth_width<N>(), R2SEL>(a);
}

__global__ __launch_bounds__(64) void sh_group_kernel(const ShArgs* tab, GroupCall g) {
  ShArgs a = tab[blockIdx.z];
  if (blockIdx.y >= static_cast<uint32_t>(a.M) || a.levels == 0) return;  // uniform over the block
  a.sh = rebase(g.ws, a.sh);
  group_key(g, &a.key0, &a.key1);
  a.t = g.t;
  a.t_dev = g.t_dev;
  sh_body(a);
}

// The row passes of a group, chosen as row_launch chooses them for one
// instance (the records share the kernel-deciding fields).
template <int N>
hipError_t row_group_launch(const RowArgs& proto, const RowArgs* tab, uint32_t count, int64_t pairs,
                            const GroupCall& g, hipStream_t s) {
  constexpr int G = row_groups<N>();
  const uint32_t P = static_cast<uint32_t>(pairs);
  // halves that are not whole waves, or a single realization on the pair
  // schedule: one group of threads per row (as row_launch chooses)
  const bool small = (pair_rows<N>() * (N / kE)) % 64 != 0 || solo_forward<N>(proto.R, proto.backward, g.ck);
  if (proto.phase_out) return hipErrorInvalidValue;
  if (proto.screen_mode == ROW_NO_SCREEN) {
    hipLaunchKernelGGL((row_pass_group_kernel<N, ROW_NO_SCREEN>), dim3(N / G, P, count), dim3(row_block<N>()), 0,
                       s, tab, g);
  } else if (proto.screen_mode != ROW_SCRATCH) {
    return hipErrorInvalidValue;
  } else if (proto.backward) {
    if (small)
      hipLaunchKernelGGL((row_pass_group_bwd_kernel<N>), dim3(N / G, P, count), dim3(row_block<N>()), 0, s, tab, g);
    else
      hipLaunchKernelGGL((row_pair_group_bwd_kernel<N>), dim3(N / pair_rows<N>(), P, count), dim3(pair_block<N>()),
                         0, s, tab, g);
  } else if (small) {
    hipLaunchKernelGGL((row_pass_group_kernel<N, ROW_SCRATCH>), dim3(N / G, P, count), dim3(row_block<N>()), 0, s,
                       tab, g);
  } else {
    bool relay = false;
    if constexpr (relay_fits<N>() && N <= 1024) {
      if (!g.ck && !proto.conj_tables && !proto.pre) {
        hipLaunchKernelGGL((row_relay_group_kernel<N>), dim3(N / (2 * relay_rows<N>()), P, count),
                           dim3(relay_block<N>()), 0, s, tab, g);
        relay = true;
      }
    }
    if (!relay)
      hipLaunchKernelGGL((row_pair_group_kernel<N>), dim3(N / pair_rows<N>(), P, count), dim3(pair_block<N>()), 0, s,
                         tab, g);
  }
  return hipGetLastError();
}

template <int N, int R2SEL>
hipError_t col_group_launch_r(const ColArgs& proto, const ColArgs* tab, uint32_t count, const GroupCall& g,
                              hipStream_t s) {
  if constexpr (!radix_built(N, R2SEL)) {
    return hipErrorInvalidValue;
  } else {
    const dim3 grid(static_cast<uint32_t>((N / col_width<N>()) * proto.R), count), block(col_width<N>() * (N / kE));
    if (!proto.angular)
      hipLaunchKernelGGL((col_pass_group_kernel<N, TF_FRESNEL_ONLY, R2SEL>), grid, block, 0, s, tab, g);
    else if (proto.as_table)
      hipLaunchKernelGGL((col_pass_group_kernel<N, TF_AS_TABLE, R2SEL>), grid, block, 0, s, tab, g);
    else
      hipLaunchKernelGGL((col_pass_group_kernel<N, TF_AS_FP32, R2SEL>), grid, block, 0, s, tab, g);
    return hipGetLastError();
  }
}

template <int N>
hipError_t col_group_launch(const ColArgs& proto, const ColArgs* tab, uint32_t count, const GroupCall& g,
                            hipStream_t s) {
  switch (proto.radix) {
    case 0: return col_group_launch_r<N, 0>(proto, tab, count, g, s);
    case 4: return col_group_launch_r<N, 4>(proto, tab, count, g, s);
    case 8: return col_group_launch_r<N, 8>(proto, tab, count, g, s);
    default: return hipErrorInvalidValue;
  }
}

template <int N, int R2SEL>
hipError_t synth_group_launch_r(const SynthArgs& proto, const SynthArgs* tab, uint32_t count, const GroupCall& g,
                                hipStream_t s) {
  if constexpr (!radix_built(N, R2SEL)) {
    return hipErrorInvalidValue;
  } else {
    const dim3 grid(static_cast<uint32_t>((N / synth_width<N>()) * proto.P), count);
    hipLaunchKernelGGL((synth_group_kernel<N, R2SEL>), grid, dim3(synth_width<N>() * (N / kE)), 0, s, tab, g);
    return hipGetLastError();
  }
}

template <int N>
hipError_t synth_group_launch(const SynthArgs& proto, const SynthArgs* tab, uint32_t count, const GroupCall& g,
                              hipStream_t s) {
  if (proto.spectra || proto.evolve) return hipErrorInvalidValue;  // synthesised screens only
  switch (proto.radix) {
    case 0: return synth_group_launch_r<N, 0>(proto, tab, count, g, s);
    case 4: return synth_group_launch_r<N, 4>(proto, tab, count, g, s);
    case 8: return synth_group_launch_r<N, 8>(proto, tab, count, g, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

#define TURPY_DISPATCH_N(n, FN, ...)            \
  switch (n) {                                  \
    case 16: return FN<16>(__VA_ARGS__);        \
    case 32: return FN<32>(__VA_ARGS__);        \
    case 64: return FN<64>(__VA_ARGS__);        \
    case 128: return FN<128>(__VA_ARGS__);      \
    case 256: return FN<256>(__VA_ARGS__);      \
    case 512: return FN<512>(__VA_ARGS__);      \
    case 1024: return FN<1024>(__VA_ARGS__);    \
    case 2048: return FN<2048>(__VA_ARGS__);    \
    default: return hipErrorInvalidValue;       \
  }

hipError_t launch_row(int n, const RowArgs& a, int64_t pairs, hipStream_t s) {
  TURPY_DISPATCH_N(n, row_launch, a, pairs, s)
}
template <int N>
hipError_t row_moments_launch(const RowArgs& a, float* moments, hipStream_t s) {
  hipLaunchKernelGGL(row_moments_kernel<N>, dim3(N), dim3(moment_chunks(N) * (N / kE)), 0, s, a, moments);
  return hipGetLastError();
}
hipError_t launch_row_moments(int n, const RowArgs& a, float* moments, hipStream_t s) {
  TURPY_DISPATCH_N(n, row_moments_launch, a, moments, s)
}
hipError_t launch_col(int n, const ColArgs& a, hipStream_t s) { TURPY_DISPATCH_N(n, col_launch, a, s) }
hipError_t launch_synth(int n, const SynthArgs& a, hipStream_t s) { TURPY_DISPATCH_N(n, synth_launch, a, s) }

hipError_t launch_row_group(int n, const RowArgs& proto, const RowArgs* tab, uint32_t count, int64_t pairs,
                            const GroupCall& g, hipStream_t s) {
  TURPY_DISPATCH_N(n, row_group_launch, proto, tab, count, pairs, g, s)
}
hipError_t launch_col_group(int n, const ColArgs& proto, const ColArgs* tab, uint32_t count, const GroupCall& g,
                            hipStream_t s) {
  TURPY_DISPATCH_N(n, col_group_launch, proto, tab, count, g, s)
}
hipError_t launch_synth_group(int n, const SynthArgs& proto, const SynthArgs* tab, uint32_t count,
                              const GroupCall& g, hipStream_t s) {
  TURPY_DISPATCH_N(n, synth_group_launch, proto, tab, count, g, s)
}
hipError_t launch_sh_group(const ShArgs* tab, uint32_t count, int64_t pairs, int max_screens, const GroupCall& g,
                           hipStream_t s) {
  hipLaunchKernelGGL(sh_group_kernel, dim3(static_cast<uint32_t>(pairs), static_cast<uint32_t>(max_screens), count),
                     dim3(64), 0, s, tab, g);
  return hipGetLastError();
}

hipError_t launch_sh(const ShArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(sh_kernel, dim3(static_cast<uint32_t>(a.P), a.M), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_evolve(const EvolveArgs& a, hipStream_t s) {
  const int64_t total = a.P * a.M * static_cast<int64_t>(a.n / 2) * a.n;
  hipLaunchKernelGGL(evolve_kernel, dim3(static_cast<uint32_t>((total + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_stats(const StatsArgs& a, hipStream_t s) {
  const int64_t np = static_cast<int64_t>(a.n) * a.n;
  hipLaunchKernelGGL(stats_kernel, dim3(static_cast<uint32_t>((np + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_nonfinite(const float* x, int64_t count, unsigned long long* counter, hipStream_t s) {
  hipLaunchKernelGGL(clear_counter_kernel, dim3(1), dim3(1), 0, s, counter);
  const int64_t blocks = std::min<int64_t>((count + 255) / 256, 8192);
  hipLaunchKernelGGL(nonfinite_kernel, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, s, x, count, counter);
  return hipGetLastError();
}

hipError_t launch_finalize(const FinalizeArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(1024), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_noise(const NoiseArgs& a, hipStream_t s) {
  const int64_t total = a.pairs * static_cast<int64_t>(a.n / 2) * a.n;
  hipLaunchKernelGGL(noise_kernel, dim3(static_cast<uint32_t>((total + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_sum_planes(const float2* in, int64_t R, int64_t count, float2* out, hipStream_t s) {
  hipLaunchKernelGGL(sum_planes_kernel, dim3(static_cast<uint32_t>((count + 255) / 256)), dim3(256), 0, s, in, R,
                     count, out);
  return hipGetLastError();
}

hipError_t launch_copy(const float2* in, int64_t in_stride, float2* out, int64_t count, int64_t R,
                       hipStream_t s) {
  const int64_t total = count * R;
  hipLaunchKernelGGL(copy_kernel, dim3(static_cast<uint32_t>((total + 255) / 256)), dim3(256), 0, s, in,
                     in_stride, out, count, R);
  return hipGetLastError();
}

}  // namespace turpy
