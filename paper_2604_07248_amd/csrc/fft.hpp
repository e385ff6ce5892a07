// Stockham autosort FFT building blocks for gfx950.
//
// A length-N transform is carried by a group of T = N / E threads; thread t
// holds E elements in registers, element slot m holding index t + T*m (the
// "strided" layout).  Every pass reads its inputs in that layout, multiplies
// by the pass twiddles, does a radix-R DFT in registers and, except for the
// last pass, scatters its outputs to LDS at their Stockham positions; after a
// barrier the next pass reads the strided layout back.  The last pass leaves
// its outputs in registers, already in the strided layout and in natural
// frequency order, so a forward transform, a pointwise multiply and an inverse
// transform chain without an LDS round trip between them.
//
// Radix plan for E = 16: first pass radix 16 (no twiddles), second pass radix
// R2 (default min(16, N/16)) at sub-length 16, third pass radix N/(16 R2) at
// sub-length 16 R2.
#pragma once

#include "device_common.hpp"

namespace turpy {

// exp(-+ i theta) with (c, s) = (cos theta, sin theta); forward uses exp(-i theta).
template <bool INV>
__device__ __forceinline__ float2 c_rot(float2 a, float c, float s) {
  const float sn = INV ? s : -s;
  return make_float2(a.x * c - a.y * sn, a.x * sn + a.y * c);
}
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 c_quarter(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <bool INV>
__device__ __forceinline__ void dft2(float2& a, float2& b) {
  const float2 t = a;
  a = c_add(t, b);
  b = c_sub(t, b);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  const float2 t0 = c_add(a0, a2), t1 = c_sub(a0, a2);
  const float2 t2 = c_add(a1, a3), t3 = c_quarter<INV>(c_sub(a1, a3));
  a0 = c_add(t0, t2);
  a2 = c_sub(t0, t2);
  a1 = c_add(t1, t3);
  a3 = c_sub(t1, t3);
}

constexpr float kC8 = 0.70710678118654752f;   // cos(pi/4)
constexpr float kC16 = 0.92387953251128674f;  // cos(pi/8)
constexpr float kS16 = 0.38268343236508977f;  // sin(pi/8)

// radix-8 as 2 x 4: index n = 2 n1 + n2, output k = k1 + 4 k2
template <bool INV>
__device__ __forceinline__ void dft8(float2* v) {
  float2 a0 = v[0], a1 = v[2], a2 = v[4], a3 = v[6];
  float2 b0 = v[1], b1 = v[3], b2 = v[5], b3 = v[7];
  dft4<INV>(a0, a1, a2, a3);
  dft4<INV>(b0, b1, b2, b3);
  b1 = c_rot<INV>(b1, kC8, kC8);
  b2 = c_quarter<INV>(b2);
  b3 = c_rot<INV>(b3, -kC8, kC8);
  v[0] = c_add(a0, b0); v[4] = c_sub(a0, b0);
  v[1] = c_add(a1, b1); v[5] = c_sub(a1, b1);
  v[2] = c_add(a2, b2); v[6] = c_sub(a2, b2);
  v[3] = c_add(a3, b3); v[7] = c_sub(a3, b3);
}

// radix-16 as 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2; inner twiddles W16^(n2 k1)
template <bool INV>
__device__ __forceinline__ void dft16(float2* v) {
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft4<INV>(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
  // A[n2][k1] sits in v[4*k1 + n2]
  v[4 * 1 + 1] = c_rot<INV>(v[4 * 1 + 1], kC16, kS16);   // W^1
  v[4 * 2 + 1] = c_rot<INV>(v[4 * 2 + 1], kC8, kC8);     // W^2
  v[4 * 3 + 1] = c_rot<INV>(v[4 * 3 + 1], kS16, kC16);   // W^3
  v[4 * 1 + 2] = c_rot<INV>(v[4 * 1 + 2], kC8, kC8);     // W^2
  v[4 * 2 + 2] = c_quarter<INV>(v[4 * 2 + 2]);           // W^4
  v[4 * 3 + 2] = c_rot<INV>(v[4 * 3 + 2], -kC8, kC8);    // W^6
  v[4 * 1 + 3] = c_rot<INV>(v[4 * 1 + 3], kS16, kC16);   // W^3
  v[4 * 2 + 3] = c_rot<INV>(v[4 * 2 + 3], -kC8, kC8);    // W^6
  v[4 * 3 + 3] = c_rot<INV>(v[4 * 3 + 3], -kC16, -kS16); // W^9
  float2 out[16];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    float2 a0 = v[4 * k1 + 0], a1 = v[4 * k1 + 1], a2 = v[4 * k1 + 2], a3 = v[4 * k1 + 3];
    dft4<INV>(a0, a1, a2, a3);
    out[k1] = a0; out[k1 + 4] = a1; out[k1 + 8] = a2; out[k1 + 12] = a3;
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = out[i];
}

template <int R, bool INV>
__device__ __forceinline__ void dft(float2* v) {
  if constexpr (R == 2) dft2<INV>(v[0], v[1]);
  else if constexpr (R == 4) dft4<INV>(v[0], v[1], v[2], v[3]);
  else if constexpr (R == 8) dft8<INV>(v);
  else if constexpr (R == 16) dft16<INV>(v);
  else static_assert(R == 2 || R == 4 || R == 8 || R == 16, "unsupported radix");
}

// LDS addressing of one row transform: one pad slot per 16 elements keeps the
// stride-16 Stockham scatters free of bank conflicts.  For a group of T
// threads (T a multiple of 16) element t + T m sits at strided(t)[m * step],
// one base address and immediate offsets.
struct RowLds {
  float2* base;
  __device__ __forceinline__ float2& operator[](int i) const { return base[i + (i >> 4)]; }
  static constexpr int words(int n) { return n + n / 16; }
  template <int T>
  static constexpr bool strided_ok() { return T % 16 == 0; }
  template <int T>
  static constexpr int step() { return T + T / 16; }
  __device__ __forceinline__ float2* strided(int t) const { return base + t + (t >> 4); }
};

// LDS addressing of a strip of K columns transformed along the row index:
// element (row, c) at row*K + c.
template <int K>
struct ColLds {
  float2* base;
  int c;
  __device__ __forceinline__ float2& operator[](int i) const { return base[i * K + c]; }
  static constexpr int words(int n) { return n * K; }
  template <int T>
  static constexpr bool strided_ok() { return true; }
  template <int T>
  static constexpr int step() { return T * K; }
  __device__ __forceinline__ float2* strided(int t) const { return base + t * K + c; }
};

// Read the strided layout x[m] = element t + T m back from LDS.
template <int T, int E, class Lds>
__device__ __forceinline__ void lds_gather(float2 (&x)[E], const Lds& lds, int t) {
  if constexpr (Lds::template strided_ok<T>()) {
    const float2* p = lds.strided(t);
#pragma unroll
    for (int m = 0; m < E; ++m) x[m] = p[m * Lds::template step<T>()];
  } else {
#pragma unroll
    for (int m = 0; m < E; ++m) x[m] = lds[t + T * m];
  }
}

// Ordering of an LDS exchange.  A transform whose T threads sit inside one
// wavefront (T <= 64, groups aligned to the wave) needs no block barrier: the
// wave waits for its own outstanding LDS operations (lgkmcnt(0)) and the
// compiler is kept from moving LDS accesses across the point.  Otherwise a
// block-wide barrier.
template <bool WAVE>
__device__ __forceinline__ void lds_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0), vmcnt / expcnt untouched
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// One Stockham pass loading each twiddle right where it is used.
template <int N, int E, int R, int NS, bool INV, bool LAST, bool WAVE, class Lds>
__device__ __forceinline__ void stockham_pass(float2 (&x)[E], const Lds& lds, int t,
                                              const float2* __restrict__ tw) {
  constexpr int T = N / E;
  constexpr int B = E / R;
#pragma unroll
  for (int q = 0; q < B; ++q) {
    const int j = t + T * q;
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = x[q + B * r];
    if constexpr (NS > 1) {
      const int k = j & (NS - 1);
      constexpr int STRIDE = N / (NS * R);
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const float2 w = tw[r * k * STRIDE];
        v[r] = INV ? c_mulc(v[r], w) : c_mul(v[r], w);
      }
    }
    dft<R, INV>(v);
    if constexpr (LAST) {
#pragma unroll
      for (int r = 0; r < R; ++r) x[q + B * r] = v[r];
    } else {
      const int k = j & (NS - 1);
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[base + r * NS] = v[r];
    }
  }
  if constexpr (!LAST) {
    lds_sync<WAVE>();
    lds_gather<T>(x, lds, t);
    lds_sync<WAVE>();
  }
}

// Full length-N transform of the strided-layout registers (unnormalised in
// both directions; forward uses exp(-2 pi i n k / N)).
// WAVE: the T = N/E threads of the transform lie in one wavefront (see lds_sync).
// R2SEL: radix of the second pass (0: min(16, N/16)); the third pass takes the
// rest, N / (16 R2SEL), at sub-length 16 R2SEL.  Every plan leaves its outputs
// in the same strided natural-order layout (the last pass writes output index
// j + (N/R) r back to slot q + (E/R) r, the slot it read).
template <int N, int R2SEL>
constexpr int second_radix() {
  return R2SEL ? R2SEL : (N / 16 >= 16 ? 16 : N / 16);
}
template <int N, int R2SEL>
constexpr int fft_passes() {
  return N == 16 ? 1 : (N / 16 == second_radix<N, R2SEL>() ? 2 : 3);
}

template <int N, int E, bool INV, bool WAVE = false, int R2SEL = 0, class Lds>
__device__ __forceinline__ void fft(float2 (&x)[E], const Lds& lds, int t, const float2* __restrict__ tw) {
  static_assert(E == 16, "radix plan written for 16 elements per thread");
  static_assert(N >= 16 && N <= 4096 && (N & (N - 1)) == 0, "N must be a power of two in 16..4096");
  static_assert(!WAVE || N / E <= 64, "a wave-local transform needs at most 64 threads");
  constexpr int REM1 = N / 16;
  stockham_pass<N, E, 16, 1, INV, REM1 == 1, WAVE>(x, lds, t, tw);
  if constexpr (REM1 > 1) {
    constexpr int R2 = second_radix<N, R2SEL>();
    static_assert(REM1 % R2 == 0 && R2 <= 16 && REM1 / R2 <= 16, "unsupported radix plan");
    constexpr int REM2 = REM1 / R2;
    stockham_pass<N, E, R2, 16, INV, REM2 == 1, WAVE>(x, lds, t, tw);
    if constexpr (REM2 > 1) stockham_pass<N, E, REM2, 16 * R2, INV, true, WAVE>(x, lds, t, tw);
  }
}

// Copy the N-entry twiddle table into LDS once per block: the passes then
// read their per-lane twiddles with LDS loads instead of divergent global
// gathers.  Block-wide barrier at the end.
template <int N>
__device__ __forceinline__ const float2* stage_twiddles(float2* lds_tw, const float2* __restrict__ tw) {
  for (int i = threadIdx.x; i < N; i += blockDim.x) lds_tw[i] = tw[i];
  __syncthreads();
  return lds_tw;
}

// Barriers executed by fft<N, 16, ...>: a group with no transform to do calls
// this so that every thread of a block passes the same barrier sequence.
template <int N, bool WAVE = false, int R2SEL = 0>
__device__ __forceinline__ void idle_fft() {
  if constexpr (WAVE) return;
#pragma unroll
  for (int i = 0; i < 2 * (fft_passes<N, R2SEL>() - 1); ++i) __syncthreads();
}

}  // namespace turpy
