// Device helpers for gfx950: complex arithmetic, the Philox4x32-10 generator,
// Box-Muller normals and revolution-based sine/cosine.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace turpy {

// Poisoned-LDS test builds (TURPY_LDS_POISON, libturpy_poison.so): every LDS
// array is filled with all-ones words (NaN as float and as double) before a
// kernel uses it, so a read of LDS that no thread wrote turns the result into
// NaN.  Other builds compile the macro to nothing.
#ifdef TURPY_LDS_POISON
template <class T, size_t S>
__device__ __forceinline__ void poison_lds(T (&arr)[S]) {
  uint32_t* w = reinterpret_cast<uint32_t*>(arr);
  for (size_t i = threadIdx.x; i < sizeof(arr) / sizeof(uint32_t); i += blockDim.x) w[i] = 0xFFFFFFFFu;
  __syncthreads();
}
#define TURPY_LDS_INIT(arr) ::turpy::poison_lds(arr)
#else
#define TURPY_LDS_INIT(arr) ((void)0)
#endif

// Global load of a complex value, with the non-temporal (nt) cache policy
// when NT is set.
typedef float float2_nt __attribute__((ext_vector_type(2)));
template <bool NT>
__device__ __forceinline__ float2 ld_s(const float2* p) {
  if constexpr (NT) {
    const float2_nt w = __builtin_nontemporal_load(reinterpret_cast<const float2_nt*>(p));
    return make_float2(w.x, w.y);
  } else {
    return *p;
  }
}

// Global stores with the non-temporal (nt) cache policy when NT is set: for
// outputs that no kernel of the same pass sequence reads back soon
// (checkpoints and dL/dphi, read by the adjoint or the caller), which then do
// not displace the field planes the next pass reads from the last-level cache.
template <bool NT>
__device__ __forceinline__ void st_s(float2* p, float2 v) {
  if constexpr (NT) {
    const float2_nt w = {v.x, v.y};
    __builtin_nontemporal_store(w, reinterpret_cast<float2_nt*>(p));
  } else {
    *p = v;
  }
}
template <bool NT>
__device__ __forceinline__ void st_f(float* p, float v) {
  if constexpr (NT) {
    __builtin_nontemporal_store(v, p);
  } else {
    *p = v;
  }
}

__device__ __forceinline__ float2 c_add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 c_sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 c_mul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 c_mulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 c_scale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 products
// with the multipliers 0xD2511F53 / 0xCD9E8D57, key advanced by the Weyl
// constants 0x9E3779B9 / 0xBB67AE85 between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    if (i > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c.x;
    const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c.z;
    // three-input exclusive or in one gfx950 instruction (truth table 0x96)
    c = make_uint4(__builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(p1 >> 32), c.y, k0, 0x96),
                   static_cast<uint32_t>(p1),
                   __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(p0 >> 32), c.w, k1, 0x96),
                   static_cast<uint32_t>(p0));
  }
  return c;
}

// Uniform in (0, 1): (floor(v / 512) + 1/2) * 2^-23, exact in FP32.
__device__ __forceinline__ float u01(uint32_t v) {
  return (static_cast<float>(v >> 9) + 0.5f) * 0x1p-23f;
}

// sin / cos of 2*pi*x (the hardware transcendental units take their argument
// in revolutions).  The argument is first reduced to [-1/2, 1/2]: x - rint(x)
// is exact in FP32 for every finite x, so the only error beyond the hardware
// units' own is the rounding already in x (absolute, about |x| * 2^-24
// revolutions).
__device__ __forceinline__ void sincos_rev(float x, float* s, float* c) {
  const float r = x - rintf(x);
  *s = __builtin_amdgcn_sinf(r);
  *c = __builtin_amdgcn_cosf(r);
}

// Complex unit-variance-per-component normal from two words:
// rho = sqrt(-2 ln u(va)), theta = 2 pi u(vb).
__device__ __forceinline__ float2 box_muller(uint32_t va, uint32_t vb) {
  const float ua = u01(va);
  const float ub = u01(vb);
  // hardware square root (about 1 ulp): the argument is at least about 2^-23,
  // far from the denormal range that the correctly rounded expansion guards
  const float rho = __builtin_amdgcn_sqrtf(-2.0f * 0.69314718055994531f * __builtin_amdgcn_logf(ua));
  float s, c;
  sincos_rev(ub, &s, &c);
  return make_float2(rho * c, rho * s);
}

// Ensemble moments of the intensity (Sec. 3.3) as compensated (Kahan) sums:
// per pixel (s1, c1) over I = |u|^2 and (s2, c2) over I^2, the true sums being
// about s - c.  Every kernel that accumulates moments goes through these
// helpers, whose multiplies never fuse with a neighbouring add (contraction
// off), so the same inputs in the same order give the same bits in every
// kernel that inlines them.
__device__ __forceinline__ void kahan_add(float& s, float& c, float v) {
#pragma clang fp contract(off)
  const float y = v - c;
  const float t = s + y;
  c = (t - s) - y;
  s = t;
}
// Join a compensated partial sum (ps, pc) into (s, c).
__device__ __forceinline__ void kahan_join(float& s, float& c, float ps, float pc) {
#pragma clang fp contract(off)
  const float y = ps - (c + pc);
  const float t = s + y;
  c = (t - s) - y;
  s = t;
}
__device__ __forceinline__ void moment_add(float& s1, float& c1, float& s2, float& c2, float2 u) {
#pragma clang fp contract(off)
  const float i = u.x * u.x + u.y * u.y;
  kahan_add(s1, c1, i);
  kahan_add(s2, c2, i * i);
}

// Counter words for the noise layout (e, t, pair, tag << 28 | screen).
__device__ __forceinline__ uint4 noise_counter(uint32_t e, uint32_t t, uint32_t pair, uint32_t tag,
                                               uint32_t screen) {
  return make_uint4(e, t, pair, (tag << 28) | screen);
}

}  // namespace turpy
