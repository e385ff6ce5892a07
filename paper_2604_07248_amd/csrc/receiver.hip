// Dual-domain two-mask receiver (Sec. 2.5, Sec. 4.1) and its adjoint on gfx950.
//
// Forward:  U1 = A u exp(i theta1)            (row pass, then FFT along x)
//           Z  = DFT{U1} exp(i theta2')       (column pass: FFT along y, mask / N, IFFT)
//           u_out = IDFT{Z}                   (row pass: IFFT along x / N)
// The mask gradients are sums over the batch; each block accumulates a fixed
// chunk of batch elements in registers and writes one partial plane, and a
// reduction kernel adds the partials in a fixed order (deterministic).
#include "fft.hpp"
#include "kernels.hpp"
#include "layout.hpp"

namespace turpy {

namespace {

__device__ __forceinline__ float aperture(int i0, int i1, int n, double dx, double r2) {
  const double x = (i1 - n / 2) * dx, y = (i0 - n / 2) * dx;
  return (x * x + y * y) <= r2 ? 1.0f : 0.0f;
}

// exp(i theta) with theta in radians.
__device__ __forceinline__ float2 phase(float theta) {
  float s, c;
  sincos_rev(theta * 0.15915494309189535f, &s, &c);
  return make_float2(c, s);
}

// theta2 stored centred: natural bin k maps to centred index (k + n/2) mod n.
__device__ __forceinline__ size_t centred(int k0, int k1, int n) {
  return static_cast<size_t>((k0 + n / 2) & (n - 1)) * n + ((k1 + n / 2) & (n - 1));
}

template <int N>
__global__ __launch_bounds__(row_block<N>()) void recv_row_in_kernel(RecvArgs a) {
  constexpr int T = N / kE;
  constexpr int G = row_groups<N>();
  __shared__ float2 smem[G * RowLds::words(N)];
  TURPY_LDS_INIT(smem);
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  const int i0 = blockIdx.x * G + g;
  const int64_t b = blockIdx.y;
  const RowLds lds{smem + g * RowLds::words(N)};
  __shared__ float2 tw_lds[N];
  const float2* tw = stage_twiddles<N>(tw_lds, a.tw);
  const size_t row = static_cast<size_t>(i0) * N;
  const float2* src = a.u + b * static_cast<int64_t>(N) * N + row;
  float2 x[kE];
#pragma unroll
  for (int m = 0; m < kE; ++m) {
    const int i1 = t + T * m;
    const float amp = aperture(i0, i1, N, a.dx, a.radius2);
    x[m] = c_scale(c_mul(src[i1], phase(a.theta1[row + i1])), amp);
  }
  fft<N, kE, false>(x, lds, t, tw);
  float2* dst = a.out + b * static_cast<int64_t>(N) * N + row;
#pragma unroll
  for (int m = 0; m < kE; ++m) (dst + t)[T * m] = x[m];
}

template <int N>
__global__ __launch_bounds__(col_block<N>()) void recv_col_kernel(RecvArgs a) {
  constexpr int T = N / kE;
  constexpr int K = col_width<N>();
  constexpr int STRIPS = N / K;
  __shared__ float2 smem[ColLds<K>::words(N)];
  TURPY_LDS_INIT(smem);
  const uint32_t bid = xcd_remap(blockIdx.x, gridDim.x);
  const int strip = bid % STRIPS;
  const int64_t b = bid / STRIPS;
  const int c = threadIdx.x % K, t = threadIdx.x / K;
  const int k1 = strip * K + c;
  const ColLds<K> lds{smem, c};
  __shared__ float2 tw_lds[N];
  const float2* tw = stage_twiddles<N>(tw_lds, a.tw);
  const size_t plane = static_cast<size_t>(N) * N;
  const float2* src = a.in + b * plane + k1;
  float2 x[kE];
#pragma unroll
  for (int m = 0; m < kE; ++m) x[m] = (src + static_cast<size_t>(t) * N)[static_cast<size_t>(T * m) * N];
  fft<N, kE, false>(x, lds, t, tw);
  constexpr float inv_n = 1.0f / N;
#pragma unroll
  for (int m = 0; m < kE; ++m) {
    const int k0 = t + T * m;
    float2 h = phase(a.theta2[centred(k0, k1, N)]);
    if (a.conj_mask) h.y = -h.y;
    x[m] = c_scale(c_mul(x[m], h), inv_n);
  }
  fft<N, kE, true>(x, lds, t, tw);
  float2* dst = a.out + b * plane + k1;
#pragma unroll
  for (int m = 0; m < kE; ++m) (dst + static_cast<size_t>(t) * N)[static_cast<size_t>(T * m) * N] = x[m];
}

// Column half of the adjoint.  in = row-FFT of U1 (X after the column FFT),
// in2 = row-FFT of g_out (G after the column FFT).  Accumulates
// Im(conj(X M2) G) / N^2 over the block's batch chunk into partial[chunk] and
// writes IFFT_y(conj(M2) G / N) back over in2's rows in out.
template <int N>
__global__ __launch_bounds__(col_block<N>()) void recv_col_grad_kernel(RecvArgs a) {
  constexpr int T = N / kE;
  constexpr int K = col_width<N>();
  constexpr int STRIPS = N / K;
  __shared__ float2 smem[ColLds<K>::words(N)];
  TURPY_LDS_INIT(smem);
  const int strip = blockIdx.x % STRIPS;
  const int chunk = blockIdx.x / STRIPS;
  const int c = threadIdx.x % K, t = threadIdx.x / K;
  const int k1 = strip * K + c;
  const ColLds<K> lds{smem, c};
  __shared__ float2 tw_lds[N];
  const float2* tw = stage_twiddles<N>(tw_lds, a.tw);
  const size_t plane = static_cast<size_t>(N) * N;
  const int64_t per = (a.batch + a.chunks - 1) / a.chunks;
  const int64_t b0 = chunk * per, b1 = b0 + per < a.batch ? b0 + per : a.batch;
  float2 mask[kE];
#pragma unroll
  for (int m = 0; m < kE; ++m) mask[m] = phase(a.theta2[centred(t + T * m, k1, N)]);
  float acc[kE];
#pragma unroll
  for (int m = 0; m < kE; ++m) acc[m] = 0.0f;
  constexpr float inv_n = 1.0f / N;
  constexpr float inv_n2 = 1.0f / (static_cast<float>(N) * N);
  for (int64_t b = b0; b < b1; ++b) {
    float2 x[kE], gg[kE];
    const float2* sx = a.in + b * plane + k1;
    const float2* sg = a.in2 + b * plane + k1;
#pragma unroll
    for (int m = 0; m < kE; ++m) x[m] = (sx + static_cast<size_t>(t) * N)[static_cast<size_t>(T * m) * N];
    fft<N, kE, false>(x, lds, t, tw);
#pragma unroll
    for (int m = 0; m < kE; ++m) gg[m] = (sg + static_cast<size_t>(t) * N)[static_cast<size_t>(T * m) * N];
    fft<N, kE, false>(gg, lds, t, tw);
#pragma unroll
    for (int m = 0; m < kE; ++m) {
      const float2 z = c_mul(x[m], mask[m]);
      acc[m] += (z.x * gg[m].y - z.y * gg[m].x) * inv_n2;  // Im(conj(Z) G) / N^2
      gg[m] = c_scale(c_mulc(gg[m], mask[m]), inv_n);
    }
    fft<N, kE, true>(gg, lds, t, tw);
    float2* dst = a.out + b * plane + k1;
#pragma unroll
    for (int m = 0; m < kE; ++m) (dst + static_cast<size_t>(t) * N)[static_cast<size_t>(T * m) * N] = gg[m];
  }
  float* part = a.partial + static_cast<size_t>(chunk) * plane + k1;
#pragma unroll
  for (int m = 0; m < kE; ++m) (part + static_cast<size_t>(t) * N)[static_cast<size_t>(T * m) * N] = acc[m];
}

// Row half of the adjoint.  in = output of recv_col_grad (row-spectral g path):
// g_U1 = IFFT_x(in) / N; with U1 = A u exp(i theta1) recomputed,
// partial[chunk] += Im(conj(U1) g_U1) and out = A exp(-i theta1) g_U1 (if set).
template <int N>
__global__ __launch_bounds__(row_block<N>()) void recv_row_grad_kernel(RecvArgs a) {
  constexpr int T = N / kE;
  constexpr int G = row_groups<N>();
  __shared__ float2 smem[G * RowLds::words(N)];
  TURPY_LDS_INIT(smem);
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  const int i0 = blockIdx.x * G + g;
  const int chunk = blockIdx.y;
  const RowLds lds{smem + g * RowLds::words(N)};
  __shared__ float2 tw_lds[N];
  const float2* tw = stage_twiddles<N>(tw_lds, a.tw);
  const size_t plane = static_cast<size_t>(N) * N;
  const size_t row = static_cast<size_t>(i0) * N;
  const int64_t per = (a.batch + a.chunks - 1) / a.chunks;
  const int64_t b0 = chunk * per, b1 = b0 + per < a.batch ? b0 + per : a.batch;
  float2 w[kE];  // A exp(i theta1)
#pragma unroll
  for (int m = 0; m < kE; ++m) {
    const int i1 = t + T * m;
    w[m] = c_scale(phase(a.theta1[row + i1]), aperture(i0, i1, N, a.dx, a.radius2));
  }
  float acc[kE];
#pragma unroll
  for (int m = 0; m < kE; ++m) acc[m] = 0.0f;
  constexpr float inv_n = 1.0f / N;
  for (int64_t b = b0; b < b1; ++b) {
    float2 x[kE];
    const float2* src = a.in + b * plane + row;
#pragma unroll
    for (int m = 0; m < kE; ++m) x[m] = (src + t)[T * m];
    fft<N, kE, true>(x, lds, t, tw);
    const float2* us = a.u + b * plane + row;
#pragma unroll
    for (int m = 0; m < kE; ++m) {
      const float2 gu1 = c_scale(x[m], inv_n);
      const float2 u1 = c_mul((us + t)[T * m], w[m]);
      acc[m] += u1.x * gu1.y - u1.y * gu1.x;  // Im(conj(U1) g_U1)
      x[m] = c_mulc(gu1, w[m]);               // A exp(-i theta1) g_U1
    }
    if (a.out) {
      float2* dst = a.out + b * plane + row;
#pragma unroll
      for (int m = 0; m < kE; ++m) (dst + t)[T * m] = x[m];
    }
  }
  float* part = a.partial + static_cast<size_t>(chunk) * plane + row;
#pragma unroll
  for (int m = 0; m < kE; ++m) (part + t)[T * m] = acc[m];
}

__global__ __launch_bounds__(256) void recv_reduce_kernel(const float* partial, int chunks, int n, float* grad,
                                                          int centre_shift) {
  const int64_t np = static_cast<int64_t>(n) * n;
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= np) return;
  float s = 0.0f;
  for (int c = 0; c < chunks; ++c) s += partial[c * np + p];
  int64_t q = p;
  if (centre_shift) {
    const int k0 = static_cast<int>(p / n), k1 = static_cast<int>(p % n);
    q = static_cast<int64_t>((k0 + n / 2) & (n - 1)) * n + ((k1 + n / 2) & (n - 1));
  }
  grad[q] = s;
}

template <int N>
hipError_t row_in_launch(const RecvArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(recv_row_in_kernel<N>, dim3(N / row_groups<N>(), static_cast<uint32_t>(a.batch)),
                     dim3(row_block<N>()), 0, s, a);
  return hipGetLastError();
}
template <int N>
hipError_t col_launch(const RecvArgs& a, hipStream_t s) {
  const uint64_t blocks = static_cast<uint64_t>(N / col_width<N>()) * a.batch;
  hipLaunchKernelGGL(recv_col_kernel<N>, dim3(static_cast<uint32_t>(blocks)), dim3(col_block<N>()), 0, s, a);
  return hipGetLastError();
}
template <int N>
hipError_t col_grad_launch(const RecvArgs& a, hipStream_t s) {
  const uint32_t blocks = static_cast<uint32_t>(N / col_width<N>()) * a.chunks;
  hipLaunchKernelGGL(recv_col_grad_kernel<N>, dim3(blocks), dim3(col_block<N>()), 0, s, a);
  return hipGetLastError();
}
template <int N>
hipError_t row_grad_launch(const RecvArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(recv_row_grad_kernel<N>, dim3(N / row_groups<N>(), a.chunks), dim3(row_block<N>()), 0, s, a);
  return hipGetLastError();
}

}  // namespace

#define TURPY_RECV_DISPATCH(FN, ...)          \
  switch (a.n) {                              \
    case 16: return FN<16>(__VA_ARGS__);      \
    case 32: return FN<32>(__VA_ARGS__);      \
    case 64: return FN<64>(__VA_ARGS__);      \
    case 128: return FN<128>(__VA_ARGS__);    \
    case 256: return FN<256>(__VA_ARGS__);    \
    case 512: return FN<512>(__VA_ARGS__);    \
    case 1024: return FN<1024>(__VA_ARGS__);  \
    case 2048: return FN<2048>(__VA_ARGS__);  \
    default: return hipErrorInvalidValue;     \
  }

hipError_t launch_recv_row_in(const RecvArgs& a, hipStream_t s) { TURPY_RECV_DISPATCH(row_in_launch, a, s) }
hipError_t launch_recv_col(const RecvArgs& a, hipStream_t s) { TURPY_RECV_DISPATCH(col_launch, a, s) }
hipError_t launch_recv_col_grad(const RecvArgs& a, hipStream_t s) { TURPY_RECV_DISPATCH(col_grad_launch, a, s) }
hipError_t launch_recv_row_grad(const RecvArgs& a, hipStream_t s) { TURPY_RECV_DISPATCH(row_grad_launch, a, s) }

hipError_t launch_recv_reduce(const RecvArgs& a, float* grad, int centre_shift, hipStream_t s) {
  const int64_t np = static_cast<int64_t>(a.n) * a.n;
  hipLaunchKernelGGL(recv_reduce_kernel, dim3(static_cast<uint32_t>((np + 255) / 256)), dim3(256), 0, s, a.partial,
                     a.chunks, a.n, grad, centre_shift);
  return hipGetLastError();
}

}  // namespace turpy
