// Launch geometry shared by the kernel files: elements per thread, rows per
// row-pass block, columns per column-pass strip, XCD-aware block order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace turpy {

constexpr int kE = 16;  // elements per thread in every transform

template <int N>
constexpr int row_groups() {  // rows per block of the row kernels
  return (256 / (N / kE)) < N ? (256 / (N / kE)) : N;
}
template <int N>
constexpr int row_block() { return row_groups<N>() * (N / kE); }
// Columns per block of the column pass and of the screen synthesis, per grid
// size, when no tuned choice is set: the fastest of 4, 8 and 16 measured on
// MI355X at constant R N^2 (column pass: 16 up to N = 512, 8 above;
// synthesis, whose VALU load per element is higher, 4 from N = 1024).
constexpr int default_col_width(int n) { return n >= 1024 ? 8 : (n >= 256 ? 16 : 8); }
constexpr int default_synth_width(int n) { return n >= 1024 ? 4 : default_col_width(n); }
template <int N>
constexpr int col_width() { return default_col_width(N); }
template <int N>
constexpr int col_block() { return col_width<N>() * (N / kE); }
template <int N>
constexpr int synth_width() { return default_synth_width(N); }

// A strip of K columns is built for grid size N when its block (K N / 16
// threads) stays within 1024 threads and its LDS (K N complex words beside
// the N-entry twiddle and chirp tables) within the 160 KiB of a CU.  At
// N = 2048 this excludes 16 columns.
template <int N, int K>
constexpr bool strip_fits() {
  return K <= N && K * (N / kE) <= 1024 && (static_cast<long>(K) * N + 2L * N) * 8 <= 160L * 1024;
}
constexpr bool strip_fits_rt(int n, int k) {
  return (k == 4 || k == 8 || k == 16) && k <= n && k * (n / kE) <= 1024 &&
         (static_cast<long>(k) * n + 2L * n) * 8 <= 160L * 1024;
}

// Ensemble moments: the R realizations are summed in C contiguous chunks,
// chunk c holding realizations [c R / C, (c + 1) R / C), and the compensated
// sums of the non-empty chunks are joined into the stored ones in chunk order.
// C = 256 / (N / 16) clamped to [4, 64] depends on N alone: a block of the
// fused final row pass (one row, C chunks of N / 16 threads) then has 256
// threads for N = 64..1024.
constexpr int moment_chunks(int n) {
  return (256 / (n / kE)) < 4 ? 4 : ((256 / (n / kE)) > 64 ? 64 : 256 / (n / kE));
}

// Row-pair pass: each half of a block (whole waves for N >= 64) carries one
// realization of a pair over `pair_rows` rows.
template <int N>
constexpr int pair_rows() {
  return (128 / (N / kE)) < 1 ? 1 : ((128 / (N / kE)) < N ? (128 / (N / kE)) : N);
}
template <int N>
constexpr int pair_block() { return 2 * pair_rows<N>() * (N / kE); }

// Relay row pass: two workers of `relay_rows` rows each per block, over two
// row groups (2 relay_rows <= N).  Used where a worker is whole waves.
template <int N>
constexpr int relay_rows() { return pair_rows<N>() < N / 2 ? pair_rows<N>() : N / 2; }
template <int N>
constexpr int relay_block() { return 2 * relay_rows<N>() * (N / kE); }
template <int N>
constexpr bool relay_fits() { return (relay_rows<N>() * (N / kE)) % 64 == 0; }

// Spread a 1-D block index so that consecutive logical tiles land on the same
// XCD (blocks are dealt round-robin over the 8 XCDs, each with its own L2).
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t nb) {
  if (nb % 8u != 0u) return b;
  return (b % 8u) * (nb / 8u) + b / 8u;
}

// Strip and plane of block b of a column pass over R planes of `strips`
// strips: plane-major, the planes from last to first, each XCD taking one
// contiguous eighth of every plane's strips (neighbouring strips, which share
// cache lines, stay on one XCD's L2).  The row passes run the planes from
// first to last, so a column pass starts on the planes the row pass before it
// wrote last, and the row pass after it on the planes it wrote last.  With a
// strip count that is not a multiple of 8: xcd_remap over (plane, strip).
__device__ __forceinline__ void col_tile(uint32_t b, uint32_t nb, int strips, int64_t R, int* strip, int64_t* r) {
  if (strips % 8 == 0) {
    const uint32_t x = b % 8u, i = b / 8u;
    const int per = strips / 8;
    *strip = static_cast<int>(x) * per + static_cast<int>(i % static_cast<uint32_t>(per));
    *r = R - 1 - static_cast<int64_t>(i / static_cast<uint32_t>(per));
  } else {
    const uint32_t t = xcd_remap(b, nb);
    *strip = static_cast<int>(t % static_cast<uint32_t>(strips));
    *r = t / static_cast<uint32_t>(strips);
  }
}

}  // namespace turpy
