// Launch interface between the host runtime (api.hip) and the gfx950 kernels
// (kernels.hip).  Plain structs of device pointers and scalars.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace turpy {

// Philox counter tags of the noise layout.
constexpr uint32_t TAG_MAIN = 1;
constexpr uint32_t TAG_SH = 2;
constexpr uint32_t TAG_AR = 3;
constexpr uint32_t TAG_AR_SH = 4;  // AR innovations of the subharmonic coefficients

// Screen source inside a row pass.
enum RowScreen : int { ROW_NO_SCREEN = 0, ROW_SCRATCH = 1, ROW_MATERIALIZED = 2 };

struct RowArgs {
  const float2* tw;         // twiddles exp(-2 pi i k / N), [N]
  const float2* in;         // field rows, realization r at in + r * in_stride
  int64_t in_stride;        // elements between realizations (0: shared source)
  float2* out;              // [R][N][N]
  int64_t R;                // realizations
  int in_spectral;          // input rows in the row-spectral domain: inverse row transform first
  int out_spectral;         // forward row transform at the end
  const float2* pre;        // per-column factor before the inverse transform, or NULL
  const float2* post;       // per-column factor after the forward transform, or NULL
  int conj_tables;          // use conj(pre), conj(post)
  float scale;              // normalisation folded into the pointwise step
  int screen_mode;          // RowScreen
  const float2* scratch;    // [P][N][N] column-transformed complex screen, revolutions
  const float* screens;     // [R][M][N][N] radians (materialised)
  int screen;               // screen index s
  int M;                    // screens per path
  int sh_levels;            // 0..3
  const float2* sh;         // [P][M][32] subharmonic coefficients, [24] = their grid mean
  float sh_scale;           // to revolutions: 1 (synthesised) or 1/(2 pi) (AR state, radians)
  const float2* sh_phasor;  // [3][N] exp(2 pi i (i - N/2) / (N 3^p))
  int backward;             // 0: W = U e^{i phi}; 1: adjoint (read checkpoint, write dL/dphi, e^{-i phi})
  float2* ckpt_out;         // [R][M][N][N] field after the screen, or NULL (backward: as rebuilt)
  const float2* ckpt_in;    // backward: same layout
  int ckpt_single;          // 1: ckpt_out / ckpt_in hold this screen only, [R][N][N]
  float* grad_screens;      // backward: [R][M][N][N] dL/dphi, or NULL
  float* phase_out;         // [R][M][N][N] radians: write the screens themselves, or NULL
  int waves;                // occupancy hint of the screen row passes (2, 3, 4; 0: the default)
};

struct ColArgs {
  const float2* tw;
  const float2* in;         // realization r at in + r * in_stride
  int64_t in_stride;
  float2* out;              // [R][N][N]
  int64_t R;
  const float2* table;      // h[k0] / N for this distance, [N]
  int conj_table;
  int angular;              // angular-spectrum correction on top of the separable Fresnel chirp
  const float2* as_table;   // [N^2/2 + 1]: H_as / H_fresnel at q = k0^2 + k1^2 (signed bins), or NULL
  float as_b;               // (2 pi df)^2 / k^2: kappa^2 / k^2 per unit of q
  float as_c;               // -dz (2 pi df)^4 / (4 pi k^3): revolutions per q^2 / (1 + sqrt(1 - B q))^2
  int width;                // columns per block (4, 8, 16), 0: the built-in choice for N
  int radix;                // radix of the transforms' second pass (0: the default plan)
};

struct SynthArgs {
  const float2* tw;
  float2* scratch;          // [P][N][N]
  int64_t P;                // realization pairs
  uint32_t key0, key1;      // Philox key (seed)
  uint32_t t;               // time step
  const uint32_t* t_dev;    // or, when set, read here at run time
  uint32_t screen;
  uint32_t tag;
  float amp;                // sqrt(0.023) r0^(-5/6) df / (2 pi): revolutions
  float df2;                // df^2
  float inner;              // log2(e) / (2 fm^2), 0 when no inner-scale cutoff
  float f02;                // f0^2
  float q;                  // alpha / 4: exponent of (f^2 + f0^2) in the amplitude
  // spectra source (ROW_SCRATCH from stored spectra) instead of noise
  const float2* spectra;    // [P][M][N][N] radians, or NULL for synthesis
  int M;
  int width;                // columns per block (4, 8, 16), 0: the built-in choice for N
  int radix;                // radix of the transform's second pass (0: the default plan)
  // AR step fused into the read of the stored spectra (Eq. 4 then Eq. 5 with
  // innovations drawn at the time step): the evolved spectrum is written back
  // to `state` (the same array as `spectra`) and transformed
  int evolve;
  float2* state;
  uint32_t ar_tag;          // innovation tag
  float alpha_f, blend;     // alpha and sqrt(1 - alpha^2), rounded from FP64
  double sx, sy;            // frozen-flow shift in pixels
  float amp_rad;            // sqrt(0.023) r0^(-5/6) df of this screen: radians
};

struct ShArgs {
  float2* sh;               // [P][M][32], in place for an AR step
  int64_t P;
  int M;
  int levels;
  int n;                    // grid size (translation phase of an AR step)
  uint32_t key0, key1, t, tag;
  const uint32_t* t_dev;    // time step read at run time when set
  const float* amp;         // [M][3][2] amplitude (revolutions) for |offset|^2 = 1, 2
  float scale;              // output units per revolution: 1, or 2 pi for radians
  int ar;                   // 0: fresh coefficients; 1: Eq. 4 + Eq. 5 step of the stored ones
  double alpha, sx, sy;     // AR step: blend and translation in pixels
  float2 mean_fac[3];       // mean over the grid of exp(2 pi i (i - N/2)/(N 3^p))
};

// A grouped launch of an uneven batch runs one pass of many path instances:
// instance i's argument record is tab[i], i the block's z index (y for the
// column-pass and synthesis kernels, whose x index is 1-D).  In a record the
// pointers into a call's buffers hold byte offsets, which the launch adds to
// the bases below; the key words of the noise records hold the instance's
// seed offset (low, high word), to which the launch adds its seed.  Pointers
// to plan tables (twiddles, transfer functions) are absolute.
struct GroupCall {
  const char* in;           // fields the pass reads: the call's u_in, or u_out
  char* out;                // fields it writes: u_out
  char* ws;                 // the group's workspace
  char* ck;                 // checkpoints the pass writes (forward) or reads (adjoint), or NULL
  char* gs;                 // adjoint: dL/dphi, or NULL
  uint64_t seed;
  uint32_t t;
  const uint32_t* t_dev;    // time step read at run time when set
};

struct EvolveArgs {
  float2* spectra;          // [P][M][N][N] radians, in place
  int64_t P;
  int M;
  int n;
  int log2n;
  uint32_t key0, key1, t, tag;
  const uint32_t* t_dev;    // time step read at run time when set
  float alpha_f;            // alpha and sqrt(1 - alpha^2), rounded from FP64
  float blend;
  double sx, sy;            // shift in pixels
  int init;                 // 1: overwrite with fresh spectra (t = 0)
  const float* amp;         // [M] sqrt(0.023) r0^(-5/6) df: radians
  float df2, inner, f02, q;
};

struct StatsArgs {
  const float2* u;
  int64_t batch;
  int n;
  float* moments;           // [4][n][n]
};

struct FinalizeArgs {
  const float* moments;
  int n;
  double dx;
  double count;
  float* si_map;
  double* summary;          // [8], see turpy_stats
  const float* weight;      // [n][n] per-pixel weights of the SI region sums, or NULL (all 1)
  double power_fraction;    // > 0: SI region = power-cutoff region; 0: the central region
};

struct NoiseArgs {
  float2* out;              // [pairs][n][n]
  int64_t pairs;
  int n;
  uint32_t key0, key1, t, tag, screen;
};

struct RecvArgs {
  const float2* tw;
  int n;
  int64_t batch;
  double dx;
  double radius2;           // (aperture diameter / 2)^2
  const float* theta1;      // [n][n] real-space mask (radians)
  const float* theta2;      // [n][n] Fourier-plane mask, centred (fftshift) order
  const float2* u;          // receiver input fields [batch][n][n]
  const float2* in;         // pass input [batch][n][n]
  const float2* in2;        // second pass input (gradient path)
  float2* out;              // pass output [batch][n][n]
  float* partial;           // [chunks][n][n] per-chunk mask-gradient sums
  int chunks;               // number of batch chunks
  int conj_mask;            // use exp(-i theta2)
};

hipError_t launch_row(int n, const RowArgs& a, int64_t pairs, hipStream_t s);
// Grouped launches over `count` instances (records in device memory, `proto`
// one of them as built on the host, for the kernel choice).  The row passes
// take the screen-free and the synthesised-screen forms, forward and adjoint;
// the column pass and synthesis the default strip width with the record's
// radix.
hipError_t launch_row_group(int n, const RowArgs& proto, const RowArgs* tab, uint32_t count, int64_t pairs,
                            const GroupCall& g, hipStream_t s);
hipError_t launch_col_group(int n, const ColArgs& proto, const ColArgs* tab, uint32_t count, const GroupCall& g,
                            hipStream_t s);
hipError_t launch_synth_group(int n, const SynthArgs& proto, const SynthArgs* tab, uint32_t count,
                              const GroupCall& g, hipStream_t s);
// grid (pairs, max_screens, count); blocks beyond an instance's screens or
// with no subharmonic levels exit at once
hipError_t launch_sh_group(const ShArgs* tab, uint32_t count, int64_t pairs, int max_screens, const GroupCall& g,
                           hipStream_t s);
// The plain final row pass (in spectral, out real, no screen, no pre/post
// factor) with the ensemble moments added into moments [4][n][n].
hipError_t launch_row_moments(int n, const RowArgs& a, float* moments, hipStream_t s);
hipError_t launch_col(int n, const ColArgs& a, hipStream_t s);
hipError_t launch_synth(int n, const SynthArgs& a, hipStream_t s);
hipError_t launch_sh(const ShArgs& a, hipStream_t s);
hipError_t launch_evolve(const EvolveArgs& a, hipStream_t s);
hipError_t launch_stats(const StatsArgs& a, hipStream_t s);
// Count of NaN and infinite values among x[0..count) into *counter (cleared first).
hipError_t launch_nonfinite(const float* x, int64_t count, unsigned long long* counter, hipStream_t s);
hipError_t launch_finalize(const FinalizeArgs& a, hipStream_t s);
// receiver passes (receiver.hip)
hipError_t launch_recv_row_in(const RecvArgs& a, hipStream_t s);     // U1 = A u e^{i th1}, FFT along x
hipError_t launch_recv_col(const RecvArgs& a, hipStream_t s);        // FFT_y, x e^{+-i th2}/N, IFFT_y
hipError_t launch_recv_col_grad(const RecvArgs& a, hipStream_t s);   // th2 gradient partials + gradient path
hipError_t launch_recv_row_grad(const RecvArgs& a, hipStream_t s);   // th1 gradient partials + grad u
hipError_t launch_recv_reduce(const RecvArgs& a, float* grad, int centre_shift, hipStream_t s);
hipError_t launch_noise(const NoiseArgs& a, hipStream_t s);
// out[p] = sum over r < R of in[r * count + p] (in order, compensated)
hipError_t launch_sum_planes(const float2* in, int64_t R, int64_t count, float2* out, hipStream_t s);
hipError_t launch_copy(const float2* in, int64_t in_stride, float2* out, int64_t count, int64_t R,
                       hipStream_t s);

}  // namespace turpy
