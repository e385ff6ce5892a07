/*
 * turpy.h -- C ABI of the MI355X (gfx950) split-step turbulence propagator.
 *
 * The library computes the data-parallel hot path of TurPy (arXiv 2604.07248):
 * phase-screen synthesis from the modified von Karman PSD with Lane
 * subharmonics, split-step Fresnel / angular-spectrum propagation of batched
 * complex64 fields through those screens, AR(1) + frozen-flow evolution of the
 * stored screen spectra, the adjoint of the propagation, ensemble statistics
 * and the dual-domain two-mask receiver.
 *
 * Conventions shared by every call
 *  - Arrays are row-major [batch][screen][y][x]; complex values are interleaved
 *    (re, im) float pairs (complex64).  Index i0 is y, i1 is x; a pixel's
 *    centred coordinate is (i - N/2) dx.
 *  - All array arguments are DEVICE pointers owned by the caller (for example
 *    PyTorch tensors), 16-byte aligned at least; nothing here allocates or frees
 *    caller memory.  Plans own small device tables (twiddles, transfer-function
 *    chirps, subharmonic phasors) that turpy_plan_destroy releases.
 *  - Calls are asynchronous and stream-ordered on the given hipStream_t
 *    (passed as void*; NULL means the default stream).  Input validation runs on
 *    the host before anything is launched: on any non-OK status nothing has been
 *    enqueued, and turpy_last_error() returns a message for this thread.
 *  - Noise is Philox4x32-10 keyed by the 64-bit seed with counter
 *    (e, t, j, tag<<28 | s): t time step, j realization pair, s screen, tag 1
 *    main spectrum / 2 subharmonics / 3 AR innovation / 4 AR innovation of the
 *    subharmonic coefficients.  Realizations 2j and
 *    2j+1 take the real and imaginary parts of one complex screen.
 *  - Gradients follow PyTorch's convention for real losses:
 *    g = dL/dRe(u) + i dL/dIm(u).
 */
#ifndef TURPY_H_
#define TURPY_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TURPY_OK = 0,
  TURPY_E_INVALID = 1,      /* malformed argument or descriptor              */
  TURPY_E_UNSUPPORTED = 2,  /* well-formed but outside what is implemented   */
  TURPY_E_ALIASING = 3,     /* a step exceeds the transfer-function sampling limit (Sec. 2.4, Eq. 7) */
  TURPY_E_WORKSPACE = 4,    /* workspace NULL or smaller than turpy_workspace_size() */
  TURPY_E_HIP = 5,          /* a HIP runtime call failed (message has the HIP error) */
  TURPY_E_CAPACITY = 6,     /* a host output array is smaller than the result */
  TURPY_E_NONFINITE = 7     /* TURPY_CHECK_FINITE: an output holds a NaN or an infinity */
} turpy_status;

typedef enum { TURPY_TF_FRESNEL = 0, TURPY_TF_ANGULAR_SPECTRUM = 1 } turpy_tf_kind;

/* Where the screens of a propagation come from. */
typedef enum {
  TURPY_SCREENS_SYNTH = 0,        /* synthesised from (seed, t) inside the passes (Eq. S16, Eq. 2-3) */
  TURPY_SCREENS_MATERIALIZED = 1, /* float [R][M][N][N] radians supplied by the caller               */
  TURPY_SCREENS_SPECTRA = 2       /* an AR state (turpy_evolve): pair spectra and, with subharmonic
                                     levels, their subharmonic coefficients                        */
} turpy_screen_src;

/* Plan flags. */
#define TURPY_ALLOW_ALIASING 1u      /* accept steps beyond the Eq. 7 limit */
#define TURPY_SCREEN_CHECKPOINTS 2u  /* checkpoints also keep each screen's column half, so that the
                                        adjoint reads the screens instead of synthesising them again
                                        (turpy_checkpoint_size) */
#define TURPY_CHECK_FINITE 4u        /* every call of the plan counts the NaN and infinite values in
                                        its outputs (fields, checkpoints, gradients, screens) and
                                        returns TURPY_E_NONFINITE, naming the output, when there are
                                        any.  The check synchronises the stream, so such calls cannot
                                        be captured in a graph (TURPY_E_INVALID on a capturing
                                        stream); the outputs are written either way */

/* One propagation path (Sec. 2.1, Fig. 1A inputs). */
typedef struct turpy_path {
  int32_t n;                /* grid size N: power of two, 16..2048                              */
  int32_t num_screens;      /* M >= 0                                                           */
  double dx;                /* grid spacing [m], > 0                                            */
  double wavelength;        /* vacuum wavelength [m], > 0                                       */
  double n0;                /* mean refractive index, > 0                                       */
  const double* dz;         /* HOST [M+1]: diffraction distance before screen i (i < M) and after the
                               last screen (i = M), each >= 0; dz[i] for 0 < i < M must be > 0    */
  const double* cn2dz;      /* HOST [M]: integral of Cn^2 over screen i's interval [m^(1/3)], >= 0 */
  double l0;                /* inner scale [m]; <= 0 disables the inner-scale cutoff            */
  double L0;                /* outer scale [m]; <= 0 or infinite disables it                    */
  int32_t sh_levels;        /* Lane subharmonic levels 0..3 (scale 3 per level, Sec. 2.2)        */
  int32_t tf_kind;          /* turpy_tf_kind                                                    */
  int32_t inner_scale_conv; /* 0: fm = 1/l0 (Eq. S17 as printed, in cycles/m); 1: fm = 5.92/(2 pi l0) */
  int64_t realizations;     /* R >= 1                                                           */
  double psd_alpha;         /* power law of the PSD, W ~ f^-alpha (App. B Eq. S12/S15, Table S1);
                               0 selects 11/3 (Eq. S17); otherwise 2 < alpha < 6               */
} turpy_path;

typedef struct turpy_plan turpy_plan;

/* Operations for turpy_workspace_size. */
typedef enum {
  TURPY_OP_SCREEN_GENERATE = 0,
  TURPY_OP_PROPAGATE = 1,
  TURPY_OP_PROPAGATE_BACKWARD = 2,
  TURPY_OP_EVOLVE = 3,
  TURPY_OP_PROPAGATE_BACKWARD_REVERSIBLE = 4,
  TURPY_OP_TUNE = 5
} turpy_op;

/* Library version string (static storage). */
const char* turpy_version(void);

/* Message for the last non-OK status returned on this thread (static
 * thread-local storage; empty string when none). */
const char* turpy_last_error(void);

/* Validate `path`, compute the per-screen scalars (Fried parameter r0_i from
 * Eq. S18 and the PSD scale of Eq. S17), and build the FP64-derived tables on
 * the current HIP device: FFT twiddles, per-distance Fresnel chirps
 * exp(-i pi (lambda/n0) dz f^2) with exact FP64 range reduction, and the
 * subharmonic phasors of Eq. 2.  The host arrays dz/cn2dz are copied; the
 * caller may free them on return.  *out receives a plan owned by the caller
 * (release with turpy_plan_destroy).  Errors: INVALID (NULL pointers, N not a
 * power of two, non-finite or negative values), UNSUPPORTED (N outside 16..2048,
 * sh_levels > 3, a zero interior distance), ALIASING (a distance beyond
 * N dx^2 n0 / lambda, Eq. 7 with the Nyquist frequency, unless flags has
 * TURPY_ALLOW_ALIASING), HIP. */
turpy_status turpy_plan_create(turpy_plan** out, const turpy_path* path, uint32_t flags);
/* Releases the plan's device tables with hipFree, which waits for the device:
 * not while any stream of the device is being captured into a graph (a
 * capture in global mode is then invalidated), and not while the plan's work
 * is still to run.  NULL is accepted. */
turpy_status turpy_plan_destroy(turpy_plan* plan);

/* Bytes of the checkpoint buffer of turpy_propagate / turpy_propagate_backward:
 * complex64 fields [R][M][N][N] (the field just after each screen), followed,
 * for a plan created with TURPY_SCREEN_CHECKPOINTS, by the column halves of
 * the screens complex64 [M][ceil(R/2)][N][N] (each pair's screen after its
 * inverse transform along y, in revolutions; synthesised or stored-spectrum
 * screens only).  The forward pass writes both; the adjoint reads both and
 * then synthesises no screen: the same bytes move, and the adjoint's
 * synthesis work is saved for M ceil(R/2) N^2 8 bytes of memory. */
turpy_status turpy_checkpoint_size(const turpy_plan* plan, size_t* bytes);

/* Bytes of device workspace an operation needs for this plan (0 allowed). */
turpy_status turpy_workspace_size(const turpy_plan* plan, int32_t op, size_t* bytes);

/* Phase screens (App. B Eq. S16 with the Eq. S17 PSD, Sec. 2.2 Eq. 2-3, piston
 * removed): writes float screens[R][M][N][N] in radians for time step t (0 for
 * static screens).  `ws` must hold turpy_workspace_size(TURPY_OP_SCREEN_GENERATE). */
turpy_status turpy_screen_generate(turpy_plan* plan, uint64_t seed, int64_t t, float* screens,
                                   void* ws, size_t ws_bytes, void* stream);

/* Forward split-step (Sec. 2.1 Eq. 1): for i < M, diffract by dz[i] and
 * multiply by exp(i phi_i); finally diffract by dz[M].
 *  u_in       complex64 [R][N][N] (u_in_stride = N*N) or one shared source
 *             [N][N] (u_in_stride = 0).  Read only.  May equal u_out only when
 *             u_in_stride = N*N.
 *  src/screens_or_spectra  per turpy_screen_src (NULL for SYNTH).
 *  u_out      complex64 [R][N][N], written.
 *  checkpoints turpy_checkpoint_size bytes or NULL: the field just after
 *             each screen (complex64 [R][M][N][N]) and, with
 *             TURPY_SCREEN_CHECKPOINTS, the screens' column halves, for
 *             turpy_propagate_backward.
 *  ws         turpy_workspace_size(TURPY_OP_PROPAGATE) bytes. */
turpy_status turpy_propagate(turpy_plan* plan, uint64_t seed, int64_t t, const void* u_in,
                             int64_t u_in_stride, int32_t src, const void* screens_or_spectra,
                             void* u_out, void* checkpoints, void* ws, size_t ws_bytes, void* stream);

/* turpy_propagate without a workspace argument, for callers that cannot
 * allocate device memory (code under graph capture, tight serving loops,
 * harnesses that forbid allocation).  It allocates nothing: its scratch
 * (screen planes, subharmonic coefficients, the shared-source plane) lives in
 * a fixed 64 MiB device array of the library, one per GPU, held until the
 * process ends; the array's address is looked up by turpy_plan_create.  Other
 * arguments and results as turpy_propagate (bit-identical).  A plan whose
 * turpy_workspace_size(TURPY_OP_PROPAGATE) exceeds 64 MiB is refused with
 * TURPY_E_WORKSPACE (N = 1024: at most 14 realizations; N = 512: 62).
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind (no part of it needs to start at zero): calls that overlap on one
 * GPU -- on different streams, or from different threads -- race. */
turpy_status turpy_propagate_static(turpy_plan* plan, uint64_t seed, int64_t t, const void* u_in,
                                    int64_t u_in_stride, int32_t src, const void* screens_or_spectra, void* u_out,
                                    void* checkpoints, void* stream);

/* Screen-spectrum evolution (Sec. 2.3) of an AR state, in place.  The state
 * (turpy_state_size bytes, device memory) is complex64 spectra
 * [ceil(R/2)][M][N][N] in radians, followed, when the plan has subharmonic
 * levels, by [ceil(R/2)][M][32] complex64 subharmonic coefficients in radians
 * (the 24 points of Eq. 2, level-major in the offset order (m, n) = (-1,-1),
 * (-1,0), (-1,1), (0,-1), (0,1), (1,-1), (1,0), (1,1); then their grid mean;
 * then padding).  With t == 0: the static main spectra of Eq. S16 (DC zero)
 * and the static subharmonic coefficients, so that the state reproduces the
 * synthesised screens of t = 0.  With t >= 1: the frozen-flow shift of Eq. 4
 * by (shift_x, shift_y) pixels (= T v / dx), then the AR(1) blend of Eq. 5 with
 * innovation noise drawn at time step t; the subharmonic coefficients take
 * the same two steps at their frequencies (n, m) df / 3^p (innovation tag 4).
 * 0 <= alpha <= 1. */
turpy_status turpy_evolve(turpy_plan* plan, uint64_t seed, int64_t t, double alpha, double shift_x,
                          double shift_y, void* spectra, void* ws, size_t ws_bytes, void* stream);

/* The complex normals N_c of a spectrum on their own (App. B Eq. S16; the
 * same numbers the synthesis and the evolution draw inside their kernels):
 * out complex64 [pairs][n][n] (device), bin (k0, k1) of pair j from the
 * Philox counter (k0 n + k1, t, j, tag << 28 | screen) for k0 < n/2 (words 0-1,
 * Box-Muller) and the bin (k0 + n/2, k1) from the same block (words 2-3).
 * tag: 1 main spectrum, 3 AR innovation (others accepted).  For building the
 * path one operation per kernel (a baseline) or inspecting the noise.
 * Errors: INVALID for n not a power of two in 2..65536, tag outside 1..15,
 * screen outside 0..2^28-1, t outside 0..2^32-1. */
turpy_status turpy_noise(int32_t n, int64_t pairs, uint64_t seed, int64_t t, int32_t tag, int32_t screen, void* out,
                         void* stream);

/* One time step of the autoregressive path (Sec. 2.3 then Sec. 2.1): the AR
 * step of turpy_evolve (t >= 1) followed by turpy_propagate from the evolved
 * state (src TURPY_SCREENS_SPECTRA), with the evolution of each screen's
 * spectra done inside that screen's synthesis pass: the state is read once,
 * evolved in registers (Eq. 4 translation with the phase reduced in FP64, then
 * the Eq. 5 blend with innovations of tag 3 at step t), written back, and
 * transformed along y in the same pass, which saves the separate evolution
 * pass's read and write of the whole state.  Results equal turpy_evolve then
 * turpy_propagate up to FP32 rounding.  Subharmonic coefficients take their
 * step in a small kernel first.  Arguments as for turpy_evolve and
 * turpy_propagate; ws: turpy_workspace_size(TURPY_OP_PROPAGATE) bytes.
 * Errors: INVALID for t < 1 (initialise the state with turpy_evolve at t = 0),
 * alpha outside [0, 1], non-finite shifts. */
turpy_status turpy_evolve_propagate(turpy_plan* plan, uint64_t seed, int64_t t, double alpha, double shift_x,
                                    double shift_y, void* state, const void* u_in, int64_t u_in_stride,
                                    void* u_out, void* checkpoints, void* ws, size_t ws_bytes, void* stream);

/* Device-resident time step, for graph replays.  With dev_t set (a uint32
 * in device memory, 4-byte aligned), every kernel of this plan that draws
 * noise (screen synthesis, subharmonics, AR innovations) reads its time step
 * from *dev_t when it runs, instead of the t passed to the call; a captured
 * call then draws fresh noise on each replay after the caller updates *dev_t.
 * turpy_evolve still decides initialisation (t == 0) from its t argument.
 * NULL restores the argument.  The pointer is kept; the memory stays the
 * caller's. */
turpy_status turpy_plan_bind_time(turpy_plan* plan, const void* dev_t);

/* Ensemble moments taken inside the forward pass (Sec. 3.3).  With moments
 * set (float [4][N][N] in device memory, the layout of turpy_stats), every
 * forward call of this plan (turpy_propagate, turpy_evolve_propagate,
 * turpy_propagate_static) also adds its R output fields to those sums, with
 * the same bits as a turpy_stats(N, dx, R, u_out, moments, 0, 0, ...) call
 * after it.  Where the pass ends with a plain inverse row transform (a
 * distance after the last screen) the sums are taken inside that transform
 * and the output planes are not read back; otherwise the moment kernel runs
 * after it.  The caller keeps the realization count for the finalize call.
 * NULL unbinds.  The pointer is kept; the memory stays the caller's. */
turpy_status turpy_plan_bind_moments(turpy_plan* plan, float* moments);

/* Bytes of the plan's AR state (see turpy_evolve). */
turpy_status turpy_state_size(const turpy_plan* plan, size_t* bytes);

/* Adjoint of turpy_propagate with the same plan, seed, t and screens: the
 * gradients of a real loss through the split-step of Sec. 2.1 Eq. 1, which
 * the paper differentiates end to end to train optics placed before and after
 * the path (Sec. 1, Sec. 4).  Each diffraction step's adjoint is the same step
 * with conj(H); through screen i, dL/dphi_i = Im(conj(W_i) g) with W_i the
 * field just after the screen, then g <- exp(-i phi_i) g.
 *  grad_u_out  complex64 [R][N][N], read only.
 *  checkpoints turpy_checkpoint_size bytes written by the forward call with
 *              the same plan (NULL allowed when M = 0); with
 *              TURPY_SCREEN_CHECKPOINTS the screens are read from it.
 *  grad_u_in   dL/du_in or NULL.  grad_u_in_stride = N*N: complex64
 *              [R][N][N], one gradient per realization (also used as the
 *              working buffer).  grad_u_in_stride = 0: complex64 [N][N], the
 *              gradient of a source shared by every realization (the forward
 *              call's u_in_stride = 0), i.e. the sum over realizations; the
 *              sum is taken right after screen 0 (Kahan-compensated, in
 *              realization order) and the first diffraction's adjoint runs
 *              once on it.  Other strides: TURPY_E_INVALID.
 *  grad_screens float [R][M][N][N] dL/dphi_i, or NULL.
 *  ws          turpy_workspace_size(TURPY_OP_PROPAGATE_BACKWARD) bytes. */
turpy_status turpy_propagate_backward(turpy_plan* plan, uint64_t seed, int64_t t, const void* grad_u_out,
                                      const void* checkpoints, int32_t src, const void* screens_or_spectra,
                                      void* grad_u_in, int64_t grad_u_in_stride, float* grad_screens, void* ws,
                                      size_t ws_bytes, void* stream);

/* The adjoint of turpy_propagate without checkpoints (same operation as
 * turpy_propagate_backward, Sec. 2.1 Eq. 1).  When every step of the path is
 * unitary -- Fresnel transfer functions, or angular-spectrum ones whose bins
 * all propagate -- the forward field at each screen plane is rebuilt by
 * running the same adjoint steps on the forward output: the memory of the
 * [R][M][N][N] checkpoints is replaced by two [R][N][N] fields in the
 * workspace, at the price of a second chain of passes.  Results equal
 * turpy_propagate_backward's up to FP32 rounding (the rebuilt fields carry the
 * rounding of both chains).  A plan whose angular-spectrum grid has evanescent
 * bins (|H| < 1, the plan keeps its FP64 table) is not unitary: the call
 * returns TURPY_E_UNSUPPORTED and enqueues nothing.
 *  u_out   complex64 [R][N][N], the output of the forward call with the same
 *          plan, seed, t and screens; read only.  May be NULL when M = 0.
 *  Other arguments as for turpy_propagate_backward; ws holds
 *  turpy_workspace_size(TURPY_OP_PROPAGATE_BACKWARD_REVERSIBLE) bytes. */
turpy_status turpy_propagate_backward_reversible(turpy_plan* plan, uint64_t seed, int64_t t,
                                                 const void* grad_u_out, const void* u_out, int32_t src,
                                                 const void* screens_or_spectra, void* grad_u_in,
                                                 int64_t grad_u_in_stride, float* grad_screens, void* ws,
                                                 size_t ws_bytes, void* stream);

/* Ensemble statistics of received fields (Sec. 3.2-3.3, Eq. S25; Sec. 4.1).
 *  If batch > 0: accumulate I = |u|^2 of u[batch][n][n] into
 *  moments float [4][n][n] = (sum I, its compensation, sum I^2, its
 *  compensation), Kahan-compensated; zero `moments` before the first batch.
 *  The batch is summed in C = clamp(256 / (n / 16), 4, 64) contiguous chunks,
 *  chunk c holding entries [c batch / C, (c + 1) batch / C) in order, and the
 *  compensated sums of the non-empty chunks join the stored ones in chunk
 *  order: a fixed order for a given (n, batch), bitwise reproducible.
 *  If finalize != 0: with count = total realizations accumulated and
 *  m = sums / count, write si_map float [n][n] = m2/m1^2 - 1 (may be NULL)
 *  and summary double[8] (device):
 *    [0] SI averaged over the region, weighted: sum w SI / sum w;
 *    [1] W_2nd = sqrt(2 sum r^2 m1 / sum m1);
 *    [2] W_fit, least-squares fit of ln m1 = a - 2 r^2/W^2 over m1 >= e^-2 max m1;
 *    [3] count;
 *    [4] sum w SI over the region (the summed scintillation of Sec. 4.1);
 *    [5] sum w over the region;
 *    [6] the region's threshold intensity (power cutoff), else 0;
 *    [7] 0.
 *  The region: power_fraction = 0 selects the central pixels |i - n/2| < n/4
 *  in both directions; 0 < power_fraction <= 1 the power-cutoff region of
 *  Sec. 4.1 (99.9 % there): the pixels with m1 >= t, t the largest value for
 *  which they hold power_fraction of sum m1 (decided on m1 rounded to FP32).
 *  weight: float [n][n] device weights (an aperture mask, for instance) or
 *  NULL for 1.  Errors: INVALID for power_fraction outside [0, 1]. */
turpy_status turpy_stats(int32_t n, double dx, int64_t batch, const void* u, float* moments, int64_t count,
                         int32_t finalize, const float* weight, double power_fraction, float* si_map,
                         double* summary, void* stream);

/* Set-up of the plan-less receiver calls for grid size n on the current
 * device: builds their FP64-generated twiddle table (allocates and uploads
 * synchronously; not for a capturing stream).  Idempotent; the tables live
 * until the process ends.  turpy_receiver / turpy_receiver_backward return
 * TURPY_E_INVALID for an n not set up on the current device. */
turpy_status turpy_receiver_setup(int32_t n);

/* Dual-domain two-mask receiver (Sec. 2.5, Sec. 4.1):
 *  U1 = A u exp(i theta1) (A: disc of `aperture_diameter` metres centred on
 *  pixel (n/2, n/2)); Z = DFT{U1} exp(i theta2') with theta2' the natural-order
 *  view of theta2 (theta2 stored centred, fftshift order);
 *  u_out = IDFT{Z} (1/n^2 inverse).  u, u_out complex64 [batch][n][n] (must
 *  not alias); theta1, theta2 float [n][n] radians.  The forward pass needs no
 *  workspace (ws may be NULL).  n: power of two 16..2048. */
turpy_status turpy_receiver_workspace_size(int32_t n, int64_t batch, size_t* bytes);
turpy_status turpy_receiver(int32_t n, double dx, double aperture_diameter, int64_t batch, const void* u,
                            const float* theta1, const float* theta2, void* u_out, void* ws,
                            size_t ws_bytes, void* stream);

/* Adjoint of turpy_receiver: given grad_out [batch][n][n] returns
 * grad_u [batch][n][n] (or NULL), and dL/dtheta1, dL/dtheta2 float [n][n]
 * summed over the batch (theta2 gradient in centred order; either may be
 * NULL).  The batch sums are taken in a fixed order (bitwise reproducible).
 * ws: turpy_receiver_workspace_size(n, batch) bytes. */
turpy_status turpy_receiver_backward(int32_t n, double dx, double aperture_diameter, int64_t batch,
                                     const void* u, const float* theta1, const float* theta2,
                                     const void* grad_out, void* grad_u, float* grad_theta1,
                                     float* grad_theta2, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Uneven batches: many path instances, each with its own grid size, screen
 * count, wavelength and distances, propagated by one call on the caller's
 * stream.  Instances that share the grid size, the realization count and the
 * transfer-function form, have every distance > 0 and at most 2^20 pixels
 * per pass (R N^2; larger ones fill the GPU alone) run in groups: each pass of
 * the forward pass and of the adjoint is one launch over the group's members.
 * A group holds as many members as keep its working set (fields and
 * workspace of its members) within the group limit (turpy_batch_group_limit).
 * Groups and the other instances are spread over a few internal streams of
 * default priority (longest processing time first, cost R N^2 (M + 1)),
 * forked from and joined back to the caller's stream with events; nothing is
 * allocated and no memset is issued, so the calls can be captured in a HIP
 * graph.  Screens
 * are synthesised (Eq. S16, Eq. 2-3); instance i draws its noise with the key
 * seed + i * 0x9E3779B97F4A7C15 (mod 2^64), otherwise exactly as
 * turpy_propagate with its own plan.  Not thread-safe (one call at a time per
 * batch).
 * ------------------------------------------------------------------------- */
typedef struct turpy_batch turpy_batch;

/* paths [num_paths] as for turpy_plan_create (the dz / cn2dz arrays are read
 * here only); field_offsets [num_paths]: element (complex64) offset of
 * instance i's fields [R_i][N_i][N_i] in the packed field buffers; the fields
 * of different instances must not overlap (TURPY_E_INVALID).  A path that
 * fails turpy_plan_create's validation fails the batch with its status.
 * flags as for turpy_plan_create, except TURPY_SCREEN_CHECKPOINTS
 * (TURPY_E_INVALID). */
turpy_status turpy_batch_create(turpy_batch** out, const turpy_path* paths, const int64_t* field_offsets,
                                int32_t num_paths, uint32_t flags);
/* Releases the batch's plans and device records (hipFree): the conditions
 * of turpy_plan_destroy apply.  NULL is accepted. */
turpy_status turpy_batch_destroy(turpy_batch* batch);
/* turpy_plan_bind_time for every instance of the batch. */
turpy_status turpy_batch_bind_time(turpy_batch* batch, const void* dev_t);
/* Working-set limit of a group, in bytes, for batches created from now on
 * (process-wide; 0 restores the default, 1 GiB).  It bounds a group's
 * workspace; a member alone beyond the limit runs its own plan's calls. */
turpy_status turpy_batch_group_limit(size_t bytes);
/* op: TURPY_OP_PROPAGATE, TURPY_OP_PROPAGATE_BACKWARD or TURPY_OP_TUNE. */
turpy_status turpy_batch_workspace_size(const turpy_batch* batch, int32_t op, size_t* bytes);
/* u_in / u_out: packed fields (instance i at field_offsets[i], one source
 * plane per realization; u_in == u_out allowed).  checkpoints (NULL = none):
 * packed instance after instance, [R_i][M_i][N_i][N_i] each, in order i. */
turpy_status turpy_batch_propagate(turpy_batch* batch, uint64_t seed, int64_t t, const void* u_in, void* u_out,
                                   void* checkpoints, void* ws, size_t ws_bytes, void* stream);
/* The adjoint of turpy_batch_propagate: grad_u_out / grad_u_in packed like
 * the fields, checkpoints and grad_screens (float) packed like the
 * checkpoints; grad_u_in or grad_screens may be NULL. */
turpy_status turpy_batch_propagate_backward(turpy_batch* batch, uint64_t seed, int64_t t, const void* grad_u_out,
                                            const void* checkpoints, void* grad_u_in, float* grad_screens,
                                            void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Screen placement (Sec. 2.4; App. C Eq. S18-S21).  Host arithmetic only: no
 * device memory, no stream and no GPU are involved.
 * ------------------------------------------------------------------------- */
typedef enum {
  TURPY_CN2_UNIFORM = 0,         /* Cn2(z) = cn2                                                     */
  TURPY_CN2_HUFNAGEL_VALLEY = 1, /* Eq. S21 with ground constant A [m^-2/3] and wind speed V [m/s];
                                    z is the height above the ground (vertical path from the ground) */
  TURPY_CN2_TABLE = 2            /* piecewise linear through (z[i], values[i]), count >= 1, z strictly
                                    increasing; constant beyond the first and the last point         */
} turpy_cn2_kind;

typedef struct turpy_cn2_profile {
  int32_t kind;                  /* turpy_cn2_kind                                                   */
  double cn2;                    /* UNIFORM: Cn2 >= 0                                                */
  double A, V;                   /* HUFNAGEL_VALLEY: A >= 0, V >= 0                                  */
  const double* z;               /* TABLE: HOST [count] positions [m]                                */
  const double* values;          /* TABLE: HOST [count] Cn2 >= 0                                     */
  int64_t count;                 /* TABLE: number of points                                          */
} turpy_cn2_profile;

/* Screen placement along [0, length] for a grid of n points spaced dx
 * (Sec. 2.4).  In order:
 *  1. `initial` >= 1 equal intervals;
 *  2. every interval whose Rytov variance (Eq. S19 over the interval, with
 *     k = 2 pi n0 / wavelength) exceeds rytov_limit is halved, until none does;
 *  3. neighbours are merged, left to right, while the merged interval stays
 *     within the limit;
 *  4. the interior boundaries move, keeping their number, to equal shares of
 *     the cumulative Rytov variance interpolated linearly between the current
 *     boundaries; step 2 is repeated;
 *  5. every interval longer than the Eq. 7 step (N dx / 2) sqrt(n0^2 k0^2 -
 *     kappa0^2) / kappa0, kappa0 = 2 pi / dx, k0 = 2 pi / wavelength, is halved
 *     until none is.
 * One screen sits at the middle of each interval.  Outputs, HOST arrays sized
 * by max_screens: dz [M+1] in the layout of turpy_path.dz, cn2dz [M] the
 * integral of Cn2 over each interval, rytov [M] Eq. S19 of each interval (may
 * be NULL); *num_screens = M.  Integrals use composite Gauss-Legendre
 * quadrature (relative error near 1e-13 for the profiles above).
 * Errors: TURPY_E_INVALID for a malformed profile or argument, for dx <=
 * wavelength / n0 (Eq. 7 has no real step) or when more than 65536 intervals
 * would be needed; TURPY_E_CAPACITY when M > max_screens (*num_screens then
 * holds M and the arrays are untouched). */
turpy_status turpy_place_screens(const turpy_cn2_profile* profile, double length, double wavelength, double n0,
                                 int32_t n, double dx, double rytov_limit, int32_t initial, int32_t max_screens,
                                 int32_t* num_screens, double* dz, double* cn2dz, double* rytov);

/* ---------------------------------------------------------------------------
 * Launch-configuration tuning.  Three choices are searched, none of which
 * changes what is computed beyond FP32 rounding order:
 *  - the column pass (FFT along y, transfer function, inverse FFT; Sec. 2.1)
 *    and the column half of the screen synthesis (Eq. S16) run one block per
 *    strip of K adjacent columns of a plane, K in {4, 8, 16} (K N / 16
 *    threads per block, at most 1024, and K N complex words of LDS; at
 *    N = 2048 K = 16 does not fit): K sets the block size, the occupancy and
 *    the width of each memory segment; results are bit-identical for every K;
 *  - the radix plan of their transforms: every transform starts with a
 *    radix-16 pass; the second pass has radix R2 (default min(16, N/16)) and
 *    the third N / (16 R2); R2 in {8, 4} is also built for N = 512 and 1024
 *    and R2 = 8 for N = 2048 (other plans round differently, within the
 *    oracle tolerance);
 *  - the occupancy hint of the screen row passes, forward and adjoint: the
 *    minimum waves per SIMD (2, 3 or 4) the register allocation must allow;
 *    3 is the default, 2 and 4 are built for N >= 256 (bit-identical results).
 * A plan starts from the built-in choices (measured on MI355X), or from the
 * process-wide cache when it holds an entry for the plan's key:
 *   (device architecture, kernel, N, batch class = bit length of the number
 *    of planes one launch covers: R for the column pass, ceil(R/2) for the
 *    synthesis and the row passes).
 * ------------------------------------------------------------------------- */
typedef enum {
  TURPY_TUNE_COL_FRESNEL = 0,   /* column pass, Fresnel transfer function               */
  TURPY_TUNE_COL_ANGULAR = 1,   /* column pass, angular spectrum, every bin propagating */
  TURPY_TUNE_COL_AS_TABLE = 2,  /* column pass, angular spectrum with evanescent bins   */
  TURPY_TUNE_SYNTH = 3,         /* column half of the screen synthesis                  */
  TURPY_TUNE_ROW_FWD = 4,       /* forward screen row pass (no checkpoints)             */
  TURPY_TUNE_ROW_BWD = 5,       /* adjoint screen row pass                              */
  TURPY_TUNE_SYNTH_AR = 6       /* the synthesis with the AR step fused into it
                                   (turpy_evolve_propagate): its own choice, since
                                   the best strip differs from the plain synthesis's */
} turpy_tune_kernel;

#define TURPY_TUNE_FORCE 1u     /* measure even when the cache holds the key */

typedef struct turpy_tune_entry {
  char arch[32];                /* device architecture, e.g. "gfx950" (NUL-terminated)             */
  int32_t kernel;               /* turpy_tune_kernel                                                */
  int32_t n;                    /* grid size                                                        */
  int32_t batch_class;          /* bit length of the planes per launch                              */
  int32_t width;                /* columns per block (4, 8, 16); 0 for the row kernels              */
  int32_t radix;                /* second-pass radix (0: default plan); 0 for the row kernels       */
  int32_t waves;                /* occupancy hint of the row kernels (2, 3, 4); 0 for the others    */
  int32_t configs;              /* configurations measured (0 when put by hand)                     */
  float us;                     /* microseconds per launch of the chosen configuration              */
  float us_default;             /* of the built-in configuration (0: not measured)                  */
} turpy_tune_entry;

/* The launch choices of a plan (0 in set_config: the built-in choice). */
typedef struct turpy_launch_config {
  int32_t col_width, col_radix;     /* column pass                               */
  int32_t synth_width, synth_radix; /* column half of the synthesis              */
  int32_t row_waves;                /* forward screen row passes                 */
  int32_t row_waves_bwd;            /* adjoint screen row passes                 */
  int32_t ar_width, ar_radix;       /* the synthesis with the AR step fused      */
} turpy_launch_config;

/* Time every launch configuration of the plan's column pass (its
 * transfer-function kind, distance 0, all R planes in place), and, when the
 * plan has screens, of its synthesis (all ceil(R/2) scratch planes; once
 * plain and once with the AR step fused, on workspace planes as the state)
 * and of its forward and adjoint row passes for screen 0 (workspace planes), with
 * HIP events on `stream`, and keep the fastest of each in the plan and in the
 * cache.  A key already in the cache is applied without measuring unless
 * flags has TURPY_TUNE_FORCE.  Each configuration: one launch, then 3
 * repetitions of a loop of launches lasting about 2 ms; the minimum
 * per-launch time counts.  ws: turpy_workspace_size(TURPY_OP_TUNE) bytes of
 * device memory, zeroed and overwritten here (no caller data is touched).
 * Synchronises `stream`: it cannot be captured in a graph (TURPY_E_INVALID
 * while the stream captures).  col_width / synth_width (may be NULL) receive
 * the strip widths now in the plan (turpy_plan_config has every choice). */
turpy_status turpy_plan_tune(turpy_plan* plan, uint32_t flags, void* ws, size_t ws_bytes, void* stream,
                             int32_t* col_width, int32_t* synth_width);
/* The strip widths the plan's launches use now. */
turpy_status turpy_plan_widths(const turpy_plan* plan, int32_t* col_width, int32_t* synth_width);
/* Set the strip widths directly: 0 restores the built-in choice; any other
 * value must be a width built for the plan's N (TURPY_E_INVALID otherwise,
 * and the plan is unchanged). */
turpy_status turpy_plan_set_widths(turpy_plan* plan, int32_t col_width, int32_t synth_width);
/* Every launch choice of the plan now (built-in choices filled in). */
turpy_status turpy_plan_config(const turpy_plan* plan, turpy_launch_config* config);
/* Set every launch choice (0 fields: built-in); TURPY_E_INVALID for a
 * choice not built for the plan's N (the plan is then unchanged). */
turpy_status turpy_plan_set_config(turpy_plan* plan, const turpy_launch_config* config);
/* The cache (host memory, process-wide, guarded by a lock): get copies up to
 * `capacity` entries in key order and sets *count to the number held (so a
 * call with capacity 0 sizes the array); put inserts or replaces entries by
 * key (TURPY_E_INVALID for a choice not built for the entry's n or an unknown
 * kernel; entries before the bad one are kept); clear empties it.  Plans
 * created afterwards start from the cached choices; existing plans keep
 * theirs.  These three calls touch no device. */
turpy_status turpy_tune_cache_get(turpy_tune_entry* entries, int32_t capacity, int32_t* count);
turpy_status turpy_tune_cache_put(const turpy_tune_entry* entries, int32_t count);
turpy_status turpy_tune_cache_clear(void);
/* turpy_plan_tune for every instance of the batch (each distinct key is
 * measured once; later instances take it from the cache).  ws:
 * turpy_batch_workspace_size(TURPY_OP_TUNE) bytes; synchronises `stream`. */
turpy_status turpy_batch_tune(turpy_batch* batch, uint32_t flags, void* ws, size_t ws_bytes, void* stream);

/* Per-kernel timing for benchmarking.  turpy_profile(1) clears the record and
 * starts bracketing every kernel the library enqueues with a pair of HIP events
 * on that kernel's stream; turpy_profile(0) stops recording.  Kernel families:
 * "row_fwd", "row_bwd", "row_plain", "row_moments", "col", "synth", "sh", "evolve",
 * "stats", "finalize", "copy", "sum", "noise", "nonfinite", "recv_row", "recv_col",
 * "recv_col_grad", "recv_row_grad", "recv_reduce".  turpy_profile_read waits for the recorded events and
 * returns the launch count and summed duration (ms) of one family (zero when it
 * never ran).  turpy_profile_only(family) restricts the bracketing to one
 * family (the others launch with no events around them, so that timing one
 * kernel perturbs the rest of a pass as little as possible); NULL or "" times
 * every family again.  The family string is copied.  Host-side state,
 * process-wide; not thread-safe. */
turpy_status turpy_profile(int32_t enable);
turpy_status turpy_profile_only(const char* family);
turpy_status turpy_profile_read(const char* family, int64_t* launches, double* total_ms);

/* Launch-failure injection, for testing error handling from the host: with
 * k > 0, the k-th kernel launch the library enqueues from now on (any plan,
 * batch or thread; counting from 1) is not enqueued, and the entry point that
 * enqueues it returns TURPY_E_HIP with a message saying the failure was
 * injected, exactly as it would for a failed launch.  The countdown then
 * disarms; k = 0 disarms it at once.  The outputs of the failed call (and an
 * AR state it was updating) are undefined; plans and batches stay usable. */
turpy_status turpy_debug_fail_launch(int64_t k);

#ifdef __cplusplus
}
#endif

#endif /* TURPY_H_ */
