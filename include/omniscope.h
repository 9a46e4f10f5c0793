/*
 * omniscope.h -- C ABI of the MI355X (gfx950) hierarchical-grid correlator.
 *
 * What it computes (Tegmark & Zaldarriaga, "Omniscopes", Sec. II):
 *   Antennas sit on an L-level hierarchy of rectangular grids,
 *   r = sum_l A_l (i_lx, i_ly)  (Sec. II.D, Eq. GridEq).  One channel's voltages
 *   at one time form the 2L-dimensional hypercube F_{i_1 ... i_2L}.  The
 *   visibility hypercube, i.e. every antenna pair's correlation summed over all
 *   pairs sharing the same index difference Delta, is
 *
 *       V_f[Delta] = sum_t sum_j x_{t,f,j} conj(x_{t,f,j-Delta}),
 *       Delta_k in [-(n_k-1), n_k-1]          (Sec. II.D, Eq. ProofEq2)
 *
 *   and is computed the fast way (Sec. II.A, II.C): zero-pad every axis to
 *   m_k = 2 n_k, 2L-dimensional DFT, square modulus, sum over the time samples,
 *   one inverse DFT per channel.  The lattice matrices A_l never enter the
 *   arithmetic (Sec. II.D); they only label each output cell with its physical
 *   baseline (omni_baselines).
 *
 * Conventions shared by every entry point
 *   - Every call returns OMNI_OK (0) or a negative omni_status.  No C++
 *     exception crosses this boundary.  omni_last_error() gives a message for
 *     the most recent failure on the calling thread.
 *   - Diagnostics: the environment variable OMNI_LOG_LEVEL (read once per
 *     process) makes the library write to stderr: 1 = every failure as it is
 *     returned, 2 = also each new plan's description and every autotuner
 *     decision.  Unset or 0: silent.  The main entry points (plan, correlate,
 *     direct, F-engine, hybrid, fold) push a roctx range named after the call
 *     (rocprofv3 --marker-trace records them).
 *   - Axis order: axis 2l is level l's x index, axis 2l+1 its y index, levels
 *     in the caller's order (outermost first is the natural choice).  The
 *     antenna index a of a voltage sample is row-major over these axes.
 *   - Voltages: device memory [T][F][N] samples, 256-byte aligned, in one of
 *       OMNI_CF32 interleaved float32 (re, im)                 8 bytes/sample
 *       OMNI_CI8  interleaved int8 (re, im)                    2 bytes/sample
 *       OMNI_CI4  one byte, re = high nibble, im = low nibble,
 *                 two's complement, values in [-7, 7]         1 byte/sample
 *   - Visibilities: device memory, complex64 (float re, float im),
 *     [F][2n_1-1]...[2n_d-1] row-major, Delta_k stored at index Delta_k+n_k-1
 *     (centred).  V is Hermitian: V[-Delta] = conj V[Delta]; V[0] is the total
 *     power.  Plain sums: no 1/T and no per-pair normalisation.
 *   - The caller owns voltage and visibility buffers; the plan owns its
 *     twiddle tables, accumulators and workspace.  A plan is not re-entrant:
 *     calls on one plan must not overlap; distinct plans are independent.
 *   - omni_correlate* are asynchronous on the caller's HIP stream; results are
 *     valid once that stream has been synchronised.
 */
#ifndef OMNISCOPE_H
#define OMNISCOPE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  OMNI_OK = 0,
  OMNI_E_INVAL = -1,  /* null pointer, bad enum, bad size or flag            */
  OMNI_E_SHAPE = -2,  /* grid dimensions outside what a plan supports        */
  OMNI_E_GEOM = -3,   /* non-finite lattice matrix, or two antennas collide  */
  OMNI_E_NODEV = -4,  /* no usable gfx950 device                             */
  OMNI_E_NOMEM = -5,  /* device allocation failed or plan exceeds memory     */
  OMNI_E_HIP = -6,    /* a HIP runtime call failed (message has the detail)  */
  OMNI_E_STATE = -7   /* call not valid for this plan (e.g. host-only plan)  */
} omni_status;

typedef enum { OMNI_CF32 = 0, OMNI_CI8 = 1, OMNI_CI4 = 2 } omni_dtype;

/* Arithmetic form of the forward transforms.
 *   OMNI_FORM_FP32 : float32 DFT stages on the vector ALUs, float32 twiddles.
 *                    Error <= 1e-5 of the zero-lag power.
 *   OMNI_FORM_MIXED: float16 MFMA DFT stages with float32 accumulation,
 *                    twiddles split into float16 hi + lo parts, per-stage
 *                    power-of-two scaling.  Error <= 2e-3 of zero-lag power.
 * Both forms integrate |X|^2 in float32 over short blocks of time samples and
 * then in float64, and run the inverse transform with float64 sums (complex
 * float32 between its axes). */
typedef enum { OMNI_FORM_FP32 = 0, OMNI_FORM_MIXED = 1 } omni_form;

/* omni_opts.flags */
#define OMNI_PLAN_HOST_ONLY 0x1u /* geometry only: no device resources; correlate -> OMNI_E_STATE */
#define OMNI_PLAN_TIMING 0x2u    /* record HIP events around each stage of every correlate call  */
#define OMNI_PLAN_GRAPH 0x8u     /* run every correlate call as one HIP graph whose arrays are     \
                                    parallel branches (first call captured, later calls replay)  */
/* Beam-space ("digital pointing") variant of Appendix A, steps 4-5: the lowest
 * level (the last level, axes d-2 and d-1) consists of fully sampled n_x x n_y
 * blocks; every block is Fourier transformed over those two axes without zero
 * padding (pointing b = (b_x, b_y): B_b = sum_j x_j exp(-2 pi i (b_x j_x / n_x +
 * b_y j_y / n_y))), and each pointing is correlated over the outer levels as in
 * Sec. II (padded transforms, square modulus, time sum, inverse along the outer
 * axes only).  Visibilities: complex64 [F][2n_1-1]...[2n_{d-2}-1][n_x][n_y]
 * (pointings last).  Since the unpadded transform of a block is the
 * zero-padded one (m = 2n) at its even cells, B_b = X[2b], a grid whose
 * ordinary plan has a fixed-shape kernel (matrix-core or compile-time shape)
 * runs that kernel unchanged and keeps the even cells of the block axes
 * before the inverse; other grids run the general kernel with the block axes
 * unpadded.  Needs at least two levels and more than one block;
 * omni_baselines, the fold and the direct correlator refuse such plans
 * (OMNI_E_STATE). */
#define OMNI_PLAN_BEAMS 0x10u

/* flags argument of omni_correlate* */
#define OMNI_NO_RESET 0x1u    /* add this call's samples to the running accumulator            */
#define OMNI_NO_FINALIZE 0x2u /* skip the inverse transform (vis is not touched, may be NULL)  */

/* omni_opts.tune: the plan-time autotuner times candidate schedules (short-DFT
 * length cap x time slicing of the vector-ALU kernels; time slicing and the
 * float32 block of the matrix-core kernels) on an all-zero input of a few
 * samples with HIP events, and keeps the fastest.  The schedule changes only
 * speed, never the result beyond rounding order. */
typedef enum {
  OMNI_TUNE_OFF = 0,    /* the planner's fixed schedule                                   */
  OMNI_TUNE_CACHE = 1,  /* the schedule stored for this array in tune_cache, else search  */
  OMNI_TUNE_SEARCH = 2  /* always search; the result is appended to tune_cache if named   */
} omni_tune;

typedef struct {
  omni_dtype dtype;   /* sample format of the voltages                        */
  omni_form form;     /* arithmetic form of the forward transform             */
  int32_t time_block; /* samples per float32 block before the float64 add; 0 = default (64, mixed 1024) */
  uint32_t flags;     /* OMNI_PLAN_* flags                                    */
  int32_t tune;       /* omni_tune                                            */
  const char* tune_cache; /* text file of tuned schedules (one line per array key), or NULL;
                             read and appended at plan time only, never by correlate calls */
  int32_t chunk_T;    /* grids transformed partly by front passes (one channel's Fourier grid too
                         large for one work-group share): at most this many time samples per chunk
                         of the front workspace; 0 = the planner's choice (<= 256 samples, <= 8 GiB
                         per workspace, 16 GiB in the mixed form).  Smaller chunks use less memory. */
} omni_opts;

typedef struct omni_plan_s* omni_plan_t;

/* Plan one array: the n-level hierarchy of rectangular grids of Sec. II.D
 * (antenna positions r = sum_l A_l (i_lx, i_ly), Eq. GridEq) laid out as the
 * 2L-dimensional hypercube whose zero-padded transform (Sec. II.A, II.C: every
 * axis padded to m_k = 2 n_k, so that the circular correlation holds the whole
 * linear one) the correlate calls take.  The plan fixes the axis order, the
 * fold moduli of every axis' pruned DFT, the kernels and the workspaces.
 *   levels : L >= 1 levels of the hierarchy (d = 2L axes, d <= 8).
 *   dims   : [L][2] int32 (n_x, n_y) per level; each >= 1; N = prod n <= 2^22.
 *   A      : [L][2][2] float64 row-major; column c is the level's lattice vector
 *            of index c, in wavelengths at the reference frequency.  Used only
 *            for omni_baselines and the position-collision check; may be NULL
 *            (then no check and omni_baselines returns OMNI_E_STATE).
 *   nchan  : F >= 1 frequency channels.
 *   opts   : may be NULL (CF32, FP32 form, defaults).
 * On success *out holds a new plan (free with omni_destroy).  Device resources
 * (twiddles from a float64 generator kernel, accumulators, workspace) are
 * allocated on the current HIP device.  Errors: OMNI_E_INVAL, OMNI_E_SHAPE,
 * OMNI_E_GEOM, OMNI_E_NODEV, OMNI_E_NOMEM, OMNI_E_HIP. */
int omni_plan(omni_plan_t* out, int32_t levels, const int32_t* dims, const double* A, int32_t nchan,
              const omni_opts* opts);

/* One array of a batched plan (same fields as omni_plan's arguments). */
typedef struct {
  int32_t levels;
  const int32_t* dims; /* [levels][2] */
  const double* A;     /* [levels][2][2] or NULL */
  int32_t nchan;
} omni_array_desc;

/* Plan several arrays (possibly of different shapes) that are always
 * correlated together, in one launch sequence, with a common T: the same
 * per-channel correlation of Sec. II.D, Eq. ProofEq2 repeated over arrays and
 * frequency channels (Appendix A: the procedure is repeated for every
 * frequency bin of interest).  Sample format and form are shared.  Array i of
 * the plan is arrays[i].  Errors as for omni_plan. */
int omni_plan_batch(omni_plan_t* out, int32_t n_arrays, const omni_array_desc* arrays, const omni_opts* opts);

/* Correlate T time samples (T >= 0) of every channel: the visibility
 * hypercube V_f[Delta] of Sec. II.D, Eq. ProofEq2 (every pair's product summed
 * over the pairs sharing the index difference Delta), computed as in Sec. II.A
 * and II.C: zero-padded d-dimensional DFT of each sample's hypercube, square
 * modulus, sum over the samples (the time integration of Sec. II.A), one
 * inverse DFT per channel.  Integer samples give Gaussian-integer visibilities
 * which the float32 form reproduces to 1e-5 and the mixed form to 2e-3 of the
 * channel's zero-lag power.
 *   volt   : device [T][F][N] samples in the plan's format (may be NULL iff T == 0).
 *   vis    : device complex64 [F][2n_1-1]...[2n_d-1]; may be NULL with OMNI_NO_FINALIZE.
 *   stream : hipStream_t, or NULL for the default stream.
 *   flags  : OMNI_NO_RESET, OMNI_NO_FINALIZE.
 * Without OMNI_NO_RESET the plan's float64 accumulator restarts at zero; with
 * it, this call's samples are added (a long integration split over calls, or
 * resumed from omni_accumulator_set, equals the single call up to rounding).
 * T == 0 with no flags yields all-zero visibilities.
 * Errors: OMNI_E_INVAL (bad pointer/T/flags), OMNI_E_STATE (host-only plan),
 * OMNI_E_HIP. */
int omni_correlate(omni_plan_t plan, const void* volt, int64_t T, void* vis, void* stream, uint32_t flags);

/* Batched form of omni_correlate (same computation per array, Sec. II.D,
 * Eq. ProofEq2): volt[i] / vis[i] belong to array i of the batch plan, each in
 * that array's layout; all arrays share T.  volt and vis are host arrays of
 * n_arrays device pointers, read during the call only.
 * Without OMNI_PLAN_GRAPH the arrays run one after another on `stream`.  With
 * it, the plan captures its first call (all arrays, all stages) into one HIP
 * graph in which each array is an independent branch on a stream of its own,
 * so that the arrays' kernels overlap and fill each other's tails; the graph
 * is launched on `stream` and every later call replays it.  Later calls must
 * repeat the first call's T, flags and volt / vis pointers (the buffers'
 * contents may change): any other call returns OMNI_E_STATE (make another
 * plan for another call shape).  Results are identical to the sequential
 * form.  The graph holds no memset nodes. */
int omni_correlate_batch(omni_plan_t plan, const void* const* volt, int64_t T, void* const* vis, void* stream,
                         uint32_t flags);

/* Direct N^2 correlator on the GPU, the comparison baseline for the FFT forms
 * (the generic correlator whose cost grows as the number of antenna pairs,
 * Sec. I): every pair's product x_a conj(x_b) summed over the T samples and
 * binned by index difference Delta = idx(a) - idx(b), i.e. the visibility
 * hypercube of Sec. II.D, Eq. ProofEq2, by its definition.  Same input and
 * output layout as omni_correlate (complex64 [F][2n_1-1]...[2n_d-1], centred).
 * Integer samples only (plan dtype OMNI_CI8 or OMNI_CI4); int8 matrix-core
 * products with int32 sums over at most 32768 samples per launch and int64
 * sums after that, so the result is exact up to its final rounding to float32.
 * Requires a single-array plan with N a multiple of 128, fewer than 2^23 pairs
 * of blocks of 128 consecutive antennas, and at most 2048 index differences
 * per block pair (prod_k (2 e_k + 1) <= 2048, e_k the largest extent of a block
 * along axis k: 465 for a 16 x 16 grid, 675 for 8x8 tiles of 8x8).  The first
 * call allocates the plan's direct-correlator buffers (F x cells x 16 bytes of
 * int64 sums, the block-pair list); the call does not touch the plan's FFT
 * accumulator.  Asynchronous on `stream`, like omni_correlate.
 *   volt : device [T][F][N] samples, 8-byte (ci8) / 4-byte (ci4) aligned; may be NULL iff T == 0.
 *   vis  : device complex64 visibilities (written, never read).
 * Errors: OMNI_E_INVAL (bad pointer, alignment or T), OMNI_E_STATE (host-only
 * or batch plan, float samples), OMNI_E_SHAPE (N or block boxes outside the
 * limits above), OMNI_E_NOMEM, OMNI_E_HIP. */
int omni_direct_correlate(omni_plan_t plan, const void* volt, int64_t T, void* vis, void* stream);

/* omni_direct_correlate for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same computation, arguments, layouts and errors, and the
 * same visibilities bit for bit, but every buffer the direct correlator needs
 * beyond volt and vis (the int64 half-sums, the block pairs and block boxes,
 * which omni_direct_correlate allocates on its first call) lives in a fixed
 * 64 MiB device array of the library, one per device, held until the process
 * ends.  The call makes no device allocation.  It needs
 *   F x prod_k(2 n_k - 1) x 16 + (N/128)(N/128 + 1) x 4 + (N/128) x 64 bytes
 * (rounded to 256-byte blocks) of that array and returns OMNI_E_NOMEM, with
 * the sizes in the message, when they exceed 64 MiB (8 x 8 tiles of 8 x 8
 * antennas: up to 82 channels).  Every call on a device shares that device's
 * array and overwrites what the last call left there, so calls that overlap
 * on one device (another stream, another thread, another plan) race: order
 * them on one stream.  The array's address is looked up on the first call on
 * each device. */
int omni_direct_correlate_noalloc(omni_plan_t plan, const void* volt, int64_t T, void* vis, void* stream);

/* Number of arrays in the plan (1 for omni_plan).  Planning metadata, no
 * passage of the paper.  Errors: OMNI_E_INVAL (NULL argument). */
int omni_n_arrays(omni_plan_t plan, int32_t* n);

/* Visibility shape of array `array`: *ndim = 1 + d, shape = [F, 2n_1-1, ...],
 * one cell per index difference Delta_k in [-(n_k-1), n_k-1] (the index range
 * of Sec. II.D, Eq. ProofEq2; Sec. II.C's worked example has 2n-1 = 5 and 3
 * cells for n = 3 and 2); an OMNI_PLAN_BEAMS plan ends in [n_x, n_y]
 * pointings instead.  shape is host memory of at least 9 entries.
 * Errors: OMNI_E_INVAL (NULL argument, array out of range). */
int omni_vis_shape(omni_plan_t plan, int32_t array, int32_t* ndim, int64_t* shape);

/* Physical baseline of every visibility cell of array `array`:
 * uv[cell][2] = sum_l A_l (Delta_lx, Delta_ly) in wavelengths at the reference
 * frequency (Sec. II.D, Eq. GridEq applied to an index difference), cells in
 * the visibility layout.  uv is host memory of prod(2n_k-1)*2 doubles, written.
 * Errors: OMNI_E_INVAL (NULL argument, array out of range), OMNI_E_STATE
 * (planned without A). */
int omni_baselines(omni_plan_t plan, int32_t array, double* uv);

/* Size in bytes of the plan's float64 accumulator, the integration state
 * sum_t |X_t[kappa]|^2 of Sec. II.A (squared transforms summed over the time
 * samples before the single inverse transform): sum over arrays of
 * F * prod(2 n_k) doubles, [array][F][kappa_1]...[kappa_d], natural frequency
 * order.  Errors: OMNI_E_INVAL (NULL argument). */
int omni_accumulator_bytes(omni_plan_t plan, size_t* bytes);

/* Copy the accumulator (the time-summed power of Sec. II.A, layout as in
 * omni_accumulator_bytes) to / from `buf` (host or device memory owned by the
 * caller; `bytes` must equal omni_accumulator_bytes).  Synchronous with respect
 * to `stream`.  Together with OMNI_NO_RESET this checkpoints and resumes an
 * integration: the sum over time is linear, so a split integration equals the
 * whole one up to rounding.  Errors: OMNI_E_INVAL (NULL, wrong size),
 * OMNI_E_STATE (host-only plan), OMNI_E_HIP. */
int omni_accumulator_get(omni_plan_t plan, void* buf, size_t bytes, void* stream);
int omni_accumulator_set(omni_plan_t plan, const void* buf, size_t bytes, void* stream);

/* A JSON description of the schedule the planner chose (axis order, fold
 * moduli, work-group split, kernel variants, time chunk of the front passes).
 * Planning metadata, no passage of the paper.  Writes at most len bytes of
 * host memory including the terminating NUL (buf may be NULL when len is 0);
 * *needed receives the full length.  Errors: OMNI_E_INVAL (NULL plan). */
int omni_plan_describe(omni_plan_t plan, char* buf, size_t len, size_t* needed);

/* Stages timed by a plan made with OMNI_PLAN_TIMING. */
typedef enum {
  OMNI_STAGE_FORWARD = 0, /* forward transform + |X|^2 + time integration kernel(s)  */
  OMNI_STAGE_REDUCE = 1,  /* partial-sum reduction into the float64 accumulator      */
  OMNI_STAGE_INVERSE = 2, /* inverse transform to visibilities                       */
  OMNI_STAGE_CALL = 3,    /* the whole correlate call, on the caller's stream        */
  OMNI_STAGE_KERNEL = 4   /* per call, the mean duration of one launch of the main forward kernel (the
                             fused or matrix-core kernel that squares and integrates; front passes,
                             reduction and inverse excluded), over up to 16 launches per call */
} omni_stage;

/* Measurement support, no passage of the paper.
 * Durations in milliseconds of `stage` over the most recent correlate calls
 * (oldest first; at most 256 calls are remembered; for a batch plan the
 * stage spans all arrays).  Waits for the recorded events.  Writes at most
 * `max` values to ms and the count to *n.  OMNI_E_STATE without
 * OMNI_PLAN_TIMING, and for stages 0-2 and 4 of an OMNI_PLAN_GRAPH plan (its
 * arrays' stages overlap; only OMNI_STAGE_CALL is recorded).  Stage 4 keeps the
 * 32 most recent calls. */
int omni_stage_times(omni_plan_t plan, int32_t stage, int32_t max, float* ms, int32_t* n);

/* ---- F-engine ahead of the correlator ------------------------------------
 *
 * Appendix A, steps 2-3: each antenna's data are Fourier transformed in the
 * time domain (and calibrated), then arranged per frequency bin as the
 * hypercube the correlator takes.  Reading: raw real samples, one int8 per
 * antenna and instant, antenna-major; blocks of 2F consecutive samples, one
 * DFT per block, no window, bins k = 0 .. F-1 (the Nyquist bin dropped):
 *   X[n][t][k] = sum_{j < 2F} raw[n][2F t + j] exp(-2 pi i j k / 2F);
 * calibration and requantisation scale in one complex gain per antenna and
 * channel, Y = gains[n][k] X[n][t][k]; real and imaginary parts rounded to
 * the nearest integer (ties to even) and clipped to [-7, 7] (ci4) or
 * [-127, 127] (ci8); written in the correlator's sample layout [t][k][n]
 * (the corner turn).  The transform runs on the int8 matrix cores: the
 * samples times a three-part int8 split of the DFT matrix (each coefficient
 * within 6.1e-8), summed exactly in int32, combined and scaled in float32.
 * A code can differ from the exact value's by one only where the exact value
 * lies within that error (far below 1e-5 of sum_j |raw| |gain|) of a
 * rounding boundary.
 *   raw   : device int8 [N][2 F T], 16-byte aligned.
 *   N, T  : antennas (>= 1) and blocks (time samples of the output, >= 0).
 *   F     : channels, 16, 32 or 64.
 *   gains : device complex64 [N][F].
 *   dtype : OMNI_CI4 (volt: uint8 [T][F][N]) or OMNI_CI8 (volt: int8 [T][F][N][2]).
 *   volt  : device output, written.
 * Asynchronous on `stream`.  Errors: OMNI_E_INVAL (NULL, alignment, dtype,
 * N or T), OMNI_E_SHAPE (F, sizes), OMNI_E_HIP. */
int omni_fengine(const void* raw, int64_t N, int64_t T, int32_t F, const void* gains, int32_t dtype, void* volt,
                 void* stream);

/* ---- Hybrid tiles ---------------------------------------------------------
 *
 * Sec. III (the hybrid-tile paragraph): the array is P rectangular tiles of
 * n_x x n_y antennas, translated relative to one another by arbitrary
 * amounts.  Inside a tile the FFT method applies; the tiles' transforms
 * (synthesized beams) are correlated between tiles by brute force.  The call
 * computes, for every ordered pair of tiles (p, q) and index difference Delta
 * inside the tile grid,
 *   C_pq[Delta] = sum_t sum_{j, j-Delta in the tile} x_p[t][j] conj(x_q[t][j - Delta])
 * (C_pp is tile p's own visibility hypercube of Sec. II.D, Eq. ProofEq2), as:
 * zero-padded 2-D transform of every tile and sample (m = 2n per axis), the
 * cross-power sums S_pq[kappa] = sum_t Y_p conj(Y_q) per Fourier cell (float32
 * over a chunk of samples, then float64), one inverse transform per pair.
 * Physical baseline of cell (p, q, Delta): o_p - o_q + A Delta. */
typedef struct omni_hybrid_s* omni_hybrid_t;

/* Plan P tiles (2, 4, 8, 16 or 32) of n_x x n_y antennas (each side 1, 2, 4,
 * 8, 16 or 32), nchan channels, samples in format dtype (omni_dtype).
 *   offsets : [P][2] float64 tile offsets o_p, or NULL (metadata only).
 *   A       : [2][2] float64 row-major lattice matrix of a tile (columns =
 *             lattice vectors), or NULL (metadata only).
 * Allocates on the current device (gfx950).  Errors: OMNI_E_INVAL,
 * OMNI_E_SHAPE, OMNI_E_NODEV, OMNI_E_NOMEM, OMNI_E_HIP. */
int omni_hybrid_plan(omni_hybrid_t* out, int32_t P, int32_t nx, int32_t ny, int32_t nchan, int32_t dtype,
                     const double* offsets, const double* A);

/* Correlate T samples (T >= 0).
 *   volt : device [T][F][P n_x n_y] samples, tile-major (antenna p n_x n_y +
 *          i_x n_y + i_y), in the plan's format; may be NULL iff T == 0.
 *   vis  : device complex64 [F][P][P][2 n_x - 1][2 n_y - 1] (written; may be
 *          NULL with OMNI_NO_FINALIZE).
 *   flags: OMNI_NO_RESET (add to the running sums), OMNI_NO_FINALIZE.
 * Asynchronous on `stream`.  Errors: OMNI_E_INVAL, OMNI_E_STATE (other
 * device), OMNI_E_HIP. */
int omni_hybrid_correlate(omni_hybrid_t h, const void* volt, int64_t T, void* vis, void* stream, uint32_t flags);

/* uv[p][q][Delta_x][Delta_y][2] = o_p - o_q + A (Delta_x, Delta_y) (host
 * memory, written).  Errors: OMNI_E_INVAL, OMNI_E_STATE (no offsets or A). */
int omni_hybrid_baselines(omni_hybrid_t h, double* uv);

/* Release a hybrid plan (waits for the device first).  NULL is a no-op. */
int omni_hybrid_destroy(omni_hybrid_t h);

/* ---- Physical-baseline fold and baseline distributions -------------------
 *
 * Sec. II.D: hypercube cell Delta holds every antenna pair whose index tuples
 * differ by Delta, at physical separation b(Delta) = sum_k Delta_k a_k
 * (Eq. GridEq applied to an index difference).  Where several cells share one
 * separation (the 3-level layout of Fig. 1), the physical correlation at b is
 * their sum: the fold.  Sec. III draws each layout's two-dimensional baseline
 * distribution d (the layout map correlated with its parity reversal, which is
 * the fold of the visibilities of an all-ones input at one time sample) with
 * the origin zeroed on an asinh(4 d / d_max) intensity scale, bins it radially
 * and, for comparisons, smooths the radial distribution with a sliding boxcar.
 *
 * Pixels: cell Delta goes to pixel (rint(b_x / du), rint(b_y / dv)) relative to
 * the image centre, rint rounding half to even (the exact fold for integer
 * lattice vectors and du = dv = 1; nearest-pixel gridding otherwise).  The
 * image is [ny][nx], row = y, ny = 2 cy + 1, nx = 2 cx + 1, the zero baseline
 * at (cy, cx), cx = rint(X / du) with X = sum over lattice vectors of
 * |a_x| (n - 1) (the largest |b_x|), cy likewise.  Radial bin of pixel
 * (ix, iy) (offsets from the centre): floor(sqrt((ix du)^2 + (iy dv)^2) *
 * radius_scale / dr).  Pixel and bin follow from correctly rounded float64
 * operations in that order. */
typedef struct omni_fold_s* omni_fold_t;

typedef struct {
  double du, dv;        /* pixel size along x and y, in the units of A (> 0)               */
  double dr;            /* radial bin width, after radius_scale (> 0)                       */
  double radius_scale;  /* factor on |b| before radial binning (> 0; 1: none).  Sec. III's
                           comparison rescales every layout to the same largest baseline.    */
  int32_t boxcar;       /* odd width, in radial bins, of the centred sliding mean (1: none)  */
  int32_t zero_origin;  /* nonzero: omni_fold writes 0 to the zero-baseline pixel (Sec. III) */
} omni_fold_opts;

/* Plan the fold of array `array` of `plan` (which must carry lattice
 * matrices): computes every cell's pixel and every pixel's radial bin on the
 * device and keeps them grouped (cells sorted by pixel, pixels by bin), so
 * that each fold call is a gather with a fixed summation order.  opts may be
 * NULL (du = dv = dr = radius_scale = 1, no boxcar, origin kept).  Allocates
 * about 8 bytes per cell and per pixel on the plan's device (which must be
 * current) and synchronises it.  Errors: OMNI_E_INVAL (NULL, bad options,
 * array out of range), OMNI_E_STATE (host-only plan, no A, other device),
 * OMNI_E_SHAPE (image of 2^31 pixels or more), OMNI_E_NOMEM, OMNI_E_HIP. */
int omni_fold_plan(omni_fold_t* out, omni_plan_t plan, int32_t array, const omni_fold_opts* opts);

/* Image extent [ny][nx] and number of radial bins (host outputs). */
int omni_fold_shape(omni_fold_t fold, int64_t* ny, int64_t* nx, int64_t* nbins);

/* Fold visibilities: image[f][p] = sum of vis[f][cell] over the cells of
 * pixel p, in float64 (ascending cell order), f < nchan.
 *   vis   : device complex64 [nchan][prod(2 n_k - 1)] in the layout omni_correlate writes.
 *   image : device complex128 [nchan][ny][nx], written.
 *   nchan : 1 .. F of the array.
 * Asynchronous on `stream`.  Errors: OMNI_E_INVAL, OMNI_E_SHAPE (nchan),
 * OMNI_E_STATE (other device), OMNI_E_HIP. */
int omni_fold(omni_fold_t fold, const void* vis, int32_t nchan, void* image, void* stream);

/* Baseline-distribution products of Sec. III from the real part d of a
 * folded image (device complex128 [nchan][ny][nx], e.g. omni_fold's output for
 * an all-ones input, made with zero_origin):
 *   map    : device float64 [nchan][ny][nx] = asinh(4 d / d_max), d_max the
 *            channel's largest pixel (1 if that is not positive); may be NULL.
 *   hist   : device float64 [nchan][nbins], the sum of d over each radial bin;
 *            may be NULL.
 *   smooth : device float64 [nchan][nbins], the centred boxcar mean of hist
 *            over `boxcar` bins, bins beyond either end counting as zero; may be
 *            NULL (needs hist).
 * Asynchronous on `stream`; deterministic.  Errors: OMNI_E_INVAL (NULL image,
 * smooth without hist), OMNI_E_SHAPE (nchan), OMNI_E_STATE, OMNI_E_HIP. */
int omni_baseline_profile(omni_fold_t fold, const void* image, int32_t nchan, void* map, void* hist, void* smooth,
                          void* stream);

/* Release a fold (waits for the device first).  NULL is a no-op. */
int omni_fold_destroy(omni_fold_t fold);

/* Release the plan and everything it owns on the device (waits for the
 * device first).  NULL is a no-op.  Always returns OMNI_OK. */
int omni_destroy(omni_plan_t plan);

/* Static text for a status code (never NULL; "unknown status" otherwise). */
const char* omni_strerror(int code);

/* Detail of the last failure on the calling thread ("" if none); the text is
 * owned by the library and valid until the thread's next failing call. */
const char* omni_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* OMNISCOPE_H */
