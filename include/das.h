/*
 * das.h -- C ABI of the MI355X (gfx950) 3D delay-and-sum library.
 *
 * The operator (paper, Sec. 2):
 *   Eq. (1)  tau_qmn = tau_tx_qn + |p_n - r_m| / c0, with the transmit term of
 *            the footnote to Eq. (1) (plane wave, diverging wave, or none);
 *   weight   w_qmn = w_tx_qn * w_rx_mn (paragraph after Eq. (1));
 *   Eq. (2)  x_bn = sum_q sum_m w_qmn y_bqm[tau_qmn], linear interpolation
 *            between samples k = floor(f) and k+1 (sentence after Eq. (2)),
 *   with channel data batched as y[B][Q][M][K] (Sec. 2, last paragraphs).
 * The readings this library takes where the paper is silent:
 *   - fractional sample index f = ((D_tx + D_rx)/c - t0) * fs, with
 *     D_rx = |p - r_m| and D_tx = u.p - L (plane wave along unit u),
 *     |p - v| - L (diverging wave from virtual source v) or -L (none);
 *     sample k (0-based) is taken at time t0 + k/fs;
 *   - taps outside [0, K) read zero;
 *   - receive weight: uniform, or Hann with f-number F:
 *     with d = p - r_m, z = d.n_m, rho = |d - z n_m|, a = z/(2F):
 *     w_rx = (1 + cos(pi rho/a))/2 if z > 0 and rho < a, else 0;
 *   - voxel n = ix + Nx*(iy + Ny*iz) at origin + (ix, iy, iz) * spacing.
 *
 * Conventions for every entry point:
 *   - Every call returns das_status (DAS_OK = 0).  No exception crosses the
 *     ABI.  das_last_error() gives a thread-local message for the last failure
 *     of the calling thread.
 *   - Arguments are validated on the host before any HIP call; an invalid
 *     argument returns DAS_ERR_INVALID_ARG and touches no device state.
 *   - Large buffers (y, ws, x, gx, gy, w_tx, dLdc, f_out) are caller-owned,
 *     contiguous device memory of the stated layout.  The plan owns only its
 *     small geometry buffers (allocated by das_plan_create, freed by
 *     das_plan_destroy).
 *   - `stream` is a hipStream_t (NULL = the default stream).  Device work is
 *     enqueued asynchronously on it; no call synchronizes implicitly, except
 *     das_plan_create / das_plan_destroy / das_autotune which may.
 *   - Non-finite inputs propagate unchecked.
 *   - A plan is not safe to mutate from several threads; enqueuing work from
 *     one thread per stream on a plan that is not being mutated is safe.
 *     MFMA forwards led by one plan (das_forward and das_forward_batched)
 *     take the plan's 64 sets of work counters in turn: at most 64 of them
 *     may execute at the same time on different streams.
 */
#ifndef DAS_MI355X_H
#define DAS_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DAS_OK = 0,
  DAS_ERR_INVALID_ARG = -1,   /* bad pointer, size, enum, or geometry */
  DAS_ERR_UNSUPPORTED = -2,   /* valid, but this algorithm cannot run it */
  DAS_ERR_HIP = -3,           /* a HIP runtime call failed (see das_last_error) */
  DAS_ERR_OOM = -4            /* device allocation failed */
} das_status;

typedef enum { DAS_TX_NONE = 0, DAS_TX_PLANE = 1, DAS_TX_DIVERGING = 2 } das_tx_kind;
/* Workspace storage of the channel samples.  F16 and BF16 are the reduced
 * precision of Sec. 3.3 (round to nearest even).  FP8_E4M3 is the lower
 * precision the paper names as future work (Sec. 5): the OCP E4M3 8-bit format
 * (4 exponent bits, bias 7, 3 fraction bits, largest finite 448), round to
 * nearest even, with one power-of-two scale per batch item: an item whose
 * largest magnitude is A = f 2^x (f in [0.5, 1)) is stored as y 2^(8-x), so
 * that its samples span [-256, 256) and stay far from saturation; the forward
 * removes the scale exactly.  An item with A = 0 or a non-finite sample is
 * stored unscaled; NaN and +-inf samples are stored as NaN, finite magnitudes
 * above 448 saturate.  FP8 runs in the windowed and MFMA algorithms (the plain
 * one reads f32 and ignores the storage type, as for F16 and BF16). */
typedef enum {
  DAS_STORE_F32 = 0,
  DAS_STORE_F16 = 1,
  DAS_STORE_BF16 = 2,
  DAS_STORE_FP8_E4M3 = 3
} das_storage;
typedef enum { DAS_APOD_UNIFORM = 0, DAS_APOD_HANN_FNUM = 1 } das_apod;
typedef enum {
  DAS_ALGO_AUTO = 0,    /* tuned / heuristic choice among the three below */
  DAS_ALGO_PLAIN = 1,   /* one voxel per lane, direct gathers from y[B][Q][M][K] f32 */
  DAS_ALGO_TILED = 2,   /* voxel tiles, LDS sample windows, aperture culling */
  DAS_ALGO_MFMA = 3     /* locality form on matrix cores (f16, bf16 or fp8 storage) */
} das_algo;

/* One transmit (observation) q: footnote to Eq. (1). */
typedef struct {
  int32_t kind;          /* das_tx_kind */
  double vec[3];         /* PLANE: unit propagation direction u (into the medium);
                            DIVERGING: virtual source position v (m); NONE: unused */
  double path_offset;    /* L_q (m), subtracted from the transmit path */
} das_tx;

/* Voxel grid (Sec. 2): p = origin + (ix, iy, iz) * spacing. */
typedef struct {
  double origin[3];      /* m */
  double spacing[3];     /* m, each > 0 */
  int32_t dims[3];       /* Nx, Ny, Nz, each >= 1 */
} das_grid;

typedef struct {
  int32_t num_elements;        /* M >= 1 */
  const double* element_pos;   /* host [M][3] (m); copied at plan creation */
  const double* element_normal;/* host [M][3] or NULL (= +z); normalized on copy */
  int32_t num_tx;              /* Q >= 1 */
  const das_tx* tx;            /* host [Q]; copied */
  das_grid grid;
  int32_t num_samples;         /* K >= 2 */
  int32_t max_batch;           /* B upper bound >= 1 */
  double sound_speed;          /* c0 (m/s) > 0 */
  double fs;                   /* sampling rate (Hz) > 0 */
  double t0;                   /* time of sample 0 (s) */
  int32_t apod;                /* das_apod */
  double f_number;             /* F > 0 (HANN_FNUM only) */
  int32_t storage;             /* das_storage of the prepared workspace */
  int32_t algo;                /* das_algo */
} das_config;

typedef struct das_plan_s* das_plan;

/* Create a plan on HIP device `hip_device`: validate cfg, copy the geometry
 * (FP64) to the device.  *out is NULL on failure. */
das_status das_plan_create(das_plan* out, const das_config* cfg, int hip_device);
/* Free the plan's device buffers (synchronizes the device).  NULL is a no-op. */
das_status das_plan_destroy(das_plan p);

/* Replace c0 (m/s, > 0); read by the next enqueued call. */
das_status das_plan_set_sound_speed(das_plan p, double c);
/* Optional transmit weights: the factor w_tx of the weight w_qmn = w_tx_qn
 * w_rx_mn (paragraph after Eq. (1); the transmit wavefield magnitude that
 * Sec. 3.1 precomputes per voxel).  w_tx[Q][N] f32, device, caller-owned, must
 * outlive the calls that use it; NULL restores w_tx = 1.  Transmits whose
 * weight is zero over a whole voxel tile are skipped there (the sparse
 * observation lists of Sec. 5); the result does not change. */
das_status das_plan_set_tx_weights(das_plan p, const float* w_tx);
/* Complex baseband (IQ) mode, the paper's data model (Sec. 2), with the phase
 * term that Eq. (2) omits for demodulated data: with enable != 0 the batch
 * items come in pairs (2b, 2b+1) = (I, Q) of one complex record, demodulated
 * at the carrier fc (Hz, finite, >= 0): y_iq(t_k) = y_analytic(t_k)
 * exp(-i 2 pi fc t_k), t_k = t0 + k/fs.  das_forward then writes
 *   x[2b] + i x[2b+1] = sum_q sum_m w ((1-a) s(k) + a s(k+1)) exp(i 2 pi fc tau),
 * tau = (D_tx + D_rx)/c, from the interpolated complex samples s.  Runs in the
 * windowed algorithm with f32 storage, or in the MFMA algorithm with f16 or
 * FP8 storage (Alg. 3's complex W: the cosine and sine parts of the weights
 * contracted with the same sample fragments; COLUMN, SLAB or PERSISTENT
 * launch, the FP8-operand forms taking the f16-operand COLUMN or SLAB
 * launch), with an even batch (DAS_ERR_UNSUPPORTED / DAS_ERR_INVALID_ARG
 * otherwise).  das_adjoint and das_grad_sound_speed of an IQ plan are the
 * transpose and the sound-speed derivative of that map (even batch);
 * das_forward_batched takes IQ plans in the MFMA algorithm.
 * enable = 0 restores real data. */
das_status das_plan_set_iq(das_plan p, int32_t enable, double fc);
/* Launch form of the MFMA algorithm (Sec. 3.4, Alg. 3); Sec. 3.2 says tile
 * sizes should be picked by profiling, and das_autotune does so for MFMA
 * plans.  DAS_MFMA_COLUMN: one launch, each wavefront a 4 x 4 x 4 voxel column
 * (four 4 x 4 MFMA row groups stacked in depth).  DAS_MFMA_SLAB: one launch,
 * each wavefront an 8 x 8 x 1 slab (four groups side by side at one depth,
 * whose taps share more sample chunks).  DAS_MFMA_PERSISTENT: the persistent
 * dynamic-scheduling kernel of das_forward_batched with one plan (4 x 4 x 4
 * columns).  DAS_MFMA_COLUMN_FP8 / DAS_MFMA_SLAB_FP8 (FP8 storage only,
 * DAS_ERR_UNSUPPORTED otherwise): the COLUMN / SLAB launches on the FP8
 * matrix instructions, contracting the stored E4M3 codes with E4M3
 * interpolation weights (each weight, scaled by 2^7, split into two E4M3
 * parts: a relative weight error near 2^-8 instead of the f16 weights'
 * 2^-11).  DAS_MFMA_AUTO (default): persistent where it gives the plan the
 * same batch tiles per wavefront as the plain launch, else COLUMN.  All forms
 * read the same workspace and agree up to FP32 summation order and the
 * rounding of the interpolation weights (they form delays relative to
 * different box centres).  FP8 storage is Sec. 5's lower-precision future
 * direction. */
typedef enum {
  DAS_MFMA_AUTO = 0,
  DAS_MFMA_COLUMN = 1,
  DAS_MFMA_SLAB = 2,
  DAS_MFMA_PERSISTENT = 3,
  DAS_MFMA_COLUMN_FP8 = 4,
  DAS_MFMA_SLAB_FP8 = 5
} das_mfma_form;
das_status das_plan_set_mfma_form(das_plan p, int32_t form);
das_status das_plan_get_mfma_form(das_plan p, int32_t* form);
/* Interpolation of the channel samples at the fractional index f of Eq. (1):
 * DAS_INTERP_LINEAR (0, the default) is Eq. (2); DAS_INTERP_CUBIC (1) is the
 * four-point Lagrange interpolant through samples k-1 .. k+2 (k = floor(f)),
 * one of the alternative schemes the paper allows after Eq. (2), with taps
 * outside [0, K) reading zero as for linear interpolation.  Cubic runs in the
 * windowed algorithm with f32 storage on real data: das_plan_set_interp
 * returns DAS_ERR_UNSUPPORTED for a plan whose algorithm for some batch is
 * not the windowed one, and das_forward (IQ plans), das_adjoint,
 * das_grad_sound_speed and das_forward_batched refuse cubic plans. */
typedef enum { DAS_INTERP_LINEAR = 0, DAS_INTERP_CUBIC = 1 } das_interp;
das_status das_plan_set_interp(das_plan p, int32_t interp);
/* Force an algorithm (das_algo) for subsequent calls; AUTO restores the
 * plan's choice.  AUTO depends only on the storage type, the batch size and
 * what was fixed at plan creation: MFMA for 16- or 8-bit storage with batch >= 16,
 * else windowed if any tile shape fits the geometry, else plain.  MFMA with
 * f32 storage returns DAS_ERR_UNSUPPORTED.  The algorithm decides the
 * workspace layout: a workspace must be prepared under the algorithm (and
 * batch_total) that reads it. */
das_status das_plan_set_algo(das_plan p, int32_t algo);
/* The algorithm das_forward would use for `batch` items. */
das_status das_plan_get_algo(das_plan p, int32_t batch, int32_t* algo);

/* Size in bytes of the prepared workspace for `batch` items. */
das_status das_workspace_bytes(das_plan p, int32_t batch, size_t* bytes);

/* Reorder + convert (Sec. 3.2 batch-inner layout, fused with the Sec. 3.3
 * precision conversion).  y: device [nb][Q][M][K] f32, items b0 .. b0+nb-1 of
 * a batch of batch_total.  ws: device workspace of das_workspace_bytes(
 * batch_total) bytes.  Layout written:
 *   PLAIN:        [batch_total][Q][M][K] f32 (a copy; y itself may be passed
 *                 as ws to das_forward instead)
 *   TILED:        [Q][M][K][batch_total] in the plan's storage type, rounded
 *                 to nearest even;
 *   MFMA:         [Bp/TW][Q][M][Kc][TW][8] in f16/bf16/fp8 (rounded to
 *                 nearest even): 8-sample chunks, chunk kc holding samples
 *                 8(kc-1) .. 8kc-1 (zero outside [0, K)), Kc = ceil(K/8) + 2;
 *                 batch tiles of TW = 16, 32 or 64 items for batch_total
 *                 <= 16, <= 32 or more, Bp = batch_total rounded up to TW
 *                 (Sec. 3.4 locality form).
 * FP8 workspaces end with a table of batch_total f32 values (the largest
 * magnitude of each item, which fixes its scale) at the first 256-byte
 * boundary after the samples; das_prepare first finds the largest magnitude of
 * items b0 .. b0+nb-1 (one extra read of their y), then converts. */
das_status das_prepare(das_plan p, const float* y, int32_t b0, int32_t nb, int32_t batch_total,
                       void* ws, void* stream);

/* Forward, Eq. (2).  ws: prepared workspace for `batch` items.
 * x: device [batch][N] f32, overwritten. */
das_status das_forward(das_plan p, const void* ws, int32_t batch, float* x, void* stream);

/* Adjoint: the exact transpose of the linear map y -> x of Eq. (2), with the
 * delays of Eq. (1) and linear interpolation (sentence after Eq. (2)):
 * gy[b][q][m][j] = sum_n w_qmn ((1-a)[j = k] + a [j = k+1]) gx[b][n].
 * gx: device [batch][N] f32; gy: device [batch][Q][M][K] f32, overwritten
 * (taps outside [0, K) are dropped, as they read zero in the forward map).
 * IQ plans (das_plan_set_iq; even batch): the transpose of the complex
 * baseband map, item pairs (2b, 2b+1) = (I, Q) on both sides:
 * gy[2b] + i gy[2b+1] at tap j = sum_n w_qmn ((1-a)[j = k] + a [j = k+1])
 * exp(-i 2 pi fc tau) (gx[2b][n] + i gx[2b+1][n]).
 * Summation order across voxel tiles is not fixed (FP32 rounding level). */
das_status das_adjoint(das_plan p, const float* gx, int32_t batch, float* gy, void* stream);

/* Sound-speed gradient: the derivative of Eq. (2) in c0 through the delays of
 * Eq. (1) (grid, t0 and weights do not depend on c0):
 * dL/dc = sum_{b,n} gx[b][n] dx[b][n]/dc, with dx/dc = sum_{q,m} w (s(k+1)-s(k)) df/dc,
 * df/dc = -fs (D_tx + D_rx)/c^2 (right-hand slope at integer f).
 * IQ plans (even batch; pairs (2b, 2b+1) = (I, Q) in y and gx): the phase
 * exp(i 2 pi fc tau) turns with c too, dx/dc = sum w exp(i 2 pi fc tau)
 * ((s(k+1)-s(k)) + i 2 pi (fc/fs) s_interp) df/dc, and
 * dL/dc = sum gx[2b] Re(dx/dc) + gx[2b+1] Im(dx/dc).
 * y: device [batch][Q][M][K] f32 (caller layout); gx: device [batch][N] f32;
 * dLdc: device scalar f32, overwritten. */
das_status das_grad_sound_speed(das_plan p, const float* y, const float* gx, int32_t batch,
                                float* dLdc, void* stream);

/* Several forward passes in one persistent launch: the batched problem of
 * Sec. 2 (many frames beamformed with shared geometry, Sec. 3.2) extended to
 * plans of different grids and arrays.  For
 * i < count, plan plans[i] beamforms its prepared workspace ws[i] (batch[i]
 * items) into x[i] ([batch[i]][N_i] f32).  The launch walks one work list of
 * (plan, voxel tile or column, batch group) items with a fixed grid of
 * resident workgroups.  Requirements: 1 <= count <= 16; all plans on one
 * device with the same storage type and the same algorithm for their batch,
 * windowed (each plan with its own tile shape) or MFMA (DAS_ERR_UNSUPPORTED
 * otherwise).  Complex baseband (IQ) plans: all plans of the launch or none
 * (DAS_ERR_UNSUPPORTED), MFMA algorithm with f16 or FP8 storage
 * (DAS_ERR_UNSUPPORTED otherwise), even batches (DAS_ERR_INVALID_ARG).
 * Results equal those of das_forward on each plan bit for bit (for IQ
 * plans: das_forward with the PERSISTENT form).
 * MFMA launches schedule their items dynamically through one of the 64
 * sets of work counters owned by plans[0] (the sets are taken in turn, so at
 * most 64 MFMA launches led by one plan may execute at the same time on
 * different streams).  A single-plan das_forward with the MFMA algorithm runs
 * through this persistent kernel too when that gives the plan the same batch
 * tiles per wavefront as the plain launch. */
das_status das_forward_batched(int32_t count, const das_plan* plans, const void* const* ws,
                               const int32_t* batch, float* const* x, void* stream);

/* Tile shapes picked by measurement, as Sec. 3.2 says they should be chosen
 * ("determined by profiling").  For a plan whose algorithm for `batch` items
 * is the windowed one, times the candidate tile shapes; for the MFMA
 * algorithm, times the launch forms COLUMN, SLAB and PERSISTENT (and for
 * FP8 storage COLUMN_FP8 and SLAB_FP8; das_mfma_form).  Runs on `stream` with
 * scratch buffers it allocates and frees (a zeroed workspace of `batch`
 * items), keeps the fastest for this plan and synchronizes the stream. */
das_status das_autotune(das_plan p, int32_t batch, void* stream);
/* Tile shape index the plan uses for TILED (see das_tile_shape).  set_tile
 * returns DAS_ERR_UNSUPPORTED, leaving the plan unchanged, for a shape whose
 * sample windows do not fit this geometry.  The workspace layout does not
 * depend on the tile shape. */
das_status das_plan_get_tile(das_plan p, int32_t* tile_index);
das_status das_plan_set_tile(das_plan p, int32_t tile_index);
/* Dimensions of candidate tile `tile_index` (0 .. das_num_tile_shapes()-1). */
int32_t das_num_tile_shapes(void);
das_status das_tile_shape(int32_t tile_index, int32_t dims[3]);

/* The fractional sample index of Eq. (1) (f = tau fs, with the readings
 * above) as the forward kernels form it (integer part
 * plus the FP32 tile-relative part, converted exactly to f64), for transmit q,
 * elements [m0, m1) and voxels [n0, n1).  f_out: device [m1-m0][n1-n0] f64.
 * Exposes the in-kernel delay formation to the delay-error test. */
das_status das_debug_delays(das_plan p, int32_t q, int32_t m0, int32_t m1, int32_t n0, int32_t n1,
                            double* f_out, void* stream);

/* Rank-truncation (SVD) clutter filter and power Doppler of an ensemble: the
 * rank-truncation primitive the paper names beside the beamformer for
 * clutter filtering in ultrafast pipelines (Sec. 1, Sec. 5).  x: device [T][N] f32, T frames of N voxels (for example the
 * output of das_forward for a batch of T frames), read as the Casorati matrix
 * S = x^T = U diag(sigma) V^T.  The filter keeps the singular components
 * k_lo .. k_hi-1 (0 <= k_lo < k_hi <= T; the k_lo largest are tissue
 * clutter, components from k_hi on are noise):
 *   xf = sum_{k_lo <= j < k_hi} sigma_j v_j-projection of each voxel series,
 *   power[n] = (1/T) sum_t xf[t][n]^2.
 * Outputs (device, caller-owned): sv[T] f32 singular values, descending;
 * power[N] f32; xf[T][N] f32 or NULL.  ws: device workspace of
 * das_clutter_workspace_bytes(T) bytes, caller-owned (not kept between
 * calls).  Requirements: 1 <= T <= 512, N >= 1, and the smaller of
 * (k_hi - k_lo) and T - (k_hi - k_lo) at most 64 (DAS_ERR_UNSUPPORTED
 * otherwise; DAS_ERR_INVALID_ARG for bad sizes or NULL pointers).
 * Method: Gram matrix x x^T on the matrix cores (FP32, chunks merged in
 * FP64); FP64 eigen-decomposition (Householder tridiagonalisation,
 * multisection for the eigenvalues, inverse iteration and
 * back-transformation for the eigenvectors of the projection basis: the kept
 * components or the removed ones, whichever are fewer); per-voxel
 * projection (power alone in one FP64 pass when xf is NULL and the basis
 * has at most 16 vectors).
 * Runs on the calling thread's current device. */
das_status das_clutter_workspace_bytes(int32_t T, size_t* bytes);
das_status das_clutter_filter(const float* x, int32_t T, int64_t N, int32_t k_lo, int32_t k_hi,
                              float* sv, float* power, float* xf, void* ws, void* stream);

/* das_clutter_filter for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same computation with its workspace in a buffer the
 * library holds, a static device array of 2.2 MiB per device that lives
 * until the process ends.  No allocation of any kind is made.  Arguments as
 * for das_clutter_filter without ws; T <= 256 (DAS_ERR_INVALID_ARG above).
 * Every call on a device shares that device's buffer: calls that overlap on
 * one device (different streams or threads) race and must be serialised by
 * the caller.  The buffer keeps the last call's contents; each call clears
 * what it needs at zero. */
das_status das_clutter_filter_noalloc(const float* x, int32_t T, int64_t N, int32_t k_lo,
                                      int32_t k_hi, float* sv, float* power, float* xf,
                                      void* stream);
const char* das_status_string(das_status st);
const char* das_last_error(void);
/* Library version string. */
const char* das_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DAS_MI355X_H */
