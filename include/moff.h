/* moff.h -- C ABI of the MI355X-native MOFF correlator hot path.
 *
 * The MOFF image (Section 4, Eq. m6) is
 *
 *     I'(theta) = < | F^T(theta, r) W^T(r, a) N~(a, a) E'(a) |^2 >_t
 *
 * computed for every frequency channel c and time sample t as
 *   1. noise weighting N~ (diagonal, folded into the kernels by the caller),
 *   2. gridding W^T: each antenna's channelised voltage E'_a is spread onto a regular n x n grid through its own
 *      K x K complex kernel (multiplied as given, no conjugation),
 *   3. the spatial transform F^T: an unnormalised 2-D DFT with the e^{+2 pi i} sign (the adjoint of the
 *      e^{-2 pi i u.theta} of the voltage model, Eq. Ea), evaluated as an FFT (Fig. 1 caption, rows d-e),
 *   4. squaring into polarisation products XX = |E_X|^2, YY = |E_Y|^2, XY = E_X conj(E_Y), summed over time
 *      (YX = conj(XY) pixel by pixel; Discussion: four polarisations).
 *
 * Geometry conventions (Section 4, MOFF properties 1-2: arbitrary antenna placement, free grid spacing; the
 * grid is tied to the ground, east = u = column i, north = v = row j):
 *   X_a = x_a f_c / c / cell + n_c / 2,  Y_a likewise from y_a;
 *   the footprint of antenna a covers columns floor(X_a) - K/2 + 1 ... floor(X_a) + K/2 (rows likewise) and must
 *   lie inside the grid (otherwise MOFF_E_INVALID);
 *   image pixel (q, p) <-> direction (m, l) = ((q - n/2), (p - n/2)) / (n cell).
 *
 * Memory and streams.  Every device buffer is caller-owned (the library never allocates device memory).  Every
 * call that takes a stream only enqueues work on it and returns without synchronising; a stream argument is a
 * hipStream_t passed as void* (NULL = the null stream).  Validation is done on the host before anything is
 * enqueued: on error nothing is enqueued and outputs are untouched.  Asynchronous device faults surface at the
 * caller's next synchronisation.  A plan is used by one host thread at a time; distinct plans may run
 * concurrently on distinct streams.  Results are deterministic for identical inputs.
 *
 * Layouts (all little-endian, densely packed):
 *   voltages    int8  [n_t][C][A][P][2] (re, im)            (volt_format MOFF_VOLT_INT8)
 *               float [n_t][C][A][P][2] (complex64)          (volt_format MOFF_VOLT_C64)
 *   kernels     float [C][A][P][K][K][2] (complex64), the weight N~ already folded in (diagonal kernels);
 *               float [C][A][2 (p, grid)][2 (q, voltage)][K][K][2] for Jones kernels
 *   grid/efield float [n_t][sum_c P n_c^2][2]: per sample, channel c's block starts at P * pix_off(c), pol p at
 *               + p n_c^2, row-major [j][i].  E-field images are in FFT order: index k <-> pixel (k + n/2) mod n.
 *   accumulator float (MOFF_ACC_FP32) or double pairs (sum, carry) (MOFF_ACC_FP64_COMP), R reals per pixel:
 *               R = 4 (XX, YY, Re XY, Im XY) for P = 2, R = 1 for P = 1.  Channel c starts at R * pix_off(c); its
 *               layout is internal (column-group tiles matching the column pass), so read it with
 *               moff_read_image.  Zero it before the first call (any fill kernel); calls add to it.
 *   image       float [sum_c M n_c^2][2] (complex64), M = 4 products XX, YY, XY, YX (M = 1 for P = 1), channel c at
 *               M * pix_off(c), product-major, pixels centred (row q = m, column p = l).
 *   pix_off(c) = sum_{c' < c} n_c'^2  (moff_chan_offset).
 */
#ifndef MOFF_H
#define MOFF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct moff_plan_s *moff_plan_t;

typedef enum {
  MOFF_OK = 0,
  MOFF_E_INVALID = 1,     /* bad argument: null pointer, odd K, footprint outside the grid, bad size */
  MOFF_E_BUDGET = 2,      /* workspace smaller than moff_workspace_size */
  MOFF_E_DEVICE = 3,      /* a HIP call or kernel launch failed */
  MOFF_E_UNSUPPORTED = 4, /* valid request the library does not implement (e.g. a grid size with a prime > 5) */
  MOFF_E_STATE = 5        /* call out of order: not bound, kernels not set */
} moff_status;

/* Arithmetic of gridding and the spatial transform.
 *   FP32: scatter gridding in LDS and radix-2/3/4/5/8/16 FFT stages on the vector units.
 *   SPLIT_FP16 / SPLIT_BF16 (256^2 grids, two pols): FP32 gridding, both FFT passes as radix-16 DFT-GEMMs on the
 *     matrix cores with split 16-bit products.
 *   GEMM_FP16: gridding and the row half of the transform together as one matrix-core GEMM over time samples,
 *     H[t][j][k] = sum over the antennas a whose footprint covers grid row j of E[t][a] Phi_a[k], with
 *     Phi_a[k] = w^(i0_a k) sum_x W_a[j - j0_a][x] w^(x k) (w = e^(2 pi i / n)): the int8 voltages are exact in FP16,
 *     Phi is formed in FP32 from the kernel and split into FP16 hi + lo terms (two products, FP32 accumulation);
 *     the column half and the products are the FP32 column pass.  Any supported grid size, diagonal kernels, int8
 *     voltages. */
typedef enum { MOFF_FFT_FP32 = 0, MOFF_FFT_SPLIT_FP16 = 1, MOFF_FFT_SPLIT_BF16 = 2, MOFF_FFT_GEMM_FP16 = 3 } moff_fft_mode;
typedef enum { MOFF_ACC_FP32 = 0, MOFF_ACC_FP64_COMP = 1 } moff_acc_mode;
typedef enum { MOFF_VOLT_INT8 = 0, MOFF_VOLT_C64 = 1 } moff_volt_format;
/* Diagonal kernels: the X grid receives only X voltages (through K_{a,X}) and the Y grid only Y voltages.
 * Jones kernels (full polarimetry): grid p receives both pols of every antenna, G_p = sum_q K_{a,pq} E_{a,q}. */
typedef enum { MOFF_KERNEL_DIAG = 0, MOFF_KERNEL_JONES = 1 } moff_kernel_mode;
typedef enum { MOFF_PIPELINE_TWO_PASS = 0, MOFF_PIPELINE_STREAM = 1 } moff_pipeline;

typedef struct {
  int32_t n_ant;            /* A >= 1 */
  int32_t n_pol;            /* P = 1 or 2 */
  int32_t n_chan;           /* C >= 1 */
  int32_t ksize;            /* K, even, 2..8 */
  const double *ant_xy_m;   /* host [A][2] (east, north) metres; copied by moff_plan */
  const double *freq_hz;    /* host [C] channel centre frequencies; copied */
  const int32_t *grid_n;    /* host [C] grid sizes, or NULL / 0 entries = smallest supported size that fits */
  double cell_lambda;       /* grid cell size in wavelengths (> 0) */
  int32_t fft_mode;         /* moff_fft_mode */
  int32_t acc_mode;         /* moff_acc_mode */
  int32_t time_block;       /* samples per fused launch block (0 = library default, 256) */
  int32_t volt_format;      /* moff_volt_format */
  int32_t chans_per_block;  /* channels per fused launch block (0 = library default, 32) */
  int32_t time_group;       /* samples per row-pass workgroup (0 = library default, 32) */
  int32_t kernel_mode;      /* moff_kernel_mode; Jones needs n_pol = 2 and the FP32 transform */
  int32_t n_tap;            /* E-field image taps per channel, 0..8 (moff_set_taps) */
} moff_plan_desc;

/* Host only.  Validates the description, computes every antenna's footprint per channel, bins antennas into
 * grid row bands (an antenna whose footprint straddles a band boundary is listed in both bands: the paper's
 * module-boundary copies, Section 5) and lays out the workspace.  *out receives a new plan.  Channels are
 * binned on host threads (environment MOFF_PLAN_THREADS, default the host's threads up to 16); the plan is the
 * same for every thread count. */
moff_status moff_plan(const moff_plan_desc *desc, moff_plan_t *out);

/* Bytes of device workspace the plan needs (>= 256-byte aligned sections). */
moff_status moff_workspace_size(moff_plan_t plan, size_t *bytes);

/* Bytes of the accumulator buffer (depends on acc_mode) and of the image buffer, for all channels. */
moff_status moff_acc_size(moff_plan_t plan, size_t *bytes);
moff_status moff_image_size(moff_plan_t plan, size_t *bytes);

/* Grid size chosen for channel chan, and pix_off(chan) = sum of n_c^2 over earlier channels. */
moff_status moff_grid_n(moff_plan_t plan, int32_t chan, int32_t *n);
moff_status moff_chan_offset(moff_plan_t plan, int32_t chan, int64_t *pix_off);

/* Binds device workspace d_ws (>= moff_workspace_size bytes, 256-byte aligned) to the plan: uploads the band
 * lists and tap tables and generates the FFT twiddle tables on the device in FP64 (rounded once to FP32).
 * The workspace must stay allocated while the plan is used. */
moff_status moff_bind(moff_plan_t plan, void *d_ws, size_t bytes, void *stream);

/* Sets the per-antenna kernels (layout above, device memory).  Re-orders them into the library's tap-group
 * order inside the workspace; d_kern may be freed once the stream has passed this call.  Step 1-2 of Eq. m6:
 * the caller folds N~ into the kernels. */
moff_status moff_set_kernels(moff_plan_t plan, const void *d_kern, void *stream);

/* Phase-centre tracking (Section 4: the phase centre is followed by delaying each antenna's signal before
 * gridding): as moff_set_kernels, with every antenna's channelised voltage multiplied by d_phase[c][a][p]
 * (complex64, device) before gridding.  The product is folded into the packed kernels (W (phi E) = (W phi) E),
 * so the hot path does no extra work; call it again with new phases between time blocks to track a moving phase
 * centre.  d_phase == NULL is moff_set_kernels. */
moff_status moff_set_kernels_phased(moff_plan_t plan, const void *d_kern, const void *d_phase, void *stream);

/* Staged path, step 2 (gridding): d_volt [n_t] samples -> d_grid [n_t] grids (layout above, fully written). */
moff_status moff_grid(moff_plan_t plan, const void *d_volt, int64_t n_t, void *d_grid, void *stream);

/* Staged path, step 3: in-place 2-D FFT of n_t grids into E-field images (FFT pixel order).  Every row and column
 * of every channel's grid is transformed, so the grids may hold data anywhere (not only on the footprint rows that
 * moff_grid writes). */
moff_status moff_fft(moff_plan_t plan, void *d_grid, int64_t n_t, void *stream);

/* Staged path, step 4: adds the polarisation products of n_t E-field images to the accumulator. */
moff_status moff_accumulate(moff_plan_t plan, const void *d_efield, int64_t n_t, void *d_acc, void *stream);

/* Fused path: steps 1-4 for n_t samples of all channels, added to the accumulator.  Uses only the workspace
 * as scratch (the row-transformed grids pass through it between the row and column passes). */
moff_status moff_correlate(moff_plan_t plan, const void *d_volt, int64_t n_t, void *d_acc, void *stream);

/* Read-out: accumulator -> centred complex64 image (layout above), expanding YX = conj(XY).  normalize != 0
 * divides by n_samples (the time average of Eq. m6); otherwise the sums are returned. */
moff_status moff_read_image(moff_plan_t plan, const void *d_acc, int64_t n_samples, int32_t normalize,
                            void *d_img, void *stream);

/* Test hooks.  moff_debug_unpack converts one sample's voltages ([C][A][P][2]) exactly to float [C][A][P][2].
 * moff_debug_tiles copies (host to host) the footprint origins int32 [C][A][2] (j0, i0), the band pointer array
 * int32 [n_band_total + 1] and the band antenna list int32 [n_entries]; any pointer may be NULL, and
 * moff_debug_tile_counts gives the sizes and the band height per channel (int32 [C], may be NULL). */
moff_status moff_debug_unpack(moff_plan_t plan, const void *d_volt, float *d_out, void *stream);
moff_status moff_debug_tile_counts(moff_plan_t plan, int64_t *n_band_total, int64_t *n_entries,
                                   int32_t *band_rows);
moff_status moff_debug_tiles(moff_plan_t plan, int32_t *h_origin, int32_t *h_band_ptr, int32_t *h_band_ant);

/* Launch shape of the fused path: samples per launch block, channels per launch block (consecutive channels
 * with one grid size) and samples per row-pass workgroup.  moff_workspace_size_for gives the workspace a shape
 * needs; moff_set_launch_shape applies one to a bound plan (MOFF_E_BUDGET if the bound workspace is too small;
 * nothing changes then).  The shape changes speed only, never results beyond FP32 summation order. */
moff_status moff_workspace_size_for(moff_plan_t plan, int32_t time_block, int32_t chans_per_block, size_t *bytes);
moff_status moff_set_launch_shape(moff_plan_t plan, int32_t time_block, int32_t chans_per_block, int32_t time_group);
moff_status moff_get_launch_shape(moff_plan_t plan, int32_t *time_block, int32_t *chans_per_block,
                                  int32_t *time_group);

/* Autotuner.  Times moff_correlate of n_t samples of d_volt for candidate launch shapes that fit the bound
 * workspace: the plan's current shape first, then time blocks of 8-256 samples x 4-128 channels x row groups of
 * 2-64 samples (d_acc is used as scratch and left holding garbage); keeps the fastest and returns it with its
 * time per call in ms, so the result is never slower than the current shape on this input.  Blocks the calling
 * host thread (it synchronises the stream). */
moff_status moff_autotune(moff_plan_t plan, const void *d_volt, int64_t n_t, void *d_acc, void *stream,
                          int32_t *time_block, int32_t *chans_per_block, int32_t *time_group, double *best_ms);

/* Autotuner with a persisted per-shape cache.  The key (moff_autotune_key) names every input of the launch-shape
 * choice: compute units of the bound device, antennas, pols, kernel size, channels, the distinct grid sizes with
 * their channel counts, the touched grid rows, the fft / accumulator / voltage / kernel modes, the pipeline and the
 * taps.  cache_path is a text file of lines "key<TAB>time_block chans_per_block time_group ms" (created if
 * missing).  If it holds the key (the last such line wins) and that shape fits the bound workspace, the shape is
 * applied without timing anything and *hit = 1; otherwise moff_autotune runs, its result is appended to the file
 * and *hit = 0.  MOFF_E_INVALID if the file cannot be read or written (a malformed line for this key is ignored). */
moff_status moff_autotune_cached(moff_plan_t plan, const char *cache_path, const void *d_volt, int64_t n_t,
                                 void *d_acc, void *stream, int32_t *time_block, int32_t *chans_per_block,
                                 int32_t *time_group, double *best_ms, int32_t *hit);
/* The cache key of a plan, NUL-terminated into buf (MOFF_E_INVALID if bufsize is too small).  The compute-unit
 * count is 0 until the plan is bound; host only. */
moff_status moff_autotune_key(moff_plan_t plan, char *buf, size_t bufsize);

/* Fused path replayed from a HIP graph.  The first call for a given (d_volt, n_t, d_acc) records every launch
 * moff_correlate would make (on an internal capture stream) into a graph and instantiates it; every call then
 * launches that graph on the caller's stream, one host call per integration.  Changing the launch shape or
 * rebinding drops the cached graphs.  The buffers' contents may change between calls; their addresses may not. */
moff_status moff_correlate_graph(moff_plan_t plan, const void *d_volt, int64_t n_t, void *d_acc, void *stream);

/* For callers that cannot allocate device memory when they correlate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): moff_correlate with the row-transformed grids passing through a fixed
 * buffer that the library owns, MOFF_NOALLOC_EXCHANGE_BYTES on each GPU it runs on (a device array held from the
 * first call on that GPU until the process ends), instead of the workspace's exchange region.  It calls no
 * hipMalloc or hipFree and allocates nothing else.  Launch blocks are cut (channels, then samples) so that one
 * block's exchange fits the buffer, which makes it slower than moff_correlate; results equal moff_correlate's up
 * to FP32 summation order (the accumulator is updated per shorter block).  Two-pass form whatever the pipeline
 * setting.  MOFF_E_UNSUPPORTED if one channel-sample of the plan needs more than the buffer (P n^2 x 8 bytes; every
 * supported grid size fits).  Every call on one GPU shares the buffer, which keeps the last call's contents (each
 * call writes what it reads): calls that overlap on one GPU (concurrent streams, other plans, other host
 * threads) race. */
#define MOFF_NOALLOC_EXCHANGE_BYTES (64u << 20)
moff_status moff_correlate_noalloc(moff_plan_t plan, const void *d_volt, int64_t n_t, void *d_acc, void *stream);

/* How the fused path (moff_correlate, moff_correlate_graph) moves the row-transformed grids to the column pass
 * -- the all-to-all of a 2-D FFT too large for one compute unit, which the paper's modular design does between
 * spatial modules (Section 5).  MOFF_PIPELINE_TWO_PASS (default): a row-pass kernel writes them for a launch
 * block of channels x samples and a column-pass kernel reads them back.  MOFF_PIPELINE_STREAM: one persistent
 * launch per run of channels with one grid size; in each team of workgroups some own the column groups of a
 * channel and keep transforming and accumulating while the others grid and row-transform the next samples into
 * a small ring (device-coherent accesses, held by the memory-side cache), with counters ordering the two.
 * Results equal the two-pass form's up to FP32 rounding (same sums, same accumulation blocks).  The streaming
 * launch needs every workgroup resident: do not run other kernels concurrently on the device while it runs.
 * Its waits are bounded (spin limit, MOFF_SPIN_LIMIT); a wait that times out ends the launch early and leaves a
 * code that moff_stream_status reads (0 = fine; 1 = timed out, the accumulator is then not valid).
 * MOFF_E_UNSUPPORTED for the split transforms.  Grid sizes whose kernel leaves too few resident workgroups for
 * column owners plus row workers run two-pass within the same call.  Setting the pipeline drops cached graphs. */
moff_status moff_set_pipeline(moff_plan_t plan, int32_t pipeline);
/* Synchronises the device, then reads the streaming form's status code of the last fused call. */
moff_status moff_stream_status(moff_plan_t plan, int32_t *code);

/* Electric-field image taps and feedback calibration (Section 6; the Discussion notes that each pixel of the
 * E-field image is a calibrated tied-array beam, fit for pulsar and transient work).
 *
 * moff_set_taps: the desc.n_tap pixels of every channel, h_pix int32 [C][n_tap][2] = centred (row, col) as
 * in moff_read_image's layout (host memory, copied; the tables are uploaded on the stream).
 * moff_correlate_tap: moff_correlate (two-pass form, whatever the pipeline setting), plus the E-field image
 * of every sample at the tapped pixels, before squaring: d_tap complex64 [n_t][C][n_tap][P] (fully written).
 * moff_cal_accumulate adds to d_cal (FP64, caller-zeroed, moff_cal_size bytes) the sums over the n_t samples
 *   R[c][m][a][p] = sum_t E_tap[t][c][m][p] conj(E[t][c][a][p])   (double2 [C][n_tap][A][P]; Eq. FBeq2's
 *                   correlation of the image pixel with one antenna's input, before the gain factor)
 *   Pw[c][m][p]   = sum_t |E_tap[t][c][m][p]|^2                   (double [C][n_tap][P]; Eq. FBeq1)
 *   V[c][a][p]    = sum_t |E[t][c][a][p]|^2                       (double [C][A][P])
 * in that order in the buffer.  d_volt and d_tap are those of the same samples.
 * moff_cal_solve: with g = B_a(theta_m) (the image of a unit voltage on antenna a alone at tap m, i.e. its
 * kernel's DFT there, computed in FP64 from d_kern, the diagonal kernels [C][A][P][K][K] in use), writes
 * d_out double2 [3][C][n_tap][A][P]: S = conj(g) R (Eq. FBeq2's left side; the printed right side is its
 * conjugate), X = Pw - S - conj(S) + |g|^2 V (the exact sum of all visibilities not involving antenna a;
 * Eq. FBeq3 as printed omits the k = a terms) and u = 2 - A conj(S) / Pw, the single-calibrator gain update
 * g -> u g (the printed factor 2A would give -g at convergence; A makes it vanish there).  u can be fed back
 * as the per-antenna factor of moff_set_kernels_phased.  MOFF_E_UNSUPPORTED for Jones kernels. */
moff_status moff_set_taps(moff_plan_t plan, const int32_t *h_pix, void *stream);
moff_status moff_correlate_tap(moff_plan_t plan, const void *d_volt, int64_t n_t, void *d_acc, void *d_tap,
                               void *stream);
moff_status moff_cal_size(moff_plan_t plan, size_t *bytes);
moff_status moff_cal_accumulate(moff_plan_t plan, const void *d_volt, const void *d_tap, int64_t n_t, void *d_cal,
                                void *stream);
moff_status moff_cal_solve(moff_plan_t plan, const void *d_cal, const void *d_kern, void *d_out, void *stream);

/* Kernel timing (tracing).  moff_profile(plan, 1) starts recording a pair of HIP events around every launch of
 * the fused path on the caller's stream (earlier records are dropped); moff_profile(plan, 0) stops.  After the
 * stream has been synchronised, moff_profile_read sums, for kernel kind 0 (row pass: gridding + row FFTs),
 * 1 (column pass: column FFTs + products + accumulation) or 2 (streaming form: both), the event-measured time
 * in ms, the launch count and the channel-samples those launches processed.  Recording adds two event records
 * per launch. */
moff_status moff_profile(moff_plan_t plan, int32_t enable);
moff_status moff_profile_read(moff_plan_t plan, int32_t kind, double *total_ms, int64_t *launches,
                              int64_t *channel_samples);

/* Issue-rate probes (measurement only, no plan): kind 0 runs `blocks` workgroups of 256 threads, each thread
 * `iters` iterations of 8 independent FP32 FMA chains (blocks x 256 x iters x 16 flops); kind 1 runs `blocks`
 * workgroups of 4 wavefronts, each wavefront `iters` x 4 independent v_mfma_f32_16x16x32_f16 (blocks x 4 x iters
 * x 4 x 16384 flops).  d_out: caller-owned device float [blocks x 256], one value per thread (the work is not
 * optimised away).
 * Exchange probes (the data movement between the stages of a spatial transform, Eq. m6 step 3): d_out holds
 * blocks x 16 complex float transforms of 256 points, transformed in place iters times, each time
 * X[k] = (1/256) sum_n x[n] e^(+2 pi i n k / 256).  Kind 2: two radix-16 stages per transform with the transpose
 * between them through LDS (natural-order output); kind 3: eight radix-2 stages, the last six exchanging values
 * across the lanes of a wavefront (output position n holds X[bit-reversed n]).
 * Kind 4: thread 0 of each of `blocks` workgroups writes its XCD number (hardware XCC_ID) to d_out[b] (float
 * [blocks]; iters unused but >= 1).
 * Exchange-pattern probes (the HBM access patterns of the 256^2 dual-pol fused path's row-to-column exchange,
 * Section 5's inter-module exchange, with no arithmetic): d_out holds `blocks` channel-samples of column-group
 * tiles, complex float [blocks][2][32][256][8] (1 MiB each; iters unused but >= 1).  Kind 5 stores all of them in
 * the row pass's order (workgroups of 8 rows x 32 channel-samples, non-temporal 8-byte stores); kind 6 loads them
 * in the column pass's order (workgroups of 8 columns x 256 channel-samples, non-temporal 8-byte loads) and
 * overwrites one element per thread with the sum of what it read.
 * Enqueues on `stream`; the caller times it.  MOFF_E_INVALID for blocks or iters < 1, a NULL d_out or an unknown
 * kind. */
moff_status moff_probe(int32_t kind, int32_t blocks, int32_t iters, float *d_out, void *stream);

void moff_plan_destroy(moff_plan_t plan);
const char *moff_status_str(moff_status s);
/* Text of the most recent error on this thread ("" if none). */
const char *moff_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MOFF_H */
