/*
 * rl.h - C ABI of the MI355X (gfx950) Richardson-Lucy deconvolution library.
 *
 * Operation (paper §4.3, paragraph "Richardson-Lucy algorithm"): iterative
 * deconvolution under a Poisson noise model.  One iteration of the estimate u
 * against the observed volume d with the PSF h is
 *
 *     q = H u                      forward blur  (convolution with h, see rl_boundary)
 *     r = d / q  where q > 1e-12, else 0
 *     c = H^T r                    back-projection with the mirrored PSF
 *     u = u * max(c, 0)
 *
 * where H uses the PSF normalised to unit sum (in FP64) with its centre at
 * voxel floor(p/2) on each axis, and H^T is the exact adjoint of H (the
 * correlation; in the frequency domain a multiplication by the conjugate
 * transfer function).  By default image and PSF have the same ZYX shape, as in
 * the paper's experiment (§4.3, paragraph "Dataset description");
 * rl_options.psf_shape admits a smaller PSF.
 *
 * Conventions shared by every call:
 *   - Volumes are dense, C-ordered float32 arrays [Z][Y][X], X contiguous,
 *     shape given as {nz, ny, nx}.
 *   - Every data pointer is a DEVICE pointer on the plan's GPU, owned by the
 *     caller, at least 16-byte aligned, covering nz*ny*nx floats.
 *   - Transform lengths.  nx must be even, 4 <= nx <= 4096, with nx/2 =
 *     o * 2^a, o in {1, 3, 5, 7, 9, 15}, split over a power-of-two number of
 *     threads <= 64, each holding E in {1..10, 12, 14, 15, 16, 18, 20, 24, 30}
 *     elements that carry every odd factor of nx/2 (e.g. nx = 2560).  ny and nz
 *     are 2^a 3^b 5^c 7^d <= 4096: where an E carries the whole odd part the
 *     rule is the same (threads <= 1024), else E needs each odd prime once and
 *     the thread count carries the rest (e.g. 2160 = 16 * 135 as 30 elements on
 *     72 threads).  At most 8 radix stages (16, 8, 4, 2, then 7, 5, 3), and a
 *     pencil's work-group must fit the LDS (length x lanes x 8 bytes <= 160 KB).
 *     Other lengths return RL_E_UNSUPPORTED (for the zero boundary the rule
 *     applies to the padded transform grid).
 *   - Environment: RLMI_TUNE_CACHE (see rl_options.autotune); RLMI_AUTOTUNE=1
 *     or 0 turns the autotuner on or off for every plan whatever its options
 *     say; RLMI_SYNC_DEBUG=1 synchronises the plan's stream after every kernel
 *     launch (outside graph capture) and reports an execution fault as
 *     RL_E_DEVICE against the launch that caused it (slow; for debugging).
 *     Each is read once per process.
 *   - All argument checks run before any device work; a failing call leaves
 *     every buffer untouched.  No call aborts, exits or throws.
 *   - Work is enqueued on the plan's stream (default: the null stream) and
 *     returns without waiting, except where a call says it synchronises.
 *     Faults during execution surface at the next synchronising call.
 *   - A plan is not re-entrant: use it from one host thread / stream at a time.
 *   - Error detail for the last failing call on this thread: rl_last_error().
 */
#ifndef RL_H_
#define RL_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rl_plan_s* rl_plan; /* opaque, owned by the library */

typedef enum {
  RL_OK = 0,
  RL_E_INVALID = 1,     /* bad argument: NULL, misaligned, wrong size, bad PSF, ... */
  RL_E_UNSUPPORTED = 2, /* valid request this library does not implement */
  RL_E_NOMEM = 3,       /* device allocation failed */
  RL_E_DEVICE = 4,      /* no usable GPU, or a HIP runtime / launch error */
  RL_E_NUMERIC = 5,     /* non-finite flux detected at a synchronising call */
  RL_E_INTERNAL = 6     /* unexpected internal failure */
} rl_status;

/*
 * Boundary of the blur.  The PSF (shape p <= the volume's per axis, centre
 * voxel floor(p/2), normalised to unit sum) acts as
 *   (H x)[i] = sum_m h[m] x[i - (m - floor(p/2))]
 * PERIODIC: indices wrap around the volume (circular convolution); the volume's
 *   dimensions must be transform lengths (see rl_plan_create).
 * ZERO: x is zero outside the volume (linear convolution, output kept on the
 *   volume's grid).  The library transforms on a padded grid of at least
 *   n + floor(p/2) per axis (rounded up to a transform length; rl_plan_get_grid),
 *   so the volume may have any dimensions whose padded grid is supported.  The
 *   adjoint is the linear correlation; the update is unchanged, so the flux
 *   sum(u) is still conserved.  Single-volume plans only.
 */
typedef enum {
  RL_BOUNDARY_PERIODIC = 0,
  RL_BOUNDARY_ZERO = 1
} rl_boundary;

typedef enum {
  RL_PRECISION_FP32 = 0,       /* FP32 transforms, FP64 twiddle generation and sums */
  RL_PRECISION_SPLIT_BF16 = 1, /* radix-16 butterflies of the Y and Z transforms as 32x32
                                  real DFT matrices on MFMA, operands split into BF16
                                  hi + lo, three products accumulated in FP32; other
                                  stages, twiddles, the elementwise steps and all sums as
                                  in FP32 mode.  The X transforms (fused with the ratio
                                  and the update) keep FP32 radix-8/4 butterflies unless
                                  rl_options.x_elems = 16 asks for radix-16 stages there,
                                  which then run on MFMA too */
  RL_PRECISION_SPLIT_FP16 = 2  /* the same with FP16 hi + lo and a power-of-two scale
                                  per 16-point DFT */
} rl_precision;

/* Iteration scheme (rl_options.accel). */
typedef enum {
  RL_ACCEL_NONE = 0,           /* plain Richardson-Lucy */
  RL_ACCEL_BIGGS_ANDREWS = 1   /* first-order vector extrapolation of Biggs & Andrews,
                                  Applied Optics 36(8), 1997 (the acceleration behind the
                                  CUDA deconvolution tool of the paper's related work):
                                  each iteration starts from y_k = max(x_k + alpha_k h_k, 0),
                                  h_k = x_k - x_{k-1},
                                  alpha_k = <g_{k-1}, g_{k-2}> / <g_{k-2}, g_{k-2}> clipped
                                  to [0, 1], g_k = x_{k+1} - y_k; alpha_0 = alpha_1 = 0 */
} rl_accel;

/* Options for rl_plan_create_ex.  Zero-initialise, then set fields. */
typedef struct {
  int precision;  /* rl_precision */
  void* stream;   /* hipStream_t to enqueue on; NULL = null stream */
  int tile_x;     /* work-group width of the Y/Z passes in complex elements: 1..16 =
                     columns of one 16-column tile, 32/64 = 2/4 whole tile rows (Z
                     pass only); 0 = library default; out of range = RL_E_INVALID */
  int x_elems;    /* elements per thread of the X-pass transforms (length nx/2); 0 =
                     default; must divide nx/2 leaving a power-of-two thread count
                     <= 64, carry every odd factor of nx/2 and be even when
                     nx/2 is (else RL_E_INVALID) */
  int yz_elems;   /* the same for the Y and Z transforms (lengths ny and nz) */
  int autotune;   /* 1: at plan creation, time candidate elements-per-thread and
                     work-group widths for each pass on this GPU and keep the
                     fastest (adds tens of ms; needs 8 bytes per voxel of
                     temporary device memory).  With RLMI_TUNE_CACHE naming a
                     text file, results are read from / appended to it, keyed
                     by GPU architecture, HIP runtime version, shape and
                     precision; the
                     last line of a key wins, and a line whose configuration
                     does not fit the shape is ignored (the plan tunes afresh
                     and appends a new line). */
  int accel;      /* rl_accel.  RL_ACCEL_BIGGS_ANDREWS keeps two more plan-owned
                     volumes (8 bytes per voxel: the last step h and change g) and
                     costs one more X pass and a one-work-group reduction per
                     iteration; single-volume plans only (rl_plan_create_batch
                     returns RL_E_UNSUPPORTED). */
  int64_t psf_shape[3]; /* {pz, py, px} of the PSF passed to rl_plan_create_ex;
                     {0, 0, 0} = the volume's shape.  Each must be in [1, the
                     volume's dimension] (else RL_E_INVALID); the PSF is centred
                     at voxel floor(p/2) and zero beyond its extent.  Single-
                     volume plans only. */
  int batch_mode; /* rl_batch_mode, batch plans only (single-volume plans ignore it) */
} rl_options;

/* How rl_iterate_batch runs one iteration of all volumes (rl_options.batch_mode). */
typedef enum {
  RL_BATCH_AUTO = 0,       /* RL_BATCH_GRAPH (RL_BATCH_PERSISTENT is switched off) */
  RL_BATCH_PERSISTENT = 1, /* one persistent kernel launch per iteration: work-groups
                              of 128 threads take the tiles of every pass of every
                              volume from per-XCD work queues in pass-major order and
                              wait on per-(volume, pass) completion counters; each
                              volume's tiles run on one XCD.  Switched off in this
                              library: its completion waits did not finish on MI355X,
                              and plan creation returns RL_E_UNSUPPORTED */
  RL_BATCH_GRAPH = 2       /* per-pass kernels of each shape class: one hipGraph of
                              one iteration per class, replayed on the class's own
                              stream */
} rl_batch_mode;

/*
 * Create a plan for volumes of shape {nz, ny, nx} blurred by `psf`
 * (device pointer, the same shape; rl_options.psf_shape allows a smaller one).
 * The PSF is read only during this call: it must be finite, >= 0 and have a
 * positive sum (else RL_E_INVALID); it is normalised to unit sum in FP64 and
 * its transfer function is stored in the plan (plan-owned device memory, about
 * 8 bytes per voxel of the transform grid including the spectrum workspace).
 * Periodic boundary: each dimension must be a transform length as stated
 * above (else RL_E_UNSUPPORTED).  Zero boundary: those limits apply to the padded grid.
 * Synchronous: returns after all device work is done.  On success *out
 * receives the plan; on failure *out is set to NULL.
 */
rl_status rl_plan_create(const int64_t shape[3], const float* psf, int boundary,
                         rl_plan* out);

/* As rl_plan_create, with options (may be NULL for defaults). */
rl_status rl_plan_create_ex(const int64_t shape[3], const float* psf, int boundary,
                            const rl_options* opt, rl_plan* out);

/*
 * Run exactly n_iter Richardson-Lucy iterations in place on `estimate`
 * (device, read/write), starting from its current contents, against
 * `observed` (device, read-only).  n_iter == 0 is a no-op; n_iter < 0 is
 * RL_E_INVALID.  The FP64 total flux sum(u) after each iteration is kept on
 * the device for rl_plan_get_flux.  Asynchronous on the plan's stream;
 * `observed` and `estimate` must stay valid until that work completes.
 * Calling again continues the iteration (resume).  With extrapolation
 * (rl_options.accel) every call starts the extrapolation afresh from
 * `estimate` (alpha_0 = alpha_1 = 0 again), so a split run differs from an
 * unsplit one.
 */
rl_status rl_iterate(rl_plan p, const float* observed, float* estimate, int n_iter);

/*
 * rl_iterate for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * plain iteration, kernels and results as rl_iterate, with its per-iteration flux
 * partials in a fixed device array of the library (8 MiB, 2^20 FP64 values, one
 * per GPU, held until the process ends) instead of plan memory that rl_iterate
 * grows for long calls.  The call makes no device allocation.  Limits (else
 * RL_E_INVALID, nothing enqueued): n_iter times the plan's X-pass work-group
 * count <= 2^20, and n_iter <= the plan's flux capacity (128, or the longest
 * earlier rl_iterate call).  Plain single-volume plans without per-launch
 * timing only (else RL_E_UNSUPPORTED).  Every call on a GPU shares that GPU's
 * array: calls that overlap in time on one GPU (other streams, other plans,
 * other host threads) race and give wrong flux values; order them.  The array
 * keeps the last call's contents, which no call reads before writing.
 * rl_plan_get_flux returns the flux as after rl_iterate.
 */
rl_status rl_iterate_noalloc(rl_plan p, const float* observed, float* estimate, int n_iter);

/*
 * out = H x: circular convolution of x (device) with the plan's normalised PSF,
 * exactly the forward operator rl_iterate uses.  `out` may alias `x`.
 * Asynchronous on the plan's stream.
 */
rl_status conv3d_fft(rl_plan p, const float* x, float* out);

/*
 * Batched form: `count` independent volumes, volume v of shape
 * {shapes[3v], shapes[3v+1], shapes[3v+2]} with its own PSF psfs[v] (device
 * pointers, each the shape of its volume), deconvolved together.  Volumes of
 * equal shape form one class; each class keeps its spectra and transfer
 * functions back to back.  Constraints per volume as for rl_plan_create;
 * opt->tile_x must be 0; opt->autotune tunes each shape once.  Synchronous.
 * The plan's stream (opt->stream) orders calls; the library forks private
 * streams, one per class, from it and joins them back.
 */
rl_status rl_plan_create_batch(int count, const int64_t* shapes, const float* const* psfs,
                               int boundary, const rl_options* opt, rl_plan* out);

/*
 * n_iter iterations of every volume of a batch plan: observed[v] and
 * estimate[v] are device pointers (host arrays of `count` pointers, read
 * during the call).  One iteration of one shape class is one hipGraph launch
 * (captured on the first call, replayed afterwards) on the class's private
 * stream; the classes run their iterations independently and join the plan's
 * stream once, at the end of the call.  rl_plan_get_flux then returns
 * count * n_iter values,
 * volume-major (flux[v * n_iter + t]).  Asynchronous like rl_iterate.
 */
rl_status rl_iterate_batch(rl_plan p, const float* const* observed, float* const* estimate,
                           int n_iter);

/*
 * Metric-guided automatic stopping (paper §4.3: the iteration count is chosen by
 * monitoring an image-quality metric between consecutive iterations and stopping
 * once its improvement falls below a configurable threshold).
 *   RL_STOP_LOGLIK: l_k = sum over q > 1e-12 of (d log q - q), q = H u_k, the
 *     Poisson log-likelihood RL maximises, evaluated for the estimate entering
 *     iteration k (computed inside that iteration's ratio pass).  Stops at
 *     iteration k >= 1 when (l_k - l_{k-1}) / |l_k| < threshold; iteration k is
 *     then not carried out (k iterations done).  Values are FP64 sums of FP32
 *     blurs: improvements below ~1e-7 are rounding.
 *   RL_STOP_CHANGE: m_k = ||u_{k+1} - u_k|| / ||u_k|| after iteration k; stops
 *     when m_k < threshold (k + 1 iterations done).
 *   RL_STOP_PSNR: scale-invariant PSNR of u_{k+1} against `reference` (device,
 *     the volume's shape): 20 log10(max g - min g) - 10 log10(mean squared
 *     residual of the least-squares affine fit of u to g); stops at k >= 1 when
 *     psnr_k - psnr_{k-1} < threshold (dB; k + 1 iterations done).
 *   RL_STOP_SSIM: mean SSIM of u_{k+1} against `reference` (see rl_ssim); stops at
 *     k >= 1 when ssim_k - ssim_{k-1} < threshold (k + 1 iterations done).  Runs
 *     three window-sum passes after each update (about 170 bytes per voxel).
 *   RL_STOP_FSC: single-image Fourier shell correlation resolution of u_{k+1}
 *     (no reference; paper §4.3 lists FRC/FSC among its metrics): the FSC of the
 *     two diagonal half-size sub-volumes u[0::2, 0::2, 0::2] and u[1::2, 1::2, 1::2]
 *     (rl_split_diagonal) with fsc_bins shells and crossing threshold
 *     fsc_threshold (rl_fsc), in cycles per voxel of the half-size volumes; stops
 *     at k >= 1 when res_k - res_{k-1} < threshold (k + 1 iterations done).  Needs
 *     a periodic plan with even dimensions whose halves are transform lengths
 *     (else RL_E_UNSUPPORTED).  After each update the split, two half-size
 *     forward transforms and the shell sums run on the device (about 10 bytes per
 *     voxel); a transform-only plan of the half shape and its buffers (about 3.5
 *     bytes per voxel) are allocated on first use and kept with the plan.
 * No stop happens before min_iter iterations are done.  The metric is
 * accumulated in FP64 inside the passes (no extra pass over the volume; PSNR
 * reads the reference, 4 bytes per voxel per iteration).
 */
typedef enum {
  RL_STOP_LOGLIK = 1,
  RL_STOP_CHANGE = 2,
  RL_STOP_PSNR = 3,
  RL_STOP_SSIM = 4,
  RL_STOP_FSC = 5
} rl_stop_metric;

typedef struct {
  int metric;              /* rl_stop_metric */
  double threshold;        /* finite */
  int min_iter;            /* >= 0 */
  const float* reference;  /* RL_STOP_PSNR and RL_STOP_SSIM: device, the volume's shape */
  int fsc_bins;            /* RL_STOP_FSC: shells, 0 = 64, else in [2, 1024] */
  double fsc_threshold;    /* RL_STOP_FSC: FSC crossing level, 0 = 1/7, else finite */
} rl_stop_rule;

/*
 * At most max_iter iterations of rl_iterate on a single-volume plan without
 * extrapolation (else RL_E_UNSUPPORTED), ended early by `rule`.  The whole call
 * is enqueued at once; a one-work-group kernel evaluates the rule after each
 * check and sets a device flag, after which every remaining launch of the call
 * returns at once, so no host synchronisation is needed.  Asynchronous like
 * rl_iterate.  rl_plan_get_flux then returns the flux of the iterations done.
 */
rl_status rl_iterate_stop(rl_plan p, const float* observed, float* estimate, int max_iter,
                          const rl_stop_rule* rule);

/*
 * After rl_iterate_stop (else RL_E_INVALID): iterations carried out in
 * *n_done, and the metric value of every check in history[0 .. min(cap, n) - 1]
 * with n in *n_history (LOGLIK: l_0 .. l_k; CHANGE, PSNR, SSIM and FSC: one value
 * per iteration done).  Synchronises the plan's stream.
 */
rl_status rl_plan_get_stop(rl_plan p, int* n_done, double* history, int cap, int* n_history);

/*
 * Structural similarity (paper §4.3 lists SSIM against ground truth among its
 * metrics; Wang et al. 2004) of u against `reference` (device, the plan's volume
 * shape, every dimension >= 7, else RL_E_UNSUPPORTED): 7x7x7 uniform windows
 * lying inside the volume, sample (co)variances (normalised by 342),
 * C1 = (0.01 L)^2, C2 = (0.03 L)^2 with L = max - min of the reference;
 * *value = mean over the windows.  Window sums in FP64; buffers of about
 * 80 bytes per voxel are allocated on first use.  Synchronous.
 */
rl_status rl_ssim(rl_plan p, const float* u, const float* reference, double* value);

/*
 * Fourier shell correlation (paper §3 and §4.3: FRC/FSC and a single-image
 * FRC-derived resolution are among its quality metrics) of volumes a and b
 * (device, the plan's shape; periodic single-volume plans, else
 * RL_E_UNSUPPORTED), with the plan's transforms: F = DFT(a), G = DFT(b);
 * shell s = floor(rho / 0.5 * nbins) of each frequency, rho = sqrt(sum_i
 * (k_i / n_i)^2) with k_i the signed index in [-n_i/2, n_i/2) (shells 0 ..
 * nbins-1 cover rho < 0.5 cycles per voxel, shell nbins the corners beyond);
 * curve[s] = sum_s Re(F conj G) / sqrt(sum_s |F|^2 sum_s |G|^2) (0 if a
 * denominator is 0) for s = 0 .. nbins (host array of nbins + 1).
 * *resolution (may be NULL): the frequency, in cycles per voxel, where the
 * curve first drops below `threshold` (shell s >= 1, interpolated linearly
 * between the centres (s - 0.5) * 0.5 / nbins and (s + 0.5) * 0.5 / nbins);
 * 0.5 if it never does.  nbins in [2, 1024].  Uses the plan's spectrum
 * workspace and a second one allocated on first use; synchronous.
 * Shell sums are accumulated with shared-memory atomics, so their last bits
 * may vary between calls.
 */
rl_status rl_fsc(rl_plan p, const float* a, const float* b, int nbins, double threshold,
                 double* curve, double* resolution);

/*
 * Single-image split: a = u[0::2, 0::2, 0::2], b = u[1::2, 1::2, 1::2] of the
 * dense volume u of `shape` (every dimension even; a and b hold shape/2 each;
 * all device pointers).  Asynchronous on `hip_stream`.  rl_fsc of a and b on a
 * plan of the half shape gives the single-image FSC.
 */
rl_status rl_split_diagonal(const float* u, const int64_t shape[3], float* a, float* b,
                            void* hip_stream);

/* Release the plan and its device memory (waits for its pending work). NULL is a no-op. */
void rl_plan_destroy(rl_plan p);

/* Enqueue later work of this plan on `hip_stream` (a hipStream_t; NULL = null stream). */
rl_status rl_plan_set_stream(rl_plan p, void* hip_stream);

/*
 * Copy the per-iteration FP64 flux of the most recent rl_iterate call into
 * flux[0 .. min(cap, n) - 1] and its length n into *n_written.  Synchronises
 * the plan's stream.  Returns RL_E_NUMERIC if any value is not finite (this is
 * also where a NaN/Inf in the inputs is reported).
 */
rl_status rl_plan_get_flux(rl_plan p, double* flux, int cap, int* n_written);

/*
 * Extrapolated plans (accel = RL_ACCEL_BIGGS_ANDREWS): copy the FP64 weight
 * alpha_k used by iteration k = 0 .. n-1 of the most recent rl_iterate call
 * into alpha[0 .. min(cap, n) - 1] and n into *n_written.  Synchronises the
 * plan's stream.  RL_E_INVALID for a plan without extrapolation.
 */
rl_status rl_plan_get_alpha(rl_plan p, double* alpha, int cap, int* n_written);

/* Shape {nz, ny, nx} of the plan's volumes and the number of complex columns
 * the plan stores per half-spectrum row (grid nx/2 + 1 rounded up to whole
 * 16-column tiles). */
rl_status rl_plan_get_info(rl_plan p, int64_t shape[3], int64_t* spectrum_pitch);

/* Transform grid {nz, ny, nx}: the volume's shape for the periodic boundary,
 * the padded grid for the zero boundary (batch plans: the first volume's). */
rl_status rl_plan_get_grid(rl_plan p, int64_t grid[3]);

/* Launch configuration in use: out = {X elements per thread, Y elements per
 * thread, Y work-group lanes, Z elements per thread, Z work-group lanes,
 * 1 if chosen by the autotuner else 0, 1 if the Z grid runs row groups
 * fastest else 0, 1 if a batch plan runs the persistent kernel else 0 (always 0
 * while that kernel is switched off)}
 * (batch plans: the first volume's shape class). */
rl_status rl_plan_get_launch(rl_plan p, int out[8]);

/*
 * Per-kernel timing with HIP events (measurement support).  When enabled,
 * every kernel the plan launches is bracketed by events on the plan's stream.
 * rl_plan_get_timing synchronises and returns, for each kernel kind k in
 * [0, RL_KERNEL_KINDS), the number of launches and their summed duration in
 * milliseconds since timing was enabled; it then clears the counters.
 */
enum {
  RL_KERNEL_X_R2C = 0,    /* X pass: real rows -> half spectrum */
  RL_KERNEL_X_C2R = 1,    /* X pass: half spectrum -> real rows */
  RL_KERNEL_X_RATIO = 2,  /* X pass: inverse, ratio d/q, forward */
  RL_KERNEL_X_UPDATE = 3, /* X pass: inverse, multiplicative update + flux, forward */
  RL_KERNEL_Y = 4,        /* Y pass, forward or inverse */
  RL_KERNEL_Z_OTF = 5,    /* Z pass: forward, times (conj) transfer function, inverse */
  RL_KERNEL_Z = 6,        /* Z pass, forward only (plan creation) */
  RL_KERNEL_OTHER = 7,    /* twiddles, PSF reduction and preparation */
  RL_KERNEL_KINDS = 8
};
rl_status rl_plan_set_timing(rl_plan p, int enable); /* RL_E_UNSUPPORTED for batch plans */
rl_status rl_plan_get_timing(rl_plan p, int count[RL_KERNEL_KINDS], double ms[RL_KERNEL_KINDS]);

/*
 * Steady-state duration of one pass (measurement support): launches the pass
 * of kind RL_KERNEL_X_RATIO, RL_KERNEL_X_UPDATE, RL_KERNEL_Y (forward) or
 * RL_KERNEL_Z_OTF `reps` times back to back on the plan's spectrum workspace
 * (with `observed` / `estimate` as the real operands of the X passes; the
 * update pass overwrites `estimate` and the workspace) and returns the average
 * time per launch in milliseconds from two HIP events around the burst.
 * Synchronises.  Single-volume plans only.
 */
rl_status rl_plan_time_pass(rl_plan p, int kind, const float* observed, float* estimate,
                            int reps, double* ms_per_launch);

/*
 * Kernels of one pass kind as a profiler names them (measurement support):
 * writes the kernel template name(s) used for kind RL_KERNEL_X_RATIO,
 * RL_KERNEL_X_UPDATE, RL_KERNEL_Y or RL_KERNEL_Z_OTF into name[0 .. cap-1]
 * (NUL-terminated; two names joined by '|' where the pass has a forward and an
 * inverse, or a plain and a conjugate, variant, e.g.
 * "k_pencil<8, 0, 1024, 0>|k_pencil<8, 1, 1024, 0>"; pencils compiled for their
 * length are named k_pencil_ct<E, mode, precision, length>, X rows compiled for
 * theirs carry the row length as the last argument of k_xrow) and the number of
 * threads one launch runs (work-groups times work-group size) into *threads.
 * RL_E_INVALID if cap is too small.  Single-volume plans only.
 */
rl_status rl_plan_get_pass_kernel(rl_plan p, int kind, char* name, size_t cap, int64_t* threads);

/*
 * Bandwidth probe (measurement support): copy `bytes` bytes (multiple of 16)
 * from device `src` to device `dst` with a plain streaming kernel on
 * `hip_stream`.  Used to calibrate hardware byte counters against a known
 * amount of traffic.
 */
rl_status rl_probe_copy(const void* src, void* dst, size_t bytes, void* hip_stream);

/* Static text for a status code. */
const char* rl_status_string(rl_status s);

/* Detail of the last failing call made by this thread ("" if none). */
const char* rl_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RL_H_ */
