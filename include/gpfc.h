/*
 * gpfc.h - C ABI of the MI355X (gfx950) phase-fold + box-SNR library.
 *
 * Method: GPU phase folding of Wang, Ge, Willis, Wang, Zhao, "The GPU Phase
 * Folding and Deep Learning Method for Detecting Exoplanet Transits"
 * (MNRAS 2024, arXiv:2312.02063). A light curve is folded at every trial
 * period of a grid (Sec. 2.1, Sec. 2.3); each folded curve is binned in phase
 * and scored.
 *
 * Conventions for every call below
 *  - Array arguments are DEVICE pointers (e.g. torch tensors' data_ptr()) on
 *    the plan's device, unless the comment says "host". The caller allocates
 *    and owns them; the library never frees caller memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream). Work
 *    is enqueued asynchronously on it; outputs are valid once the stream has
 *    reached that point.
 *  - Return value: GPFC_OK (0) or a negative error code. Argument checks run
 *    on the host before any GPU work is enqueued; on an argument error nothing
 *    is enqueued and no output is touched. No C++ exception crosses the ABI.
 *  - A plan (and its device workspace) must not be used by two host threads,
 *    or by two streams that run concurrently, at the same time.
 *  - Layout of per-period outputs: row-major [k][nbins].
 *  - Phase zero is t = 0 of the caller's time scale; t need not be sorted.
 */
#ifndef GPFC_H
#define GPFC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GPFC_OK 0
#define GPFC_EINVAL (-1)   /* null pointer, negative size, nbins < 1, bad widths,
                              non-finite t or flux (reported by gpfc_sync / gpfc_curve_stats) */
#define GPFC_ENOTSUP (-2)  /* nbins not a power of two in [1, 4096] (or outside the
                              narrower range a call states) */
#define GPFC_ERANGE (-3)   /* n or k beyond what the call takes */
#define GPFC_ENOMEM (-4)   /* device workspace allocation failed */
#define GPFC_EDEVICE (-5)  /* a HIP call failed; gpfc_last_error() has the text */
#define GPFC_EIO (-6)      /* a network file could not be written, read, or is not one */

#define GPFC_MAX_SAMPLES 2147483647LL   /* 2^31 - 1 samples per curve */
#define GPFC_MAX_PACKED 262143          /* 2^18 - 1: curves the fused kernels fold in one
                                           pass (the packed 64-bit bin counter); longer
                                           single curves take the general path */
#define GPFC_MAX_NBINS 4096
#define GPFC_FUSED_MAX_NBINS 256        /* nbins of the fused kernels, the batch and the survey */
#define GPFC_MAX_WIDTHS 24

typedef struct gpfc_plan gpfc_plan;

/* Curve statistics (host struct), filled by gpfc_curve_stats. */
typedef struct gpfc_curve {
    double mean;     /* mean flux, FP64 */
    double sigma;    /* sample std of flux (ddof 1): the per-point noise of Eq. 2 (Sec. 2.6); 0 if n < 2 */
    double ref;      /* reference flux on the fixed-point grid (multiple of qscale) */
    double qscale;   /* 2^e: weight of one fixed-point unit of a bin sum */
    double tmax;     /* max |t| */
    double maxdev;   /* max |flux - ref| */
    int64_t n;       /* samples */
    int32_t exact;   /* 1: bin sums are exact (every flux - ref is an integer multiple of the
                        fixed-point unit); 0: each sample's deviation was rounded to a unit of
                        about maxdev * 2^-52 (flux spanning more than 53 bits of range) */
    int32_t finite;  /* 1: every t and flux is finite; 0 makes all results unspecified and
                        is reported as GPFC_EINVAL by gpfc_curve_stats and gpfc_sync */
    int32_t words;   /* 1: one 27-bit fixed-point word per sample; 2: two words (deviations
                        needing more than 27 bits, e.g. zero-centred flux): the fused folds
                        then take two passes of 32 periods per block */
    int32_t pad;
} gpfc_curve;

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int32_t gpfc_version(void);

/* Static text for an error code. */
const char *gpfc_strerror(int32_t code);

/* Text of the last GPFC_EDEVICE on the calling host thread ("" if none). */
const char *gpfc_last_error(void);

/*
 * Create a plan on HIP device `device`. A plan owns a device workspace that
 * grows on demand (hipMalloc, so the first call at a new size is not
 * capturable) and a box-width set, initially the default set: the distinct
 * integers nearest to sqrt(2)^j in [1, nbins/2]. *out receives the plan.
 */
int32_t gpfc_plan_create(gpfc_plan **out, int32_t device);

/*
 * Plan options (host struct) for gpfc_plan_create_opts; zero fields take the
 * defaults of gpfc_plan_create.
 *   widths[nw]      box widths, as gpfc_plan_set_widths (nw = 0: default set)
 *   split           sample split, as gpfc_plan_set_split (0: automatic)
 *   tune_cache      autotuner cache path gpfc_autotune uses when its own
 *                   cache_path is NULL (NULL or "": none); copied
 *   workspace_bytes largest device workspace a chunk of the general path
 *                   (nbins > 256 or n > GPFC_MAX_PACKED) may take
 *                   (0: 1 GiB; at least one 64-period chunk is always taken)
 * The fold's precision is not an option: bin counts and sums are exact
 * integers (gpfc_fold_f32_prepared gives the FP32 forms for comparison).
 */
typedef struct gpfc_plan_opts {
    int32_t device;
    int32_t nw;
    int32_t widths[GPFC_MAX_WIDTHS];
    int32_t split;
    int32_t pad;
    const char *tune_cache;
    int64_t workspace_bytes;
} gpfc_plan_opts;

int32_t gpfc_plan_create_opts(gpfc_plan **out, const gpfc_plan_opts *opts_host);

/* Free a plan and its workspace (synchronises the device first). NULL is a no-op. */
int32_t gpfc_plan_destroy(gpfc_plan *plan);

/*
 * Set the box widths (host array, in coarse bins, 1 <= w < GPFC_MAX_NBINS,
 * strictly ascending, at most GPFC_MAX_WIDTHS). nw = 0 restores the default
 * set. Widths not below nbins are skipped when a fold with that nbins is
 * scored. The fused kernels hold 16 widths: with more below nbins, single
 * curves take the general path and batches and surveys return GPFC_ENOTSUP.
 */
int32_t gpfc_plan_set_widths(gpfc_plan *plan, const int32_t *widths_host, int32_t nw);

/*
 * Curve statistics (mean, sigma for Eq. 2's per-point noise, fixed-point
 * grid): t f64[n], flux f32[n]. Synchronous: waits for `stream`, then fills
 * the host struct *out. Returns GPFC_EINVAL (after filling *out, finite = 0)
 * when some t or flux is not finite.
 */
int32_t gpfc_curve_stats(gpfc_plan *plan, const double *t, const float *flux, int64_t n,
                         gpfc_curve *out_host, void *stream);

/*
 * Phase fold (Sec. 2.3, five-step fold with equal-width bins; Fig. 4 panels
 * a, b, d, e): for each trial period P_j and sample i, the bin is
 *   b = floor(nbins * (x - floor(x))),  x = RN(t_i / P_j)  (binary64),
 * clamped to nbins - 1 - bit-identical to that IEEE sequence. Outputs:
 *   sums   f64[k][nbins]  sum of flux in the bin (0 if empty)
 *   counts i32[k][nbins]  samples in the bin
 *   means  f64[k][nbins]  sums / counts, NaN if empty (may be NULL)
 * Inputs: t f64[n], flux f32[n], periods f64[k]; nbins a power of two in
 * [1, 4096]; n <= GPFC_MAX_SAMPLES; k < 2^31. A period that is not finite and
 * > 0 gives an all-zero row (means NaN). n = 0 or k = 0 is valid. Bin sums are
 * count * ref + (exact fixed-point deviation sum), each term rounded once to
 * binary64 (see gpfc_curve.exact). nbins <= 256 with n <= GPFC_MAX_PACKED runs
 * the fused LDS kernel; other shapes run the general path (integer histograms
 * of sample parts accumulated in a plan workspace that grows on demand), with
 * identical results where both apply. Non-finite t or flux makes the results
 * unspecified and is reported by the next gpfc_sync.
 */
int32_t gpfc_fold(gpfc_plan *plan, const double *t, const float *flux, int64_t n,
                  const double *periods, int64_t k, int32_t nbins,
                  double *sums, int32_t *counts, double *means, void *stream);

/*
 * Box-transit SNR of materialised folds (the statistic of Eq. 2, Sec. 2.6,
 * over the BLS box of Sec. 3.1). For every row of sums/counts ([k][nbins] as
 * gpfc_fold writes them), over each width w of the plan's set and each
 * circular start s, with n_in/D_in the box's count and flux-deviation sum:
 *   depth = (S - D_in)/(n - n_in) - D_in/n_in,
 *   snr   = depth * sqrt(n_in (n - n_in) / n) / sigma,
 * keeping the largest positive snr (ties: smaller w, then smaller s).
 * Outputs f32 snr[k], i32 start[k], i32 width[k] (in coarse bins), f32
 * depth[k]; a row with no positive box gives snr = depth = 0 and
 * start = width = -1. sigma is the curve's per-point noise (host value,
 * e.g. gpfc_curve.sigma); sigma not > 0 gives that empty result for every row.
 * nbins a power of two in [1, 4096]. Boxes are compared in FP32 and the
 * winner evaluated in FP64 (a near-tie may pick a box whose FP64 SNR is
 * within FP32 rounding of the largest).
 */
int32_t gpfc_score(gpfc_plan *plan, const double *sums, const int32_t *counts, int64_t k,
                   int32_t nbins, double sigma, float *snr, int32_t *start, int32_t *width,
                   float *depth, void *stream);

/*
 * Fused fold + score: the fold of gpfc_fold followed by the box-SNR of
 * gpfc_score with sigma = the curve's sample std, without materialising the
 * folded curves (16 bytes written per period) when nbins <= 256 and
 * n <= GPFC_MAX_PACKED; other shapes materialise chunks of folds in the plan's
 * workspace. Same inputs as gpfc_fold; same outputs as gpfc_score.
 */
int32_t gpfc_fold_score(gpfc_plan *plan, const double *t, const float *flux, int64_t n,
                        const double *periods, int64_t k, int32_t nbins, float *snr,
                        int32_t *start, int32_t *width, float *depth, void *stream);

/*
 * Prepare a curve once for several folds: runs the curve statistics and
 * writes the plan's prepared curve (times and fixed-point flux, Sec. 2.3's
 * input to the fold) into its workspace. The *_prepared calls below then fold
 * that curve against any number of period arrays; a later gpfc_prepare,
 * gpfc_fold, gpfc_fold_score or gpfc_curve_stats on the same plan replaces
 * it. Same input contract as gpfc_fold.
 */
int32_t gpfc_prepare(gpfc_plan *plan, const double *t, const float *flux, int64_t n, void *stream);

/* gpfc_fold on the plan's prepared curve (GPFC_EINVAL if none). */
int32_t gpfc_fold_prepared(gpfc_plan *plan, const double *periods, int64_t k, int32_t nbins,
                           double *sums, int32_t *counts, double *means, void *stream);

/*
 * gpfc_fold_score on the plan's prepared curve (GPFC_EINVAL if none).
 * zfold (may be NULL; needs 16 <= nbins <= 256): also writes each period's folded
 * curve normalised for the learned scorer (Sec. 2.1: scaled to unit noise
 * before the CNN), as bfloat16 [k][nbins]: bin means minus their mean over
 * the non-empty bins, divided by their standard deviation (ddof 0); empty bins
 * and a zero spread give 0.
 */
int32_t gpfc_fold_score_prepared(gpfc_plan *plan, const double *periods, int64_t k,
                                 int32_t nbins, float *snr, int32_t *start, int32_t *width,
                                 float *depth, uint16_t *zfold, void *stream);

/*
 * gpfc_fold on the prepared curve with FP32 bin sums, for precision studies:
 * compensated = 0 adds float(flux - ref) with plain float LDS atomics;
 * compensated = 1 also accumulates each addition's exact rounding error
 * (TwoSum on the atomic's returned old value) in a second float array. Counts
 * and bins are those of gpfc_fold; sums are count * ref + sum (+ error).
 * Float LDS atomics run far slower than the integer ones gpfc_fold uses.
 */
int32_t gpfc_fold_f32_prepared(gpfc_plan *plan, const double *periods, int64_t k, int32_t nbins,
                               int32_t compensated, double *sums, int32_t *counts, double *means,
                               void *stream);

/*
 * The paper's own two-tier fold (Sec. 2.3 steps 1-5, Fig. 4) of the
 * prepared curve: each sample goes to one of 4096 equal-width intermediate
 * phase bins (same bin definition as gpfc_fold at 4096 bins); the bins are
 * then merged left to right into nbins final bins that hold N / nbins points
 * each, a bin straddling a boundary split in proportion (each part carries
 * its mean flux times the points it takes). Outputs (device, either may be
 * NULL but not both): means f64[k][nbins] (NaN for an invalid period or an
 * empty curve) and zfold u16[k][nbins], bfloat16 z-scores of the means (the
 * network's input). 1 <= nbins <= 256, any integer; n <= GPFC_MAX_PACKED
 * (GPFC_ERANGE beyond).
 */
int32_t gpfc_fold_eqcount_prepared(gpfc_plan *plan, const double *periods, int64_t k,
                                   int32_t nbins, double *means, uint16_t *zfold, void *stream);

/*
 * Sample split of the fold + score of one curve: a grid of fewer 64-period
 * tiles than compute units leaves most of the chip idle, so each tile's
 * samples can be split over `split` blocks whose histograms are merged with
 * exact 64-bit integer atomics (results are identical for every split).
 * split = 0 (default): the value gpfc_autotune found for the prepared
 * curve's n, the grid size and nbins, else one block per compute unit;
 * 1..GPFC_MAX_SPLIT: forced. Applies to gpfc_fold_score and
 * gpfc_fold_score_prepared.
 */
#define GPFC_MAX_SPLIT 64
int32_t gpfc_plan_set_split(gpfc_plan *plan, int32_t split);

/*
 * Autotuner of the block shape for the prepared curve at these periods and
 * nbins: times every power-of-two split the grid allows (3 runs each, HIP
 * events on `stream`; synchronous; allocates a temporary output) and keeps
 * the fastest in the plan. With cache_path (may be NULL) a line
 * "<device> <n> <k> <nbins> <split>" is looked up first (then nothing is
 * timed) and appended after timing. split_out, ms_out (may be NULL): the
 * choice and its time (-1 when taken from the cache).
 */
int32_t gpfc_autotune(gpfc_plan *plan, const double *periods, int64_t k, int32_t nbins,
                      const char *cache_path, int32_t *split_out, float *ms_out, void *stream);

/*
 * Multi-curve batch: many light curves folded and scored in one persistent
 * launch (the paper processes a catalogue curve after curve, overlapping the fold of one
 * curve with the network on the previous one, Sec. 3.3).
 * Setup (synchronous, allocates): sample_offsets_host[n_curves + 1] and
 * period_offsets_host[n_curves + 1] (HOST arrays, starting at 0) cut the
 * concatenated t / flux and periods arrays into curves. Work items (a curve
 * and a block of 64 of its periods) are queued longest curve first. A later
 * setup (or gpfc_survey_setup) replaces the batch. Each curve holds at most
 * GPFC_MAX_PACKED samples (GPFC_ERANGE beyond); batch folds take
 * nbins <= GPFC_FUSED_MAX_NBINS.
 */
int32_t gpfc_batch_setup(gpfc_plan *plan, const int64_t *sample_offsets_host,
                         const int64_t *period_offsets_host, int32_t n_curves);

/*
 * Fold and score every curve of the batch at its own periods: per-curve
 * statistics, packing, then one persistent kernel (one block per compute
 * unit pulling work items from a device counter). t f64[total samples],
 * flux f32[...], periods f64[total periods]; outputs indexed like periods
 * (snr, start, width, depth as gpfc_score; zfold as gpfc_fold_score_prepared,
 * [total periods][nbins], may be NULL). Allocates nothing.
 */
int32_t gpfc_batch_fold_score(gpfc_plan *plan, const double *t, const float *flux,
                              const double *periods, int32_t nbins, float *snr, int32_t *start,
                              int32_t *width, float *depth, uint16_t *zfold, void *stream);

/*
 * Record the gpfc_batch_fold_score launch sequence for these buffers into a
 * HIP graph held by the plan (kernel nodes only). `stream` must be a created
 * stream, not the null stream. gpfc_batch_replay launches the graph on any
 * stream; the buffers must stay valid while replays run.
 */
int32_t gpfc_batch_capture(gpfc_plan *plan, const double *t, const float *flux,
                           const double *periods, int32_t nbins, float *snr, int32_t *start,
                           int32_t *width, float *depth, uint16_t *zfold, void *stream);
int32_t gpfc_batch_replay(gpfc_plan *plan, void *stream);

/* Per-curve statistics of the last batch run (host array of n_curves); synchronous. */
int32_t gpfc_batch_curve_stats(gpfc_plan *plan, gpfc_curve *out_host, void *stream);

/*
 * Plain GPU fold, the baseline the paper's own design resembles (Sec. 2.3,
 * Sec. 2.4: atomic accumulation, one thread per sample and period): IEEE
 * division per update and device-memory atomics. Same contract and outputs
 * as gpfc_fold without means (sums accumulate in FP64 atomics, so they
 * differ from gpfc_fold's only in rounding order).
 */
int32_t gpfc_fold_naive(gpfc_plan *plan, const double *t, const float *flux, int64_t n,
                        const double *periods, int64_t k, int32_t nbins, double *sums,
                        int32_t *counts, void *stream);

/* ------------------------------------------------------------------------
 * Learned scorer (Sec. 2.5: a convolutional network scores each noise-
 * normalised fold; cross-entropy, Adam). Network: 4 x [circular conv1d,
 * kernel 5, padding 2 by wrap-around -> ReLU -> max-pool 2] with
 * 1->16->32->64->64 channels over 256 positions, then fully connected
 * 1024->256->64->1 with ReLU between and a sigmoid output.
 * Parameters (FP32, 312,449 values) in the canonical layout: conv l weight
 * [Cout][Cin][5] then bias, l = 1..4; fc weight [out][in] then bias for
 * 1024->256, 256->64, 64->1; the flatten after block 4 is channel-major
 * (channel * 16 + position). Inputs x are [B][256] normalised folds, either
 * bfloat16 bits (x_f32 = 0, as gpfc_fold_score_prepared's zfold) or FP32.
 * GPFC_CNN_BF16 runs convolutions 2-4 and the first two fully connected
 * layers on bf16 matrix cores with FP32 accumulation; GPFC_CNN_FP32 runs them
 * in FP32 (for checking). Master weights, gradients and Adam moments are
 * always FP32. All pointers are device pointers.
 * ------------------------------------------------------------------------ */
#define GPFC_CNN_BF16 0
#define GPFC_CNN_FP32 1

typedef struct gpfc_cnn gpfc_cnn;

/* Number of parameters (312,449). */
int32_t gpfc_cnn_nparams(void);

/* Text of the last GPFC_EDEVICE of a gpfc_cnn_* call on this thread. */
const char *gpfc_cnn_last_error(void);

/* Create a network on `device` with activation buffers for up to max_batch inputs. */
int32_t gpfc_cnn_create(gpfc_cnn **out, int32_t device, int32_t precision, int64_t max_batch);
int32_t gpfc_cnn_destroy(gpfc_cnn *cnn);

/* Copy params f32[nparams] in; resets the Adam moments and step count. */
int32_t gpfc_cnn_set_params(gpfc_cnn *cnn, const float *params, void *stream);
/* Copy the current parameters out to f32[nparams]. */
int32_t gpfc_cnn_get_params(gpfc_cnn *cnn, float *out, void *stream);

/*
 * Write the parameters to a file at host path `path` (an 8-byte tag
 * "GPFCCNN1", the int64 parameter count, then the FP32 parameters in the
 * canonical order, little-endian), or read such a file back (as
 * gpfc_cnn_set_params: resets the Adam state). Both wait for `stream`.
 * GPFC_EIO when the file cannot be written or read, or is not a network file
 * of this architecture (wrong tag, count or length); the network is then
 * unchanged.
 */
int32_t gpfc_cnn_save(gpfc_cnn *cnn, const char *path, void *stream);
int32_t gpfc_cnn_load(gpfc_cnn *cnn, const char *path, void *stream);

/*
 * Inference path of a bf16 network: on = 1 (the default), the four
 * convolution blocks run as one fused kernel (8 waves per compute unit) that
 * keeps the convolution weights in LDS and every activation in a wave's own
 * LDS slice, each wave taking whole inputs on its own (no block-wide waits);
 * 2, the same fused stack over tiles of 8 inputs in lockstep; 0, layer by
 * layer through device memory. All give bit-identical logits. The setting
 * also selects the training path of a bf16 network: fused (on != 0; the
 * input must be 16-byte aligned, else the layer path is taken) or layer by
 * layer (0). Both give the same loss and fully connected gradients bit for
 * bit; the convolution weight gradients differ only in FP32 summation order.
 */
int32_t gpfc_cnn_set_fused(gpfc_cnn *cnn, int32_t on);

/* Logits f32[B] (sigmoid of a logit is the transit score). B <= max_batch. */
int32_t gpfc_cnn_forward(gpfc_cnn *cnn, const void *x, int32_t x_f32, int64_t B, float *logits,
                         void *stream);

/*
 * Mean binary cross-entropy with logits against labels f32[B] (1 = transit)
 * and its gradient, kept in the network for gpfc_cnn_adam; also copied to
 * loss_out (f32[1]) and grad_out (f32[nparams]) when they are not NULL.
 */
int32_t gpfc_cnn_backward(gpfc_cnn *cnn, const void *x, int32_t x_f32, const float *labels,
                          int64_t B, float *loss_out, float *grad_out, void *stream);

/*
 * FP8 inference of a bf16 network: calibration runs the bf16 forward on
 * x[B][256] and records the largest activation entering each matrix-core
 * layer (accumulated over calls unless reset != 0; synchronous). Forward in
 * FP8 then rounds each layer's input, scaled so that maximum maps to 448, and
 * its weights, scaled per output channel, to OCP E4M3, multiplies on the FP8
 * matrix cores with FP32 accumulation and rescales in the epilogue.
 * GPFC_EINVAL if the network is not bf16 or not calibrated.
 */
int32_t gpfc_cnn_calibrate_fp8(gpfc_cnn *cnn, const void *x, int32_t x_f32, int64_t B,
                               int32_t reset, void *stream);
int32_t gpfc_cnn_forward_fp8(gpfc_cnn *cnn, const void *x, int32_t x_f32, int64_t B, float *logits,
                             void *stream);

/* One bias-corrected Adam step on the FP32 masters with the last gradient
 * (the step count lives on the device; gpfc_cnn_set_params resets it). */
int32_t gpfc_cnn_adam(gpfc_cnn *cnn, float lr, float beta1, float beta2, float eps, void *stream);

/* One training step: gpfc_cnn_backward on x[B][256] and labels[B] (mean
 * loss to loss_out, f32[1], when not NULL), then gpfc_cnn_adam. */
int32_t gpfc_cnn_train_step(gpfc_cnn *cnn, const void *x, int32_t x_f32, const float *labels,
                            int64_t B, float lr, float beta1, float beta2, float eps,
                            float *loss_out, void *stream);

/*
 * A whole training step (gpfc_cnn_backward then gpfc_cnn_adam) recorded
 * into a HIP graph held by the network, for the launch-bound small batches
 * of training: replays read x[B][256] and labels[B] from the same buffers
 * (fill them before each replay), re-pack the weights the previous step
 * changed, and write the step's mean loss to loss_out (f32[1], may be NULL).
 * `stream` must be a created stream, not the null stream. A later capture
 * replaces the graph.
 */
int32_t gpfc_cnn_train_capture(gpfc_cnn *cnn, const void *x, int32_t x_f32, const float *labels,
                               int64_t B, float lr, float beta1, float beta2, float eps,
                               float *loss_out, void *stream);
int32_t gpfc_cnn_train_replay(gpfc_cnn *cnn, void *stream);

/*
 * The paper's own scoring network (Sec. 2.5, Fig. 5): the 256-bin normalised
 * fold read row-major as a 16 x 16 image; circular (wrap-around in both axes,
 * same-size) 2-D convolutions of 128 then 256 filters with 3 x 3 kernels, each
 * followed by ReLU; a global max-pool over the 256 positions, whose 256 values
 * are read row-major as a new one-channel 16 x 16 image; the same with 5 x 5
 * kernels (128 then 256 filters, global max-pool); a dense layer of 128 ReLU
 * units, dropout, and a dense output unit whose sigmoid is the transit
 * probability. The kernel sides, the reshape order and the hidden width are
 * readings: the text names the layer types and filter counts only.
 * Parameters (FP32, flat, gpfc_pnet_nparams() = 1,152,257 values): w1
 * [128][1][3][3], b1 [128], w2 [256][128][3][3], b2 [256], w3 [128][1][5][5],
 * b3 [128], w4 [256][128][5][5], b4 [256], w5 [128][256], b5 [128], w6 [128],
 * b6 [1]; a convolution is a cross-correlation,
 *   y[f][r][c] = b[f] + sum w[f][i][u][v] x[i][(r+u-p) mod 16][(c+v-p) mod 16], p = (side-1)/2;
 * a global max-pool routes its gradient to the first position of the maximum
 * in row-major order. precision: GPFC_CNN_BF16 (matrix cores on bf16 weights
 * and activations, FP32 accumulation, biases FP32) or GPFC_CNN_FP32.
 * max_batch: inputs per internal pass (device memory ~160 KB per input in
 * bf16, twice that in FP32, plus 230 MB of gradient chunk sums); forward
 * takes any batch in passes of it, backward at most max_batch. All arrays are device pointers; calls are
 * asynchronous on `stream`. x: [B][256] bf16 bits (x_f32 = 0) or FP32.
 */
typedef struct gpfc_pnet gpfc_pnet;
int32_t gpfc_pnet_nparams(void);
const char *gpfc_pnet_last_error(void);
int32_t gpfc_pnet_create(gpfc_pnet **out, int32_t device, int32_t precision, int64_t max_batch);
int32_t gpfc_pnet_destroy(gpfc_pnet *net);
/*
 * bf16 forward path: on = 1 (default) runs each convolution pair as one fused
 * kernel per input (activation tile in LDS, pooling in the epilogue); on = 0
 * layer by layer through HBM. Same results bit for bit.
 */
int32_t gpfc_pnet_set_fused(gpfc_pnet *net, int32_t on);
/* Copy in FP32 parameters (device, flat order above); resets Adam. */
int32_t gpfc_pnet_set_params(gpfc_pnet *net, const float *params, void *stream);
int32_t gpfc_pnet_get_params(gpfc_pnet *net, float *params, void *stream);
/* Logits f32 [B] (inference: no dropout). GPFC_EINVAL before set_params. */
int32_t gpfc_pnet_forward(gpfc_pnet *net, const void *x, int32_t x_f32, int64_t B, float *logits,
                          void *stream);
/*
 * Forward with the dropout keep mask keep [B][128] (each entry 0 or
 * 1/(1 - rate), drawn by the caller; NULL: no dropout), then the gradient of
 * the mean binary cross-entropy with logits (labels f32 [B] in {0, 1}) into
 * the network's gradient buffer (gpfc_pnet_get_grads). logits [B] receives
 * the forward's logits, loss (device f32, may be NULL) the mean loss.
 * B <= max_batch (GPFC_ERANGE beyond).
 */
int32_t gpfc_pnet_backward(gpfc_pnet *net, const void *x, int32_t x_f32, const float *labels,
                           const float *keep, int64_t B, float *logits, float *loss, void *stream);
int32_t gpfc_pnet_get_grads(gpfc_pnet *net, float *grads, void *stream);
/* One Adam step (bias-corrected) on the FP32 masters from the last gradient. */
int32_t gpfc_pnet_adam(gpfc_pnet *net, float lr, float beta1, float beta2, float eps, void *stream);

/* ------------------------------------------------------------------------
 * Per-curve reduction (Sec. 2.1: a curve's detection is the trial period
 * with the best score; Sec. 3.2: the maximum score over trial periods is the
 * statistic thresholded for the ROC). For each of `rows` rows of `len`
 * scores values[rows][len]: the `top` best entries, best first, ordered by
 * value descending and then by index ascending, into out_val[rows][top] and
 * out_idx[rows][top] (index within the row). NaN values are skipped, and so
 * is every entry whose gate[rows][len] value is not >= gate_min when gate is
 * not NULL (a NaN gate never passes). Places without an entry get -inf and
 * -1. 1 <= top <= 64; len < 2^32 (GPFC_ERANGE beyond). Device pointers;
 * asynchronous on `stream`. A few long rows are split over many blocks whose
 * lists are merged, with stream-ordered scratch memory (not inside a graph
 * capture, where a row takes one block).
 * ------------------------------------------------------------------------ */
#define GPFC_MAX_TOP 64
int32_t gpfc_topk(const float *values, int64_t rows, int64_t len, const float *gate,
                  float gate_min, int32_t top, float *out_val, int64_t *out_idx, void *stream);

/*
 * Periodogram post-processing, per row of `len` scores (a curve's box-SNR or
 * network periodogram over its trial periods): SDE (Eq. 3) = (max - mean) /
 * sd over the non-NaN scores (sd with ddof 0; 0 when sd = 0); peaks (Sec. 4.2:
 * the best peak among those higher than 3 sigma and wider than 3 points) =
 * maximal runs of consecutive scores > mean + nsigma * sd (a NaN ends a run)
 * longer than min_width, valued by their maximum (index: its first
 * position), ordered by value descending then index ascending; n_peaks counts
 * them all and the first max_peaks (1..GPFC_MAX_PEAKS) are returned (value
 * -inf, index -1, width 0 where missing). With periods f64[len] (may be NULL)
 * peak_harmonic holds 1 for the best peak, h (2, 3) for a peak at h times its
 * period and -h at 1/h of it (within 1e-3 relative), else 0. Outputs: sde,
 * mean, sd f32[rows]; n_peaks i32[rows]; peak_val f32, peak_idx i64,
 * peak_width i32, peak_harmonic i32, each [rows][max_peaks]. Device pointers.
 */
#define GPFC_MAX_PEAKS 8
int32_t gpfc_periodogram_peaks(const float *values, int64_t rows, int64_t len,
                               const double *periods, float nsigma, int32_t min_width,
                               int32_t max_peaks, float *sde, float *mean, float *sd,
                               int32_t *n_peaks, float *peak_val, int64_t *peak_idx,
                               int32_t *peak_width, int32_t *peak_harmonic, void *stream);

/* ------------------------------------------------------------------------
 * Survey: many curves of uneven length, each folded and scored at the same
 * K trial periods, and each fold scored by the network (the paper searches
 * a catalogue curve by curve, Sec. 3.3 and Sec. 4; here the curves share one
 * persistent launch per chunk). Setup (synchronous, allocates):
 * sample_offsets_host[n_curves + 1] (HOST, from 0) cut the concatenated
 * t / flux into curves; every curve uses periods[0..k). Curves are taken in
 * chunks of max(1, chunk_folds / k) consecutive curves; a chunk's work items
 * (a curve and 64 of its periods) run longest curve first in one persistent
 * launch, which writes the chunk's bfloat16 normalised folds to a workspace
 * of chunk_folds (at least k) x 256 values; the network then scores them.
 * chunk_folds = 0: no network, all curves in one launch, no workspace.
 * A later gpfc_survey_setup or gpfc_batch_setup replaces it.
 * ------------------------------------------------------------------------ */
typedef struct gpfc_survey_out {
    float *snr;              /* [n_curves][k] box-SNR, as gpfc_score */
    int32_t *start;          /* [n_curves][k] */
    int32_t *width;          /* [n_curves][k] */
    float *depth;            /* [n_curves][k] */
    float *logits;           /* [n_curves][k] network logits; NULL: no network */
    int32_t cnn_fp8;         /* 1: FP8 E4M3 inference (calibrated bf16 network) */
    int32_t top;             /* 0..64 best entries per curve; 0: no reduction */
    float *box_val;          /* [n_curves][top] best box-SNRs and their period indices */
    int64_t *box_idx;
    float *cnn_val;          /* [n_curves][top] best logits (needs logits), or NULL */
    int64_t *cnn_idx;
    float judge_snr;         /* the best logits among periods with snr >= judge_snr */
    float *judged_val;       /* [n_curves][top], or NULL */
    int64_t *judged_idx;
} gpfc_survey_out;

int32_t gpfc_survey_setup(gpfc_plan *plan, const int64_t *sample_offsets_host, int32_t n_curves,
                          int64_t k, int64_t chunk_folds);

/*
 * Run the survey: per-curve statistics and packing, then per chunk the
 * persistent fold + box-SNR (+ normalised folds) launch and, with a network
 * (cnn not NULL, nbins 256, out->logits not NULL), its forward pass over the
 * chunk's folds in batches of at most its max_batch; then the per-curve
 * reductions of out->top. t f64[total samples], flux f32[...], periods
 * f64[k]. GPFC_EINVAL for a plan without a survey setup, missing outputs, a
 * network without a workspace or an uncalibrated FP8 request.
 */
int32_t gpfc_survey_run(gpfc_plan *plan, gpfc_cnn *cnn, const double *t, const float *flux,
                        const double *periods, int32_t nbins, const gpfc_survey_out *out,
                        void *stream);

/*
 * Record gpfc_survey_run's whole launch sequence for these buffers into the
 * plan's HIP graph (kernel nodes only; replay with gpfc_batch_replay). The
 * graph converts the network's FP32 master weights to its working copies
 * itself, so each replay uses the weights current at that time (and, for
 * FP8, the current calibration). `stream` must be a created stream, not the
 * null stream.
 */
int32_t gpfc_survey_capture(gpfc_plan *plan, gpfc_cnn *cnn, const double *t, const float *flux,
                            const double *periods, int32_t nbins, const gpfc_survey_out *out,
                            void *stream);

/*
 * Autotuner of the survey's shapes (the many-star batch of form 2): for every
 * chunk size chunks_host[i] (folds per chunk, >= k with a network) and every
 * network pass size nets_host[j] (inputs per network call, <= the network's
 * max_batch; n_net = 0: the max_batch alone), sets the survey up (as
 * gpfc_survey_setup with sample_offsets_host[n_curves + 1]) and times
 * gpfc_survey_run with HIP events on `stream` (one warm-up run, one timed
 * run, scratch outputs); keeps the fastest pair: the plan is left set up with
 * that chunk size and later survey runs call the network with that pass size.
 * A cache file (cache_path, else the plan's tune cache; NULL: none) holds
 * lines "<device> survey <curves> <samples> <k> <nbins> <chunk> <net batch>";
 * a cached shape is taken without timing, a new one appended. cnn NULL tunes
 * nothing (one launch, no network). Synchronous; allocates 20 bytes per fold
 * of scratch outputs while timing. chunk_out, net_out, ms_out: host, may be
 * NULL (ms_out -1 when the shape came from the cache).
 */
int32_t gpfc_survey_autotune(gpfc_plan *plan, gpfc_cnn *cnn, const int64_t *sample_offsets_host,
                             int32_t n_curves, const double *t, const float *flux,
                             const double *periods, int64_t k, int32_t nbins,
                             const int64_t *chunks_host, int32_t n_chunk, const int64_t *nets_host,
                             int32_t n_net, const char *cache_path, int64_t *chunk_out,
                             int64_t *net_out, float *ms_out, void *stream);

/*
 * Roofline micro-benchmarks of the running GPU (the measured counterpart of
 * the paper's breakdown of where its GPU fold spends its time, Sec. 2.4,
 * Table 1): the denominators the fold's throughput is judged against.
 *   GPFC_ROOF_LDS_U64   conflict-free 64-bit LDS integer atomics, in the
 *                       fold's histogram layout (the fold's only operation
 *                       per sample-period update): lane-ops/s
 *   GPFC_ROOF_LDS_U32   the same with 32-bit integer atomics: lane-ops/s
 *   GPFC_ROOF_LDS_F32   32-bit float LDS atomics (the FP32 study fold): lane-ops/s
 *   GPFC_ROOF_FP64_FMA  independent FP64 FMAs: flop/s (2 per FMA)
 *   GPFC_ROOF_HBM_COPY  a 1 GiB device-to-device copy: bytes read + written per s
 * Synchronous on `stream` (device `device`); allocates and frees its own
 * buffers (2 GiB for the copy). rate_out (host) gets the rate, ms_out (host,
 * may be NULL) the average launch time.
 */
#define GPFC_ROOF_LDS_U64 0
#define GPFC_ROOF_LDS_U32 1
#define GPFC_ROOF_LDS_F32 2
#define GPFC_ROOF_FP64_FMA 3
#define GPFC_ROOF_HBM_COPY 4
int32_t gpfc_roof_probe(int32_t device, int32_t kind, double *rate_out, double *ms_out,
                        void *stream);

/*
 * For callers that cannot allocate device memory (code being captured into a
 * HIP graph, tight serving loops, harnesses that forbid hipMalloc): the fused
 * fold + score of gpfc_fold_score with no plan and no allocation. The curve
 * statistics and the prepared curve go to a static device buffer the library
 * owns, GPFC_NOALLOC_BYTES on each GPU it runs on, held until the process
 * ends; the caller passes device inputs and outputs as for gpfc_fold_score.
 * Runs on the current HIP device, asynchronously on `stream`, with the
 * default box widths and one block per 64 periods. Results equal those of
 * gpfc_fold_score with the default widths, bit for bit.
 * Limits: n <= GPFC_NOALLOC_MAX_SAMPLES (GPFC_ERANGE beyond), nbins a power of
 * two in [1, 256] (GPFC_ENOTSUP otherwise), k < 2^31; argument errors are
 * returned before any HIP call. Every call on one GPU shares that GPU's
 * buffer, which keeps the last call's contents (nothing in it needs to start
 * at zero): calls that overlap on one GPU (two streams, or two host threads)
 * race and give wrong results, so serialise them. Non-finite input is
 * reported by the next gpfc_sync.
 */
#define GPFC_NOALLOC_MAX_SAMPLES 131072
#define GPFC_NOALLOC_BYTES 3146496   /* 256 + (131072 + 16) x 24 bytes, rounded up to 256 */
int32_t gpfc_fold_score_noalloc(const double *t, const float *flux, int64_t n,
                                const double *periods, int64_t k, int32_t nbins, float *snr,
                                int32_t *start, int32_t *width, float *depth, void *stream);

/*
 * Light-curve pre-processing (Sec. 2.2, Fig. 3): segments, spline continuum,
 * division, edge crop, for one time-sorted curve t f64[n], flux f32[n], with
 * optional known-transit flags transit u8[n] (nonzero: masked; may be NULL).
 *  1. A new segment starts where the time step from the previous sample
 *     exceeds gap_cadences x cadence, or where an unmasked sample's flux step
 *     from the previous unmasked sample exceeds jump_sigma standard deviations
 *     (sample std, ddof 1, of the unmasked flux): a masked transit's dip does
 *     not split its segment.
 *  2. Per segment and per knot spacing h of the list: a least-squares cubic
 *     B-spline with uniform knots (L = max(1, ceil(span / h)) spans, L + 3
 *     basis functions) fitted to the unmasked, unclipped points; points with
 *     |residual| > clip_sigma x the residual scatter (ddof 0) of the fitted
 *     points are clipped (masked points never) and the fit repeated until the
 *     clipped set repeats, at most max_fits fits (the last fit and the set it
 *     used are kept); BIC = n ln(RSS / n) + m ln n over its n fitted points and
 *     m basis functions. A spacing with fewer than 2m fitted points, or whose
 *     normal equations are singular, is not tried; the smallest BIC wins
 *     (ties: the earlier spacing).
 *  3. flux_out f64[n] = flux / continuum over each segment (0 in dropped
 *     segments).
 *  4. keep_out u8[n] = 1 for points at least `edge` points from both ends of
 *     their segment and not clipped by the chosen fit; a segment of at most
 *     2 edge points, or with no tried spacing, is dropped (all 0).
 * The kept points in time order are the stitched curve (step 5). FP64
 * arithmetic; results are deterministic. opts_host NULL takes the defaults
 * (cadence 0.020428 d, 30 cadences, 5 sigma, 3 sigma, edge 30, 10 fits,
 * spacings 0.5, 0.75, 1, 1.5, 2, 3, 5 d); otherwise every field is used as
 * given (cadence, gap, jump and clip > 0; edge >= 0; 1 <= max_fits <= 100;
 * 1 <= n_spacings <= 8 ascending spacings > 0). Synchronous (waits for
 * `stream`); uses the plan's workspace (about 34 bytes per sample per
 * spacing). Returns GPFC_ERANGE if a segment would need more than 2048 basis
 * functions at some spacing. info_host (may be NULL) receives the segment
 * count, the number of kept segments and the status bits (1: basis limit,
 * 2: a singular system was skipped).
 */
#define GPFC_DETREND_MAX_SPACINGS 8
typedef struct gpfc_detrend_opts {
    double cadence;
    double gap_cadences;
    double jump_sigma;
    double clip_sigma;
    int32_t edge;
    int32_t max_fits;
    int32_t n_spacings;
    int32_t pad;
    double spacings[GPFC_DETREND_MAX_SPACINGS];
} gpfc_detrend_opts;
typedef struct gpfc_detrend_info {
    int32_t n_segments;
    int32_t n_kept_segments;
    int32_t status;
    int32_t pad;
} gpfc_detrend_info;
int32_t gpfc_detrend(gpfc_plan *plan, const double *t, const float *flux, const uint8_t *transit,
                     int64_t n, const gpfc_detrend_opts *opts_host, double *flux_out,
                     uint8_t *keep_out, gpfc_detrend_info *info_host, void *stream);

/*
 * hipStreamSynchronize(stream); reports an asynchronous device error
 * (GPFC_EDEVICE), then GPFC_EINVAL if a curve statistics pass on the stream's
 * device has seen a non-finite t or flux since the last gpfc_sync or
 * gpfc_curve_stats (a per-device flag, which this call clears: with several
 * streams on one device, the next gpfc_sync on any of them reports it).
 */
int32_t gpfc_sync(void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GPFC_H */
