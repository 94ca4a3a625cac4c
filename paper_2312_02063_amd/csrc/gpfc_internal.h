// Internal declarations shared by the host entry points and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

struct gpfc_cnn;

namespace gpfc {

// Largest batch a network's workspace takes (defined in gpfc_cnn.hip).
int64_t cnn_max_batch(const gpfc_cnn* c);

// One packed histogram bin: the sample count in bits [46, 64) and the sum of
// (q_i + 2^27) in bits [0, 46), q_i being the sample's flux deviation in
// fixed-point units of 2^e. Both fields add as one 64-bit integer without
// carrying into each other for n < 2^18 samples, so a single integer LDS
// atomic accumulates count and flux sum exactly and in any order.
//
// A curve whose deviations need more than 27 bits of fixed-point range (for
// example zero-centred flux, whose small values carry fine ulps) is packed in
// two words per sample: q = q_hi 2^27 + q_lo, q in units of 2^e_lo, q_hi and
// q_lo each a packed word as above; bin sums then stay exact for up to 53 bits
// of range.
constexpr int kCountShift = 46;
constexpr uint64_t kSumMask = (uint64_t(1) << kCountShift) - 1;
constexpr int64_t kBias = int64_t(1) << 27;
constexpr int kLoBits = 27;        // weight of q_hi in units of q_lo
constexpr int kFineBins = 256;     // bins of the fused kernels' LDS histogram
constexpr int kPeriodsPerBlock = 64;
constexpr int kMaxWidths = 24;     // box widths a plan holds
constexpr int kFusedWidths = 16;   // box widths the fused scorer holds
constexpr int kMaxBins = 4096;     // largest nbins (general path)
constexpr int64_t kPartSamples = 262128;   // samples per packed part (< 2^18, multiple of 16)

// Device-resident curve description written by k_curve_stats.
struct CurveInfo {
    double mean;
    double sigma;
    double ref;       // multiple of 2^e
    double qscale;    // 2^e
    double tmax;      // max |t|
    double maxdev;    // max |flux - ref|
    int64_t n;
    int32_t e;        // exponent of the unit of the (high) packed word
    int32_t exact;
    int32_t finite;
    int32_t words;    // 1: one packed word per sample; 2: high and low words
    int32_t e_lo;     // exponent of the low word's unit (words == 2; e = e_lo + 27)
    int32_t pad;
};

// Prepared sample: time and packed contribution (16 bytes).
struct Rec {
    double t;
    uint64_t c;
};

// One curve of a multi-curve batch: where its prepared records and periods
// start, its per-wave slice length, its number of periods, where its rows of
// the score outputs start and where its rows of the normalised folds start.
struct BatchCurve {
    int64_t rec_off;
    int64_t per;
    int64_t p_off;
    int64_t k;
    int64_t o_off;
    int64_t z_off;
};

struct Widths {
    int32_t w[kMaxWidths];
    int32_t n;
};

// Light-curve pre-processing (gpfc_detrend.hip).
constexpr int kDetrendMaxBasis = 2048;   // spline basis functions a segment's fit may use
constexpr int kDetrendMaxSpacings = 8;
struct DetrendParams {
    double cadence, gap_cadences, jump_sigma, clip_sigma;
    int32_t edge, max_fits, n_spacings, pad;
    double spacings[kDetrendMaxSpacings];
};
struct DetrendWs {
    int32_t* seg;       // segment starts [n + 2]
    int32_t* status;    // bit 0: a segment needed more than kDetrendMaxBasis functions;
                        // bit 1: a normal-equation system was singular
    int32_t* nseg;      // segments found
    int32_t* chosen;    // spacing index chosen per segment (-1: dropped)
    double* bic;
    double* coef;
    uint8_t* clip;
    int8_t* state;
};
size_t detrend_workspace_bytes(int64_t n, int32_t ns);
DetrendWs detrend_carve(void* ws, int64_t n, int32_t ns);
hipError_t launch_detrend(const double* t, const float* flux, const uint8_t* tr, int64_t n,
                          const DetrendParams& prm, const DetrendWs& w, double* out, uint8_t* keep,
                          hipStream_t s);

// Whether a curve statistics pass on the current device has seen a
// non-finite time or flux since the last call (which clears the flag);
// synchronous.
hipError_t take_input_fault(int32_t* fault);

// Launchers (defined in gpfc_kernels.hip). Each returns the HIP error of the launch.
// `lo` is the low-word array parallel to the records (read only for
// two-word curves; the kernels decide from the device-side CurveInfo).
hipError_t launch_curve_stats(const double* t, const float* flux, int64_t n, CurveInfo* info,
                              hipStream_t s);
// Records the prepared curve of n samples occupies (padding included).
int64_t prepared_len(int64_t n);
// Records per wave slice of a prepared curve of n samples.
int64_t slice_len(int64_t n);
hipError_t launch_pack(const double* t, const float* flux, int64_t n, const CurveInfo* info,
                       Rec* rec, uint64_t* lo, hipStream_t s);
hipError_t launch_fold(const Rec* rec, const uint64_t* lo, int64_t n, const double* periods,
                       int64_t k, int32_t nbins, const CurveInfo* info, double* sums,
                       int32_t* counts, double* means, hipStream_t s);
hipError_t launch_fold_score(const Rec* rec, const uint64_t* lo, int64_t n,
                             const double* periods, int64_t k, int32_t nbins,
                             const CurveInfo* info, const Widths& widths, float* snr,
                             int32_t* start, int32_t* width, float* depth, uint16_t* zfold,
                             hipStream_t s);
// Fold + score with the samples of each 64-period tile split over `split`
// blocks merged through gh (tiles x 2 halves x 256 x 64 u64, zero on entry
// and on exit) and arrivals (tiles x 2 int32, zero on entry and on exit).
hipError_t launch_fold_score_split(const Rec* rec, const uint64_t* lo, int64_t n,
                                   const double* periods, int64_t k, int32_t nbins,
                                   const CurveInfo* info, const Widths& widths, int32_t split,
                                   unsigned long long* gh, int32_t* arrivals, float* snr,
                                   int32_t* start, int32_t* width, float* depth, uint16_t* zfold,
                                   hipStream_t s);
// The two-tier equal-count fold: means f64[k][nbins] and/or bf16 z-scores.
hipError_t launch_fold_eqcount(const Rec* rec, const uint64_t* lo, int64_t n,
                               const double* periods, int64_t k, int32_t nbins,
                               const CurveInfo* info, double* means, uint16_t* zfold,
                               hipStream_t s);
hipError_t launch_batch_prepare(const double* t, const float* flux, const int64_t* soff,
                                const int64_t* roff, int32_t n_curves, int64_t max_records,
                                CurveInfo* infos, Rec* rec, uint64_t* lo, hipStream_t s);
hipError_t launch_batch_fold_score(const Rec* rec, const uint64_t* lo, const BatchCurve* curves,
                                   const int2* items, int32_t n_items, int32_t* counter,
                                   const CurveInfo* infos, const double* periods, int32_t nbins,
                                   const Widths& widths, int32_t grid, float* snr, int32_t* start,
                                   int32_t* width, float* depth, uint16_t* zfold, hipStream_t s);
hipError_t launch_fold_f32(const Rec* rec, const uint64_t* lo, int64_t n, const double* periods,
                           int64_t k, int32_t nbins, int32_t compensated, const CurveInfo* info,
                           double* sums, int32_t* counts, double* means, hipStream_t s);
hipError_t launch_score(const double* sums, const int32_t* counts, int64_t k, int32_t nbins,
                        double sigma, const Widths& widths, float* snr, int32_t* start,
                        int32_t* width, float* depth, hipStream_t s);

// General path (any n, nbins up to 4096): integer histograms of a block of
// k periods accumulated part by part (parts of fewer than 2^18 samples), in
// global memory: cnt u32 [k][nbins], shi / slo i64 [k][nbins] (sums of the
// high / low fixed-point words).
// Fold records [r0, r1) (r1 - r0 <= kPartSamples) into them: first != 0
// overwrites, else adds. The low-word pass (use_lo) does nothing for a
// one-word curve.
hipError_t launch_fold_wide(const Rec* rec, const uint64_t* lo, int64_t r0, int64_t r1,
                            const double* periods, int64_t k, int32_t nbins,
                            const CurveInfo* info, int32_t use_lo, int32_t first, uint32_t* cnt,
                            int64_t* shi, int64_t* slo, hipStream_t s);
// Sums f64 = cnt ref + shi 2^e + slo 2^e_lo (0 for an invalid period),
// counts i32 and means f64 (NaN when empty; may be NULL) of those histograms.
hipError_t launch_wide_finish(const uint32_t* cnt, const int64_t* shi, const int64_t* slo,
                              const double* periods, int64_t k, int32_t nbins,
                              const CurveInfo* info, double* sums, int32_t* counts, double* means,
                              hipStream_t s);
// Box-SNR of materialised folds at any nbins <= 4096 and up to kMaxWidths
// widths (FP64 prefix sums, FP32 box scan, winner in FP64).
hipError_t launch_score_wide(const double* sums, const int32_t* counts, int64_t k, int32_t nbins,
                             double sigma, const double* sigma_dev, const Widths& widths,
                             float* snr, int32_t* start, int32_t* width, float* depth,
                             hipStream_t s);
// bf16 z-scored folds (the network input) of materialised folds.
hipError_t launch_zfold_rows(const double* sums, const int32_t* counts, int64_t k, int32_t nbins,
                             uint16_t* zfold, hipStream_t s);
// Best `top` (<= 64) entries of each of `rows` rows of `len` scores (value
// descending, index ascending; NaN and entries with gate < gate_min skipped).
hipError_t launch_topk(const float* values, int64_t rows, int64_t len, const float* gate,
                       float gate_min, int32_t top, float* out_val, int64_t* out_idx, hipStream_t s);
// SDE, mean, sd, peak count and the best max_peaks (<= 8) peaks of each row.
hipError_t launch_periodogram(const float* values, int64_t rows, int64_t len, const double* periods,
                              float nsigma, int32_t min_width, int32_t max_peaks, float* sde,
                              float* mean, float* sd, int32_t* n_peaks, float* pval, int64_t* pidx,
                              int32_t* pwidth, int32_t* pharm, hipStream_t s);
hipError_t launch_fold_naive(const double* t, const float* flux, int64_t n,
                             const double* periods, int64_t k, int32_t nbins, double* sums,
                             int32_t* counts, hipStream_t s);

}  // namespace gpfc
