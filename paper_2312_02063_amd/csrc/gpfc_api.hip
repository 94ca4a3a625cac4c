// Host side of the C ABI declared in include/gpfc.h: argument checks (before
// any HIP call), plans and their device workspace, error reporting.
#include <math.h>
#include <stddef.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/gpfc.h"
#include "gpfc_internal.h"

using gpfc::CurveInfo;
using gpfc::Widths;

// Curves [c0, c1) of a survey and their work items [i0, i1).
struct SurveyChunk {
    int32_t c0, c1;
    int32_t i0, i1;
};

struct gpfc_plan {
    int32_t device = 0;
    gpfc::Rec* rec = nullptr;     // prepared curve: times and packed contributions
    uint64_t* lo = nullptr;       // low packed words of a two-word curve (parallel to rec)
    int64_t cap = 0;              // records rec (and lo) can hold
    CurveInfo* info = nullptr;    // device-resident curve description
    int64_t n = -1;               // samples of the prepared curve (-1: none)
    int32_t widths[GPFC_MAX_WIDTHS];
    int32_t nw = 0;               // 0: default set
    int32_t n_cu = 0;             // compute units (persistent grid size)
    // multi-curve batch (gpfc_batch_setup)
    int32_t b_curves = -1;
    int64_t b_samples = 0, b_periods = 0, b_records = 0, b_max_records = 0;
    int32_t b_items = 0;
    void* b_dev = nullptr;        // one allocation: offsets, curves, items, counter, infos, records
    int64_t* b_soff = nullptr;
    int64_t* b_roff = nullptr;
    gpfc::BatchCurve* b_curve = nullptr;
    int2* b_item = nullptr;
    int32_t* b_counter = nullptr;
    CurveInfo* b_info = nullptr;
    gpfc::Rec* b_rec = nullptr;
    uint64_t* b_lo = nullptr;
    // survey (gpfc_survey_setup): shared period grid, curves in chunks
    bool b_survey = false;
    int64_t s_k = 0;                   // periods per curve
    uint16_t* s_zbuf = nullptr;        // normalised folds of one chunk (inside b_dev)
    uint16_t* s_zbuf2 = nullptr;       // a second chunk buffer (several chunks: double buffering)
    int64_t s_zfolds = 0;              // folds s_zbuf holds (0: no workspace)
    hipStream_t s_net = nullptr;       // the network's stream in a pipelined survey
    int64_t s_net_batch = 0;           // inputs per network call (0: the network's max_batch)
    hipEvent_t s_ev[4] = {};           // fold done / network done, per chunk buffer
    std::vector<SurveyChunk> s_chunks;
    // sample split of the single-curve fold + score (k_fold_score_split)
    int32_t split = 0;                 // 0: automatic
    int64_t tuned_n = -1, tuned_k = -1;
    int32_t tuned_nbins = 0, tuned_split = 1;
    unsigned long long* split_gh = nullptr;   // n_cu tiles x 256 x 64, zero between launches
    int32_t* split_arrivals = nullptr;        // n_cu counters, zero between launches
    char device_name[64] = "";
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    // general path (nbins > 256 or n > GPFC_MAX_PACKED): per-chunk integer
    // histograms and materialised folds
    void* w_buf = nullptr;
    size_t w_cap = 0;
    int64_t w_limit = int64_t(1) << 30;       // bytes a chunk's workspace may take
    char tune_cache[512] = "";                // default autotuner cache path ("" none)
    // pre-processing (gpfc_detrend)
    void* d_buf = nullptr;
    size_t d_cap = 0;
};

namespace {

thread_local char g_last_error[256] = "";

int32_t device_error(hipError_t e, const char* what) {
    snprintf(g_last_error, sizeof(g_last_error), "%s: %s", what, hipGetErrorString(e));
    return GPFC_EDEVICE;
}

bool pow2_in_range(int32_t nbins) {
    return nbins >= 1 && nbins <= GPFC_MAX_NBINS && (nbins & (nbins - 1)) == 0;
}

// The fused kernels take nbins <= 256 and curves of at most GPFC_MAX_PACKED samples.
bool fused_shape(int64_t n, int32_t nbins) {
    return nbins <= gpfc::kFineBins && n <= GPFC_MAX_PACKED;
}

// Distinct integers nearest sqrt(2)^j in [1, max(1, nbins/2)], ascending.
Widths default_widths(int32_t nbins) {
    Widths w{};
    int32_t last = 0;
    const int32_t wmax = nbins / 2 > 0 ? nbins / 2 : 1;
    double v = 1.0;
    for (int j = 0; j < 64 && w.n < gpfc::kMaxWidths; ++j) {
        const int32_t r = (int32_t)floor(v + 0.5);
        if (r > wmax) break;
        if (r != last) w.w[w.n++] = r;
        last = r;
        v *= 1.4142135623730951;
    }
    return w;
}

// The plan's widths that fit nbins (w < nbins), in order.
Widths plan_widths(const gpfc_plan* p, int32_t nbins) {
    if (p->nw == 0) return default_widths(nbins);
    Widths w{};
    for (int i = 0; i < p->nw; ++i)
        if (p->widths[i] < nbins) w.w[w.n++] = p->widths[i];
    return w;
}

// The fused scorer holds kFusedWidths widths; more go to the general scorer.
bool fused_widths(const gpfc_plan* p, int32_t nbins) {
    return plan_widths(p, nbins).n <= gpfc::kFusedWidths;
}

int32_t check_fold_args(const gpfc_plan* p, const void* t, const void* flux, int64_t n,
                        const void* periods, int64_t k, int32_t nbins) {
    if (!p) return GPFC_EINVAL;
    if (n < 0 || k < 0) return GPFC_EINVAL;
    if (n > 0 && (!t || !flux)) return GPFC_EINVAL;
    if (k > 0 && !periods) return GPFC_EINVAL;
    if (nbins < 1) return GPFC_EINVAL;
    if (!pow2_in_range(nbins)) return GPFC_ENOTSUP;
    if (n > GPFC_MAX_SAMPLES) return GPFC_ERANGE;
    if (k > 0x7fffffffLL) return GPFC_ERANGE;
    return GPFC_OK;
}

// Make the workspace hold n samples, then run the curve statistics and the
// packing kernels on `s`.
int32_t prepare_curve(gpfc_plan* p, const double* t, const float* flux, int64_t n, hipStream_t s) {
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return device_error(e, "hipSetDevice");
    if (!p->info) {
        e = hipMalloc(&p->info, sizeof(CurveInfo));
        if (e != hipSuccess) return e == hipErrorOutOfMemory ? GPFC_ENOMEM : device_error(e, "hipMalloc");
    }
    const int64_t need = gpfc::prepared_len(n);
    if (need > p->cap) {
        const int64_t want = need < 8192 ? 8192 : need;
        gpfc::Rec* buf = nullptr;
        uint64_t* lbuf = nullptr;
        e = hipMalloc(&buf, (size_t)want * sizeof(gpfc::Rec));
        if (e == hipSuccess) e = hipMalloc(&lbuf, (size_t)want * sizeof(uint64_t));
        if (e != hipSuccess) {
            if (buf) (void)hipFree(buf);
            return e == hipErrorOutOfMemory ? GPFC_ENOMEM : device_error(e, "hipMalloc");
        }
        if (p->rec) {
            (void)hipDeviceSynchronize();
            (void)hipFree(p->rec);
            (void)hipFree(p->lo);
        }
        p->rec = buf;
        p->lo = lbuf;
        p->cap = want;
    }
    e = gpfc::launch_curve_stats(t, flux, n, p->info, s);
    if (e != hipSuccess) return device_error(e, "k_curve_stats launch");
    e = gpfc::launch_pack(t, flux, n, p->info, p->rec, p->lo, s);
    if (e != hipSuccess) return device_error(e, "k_pack launch");
    p->n = n;
    return GPFC_OK;
}

int32_t check_prepared(const gpfc_plan* p, const void* periods, int64_t k, int32_t nbins) {
    if (!p || p->n < 0 || k < 0 || (k > 0 && !periods) || nbins < 1) return GPFC_EINVAL;
    if (!pow2_in_range(nbins)) return GPFC_ENOTSUP;
    if (k > 0x7fffffffLL) return GPFC_ERANGE;
    return GPFC_OK;
}

// Device address of the prepared curve's sigma.
const double* sigma_dev(const gpfc_plan* p) {
    return (const double*)((const char*)p->info + offsetof(CurveInfo, sigma));
}

// Make the general path's workspace hold `bytes`.
int32_t wide_reserve(gpfc_plan* p, size_t bytes) {
    if (bytes <= p->w_cap) return GPFC_OK;
    void* buf = nullptr;
    hipError_t e = hipMalloc(&buf, bytes);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? GPFC_ENOMEM : device_error(e, "hipMalloc");
    if (p->w_buf) {
        (void)hipDeviceSynchronize();
        (void)hipFree(p->w_buf);
    }
    p->w_buf = buf;
    p->w_cap = bytes;
    return GPFC_OK;
}

// General path of the prepared curve (any n, nbins up to 4096): per chunk of
// periods, every part of fewer than 2^18 samples is folded into integer
// histograms (high words, then low words of a two-word curve), which become
// sums / counts / means, then box-SNR and normalised folds. Materialised
// outputs (sums, counts, means) go to the caller's buffers when given,
// otherwise to the workspace; snr != NULL scores, zfold != NULL normalises.
int32_t wide_run(gpfc_plan* p, const double* periods, int64_t k, int32_t nbins, double* sums,
                 int32_t* counts, double* means, float* snr, int32_t* start, int32_t* width,
                 float* depth, uint16_t* zfold, hipStream_t s) {
    if (k == 0) return GPFC_OK;
    const bool own = sums == nullptr;   // materialise into the workspace
    const int64_t per_period = (int64_t)nbins * (4 + 8 + 8 + (own ? 8 + 4 : 0));
    int64_t kc = std::max<int64_t>(64, p->w_limit / per_period) / 64 * 64;
    kc = std::min<int64_t>(kc, (k + 63) / 64 * 64);
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t b_cnt = al((size_t)kc * nbins * 4), b_s = al((size_t)kc * nbins * 8);
    const size_t total = b_cnt + 2 * b_s + (own ? b_s + b_cnt : 0);
    int32_t rc = wide_reserve(p, total);
    if (rc != GPFC_OK) return rc;
    char* base = (char*)p->w_buf;
    uint32_t* cnt = (uint32_t*)base;
    int64_t* shi = (int64_t*)(base + b_cnt);
    int64_t* slo = (int64_t*)(base + b_cnt + b_s);
    double* wsums = own ? (double*)(base + b_cnt + 2 * b_s) : nullptr;
    int32_t* wcounts = own ? (int32_t*)(base + b_cnt + 3 * b_s) : nullptr;
    const int64_t recs = gpfc::prepared_len(p->n);
    const Widths W = plan_widths(p, nbins);
    for (int64_t c0 = 0; c0 < k; c0 += kc) {
        const int64_t kn = std::min(kc, k - c0);
        const double* per = periods + c0;
        hipError_t e = hipSuccess;
        for (int64_t r0 = 0; r0 < recs && e == hipSuccess; r0 += gpfc::kPartSamples) {
            const int64_t r1 = std::min(recs, r0 + gpfc::kPartSamples);
            for (int use_lo = 0; use_lo < 2 && e == hipSuccess; ++use_lo)
                e = gpfc::launch_fold_wide(p->rec, p->lo, r0, r1, per, kn, nbins, p->info, use_lo,
                                           r0 == 0, cnt, shi, slo, s);
        }
        if (e != hipSuccess) return device_error(e, "k_fold_wide launch");
        double* os = own ? wsums : sums + c0 * nbins;
        int32_t* oc = own ? wcounts : counts + c0 * nbins;
        double* om = (own || !means) ? nullptr : means + c0 * nbins;
        e = gpfc::launch_wide_finish(cnt, shi, slo, per, kn, nbins, p->info, os, oc, om, s);
        if (e == hipSuccess && snr)
            e = gpfc::launch_score_wide(os, oc, kn, nbins, 0.0, sigma_dev(p), W, snr + c0,
                                        start + c0, width + c0, depth + c0, s);
        if (e == hipSuccess && zfold)
            e = gpfc::launch_zfold_rows(os, oc, kn, nbins, zfold + c0 * nbins, s);
        if (e != hipSuccess) return device_error(e, "general path launch");
    }
    return GPFC_OK;
}

// Device buffer of gpfc_fold_score_noalloc: CurveInfo (padded to 256 bytes),
// then the prepared records and low words of up to GPFC_NOALLOC_MAX_SAMPLES
// samples (prepared_len pads a curve to whole 256-sample blocks plus 16).
constexpr size_t kNoAllocInfoBytes = 256;
constexpr int64_t kNoAllocRecs = (GPFC_NOALLOC_MAX_SAMPLES + 255) / 256 * 256 + 16;
static_assert(sizeof(CurveInfo) <= kNoAllocInfoBytes, "CurveInfo must fit its slot");
static_assert(kNoAllocInfoBytes + kNoAllocRecs * (sizeof(gpfc::Rec) + sizeof(uint64_t)) <=
                  (size_t)GPFC_NOALLOC_BYTES,
              "GPFC_NOALLOC_BYTES must hold the statistics and the records");

constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mu;
char* g_noalloc_ptr[kNoAllocDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[GPFC_NOALLOC_BYTES];

namespace {

// Device address of `scratch` on the current device, looked up once per device
// (with that device current) and kept.
int32_t noalloc_base(char** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return device_error(e, "hipGetDevice");
    if (dev < 0 || dev >= kNoAllocDevices) return GPFC_EINVAL;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return device_error(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return device_error(hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        g_noalloc_ptr[dev] = static_cast<char*>(ptr);
    }
    *out = g_noalloc_ptr[dev];
    return GPFC_OK;
}

}  // namespace

extern "C" {

int32_t gpfc_version(void) { return 100; }

const char* gpfc_strerror(int32_t code) {
    switch (code) {
        case GPFC_OK: return "ok";
        case GPFC_EINVAL: return "invalid argument";
        case GPFC_ENOTSUP: return "nbins not supported (a power of two in [1, 4096]; [1, 256] or [16, 256] for some calls)";
        case GPFC_ERANGE: return "size out of range (too many samples or periods for the call)";
        case GPFC_ENOMEM: return "device memory allocation failed";
        case GPFC_EDEVICE: return "HIP device error";
        case GPFC_EIO: return "network file could not be written or read, or is not a network file";
        default: return "unknown error";
    }
}

const char* gpfc_last_error(void) { return g_last_error; }

int32_t gpfc_plan_create(gpfc_plan** out, int32_t device) {
    if (!out) return GPFC_EINVAL;
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return device_error(e, "hipGetDeviceCount");
    if (device < 0 || device >= count) return GPFC_EINVAL;
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return device_error(e, "hipGetDeviceProperties");
    gpfc_plan* p = new (std::nothrow) gpfc_plan();
    if (!p) return GPFC_ENOMEM;
    p->device = device;
    p->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 1;
    snprintf(p->device_name, sizeof(p->device_name), "%s", prop.gcnArchName);
    for (char* c = p->device_name; *c; ++c)
        if (*c == ' ' || *c == ':') *c = '_';
    e = hipSetDevice(device);
    // two 32-period halves per tile (a two-word curve merges them separately)
    const size_t gh_bytes = (size_t)2 * p->n_cu * gpfc::kFineBins * 64 * sizeof(unsigned long long);
    if (e == hipSuccess) e = hipMalloc(&p->split_gh, gh_bytes);
    if (e == hipSuccess) e = hipMalloc(&p->split_arrivals, sizeof(int32_t) * 2 * p->n_cu);
    if (e == hipSuccess) e = hipMemset(p->split_gh, 0, gh_bytes);
    if (e == hipSuccess) e = hipMemset(p->split_arrivals, 0, sizeof(int32_t) * 2 * p->n_cu);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        if (p->split_gh) (void)hipFree(p->split_gh);
        if (p->split_arrivals) (void)hipFree(p->split_arrivals);
        delete p;
        return e == hipErrorOutOfMemory ? GPFC_ENOMEM : device_error(e, "plan workspace");
    }
    *out = p;
    return GPFC_OK;
}

int32_t gpfc_plan_create_opts(gpfc_plan** out, const gpfc_plan_opts* o) {
    if (!out) return GPFC_EINVAL;
    *out = nullptr;
    if (!o || o->nw < 0 || o->nw > GPFC_MAX_WIDTHS || o->split < 0 || o->split > GPFC_MAX_SPLIT ||
        o->workspace_bytes < 0)
        return GPFC_EINVAL;
    if (o->tune_cache && strlen(o->tune_cache) >= sizeof(((gpfc_plan*)nullptr)->tune_cache))
        return GPFC_EINVAL;
    for (int i = 0; i < o->nw; ++i) {
        if (o->widths[i] < 1 || o->widths[i] >= GPFC_MAX_NBINS) return GPFC_EINVAL;
        if (i > 0 && o->widths[i] <= o->widths[i - 1]) return GPFC_EINVAL;
    }
    gpfc_plan* p = nullptr;
    const int32_t rc = gpfc_plan_create(&p, o->device);
    if (rc != GPFC_OK) return rc;
    for (int i = 0; i < o->nw; ++i) p->widths[i] = o->widths[i];
    p->nw = o->nw;
    p->split = o->split;
    if (o->tune_cache) snprintf(p->tune_cache, sizeof(p->tune_cache), "%s", o->tune_cache);
    if (o->workspace_bytes > 0) p->w_limit = o->workspace_bytes;
    *out = p;
    return GPFC_OK;
}

int32_t gpfc_plan_destroy(gpfc_plan* p) {
    if (!p) return GPFC_OK;
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    if (p->rec) (void)hipFree(p->rec);
    if (p->lo) (void)hipFree(p->lo);
    if (p->info) (void)hipFree(p->info);
    if (p->w_buf) (void)hipFree(p->w_buf);
    if (p->d_buf) (void)hipFree(p->d_buf);
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->b_dev) (void)hipFree(p->b_dev);
    if (p->split_gh) (void)hipFree(p->split_gh);
    if (p->split_arrivals) (void)hipFree(p->split_arrivals);
    for (hipEvent_t& ev : p->s_ev)
        if (ev) (void)hipEventDestroy(ev);
    if (p->s_net) (void)hipStreamDestroy(p->s_net);
    delete p;
    return GPFC_OK;
}

int32_t gpfc_plan_set_widths(gpfc_plan* p, const int32_t* widths, int32_t nw) {
    if (!p || nw < 0 || nw > GPFC_MAX_WIDTHS || (nw > 0 && !widths)) return GPFC_EINVAL;
    for (int i = 0; i < nw; ++i) {
        if (widths[i] < 1 || widths[i] >= GPFC_MAX_NBINS) return GPFC_EINVAL;
        if (i > 0 && widths[i] <= widths[i - 1]) return GPFC_EINVAL;
    }
    for (int i = 0; i < nw; ++i) p->widths[i] = widths[i];
    p->nw = nw;
    return GPFC_OK;
}

int32_t gpfc_curve_stats(gpfc_plan* p, const double* t, const float* flux, int64_t n,
                         gpfc_curve* out, void* stream) {
    int32_t rc = check_fold_args(p, t, flux, n, (const void*)1, 0, 1);
    if (rc != GPFC_OK) return rc;
    if (!out) return GPFC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    rc = prepare_curve(p, t, flux, n, s);
    if (rc != GPFC_OK) return rc;
    CurveInfo ci;
    hipError_t e = hipMemcpyAsync(&ci, p->info, sizeof(ci), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_error(e, "curve stats copy");
    out->mean = ci.mean;
    out->sigma = ci.sigma;
    out->ref = ci.ref;
    out->qscale = ci.qscale;
    out->tmax = ci.tmax;
    out->maxdev = ci.maxdev;
    out->n = ci.n;
    out->exact = ci.exact;
    out->finite = ci.finite;
    out->words = ci.words;
    if (!ci.finite) {
        int32_t fault = 0;
        (void)gpfc::take_input_fault(&fault);   // reported here, not again at gpfc_sync
        return GPFC_EINVAL;
    }
    return GPFC_OK;
}

int32_t gpfc_prepare(gpfc_plan* p, const double* t, const float* flux, int64_t n, void* stream) {
    int32_t rc = check_fold_args(p, t, flux, n, (const void*)1, 0, 1);
    if (rc != GPFC_OK) return rc;
    return prepare_curve(p, t, flux, n, (hipStream_t)stream);
}

int32_t gpfc_fold_prepared(gpfc_plan* p, const double* periods, int64_t k, int32_t nbins,
                           double* sums, int32_t* counts, double* means, void* stream) {
    int32_t rc = check_prepared(p, periods, k, nbins);
    if (rc != GPFC_OK) return rc;
    if (k > 0 && (!sums || !counts)) return GPFC_EINVAL;
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return device_error(e, "hipSetDevice");
    if (!fused_shape(p->n, nbins))
        return wide_run(p, periods, k, nbins, sums, counts, means, nullptr, nullptr, nullptr,
                        nullptr, nullptr, (hipStream_t)stream);
    e = gpfc::launch_fold(p->rec, p->lo, p->n, periods, k, nbins, p->info, sums, counts, means,
                          (hipStream_t)stream);
    if (e != hipSuccess) return device_error(e, "k_fold launch");
    return GPFC_OK;
}

// Largest power of two <= x (x >= 1).
static int32_t pow2_floor(int64_t x) {
    int32_t r = 1;
    while ((int64_t)r * 2 <= x) r *= 2;
    return r;
}

// Sample split for a fold + score of the prepared curve (n samples) at k
// periods: the forced value, else the autotuned one for this shape, else
// enough blocks per 64-period tile to give every compute unit one block,
// keeping at least 256 records per wave per part. Measured on MI355X: a
// 4,000-sample curve (256 records per wave) is fastest unsplit even at 16
// tiles (35 us; split 2 takes 47 us), a 65,000-sample one at 16 tiles with 8
// parts (119 us against 293 us unsplit), a 20,000-sample one with 4.
static int32_t resolve_split(const gpfc_plan* p, int64_t n, int64_t k, int32_t nbins) {
    const int64_t tiles = (k + 63) / 64;
    if (tiles == 0 || tiles > p->n_cu) return 1;
    int32_t sp;
    if (p->split > 0) sp = p->split;
    else if (p->tuned_n == n && p->tuned_k == k && p->tuned_nbins == nbins) sp = p->tuned_split;
    else {
        const int64_t per = gpfc::slice_len(n);
        sp = pow2_floor(std::max<int64_t>(1, std::min<int64_t>(p->n_cu / tiles, per / 256)));
    }
    return std::max(1, std::min(sp, GPFC_MAX_SPLIT));
}

static hipError_t enqueue_fold_score(gpfc_plan* p, int64_t n, const double* periods, int64_t k,
                                     int32_t nbins, float* snr, int32_t* start, int32_t* width,
                                     float* depth, uint16_t* zfold, int32_t split, hipStream_t s) {
    if (split <= 1)
        return gpfc::launch_fold_score(p->rec, p->lo, n, periods, k, nbins, p->info,
                                       plan_widths(p, nbins), snr, start, width, depth, zfold, s);
    return gpfc::launch_fold_score_split(p->rec, p->lo, n, periods, k, nbins, p->info,
                                         plan_widths(p, nbins), split, p->split_gh,
                                         p->split_arrivals, snr, start, width, depth, zfold, s);
}

// Fold + score of the prepared curve: the fused kernels, or the general path
// for shapes they do not take.
static int32_t run_fold_score(gpfc_plan* p, const double* periods, int64_t k, int32_t nbins,
                              float* snr, int32_t* start, int32_t* width, float* depth,
                              uint16_t* zfold, hipStream_t s) {
    if (!fused_shape(p->n, nbins) || !fused_widths(p, nbins))
        return wide_run(p, periods, k, nbins, nullptr, nullptr, nullptr, snr, start, width, depth,
                        zfold, s);
    const hipError_t e = enqueue_fold_score(p, p->n, periods, k, nbins, snr, start, width, depth,
                                            zfold, resolve_split(p, p->n, k, nbins), s);
    return e == hipSuccess ? GPFC_OK : device_error(e, "k_fold_score launch");
}

int32_t gpfc_fold_score_prepared(gpfc_plan* p, const double* periods, int64_t k, int32_t nbins,
                                 float* snr, int32_t* start, int32_t* width, float* depth,
                                 uint16_t* zfold, void* stream) {
    int32_t rc = check_prepared(p, periods, k, nbins);
    if (rc != GPFC_OK) return rc;
    if (k > 0 && (!snr || !start || !width || !depth)) return GPFC_EINVAL;
    if (zfold && (nbins < 16 || nbins > gpfc::kFineBins)) return GPFC_ENOTSUP;
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return device_error(e, "hipSetDevice");
    return run_fold_score(p, periods, k, nbins, snr, start, width, depth, zfold,
                          (hipStream_t)stream);
}

// Cache lines: "<device> <n> <k> <nbins> <split>".
static bool cache_lookup(const char* path, const char* dev, int64_t n, int64_t k, int32_t nbins,
                         int32_t* split) {
    if (!path) return false;
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char line[512], name[64], extra[8];
    long long cn, ck;
    int cb, cs;
    bool found = false;
    while (fgets(line, sizeof(line), f))   // fold lines have exactly five fields
        if (sscanf(line, "%63s %lld %lld %d %d %7s", name, &cn, &ck, &cb, &cs, extra) == 5 &&
            !strcmp(name, dev) && cn == n && ck == k && cb == nbins && cs >= 1 && cs <= GPFC_MAX_SPLIT) {
            *split = cs;
            found = true;
        }
    fclose(f);
    return found;
}

int32_t gpfc_autotune(gpfc_plan* p, const double* periods, int64_t k, int32_t nbins,
                      const char* cache_path, int32_t* split_out, float* ms_out, void* stream) {
    int32_t rc = check_prepared(p, periods, k, nbins);
    if (rc != GPFC_OK) return rc;
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return device_error(e, "hipSetDevice");
    const int64_t tiles = (k + 63) / 64;
    int32_t best = 1;
    float best_ms = -1.0f;
    if (!cache_path && p->tune_cache[0]) cache_path = p->tune_cache;
    if (!fused_shape(p->n, nbins) || !fused_widths(p, nbins)) {
        // the general path has no sample split to tune
    } else if (cache_lookup(cache_path, p->device_name, p->n, k, nbins, &best)) {
        // known shape: no timing
    } else if (tiles >= 1 && tiles <= p->n_cu) {
        hipStream_t s = (hipStream_t)stream;
        void* out = nullptr;
        e = hipMalloc(&out, (size_t)k * 16);
        if (e != hipSuccess) return e == hipErrorOutOfMemory ? GPFC_ENOMEM : device_error(e, "hipMalloc");
        float* snr = (float*)out;
        int32_t* st = (int32_t*)(snr + k);
        int32_t* wd = st + k;
        float* dp = (float*)(wd + k);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        const int64_t per = gpfc::slice_len(p->n);
        for (int32_t sp = 1; e == hipSuccess && sp <= GPFC_MAX_SPLIT; sp *= 2) {
            if (sp > 1 && (tiles * sp > 4 * (int64_t)p->n_cu || per / sp < 32)) break;
            e = enqueue_fold_score(p, p->n, periods, k, nbins, snr, st, wd, dp, nullptr, sp, s);
            if (e == hipSuccess) e = hipEventRecord(e0, s);
            for (int r = 0; r < 3 && e == hipSuccess; ++r)
                e = enqueue_fold_score(p, p->n, periods, k, nbins, snr, st, wd, dp, nullptr, sp, s);
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            ms /= 3.0f;
            if (e == hipSuccess && (best_ms < 0.0f || ms < best_ms)) {
                best_ms = ms;
                best = sp;
            }
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipStreamSynchronize(s);
        (void)hipFree(out);
        if (e != hipSuccess) return device_error(e, "autotune");
        if (cache_path) {
            FILE* f = fopen(cache_path, "a");
            if (f) {
                fprintf(f, "%s %lld %lld %d %d\n", p->device_name, (long long)p->n, (long long)k,
                        nbins, best);
                fclose(f);
            }
        }
    }
    p->tuned_n = p->n;
    p->tuned_k = k;
    p->tuned_nbins = nbins;
    p->tuned_split = best;
    if (split_out) *split_out = best;
    if (ms_out) *ms_out = best_ms;
    return GPFC_OK;
}

int32_t gpfc_fold_f32_prepared(gpfc_plan* p, const double* periods, int64_t k, int32_t nbins,
                               int32_t compensated, double* sums, int32_t* counts, double* means,
                               void* stream) {
    int32_t rc = check_prepared(p, periods, k, nbins);
    if (rc != GPFC_OK) return rc;
    if (nbins > gpfc::kFineBins) return GPFC_ENOTSUP;
    if (k > 0 && (!sums || !counts)) return GPFC_EINVAL;
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return device_error(e, "hipSetDevice");
    e = gpfc::launch_fold_f32(p->rec, p->lo, p->n, periods, k, nbins, compensated, p->info, sums,
                              counts, means, (hipStream_t)stream);
    if (e != hipSuccess) return device_error(e, "k_fold_f32 launch");
    return GPFC_OK;
}

int32_t gpfc_fold(gpfc_plan* p, const double* t, const float* flux, int64_t n,
                  const double* periods, int64_t k, int32_t nbins, double* sums, int32_t* counts,
                  double* means, void* stream) {
    int32_t rc = check_fold_args(p, t, flux, n, periods, k, nbins);
    if (rc != GPFC_OK) return rc;
    if (k > 0 && (!sums || !counts)) return GPFC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    rc = prepare_curve(p, t, flux, n, s);
    if (rc != GPFC_OK) return rc;
    if (!fused_shape(n, nbins))
        return wide_run(p, periods, k, nbins, sums, counts, means, nullptr, nullptr, nullptr,
                        nullptr, nullptr, s);
    hipError_t e = gpfc::launch_fold(p->rec, p->lo, n, periods, k, nbins, p->info, sums, counts,
                                     means, s);
    if (e != hipSuccess) return device_error(e, "k_fold launch");
    return GPFC_OK;
}

int32_t gpfc_fold_eqcount_prepared(gpfc_plan* p, const double* periods, int64_t k, int32_t nbins,
                                   double* means, uint16_t* zfold, void* stream) {
    if (!p || p->n < 0 || k < 0 || (k > 0 && !periods)) return GPFC_EINVAL;
    if (nbins < 1 || nbins > gpfc::kFineBins) return GPFC_ENOTSUP;
    if (k > 0 && !means && !zfold) return GPFC_EINVAL;
    if ((k + 3) / 4 > 0x7fffffffLL || p->n > GPFC_MAX_PACKED) return GPFC_ERANGE;
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return device_error(e, "hipSetDevice");
    e = gpfc::launch_fold_eqcount(p->rec, p->lo, p->n, periods, k, nbins, p->info, means, zfold,
                                  (hipStream_t)stream);
    if (e != hipSuccess) return device_error(e, "k_fold_eqcount launch");
    return GPFC_OK;
}

int32_t gpfc_plan_set_split(gpfc_plan* p, int32_t split) {
    if (!p || split < 0 || split > GPFC_MAX_SPLIT) return GPFC_EINVAL;
    p->split = split;
    return GPFC_OK;
}

int32_t gpfc_fold_score(gpfc_plan* p, const double* t, const float* flux, int64_t n,
                        const double* periods, int64_t k, int32_t nbins, float* snr,
                        int32_t* start, int32_t* width, float* depth, void* stream) {
    int32_t rc = check_fold_args(p, t, flux, n, periods, k, nbins);
    if (rc != GPFC_OK) return rc;
    if (k > 0 && (!snr || !start || !width || !depth)) return GPFC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    rc = prepare_curve(p, t, flux, n, s);
    if (rc != GPFC_OK) return rc;
    return run_fold_score(p, periods, k, nbins, snr, start, width, depth, nullptr, s);
}

int32_t gpfc_score(gpfc_plan* p, const double* sums, const int32_t* counts, int64_t k,
                   int32_t nbins, double sigma, float* snr, int32_t* start, int32_t* width,
                   float* depth, void* stream) {
    if (!p || k < 0 || nbins < 1) return GPFC_EINVAL;
    if (!pow2_in_range(nbins)) return GPFC_ENOTSUP;
    if (k > 0 && (!sums || !counts || !snr || !start || !width || !depth)) return GPFC_EINVAL;
    if (k > 0x7fffffffLL) return GPFC_ERANGE;
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return device_error(e, "hipSetDevice");
    if (nbins > gpfc::kFineBins || !fused_widths(p, nbins))
        e = gpfc::launch_score_wide(sums, counts, k, nbins, sigma, nullptr, plan_widths(p, nbins),
                                    snr, start, width, depth, (hipStream_t)stream);
    else
        e = gpfc::launch_score(sums, counts, k, nbins, sigma, plan_widths(p, nbins), snr, start,
                               width, depth, (hipStream_t)stream);
    if (e != hipSuccess) return device_error(e, "k_score launch");
    return GPFC_OK;
}

int32_t gpfc_fold_naive(gpfc_plan* p, const double* t, const float* flux, int64_t n,
                        const double* periods, int64_t k, int32_t nbins, double* sums,
                        int32_t* counts, void* stream) {
    int32_t rc = check_fold_args(p, t, flux, n, periods, k, nbins);
    if (rc != GPFC_OK) return rc;
    if (k > 0 && (!sums || !counts)) return GPFC_EINVAL;
    if (k > 0x7fffffffLL) return GPFC_ERANGE;
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return device_error(e, "hipSetDevice");
    e = gpfc::launch_fold_naive(t, flux, n, periods, k, nbins, sums, counts, (hipStream_t)stream);
    if (e != hipSuccess) return device_error(e, "k_fold_naive launch");
    return GPFC_OK;
}

// Allocate and upload a batch: per-curve offsets, curve table, work items,
// counter, curve statistics, prepared records and `extra` bytes of workspace
// (returned in *extra_ptr). Replaces any earlier batch or survey.
static int32_t batch_upload(gpfc_plan* p, const int64_t* soff, int32_t n_curves,
                            const std::vector<int64_t>& roff,
                            const std::vector<gpfc::BatchCurve>& curves,
                            const std::vector<int2>& it, int64_t periods, size_t extra,
                            void** extra_ptr) {
    const int64_t recs = roff[n_curves];
    const int64_t items = (int64_t)it.size();
    int64_t maxr = 0;
    for (int32_t c = 0; c < n_curves; ++c) maxr = std::max<int64_t>(maxr, roff[c + 1] - roff[c]);
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return device_error(e, "hipSetDevice");
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t sz_off = al(sizeof(int64_t) * (n_curves + 1));
    const size_t sz_cur = al(sizeof(gpfc::BatchCurve) * (n_curves > 0 ? n_curves : 1));
    const size_t sz_it = al(sizeof(int2) * (items > 0 ? items : 1));
    const size_t sz_ctr = 256;
    const size_t sz_inf = al(sizeof(CurveInfo) * (n_curves > 0 ? n_curves : 1));
    const size_t sz_rec = al(sizeof(gpfc::Rec) * (recs > 0 ? recs : 1));
    const size_t sz_lo = al(sizeof(uint64_t) * (recs > 0 ? recs : 1));
    const size_t total = 2 * sz_off + sz_cur + sz_it + sz_ctr + sz_inf + sz_rec + sz_lo + al(extra);
    if (p->graph_exec) { (void)hipGraphExecDestroy(p->graph_exec); p->graph_exec = nullptr; }
    if (p->graph) { (void)hipGraphDestroy(p->graph); p->graph = nullptr; }
    if (p->b_dev) {
        (void)hipDeviceSynchronize();
        (void)hipFree(p->b_dev);
        p->b_dev = nullptr;
    }
    p->b_curves = -1;
    p->b_survey = false;
    p->s_zbuf = nullptr;
    p->s_zbuf2 = nullptr;
    p->s_zfolds = 0;
    p->s_chunks.clear();
    e = hipMalloc(&p->b_dev, total);
    if (e != hipSuccess) {
        p->b_dev = nullptr;
        return e == hipErrorOutOfMemory ? GPFC_ENOMEM : device_error(e, "hipMalloc");
    }
    char* base = (char*)p->b_dev;
    p->b_soff = (int64_t*)base; base += sz_off;
    p->b_roff = (int64_t*)base; base += sz_off;
    p->b_curve = (gpfc::BatchCurve*)base; base += sz_cur;
    p->b_item = (int2*)base; base += sz_it;
    p->b_counter = (int32_t*)base; base += sz_ctr;
    p->b_info = (CurveInfo*)base; base += sz_inf;
    p->b_rec = (gpfc::Rec*)base; base += sz_rec;
    p->b_lo = (uint64_t*)base; base += sz_lo;
    *extra_ptr = extra ? (void*)base : nullptr;
    e = hipMemcpy(p->b_soff, soff, sizeof(int64_t) * (n_curves + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->b_roff, roff.data(), sizeof(int64_t) * (n_curves + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess && n_curves > 0)
        e = hipMemcpy(p->b_curve, curves.data(), sizeof(gpfc::BatchCurve) * n_curves, hipMemcpyHostToDevice);
    if (e == hipSuccess && items > 0)
        e = hipMemcpy(p->b_item, it.data(), sizeof(int2) * items, hipMemcpyHostToDevice);
    if (e != hipSuccess) return device_error(e, "batch table upload");
    p->b_curves = n_curves;
    p->b_samples = soff[n_curves];
    p->b_periods = periods;
    p->b_records = recs;
    p->b_max_records = maxr;
    p->b_items = (int32_t)items;
    return GPFC_OK;
}

// Work items of curves [c0, c1): every block of 64 periods, longest curve first.
static void push_items(std::vector<int2>& it, const int64_t* soff, int32_t c0, int32_t c1,
                       const std::vector<gpfc::BatchCurve>& curves) {
    std::vector<int32_t> order;
    for (int32_t c = c0; c < c1; ++c) order.push_back(c);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return soff[a + 1] - soff[a] > soff[b + 1] - soff[b];
    });
    for (int32_t c : order)
        for (int64_t j = 0; j < (curves[c].k + 63) / 64; ++j) it.push_back(make_int2(c, (int)j));
}

int32_t gpfc_batch_setup(gpfc_plan* p, const int64_t* soff, const int64_t* poff, int32_t n_curves) {
    if (!p || !soff || !poff || n_curves < 0) return GPFC_EINVAL;
    if (soff[0] != 0 || poff[0] != 0) return GPFC_EINVAL;
    int64_t recs = 0, items = 0;
    std::vector<int64_t> roff(n_curves + 1);
    std::vector<gpfc::BatchCurve> curves(n_curves);
    roff[0] = 0;
    for (int32_t c = 0; c < n_curves; ++c) {
        const int64_t n = soff[c + 1] - soff[c];
        const int64_t k = poff[c + 1] - poff[c];
        if (n < 0 || k < 0) return GPFC_EINVAL;
        if (n > GPFC_MAX_PACKED) return GPFC_ERANGE;
        curves[c] = gpfc::BatchCurve{recs, gpfc::slice_len(n), poff[c], k, poff[c], poff[c]};
        recs += gpfc::prepared_len(n);
        roff[c + 1] = recs;
        items += (k + 63) / 64;
    }
    if (items > 0x7fffffffLL) return GPFC_ERANGE;
    std::vector<int2> it;
    it.reserve((size_t)items);
    push_items(it, soff, 0, n_curves, curves);
    void* unused = nullptr;
    return batch_upload(p, soff, n_curves, roff, curves, it, poff[n_curves], 0, &unused);
}

int32_t gpfc_survey_setup(gpfc_plan* p, const int64_t* soff, int32_t n_curves, int64_t k,
                          int64_t chunk_folds) {
    if (!p || !soff || n_curves < 0 || k < 0 || chunk_folds < 0) return GPFC_EINVAL;
    if (soff[0] != 0) return GPFC_EINVAL;
    const int64_t per_chunk = chunk_folds == 0 ? std::max<int32_t>(n_curves, 1)
                                               : std::max<int64_t>(1, k > 0 ? chunk_folds / k : n_curves);
    const int64_t zfolds = chunk_folds == 0 ? 0 : per_chunk * k;
    if ((int64_t)n_curves * k > (int64_t(1) << 40)) return GPFC_ERANGE;
    int64_t recs = 0, items = 0;
    std::vector<int64_t> roff(n_curves + 1);
    std::vector<gpfc::BatchCurve> curves(n_curves);
    std::vector<SurveyChunk> chunks;
    roff[0] = 0;
    for (int32_t c = 0; c < n_curves; ++c) {
        const int64_t n = soff[c + 1] - soff[c];
        if (n < 0) return GPFC_EINVAL;
        if (n > GPFC_MAX_PACKED) return GPFC_ERANGE;
        const int64_t first = c - c % per_chunk;   // first curve of this curve's chunk
        curves[c] = gpfc::BatchCurve{recs, gpfc::slice_len(n), 0, k, (int64_t)c * k, (c - first) * k};
        recs += gpfc::prepared_len(n);
        roff[c + 1] = recs;
        items += (k + 63) / 64;
    }
    if (items > 0x7fffffffLL) return GPFC_ERANGE;
    std::vector<int2> it;
    it.reserve((size_t)items);
    for (int64_t c0 = 0; c0 < n_curves; c0 += per_chunk) {
        const int32_t c1 = (int32_t)std::min<int64_t>(n_curves, c0 + per_chunk);
        const int32_t i0 = (int32_t)it.size();
        push_items(it, soff, (int32_t)c0, c1, curves);
        chunks.push_back(SurveyChunk{(int32_t)c0, c1, i0, (int32_t)it.size()});
    }
    // two chunk buffers when there are several chunks: the network of one chunk
    // runs on its own stream while the next chunk is folded into the other buffer
    const int nbuf = chunks.size() > 1 ? 2 : 1;
    const size_t zbytes = ((size_t)zfolds * gpfc::kFineBins * sizeof(uint16_t) + 255) & ~size_t(255);
    void* z = nullptr;
    int32_t rc = batch_upload(p, soff, n_curves, roff, curves, it, (int64_t)n_curves * k,
                              nbuf * zbytes, &z);
    if (rc != GPFC_OK) return rc;
    if (zfolds > 0 && nbuf == 2) {
        hipError_t e = hipSuccess;
        if (!p->s_net) e = hipStreamCreateWithFlags(&p->s_net, hipStreamNonBlocking);
        for (hipEvent_t& ev : p->s_ev)
            if (e == hipSuccess && !ev) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) return device_error(e, "survey stream setup");
    }
    p->b_survey = true;
    p->s_k = k;
    p->s_zbuf = (uint16_t*)z;
    p->s_zbuf2 = (zfolds > 0 && nbuf == 2) ? (uint16_t*)((char*)z + zbytes) : nullptr;
    p->s_zfolds = zfolds;
    p->s_chunks = chunks;
    return GPFC_OK;
}

static int32_t batch_enqueue(gpfc_plan* p, const double* t, const float* flux, const double* periods,
                             int32_t nbins, float* snr, int32_t* start, int32_t* width, float* depth,
                             uint16_t* zfold, hipStream_t s) {
    hipError_t e = gpfc::launch_batch_prepare(t, flux, p->b_soff, p->b_roff, p->b_curves,
                                              p->b_max_records, p->b_info, p->b_rec, p->b_lo, s);
    if (e != hipSuccess) return device_error(e, "batch prepare launch");
    e = gpfc::launch_batch_fold_score(p->b_rec, p->b_lo, p->b_curve, p->b_item, p->b_items, p->b_counter,
                                      p->b_info, periods, nbins, plan_widths(p, nbins), p->n_cu, snr,
                                      start, width, depth, zfold, s);
    if (e != hipSuccess) return device_error(e, "batch fold_score launch");
    return GPFC_OK;
}

static int32_t check_batch(const gpfc_plan* p, const void* t, const void* flux, const void* periods,
                           int32_t nbins, const void* snr, const void* start, const void* width,
                           const void* depth, const void* zfold) {
    if (!p || p->b_curves < 0 || p->b_survey) return GPFC_EINVAL;
    if (p->b_samples > 0 && (!t || !flux)) return GPFC_EINVAL;
    if (p->b_periods > 0 && (!periods || !snr || !start || !width || !depth)) return GPFC_EINVAL;
    if (nbins < 1) return GPFC_EINVAL;
    if (!pow2_in_range(nbins) || nbins > gpfc::kFineBins) return GPFC_ENOTSUP;
    if (zfold && nbins < 16) return GPFC_ENOTSUP;
    if (!fused_widths(p, nbins)) return GPFC_ENOTSUP;
    return GPFC_OK;
}

int32_t gpfc_batch_fold_score(gpfc_plan* p, const double* t, const float* flux, const double* periods,
                              int32_t nbins, float* snr, int32_t* start, int32_t* width, float* depth,
                              uint16_t* zfold, void* stream) {
    int32_t rc = check_batch(p, t, flux, periods, nbins, snr, start, width, depth, zfold);
    if (rc != GPFC_OK) return rc;
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return device_error(e, "hipSetDevice");
    return batch_enqueue(p, t, flux, periods, nbins, snr, start, width, depth, zfold,
                         (hipStream_t)stream);
}

// Record what `enqueue(stream)` launches into the plan's graph.
extern "C++" template <class F>
static int32_t capture_into_plan(gpfc_plan* p, hipStream_t s, F enqueue) {
    if (p->graph_exec) { (void)hipGraphExecDestroy(p->graph_exec); p->graph_exec = nullptr; }
    if (p->graph) { (void)hipGraphDestroy(p->graph); p->graph = nullptr; }
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return device_error(e, "hipStreamBeginCapture");
    int32_t rc = enqueue(s);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s, &g);
    if (rc != GPFC_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return device_error(e, "hipStreamEndCapture");
    p->graph = g;
    e = hipGraphInstantiate(&p->graph_exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        p->graph_exec = nullptr;
        return device_error(e, "hipGraphInstantiate");
    }
    return GPFC_OK;
}

int32_t gpfc_batch_capture(gpfc_plan* p, const double* t, const float* flux, const double* periods,
                           int32_t nbins, float* snr, int32_t* start, int32_t* width, float* depth,
                           uint16_t* zfold, void* stream) {
    int32_t rc = check_batch(p, t, flux, periods, nbins, snr, start, width, depth, zfold);
    if (rc != GPFC_OK) return rc;
    if (!stream) return GPFC_EINVAL;   // the null stream cannot be captured
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return device_error(e, "hipSetDevice");
    return capture_into_plan(p, (hipStream_t)stream, [&](hipStream_t s) {
        return batch_enqueue(p, t, flux, periods, nbins, snr, start, width, depth, zfold, s);
    });
}

static int32_t check_survey(const gpfc_plan* p, const gpfc_cnn* cnn, const double* t,
                            const float* flux, const double* periods, int32_t nbins,
                            const gpfc_survey_out* o) {
    if (!p || !o || !p->b_survey) return GPFC_EINVAL;
    if (p->b_samples > 0 && (!t || !flux)) return GPFC_EINVAL;
    if (p->b_periods > 0 && (!periods || !o->snr || !o->start || !o->width || !o->depth))
        return GPFC_EINVAL;
    if (nbins < 1) return GPFC_EINVAL;
    if (!pow2_in_range(nbins) || nbins > gpfc::kFineBins) return GPFC_ENOTSUP;
    if (!fused_widths(p, nbins)) return GPFC_ENOTSUP;
    const bool net = o->logits != nullptr;
    if (net && (!cnn || nbins != gpfc::kFineBins || p->s_zfolds == 0)) return GPFC_EINVAL;
    if (o->top < 0 || o->top > GPFC_MAX_TOP) return GPFC_EINVAL;
    if (o->top > 0) {
        if (!o->box_val || !o->box_idx) return GPFC_EINVAL;
        if ((o->cnn_val != nullptr) != (o->cnn_idx != nullptr)) return GPFC_EINVAL;
        if ((o->judged_val != nullptr) != (o->judged_idx != nullptr)) return GPFC_EINVAL;
        if (!net && (o->cnn_val || o->judged_val)) return GPFC_EINVAL;
    }
    return GPFC_OK;
}

static int32_t survey_enqueue(gpfc_plan* p, gpfc_cnn* cnn, const double* t, const float* flux,
                              const double* periods, int32_t nbins, const gpfc_survey_out& o,
                              hipStream_t s) {
    hipError_t e = gpfc::launch_batch_prepare(t, flux, p->b_soff, p->b_roff, p->b_curves,
                                              p->b_max_records, p->b_info, p->b_rec, p->b_lo, s);
    if (e != hipSuccess) return device_error(e, "survey prepare launch");
    const bool net = o.logits != nullptr;
    const int64_t K = p->s_k;
    // Several chunks with a network: chunk j is folded on `s` into buffer j % 2
    // while the network scores chunk j - 1 from the other buffer on p->s_net.
    // Events order the two: the network of chunk j waits for its fold, the fold
    // of chunk j + 2 waits for the network of chunk j (same buffer), and `s`
    // waits for the last networks before the per-curve best-K.
    const bool pipe = net && p->s_zbuf2 != nullptr;
    auto net_chunk = [&](const SurveyChunk& ch, const uint16_t* zb, hipStream_t ns) -> int32_t {
        const int64_t folds = (int64_t)(ch.c1 - ch.c0) * K;
        const int64_t cmb = gpfc::cnn_max_batch(cnn);
        const int64_t mb = p->s_net_batch > 0 ? std::min(p->s_net_batch, cmb) : cmb;
        for (int64_t f0 = 0; f0 < folds; f0 += mb) {
            const int64_t B = std::min<int64_t>(mb, folds - f0);
            const uint16_t* x = zb + f0 * gpfc::kFineBins;
            float* lg = o.logits + (int64_t)ch.c0 * K + f0;
            const int32_t rc = o.cnn_fp8 ? gpfc_cnn_forward_fp8(cnn, x, 0, B, lg, ns)
                                         : gpfc_cnn_forward(cnn, x, 0, B, lg, ns);
            if (rc != GPFC_OK) return rc;
        }
        return GPFC_OK;
    };
    for (size_t j = 0; j < p->s_chunks.size(); ++j) {
        const SurveyChunk& ch = p->s_chunks[j];
        const int b = (int)(j & 1);
        uint16_t* zb = (pipe && b) ? p->s_zbuf2 : p->s_zbuf;
        if (pipe && j >= 2) {
            e = hipStreamWaitEvent(s, p->s_ev[2 + b], 0);
            if (e != hipSuccess) return device_error(e, "survey stream wait");
        }
        e = gpfc::launch_batch_fold_score(p->b_rec, p->b_lo, p->b_curve, p->b_item + ch.i0, ch.i1 - ch.i0,
                                          p->b_counter, p->b_info, periods, nbins,
                                          plan_widths(p, nbins), p->n_cu, o.snr, o.start, o.width,
                                          o.depth, net ? zb : nullptr, s);
        if (e != hipSuccess) return device_error(e, "survey fold_score launch");
        if (!net) continue;
        if (!pipe) {
            const int32_t rc = net_chunk(ch, zb, s);
            if (rc != GPFC_OK) return rc;
            continue;
        }
        e = hipEventRecord(p->s_ev[b], s);
        if (e == hipSuccess) e = hipStreamWaitEvent(p->s_net, p->s_ev[b], 0);
        if (e != hipSuccess) return device_error(e, "survey stream fork");
        const int32_t rc = net_chunk(ch, zb, p->s_net);
        if (rc != GPFC_OK) return rc;
        e = hipEventRecord(p->s_ev[2 + b], p->s_net);
        if (e != hipSuccess) return device_error(e, "survey event record");
    }
    if (pipe) {
        // join: the best-K below reads every chunk's logits
        e = hipStreamWaitEvent(s, p->s_ev[2], 0);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, p->s_ev[3], 0);
        if (e != hipSuccess) return device_error(e, "survey stream join");
    }
    if (o.top > 0) {
        const int64_t rows = p->b_curves;
        e = gpfc::launch_topk(o.snr, rows, K, nullptr, 0.0f, o.top, o.box_val, o.box_idx, s);
        if (e == hipSuccess && o.cnn_val)
            e = gpfc::launch_topk(o.logits, rows, K, nullptr, 0.0f, o.top, o.cnn_val, o.cnn_idx, s);
        if (e == hipSuccess && o.judged_val)
            e = gpfc::launch_topk(o.logits, rows, K, o.snr, o.judge_snr, o.top, o.judged_val,
                                  o.judged_idx, s);
        if (e != hipSuccess) return device_error(e, "survey top-k launch");
    }
    return GPFC_OK;
}

int32_t gpfc_survey_run(gpfc_plan* p, gpfc_cnn* cnn, const double* t, const float* flux,
                        const double* periods, int32_t nbins, const gpfc_survey_out* out,
                        void* stream) {
    int32_t rc = check_survey(p, cnn, t, flux, periods, nbins, out);
    if (rc != GPFC_OK) return rc;
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return device_error(e, "hipSetDevice");
    return survey_enqueue(p, cnn, t, flux, periods, nbins, *out, (hipStream_t)stream);
}

int32_t gpfc_survey_capture(gpfc_plan* p, gpfc_cnn* cnn, const double* t, const float* flux,
                            const double* periods, int32_t nbins, const gpfc_survey_out* out,
                            void* stream) {
    int32_t rc = check_survey(p, cnn, t, flux, periods, nbins, out);
    if (rc != GPFC_OK) return rc;
    if (!stream) return GPFC_EINVAL;
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return device_error(e, "hipSetDevice");
    const gpfc_survey_out o = *out;
    return capture_into_plan(p, (hipStream_t)stream, [&](hipStream_t s) {
        return survey_enqueue(p, cnn, t, flux, periods, nbins, o, s);
    });
}

int32_t gpfc_periodogram_peaks(const float* values, int64_t rows, int64_t len, const double* periods,
                               float nsigma, int32_t min_width, int32_t max_peaks, float* sde,
                               float* mean, float* sd, int32_t* n_peaks, float* peak_val,
                               int64_t* peak_idx, int32_t* peak_width, int32_t* peak_harmonic,
                               void* stream) {
    if (rows < 0 || len < 0 || min_width < 0 || max_peaks < 1 || max_peaks > GPFC_MAX_PEAKS ||
        !(nsigma >= 0.0f))
        return GPFC_EINVAL;
    if (rows > 0x7fffffffLL) return GPFC_ERANGE;
    if (rows == 0) return GPFC_OK;
    if ((len > 0 && !values) || !sde || !mean || !sd || !n_peaks || !peak_val || !peak_idx ||
        !peak_width || !peak_harmonic)
        return GPFC_EINVAL;
    hipError_t e = gpfc::launch_periodogram(values, rows, len, periods, nsigma, min_width, max_peaks,
                                            sde, mean, sd, n_peaks, peak_val, peak_idx, peak_width,
                                            peak_harmonic, (hipStream_t)stream);
    return e == hipSuccess ? GPFC_OK : device_error(e, "k_periodogram launch");
}

int32_t gpfc_topk(const float* values, int64_t rows, int64_t len, const float* gate,
                  float gate_min, int32_t top, float* out_val, int64_t* out_idx, void* stream) {
    if (rows < 0 || len < 0 || top < 1 || top > GPFC_MAX_TOP) return GPFC_EINVAL;
    if (rows > 0x7fffffffLL || len > 0xffffffffLL) return GPFC_ERANGE;
    if (rows == 0) return GPFC_OK;
    if (!out_val || !out_idx || (len > 0 && !values)) return GPFC_EINVAL;
    hipError_t e = gpfc::launch_topk(values, rows, len, gate, gate_min, top, out_val, out_idx,
                                     (hipStream_t)stream);
    return e == hipSuccess ? GPFC_OK : device_error(e, "k_topk_rows launch");
}

int32_t gpfc_batch_replay(gpfc_plan* p, void* stream) {
    if (!p || !p->graph_exec) return GPFC_EINVAL;
    hipError_t e = hipGraphLaunch(p->graph_exec, (hipStream_t)stream);
    if (e != hipSuccess) return device_error(e, "hipGraphLaunch");
    return GPFC_OK;
}

int32_t gpfc_batch_curve_stats(gpfc_plan* p, gpfc_curve* out, void* stream) {
    if (!p || p->b_curves < 0 || (p->b_curves > 0 && !out)) return GPFC_EINVAL;
    std::vector<CurveInfo> ci(p->b_curves > 0 ? p->b_curves : 1);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (p->b_curves > 0)
        e = hipMemcpyAsync(ci.data(), p->b_info, sizeof(CurveInfo) * p->b_curves,
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_error(e, "batch curve stats copy");
    for (int32_t c = 0; c < p->b_curves; ++c) {
        out[c].mean = ci[c].mean;
        out[c].sigma = ci[c].sigma;
        out[c].ref = ci[c].ref;
        out[c].qscale = ci[c].qscale;
        out[c].tmax = ci[c].tmax;
        out[c].maxdev = ci[c].maxdev;
        out[c].n = ci[c].n;
        out[c].exact = ci[c].exact;
        out[c].finite = ci[c].finite;
        out[c].words = ci[c].words;
    }
    return GPFC_OK;
}

// Allocation-free fold + score: the curve statistics, the prepared records
// and their low words live in `scratch`, one copy per GPU at the address
// hipGetSymbolAddress reports on that device (the array's name is only a host
// stand-in and is never passed to a kernel). Layout: CurveInfo at 0, records
// at 256, low words after the records.
// Cache lines of the survey tuner: "<device> survey <curves> <samples> <k> <nbins> <chunk> <net batch>".
static bool survey_cache_lookup(const char* path, const char* dev, int32_t n_curves, int64_t samples,
                                int64_t k, int32_t nbins, int64_t* chunk, int64_t* net) {
    if (!path) return false;
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char line[512], name[64], tag[16];
    long long cc, cs, ck, ch, cn;
    int cb;
    bool found = false;
    while (fgets(line, sizeof(line), f))
        if (sscanf(line, "%63s %15s %lld %lld %lld %d %lld %lld", name, tag, &cc, &cs, &ck, &cb, &ch,
                   &cn) == 8 &&
            !strcmp(name, dev) && !strcmp(tag, "survey") && cc == n_curves && cs == samples && ck == k &&
            cb == nbins && ch >= 0 && cn >= 0) {
            *chunk = ch;
            *net = cn;
            found = true;
        }
    fclose(f);
    return found;
}

int32_t gpfc_survey_autotune(gpfc_plan* p, gpfc_cnn* cnn, const int64_t* soff, int32_t n_curves,
                             const double* t, const float* flux, const double* periods, int64_t k,
                             int32_t nbins, const int64_t* chunks, int32_t n_chunk, const int64_t* nets,
                             int32_t n_net, const char* cache_path, int64_t* chunk_out,
                             int64_t* net_out, float* ms_out, void* stream) {
    if (!p || !soff || n_curves < 1 || k < 1 || !chunks || n_chunk < 1 || n_chunk > 16 || n_net < 0 ||
        n_net > 16 || (n_net > 0 && !nets) || !t || !flux || !periods)
        return GPFC_EINVAL;
    if (!pow2_in_range(nbins) || nbins > gpfc::kFineBins) return GPFC_ENOTSUP;
    if (cnn && nbins != gpfc::kFineBins) return GPFC_EINVAL;
    const int64_t cmb = cnn ? gpfc::cnn_max_batch(cnn) : 0;
    for (int i = 0; i < n_chunk; ++i)
        if (chunks[i] < (cnn ? k : 0)) return GPFC_EINVAL;
    for (int i = 0; i < n_net; ++i)
        if (nets[i] < 1 || nets[i] > cmb) return GPFC_EINVAL;
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return device_error(e, "hipSetDevice");
    if (!cache_path && p->tune_cache[0]) cache_path = p->tune_cache;
    const int64_t samples = soff[n_curves];
    int64_t best_c = chunks[0], best_n = n_net > 0 ? nets[0] : 0;
    float best_ms = -1.0f;
    if (!survey_cache_lookup(cache_path, p->device_name, n_curves, samples, k, nbins, &best_c, &best_n)) {
        hipStream_t s = (hipStream_t)stream;
        const int64_t m = (int64_t)n_curves * k;
        void* out = nullptr;
        e = hipMalloc(&out, (size_t)m * 20);
        if (e != hipSuccess) return e == hipErrorOutOfMemory ? GPFC_ENOMEM : device_error(e, "hipMalloc");
        gpfc_survey_out o{};
        o.snr = (float*)out;
        o.start = (int32_t*)(o.snr + m);
        o.width = o.start + m;
        o.depth = (float*)(o.width + m);
        o.logits = cnn ? o.depth + m : nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        int32_t rc = GPFC_OK;
        const int nn = n_net > 0 ? n_net : 1;
        for (int ci = 0; ci < n_chunk && rc == GPFC_OK && e == hipSuccess; ++ci) {
            rc = gpfc_survey_setup(p, soff, n_curves, k, cnn ? chunks[ci] : 0);
            for (int ni = 0; ni < nn && rc == GPFC_OK && e == hipSuccess; ++ni) {
                p->s_net_batch = n_net > 0 ? nets[ni] : 0;
                rc = survey_enqueue(p, cnn, t, flux, periods, nbins, o, s);   // warm-up
                if (rc == GPFC_OK) e = hipEventRecord(e0, s);
                if (rc == GPFC_OK && e == hipSuccess) rc = survey_enqueue(p, cnn, t, flux, periods, nbins, o, s);
                if (rc == GPFC_OK && e == hipSuccess) e = hipEventRecord(e1, s);
                if (rc == GPFC_OK && e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.0f;
                if (rc == GPFC_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (rc == GPFC_OK && e == hipSuccess && (best_ms < 0.0f || ms < best_ms)) {
                    best_ms = ms;
                    best_c = chunks[ci];
                    best_n = p->s_net_batch;
                }
            }
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipStreamSynchronize(s);
        (void)hipFree(out);
        if (rc != GPFC_OK) return rc;
        if (e != hipSuccess) return device_error(e, "survey autotune");
        if (cache_path) {
            FILE* f = fopen(cache_path, "a");
            if (f) {
                fprintf(f, "%s survey %d %lld %lld %d %lld %lld\n", p->device_name, n_curves,
                        (long long)samples, (long long)k, nbins, (long long)best_c, (long long)best_n);
                fclose(f);
            }
        }
    }
    const int32_t rc = gpfc_survey_setup(p, soff, n_curves, k, cnn ? best_c : 0);
    if (rc != GPFC_OK) return rc;
    p->s_net_batch = best_n;
    if (chunk_out) *chunk_out = best_c;
    if (net_out) *net_out = best_n;
    if (ms_out) *ms_out = best_ms;
    return GPFC_OK;
}

int32_t gpfc_fold_score_noalloc(const double* t, const float* flux, int64_t n,
                                const double* periods, int64_t k, int32_t nbins, float* snr,
                                int32_t* start, int32_t* width, float* depth, void* stream) {
    if (n < 0 || k < 0 || nbins < 1) return GPFC_EINVAL;
    if (n > 0 && (!t || !flux)) return GPFC_EINVAL;
    if (k > 0 && (!periods || !snr || !start || !width || !depth)) return GPFC_EINVAL;
    if (!pow2_in_range(nbins) || nbins > gpfc::kFineBins) return GPFC_ENOTSUP;
    if (n > GPFC_NOALLOC_MAX_SAMPLES || k > 0x7fffffffLL) return GPFC_ERANGE;
    if (gpfc::prepared_len(n) > kNoAllocRecs) return GPFC_ERANGE;
    char* base = nullptr;
    const int32_t rc = noalloc_base(&base);
    if (rc != GPFC_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    CurveInfo* info = reinterpret_cast<CurveInfo*>(base);
    gpfc::Rec* rec = reinterpret_cast<gpfc::Rec*>(base + kNoAllocInfoBytes);
    uint64_t* lo = reinterpret_cast<uint64_t*>(base + kNoAllocInfoBytes + kNoAllocRecs * sizeof(gpfc::Rec));
    hipError_t e = gpfc::launch_curve_stats(t, flux, n, info, s);
    if (e != hipSuccess) return device_error(e, "k_curve_stats launch");
    e = gpfc::launch_pack(t, flux, n, info, rec, lo, s);
    if (e != hipSuccess) return device_error(e, "k_pack launch");
    e = gpfc::launch_fold_score(rec, lo, n, periods, k, nbins, info, default_widths(nbins), snr,
                                start, width, depth, nullptr, s);
    return e == hipSuccess ? GPFC_OK : device_error(e, "k_fold_score launch");
}

int32_t gpfc_detrend(gpfc_plan* p, const double* t, const float* flux, const uint8_t* transit,
                     int64_t n, const gpfc_detrend_opts* o, double* flux_out, uint8_t* keep_out,
                     gpfc_detrend_info* info, void* stream) {
    if (!p || n < 0 || (n > 0 && (!t || !flux || !flux_out || !keep_out))) return GPFC_EINVAL;
    if (n > 0x7ffffffeLL) return GPFC_ERANGE;
    gpfc::DetrendParams prm{};
    const double defaults[] = {0.5, 0.75, 1.0, 1.5, 2.0, 3.0, 5.0};
    if (!o) {
        prm.cadence = 0.020428;
        prm.gap_cadences = 30.0;
        prm.jump_sigma = 5.0;
        prm.clip_sigma = 3.0;
        prm.edge = 30;
        prm.max_fits = 10;
        prm.n_spacings = 7;
        for (int i = 0; i < 7; ++i) prm.spacings[i] = defaults[i];
    } else {
        if (!(o->cadence > 0.0) || !(o->gap_cadences > 0.0) || !(o->jump_sigma > 0.0) ||
            !(o->clip_sigma > 0.0) || o->edge < 0 || o->max_fits < 1 || o->max_fits > 100 ||
            o->n_spacings < 1 || o->n_spacings > GPFC_DETREND_MAX_SPACINGS)
            return GPFC_EINVAL;
        for (int i = 0; i < o->n_spacings; ++i)
            if (!(o->spacings[i] > 0.0) || !isfinite(o->spacings[i]) ||
                (i > 0 && !(o->spacings[i] > o->spacings[i - 1])))
                return GPFC_EINVAL;
        prm.cadence = o->cadence;
        prm.gap_cadences = o->gap_cadences;
        prm.jump_sigma = o->jump_sigma;
        prm.clip_sigma = o->clip_sigma;
        prm.edge = o->edge;
        prm.max_fits = o->max_fits;
        prm.n_spacings = o->n_spacings;
        for (int i = 0; i < o->n_spacings; ++i) prm.spacings[i] = o->spacings[i];
    }
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return device_error(e, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    const size_t bytes = gpfc::detrend_workspace_bytes(n, prm.n_spacings);
    if (bytes > p->d_cap) {
        void* buf = nullptr;
        e = hipMalloc(&buf, bytes);
        if (e != hipSuccess) return e == hipErrorOutOfMemory ? GPFC_ENOMEM : device_error(e, "hipMalloc");
        if (p->d_buf) {
            (void)hipDeviceSynchronize();
            (void)hipFree(p->d_buf);
        }
        p->d_buf = buf;
        p->d_cap = bytes;
    }
    const gpfc::DetrendWs w = gpfc::detrend_carve(p->d_buf, n, prm.n_spacings);
    e = gpfc::launch_detrend(t, flux, transit, n, prm, w, flux_out, keep_out, s);
    if (e != hipSuccess) return device_error(e, "detrend launch");
    int32_t st[2] = {0, 0};
    e = hipMemcpyAsync(st, w.status, sizeof(st), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_error(e, "detrend status");
    if (info) {
        info->n_segments = st[1];
        info->status = st[0];
        info->pad = 0;
        int32_t kept = 0;
        if (st[1] > 0) {
            std::vector<int32_t> ch((size_t)st[1]);
            e = hipMemcpy(ch.data(), w.chosen, sizeof(int32_t) * st[1], hipMemcpyDeviceToHost);
            if (e != hipSuccess) return device_error(e, "detrend segments");
            for (int32_t c : ch) kept += c >= 0;
        }
        info->n_kept_segments = kept;
    }
    return (st[0] & 1) ? GPFC_ERANGE : GPFC_OK;
}

int32_t gpfc_sync(void* stream) {
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return device_error(e, "hipStreamSynchronize");
    int dev = -1, cur = -1;
    if (stream) {
        e = hipStreamGetDevice((hipStream_t)stream, &dev);
        if (e != hipSuccess) return device_error(e, "hipStreamGetDevice");
        e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
        if (e != hipSuccess) return device_error(e, "hipSetDevice");
    }
    int32_t fault = 0;
    e = gpfc::take_input_fault(&fault);
    if (stream && cur >= 0 && cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess) return device_error(e, "input check");
    return fault ? GPFC_EINVAL : GPFC_OK;
}

}  // extern "C"
