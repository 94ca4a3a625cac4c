// Host side of the C ABI declared in include/gpfc.h: argument checks (before
// any HIP call), plans and their device workspace, error reporting.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/gpfc.h"
#include "gpfc_internal.h"

using gpfc::CurveInfo;
using gpfc::Widths;

struct gpfc_plan {
    int32_t device = 0;
    gpfc::Rec* rec = nullptr;     // prepared curve: times and packed contributions
    int64_t cap = 0;              // records rec can hold
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
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
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

Widths plan_widths(const gpfc_plan* p, int32_t nbins) {
    if (p->nw == 0) return default_widths(nbins);
    Widths w{};
    for (int i = 0; i < p->nw; ++i) w.w[w.n++] = p->widths[i];
    return w;
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
    if ((k + 63) / 64 > 0x7fffffffLL) return GPFC_ERANGE;
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
        e = hipMalloc(&buf, (size_t)want * sizeof(gpfc::Rec));
        if (e != hipSuccess) return e == hipErrorOutOfMemory ? GPFC_ENOMEM : device_error(e, "hipMalloc");
        if (p->rec) {
            (void)hipDeviceSynchronize();
            (void)hipFree(p->rec);
        }
        p->rec = buf;
        p->cap = want;
    }
    e = gpfc::launch_curve_stats(t, flux, n, p->info, s);
    if (e != hipSuccess) return device_error(e, "k_curve_stats launch");
    e = gpfc::launch_pack(t, flux, n, p->info, p->rec, s);
    if (e != hipSuccess) return device_error(e, "k_pack launch");
    p->n = n;
    return GPFC_OK;
}

int32_t check_prepared(const gpfc_plan* p, const void* periods, int64_t k, int32_t nbins) {
    if (!p || p->n < 0 || k < 0 || (k > 0 && !periods) || nbins < 1) return GPFC_EINVAL;
    if (!pow2_in_range(nbins)) return GPFC_ENOTSUP;
    if ((k + 63) / 64 > 0x7fffffffLL) return GPFC_ERANGE;
    return GPFC_OK;
}

}  // namespace

extern "C" {

int32_t gpfc_version(void) { return 100; }

const char* gpfc_strerror(int32_t code) {
    switch (code) {
        case GPFC_OK: return "ok";
        case GPFC_EINVAL: return "invalid argument";
        case GPFC_ENOTSUP: return "nbins must be a power of two in [1, 256]";
        case GPFC_ERANGE: return "size out of range (n > 262143 samples or too many periods)";
        case GPFC_ENOMEM: return "device memory allocation failed";
        case GPFC_EDEVICE: return "HIP device error";
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
    *out = p;
    return GPFC_OK;
}

int32_t gpfc_plan_destroy(gpfc_plan* p) {
    if (!p) return GPFC_OK;
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    if (p->rec) (void)hipFree(p->rec);
    if (p->info) (void)hipFree(p->info);
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->b_dev) (void)hipFree(p->b_dev);
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
    e = gpfc::launch_fold(p->rec, p->n, periods, k, nbins, p->info, sums, counts, means,
                          (hipStream_t)stream);
    if (e != hipSuccess) return device_error(e, "k_fold launch");
    return GPFC_OK;
}

int32_t gpfc_fold_score_prepared(gpfc_plan* p, const double* periods, int64_t k, int32_t nbins,
                                 float* snr, int32_t* start, int32_t* width, float* depth,
                                 uint16_t* zfold, void* stream) {
    int32_t rc = check_prepared(p, periods, k, nbins);
    if (rc != GPFC_OK) return rc;
    if (k > 0 && (!snr || !start || !width || !depth)) return GPFC_EINVAL;
    if (zfold && nbins < 16) return GPFC_ENOTSUP;
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return device_error(e, "hipSetDevice");
    e = gpfc::launch_fold_score(p->rec, p->n, periods, k, nbins, p->info, plan_widths(p, nbins),
                                snr, start, width, depth, zfold, (hipStream_t)stream);
    if (e != hipSuccess) return device_error(e, "k_fold_score launch");
    return GPFC_OK;
}

int32_t gpfc_fold_f32_prepared(gpfc_plan* p, const double* periods, int64_t k, int32_t nbins,
                               int32_t compensated, double* sums, int32_t* counts, double* means,
                               void* stream) {
    int32_t rc = check_prepared(p, periods, k, nbins);
    if (rc != GPFC_OK) return rc;
    if (k > 0 && (!sums || !counts)) return GPFC_EINVAL;
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return device_error(e, "hipSetDevice");
    e = gpfc::launch_fold_f32(p->rec, p->n, periods, k, nbins, compensated, p->info, sums, counts,
                              means, (hipStream_t)stream);
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
    hipError_t e = gpfc::launch_fold(p->rec, n, periods, k, nbins, p->info, sums, counts, means, s);
    if (e != hipSuccess) return device_error(e, "k_fold launch");
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
    hipError_t e = gpfc::launch_fold_score(p->rec, n, periods, k, nbins, p->info,
                                           plan_widths(p, nbins), snr, start, width, depth,
                                           nullptr, s);
    if (e != hipSuccess) return device_error(e, "k_fold_score launch");
    return GPFC_OK;
}

int32_t gpfc_score(gpfc_plan* p, const double* sums, const int32_t* counts, int64_t k,
                   int32_t nbins, double sigma, float* snr, int32_t* start, int32_t* width,
                   float* depth, void* stream) {
    if (!p || k < 0 || nbins < 1) return GPFC_EINVAL;
    if (!pow2_in_range(nbins)) return GPFC_ENOTSUP;
    if (k > 0 && (!sums || !counts || !snr || !start || !width || !depth)) return GPFC_EINVAL;
    if ((k + 63) / 64 > 0x7fffffffLL) return GPFC_ERANGE;
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return device_error(e, "hipSetDevice");
    e = gpfc::launch_score(sums, counts, k, nbins, sigma, plan_widths(p, nbins), snr, start, width,
                           depth, (hipStream_t)stream);
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

int32_t gpfc_batch_setup(gpfc_plan* p, const int64_t* soff, const int64_t* poff, int32_t n_curves) {
    if (!p || !soff || !poff || n_curves < 0) return GPFC_EINVAL;
    if (soff[0] != 0 || poff[0] != 0) return GPFC_EINVAL;
    int64_t recs = 0, maxr = 0, items = 0;
    std::vector<int64_t> roff(n_curves + 1);
    std::vector<gpfc::BatchCurve> curves(n_curves);
    roff[0] = 0;
    for (int32_t c = 0; c < n_curves; ++c) {
        const int64_t n = soff[c + 1] - soff[c];
        const int64_t k = poff[c + 1] - poff[c];
        if (n < 0 || k < 0) return GPFC_EINVAL;
        if (n > GPFC_MAX_SAMPLES) return GPFC_ERANGE;
        const int64_t r = gpfc::prepared_len(n);
        curves[c] = gpfc::BatchCurve{recs, gpfc::slice_len(n), poff[c], k};
        recs += r;
        roff[c + 1] = recs;
        maxr = r > maxr ? r : maxr;
        items += (k + 63) / 64;
    }
    if (items > 0x7fffffffLL) return GPFC_ERANGE;
    // Items, longest curve first (then curve, then block order).
    std::vector<int2> it;
    it.reserve((size_t)items);
    std::vector<int32_t> order(n_curves);
    for (int32_t c = 0; c < n_curves; ++c) order[c] = c;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return soff[a + 1] - soff[a] > soff[b + 1] - soff[b];
    });
    for (int32_t c : order)
        for (int64_t j = 0; j < (curves[c].k + 63) / 64; ++j) it.push_back(make_int2(c, (int)j));
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return device_error(e, "hipSetDevice");
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t sz_off = al(sizeof(int64_t) * (n_curves + 1));
    const size_t sz_cur = al(sizeof(gpfc::BatchCurve) * (n_curves > 0 ? n_curves : 1));
    const size_t sz_it = al(sizeof(int2) * (items > 0 ? items : 1));
    const size_t sz_ctr = 256;
    const size_t sz_inf = al(sizeof(CurveInfo) * (n_curves > 0 ? n_curves : 1));
    const size_t sz_rec = al(sizeof(gpfc::Rec) * (recs > 0 ? recs : 1));
    const size_t total = 2 * sz_off + sz_cur + sz_it + sz_ctr + sz_inf + sz_rec;
    if (p->graph_exec) { (void)hipGraphExecDestroy(p->graph_exec); p->graph_exec = nullptr; }
    if (p->graph) { (void)hipGraphDestroy(p->graph); p->graph = nullptr; }
    if (p->b_dev) {
        (void)hipDeviceSynchronize();
        (void)hipFree(p->b_dev);
        p->b_dev = nullptr;
    }
    p->b_curves = -1;
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
    p->b_rec = (gpfc::Rec*)base;
    e = hipMemcpy(p->b_soff, soff, sizeof(int64_t) * (n_curves + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->b_roff, roff.data(), sizeof(int64_t) * (n_curves + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess && n_curves > 0)
        e = hipMemcpy(p->b_curve, curves.data(), sizeof(gpfc::BatchCurve) * n_curves, hipMemcpyHostToDevice);
    if (e == hipSuccess && items > 0)
        e = hipMemcpy(p->b_item, it.data(), sizeof(int2) * items, hipMemcpyHostToDevice);
    if (e != hipSuccess) return device_error(e, "batch table upload");
    p->b_curves = n_curves;
    p->b_samples = soff[n_curves];
    p->b_periods = poff[n_curves];
    p->b_records = recs;
    p->b_max_records = maxr;
    p->b_items = (int32_t)items;
    return GPFC_OK;
}

static int32_t batch_enqueue(gpfc_plan* p, const double* t, const float* flux, const double* periods,
                             int32_t nbins, float* snr, int32_t* start, int32_t* width, float* depth,
                             uint16_t* zfold, hipStream_t s) {
    hipError_t e = gpfc::launch_batch_prepare(t, flux, p->b_soff, p->b_roff, p->b_curves,
                                              p->b_max_records, p->b_info, p->b_rec, s);
    if (e != hipSuccess) return device_error(e, "batch prepare launch");
    e = gpfc::launch_batch_fold_score(p->b_rec, p->b_curve, p->b_item, p->b_items, p->b_counter,
                                      p->b_info, periods, nbins, plan_widths(p, nbins), p->n_cu, snr,
                                      start, width, depth, zfold, s);
    if (e != hipSuccess) return device_error(e, "batch fold_score launch");
    return GPFC_OK;
}

static int32_t check_batch(const gpfc_plan* p, const void* t, const void* flux, const void* periods,
                           int32_t nbins, const void* snr, const void* start, const void* width,
                           const void* depth, const void* zfold) {
    if (!p || p->b_curves < 0) return GPFC_EINVAL;
    if (p->b_samples > 0 && (!t || !flux)) return GPFC_EINVAL;
    if (p->b_periods > 0 && (!periods || !snr || !start || !width || !depth)) return GPFC_EINVAL;
    if (nbins < 1) return GPFC_EINVAL;
    if (!pow2_in_range(nbins)) return GPFC_ENOTSUP;
    if (zfold && nbins < 16) return GPFC_ENOTSUP;
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

int32_t gpfc_batch_capture(gpfc_plan* p, const double* t, const float* flux, const double* periods,
                           int32_t nbins, float* snr, int32_t* start, int32_t* width, float* depth,
                           uint16_t* zfold, void* stream) {
    int32_t rc = check_batch(p, t, flux, periods, nbins, snr, start, width, depth, zfold);
    if (rc != GPFC_OK) return rc;
    if (!stream) return GPFC_EINVAL;   // the null stream cannot be captured
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return device_error(e, "hipSetDevice");
    if (p->graph_exec) { (void)hipGraphExecDestroy(p->graph_exec); p->graph_exec = nullptr; }
    if (p->graph) { (void)hipGraphDestroy(p->graph); p->graph = nullptr; }
    hipStream_t s = (hipStream_t)stream;
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return device_error(e, "hipStreamBeginCapture");
    rc = batch_enqueue(p, t, flux, periods, nbins, snr, start, width, depth, zfold, s);
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
    }
    return GPFC_OK;
}

int32_t gpfc_sync(void* stream) {
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return device_error(e, "hipStreamSynchronize");
    return GPFC_OK;
}

}  // extern "C"
