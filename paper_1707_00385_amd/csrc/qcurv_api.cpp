// qcurv_api.cpp -- the C ABI of libqcurv.so (declared in include/qcurv.h): argument
// validation, per-context scratch, batch graphs, tuning table and the hand-off to the
// HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "api_internal.h"
#include "fit_internal.h"
#include "qcurv.h"
#include "tune_table.h"

namespace {

// Host staging of one batch: descriptors, tile prefix sums and a header, copied to the
// device by the first node of the batch graph.
struct BatchStaging {
    qc::FitDesc frames[QC_MAX_BATCH];
    uint32_t first_tile[QC_MAX_BATCH + 1];
    uint32_t header[1];   // [0] frames
};

// One of the two batches a context may have in flight.
struct BatchSlot {
    BatchStaging* host = nullptr;   // pinned
    BatchStaging* dev = nullptr;
    void* list = nullptr;           // refit list storage for `capacity` entries
    uint32_t* counts = nullptr;
    int64_t capacity = 0;           // refit list entries
    size_t refit_lds = 0;           // LDS of the captured FP64 pass's workgroups
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;      // recorded after the slot's last use
    bool in_flight = false;
};

using qc::TuneEntry;
using qc::TuneKey;

TuneKey tune_key(const qc_frame* f, const qc_params* p) {
    return TuneKey{f->width, f->height, p->radius, p->iterations, p->stride, p->reject};
}

}  // namespace

struct qc_context {
    int device = 0;
    int cus = 0;
    int last_hip_error = 0;
    void* refit_storage = nullptr;     // device, refit list for `capacity` entries
    uint32_t* refit_counts = nullptr;  // device, kCountWords counters
    int64_t capacity = 0;
    hipStream_t last_stream = nullptr;
    int last_precision = 0;
    const uint32_t* last_counts = nullptr;   // counters of the last fit's list (device)
    // timing: a pool of event triples created once (qc_set_timing), the triples recorded
    // and not yet read (oldest first), the free ones, and the sums of those already read
    bool timing = false;
    std::vector<hipEvent_t> events;     // 3 per triple
    std::deque<int> pending, free_triples;
    qc_timing sums{};
    // batches
    BatchSlot slots[2];
    int next_slot = 0;
    hipStream_t capture_stream = nullptr;
    // tuned tile widths and schedules
    std::map<TuneKey, TuneEntry> tuned;
};

namespace {

qc_status hip_fail(qc_context* ctx, hipError_t e) {
    if (ctx) ctx->last_hip_error = static_cast<int>(e);
    return e == hipErrorOutOfMemory ? QC_ERR_OOM : QC_ERR_HIP;
}

// Triples of timing events per context: enough for every call of a long timed loop to
// record without waiting; beyond that the oldest triple is read (waiting for it) and reused.
constexpr int kTimingTriples = 1024;

// Folds the oldest recorded triple into the sums (waits for its last event) and frees it.
qc_status fold_oldest(qc_context* ctx) {
    const int t = ctx->pending.front();
    ctx->pending.pop_front();
    ctx->free_triples.push_back(t);
    hipEvent_t* ev = &ctx->events[3 * static_cast<size_t>(t)];
    float a = 0.f, b = 0.f;
    hipError_t e;
    if ((e = hipEventSynchronize(ev[2])) != hipSuccess || (e = hipEventElapsedTime(&a, ev[0], ev[1])) != hipSuccess ||
        (e = hipEventElapsedTime(&b, ev[1], ev[2])) != hipSuccess)
        return hip_fail(ctx, e);
    ctx->sums.calls += 1;
    ctx->sums.fit_ms += a;
    ctx->sums.refit_ms += b;
    return QC_OK;
}

// The events of a free triple for the next timed call (nullptr when timing is off).
qc_status next_triple(qc_context* ctx, hipEvent_t** ev) {
    *ev = nullptr;
    if (!ctx->timing) return QC_OK;
    if (ctx->free_triples.empty()) {
        const qc_status st = fold_oldest(ctx);
        if (st != QC_OK) return st;
    }
    const int t = ctx->free_triples.front();
    ctx->free_triples.pop_front();
    ctx->pending.push_back(t);
    *ev = &ctx->events[3 * static_cast<size_t>(t)];
    return QC_OK;
}

int sample_bytes(int32_t format) {
    switch (format) {
        case QC_DEPTH_U16: return 2;
        case QC_DEPTH_F16: return 2;
        case QC_DEPTH_F32: return 4;
        default: return 0;
    }
}

qc_status check_params(const qc_params* p) {
    if (!p) return QC_ERR_INVALID_ARG;
    if (p->radius < 1 || p->radius > QC_MAX_RADIUS) return QC_ERR_INVALID_ARG;
    if (p->normal_radius < 1 || p->normal_radius > QC_MAX_RADIUS) return QC_ERR_INVALID_ARG;
    if (p->iterations < 0 || p->iterations > 64) return QC_ERR_INVALID_ARG;
    if (!(p->k > 0.f) || !std::isfinite(p->k)) return QC_ERR_INVALID_ARG;
    if (!(p->depth_scale > 0.f) || !std::isfinite(p->depth_scale)) return QC_ERR_INVALID_ARG;
    if (p->precision < QC_PREC_MIXED || p->precision > QC_PREC_FP64) return QC_ERR_INVALID_ARG;
    if (std::isnan(p->cond_max) || std::isnan(p->step_max)) return QC_ERR_INVALID_ARG;
    if (p->tile_width != 0 && !qc::valid_tile_width(p->tile_width)) return QC_ERR_INVALID_ARG;
    if (p->reject != 0 && p->reject != 1) return QC_ERR_INVALID_ARG;
    if (p->stride < 1 || p->stride > p->radius) return QC_ERR_INVALID_ARG;
    return QC_OK;
}

qc_status check_frame(const qc_frame* f) {
    if (!f || !f->depth) return QC_ERR_INVALID_ARG;
    const int sb = sample_bytes(f->format);
    if (sb == 0) return QC_ERR_INVALID_ARG;
    if (f->width < 1 || f->height < 1) return QC_ERR_INVALID_ARG;
    // pixel indices are kept in 32 bits, tile indices in 24
    if (static_cast<int64_t>(f->width) * f->height > (int64_t{1} << 31)) return QC_ERR_INVALID_ARG;
    if (qc::refit_capacity(f->width, f->height, 8) >= (int64_t{1} << 24)) return QC_ERR_INVALID_ARG;
    if (f->pitch_bytes < static_cast<int64_t>(f->width) * sb || f->pitch_bytes % sb != 0)
        return QC_ERR_INVALID_ARG;
    const qc_intrinsics& K = f->K;
    if (!(K.fx > 0.f) || !(K.fy > 0.f) || !std::isfinite(K.fx) || !std::isfinite(K.fy) ||
        !std::isfinite(K.cx) || !std::isfinite(K.cy))
        return QC_ERR_INVALID_ARG;
    return QC_OK;
}

int64_t max_tiles(int width, int height) {
    int64_t m = 0;
    for (int tw = 8; tw <= 64; tw *= 2) m = std::max(m, qc::refit_capacity(width, height, tw));
    return m;
}

int tile_width_for(const qc_context* ctx, const qc_frame* f, const qc_params* p) {
    if (p->tile_width != 0) return p->tile_width;
    auto it = ctx->tuned.find(tune_key(f, p));
    return it != ctx->tuned.end() ? it->second.tile_width : 16;
}

// The precision a request runs at: a MIXED request with tile_width 0 takes the schedule
// qc_tune recorded for its key (FP64 throughout where that measured faster); any other
// request runs as asked.
int32_t precision_for(const qc_context* ctx, const qc_frame* f, const qc_params* p) {
    if (p->precision != QC_PREC_MIXED) return p->precision;
    // A 3x3 window (nine samples for six parameters) leaves the FP32 fit too close to
    // interpolation for the recompute criteria to bound its error: MIXED runs it in FP64.
    if (p->radius == 1) return QC_PREC_FP64;
    if (p->tile_width != 0) return p->precision;
    auto it = ctx->tuned.find(tune_key(f, p));
    return it != ctx->tuned.end() ? it->second.schedule : QC_PREC_MIXED;
}

qc::FitDesc make_desc(const qc_frame* frame, const qc_params* params, const qc_output* out,
                      int tile_w) {
    qc::FitDesc d;
    d.depth = frame->depth;
    d.format = frame->format;
    d.width = frame->width;
    d.height = frame->height;
    d.pitch = frame->pitch_bytes;
    d.fx = frame->K.fx;
    d.fy = frame->K.fy;
    d.cx = frame->K.cx;
    d.cy = frame->K.cy;
    d.scale = frame->format == QC_DEPTH_U16 ? params->depth_scale : 1.f;
    d.radius = params->radius;
    d.normal_radius = params->normal_radius;
    d.iterations = params->iterations;
    d.k = params->k;
    d.cond_max = params->cond_max;
    // step_max is stated for windows reaching up to 7 pixels from the centre; beyond, an
    // FP32 fit whose last update is smaller still can be outside the tolerance (measured
    // for dense windows at r = 10, 13 and 16 and for 25x25 sampled every 2nd pixel), so the
    // bound tightens as (7 / r)^2, r being the reach whatever the stride.
    const int r = params->radius;
    d.step_max = r > 7 ? params->step_max * (49.f / static_cast<float>(r * r)) : params->step_max;
    d.precision = params->precision;
    d.reject = params->reject;
    d.stride = params->stride;
    d.tile_w = tile_w;
    d.k1 = out->k1;
    d.k2 = out->k2;
    d.normal = out->normal;
    d.residual = out->residual;
    d.flags = out->flags;
    return d;
}

qc_status ensure_capacity(qc_context* ctx, int64_t entries) {
    if (ctx->capacity >= entries) return QC_OK;
    hipError_t e;
    if (ctx->refit_storage) {
        // the previous list may still be in use by the previous call's work, which is on
        // that call's stream (calls on one context are ordered on one stream): wait for
        // that stream only, not for other contexts' or streams' work
        if ((e = hipStreamSynchronize(ctx->last_stream)) != hipSuccess) return hip_fail(ctx, e);
        (void)hipFree(ctx->refit_storage);
        ctx->refit_storage = nullptr;
        ctx->capacity = 0;
    }
    void* p = nullptr;
    if ((e = hipMalloc(&p, qc::refit_list_bytes(entries))) != hipSuccess) return hip_fail(ctx, e);
    ctx->refit_storage = p;
    ctx->capacity = entries;
    return QC_OK;
}

void free_slot(BatchSlot& s) {
    if (s.exec) (void)hipGraphExecDestroy(s.exec);
    if (s.graph) (void)hipGraphDestroy(s.graph);
    if (s.list) (void)hipFree(s.list);
    s.exec = nullptr;
    s.graph = nullptr;
    s.list = nullptr;
    s.capacity = 0;
    s.refit_lds = 0;
}

// Makes `s` hold scratch for `entries` tiles and a graph bound to it whose FP64 pass has
// at least `refit_lds` bytes of LDS per workgroup.  The graph is the staging upload, a
// counter-reset kernel and the two persistent passes; it holds no memset node.
qc_status prepare_slot(qc_context* ctx, BatchSlot& s, int64_t entries, size_t refit_lds) {
    hipError_t e;
    if (!s.host) {
        void* h = nullptr;
        void* dv = nullptr;
        void* c = nullptr;
        if ((e = hipHostMalloc(&h, sizeof(BatchStaging), hipHostMallocDefault)) != hipSuccess)
            return hip_fail(ctx, e);
        s.host = static_cast<BatchStaging*>(h);
        if ((e = hipMalloc(&dv, sizeof(BatchStaging))) != hipSuccess) return hip_fail(ctx, e);
        s.dev = static_cast<BatchStaging*>(dv);
        if ((e = hipMalloc(&c, qc::kCountWords * sizeof(uint32_t))) != hipSuccess) return hip_fail(ctx, e);
        s.counts = static_cast<uint32_t*>(c);
        if ((e = hipEventCreate(&s.done)) != hipSuccess) return hip_fail(ctx, e);
    }
    if (s.capacity >= entries && s.refit_lds >= refit_lds && s.exec) return QC_OK;
    // keep the larger of the old and new needs, so that alternating batches do not
    // capture again and again
    const int64_t cap = std::max<int64_t>({entries, s.capacity, 1 << 16});
    const size_t lds = std::max(refit_lds, s.refit_lds);
    free_slot(s);
    void* p = nullptr;
    if ((e = hipMalloc(&p, qc::refit_list_bytes(cap))) != hipSuccess) return hip_fail(ctx, e);
    s.list = p;
    s.capacity = cap;
    s.refit_lds = lds;
    hipStream_t cs = ctx->capture_stream;
    if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return hip_fail(ctx, e);
    hipError_t le = hipMemcpyAsync(s.dev, s.host, sizeof(BatchStaging), hipMemcpyHostToDevice, cs);
    if (le == hipSuccess)
        le = qc::launch_fit_batch(s.dev->frames, s.dev->first_tile, s.dev->header, ctx->cus,
                                  s.refit_lds, qc::refit_list(s.list, s.capacity, s.counts), cs);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(ctx, le);
    }
    if (e != hipSuccess) return hip_fail(ctx, e);
    s.graph = g;
    if ((e = hipGraphInstantiate(&s.exec, g, nullptr, nullptr, 0)) != hipSuccess)
        return hip_fail(ctx, e);
    return QC_OK;
}

// ---------------------------------------------------------------------------- no-alloc
// Fixed device scratch of qc_fit_noalloc: the list counters (kCountWords words) at offset
// 0 and the list storage from kNoAllocListOffset on, for at most kNoAllocBytes -
// kNoAllocListOffset bytes of entries.  Every device the library runs on holds its own
// copy until the process ends.  In host code `scratch` only names the symbol: its device
// address comes from hipGetSymbolAddress (qc_create, once per device) and is the only one
// ever passed to kernels or copies.
constexpr size_t kNoAllocBytes = size_t{2} << 20;        // 2 MiB
constexpr size_t kNoAllocListOffset = 256;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mutex;
void* g_noalloc_ptr[kNoAllocDevices] = {};

// Called with `device` current.  Looks up the device address of `scratch` once per device.
hipError_t noalloc_setup(int device) {
    if (device >= kNoAllocDevices) return hipSuccess;   // qc_fit_noalloc reports it
    std::lock_guard<std::mutex> lock(g_noalloc_mutex);
    if (g_noalloc_ptr[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e == hipSuccess) g_noalloc_ptr[device] = p;
    return e;
}

// List entries (FP32-pass tiles) whose list fits in the fixed scratch.
int64_t noalloc_max_entries() {
    static const int64_t n = [] {
        const size_t avail = kNoAllocBytes - kNoAllocListOffset;
        int64_t m = static_cast<int64_t>(avail / qc::refit_list_bytes(1));
        while (m > 0 && qc::refit_list_bytes(m) > avail) --m;
        return m;
    }();
    return n;
}

void* noalloc_ptr(int device) {
    if (device < 0 || device >= kNoAllocDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_noalloc_mutex);
    return g_noalloc_ptr[device];
}

}  // namespace

namespace qc {

int context_device(const qc_context* ctx) { return ctx->device; }

qc_status check_request(const qc_frame* frame, const qc_params* params) {
    qc_status st = check_frame(frame);
    return st != QC_OK ? st : check_params(params);
}

}  // namespace qc

extern "C" {

void qc_params_default(qc_params* p) {
    if (!p) return;
    p->radius = 7;
    p->normal_radius = 3;
    p->iterations = 5;
    p->k = 1e-5f;
    p->reject = 0;
    p->depth_scale = 1e-3f;
    p->precision = QC_PREC_MIXED;
    p->cond_max = 15.f;
    p->step_max = 1e-1f;
    p->tile_width = 0;
    p->stride = 1;
}

qc_status qc_create(qc_context** out, int device) {
    if (!out) return QC_ERR_INVALID_ARG;
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return QC_ERR_HIP;
    if (device < 0 || device >= n) return QC_ERR_INVALID_ARG;
    qc_context* ctx = new (std::nothrow) qc_context();
    if (!ctx) return QC_ERR_OOM;
    ctx->device = device;
    int cus = 0;
    void* p = nullptr;
    if ((e = hipSetDevice(device)) != hipSuccess ||
        (e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device)) != hipSuccess ||
        (e = hipMalloc(&p, qc::kCountWords * sizeof(uint32_t))) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking)) != hipSuccess) {
        if (p) (void)hipFree(p);
        delete ctx;
        return e == hipErrorOutOfMemory ? QC_ERR_OOM : QC_ERR_HIP;
    }
    ctx->cus = cus > 0 ? cus : 1;
    ctx->refit_counts = static_cast<uint32_t*>(p);
    if ((e = noalloc_setup(device)) != hipSuccess) {
        (void)hipFree(p);
        (void)hipStreamDestroy(ctx->capture_stream);
        delete ctx;
        return QC_ERR_HIP;
    }
    *out = ctx;
    return QC_OK;
}

qc_status qc_destroy(qc_context* ctx) {
    if (!ctx) return QC_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->refit_storage) (void)hipFree(ctx->refit_storage);
    if (ctx->refit_counts) (void)hipFree(ctx->refit_counts);
    for (hipEvent_t ev : ctx->events) (void)hipEventDestroy(ev);
    for (BatchSlot& s : ctx->slots) {
        free_slot(s);
        if (s.host) (void)hipHostFree(s.host);
        if (s.dev) (void)hipFree(s.dev);
        if (s.counts) (void)hipFree(s.counts);
        if (s.done) (void)hipEventDestroy(s.done);
    }
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    delete ctx;
    return QC_OK;
}

qc_status qc_fit(qc_context* ctx, const qc_frame* frame, const qc_params* params,
                 const qc_output* out, void* stream) {
    if (!ctx) return QC_ERR_INVALID_ARG;
    qc_status st;
    if ((st = check_frame(frame)) != QC_OK) return st;
    if ((st = check_params(params)) != QC_OK) return st;
    if (!out || !out->k1 || !out->k2) return QC_ERR_INVALID_ARG;
    hipError_t e;
    if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_fail(ctx, e);
    qc_params p = *params;
    p.precision = precision_for(ctx, frame, params);
    if (p.precision != QC_PREC_FP64 &&
        (st = ensure_capacity(ctx, max_tiles(frame->width, frame->height))) != QC_OK)
        return st;
    const qc::FitDesc d = make_desc(frame, &p, out, tile_width_for(ctx, frame, params));
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t* ev = nullptr;
    if ((st = next_triple(ctx, &ev)) != QC_OK) return st;
    const qc::RefitList list = qc::refit_list(ctx->refit_storage, ctx->capacity, ctx->refit_counts);
    if ((e = qc::launch_fit(d, list, ctx->cus, s, ev)) != hipSuccess) return hip_fail(ctx, e);
    ctx->last_stream = s;
    ctx->last_precision = p.precision;
    ctx->last_counts = ctx->refit_counts;
    return QC_OK;
}

qc_status qc_fit_noalloc(qc_context* ctx, const qc_frame* frame, const qc_params* params,
                         const qc_output* out, void* stream) {
    if (!ctx) return QC_ERR_INVALID_ARG;
    qc_status st;
    if ((st = check_frame(frame)) != QC_OK) return st;
    if ((st = check_params(params)) != QC_OK) return st;
    if (!out || !out->k1 || !out->k2) return QC_ERR_INVALID_ARG;
    const int tw = tile_width_for(ctx, frame, params);
    qc_params p = *params;
    p.precision = precision_for(ctx, frame, params);
    const int64_t entries = qc::refit_capacity(frame->width, frame->height, tw);
    const int64_t max_entries = noalloc_max_entries();
    if (p.precision != QC_PREC_FP64 && entries > max_entries) return QC_ERR_TOO_LARGE;
    unsigned char* base = static_cast<unsigned char*>(noalloc_ptr(ctx->device));
    if (!base) return QC_ERR_UNSUPPORTED;
    hipError_t e;
    if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_fail(ctx, e);
    const qc::FitDesc d = make_desc(frame, &p, out, tw);
    uint32_t* counts = reinterpret_cast<uint32_t*>(base);
    const qc::RefitList list = qc::refit_list(base + kNoAllocListOffset, max_entries, counts);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((e = qc::launch_fit(d, list, ctx->cus, s, nullptr)) != hipSuccess) return hip_fail(ctx, e);
    ctx->last_stream = s;
    ctx->last_precision = p.precision;
    ctx->last_counts = counts;
    return QC_OK;
}

qc_status qc_fit_batch(qc_context* ctx, const qc_batch_item* items, int32_t n, void* stream) {
    if (!ctx || n < 0 || n > QC_MAX_BATCH || (n > 0 && !items)) return QC_ERR_INVALID_ARG;
    if (n == 0) return QC_OK;
    qc_status st;
    const int32_t prec = items[0].params.precision;
    bool per_frame = false;
    for (int32_t i = 0; i < n; ++i) {
        const qc_batch_item& it = items[i];
        if ((st = check_frame(&it.frame)) != QC_OK) return st;
        if ((st = check_params(&it.params)) != QC_OK) return st;
        if (!it.out.k1 || !it.out.k2) return QC_ERR_INVALID_ARG;
        if (it.params.precision != prec) return QC_ERR_INVALID_ARG;
        per_frame |= it.params.reject != 0 || it.params.stride != 1;
    }
    if (prec == QC_PREC_FP64) return QC_ERR_UNSUPPORTED;
    hipError_t e;
    if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_fail(ctx, e);
    hipStream_t hs = static_cast<hipStream_t>(stream);

    // Items whose tuned schedule is FP64 throughout run as per-frame FP64 launches (which
    // use no list); the others form the batch.
    std::vector<int32_t> batched;
    std::vector<qc::FitDesc> fp64_descs;
    for (int32_t i = 0; i < n; ++i) {
        const qc_batch_item& it = items[i];
        if (precision_for(ctx, &it.frame, &it.params) == QC_PREC_FP64) {
            qc_params p = it.params;
            p.precision = QC_PREC_FP64;
            fp64_descs.push_back(make_desc(&it.frame, &p, &it.out, tile_width_for(ctx, &it.frame, &it.params)));
        } else {
            batched.push_back(i);
        }
    }
    if (!fp64_descs.empty()) {
        const qc::RefitList none = qc::refit_list(nullptr, 0, ctx->refit_counts);
        for (const qc::FitDesc& d : fp64_descs)
            if ((e = qc::launch_fit(d, none, ctx->cus, hs)) != hipSuccess) return hip_fail(ctx, e);
    }
    n = static_cast<int32_t>(batched.size());
    if (n == 0) return QC_OK;

    // frames from most to least work per tile, so the long tiles start first
    std::vector<int32_t> order(batched);
    auto cost = [&](int32_t i) {
        const int r = items[i].params.radius;
        return static_cast<int64_t>(2 * r + 1) * (2 * r + 1) * std::max(1, items[i].params.iterations);
    };
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return cost(a) > cost(b); });
    std::vector<qc::FitDesc> descs(n);
    std::vector<uint32_t> first(n + 1, 0);
    for (int32_t j = 0; j < n; ++j) {
        const qc_batch_item& it = items[order[j]];
        const int tw = tile_width_for(ctx, &it.frame, &it.params);
        descs[j] = make_desc(&it.frame, &it.params, &it.out, tw);
        first[j + 1] = first[j] + static_cast<uint32_t>(qc::refit_capacity(it.frame.width, it.frame.height, tw));
    }
    if (first[n] >= (1u << 24)) return QC_ERR_INVALID_ARG;

    BatchSlot& s = ctx->slots[ctx->next_slot];
    if (s.in_flight) {
        // the slot's staging and lists may still be read by its previous batch
        if ((e = hipEventSynchronize(s.done)) != hipSuccess) return hip_fail(ctx, e);
        s.in_flight = false;
    }
    size_t refit_lds = 0;
    for (int32_t j = 0; j < n; ++j) refit_lds = std::max(refit_lds, qc::batch_refit_lds_bytes(descs[j]));
    if ((st = prepare_slot(ctx, s, first[n], refit_lds)) != QC_OK) return st;
    std::memcpy(s.host->frames, descs.data(), sizeof(qc::FitDesc) * n);
    std::memcpy(s.host->first_tile, first.data(), sizeof(uint32_t) * (n + 1));
    s.host->header[0] = static_cast<uint32_t>(n);
    if (per_frame) {
        // The batched kernels carry only the default weights of Eq. (11) and dense
        // windows: a batch holding rejection or strided frames runs as per-frame launches,
        // in order on the stream, on the slot's own list (so that two batches in flight on
        // two streams share none).
        const qc::RefitList list = qc::refit_list(s.list, s.capacity, s.counts);
        for (int32_t j = 0; j < n; ++j)
            if ((e = qc::launch_fit(descs[j], list, ctx->cus, hs)) != hipSuccess) return hip_fail(ctx, e);
    } else if (ctx->timing) {
        // timed batches run eagerly so that the two passes can be bracketed separately
        hipEvent_t* ev = nullptr;
        if ((st = next_triple(ctx, &ev)) != QC_OK) return st;
        if ((e = hipMemcpyAsync(s.dev, s.host, sizeof(BatchStaging), hipMemcpyHostToDevice, hs)) != hipSuccess ||
            (e = qc::launch_fit_batch(s.dev->frames, s.dev->first_tile, s.dev->header, ctx->cus,
                                      s.refit_lds, qc::refit_list(s.list, s.capacity, s.counts), hs,
                                      ev)) != hipSuccess)
            return hip_fail(ctx, e);
    } else if ((e = hipGraphLaunch(s.exec, hs)) != hipSuccess) {
        return hip_fail(ctx, e);
    }
    if ((e = hipEventRecord(s.done, hs)) != hipSuccess) return hip_fail(ctx, e);
    s.in_flight = true;
    ctx->next_slot ^= 1;
    return QC_OK;
}

qc_status qc_tune(qc_context* ctx, const qc_frame* frame, const qc_params* params,
                  const qc_output* out, int32_t reps, void* stream, int32_t* tile_width,
                  int32_t* schedule) {
    if (!ctx || reps < 1) return QC_ERR_INVALID_ARG;
    qc_status st;
    if ((st = check_frame(frame)) != QC_OK) return st;
    if ((st = check_params(params)) != QC_OK) return st;
    if (!out || !out->k1 || !out->k2) return QC_ERR_INVALID_ARG;
    hipError_t e;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t a = nullptr, b = nullptr;
    if ((e = hipSetDevice(ctx->device)) != hipSuccess || (e = hipEventCreate(&a)) != hipSuccess ||
        (e = hipEventCreate(&b)) != hipSuccess) {
        if (a) (void)hipEventDestroy(a);
        return hip_fail(ctx, e);
    }
    const bool timing = ctx->timing;
    ctx->timing = false;
    // milliseconds of `reps` fits with parameters p (after one warm-up fit)
    auto time_fits = [&](const qc_params& p, float* ms) {
        qc_status r = qc_fit(ctx, frame, &p, out, stream);
        if (r == QC_OK && (e = hipEventRecord(a, s)) != hipSuccess) r = hip_fail(ctx, e);
        for (int32_t i = 0; i < reps && r == QC_OK; ++i) r = qc_fit(ctx, frame, &p, out, stream);
        if (r == QC_OK && ((e = hipEventRecord(b, s)) != hipSuccess || (e = hipEventSynchronize(b)) != hipSuccess ||
                           (e = hipEventElapsedTime(ms, a, b)) != hipSuccess))
            r = hip_fail(ctx, e);
        return r;
    };
    // A candidate replaces the choice so far only if it is faster by more than kMargin:
    // the default (width 16, MIXED) stays unless another is measurably faster, so that
    // timing noise between near-equal shapes does not decide.
    constexpr float kMargin = 0.01f;
    TuneEntry best;
    float best_ms = 0.f;
    for (int tw : {16, 8, 32, 64}) {
        if (st != QC_OK) break;
        qc_params p = *params;
        p.tile_width = tw;   // an explicit width: the fit runs at the requested precision
        float ms = 0.f;
        st = time_fits(p, &ms);
        if (st == QC_OK && (tw == 16 || ms < best_ms * (1.f - kMargin))) {
            best.tile_width = tw;
            best_ms = ms;
        }
    }
    if (st == QC_OK && params->precision == QC_PREC_MIXED) {
        // the other schedule of a MIXED request: every pixel in FP64 (more accurate, and
        // faster where the FP32 pass would list many pixels for recomputation)
        qc_params p = *params;
        p.precision = QC_PREC_FP64;
        float ms = 0.f;
        st = time_fits(p, &ms);
        if (st == QC_OK && ms < best_ms * (1.f - kMargin)) best.schedule = QC_PREC_FP64;
    }
    ctx->timing = timing;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st != QC_OK) return st;
    ctx->tuned[tune_key(frame, params)] = best;
    if (tile_width) *tile_width = best.tile_width;
    if (schedule) *schedule = best.schedule;
    return QC_OK;
}

qc_status qc_tune_save(qc_context* ctx, const char* path) {
    if (!ctx || !path) return QC_ERR_INVALID_ARG;
    FILE* f = std::fopen(path, "w");
    if (!f) return QC_ERR_INVALID_ARG;
    bool ok = true;
    for (const auto& kv : ctx->tuned) ok = qc::format_tune_line(f, kv.first, kv.second) > 0 && ok;
    return std::fclose(f) == 0 && ok ? QC_OK : QC_ERR_INVALID_ARG;
}

qc_status qc_tune_load(qc_context* ctx, const char* path) {
    if (!ctx || !path) return QC_ERR_INVALID_ARG;
    FILE* f = std::fopen(path, "r");
    if (!f) return QC_ERR_INVALID_ARG;
    char line[256];
    qc_status st = QC_OK;
    std::map<TuneKey, TuneEntry> got;
    while (std::fgets(line, sizeof line, f)) {
        TuneKey k;
        TuneEntry e;
        const int r = qc::parse_tune_line(line, &k, &e, qc::valid_tile_width);
        if (r < 0) {
            st = QC_ERR_INVALID_ARG;
            break;
        }
        if (r > 0) got[k] = e;
    }
    std::fclose(f);
    if (st != QC_OK) return st;   // a malformed file changes nothing
    for (const auto& kv : got) ctx->tuned[kv.first] = kv.second;
    return QC_OK;
}

qc_status qc_last_refit_count(qc_context* ctx, uint32_t* count) {
    if (!ctx || !count) return QC_ERR_INVALID_ARG;
    *count = 0;
    if (ctx->last_precision == QC_PREC_FP64) return QC_OK;
    hipError_t e;
    if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_fail(ctx, e);
    if ((e = hipStreamSynchronize(ctx->last_stream)) != hipSuccess) return hip_fail(ctx, e);
    uint32_t counts[qc::kCountWords] = {};
    const uint32_t* src = ctx->last_counts ? ctx->last_counts : ctx->refit_counts;
    if ((e = hipMemcpy(counts, src, sizeof counts, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(ctx, e);
    *count = counts[4];   // listed pixels
    return QC_OK;
}

qc_status qc_set_timing(qc_context* ctx, int enable) {
    if (!ctx) return QC_ERR_INVALID_ARG;
    if (enable && ctx->events.empty()) {
        hipError_t e;
        if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_fail(ctx, e);
        std::vector<hipEvent_t> evs(3 * static_cast<size_t>(kTimingTriples), nullptr);
        for (hipEvent_t& x : evs)
            if ((e = hipEventCreate(&x)) != hipSuccess) {
                for (hipEvent_t y : evs)
                    if (y) (void)hipEventDestroy(y);
                return hip_fail(ctx, e);
            }
        ctx->events = std::move(evs);
        for (int t = 0; t < kTimingTriples; ++t) ctx->free_triples.push_back(t);
    }
    ctx->timing = enable != 0;
    return QC_OK;
}

qc_status qc_get_timing(qc_context* ctx, qc_timing* out, int reset) {
    if (!ctx || !out) return QC_ERR_INVALID_ARG;
    hipError_t e;
    if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_fail(ctx, e);
    qc_status st = QC_OK;
    while (!ctx->pending.empty()) {
        const qc_status s1 = fold_oldest(ctx);
        if (s1 != QC_OK) st = s1;
    }
    *out = ctx->sums;
    if (reset) ctx->sums = qc_timing{};
    return st;
}

int qc_last_hip_error(qc_context* ctx) { return ctx ? ctx->last_hip_error : 0; }

const char* qc_status_string(qc_status s) {
    switch (s) {
        case QC_OK: return "ok";
        case QC_ERR_INVALID_ARG: return "invalid argument";
        case QC_ERR_UNSUPPORTED: return "unsupported request";
        case QC_ERR_OOM: return "out of device memory";
        case QC_ERR_HIP: return "HIP runtime error";
        case QC_ERR_BUSY: return "busy";
        case QC_ERR_INTERNAL: return "internal error";
        case QC_ERR_TOO_LARGE: return "frame too large for the fixed scratch of qc_fit_noalloc";
    }
    return "unknown status";
}

}  // extern "C"
