// qcurv_api.cpp -- the C ABI of libqcurv.so (declared in include/qcurv.h): argument
// validation, per-context scratch and the hand-off to the HIP kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "fit_internal.h"
#include "qcurv.h"

struct qc_context {
    int device = 0;
    int last_hip_error = 0;
    uint32_t* refit_entries = nullptr; // device, capacity 16x4-block indices
    uint64_t* refit_masks = nullptr;   // device, capacity lane masks
    uint32_t* refit_counts = nullptr;  // device, [entries, pixels]
    int64_t capacity = 0;
    hipStream_t last_stream = nullptr;
    int last_precision = 0;
    // timing: recorded event triples not yet read, and the sums of those already read
    bool timing = false;
    std::vector<hipEvent_t> pending;
    qc_timing sums{};
};

namespace {

qc_status hip_fail(qc_context* ctx, hipError_t e) {
    if (ctx) ctx->last_hip_error = static_cast<int>(e);
    return e == hipErrorOutOfMemory ? QC_ERR_OOM : QC_ERR_HIP;
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
    if (p->reject != 0) return QC_ERR_UNSUPPORTED;
    return QC_OK;
}

qc_status check_frame(const qc_frame* f) {
    if (!f || !f->depth) return QC_ERR_INVALID_ARG;
    const int sb = sample_bytes(f->format);
    if (sb == 0) return QC_ERR_INVALID_ARG;
    if (f->width < 1 || f->height < 1) return QC_ERR_INVALID_ARG;
    // pixel indices are kept in 32 bits
    if (static_cast<int64_t>(f->width) * f->height > (int64_t{1} << 31)) return QC_ERR_INVALID_ARG;
    if (f->pitch_bytes < static_cast<int64_t>(f->width) * sb || f->pitch_bytes % sb != 0)
        return QC_ERR_INVALID_ARG;
    const qc_intrinsics& K = f->K;
    if (!(K.fx > 0.f) || !(K.fy > 0.f) || !std::isfinite(K.fx) || !std::isfinite(K.fy) ||
        !std::isfinite(K.cx) || !std::isfinite(K.cy))
        return QC_ERR_INVALID_ARG;
    return QC_OK;
}

qc_status ensure_capacity(qc_context* ctx, int64_t entries) {
    if (ctx->capacity >= entries) return QC_OK;
    hipError_t e;
    if (ctx->refit_entries) {
        // the previous lists may still be in use by enqueued work
        if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(ctx, e);
        (void)hipFree(ctx->refit_entries);
        (void)hipFree(ctx->refit_masks);
        ctx->refit_entries = nullptr;
        ctx->refit_masks = nullptr;
        ctx->capacity = 0;
    }
    void* p = nullptr;
    void* q = nullptr;
    if ((e = hipMalloc(&p, sizeof(uint32_t) * static_cast<size_t>(entries))) != hipSuccess)
        return hip_fail(ctx, e);
    if ((e = hipMalloc(&q, sizeof(uint64_t) * static_cast<size_t>(entries))) != hipSuccess) {
        (void)hipFree(p);
        return hip_fail(ctx, e);
    }
    ctx->refit_entries = static_cast<uint32_t*>(p);
    ctx->refit_masks = static_cast<uint64_t*>(q);
    ctx->capacity = entries;
    return QC_OK;
}

}  // namespace

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
    p->cond_max = 30.f;
    p->step_max = 1e-1f;
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
    if ((e = hipSetDevice(device)) != hipSuccess) {
        delete ctx;
        return QC_ERR_HIP;
    }
    void* p = nullptr;
    if ((e = hipMalloc(&p, 2 * sizeof(uint32_t))) != hipSuccess) {
        delete ctx;
        return e == hipErrorOutOfMemory ? QC_ERR_OOM : QC_ERR_HIP;
    }
    ctx->refit_counts = static_cast<uint32_t*>(p);
    *out = ctx;
    return QC_OK;
}

qc_status qc_destroy(qc_context* ctx) {
    if (!ctx) return QC_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->refit_entries) (void)hipFree(ctx->refit_entries);
    if (ctx->refit_masks) (void)hipFree(ctx->refit_masks);
    if (ctx->refit_counts) (void)hipFree(ctx->refit_counts);
    for (hipEvent_t ev : ctx->pending) (void)hipEventDestroy(ev);
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
    const int64_t entries = qc::refit_capacity(frame->width, frame->height);
    if (params->precision != QC_PREC_FP64 && (st = ensure_capacity(ctx, entries)) != QC_OK)
        return st;

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
    d.step_max = params->step_max;
    d.precision = params->precision;
    d.k1 = out->k1;
    d.k2 = out->k2;
    d.normal = out->normal;
    d.residual = out->residual;
    d.flags = out->flags;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    if (ctx->timing) {
        for (auto& x : ev)
            if ((e = hipEventCreate(&x)) != hipSuccess) return hip_fail(ctx, e);
        ctx->pending.insert(ctx->pending.end(), ev, ev + 3);
    }
    if ((e = qc::launch_fit(d, ctx->refit_entries, ctx->refit_masks, ctx->refit_counts, s,
                            ctx->timing ? ev : nullptr)) != hipSuccess)
        return hip_fail(ctx, e);
    ctx->last_stream = s;
    ctx->last_precision = params->precision;
    return QC_OK;
}

qc_status qc_last_refit_count(qc_context* ctx, uint32_t* count) {
    if (!ctx || !count) return QC_ERR_INVALID_ARG;
    *count = 0;
    if (ctx->last_precision == QC_PREC_FP64) return QC_OK;
    hipError_t e;
    if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_fail(ctx, e);
    if ((e = hipStreamSynchronize(ctx->last_stream)) != hipSuccess) return hip_fail(ctx, e);
    uint32_t counts[2] = {0, 0};
    if ((e = hipMemcpy(counts, ctx->refit_counts, sizeof counts, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(ctx, e);
    *count = counts[1];
    return QC_OK;
}

qc_status qc_set_timing(qc_context* ctx, int enable) {
    if (!ctx) return QC_ERR_INVALID_ARG;
    ctx->timing = enable != 0;
    return QC_OK;
}

qc_status qc_get_timing(qc_context* ctx, qc_timing* out, int reset) {
    if (!ctx || !out) return QC_ERR_INVALID_ARG;
    hipError_t e;
    if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_fail(ctx, e);
    qc_status st = QC_OK;
    for (size_t i = 0; i + 2 < ctx->pending.size(); i += 3) {
        hipEvent_t* ev = &ctx->pending[i];
        float a = 0.f, b = 0.f;
        if ((e = hipEventSynchronize(ev[2])) != hipSuccess ||
            (e = hipEventElapsedTime(&a, ev[0], ev[1])) != hipSuccess ||
            (e = hipEventElapsedTime(&b, ev[1], ev[2])) != hipSuccess) {
            st = hip_fail(ctx, e);
        } else {
            ctx->sums.calls += 1;
            ctx->sums.fit_ms += a;
            ctx->sums.refit_ms += b;
        }
        for (int j = 0; j < 3; ++j) (void)hipEventDestroy(ev[j]);
    }
    ctx->pending.clear();
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
    }
    return "unknown status";
}

}  // extern "C"
