// serve.cpp -- the serving loop of libqcurv.so (qc_server_* in include/qcurv.h).
//
// A worker thread moves frames through four stages:
//   submitted (depth copied into pinned staging by the caller's thread)
//   -> admitted (device memory reserved from the budget, FIFO order; upload enqueued on
//      a copy stream)
//   -> ready (upload enqueued: a batch may take the frame at once, its stream waiting for
//      the upload on the device; the staging range returns when the upload is done)
//   -> running (fitted by qc_fit_batch on one of two compute streams, at most
//      max_in_flight batches at once, up to max_batch ready frames per batch)
//   -> done (completion queued for qc_server_poll; device memory held until release).
// Frames that arrive while batches run are admitted and uploaded meanwhile and form the
// next batch, so the GPU always has the next batch queued behind the running one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "api_internal.h"
#include "qcurv.h"
#include "range_alloc.h"

namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

size_t sample_size(int32_t format) { return format == QC_DEPTH_F32 ? 4 : 2; }

struct Request {
    uint64_t ticket = 0;
    qc_request req{};           // depth points into pinned staging while queued
    size_t frame_bytes = 0;     // width * height * sample
    size_t stage_off = 0;
    bool staged = false;        // holds its pinned staging range (until its upload is done)
    size_t dev_off = 0, dev_bytes = 0;
    int64_t t_submit = 0, t_done = 0;
    hipEvent_t uploaded = nullptr;
    qc_status status = QC_OK;
    // device layout inside the pool
    void* depth = nullptr;
    float* k1 = nullptr;
    float* k2 = nullptr;
    float* normal = nullptr;
    float* residual = nullptr;
    uint8_t* flags = nullptr;
};

struct Batch {
    std::vector<Request*> reqs;
    hipEvent_t done = nullptr;
};

size_t align_up(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

struct qc_server {
    qc_context* ctx = nullptr;
    int device = 0;
    qc_server_config cfg{};
    char* dev_pool = nullptr;
    char* pin_pool = nullptr;
    qc::RangeAllocator dev_alloc, pin_alloc;
    hipStream_t copy_stream = nullptr;
    hipStream_t compute[2] = {nullptr, nullptr};
    int next_compute = 0;

    std::mutex mu;
    std::condition_variable work_cv;   // wakes the worker
    std::condition_variable done_cv;   // wakes pollers
    bool stop = false;
    uint64_t next_ticket = 1;
    std::deque<Request*> submitted, uploading, ready, completed;
    std::vector<Batch> running;
    std::map<uint64_t, Request*> all;
    qc_server_stats stats{};
    std::thread worker;

    size_t device_bytes(const qc_request& r) const {
        const size_t px = static_cast<size_t>(r.width) * r.height;
        size_t b = align_up(px * sample_size(r.format)) + 2 * align_up(px * 4);
        if (cfg.outputs & QC_OUT_NORMAL) b += align_up(px * 12);
        if (cfg.outputs & QC_OUT_RESIDUAL) b += align_up(px * 4);
        if (cfg.outputs & QC_OUT_FLAGS) b += align_up(px);
        return b;
    }

    void lay_out(Request* q) {
        const size_t px = static_cast<size_t>(q->req.width) * q->req.height;
        char* p = dev_pool + q->dev_off;
        q->depth = p;
        p += align_up(px * sample_size(q->req.format));
        q->k1 = reinterpret_cast<float*>(p);
        p += align_up(px * 4);
        q->k2 = reinterpret_cast<float*>(p);
        p += align_up(px * 4);
        if (cfg.outputs & QC_OUT_NORMAL) {
            q->normal = reinterpret_cast<float*>(p);
            p += align_up(px * 12);
        }
        if (cfg.outputs & QC_OUT_RESIDUAL) {
            q->residual = reinterpret_cast<float*>(p);
            p += align_up(px * 4);
        }
        if (cfg.outputs & QC_OUT_FLAGS) q->flags = reinterpret_cast<uint8_t*>(p);
    }

    void unstage(Request* q) {
        pin_alloc.release(q->stage_off, q->frame_bytes);
        q->staged = false;
    }

    void complete(Request* q, qc_status st) {
        q->status = st;
        q->t_done = now_ns();
        completed.push_back(q);
        stats.completed += 1;
    }

    // One pass of the worker's loop; returns true if anything moved.  Called with mu held;
    // releases it around HIP calls that may take long.
    bool step(std::unique_lock<std::mutex>& lk) {
        bool moved = false;
        // admission, FIFO: reserve device memory and enqueue the upload
        while (!submitted.empty()) {
            Request* q = submitted.front();
            size_t off = 0;
            if (!dev_alloc.alloc(q->dev_bytes, &off)) break;
            submitted.pop_front();
            q->dev_off = off;
            lay_out(q);
            const size_t row = static_cast<size_t>(q->req.width) * sample_size(q->req.format);
            hipError_t e = hipMemcpyAsync(q->depth, pin_pool + q->stage_off, row * q->req.height,
                                          hipMemcpyHostToDevice, copy_stream);
            if (e == hipSuccess) e = hipEventRecord(q->uploaded, copy_stream);
            if (e != hipSuccess) {
                pin_alloc.release(q->stage_off, q->frame_bytes);
                complete(q, QC_ERR_HIP);
                done_cv.notify_all();
            } else {
                // the frame can join a batch at once: the batch's stream waits for the
                // upload on the device; its staging range is released when it is done
                q->staged = true;
                uploading.push_back(q);
                ready.push_back(q);
            }
            moved = true;
        }
        // finished uploads (in order on the copy stream): their staging can be reused
        while (!uploading.empty() && hipEventQuery(uploading.front()->uploaded) == hipSuccess) {
            unstage(uploading.front());
            uploading.pop_front();
            moved = true;
        }
        // finished batches
        for (size_t i = 0; i < running.size();) {
            if (hipEventQuery(running[i].done) == hipSuccess) {
                // the batch waited for its frames' uploads: they are done, and a completed
                // request (which its owner may release) must hold no staging
                for (Request* q : running[i].reqs) {
                    if (q->staged) {
                        unstage(q);
                        uploading.erase(std::find(uploading.begin(), uploading.end(), q));
                    }
                    complete(q, QC_OK);
                }
                (void)hipEventDestroy(running[i].done);
                running.erase(running.begin() + static_cast<long>(i));
                done_cv.notify_all();
                moved = true;
            } else {
                ++i;
            }
        }
        // launch the next batch
        if (!ready.empty() && static_cast<int>(running.size()) < cfg.max_in_flight) {
            // a batch holds one precision (qc_fit_batch requires it): the ready frames that
            // share the oldest one's, in order; the others wait for a later batch
            Batch b;
            const int32_t prec = ready.front()->req.params.precision;
            for (auto it = ready.begin(); it != ready.end() && static_cast<int>(b.reqs.size()) < cfg.max_batch;) {
                if ((*it)->req.params.precision == prec) {
                    b.reqs.push_back(*it);
                    it = ready.erase(it);
                } else {
                    ++it;
                }
            }
            std::vector<qc_batch_item> items(b.reqs.size());
            for (size_t i = 0; i < b.reqs.size(); ++i) {
                Request* q = b.reqs[i];
                qc_batch_item& it = items[i];
                it.frame.depth = q->depth;
                it.frame.format = q->req.format;
                it.frame.width = q->req.width;
                it.frame.height = q->req.height;
                it.frame.pitch_bytes = static_cast<int64_t>(q->req.width) * sample_size(q->req.format);
                it.frame.K = q->req.K;
                it.params = q->req.params;
                it.out.k1 = q->k1;
                it.out.k2 = q->k2;
                it.out.normal = q->normal;
                it.out.residual = q->residual;
                it.out.flags = q->flags;
            }
            hipStream_t s = compute[next_compute];
            next_compute ^= 1;
            lk.unlock();
            hipError_t e = hipSuccess;
            for (Request* q : b.reqs)   // orders the batch after its frames' uploads
                if (e == hipSuccess) e = hipStreamWaitEvent(s, q->uploaded, 0);
            qc_status st = e == hipSuccess ? qc_fit_batch(ctx, items.data(), static_cast<int32_t>(items.size()), s)
                                           : QC_ERR_HIP;
            if (st == QC_OK && hipEventCreateWithFlags(&b.done, hipEventDisableTiming) != hipSuccess)
                st = QC_ERR_HIP;
            if (st == QC_OK && hipEventRecord(b.done, s) != hipSuccess) st = QC_ERR_HIP;
            lk.lock();
            stats.batches += 1;
            if (st != QC_OK) {
                if (b.done) (void)hipEventDestroy(b.done);
                for (Request* q : b.reqs) {
                    if (q->staged) {
                        // the copy engine may still read the staging: wait for it first
                        (void)hipEventSynchronize(q->uploaded);
                        unstage(q);
                        uploading.erase(std::find(uploading.begin(), uploading.end(), q));
                    }
                    complete(q, st);
                }
                done_cv.notify_all();
            } else {
                running.push_back(std::move(b));
            }
            moved = true;
        }
        return moved;
    }

    void run() {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            const bool moved = step(lk);
            const bool busy = !uploading.empty() || !running.empty();
            if (stop && submitted.empty() && !busy && ready.empty()) break;
            if (moved) continue;
            if (stop && !busy && ready.empty()) {
                // Stopping, nothing on the GPU, and the frames left wait for device memory
                // that only a release of completed results could free: no release comes
                // during destruction, so they complete with QC_ERR_BUSY instead.
                while (!submitted.empty()) {
                    Request* q = submitted.front();
                    submitted.pop_front();
                    pin_alloc.release(q->stage_off, q->frame_bytes);
                    complete(q, QC_ERR_BUSY);
                }
                done_cv.notify_all();
                continue;
            }
            // Nothing moved.  With GPU work outstanding, poll its events; otherwise every
            // change that could let work move (a submission, a release of memory, stop)
            // notifies work_cv under mu, so a plain wait cannot miss it.  (Waiting on a
            // "queue not empty" predicate would spin while the queue head waits for memory.)
            if (busy)
                work_cv.wait_for(lk, std::chrono::microseconds(20));
            else
                work_cv.wait(lk);
        }
    }
};

extern "C" {

qc_status qc_server_create(qc_context* ctx, const qc_server_config* cfg, qc_server** out) {
    if (!ctx || !cfg || !out) return QC_ERR_INVALID_ARG;
    *out = nullptr;
    if (cfg->max_batch < 1 || cfg->max_batch > QC_MAX_BATCH || cfg->max_in_flight < 1 ||
        cfg->max_in_flight > 2 || cfg->memory_budget < 4096 || cfg->staging_budget < 4096 ||
        (cfg->outputs & ~(QC_OUT_NORMAL | QC_OUT_RESIDUAL | QC_OUT_FLAGS)) != 0)
        return QC_ERR_INVALID_ARG;
    std::unique_ptr<qc_server> s(new (std::nothrow) qc_server());
    if (!s) return QC_ERR_OOM;
    s->ctx = ctx;
    s->device = qc::context_device(ctx);
    s->cfg = *cfg;
    hipError_t e;
    void* d = nullptr;
    void* h = nullptr;
    if ((e = hipSetDevice(s->device)) != hipSuccess) return QC_ERR_HIP;
    if ((e = hipMalloc(&d, cfg->memory_budget)) != hipSuccess)
        return e == hipErrorOutOfMemory ? QC_ERR_OOM : QC_ERR_HIP;
    s->dev_pool = static_cast<char*>(d);
    if ((e = hipHostMalloc(&h, cfg->staging_budget, hipHostMallocDefault)) != hipSuccess) {
        (void)hipFree(d);
        return QC_ERR_OOM;
    }
    s->pin_pool = static_cast<char*>(h);
    s->dev_alloc.reset(cfg->memory_budget);
    s->pin_alloc.reset(cfg->staging_budget);
    if (hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->compute[0], hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->compute[1], hipStreamNonBlocking) != hipSuccess) {
        for (hipStream_t st : {s->copy_stream, s->compute[0], s->compute[1]})
            if (st) (void)hipStreamDestroy(st);
        (void)hipFree(d);
        (void)hipHostFree(h);
        return QC_ERR_HIP;
    }
    s->worker = std::thread([p = s.get()] { p->run(); });
    *out = s.release();
    return QC_OK;
}

qc_status qc_server_submit(qc_server* s, const qc_request* r, uint64_t* ticket) {
    if (!s || !r || !ticket || !r->depth) return QC_ERR_INVALID_ARG;
    if (r->format < QC_DEPTH_U16 || r->format > QC_DEPTH_F32 || r->width < 1 || r->height < 1 ||
        r->pitch_bytes < static_cast<int64_t>(r->width) * static_cast<int64_t>(sample_size(r->format)))
        return QC_ERR_INVALID_ARG;
    if (r->params.precision == QC_PREC_FP64) return QC_ERR_UNSUPPORTED;
    qc_frame probe{};
    probe.depth = r->depth;
    probe.format = r->format;
    probe.width = r->width;
    probe.height = r->height;
    probe.pitch_bytes = static_cast<int64_t>(r->width) * static_cast<int64_t>(sample_size(r->format));
    probe.K = r->K;
    qc_status vs = qc::check_request(&probe, &r->params);
    if (vs != QC_OK) return vs;
    std::unique_ptr<Request> q(new (std::nothrow) Request());
    if (!q) return QC_ERR_OOM;
    q->req = *r;
    q->frame_bytes = static_cast<size_t>(r->width) * r->height * sample_size(r->format);
    q->dev_bytes = s->device_bytes(*r);
    if (q->dev_bytes > s->dev_alloc.capacity() || q->frame_bytes > s->pin_alloc.capacity())
        return QC_ERR_INVALID_ARG;
    if (hipEventCreateWithFlags(&q->uploaded, hipEventDisableTiming) != hipSuccess) return QC_ERR_HIP;
    size_t off = 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop || !s->pin_alloc.alloc(q->frame_bytes, &off)) {
            (void)hipEventDestroy(q->uploaded);
            return QC_ERR_BUSY;
        }
    }
    // pack the rows densely into the reserved staging range (outside the lock)
    const size_t row = static_cast<size_t>(r->width) * sample_size(r->format);
    const char* src = static_cast<const char*>(r->depth);
    for (int32_t y = 0; y < r->height; ++y)
        std::memcpy(s->pin_pool + off + y * row, src + static_cast<size_t>(y) * r->pitch_bytes, row);
    q->stage_off = off;
    q->t_submit = now_ns();
    std::lock_guard<std::mutex> lk(s->mu);
    q->ticket = s->next_ticket++;
    *ticket = q->ticket;
    s->all[q->ticket] = q.get();
    s->submitted.push_back(q.release());
    s->stats.submitted += 1;
    s->work_cv.notify_one();
    return QC_OK;
}

qc_status qc_server_poll(qc_server* s, qc_completion* out, int32_t max, int32_t* n, int64_t wait_us) {
    if (!s || !n || max < 0 || (max > 0 && !out)) return QC_ERR_INVALID_ARG;
    *n = 0;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->completed.empty() && wait_us > 0)
        s->done_cv.wait_for(lk, std::chrono::microseconds(wait_us), [&] { return !s->completed.empty(); });
    while (*n < max && !s->completed.empty()) {
        Request* q = s->completed.front();
        s->completed.pop_front();
        qc_completion& c = out[(*n)++];
        c.ticket = q->ticket;
        c.tag = q->req.tag;
        c.status = q->status;
        c.width = q->req.width;
        c.height = q->req.height;
        c.t_submit_ns = q->t_submit;
        c.t_done_ns = q->t_done;
        c.k1 = q->k1;
        c.k2 = q->k2;
        c.normal = q->normal;
        c.residual = q->residual;
        c.flags = q->flags;
    }
    return QC_OK;
}

qc_status qc_server_release(qc_server* s, uint64_t ticket) {
    if (!s) return QC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return QC_ERR_INVALID_ARG;
    Request* q = it->second;
    if (q->t_done == 0) return QC_ERR_BUSY;   // not finished
    if (std::find(s->completed.begin(), s->completed.end(), q) != s->completed.end())
        s->completed.erase(std::find(s->completed.begin(), s->completed.end(), q));
    if (q->depth) s->dev_alloc.release(q->dev_off, q->dev_bytes);
    if (q->uploaded) (void)hipEventDestroy(q->uploaded);
    s->all.erase(it);
    delete q;
    s->work_cv.notify_one();   // memory came back: admission may proceed
    return QC_OK;
}

qc_status qc_server_get_stats(qc_server* s, qc_server_stats* out) {
    if (!s || !out) return QC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    out->queued = s->submitted.size() + s->ready.size();
    out->device_bytes_in_use = s->dev_alloc.used();
    return QC_OK;
}

qc_status qc_server_destroy(qc_server* s) {
    if (!s) return QC_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->work_cv.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    (void)hipSetDevice(s->device);
    (void)hipDeviceSynchronize();
    for (auto& kv : s->all) {
        if (kv.second->uploaded) (void)hipEventDestroy(kv.second->uploaded);
        delete kv.second;
    }
    for (Batch& b : s->running)
        if (b.done) (void)hipEventDestroy(b.done);
    (void)hipStreamDestroy(s->copy_stream);
    (void)hipStreamDestroy(s->compute[0]);
    (void)hipStreamDestroy(s->compute[1]);
    (void)hipFree(s->dev_pool);
    (void)hipHostFree(s->pin_pool);
    delete s;
    return QC_OK;
}

}  // extern "C"
