/*
 * qcurv.h -- C ABI of libqcurv.so: per-pixel principal curvatures of a range image by
 * robust iterative fitting of a parabolic quadric patch (Spek, Li, Drummond, "A Fast
 * Method For Computing Principal Curvatures From Range Images", Section 3).
 *
 * For every pixel the library back-projects its neighbourhood with pinhole intrinsics,
 * estimates an initial normal by regression over a small window (Section 3.2.1,
 * Eq. (7)), fits the patch z = A/2 x^2 + B x y + C/2 y^2 in a rotated and shifted local
 * frame by re-weighted Gauss-Newton (Section 3.2.3, Eqs. (8)-(11)), and returns the
 * principal curvatures k1 >= k2, the eigenvalues of [[A, B], [B, C]] (Section 3.1),
 * plus optionally the refined normal (Section 3.2.4), the fit residual and flags.
 *
 * Conventions shared by every entry point:
 *   - Units: depth in metres (or integer units of depth_scale metres for U16), output
 *     curvatures in inverse metres, residual in metres.  Depth is Z along the optical
 *     axis; pixel (u, v) back-projects to (Z(u-cx)/fx, Z(v-cy)/fy, Z).
 *   - Sign: the normal points away from the camera; a surface bulging toward the camera
 *     (the visible face of a sphere) has positive curvature.
 *   - Memory: every depth and output pointer is a device pointer owned by the caller.
 *     The library never frees caller memory.  It owns only the scratch inside a context.
 *   - Streams: `stream` is a hipStream_t passed as void* (NULL = the null stream).  The
 *     fit calls enqueue work and return; results are valid once the stream reaches them.
 *   - Errors: every call returns a qc_status.  Argument errors are reported before any
 *     work is enqueued.  A pixel that cannot be fitted is not an error: its outputs are
 *     NaN and its flags have QC_FLAG_VALID clear.
 *   - Threads: a context may be used from one host thread at a time.
 */
#ifndef QCURV_H
#define QCURV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QC_OK = 0,
    QC_ERR_INVALID_ARG = -1,   /* a pointer, size or parameter is out of range */
    QC_ERR_UNSUPPORTED = -2,   /* a valid request the library does not implement */
    QC_ERR_OOM = -3,           /* device scratch could not be allocated */
    QC_ERR_HIP = -4,           /* a HIP runtime call failed (see qc_last_hip_error) */
    QC_ERR_BUSY = -5,          /* the request cannot be admitted now; retry later */
    QC_ERR_INTERNAL = -6,
    QC_ERR_TOO_LARGE = -7      /* the frame needs more scratch than qc_fit_noalloc holds */
} qc_status;

/* Depth sample formats.  U16: unsigned integer units of depth_scale metres (Kinect
 * millimetres with depth_scale = 1e-3).  F16 / F32: metres.  0 (or a non-finite
 * float) means "no depth" (Section 4.1 excludes such pixels). */
typedef enum { QC_DEPTH_U16 = 0, QC_DEPTH_F16 = 1, QC_DEPTH_F32 = 2 } qc_depth_format;

/* Arithmetic of the fit.
 *   MIXED: FP32 fit of every pixel; pixels whose equilibrated normal equations are
 *          ill-conditioned or whose last update is large are recomputed entirely in
 *          FP64 on the GPU (same input, same steps).  At radius 1 (a 3x3 window: nine
 *          samples for six parameters) every pixel is fitted in FP64, as in FP64 mode.
 *   FP32:  FP32 only (flags still mark the pixels MIXED would recompute).
 *   FP64:  FP64 for every pixel. */
typedef enum { QC_PREC_MIXED = 0, QC_PREC_FP32 = 1, QC_PREC_FP64 = 2 } qc_precision;

/* Bits of the optional per-pixel flag byte. */
#define QC_FLAG_VALID 0x01u   /* outputs hold a fit */
#define QC_FLAG_FP64 0x02u    /* the fit was computed in FP64 */
#define QC_FLAG_ILLCOND 0x04u /* the FP32 fit was judged unreliable (see qc_params) */

#define QC_MAX_RADIUS 18      /* (2r+1)^2 = 37x37, the paper's largest patch */

typedef struct {
    float fx, fy;   /* focal lengths, pixels */
    float cx, cy;   /* principal point, pixels (pixel centres at integer u, v) */
} qc_intrinsics;

typedef struct {
    int32_t radius;          /* r: fit window (2r+1)^2, 1..QC_MAX_RADIUS (Section 3.2) */
    int32_t normal_radius;   /* initial-normal window (2r_n+1)^2, 1..QC_MAX_RADIUS; 3 = 7x7 */
    int32_t iterations;      /* fixed number of re-weighted Gauss-Newton steps, 0..64 */
    float k;                 /* robust constant of Eq. (11), m^2, > 0 */
    int32_t reject;          /* 0: weights k / (k + e^2) (Eq. (11)); 1: also reject (weight 0)
                                every neighbour with e^2 >= R, R = 2 x the unweighted mean
                                of e^2 over the window at the current parameters
                                (Section 3.2.3; nothing rejected when that mean is 0).
                                MIXED also recomputes in FP64 every pixel with an FP32
                                decision too close to R to be sure of (within a relative
                                1e-4, or closer than FP32 resolves e^2 in that window) or
                                an update after the first iteration beyond 5 step_max;
                                when the residual output is requested, the decisions of
                                its own pass count too. */
    float depth_scale;       /* metres per unit of U16 depth; ignored for F16/F32 */
    int32_t precision;       /* qc_precision */
    float cond_max;          /* MIXED: refit if the equilibrated pivot ratio exceeds this */
    float step_max;          /* MIXED: refit if the last update exceeds this, or the update
                                before it exceeds 1.5 times this, measured in window units:
                                radians, t_z / h_w and h_w * (A, B, C), with h_w = r Z / fx
                                the window half-extent at the pixel; for r > 7 (any stride)
                                the bound applied is step_max * (7/r)^2 */
    int32_t tile_width;      /* FP32 pass tile: 8, 16, 32 or 64 pixels wide (256 pixels);
                                0 = the width (and, for MIXED, the schedule) qc_tune
                                recorded for this configuration, else 16 and MIXED.  Results
                                do not depend on the width. */
    int32_t stride;          /* 1..radius: the fit window takes the pixels at offsets that
                                are multiples of `stride` within +-radius (the sparsely
                                sampled large patch of the timings of Section 4), i.e.
                                (2 floor(radius/stride) + 1)^2 samples; the initial-normal
                                window stays dense.  1 (default) = every pixel. */
} qc_params;

typedef struct {
    const void* depth;       /* device pointer, `height` rows of `pitch_bytes` */
    int32_t format;          /* qc_depth_format */
    int32_t width, height;   /* pixels, each >= 1 */
    int64_t pitch_bytes;     /* bytes between rows, >= width * sample size */
    qc_intrinsics K;
} qc_frame;

typedef struct {
    float* k1;               /* required: width*height floats, row-major, dense */
    float* k2;               /* required */
    float* normal;           /* optional (NULL): width*height*3 floats, xyz per pixel */
    float* residual;         /* optional: width*height floats, weighted RMS residual, m */
    uint8_t* flags;          /* optional: width*height bytes of QC_FLAG_* bits */
} qc_output;

typedef struct qc_context qc_context;

/* Defaults: r = 7, r_n = 3, T = 5, k = 1e-5 m^2, reject = 0, depth_scale = 1e-3, MIXED,
 * cond_max = 15, step_max = 0.1, tile_width = 0, stride = 1. */
void qc_params_default(qc_params* params);

/* Creates a context bound to HIP device `device`.  *ctx receives the handle. */
qc_status qc_create(qc_context** ctx, int device);

/* Waits for the context's internal work and frees its scratch. NULL is accepted. */
qc_status qc_destroy(qc_context* ctx);

/* Fits every pixel of one frame (Section 3.2).  Asynchronous on `stream`.  The
 * context's refit scratch is reused by the next call on the same context, so calls on
 * one context must be ordered on one stream.  The first call for a larger frame grows
 * that scratch: it waits for the stream of the context's previous fit (which must still
 * exist) and allocates; later calls for frames no larger, with kernel timing off, only
 * enqueue kernels on `stream` and may be captured in a HIP graph. */
qc_status qc_fit(qc_context* ctx, const qc_frame* frame, const qc_params* params,
                 const qc_output* out, void* stream);

/* qc_fit for callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation.  Same arguments, kernels and
 * results as qc_fit (bit for bit), but the FP64 recomputation list lives in a fixed
 * 2 MiB array of device memory that the library holds on every device it runs on
 * (looked up by qc_create, kept until the process ends) instead of the context's
 * scratch: the call allocates nothing, never synchronises, and only enqueues kernels on
 * `stream` (kernel timing does not apply to it).  The array holds the lists of frames of
 * up to 13,105 FP32-pass tiles of 256 pixels (about 3.3 Mpixels; 1280x720 needs 3,600
 * at the default tile width); a larger frame in MIXED or FP32 precision is refused with QC_ERR_TOO_LARGE before
 * any work is enqueued (FP64 precision uses no list and takes any size).
 * Every call on a device shares that device's array and leaves its contents behind (the
 * call clears what must start at zero with a kernel): calls that overlap on one device,
 * from any context or stream, race and give undefined results, so order them on one
 * stream (or with events).  qc_last_refit_count reports the last call's count while no
 * later call has reused the array. */
qc_status qc_fit_noalloc(qc_context* ctx, const qc_frame* frame, const qc_params* params,
                         const qc_output* out, void* stream);

/* One frame of a batch: its depth, parameters and outputs. */
typedef struct {
    qc_frame frame;
    qc_params params;
    qc_output out;
} qc_batch_item;

#define QC_MAX_BATCH 256

/* Fits up to QC_MAX_BATCH frames of any sizes, window radii and iteration counts with one
 * persistent FP32 launch over all their tiles and one persistent FP64 recomputation
 * launch (MIXED), replayed from a HIP graph the context captures once per batch slot (and
 * again, in the call, when a batch needs a larger list or a larger LDS staging region than
 * any before it; that call may wait for work in flight on the device).  Each item's
 * outputs equal, bit for bit, those of qc_fit on the same item.  All items must use the
 * same precision, MIXED or FP32 (FP64 frames go through qc_fit).  A batch holding an item
 * with reject = 1 or stride > 1 runs as per-frame launches in item order instead.  At most two batches
 * are in flight per context; a third call first waits for the oldest.  Asynchronous on
 * `stream`; the items array itself may be reused as soon as the call returns. */
qc_status qc_fit_batch(qc_context* ctx, const qc_batch_item* items, int32_t n, void* stream);

/* Autotuning of a frame configuration (size, radius, iterations, stride, reject): runs
 * qc_fit on `frame` with each FP32-pass tile width (8, 16, 32, 64) and, for a MIXED
 * request, also in FP64 throughout, `reps` times each after one warm-up call, timed with
 * HIP events on `stream`, writing into `out` (whose contents are then undefined).  It
 * records the fastest tile width and the schedule of MIXED requests for that
 * configuration (a candidate displaces width 16 and MIXED only when more than 1 % faster): QC_PREC_MIXED (the FP32 pass plus the FP64 recomputation of the pixels
 * it lists) or QC_PREC_FP64 (every pixel in FP64: more accurate, and faster where the FP32
 * pass would list many pixels).  Later requests of that configuration with tile_width 0
 * use the recorded width, and MIXED ones the recorded schedule (their flags then mark
 * every fitted pixel QC_FLAG_FP64; qc_fit_batch runs such items as per-frame FP64
 * launches).  `tile_width` and `schedule` (either may be NULL) receive them.  Synchronous. */
qc_status qc_tune(qc_context* ctx, const qc_frame* frame, const qc_params* params,
                  const qc_output* out, int32_t reps, void* stream, int32_t* tile_width,
                  int32_t* schedule);

/* Saves / loads the recorded configurations as text lines "width height radius
 * iterations stride reject tile_width schedule" (load also accepts the older five-field
 * lines "width height radius iterations tile_width", and merges into the context's table;
 * a malformed file changes nothing and returns QC_ERR_INVALID_ARG). */
qc_status qc_tune_save(qc_context* ctx, const char* path);
qc_status qc_tune_load(qc_context* ctx, const char* path);

/* ------------------------------------------------------------------------------------
 * Serving: frames from several producers are admitted by device memory, uploaded, and
 * fitted in batches (qc_fit_batch) as they arrive: a frame that arrives while batches run
 * joins the next batch, and up to two batches overlap on the GPU.  Results stay in device
 * memory until released.  A server owns its context from creation to destruction: the
 * context must not be used by the caller meanwhile.
 * ---------------------------------------------------------------------------------- */
typedef struct qc_server qc_server;

#define QC_OUT_NORMAL 1
#define QC_OUT_RESIDUAL 2
#define QC_OUT_FLAGS 4

typedef struct {
    size_t memory_budget;    /* device bytes for resident depth + outputs, >= one frame */
    int32_t max_batch;       /* frames per batch, 1..QC_MAX_BATCH */
    int32_t max_in_flight;   /* batches on the GPU at once, 1 or 2 */
    int32_t outputs;         /* QC_OUT_* bits; k1 and k2 are always produced */
    size_t staging_budget;   /* pinned host bytes holding submitted, not yet uploaded frames */
} qc_server_config;

typedef struct {
    const void* depth;       /* host pointer; copied before qc_server_submit returns */
    int32_t format;          /* qc_depth_format */
    int32_t width, height;
    int64_t pitch_bytes;
    qc_intrinsics K;
    qc_params params;        /* MIXED or FP32 */
    uint64_t tag;            /* returned with the completion */
} qc_request;

typedef struct {
    uint64_t ticket;
    uint64_t tag;
    int32_t status;          /* qc_status of the request */
    int32_t width, height;
    int64_t t_submit_ns;     /* steady-clock times of submission and completion */
    int64_t t_done_ns;
    const float* k1;         /* device pointers, valid until qc_server_release(ticket) */
    const float* k2;
    const float* normal;
    const float* residual;
    const uint8_t* flags;
} qc_completion;

/* Starts a server on `ctx` (its device) with the given configuration.  A batch holds
 * frames of one precision: the oldest ready frame's, with the ready frames of the other
 * precision left, in order, for the next batch. */
qc_status qc_server_create(qc_context* ctx, const qc_server_config* config, qc_server** out);

/* Queues one frame; *ticket identifies it.  Returns QC_ERR_BUSY when the pinned staging
 * cannot hold the frame now (retry after polling), QC_ERR_INVALID_ARG for a frame that
 * could never be admitted (larger than the memory budget). */
qc_status qc_server_submit(qc_server* server, const qc_request* request, uint64_t* ticket);

/* Returns up to `max` completions not yet returned, waiting up to `wait_us` microseconds
 * for the first one; *n receives the count. */
qc_status qc_server_poll(qc_server* server, qc_completion* out, int32_t max, int32_t* n,
                         int64_t wait_us);

/* Frees a completed request's device buffers. */
qc_status qc_server_release(qc_server* server, uint64_t ticket);

/* Counters: submitted, completed, queued (not yet on the GPU), bytes of device memory in
 * use, batches launched. */
typedef struct {
    uint64_t submitted, completed, queued, batches;
    size_t device_bytes_in_use;
} qc_server_stats;
qc_status qc_server_get_stats(qc_server* server, qc_server_stats* out);

/* Waits for all submitted frames, stops the server and frees its memory.  Frames that
 * still wait for device memory held by unreleased results, once nothing else is on the GPU,
 * are not fitted: they complete with QC_ERR_BUSY (no release can come during destruction). */
qc_status qc_server_destroy(qc_server* server);

/* Number of pixels recomputed in FP64 by the most recent qc_fit or qc_fit_noalloc on
 * this context (MIXED), or flagged (FP32).  Synchronises with that call's stream. */
qc_status qc_last_refit_count(qc_context* ctx, uint32_t* count);

/* Kernel timing.  With timing enabled, every qc_fit on the context records HIP events
 * around its kernels on the call's stream: the FP32 (or FP64-only) fitting pass and the
 * FP64 recomputation pass.  qc_get_timing waits for the recorded events, returns the
 * sums since the last reset (milliseconds) and, if `reset` is non-zero, clears them.
 * The events come from a pool of 1024 triples that the first qc_set_timing(ctx, 1)
 * creates; a timed call only records three of them, except that once all are recorded
 * and unread the call first waits for the oldest.  Off by default. */
typedef struct {
    uint64_t calls;       /* qc_fit calls timed */
    double fit_ms;        /* summed duration of the tiled fitting pass */
    double refit_ms;      /* summed duration of the FP64 recomputation pass (MIXED) */
} qc_timing;

qc_status qc_set_timing(qc_context* ctx, int enable);
qc_status qc_get_timing(qc_context* ctx, qc_timing* out, int reset);

/* The HIP error code behind the last QC_ERR_HIP on this context (0 if none). */
int qc_last_hip_error(qc_context* ctx);

/* A static description of a status code. */
const char* qc_status_string(qc_status status);

#ifdef __cplusplus
}
#endif

#endif /* QCURV_H */
