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
    QC_ERR_UNSUPPORTED = -2,   /* a valid request this build does not implement */
    QC_ERR_OOM = -3,           /* device scratch could not be allocated */
    QC_ERR_HIP = -4,           /* a HIP runtime call failed (see qc_last_hip_error) */
    QC_ERR_BUSY = -5,          /* the request cannot be admitted now; retry later */
    QC_ERR_INTERNAL = -6
} qc_status;

/* Depth sample formats.  U16: unsigned integer units of depth_scale metres (Kinect
 * millimetres with depth_scale = 1e-3).  F16 / F32: metres.  0 (or a non-finite
 * float) means "no depth" (Section 4.1 excludes such pixels). */
typedef enum { QC_DEPTH_U16 = 0, QC_DEPTH_F16 = 1, QC_DEPTH_F32 = 2 } qc_depth_format;

/* Arithmetic of the fit.
 *   MIXED: FP32 fit of every pixel; pixels whose equilibrated normal equations are
 *          ill-conditioned or whose last update is large are recomputed entirely in
 *          FP64 on the GPU (same input, same steps).
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
    int32_t reject;          /* 0 only: the rejection variant of Eq. (11) is not built */
    float depth_scale;       /* metres per unit of U16 depth; ignored for F16/F32 */
    int32_t precision;       /* qc_precision */
    float cond_max;          /* MIXED: refit if the equilibrated pivot ratio exceeds this */
    float step_max;          /* MIXED: refit if the last update's max-norm exceeds this */
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

/* Defaults: r = 7, r_n = 3, T = 5, k = 1e-5 m^2, depth_scale = 1e-3, MIXED,
 * cond_max = 30, step_max = 0.1. */
void qc_params_default(qc_params* params);

/* Creates a context bound to HIP device `device`.  *ctx receives the handle. */
qc_status qc_create(qc_context** ctx, int device);

/* Waits for the context's internal work and frees its scratch. NULL is accepted. */
qc_status qc_destroy(qc_context* ctx);

/* Fits every pixel of one frame (Section 3.2).  Asynchronous on `stream`.  The
 * context's refit scratch is reused by the next call on the same context, so calls on
 * one context must be ordered on one stream. */
qc_status qc_fit(qc_context* ctx, const qc_frame* frame, const qc_params* params,
                 const qc_output* out, void* stream);

/* Number of pixels recomputed in FP64 by the most recent qc_fit on this context
 * (MIXED), or flagged (FP32).  Synchronises with that call's stream. */
qc_status qc_last_refit_count(qc_context* ctx, uint32_t* count);

/* Kernel timing.  With timing enabled, every qc_fit on the context records HIP events
 * around its kernels on the call's stream: the FP32 (or FP64-only) fitting pass and the
 * FP64 recomputation pass.  qc_get_timing waits for the recorded events, returns the
 * sums since the last reset (milliseconds) and, if `reset` is non-zero, clears them.
 * Timing adds two or three event records per call and is off by default. */
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
