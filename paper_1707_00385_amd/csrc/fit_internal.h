// fit_internal.h -- launch interface between the C ABI layer and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qc {

// One frame's fit as the kernels see it: plain values and device pointers only.
struct FitDesc {
    const void* depth;
    int32_t format;          // qc_depth_format
    int32_t width, height;
    int64_t pitch;           // bytes per depth row
    float fx, fy, cx, cy;
    float scale;             // metres per depth unit (1 for F16 / F32)
    int32_t radius, normal_radius, iterations;
    float k;
    float cond_max, step_max;
    int32_t precision;       // qc_precision
    float* k1;
    float* k2;
    float* normal;
    float* residual;
    uint8_t* flags;
};

// Enqueues the whole fit of one frame on `stream`.  MIXED / FP32: a tiled FP32 pass that
// lists the 16x4 pixel blocks holding unreliable fits (`entries`, with 64-bit lane
// `masks`, both of refit_capacity() entries; counts[0] = entries, counts[1] = pixels,
// zeroed here), then for MIXED an FP64 pass over those pixels.  FP64: one tiled FP64
// pass over every pixel.
// `events` (optional, 3 entries) are recorded before the fitting pass, after it, and
// after the recomputation pass.
hipError_t launch_fit(const FitDesc& d, uint32_t* entries, uint64_t* masks, uint32_t* counts,
                      hipStream_t stream, hipEvent_t* events = nullptr);

// Entries needed by launch_fit for a width x height frame.
int64_t refit_capacity(int width, int height);

}  // namespace qc
