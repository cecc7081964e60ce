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
    int32_t tile_w;          // FP32 pass tile width: 8, 16, 32 or 64 (256 / tile_w rows)
    float* k1;
    float* k2;
    float* normal;
    float* residual;
    uint8_t* flags;
};

// Enqueues the whole fit of one frame on `stream`.  MIXED / FP32: a tiled FP32 pass that
// lists the tiles holding unreliable fits (`entries`: refit_capacity() tile indices;
// `masks`: 4 x refit_capacity() 64-bit words, a 256-bit pixel mask per entry; `counts`:
// 4 words, zeroed here, counts[1] = listed pixels), then for MIXED an FP64 pass over those
// pixels.  FP64: one tiled FP64 pass over every pixel.  `events` (optional, 3 entries)
// are recorded before the fitting pass, after it, and after the recomputation pass.
hipError_t launch_fit(const FitDesc& d, uint32_t* entries, uint64_t* masks, uint32_t* counts,
                      hipStream_t stream, hipEvent_t* events = nullptr);

// Tile entries needed for a width x height frame with tiles tile_w wide (masks: 4x).
int64_t refit_capacity(int width, int height, int tile_w);
bool valid_tile_width(int tile_w);

// Enqueues the fit of a batch of frames: `frames` (device, FP32 MIXED/FP32 descriptors,
// ordered by decreasing work per tile), `first_tile` (device, n + 1 prefix sums of the
// frames' tile counts), `header` (device: [0] = n frames, [1] = 1 to recompute listed
// pixels in FP64), all read when the kernels run, so the same launches can be captured
// once and replayed with new contents.  One persistent FP32 pass of `workgroups`
// workgroups over all tiles, then one persistent FP64 pass over the listed tiles.
// Entry capacity: first_tile[n] (masks 4x); at most 256 frames.
hipError_t launch_fit_batch(const FitDesc* frames, const uint32_t* first_tile,
                            const uint32_t* header, int workgroups, uint32_t* entries,
                            uint64_t* masks, uint32_t* counts, hipStream_t stream,
                            hipEvent_t* events = nullptr);

// Dynamic LDS of the batched kernels (largest tile shape at the largest radius).
size_t batch_lds_bytes();

}  // namespace qc
