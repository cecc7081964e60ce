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
    int32_t reject;          // 1: rejection variant of Eq. (11) (per-frame kernels only)
    int32_t stride;          // fit window sampled every `stride` pixels (per-frame kernels only)
    int32_t tile_w;          // FP32 pass tile width: 8, 16, 32 or 64 (256 / tile_w rows)
    float* k1;
    float* k2;
    float* normal;
    float* residual;
    uint8_t* flags;
};

// List of the pixels whose FP32 fit is to be recomputed in FP64 (device memory).  The
// FP32 pass appends one entry per tile holding such pixels; the FP64 pass takes the
// listed pixels by rank, so its work does not depend on how they cluster in tiles.
struct RefitList {
    uint64_t* masks;     // 4 words per entry: the listed pixels (bit t = thread t of the tile)
    uint64_t* chunks;    // per 16 ranks (16 per entry at most), all the FP64 pass needs to
                         // start on them: (entry << 32) | (slot << 8) | c, with entry =
                         // (frame << 24) | tile index within the frame, slot the entry's
                         // index in `masks`, c the chunk's index within the entry
    uint32_t* counts;    // kCountWords words, 8-byte aligned, zeroed by every launch:
                         // [0] ranks handed out (each entry's pixel count rounded up to a
                         // multiple of 16, so that 16 consecutive ranks never span two
                         // entries) and [1] entries (one 64-bit counter, low word first),
                         // [2] next tile of a batched FP32 pass, [3] next rank of the FP64
                         // pass, [4] listed pixels
};
constexpr int kCountWords = 8;

// Bytes of the masks and the chunk table for `tiles` entries, and the list carved
// out of them.
size_t refit_list_bytes(int64_t tiles);
RefitList refit_list(void* storage, int64_t tiles, uint32_t* counts);

// Enqueues the whole fit of one frame on `stream`.  MIXED / FP32: a tiled FP32 pass
// (MIXED: it lists the pixels whose fit is unreliable instead of storing them; the list
// needs refit_capacity() entries), then for MIXED a persistent FP64 pass sized for `cus`
// compute units over the listed pixels.  FP64: one tiled FP64 pass over every pixel.
// `events` (optional, 3 entries) are recorded before the FP32 pass, after it, and after
// the FP64 pass.
hipError_t launch_fit(const FitDesc& d, const RefitList& list, int cus, hipStream_t stream,
                      hipEvent_t* events = nullptr);

// Tile entries needed for a width x height frame with tiles tile_w wide.
int64_t refit_capacity(int width, int height, int tile_w);
bool valid_tile_width(int tile_w);

// Enqueues the fit of a batch of frames: `frames` (device, FP32 MIXED/FP32 descriptors,
// ordered by decreasing work per tile), `first_tile` (device, n + 1 prefix sums of the
// frames' tile counts), `header` (device: [0] = n frames), all read when the kernels run,
// so the same launches can be captured once and replayed with new contents.  One
// persistent FP32 pass over all tiles, then one persistent FP64
// pass over the listed pixels of all frames.  List capacity: first_tile[n] entries; at
// most 256 frames.
// `refit_lds`: dynamic LDS of the FP64 pass's one-wave workgroups, at least the largest
// batch_refit_lds_bytes() over the batch's frames.
hipError_t launch_fit_batch(const FitDesc* frames, const uint32_t* first_tile,
                            const uint32_t* header, int cus, size_t refit_lds,
                            const RefitList& list, hipStream_t stream, hipEvent_t* events = nullptr);

// Dynamic LDS of the batched FP32 pass (largest tile shape at the largest radius), and
// the region the FP64 pass stages for a tile of frame `d`.
size_t batch_lds_bytes();
size_t batch_refit_lds_bytes(const FitDesc& d);

}  // namespace qc
