// fit_frame.h -- per-frame kernels: the FP32 tiled pass, the FP64 pass over every pixel
// and the FP64 recomputation of listed pixels, templated on the window radius (in samples),
// the rejection variant (REJ) and a strided fit window (STR); each of fit_frame*.hip
// instantiates one (REJ, STR) variant.
#pragma once

#include <atomic>

#include "fit_device.h"

namespace qc {

hipError_t launch_frame_reject(const FitDesc& d, const RefitList& list, int cus, hipStream_t st,
                               hipEvent_t* ev);
hipError_t launch_frame_strided(const FitDesc& d, const RefitList& list, int cus, hipStream_t st,
                                hipEvent_t* ev);
hipError_t launch_frame_strided_reject(const FitDesc& d, const RefitList& list, int cus,
                                       hipStream_t st, hipEvent_t* ev);

namespace {

// The tile a workgroup of a per-frame pass fits.  Workgroups are dispatched to the eight
// XCDs in turn (workgroup w to XCD w mod 8), each XCD with its own L2; the tiles are dealt
// out so that XCD x takes the x-th contiguous eighth of the frame's tiles in row-major
// order, and neighbouring tiles, which stage overlapping halos, mostly share an L2.  A
// bijection of [0, tiles): results do not depend on it.
__device__ __forceinline__ int2 xcd_tile() {
    constexpr uint32_t kXcds = 8;
    const uint32_t n = gridDim.x * gridDim.y;
    const uint32_t w = blockIdx.y * gridDim.x + blockIdx.x;
    const uint32_t x = w % kXcds, k = w / kXcds, q = n / kXcds, rem = n % kXcds;
    const uint32_t t = (x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q) + k;
    return make_int2(static_cast<int>(t % gridDim.x), static_cast<int>(t / gridDim.x));
}

// FP32 pass over one frame: one 256-lane workgroup per tile (REJ: the rejection variant
// of Eq. (11)).  Its unrolled rows with FP32 sums per row pair need ~150 registers: 3 waves per
// SIMD (the pass runs as fast at 2, 3 or 4 waves per SIMD).
template <int R, bool REJ, bool STR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(QC_F32_WAVES_PER_EU)))
void fit_tile_f32(FitDesc d, RefitList list) {
    const int2 t = xcd_tile();
    fit_tile_body<float, R, REJ, STR>(d, t.x, t.y, 0u, list);
}

// FP64 pass over every pixel of one frame: tiles 16 pixels wide, QC_F64_BLOCK lanes.
#ifndef QC_F64_BLOCK
#define QC_F64_BLOCK 64
#endif
#ifndef QC_F64_TILE_WAVES
#define QC_F64_TILE_WAVES 3
#endif
template <int R, bool REJ, bool STR>
__global__ __launch_bounds__(QC_F64_BLOCK) __attribute__((amdgpu_waves_per_eu(QC_F64_TILE_WAVES)))
void fit_tile_f64(FitDesc d, RefitList list) {
    const int2 t = xcd_tile();
    fit_tile_body<double, R, REJ, STR>(d, t.x, t.y, 0u, list);
}

// FP64 pass over the listed pixels of one frame; one wave per workgroup, persistent
// (waves loop until the ranks run out).  For each chunk the wave stages its tile plus halo
// in LDS, as the FP32 pass did, and fits the chunk's pixels from there.
template <int R, bool REJ, bool STR>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(QC_F64_WAVES_PER_EU)))
void refit_f64(FitDesc d, RefitList list) {
    extern __shared__ float2 region[];
    const uint32_t ranks = list.counts[0];
    const int tw = d.tile_w, th = 256 / tw;
    const int halo = max(R * (STR ? d.stride : 1), d.normal_radius);
    const int pitch = tw + 2 * halo;
    const int across = tiles_across(d);
    const LaneGroup<kRefitLanes> grp{static_cast<int>(threadIdx.x % kRefitLanes)};
    for (uint32_t base = first_ranks(); base < ranks; base = next_ranks(&list.counts[3])) {
        const Chunk ck = chunk_at(list, base);
        // the entry's mask is read before the tile is staged: both reads are in flight together
        const uint64_t* m = list.masks + 4 * static_cast<size_t>(ck.slot);
        const uint64_t w0 = m[0], w1 = m[1], w2 = m[2], w3 = m[3];
        const uint32_t tile = ck.entry & 0xffffffu;
        const int bx = static_cast<int>(tile % across) * tw, by = static_cast<int>(tile / across) * th;
        stage_region_wave(d, region, bx - halo, by - halo, pitch, th + 2 * halo);
        const int t = listed_thread(w0, w1, w2, w3, static_cast<int>(ck.first + threadIdx.x / kRefitLanes));
        if (t >= 0) {
            const int lx = t % tw, ly = t / tw;
            const float2* centre = region + (ly + halo) * pitch + (lx + halo);
            PixelFit<double> r;
            if constexpr (STR) {
                r = fit_pixel<double, R, kRefitLanes, REJ, true>(
                    d, LdsSource{centre, pitch}, LdsStridedSource{centre, pitch, d.stride}, bx + lx,
                    by + ly, centre->x, d.residual != nullptr, grp);
            } else {
                const LdsSource src{centre, pitch};
                r = fit_pixel<double, R, kRefitLanes, REJ>(d, src, src, bx + lx, by + ly, centre->x,
                                                           d.residual != nullptr, grp);
            }
            if (grp.part == 0) store_pixel(d, static_cast<int64_t>(by + ly) * d.width + bx + lx, r);
        }
        __syncthreads();   // the next chunk re-stages the region
    }
}

// Grid of a persistent one-wave FP64 pass: as many workgroups as can be resident at once
// with `lds` bytes each, so that every wave starts on its own first chunk (a workgroup
// waiting for a slot would hold its first chunk back until the others have drained the
// counter).  Any grid is correct; this one is cached per kernel for the last LDS size.
template <auto Kernel>
int resident_waves(size_t lds, int cus) {
    static std::atomic<uint64_t> cache{~uint64_t{0}};   // (lds << 32) | workgroups per CU
    const uint64_t c = cache.load(std::memory_order_relaxed);
    int n = static_cast<int>(c & 0xffffffffu);
    if ((c >> 32) != lds) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, Kernel, 64, lds) != hipSuccess || n < 1) n = 1;
        cache.store((static_cast<uint64_t>(lds) << 32) | static_cast<uint32_t>(n), std::memory_order_relaxed);
    }
    return n * cus;
}

template <int R, bool REJ, bool STR>
hipError_t launch_variant(const FitDesc& d, const RefitList& list, int cus, hipStream_t st,
                          hipEvent_t* ev) {
    const int reach = R * (STR ? d.stride : 1);   // pixels from the centre to the last sample
    const int halo = reach > d.normal_radius ? reach : d.normal_radius;
    hipError_t e;
    if (ev && (e = hipEventRecord(ev[0], st)) != hipSuccess) return e;
    if (d.precision == 2) {
        FitDesc d64 = d;
        d64.tile_w = kTileW;
        constexpr int th64 = QC_F64_BLOCK / kTileW;
        dim3 grid((d.width + kTileW - 1) / kTileW, (d.height + th64 - 1) / th64);
        hipLaunchKernelGGL((fit_tile_f64<R, REJ, STR>), grid, dim3(QC_F64_BLOCK), lds_bytes(kTileW, th64, halo),
                           st, d64, list);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (ev && (e = hipEventRecord(ev[1], st)) != hipSuccess) return e;
        if (ev && (e = hipEventRecord(ev[2], st)) != hipSuccess) return e;
        return hipSuccess;
    }
    const int tw = d.tile_w, th = 256 / tw;
    const size_t lds = lds_bytes(tw, th, halo);
    dim3 grid((d.width + tw - 1) / tw, (d.height + th - 1) / th);
    hipLaunchKernelGGL((fit_tile_f32<R, REJ, STR>), grid, dim3(256), lds, st, d, list);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[1], st)) != hipSuccess) return e;
    if (d.precision == 0) {
        hipLaunchKernelGGL((refit_f64<R, REJ, STR>), dim3(resident_waves<refit_f64<R, REJ, STR>>(lds, cus)),
                           dim3(64), lds, st, d, list);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (ev && (e = hipEventRecord(ev[2], st)) != hipSuccess) return e;
    return hipSuccess;
}

template <bool REJ, bool STR, int... Rs>
hipError_t dispatch_radius(int r, const FitDesc& d, const RefitList& list, int cus,
                           hipStream_t st, hipEvent_t* ev, std::integer_sequence<int, Rs...>) {
    hipError_t e = hipErrorInvalidValue;
    (void)((r == Rs + 1 ? (e = launch_variant<Rs + 1, REJ, STR>(d, list, cus, st, ev), true) : false) || ...);
    return e;
}

// The per-frame kernels for every window size: with (REJ) or without rejection, the window
// dense or (STR) sampled every d.stride pixels, r / stride samples either side.
template <bool REJ, bool STR>
hipError_t launch_frame(const FitDesc& d, const RefitList& list, int cus, hipStream_t st,
                        hipEvent_t* ev) {
    const int samples = STR ? d.radius / d.stride : d.radius;
    return dispatch_radius<REJ, STR>(samples, d, list, cus, st, ev,
                                     std::make_integer_sequence<int, kMaxRadius>{});
}

}  // namespace
}  // namespace qc
