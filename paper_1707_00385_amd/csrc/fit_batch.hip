// fit_batch.hip -- the batched form: one persistent FP32 pass over the tiles of many
// frames and one persistent FP64 pass over their listed pixels.
#include "fit_device.h"

namespace qc {
namespace {

// Persistent FP32 pass over a batch of frames.  Tiles are numbered frame after frame
// (frames ordered by the host from most to least work per tile; first_tile[f] is the
// number of the frame's first tile, first_tile[n] the total).  Workgroup b starts on tile
// b (the grid is the resident capacity, so no atomic is asked by the whole grid at once)
// and then takes the next tile number beyond the first round from counts[2] until none is
// left, so all frames share one launch.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(QC_F32_WAVES_PER_EU)))
void fit_batch_f32(const FitDesc* frames, const uint32_t* first_tile, const uint32_t* header,
                   RefitList list) {
    __shared__ uint32_t next;
    const uint32_t nf = header[0];
    if (nf == 0) return;
    const uint32_t total = first_tile[nf];
    for (uint32_t t = blockIdx.x; t < total;) {
        uint32_t lo = 0, hi = nf - 1;   // the frame holding tile t
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) / 2;
            if (first_tile[mid] <= t) lo = mid; else hi = mid - 1;
        }
        lo = __builtin_amdgcn_readfirstlane(lo);
        const FitDesc d = frames[lo];
        const int local = static_cast<int>(t - first_tile[lo]);
        const int across = tiles_across(d);
        with_radius(d.radius, [&](auto rc) {
            fit_tile_body<float, decltype(rc)::value>(d, local % across, local / across, lo, list);
        });
        if (threadIdx.x == 0) next = atomicAdd(&list.counts[2], 1u) + gridDim.x;
        __syncthreads();   // `next` is written, and the next tile may re-stage LDS
        t = __builtin_amdgcn_readfirstlane(next);
        __syncthreads();   // every lane has read `next` before thread 0 writes it again
    }
}

// Persistent FP64 pass over the listed pixels of all frames of a batch, one wave per
// workgroup, as the per-frame recomputation: each chunk's tile is staged in LDS.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(QC_F64_WAVES_PER_EU)))
void refit_batch_f64(const FitDesc* frames, RefitList list) {
    extern __shared__ float2 region[];
    const uint32_t ranks = list.counts[0];
    const LaneGroup<kRefitLanes> grp{static_cast<int>(threadIdx.x % kRefitLanes)};
    for (uint32_t base = first_ranks(); base < ranks; base = next_ranks(&list.counts[3])) {
        const Chunk ck = chunk_at(list, base);
        const uint64_t* m = list.masks + 4 * static_cast<size_t>(ck.slot);
        const uint64_t w[4] = {m[0], m[1], m[2], m[3]};
        const FitDesc d = frames[ck.entry >> 24];
        with_radius(d.radius, [&](auto rc) {
            refit_chunk<decltype(rc)::value>(d, ck.entry & 0xffffffu, w,
                                             static_cast<int>(ck.first + threadIdx.x / kRefitLanes), grp, region);
        });
    }
}

}  // namespace

size_t batch_lds_bytes() {
    // largest staging region over the supported tile shapes at the largest halo
    size_t m = 0;
    for (int tw = 8; tw <= 64; tw *= 2) {
        const size_t b = lds_bytes(tw, 256 / tw, kMaxRadius);
        m = b > m ? b : m;
    }
    return m;
}

size_t batch_refit_lds_bytes(const FitDesc& d) {
    const int halo = d.radius > d.normal_radius ? d.radius : d.normal_radius;
    return lds_bytes(d.tile_w, 256 / d.tile_w, halo);
}

hipError_t launch_fit_batch(const FitDesc* frames, const uint32_t* first_tile,
                            const uint32_t* header, int cus, size_t refit_lds,
                            const RefitList& list, hipStream_t stream, hipEvent_t* events) {
    // both passes: as many workgroups as can be resident at once, each starting on its own
    // first tile / chunk
    const size_t lds = batch_lds_bytes();
    int f32_per_cu = 0, f64_per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&f32_per_cu, fit_batch_f32, 256, lds) != hipSuccess ||
        f32_per_cu < 1)
        f32_per_cu = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&f64_per_cu, refit_batch_f64, 64, refit_lds) != hipSuccess ||
        f64_per_cu < 1)
        f64_per_cu = 1;
    hipError_t e;
    hipLaunchKernelGGL(zero_counts, dim3(1), dim3(64), 0, stream, list.counts);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (events && (e = hipEventRecord(events[0], stream)) != hipSuccess) return e;
    hipLaunchKernelGGL(fit_batch_f32, dim3(f32_per_cu * cus), dim3(256), lds, stream, frames, first_tile,
                       header, list);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (events && (e = hipEventRecord(events[1], stream)) != hipSuccess) return e;
    hipLaunchKernelGGL(refit_batch_f64, dim3(f64_per_cu * cus), dim3(64), refit_lds, stream, frames, list);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (events && (e = hipEventRecord(events[2], stream)) != hipSuccess) return e;
    return hipSuccess;
}

}  // namespace qc
