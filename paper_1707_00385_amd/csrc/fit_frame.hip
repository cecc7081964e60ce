// fit_frame.hip -- per-frame launches (default weights), the list helpers, and the entry
// that picks the variant.
#include "fit_frame.h"

namespace qc {

int64_t refit_capacity(int width, int height, int tile_w) {
    const int64_t th = 256 / tile_w;
    return ((width + tile_w - 1) / tile_w) * static_cast<int64_t>((height + th - 1) / th);
}

bool valid_tile_width(int tile_w) {
    return tile_w == 8 || tile_w == 16 || tile_w == 32 || tile_w == 64;
}

// A tile lists at most 256 pixels, i.e. 256 / kChunk = 16 chunks.
size_t refit_list_bytes(int64_t tiles) {
    return static_cast<size_t>(tiles) * (4 + 256 / kChunk) * sizeof(uint64_t);
}

RefitList refit_list(void* storage, int64_t tiles, uint32_t* counts) {
    RefitList l;
    l.masks = static_cast<uint64_t*>(storage);
    l.chunks = l.masks + 4 * static_cast<size_t>(tiles);
    l.counts = counts;
    return l;
}

hipError_t launch_fit(const FitDesc& d, const RefitList& list, int cus, hipStream_t stream,
                      hipEvent_t* events) {
    if (d.precision != 2) {
        hipLaunchKernelGGL(zero_counts, dim3(1), dim3(64), 0, stream, list.counts);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (d.stride > 1)
        return d.reject ? launch_frame_strided_reject(d, list, cus, stream, events)
                        : launch_frame_strided(d, list, cus, stream, events);
    return d.reject ? launch_frame_reject(d, list, cus, stream, events)
                    : launch_frame<false, false>(d, list, cus, stream, events);
}

}  // namespace qc
