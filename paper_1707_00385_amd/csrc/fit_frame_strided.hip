// fit_frame_strided.hip -- per-frame launches with the fit window sampled at a stride.
#include "fit_frame.h"

namespace qc {

hipError_t launch_frame_strided(const FitDesc& d, const RefitList& list, int cus, hipStream_t st,
                                hipEvent_t* ev) {
    return launch_frame<false, true>(d, list, cus, st, ev);
}

}  // namespace qc
