// fit_frame_strided_reject.hip -- per-frame launches with a strided fit window and the
// rejection variant of Eq. (11).
#include "fit_frame.h"

namespace qc {

hipError_t launch_frame_strided_reject(const FitDesc& d, const RefitList& list, int cus,
                                       hipStream_t st, hipEvent_t* ev) {
    return launch_frame<true, true>(d, list, cus, st, ev);
}

}  // namespace qc
