// fit_frame_reject.hip -- per-frame launches of the rejection variant of Eq. (11).
#include "fit_frame.h"

namespace qc {

hipError_t launch_frame_reject(const FitDesc& d, const RefitList& list, int cus, hipStream_t st,
                               hipEvent_t* ev) {
    return launch_frame<true, false>(d, list, cus, st, ev);
}

}  // namespace qc
