// api_internal.h -- helpers of the C ABI layer shared with the serving loop.
#pragma once

#include "qcurv.h"

namespace qc {

// The HIP device a context was created on.
int context_device(const qc_context* ctx);

// The argument checks of qc_fit for one frame and its parameters.
qc_status check_request(const qc_frame* frame, const qc_params* params);

}  // namespace qc
