// Mixed-precision forms (FP64 phase, FP32 transcendentals and likelihood).
#include "rlf_internal.h"

namespace rlf {

hipError_t launch_model_mixed(const ModelArgs &, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_extract_mixed(const ExtractArgs &, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_fit_mixed(const FitArgs &, hipStream_t) { return hipErrorNotSupported; }

}  // namespace rlf
