// Backward of the field MLPs and the FP64 gradient-check forms.
#include "r360_internal.h"

namespace r360 {

hipError_t launch_mlp_backward(const r360_scene*, const Workspace&, int, float*, hipStream_t) {
    return hipErrorNotSupported;
}
hipError_t launch_gradcheck_forward(const r360_scene*, const Workspace&, const double*, int64_t, double*, hipStream_t) {
    return hipErrorNotSupported;
}
hipError_t launch_gradcheck_backward(const r360_scene*, const Workspace&, const double*, int64_t, const double*,
                                     double*, hipStream_t) {
    return hipErrorNotSupported;
}

}  // namespace r360
