// Backward of the joint bilateral filter (placeholder until the kernel lands).
#include "jbfd_internal.hpp"

namespace jbfd {

size_t backward_ws_bytes(int32_t H, int32_t W) {
    return (size_t)256;
}

hipError_t launch_densify_backward(const float *, const uint8_t *, const uint8_t *,
                                   int32_t, int32_t, const FilterParams &, float,
                                   float, const float *, const float *,
                                   const float *, float *, double *, void *,
                                   hipStream_t) {
    return hipErrorNotSupported;
}

}  // namespace jbfd
