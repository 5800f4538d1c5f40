// Instantiation of one x sandwich variant (float, 6 inputs, 3 outputs); kernel in sandwich_impl.hpp.
#include "sandwich_impl.hpp"

namespace vc {
template hipError_t launch_sandwich_v<float, 6, 3, 0>(const void*, void*, const void*, const SandArgs&, const void*,
                                                const void*, const uint8_t*, int, size_t,
                                                int, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_sandwich_v<float, 6, 3, 1>(const void*, void*, const void*, const SandArgs&, const void*,
                                                const void*, const uint8_t*, int, size_t,
                                                int, hipStream_t, hipEvent_t, hipEvent_t);
}  // namespace vc
