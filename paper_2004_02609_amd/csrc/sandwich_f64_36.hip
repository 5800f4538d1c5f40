// Instantiation of one x sandwich variant (double, 3 inputs, 6 outputs); kernel in sandwich_impl.hpp.
#include "sandwich_impl.hpp"

namespace vc {
template hipError_t launch_sandwich_v<double, 3, 6, 0>(const void*, void*, const void*, const SandArgs&, const void*,
                                                const void*, const uint8_t*, int, size_t,
                                                int, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_sandwich_v<double, 3, 6, 1>(const void*, void*, const void*, const SandArgs&, const void*,
                                                const void*, const uint8_t*, int, size_t,
                                                int, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_sandwich_multi_v<double, 3, 6>(const SandScene*, int, int, const int*, const int*, int,
                                                            size_t, int, hipStream_t);
}  // namespace vc
