// Instantiation of the y pass (double); kernel in ypass_impl.hpp.
#include "ypass_impl.hpp"

namespace vc {
template hipError_t launch_ypass<double>(void*, const YArgs&, const void*, const uint8_t*, const uint8_t*, int, int,
                                      hipStream_t);
template bool ypass_args_ok<double>(const YArgs&, int, bool, size_t*, int);
template hipError_t launch_ypass_multi<double>(const YScene*, int, int, int, int, size_t, const int*, const int*,
                                            hipStream_t);
}  // namespace vc
