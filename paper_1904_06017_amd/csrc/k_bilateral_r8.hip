// Aggregation kernels instantiated for window radius R = 8.
#include "bilateral_impl.h"

namespace stereo {
hipError_t launch_bilateral_r8(const Plan& P, const BilArgs& a, int mode, hipStream_t s) {
  return bil::launch_r<8>(P, a, mode, s);
}
hipError_t launch_bilateral_persistent_r8(stereo_dtype gdt, int levels, const void* pairs,
                                           const int* tiles, int n_tiles, unsigned int* counter,
                                           int n_groups, hipStream_t s) {
  return bil::launch_persistent_r<8>(gdt, levels, static_cast<const bil::BilPair*>(pairs),
                                        tiles, n_tiles, counter, n_groups, s);
}
}  // namespace stereo
