// Aggregation kernels instantiated for window radius R = 2.
#include "bilateral_mfma16_bwd.h"

namespace stereo {
hipError_t launch_bilateral_r2(const Plan& P, const BilArgs& a, int mode, hipStream_t s) {
  if ((mode == 1 || mode == 2) && a.h2) return bilh::launch_args<2>(P, a, mode, s);
  if ((mode == 1 || mode == 2) && P.agg_engine == 1 && a.quad)
    return bilm::launch_args<2>(P, a, mode, s);
  return bil::launch_r<2>(P, a, mode, s);
}
hipError_t launch_bilateral_persistent_r2(int engine, stereo_dtype gdt, int levels, const void* pairs,
                                           const int* tiles, int n_tiles, unsigned int* counter,
                                           int n_groups, hipStream_t s) {
  const bil::BilPair* p = static_cast<const bil::BilPair*>(pairs);
  if (engine == 2) return bilh::launch_queue_r<2>(gdt, p, tiles, n_tiles, counter, n_groups, s);
  if (engine == 1) return bilm::launch_queue_r<2>(gdt, p, tiles, n_tiles, counter, n_groups, s);
  return bil::launch_persistent_r<2>(gdt, levels, p, tiles, n_tiles, counter, n_groups, s);
}
hipError_t launch_bwd16_r2(const Plan& P, const BilArgs& a, int pass, hipStream_t s) {
  return bilh::launch_bwd_args<2>(P, a, pass, s);
}
}  // namespace stereo
