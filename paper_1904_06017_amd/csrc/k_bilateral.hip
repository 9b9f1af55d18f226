// Dispatch of the aggregation launches over the compiled window radii.
#include "bilateral_mfma16.h"

namespace stereo {
hipError_t launch_bilateral_r1(const Plan&, const BilArgs&, int, hipStream_t);
hipError_t launch_bilateral_persistent_r1(int, stereo_dtype, int, const void*, const int*, int, unsigned int*, int, hipStream_t);
hipError_t launch_bilateral_r2(const Plan&, const BilArgs&, int, hipStream_t);
hipError_t launch_bilateral_persistent_r2(int, stereo_dtype, int, const void*, const int*, int, unsigned int*, int, hipStream_t);
hipError_t launch_bilateral_r3(const Plan&, const BilArgs&, int, hipStream_t);
hipError_t launch_bilateral_persistent_r3(int, stereo_dtype, int, const void*, const int*, int, unsigned int*, int, hipStream_t);
hipError_t launch_bilateral_r4(const Plan&, const BilArgs&, int, hipStream_t);
hipError_t launch_bilateral_persistent_r4(int, stereo_dtype, int, const void*, const int*, int, unsigned int*, int, hipStream_t);
hipError_t launch_bilateral_r5(const Plan&, const BilArgs&, int, hipStream_t);
hipError_t launch_bilateral_persistent_r5(int, stereo_dtype, int, const void*, const int*, int, unsigned int*, int, hipStream_t);
hipError_t launch_bilateral_r6(const Plan&, const BilArgs&, int, hipStream_t);
hipError_t launch_bilateral_persistent_r6(int, stereo_dtype, int, const void*, const int*, int, unsigned int*, int, hipStream_t);
hipError_t launch_bilateral_r7(const Plan&, const BilArgs&, int, hipStream_t);
hipError_t launch_bilateral_persistent_r7(int, stereo_dtype, int, const void*, const int*, int, unsigned int*, int, hipStream_t);
hipError_t launch_bilateral_r8(const Plan&, const BilArgs&, int, hipStream_t);
hipError_t launch_bilateral_persistent_r8(int, stereo_dtype, int, const void*, const int*, int, unsigned int*, int, hipStream_t);

hipError_t launch_bilateral(const Plan& P, const BilArgs& a, int mode, hipStream_t s) {
  switch (P.R) {
    case 1: return launch_bilateral_r1(P, a, mode, s);
    case 2: return launch_bilateral_r2(P, a, mode, s);
    case 3: return launch_bilateral_r3(P, a, mode, s);
    case 4: return launch_bilateral_r4(P, a, mode, s);
    case 5: return launch_bilateral_r5(P, a, mode, s);
    case 6: return launch_bilateral_r6(P, a, mode, s);
    case 7: return launch_bilateral_r7(P, a, mode, s);
    case 8: return launch_bilateral_r8(P, a, mode, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_bilateral_persistent(int engine, int R, stereo_dtype gdt, int levels, const void* pairs,
                                       const int* tiles, int n_tiles, unsigned int* counter,
                                       int n_groups, hipStream_t s) {
  switch (R) {
    case 1: return launch_bilateral_persistent_r1(engine, gdt, levels, pairs, tiles, n_tiles, counter, n_groups, s);
    case 2: return launch_bilateral_persistent_r2(engine, gdt, levels, pairs, tiles, n_tiles, counter, n_groups, s);
    case 3: return launch_bilateral_persistent_r3(engine, gdt, levels, pairs, tiles, n_tiles, counter, n_groups, s);
    case 4: return launch_bilateral_persistent_r4(engine, gdt, levels, pairs, tiles, n_tiles, counter, n_groups, s);
    case 5: return launch_bilateral_persistent_r5(engine, gdt, levels, pairs, tiles, n_tiles, counter, n_groups, s);
    case 6: return launch_bilateral_persistent_r6(engine, gdt, levels, pairs, tiles, n_tiles, counter, n_groups, s);
    case 7: return launch_bilateral_persistent_r7(engine, gdt, levels, pairs, tiles, n_tiles, counter, n_groups, s);
    case 8: return launch_bilateral_persistent_r8(engine, gdt, levels, pairs, tiles, n_tiles, counter, n_groups, s);
    default: return hipErrorInvalidValue;
  }
}

size_t bilateral_pair_bytes() { return sizeof(bil::BilPair); }

int h2_pitch(int R, int W) {
  switch (R) {
    case 1: return bilh::h2_pitch_for<1>(W);
    case 2: return bilh::h2_pitch_for<2>(W);
    case 3: return bilh::h2_pitch_for<3>(W);
    case 4: return bilh::h2_pitch_for<4>(W);
    case 5: return bilh::h2_pitch_for<5>(W);
    case 6: return bilh::h2_pitch_for<6>(W);
    case 7: return bilh::h2_pitch_for<7>(W);
    case 8: return bilh::h2_pitch_for<8>(W);
    default: return 0;
  }
}

void* bilateral_pair(const Plan& P, const BilArgs& a, void* out) {
  *static_cast<bil::BilPair*>(out) = bil::make_pair(P, a);
  return out;
}

}  // namespace stereo
