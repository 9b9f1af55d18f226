// Dispatch of the aggregation launches over the compiled window radii.
#include "bilateral_mfma16_bwd.h"

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

hipError_t launch_bwd16_r1(const Plan&, const BilArgs&, int, hipStream_t);
hipError_t launch_bwd16_r2(const Plan&, const BilArgs&, int, hipStream_t);
hipError_t launch_bwd16_r3(const Plan&, const BilArgs&, int, hipStream_t);
hipError_t launch_bwd16_r4(const Plan&, const BilArgs&, int, hipStream_t);
hipError_t launch_bwd16_r5(const Plan&, const BilArgs&, int, hipStream_t);

hipError_t launch_bilateral_bwd16(const Plan& P, const BilArgs& a, int pass, hipStream_t s) {
  if ((pass != 1 && pass != 2) || (a.d_first & 15)) return hipErrorInvalidValue;
  static_assert(kBwd16MaxR == 5, "one launcher per compiled radius");
  switch (P.R) {
    case 1: return launch_bwd16_r1(P, a, pass, s);
    case 2: return launch_bwd16_r2(P, a, pass, s);
    case 3: return launch_bwd16_r3(P, a, pass, s);
    case 4: return launch_bwd16_r4(P, a, pass, s);
    case 5: return launch_bwd16_r5(P, a, pass, s);
    default: return hipErrorInvalidValue;
  }
}

namespace bilh {
// Zeros in the pad columns of every row of the first blocks (both parts):
// thread t of a row: pad column t / 16 (columns [0, R), then [W + R, pitch)),
// level t % 16.
__global__ void __launch_bounds__(256) h2_pad_zero_kernel(uint16_t* __restrict__ h2,
                                                          int64_t plane, int pitch, int W,
                                                          int R) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  const int npad = pitch - W;
  if (t >= 16 * npad) return;
  const int ci = t >> 4, l = t & 15;
  const int c = ci < R ? ci : W + ci;
  const int y = blockIdx.y, bp = blockIdx.z;   // bp = 2 block + part
  h2[(int64_t)bp * plane + (int64_t)y * 16 * pitch + 64 * (c >> 2) + 4 * l + (c & 3)] = 0;
}
}  // namespace bilh

hipError_t launch_h2_pad_zero(uint16_t* h2, int64_t plane, int pitch, int W, int H, int R,
                              int nblk, hipStream_t s) {
  if (!h2 || pitch < W + R || nblk <= 0) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((16 * (pitch - W) + 255) / 256), (unsigned)H, (unsigned)(2 * nblk));
  hipLaunchKernelGGL(bilh::h2_pad_zero_kernel, grid, dim3(256), 0, s, h2, plane, pitch, W, R);
  return hipGetLastError();
}

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
