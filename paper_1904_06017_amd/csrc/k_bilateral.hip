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
// C' (FP32 blocks written by pass 1) -> the split-FP16 volume pass 2 stages,
// scaled by cprime_scale(max |C'|): level l of stored column s = x + R.
// Stored columns outside the image and levels past the tile hold zeros.
__global__ void __launch_bounds__(256) cprime_split_kernel(const float* __restrict__ src,
                                                           const unsigned int* __restrict__ gmax,
                                                           uint16_t* __restrict__ dst,
                                                           int64_t plane, int pitch, int W, int H,
                                                           int R) {
  const int l = threadIdx.x & 15;
  const int s = blockIdx.x * 16 + (threadIdx.x >> 4);
  const int y = blockIdx.y, blk = blockIdx.z;
  if (s >= (pitch >> 2)) return;
  const float S = cprime_scale(*gmax);
  const int nqx = (W + 3) >> 2;
  float v[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = 4 * s + j - R;
    v[j] = (c >= 0 && c < W)
               ? src[(((int64_t)blk * H + y) * nqx + (c >> 2)) * 64 + 4 * l + (c & 3)] * S
               : 0.0f;
  }
  typedef _Float16 h2 __attribute__((ext_vector_type(2)));
  typedef float f2 __attribute__((ext_vector_type(2)));
  const h2 h01 = __builtin_convertvector((f2){v[0], v[1]}, h2);
  const h2 h23 = __builtin_convertvector((f2){v[2], v[3]}, h2);
  const h2 l01 = __builtin_convertvector((f2){v[0] - (float)h01.x, v[1] - (float)h01.y}, h2);
  const h2 l23 = __builtin_convertvector((f2){v[2] - (float)h23.x, v[3] - (float)h23.y}, h2);
  const int64_t off = (int64_t)(2 * blk) * plane + (int64_t)y * 16 * pitch + 64 * s + 4 * l;
  *reinterpret_cast<uint2*>(dst + off) =
      make_uint2(__builtin_bit_cast(unsigned, h01), __builtin_bit_cast(unsigned, h23));
  *reinterpret_cast<uint2*>(dst + plane + off) =
      make_uint2(__builtin_bit_cast(unsigned, l01), __builtin_bit_cast(unsigned, l23));
}

}  // namespace bilh

hipError_t launch_cprime_split(const float* cblk, const unsigned int* gmax, uint16_t* h2,
                               int64_t plane, int pitch, int W, int H, int R, int levels,
                               hipStream_t s) {
  if (!cblk || !gmax || !h2 || (pitch & 7) || levels <= 0) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((pitch / 4 + 15) / 16), (unsigned)H, (unsigned)((levels + 15) / 16));
  hipLaunchKernelGGL(bilh::cprime_split_kernel, grid, dim3(256), 0, s, cblk, gmax, h2, plane,
                     pitch, W, H, R);
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
