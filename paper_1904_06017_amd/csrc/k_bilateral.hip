// Bilateral cost aggregation, Eqs. (10)-(11), with an optional fused
// winner-take-all + sub-pixel epilogue (Sec. 3.2.2, Eq. 13).
//
// E(p, d) = sum_q w(p, q) C(q, d) / sum_q w(p, q),
// w(p, q) = exp(-|p - q|^2 / sigma_s^2 - (G(p) - G(q))^2 / sigma_r^2),
// q over the (2R+1)^2 window truncated to the image.
//
// Work decomposition (VALU-bound stencil, no matrix cores):
//   * a workgroup owns a TW x TH pixel tile and walks the disparity range in
//     chunks of DC levels; for each chunk the (TW+2R) x (TH+2R) halo of costs
//     is staged in LDS as float4 quads of consecutive levels
//     ([quad][row][col], odd row pitch so that eight lanes on consecutive
//     rows hit eight different 16-byte bank groups);
//   * a thread owns PX horizontally adjacent pixels x DC levels in registers;
//     every cost quad read from LDS feeds up to PX pixels, every weight feeds
//     DC fused multiply-adds;
//   * weights are computed in registers, w = exp2(sx(dx) + sy(dy) - kr2 dG^2)
//     (the spatial factor of Eq. 31 and the range factor of Eq. 32 folded into
//     one exponent); a guide of 1e30 outside the image gives weight 0.
// Taps are summed in raster order (dy outer, dx inner) for every pixel, so
// the result does not depend on the tile shape.
#include "internal.h"

namespace stereo {
namespace {

constexpr int kThreads = 256;

template <int R, int PX, int DC, int TYT>
struct BilGeom {
  static constexpr int TXT = kThreads / TYT;
  static constexpr int TW = TXT * PX;
  static constexpr int TH = TYT;
  static constexpr int HX = TW + 2 * R;
  static constexpr int HY = TH + 2 * R;
  static constexpr int HXP = HX | 1;          // odd pitch in float4 units
  static constexpr int NQ = DC / 4;
  static constexpr size_t lds_bytes =
      sizeof(float4) * (size_t)NQ * HY * HXP + sizeof(float) * (size_t)HY * HX;
};

template <typename G>
__device__ __forceinline__ float guide_at(const G* g, int64_t pitch, int x, int y) {
  return static_cast<float>(g[(int64_t)y * pitch + x]);
}

template <int R, int PX, int DC, int TYT, typename GT, int MODE>
__global__ void __launch_bounds__(kThreads)
bilateral_kernel(const float* __restrict__ C, int64_t c_slice, int64_t c_pitch,
                 int shift, const GT* __restrict__ guide, int64_t g_pitch,
                 int W, int H, int D, float ks2, float kr2,
                 float* __restrict__ E, int16_t* __restrict__ dint,
                 float* __restrict__ dsub) {
  using Gm = BilGeom<R, PX, DC, TYT>;
  extern __shared__ float4 lds4[];
  float4* Cs = lds4;                                        // [NQ][HY][HXP]
  float* Gs = reinterpret_cast<float*>(lds4 + Gm::NQ * Gm::HY * Gm::HXP);  // [HY][HX]

  const int t = threadIdx.x;
  const int ty = t % TYT;
  const int tx = t / TYT;
  const int x0 = blockIdx.x * Gm::TW;
  const int y0 = blockIdx.y * Gm::TH;

  for (int i = t; i < Gm::HY * Gm::HX; i += kThreads) {
    const int yy = i / Gm::HX, xx = i - yy * Gm::HX;
    const int gy = y0 - R + yy, gx = x0 - R + xx;
    Gs[i] = (gy >= 0 && gy < H && gx >= 0 && gx < W) ? guide_at(guide, g_pitch, gx, gy)
                                                     : kFarGuide;
  }
  __syncthreads();

  float gp[PX];
#pragma unroll
  for (int k = 0; k < PX; ++k) gp[k] = Gs[(ty + R) * Gm::HX + tx * PX + k + R];
  float sx[2 * R + 1];
#pragma unroll
  for (int j = 0; j <= 2 * R; ++j) sx[j] = -(float)((j - R) * (j - R)) * ks2;

  float wsum[PX];
  float rinv[PX];
#pragma unroll
  for (int k = 0; k < PX; ++k) { wsum[k] = 0.0f; rinv[k] = 1.0f; }
  // running winner-take-all state per pixel (mode 1)
  float bestE[PX], Em[PX], Ep[PX], prev[PX];
  int bestD[PX];
#pragma unroll
  for (int k = 0; k < PX; ++k) {
    bestE[k] = 3.402823466e38f; Em[k] = 0.0f; Ep[k] = 0.0f; prev[k] = 0.0f; bestD[k] = 0;
  }

  for (int d0 = 0; d0 < D; d0 += DC) {
    // ---- stage the cost halo of this chunk: quads of 4 consecutive levels
    for (int i = t; i < Gm::NQ * Gm::HY * Gm::HX; i += kThreads) {
      const int q = i / (Gm::HY * Gm::HX);
      const int rem = i - q * Gm::HY * Gm::HX;
      const int yy = rem / Gm::HX, xx = rem - yy * Gm::HX;
      const int gy = y0 - R + yy, gx = x0 - R + xx;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
        const int d = d0 + 4 * q;
        const float* base = C + (int64_t)gy * c_pitch + gx;
        if (d + 0 < D) v.x = base[(int64_t)(d + 0) * c_slice + (d + 0) * shift];
        if (d + 1 < D) v.y = base[(int64_t)(d + 1) * c_slice + (d + 1) * shift];
        if (d + 2 < D) v.z = base[(int64_t)(d + 2) * c_slice + (d + 2) * shift];
        if (d + 3 < D) v.w = base[(int64_t)(d + 3) * c_slice + (d + 3) * shift];
      }
      Cs[(q * Gm::HY + yy) * Gm::HXP + xx] = v;
    }
    __syncthreads();

    float acc[PX][DC];
#pragma unroll
    for (int k = 0; k < PX; ++k)
#pragma unroll
      for (int j = 0; j < DC; ++j) acc[k][j] = 0.0f;
    const bool first = (d0 == 0);

    for (int dy = 0; dy <= 2 * R; ++dy) {
      const int row = ty + dy;
      const float sy = -(float)((dy - R) * (dy - R)) * ks2;
      const float4* crow = Cs + row * Gm::HXP + tx * PX;
      const float* grow = Gs + row * Gm::HX + tx * PX;
#pragma unroll
      for (int xx = 0; xx < PX + 2 * R; ++xx) {
        float cv[DC];
#pragma unroll
        for (int q = 0; q < Gm::NQ; ++q) {
          const float4 v = crow[q * Gm::HY * Gm::HXP + xx];
          cv[4 * q + 0] = v.x; cv[4 * q + 1] = v.y; cv[4 * q + 2] = v.z; cv[4 * q + 3] = v.w;
        }
        const float gq = grow[xx];
#pragma unroll
        for (int k = 0; k < PX; ++k) {
          const int dx = xx - k;
          if (dx < 0 || dx > 2 * R) continue;
          const float g = gp[k] - gq;
          const float w = __builtin_amdgcn_exp2f(fmaf(g * g, -kr2, sy + sx[dx]));
          if (MODE == 0 && first) wsum[k] += w;
#pragma unroll
          for (int j = 0; j < DC; ++j) acc[k][j] = fmaf(w, cv[j], acc[k][j]);
        }
      }
    }

    if (MODE == 0 && first) {
#pragma unroll
      for (int k = 0; k < PX; ++k) rinv[k] = 1.0f / wsum[k];
    }

    const int py = y0 + ty;
#pragma unroll
    for (int k = 0; k < PX; ++k) {
      const int px = x0 + tx * PX + k;
      if (MODE == 0) {
        if (py < H && px < W) {
#pragma unroll
          for (int j = 0; j < DC; ++j) {
            const int d = d0 + j;
            if (d < D) E[((int64_t)d * H + py) * W + px] = acc[k][j] * rinv[k];
          }
        }
      } else {
        // WTA on the unnormalised sums: sum_q w(p,q) is a positive per-pixel
        // constant, so the argmin and the scale-free parabola offset of
        // Eq. (13) are those of E.
#pragma unroll
        for (int j = 0; j < DC; ++j) {
          const int d = d0 + j;
          if (d < D) {
            const float e = acc[k][j];
            if (d == bestD[k] + 1) Ep[k] = e;
            if (e < bestE[k]) { Em[k] = prev[k]; bestE[k] = e; bestD[k] = d; }
            prev[k] = e;
          }
        }
      }
    }
    __syncthreads();
  }

  if (MODE == 1) {
    const int py = y0 + ty;
#pragma unroll
    for (int k = 0; k < PX; ++k) {
      const int px = x0 + tx * PX + k;
      if (py < H && px < W) {
        const int d = bestD[k];
        dint[(int64_t)py * W + px] = (int16_t)d;
        if (dsub) {
          float off = 0.0f;
          if (d > 0 && d < D - 1) {
            const float den = 2.0f * Em[k] + 2.0f * Ep[k] - 4.0f * bestE[k];
            if (den > 0.0f) off = (Em[k] - Ep[k]) / den;
          }
          dsub[(int64_t)py * W + px] = (float)d + off;
        }
      }
    }
  }
}

template <int R, int PX, int DC, int TYT, typename GT, int MODE>
hipError_t launch_one(const Plan& P, const BilArgs& a, hipStream_t s) {
  using Gm = BilGeom<R, PX, DC, TYT>;
  auto kern = bilateral_kernel<R, PX, DC, TYT, GT, MODE>;
  static bool attr_set = false;       // per instantiation; idempotent
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)Gm::lds_bytes);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  dim3 grid((P.W + Gm::TW - 1) / Gm::TW, (P.H + Gm::TH - 1) / Gm::TH);
  const Consts c = consts_of(P);
  hipLaunchKernelGGL(kern, grid, dim3(kThreads), Gm::lds_bytes, s, a.C, a.c_slice,
                     a.c_pitch, a.shift, (const GT*)a.guide, a.guide_pitch, P.W, P.H,
                     P.D, c.ks2, c.kr2, a.E, a.dint, a.dsub);
  return hipGetLastError();
}

template <int R>
hipError_t launch_r(const Plan& P, const BilArgs& a, int mode, hipStream_t s) {
  constexpr int PX = 4, DC = 8, TYT = 32;
  if (a.guide_dt == STEREO_U8)
    return mode == 0 ? launch_one<R, PX, DC, TYT, uint8_t, 0>(P, a, s)
                     : launch_one<R, PX, DC, TYT, uint8_t, 1>(P, a, s);
  return mode == 0 ? launch_one<R, PX, DC, TYT, float, 0>(P, a, s)
                   : launch_one<R, PX, DC, TYT, float, 1>(P, a, s);
}

}  // namespace

hipError_t launch_bilateral(const Plan& P, const BilArgs& a, int mode, hipStream_t s) {
  switch (P.R) {
    case 1: return launch_r<1>(P, a, mode, s);
    case 2: return launch_r<2>(P, a, mode, s);
    case 3: return launch_r<3>(P, a, mode, s);
    case 4: return launch_r<4>(P, a, mode, s);
    case 5: return launch_r<5>(P, a, mode, s);
    case 6: return launch_r<6>(P, a, mode, s);
    case 7: return launch_r<7>(P, a, mode, s);
    case 8: return launch_r<8>(P, a, mode, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace stereo
