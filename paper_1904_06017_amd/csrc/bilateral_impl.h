// Bilateral cost aggregation, Eqs. (10)-(11), with an optional fused
// winner-take-all + sub-pixel epilogue (Sec. 3.2.2, Eq. 13).
//
// E(p, d) = sum_q w(p, q) C(q, d) / sum_q w(p, q),
// w(p, q) = exp(-|p - q|^2 / sigma_s^2 - (G(p) - G(q))^2 / sigma_r^2),
// q over the (2R+1)^2 window truncated to the image.
//
// Work decomposition (VALU-bound stencil, no matrix cores):
//   * a 512-thread workgroup owns a 32 x 32 pixel tile and walks the
//     disparity range in chunks of DC levels; for each chunk the
//     (32+2R) x (32+2R) halo of costs is staged in LDS as float4 quads of
//     consecutive levels ([quad][row][col], odd row pitch so that lanes on
//     consecutive rows hit different 16-byte bank groups).  Two workgroups
//     fit a CU at DC = 8 (16 waves), so one stages while the other computes;
//   * a thread owns PX = 2 horizontally adjacent pixels x DC levels in
//     registers; every cost quad read from LDS feeds up to 2 pixels, every
//     weight feeds DC fused multiply-adds;
//   * weights are computed in registers as one exponent,
//     w = exp2(sx(dx) + sy(dy) - (G'(p) - G'(q))^2), with the guide pre-scaled
//     by sqrt(log2(e)) / sigma_r (the paper keeps pre-computed weight tables,
//     Eqs. 30-32, in constant memory; here the exponential is cheaper than a
//     per-lane table gather).  Outside the image the guide is a sentinel
//     whose weight is exactly 0.
//   * the cost volume is read either in the planar layout [level][row][col]
//     or in the level-quad-interleaved layout [level/4][row][col] float4 (one
//     16-byte load per quad).  For the target volume, which is read sheared
//     (level d from column x + d), a quad of the interleaved layout is loaded
//     whole and its four components are written to their own columns.
// Taps are summed in raster order (dy outer, dx inner) for every pixel, so
// the result does not depend on the tile shape.
#pragma once
#include <type_traits>

#include "internal.h"

namespace stereo {
namespace bil {

constexpr int kThreads = 512;
constexpr int kPX = 2;      // pixels per thread along a row
constexpr int kTYT = 32;    // thread rows = tile rows

template <int R, int PX, int DC, int TYT>
struct BilGeom {
  static constexpr int TXT = kThreads / TYT;
  static constexpr int TW = TXT * PX;
  static constexpr int TH = TYT;
  static constexpr int HX = TW + 2 * R;
  static constexpr int HY = TH + 2 * R;
  static constexpr int HXP = HX | 1;          // odd pitch in float4 units
  static constexpr int NQ = DC / 4;
  // LDS layout: [guide tile (float)] [cost quads]
  static constexpr size_t guide_bytes() {
    return (sizeof(float) * (size_t)HY * HX + 15) & ~size_t(15);
  }
  static constexpr size_t lds_bytes() {
    return guide_bytes() + sizeof(float4) * (size_t)NQ * HY * HXP;
  }
};

// Outputs and epilogue constants of one launch.
struct BilOut {
  float* E;                         // modes 0, 4
  int16_t* dint;                    // mode 1
  float* dsub;                      // mode 1 (nullable)
  float* sm_m;                      // mode 2: max_d(-E/T)
  float* sm_logZ;                   // mode 2: log sum_d exp(-E/T - m)
  float* sm_dh;                     // mode 2: soft level
  float* disp;                      // mode 2: shifted back
  float invT;
  double delta_p, c0, c1, c2;
  // modes 5, 6
  const float* gD;                  // mode 5: dL / d(shifted disparity)
  const float* cpix;                // mode 6: cost tile at the pixel
  float* aP;                        // mode 5
  float* A1;                        // mode 5
  float* A2;                        // mode 6
  float* Wp;                        // mode 5 (nullable)
  int d_first;
  float one_minus_c1;
};

// Everything one tile needs to know about its pair.
struct BilPair {
  const float* C;                   // cost volume
  int64_t c_slice, c_pitch;         // planar: floats; quad: float4 units
  int shift;                        // 1: level d is read from column x + d
  int quad;                         // 1: level-quad-interleaved layout
  const void* guide;
  int64_t g_pitch;
  int W, H, D;
  float ks2, kr2;
  BilOut o;
  const uint16_t* h2;               // split-FP16 volume (see BilArgs)
  int64_t h2_plane;
  int h2_pitch;
};

template <typename G>
__device__ __forceinline__ float guide_at(const G* g, int64_t pitch, int x, int y) {
  return static_cast<float>(g[(int64_t)y * pitch + x]);
}

template <int R, int PX, int DC, int TYT, typename GT, int MODE>
__device__ __forceinline__ void bilateral_tile(const BilPair& a, int x0, int y0,
                                               float4* lds4) {
  const float* __restrict__ C = a.C;
  const int64_t c_pitch = a.c_pitch;
  const GT* __restrict__ guide = static_cast<const GT*>(a.guide);
  const int64_t g_pitch = a.g_pitch;
  const int W = a.W, H = a.H, D = a.D;
  const float ks2 = a.ks2, kr2 = a.kr2;
  const BilOut& o = a.o;
  using Gm = BilGeom<R, PX, DC, TYT>;
  char* lds = reinterpret_cast<char*>(lds4);
  float* Gs = reinterpret_cast<float*>(lds);                                 // [HY][HX]
  float4* Cs = reinterpret_cast<float4*>(lds + Gm::guide_bytes());           // [NQ][HY][HXP]

  const int t = threadIdx.x;
  const int ty = t % TYT;
  const int tx = t / TYT;
  const float kr = sqrtf(kr2);

  for (int i = t; i < Gm::HY * Gm::HX; i += kThreads) {
    const int yy = i / Gm::HX, xx = i - yy * Gm::HX;
    const int gy = y0 - R + yy, gx = x0 - R + xx;
    const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
    // pre-scaled by sqrt(kr2): the range exponent is then -(G'(p) - G'(q))^2
    Gs[i] = in ? guide_at(guide, g_pitch, gx, gy) * kr : kFarGuide;
  }
  __syncthreads();

  float gp[PX];
#pragma unroll
  for (int k = 0; k < PX; ++k) gp[k] = Gs[(ty + R) * Gm::HX + tx * PX + k + R];
  float sx[2 * R + 1];
#pragma unroll
  for (int j = 0; j <= 2 * R; ++j) sx[j] = -(float)((j - R) * (j - R)) * ks2;

  constexpr bool NORM = (MODE == 0 || MODE == 2 || MODE == 5);   // needs sum_q w(p, q)
  // modes 5, 6 also accumulate with the second weight w(p, q) (G'(p) - G'(q))
  constexpr bool TWO = (MODE == 5 || MODE == 6);
  constexpr int PX2 = TWO ? PX : 1, DC2 = TWO ? DC : 1;
  float wsum[PX];
  float rinv[PX];
#pragma unroll
  for (int k = 0; k < PX; ++k) { wsum[k] = 0.0f; rinv[k] = 1.0f; }
  // running winner-take-all state per pixel (mode 1)
  float bestE[PX], Em[PX], Ep[PX], prev[PX];
  int bestD[PX];
  // running soft-argmin state per pixel (mode 2), base-2 exponents:
  // m2 = max_d z, Z = sum_d 2^(z - m2), S1 = sum_d d 2^(z - m2), z = -E log2(e) / T
  float m2[PX], Zs[PX], S1[PX];
#pragma unroll
  for (int k = 0; k < PX; ++k) {
    bestE[k] = 3.402823466e38f; Em[k] = 0.0f; Ep[k] = 0.0f; prev[k] = 0.0f; bestD[k] = 0;
    m2[k] = -3.402823466e38f; Zs[k] = 0.0f; S1[k] = 0.0f;
  }
  const float zscale = -o.invT * 1.4426950408889634f;
  // modes 5, 6: the two running sums per pixel (the softmax state of mode 5
  // is re-read in each pass's epilogue rather than held in registers)
  float sa[PX2], sb[PX2];
#pragma unroll
  for (int k = 0; k < PX2; ++k) { sa[k] = 0.0f; sb[k] = 0.0f; }

  // element step from level d to d + 1 (the target volume also moves one
  // column to the right per level)
  const uint32_t step = (uint32_t)a.c_slice + (uint32_t)a.shift;
  for (int d0 = 0; d0 < D; d0 += DC) {
    // ---- stage the cost halo of this chunk: quads of 4 consecutive levels.
    // Lanes run along columns (coalesced loads); offsets are 32-bit from a
    // uniform base.  Out-of-image halo entries are 0 (their weight is 0).
    if (!a.quad) {
      for (int i = t; i < Gm::HY * Gm::HX; i += kThreads) {
        const int yy = i / Gm::HX, col = i - yy * Gm::HX;
        const int gx = x0 - R + col, gy = y0 - R + yy;
        const bool ok = gx >= 0 && gx < W && gy >= 0 && gy < H;
        const uint32_t rowoff = ok ? (uint32_t)gy * (uint32_t)c_pitch + (uint32_t)gx : 0u;
#pragma unroll
        for (int q = 0; q < Gm::NQ; ++q) {
          float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
          if (ok) {
            const int d = d0 + 4 * q;
            const uint32_t o = rowoff + (uint32_t)d * step;
            if (d + 0 < D) v.x = C[o];
            if (d + 1 < D) v.y = C[o + step];
            if (d + 2 < D) v.z = C[o + 2 * step];
            if (d + 3 < D) v.w = C[o + 3 * step];
          }
          Cs[(q * Gm::HY + yy) * Gm::HXP + col] = v;
        }
      }
    } else if (!a.shift) {
      const float4* __restrict__ C4 = reinterpret_cast<const float4*>(C);
      for (int i = t; i < Gm::HY * Gm::HX; i += kThreads) {
        const int yy = i / Gm::HX, col = i - yy * Gm::HX;
        const int gx = x0 - R + col, gy = y0 - R + yy;
        const bool ok = gx >= 0 && gx < W && gy >= 0 && gy < H;
        const uint32_t rowoff = ok ? (uint32_t)gy * (uint32_t)c_pitch + (uint32_t)gx : 0u;
#pragma unroll
        for (int q = 0; q < Gm::NQ; ++q) {
          float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
          if (ok && d0 + 4 * q < D)
            v = C4[(uint32_t)((d0 >> 2) + q) * (uint32_t)a.c_slice + rowoff];
          Cs[(q * Gm::HY + yy) * Gm::HXP + col] = v;
        }
      }
    } else {
      // sheared quads: component j of the quad at extended column e holds
      // level 4q' + j of target column e - 4q' - j; 3 extra columns per row
      // cover the shear inside a quad
      const float4* __restrict__ C4 = reinterpret_cast<const float4*>(C);
      float* Csf = reinterpret_cast<float*>(Cs);
      constexpr int HXE = Gm::HX + 3;
      for (int i = t; i < Gm::HY * HXE; i += kThreads) {
        const int yy = i / HXE, c = i - yy * HXE;
        const int gy = y0 - R + yy;
        const bool rowok = gy >= 0 && gy < H;
#pragma unroll
        for (int q = 0; q < Gm::NQ; ++q) {
          const int dq = d0 + 4 * q;
          const int e = x0 - R + c + dq;
          float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
          if (rowok && dq < D && e >= 0 && e < (int)c_pitch)
            v = C4[(uint32_t)(dq >> 2) * (uint32_t)a.c_slice +
                   (uint32_t)gy * (uint32_t)c_pitch + (uint32_t)e];
          const float comp[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int col = c - j;
            if (col < 0 || col >= Gm::HX) continue;
            const int x = x0 - R + col;
            const bool ok = x >= 0 && x < W && dq + j < D;
            Csf[((q * Gm::HY + yy) * Gm::HXP + col) * 4 + j] = ok ? comp[j] : 0.0f;
          }
        }
      }
    }
    __syncthreads();

    float acc[PX][DC];
    float acc2[PX2][DC2];
#pragma unroll
    for (int k = 0; k < PX; ++k)
#pragma unroll
      for (int j = 0; j < DC; ++j) acc[k][j] = 0.0f;
#pragma unroll
    for (int k = 0; k < PX2; ++k)
#pragma unroll
      for (int j = 0; j < DC2; ++j) acc2[k][j] = 0.0f;
    const bool first = (d0 == 0);

    for (int dy = 0; dy <= 2 * R; ++dy) {
      const int row = ty + dy;
      const float sy = -(float)((dy - R) * (dy - R)) * ks2;
      const float4* crow = Cs + row * Gm::HXP + tx * PX;
      const float* grow = Gs + row * Gm::HX + tx * PX;
      // weights of this tap row first: the exponentials are independent of
      // each other and of the cost reads below
      float wr[PX][2 * R + 1];
      float wg[PX2][TWO ? 2 * R + 1 : 1];
#pragma unroll
      for (int xx = 0; xx < PX + 2 * R; ++xx) {
        const float gq = grow[xx];
#pragma unroll
        for (int k = 0; k < PX; ++k) {
          const int dx = xx - k;
          if (dx < 0 || dx > 2 * R) continue;
          const float g = gp[k] - gq;
          wr[k][dx] = __builtin_amdgcn_exp2f(fmaf(-g, g, sy + sx[dx]));
          if constexpr (TWO) wg[k][dx] = wr[k][dx] * g;
        }
      }
      if (NORM && first) {
#pragma unroll
        for (int k = 0; k < PX; ++k)
#pragma unroll
          for (int dx = 0; dx <= 2 * R; ++dx) wsum[k] += wr[k][dx];
      }
#pragma unroll
      for (int xx = 0; xx < PX + 2 * R; ++xx) {
        float cv[DC];
#pragma unroll
        for (int q = 0; q < Gm::NQ; ++q) {
          const float4 v = crow[q * Gm::HY * Gm::HXP + xx];
          cv[4 * q + 0] = v.x; cv[4 * q + 1] = v.y; cv[4 * q + 2] = v.z; cv[4 * q + 3] = v.w;
        }
#pragma unroll
        for (int k = 0; k < PX; ++k) {
          const int dx = xx - k;
          if (dx < 0 || dx > 2 * R) continue;
          const float w = wr[k][dx];
#pragma unroll
          for (int j = 0; j < DC; ++j) acc[k][j] = fmaf(w, cv[j], acc[k][j]);
          if constexpr (TWO) {
            const float w2 = wg[k][dx];
#pragma unroll
            for (int j = 0; j < DC; ++j) acc2[k][j] = fmaf(w2, cv[j], acc2[k][j]);
          }
        }
      }
    }

    if (NORM && first) {
#pragma unroll
      for (int k = 0; k < PX; ++k) rinv[k] = 1.0f / wsum[k];
    }

    const int py = y0 + ty;
#pragma unroll
    for (int k = 0; k < PX; ++k) {
      const int px = x0 + tx * PX + k;
      if (MODE == 0 || MODE == 4) {
        // mode 0: normalised E (Eq. 11); mode 4: the weighted sum alone
        if (py < H && px < W) {
#pragma unroll
          for (int j = 0; j < DC; ++j) {
            const int d = d0 + j;
            if (d < D) o.E[((int64_t)d * H + py) * W + px] = MODE == 0 ? acc[k][j] * rinv[k]
                                                                       : acc[k][j];
          }
        }
      } else if constexpr (MODE == 5) {
        // softmax adjoint: P = exp(-E/T - m - log Z), dE = g' (-1/T) P (d - dh)
        const bool in = py < H && px < W;
        float sbase = 0.0f, sgp = 0.0f, sdh = 0.0f;
        if (in) {
          const int64_t pix = (int64_t)py * W + px;
          sbase = -(o.sm_m[pix] + o.sm_logZ[pix]);
          sgp = o.gD[pix] * o.one_minus_c1 * (-o.invT);
          sdh = o.sm_dh[pix];
        }
#pragma unroll
        for (int j = 0; j < DC; ++j) {
          const int d = d0 + j;
          if (d < D) {
            const float e = acc[k][j] * rinv[k];
            const float P = __builtin_amdgcn_exp2f(fmaf(-e, o.invT, sbase) *
                                                   1.4426950408889634f);
            const float dE = sgp * P * ((float)(o.d_first + d) - sdh);
            if (in) o.E[((int64_t)d * H + py) * W + px] = dE * rinv[k];
            sa[k] = fmaf(dE, e, sa[k]);
            sb[k] = fmaf(dE, acc2[k][j], sb[k]);
          }
        }
      } else if constexpr (MODE == 6) {
        const bool in = py < H && px < W;
#pragma unroll
        for (int j = 0; j < DC; ++j) {
          const int d = d0 + j;
          if (d < D && in) {
            const int64_t oi = ((int64_t)d * H + py) * W + px;
            o.E[oi] = acc[k][j];
            sb[k] = fmaf(o.cpix[oi], acc2[k][j], sb[k]);
          }
        }
      } else if (MODE == 2) {
#pragma unroll
        for (int j = 0; j < DC; ++j) {
          const int d = d0 + j;
          if (d < D) {
            const float z = acc[k][j] * rinv[k] * zscale;
            if (z > m2[k]) {
              const float sc = __builtin_amdgcn_exp2f(m2[k] - z);
              Zs[k] = fmaf(Zs[k], sc, 1.0f);
              S1[k] = fmaf(S1[k], sc, (float)d);
              m2[k] = z;
            } else {
              const float e = __builtin_amdgcn_exp2f(z - m2[k]);
              Zs[k] += e;
              S1[k] = fmaf((float)d, e, S1[k]);
            }
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

  if constexpr (TWO) {
    // the second weight carries the guide difference scaled by sqrt(kr2)
    const float inv_kr = 1.0f / kr;
    const int py = y0 + ty;
#pragma unroll
    for (int k = 0; k < PX2; ++k) {
      const int px = x0 + tx * PX + k;
      if (py < H && px < W) {
        const int64_t pix = (int64_t)py * W + px;
        if (MODE == 5) {
          o.aP[pix] += sa[k];
          o.A1[pix] += sb[k] * inv_kr;
          if (o.Wp) o.Wp[pix] = wsum[k];
        } else {
          o.A2[pix] += -sb[k] * inv_kr;
        }
      }
    }
  }

  if (MODE == 2) {
    // soft level dh = sum_d d P(d), saved state (m, log Z) in natural units,
    // and the shift back D = dh - delta_p + d_road(u - dh + delta_p, v)
    const int py = y0 + ty;
    const float ln2 = 0.6931471805599453f;
#pragma unroll
    for (int k = 0; k < PX; ++k) {
      const int px = x0 + tx * PX + k;
      if (py < H && px < W) {
        const int64_t pix = (int64_t)py * W + px;
        const float dh = S1[k] / Zs[k];
        o.sm_m[pix] = m2[k] * ln2;
        o.sm_logZ[pix] = __builtin_amdgcn_logf(Zs[k]) * ln2;
        o.sm_dh[pix] = dh;
        const double dd = dh;
        o.disp[pix] = (float)(dd - o.delta_p + (o.c0 + o.c1 * ((double)px - dd + o.delta_p) +
                                                o.c2 * (double)py));
      }
    }
  }

  if (MODE == 1) {
    const int py = y0 + ty;
#pragma unroll
    for (int k = 0; k < PX; ++k) {
      const int px = x0 + tx * PX + k;
      if (py < H && px < W) {
        const int d = bestD[k];
        o.dint[(int64_t)py * W + px] = (int16_t)d;
        if (o.dsub) {
          float off = 0.0f;
          if (d > 0 && d < D - 1) {
            const float den = 2.0f * Em[k] + 2.0f * Ep[k] - 4.0f * bestE[k];
            if (den > 0.0f) off = (Em[k] - Ep[k]) / den;
          }
          o.dsub[(int64_t)py * W + px] = (float)d + off;
        }
      }
    }
  }
}

// Two workgroups per CU at 8 levels per pass (16 waves, 4 per SIMD): at most
// 128 VGPRs; at 16 levels the LDS allows one.
template <int R, int PX, int DC, int TYT, typename GT, int MODE>
__global__ void __launch_bounds__(kThreads, DC == 8 ? 4 : 2)
bilateral_kernel(BilPair a) {
  extern __shared__ float4 lds4[];
  using Gm = BilGeom<R, PX, DC, TYT>;
  bilateral_tile<R, PX, DC, TYT, GT, MODE>(a, blockIdx.x * Gm::TW, blockIdx.y * Gm::TH, lds4);
}

// Persistent form: each workgroup takes tiles from a queue (an integer
// counter) until the queue is empty; a tile names its pair.  Every
// workgroup leaves the loop once the counter passes n_tiles.
template <int R, int PX, int DC, int TYT, typename GT, int MODE>
__global__ void __launch_bounds__(kThreads)
bilateral_persistent_kernel(const BilPair* __restrict__ pairs, const int* __restrict__ tiles,
                            int n_tiles, unsigned int* __restrict__ counter) {
  extern __shared__ float4 lds4[];
  __shared__ int next;
  for (;;) {
    if (threadIdx.x == 0) next = (int)atomicAdd(counter, 1u);
    __syncthreads();
    const int t = next;
    __syncthreads();                       // everyone has read the slot
    if (t >= n_tiles) break;
    const int* e = tiles + 3 * t;          // (pair, x0, y0)
    bilateral_tile<R, PX, DC, TYT, GT, MODE>(pairs[e[0]], e[1], e[2], lds4);
    __syncthreads();
  }
}

inline BilPair make_pair(const Plan& P, const BilArgs& a) {
  const Consts c = consts_of(P);
  BilPair b;
  b.C = a.C; b.c_slice = a.c_slice; b.c_pitch = a.c_pitch; b.shift = a.shift; b.quad = a.quad;
  b.guide = a.guide; b.g_pitch = a.guide_pitch;
  b.W = P.W; b.H = P.H; b.D = a.levels > 0 ? a.levels : P.D;
  b.ks2 = c.ks2; b.kr2 = c.kr2;
  BilOut& o = b.o;
  o.E = a.E; o.dint = a.dint; o.dsub = a.dsub;
  o.sm_m = a.sm_m; o.sm_logZ = a.sm_logZ; o.sm_dh = a.sm_dh; o.disp = a.disp;
  o.invT = 1.0f / P.p.softargmin_T;
  o.delta_p = P.p.perspective ? (double)P.p.delta_p : 0.0;
  o.c0 = a.plane[0]; o.c1 = a.plane[1]; o.c2 = a.plane[2];
  o.gD = a.gD; o.cpix = a.cpix; o.aP = a.aP; o.A1 = a.A1; o.A2 = a.A2; o.Wp = a.Wp;
  o.d_first = a.d_first;
  o.one_minus_c1 = (float)(1.0 - a.plane[1]);
  b.h2 = a.h2; b.h2_plane = a.h2_plane; b.h2_pitch = a.h2_pitch;
  return b;
}

template <int R, int PX, int DC, int TYT, typename GT, int MODE>
hipError_t launch_one(const Plan& P, const BilArgs& a, hipStream_t s) {
  using Gm = BilGeom<R, PX, DC, TYT>;
  auto kern = bilateral_kernel<R, PX, DC, TYT, GT, MODE>;
  constexpr size_t lds = Gm::lds_bytes();
  static bool attr_set = false;       // per instantiation; idempotent
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  dim3 grid((P.W + Gm::TW - 1) / Gm::TW, (P.H + Gm::TH - 1) / Gm::TH);
  hipLaunchKernelGGL(kern, grid, dim3(kThreads), lds, s, make_pair(P, a));
  return hipGetLastError();
}

template <int R, int PX, int DC, int TYT, typename GT, int MODE>
hipError_t launch_persistent_one(const BilPair* pairs, const int* tiles, int n_tiles,
                                 unsigned int* counter, int n_groups, hipStream_t s) {
  using Gm = BilGeom<R, PX, DC, TYT>;
  auto kern = bilateral_persistent_kernel<R, PX, DC, TYT, GT, MODE>;
  constexpr size_t lds = Gm::lds_bytes();
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(kern, dim3(n_groups), dim3(kThreads), lds, s, pairs, tiles, n_tiles, counter);
  return hipGetLastError();
}

template <int R, int DC, typename GT>
hipError_t launch_rdg(const Plan& P, const BilArgs& a, int mode, hipStream_t s) {
  constexpr int PX = kPX, TYT = kTYT;
  switch (mode) {
    case 0: return launch_one<R, PX, DC, TYT, GT, 0>(P, a, s);
    case 1: return launch_one<R, PX, DC, TYT, GT, 1>(P, a, s);
    case 2: return launch_one<R, PX, DC, TYT, GT, 2>(P, a, s);
    case 4: return launch_one<R, PX, DC, TYT, GT, 4>(P, a, s);
    case 5:
    case 6:
      if constexpr (std::is_same<GT, float>::value)
        return mode == 5 ? launch_one<R, PX, DC, TYT, GT, 5>(P, a, s)
                         : launch_one<R, PX, DC, TYT, GT, 6>(P, a, s);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

// Entry points of one radius (defined in k_bilateral_r<R>.hip).
template <int R>
hipError_t launch_r(const Plan& P, const BilArgs& a, int mode, hipStream_t s) {
  const int dc = a.guide_dt == STEREO_U8 ? P.agg_levels_u8 : P.agg_levels_f32;
  if (a.guide_dt == STEREO_U8)
    return dc == 16 ? launch_rdg<R, 16, uint8_t>(P, a, mode, s)
                    : launch_rdg<R, 8, uint8_t>(P, a, mode, s);
  return dc == 16 ? launch_rdg<R, 16, float>(P, a, mode, s)
                  : launch_rdg<R, 8, float>(P, a, mode, s);
}

template <int R>
hipError_t launch_persistent_r(stereo_dtype gdt, int levels, const BilPair* pairs,
                               const int* tiles, int n_tiles, unsigned int* counter,
                               int n_groups, hipStream_t s) {
  constexpr int PX = kPX, TYT = kTYT;
  if (gdt == STEREO_U8)
    return levels == 16 ? launch_persistent_one<R, PX, 16, TYT, uint8_t, 1>(pairs, tiles, n_tiles, counter, n_groups, s)
                        : launch_persistent_one<R, PX, 8, TYT, uint8_t, 1>(pairs, tiles, n_tiles, counter, n_groups, s);
  return levels == 16 ? launch_persistent_one<R, PX, 16, TYT, float, 1>(pairs, tiles, n_tiles, counter, n_groups, s)
                      : launch_persistent_one<R, PX, 8, TYT, float, 1>(pairs, tiles, n_tiles, counter, n_groups, s);
}

}  // namespace bil
}  // namespace stereo
