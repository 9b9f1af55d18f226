// Perspective transformation (Sec. 3.1, Eq. 4), block statistics (Sec. 4.3:
// means and deviations precomputed once) and the NCC matching cost of Eq. (8).
//
// Layout: images row-major with an element pitch; statistics maps [H][W+2r]
// over block centres x in [-r, W + r) (block reads are clamped, so centres
// further out repeat the edge values); cost slices [D][H][pitch].
#include "internal.h"

namespace stereo {
namespace {

template <typename T>
__device__ __forceinline__ float ld(const T* p) { return static_cast<float>(*p); }

// tar_w(x, v) = lerp of target row v at X = x + s(x, v), where
// s = delta_p - d_road(x + delta_p, v).  The shift is evaluated in FP64 apart
// from x so that the fractional position stays exact at large x.
template <typename T>
__global__ void __launch_bounds__(256)
warp_kernel(const T* __restrict__ tar, int64_t pitch, int W, int H,
            double delta_p, double c0, double c1, double c2, int persp,
            float* __restrict__ out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  if (x >= W) return;
  const T* row = tar + (int64_t)v * pitch;
  float val;
  if (!persp) {
    val = ld(row + x);
  } else {
    const double X = (double)x + delta_p - (c0 + c1 * ((double)x + delta_p) + c2 * (double)v);
    int i0;
    float f;
    if (X <= 0.0) {
      i0 = 0; f = 0.0f;
    } else if (X >= (double)(W - 1)) {
      i0 = W - 1; f = 0.0f;
    } else {
      const double fl = floor(X);
      i0 = (int)fl;
      f = (float)(X - fl);
    }
    const int i1 = min(i0 + 1, W - 1);
    val = (1.0f - f) * ld(row + i0) + f * ld(row + i1);
  }
  out[(int64_t)v * W + x] = val;
}

// Block statistics.  One workgroup covers 64 block centres x 16 rows; the
// clamped input tile (16 + 2r rows x 64 + 2r columns, offset by -128) is
// staged in LDS, then each thread forms the mean and the population
// deviation of its blocks in two passes (mean first, then squared deviations).
constexpr int ST_TX = 64, ST_TY = 16;

template <typename T>
__global__ void __launch_bounds__(256)
block_stats_kernel(const T* __restrict__ img, int64_t pitch, int W, int H, int r,
                   float* __restrict__ mu, float* __restrict__ isd) {
  extern __shared__ float tile[];   // (ST_TY + 2r) x (ST_TX + 2r)
  const int SW = W + 2 * r;
  const int tw = ST_TX + 2 * r, th = ST_TY + 2 * r;
  const int xc0 = blockIdx.x * ST_TX - r;    // first block centre (image col)
  const int y0 = blockIdx.y * ST_TY;
  for (int i = threadIdx.x; i < tw * th; i += blockDim.x) {
    const int yy = i / tw, xx = i - yy * tw;
    const int gy = min(max(y0 - r + yy, 0), H - 1);
    const int gx = min(max(xc0 - r + xx, 0), W - 1);
    tile[i] = ld(img + (int64_t)gy * pitch + gx) - kOffset;
  }
  __syncthreads();
  const int n = (2 * r + 1) * (2 * r + 1);
  const float inv_n = 1.0f / (float)n;
  for (int o = threadIdx.x; o < ST_TX * ST_TY; o += blockDim.x) {
    const int ty = o / ST_TX, tx = o - ty * ST_TX;
    const int xi = blockIdx.x * ST_TX + tx;       // map column index
    const int y = y0 + ty;
    if (xi >= SW || y >= H) continue;
    float s = 0.0f;
    for (int i = 0; i <= 2 * r; ++i)
      for (int j = 0; j <= 2 * r; ++j) s += tile[(ty + i) * tw + tx + j];
    const float m = s * inv_n;
    float q = 0.0f;
    for (int i = 0; i <= 2 * r; ++i)
      for (int j = 0; j <= 2 * r; ++j) {
        const float e = tile[(ty + i) * tw + tx + j] - m;
        q = fmaf(e, e, q);
      }
    const float var = q * inv_n;
    mu[(int64_t)y * SW + xi] = m;
    isd[(int64_t)y * SW + xi] = (var < kFlatVar) ? 0.0f : 1.0f / sqrtf(var);
  }
}

// NCC cost, Eq. (8), in its equivalent 1 - NCC form on offset intensities:
//   C = 1 - (S/n - muX muY) / (sdX sdY),  S = sum over the block of X' Y'.
// One workgroup covers NC_TX outputs x NC_TY rows x NC_DC levels.  The
// cross sums are separable: vertical sums of products first (fixed order
// i = 0..2r), then horizontal sums (fixed order j = 0..2r); the result is
// independent of the tiling.
constexpr int NC_TX = 64, NC_TY = 16, NC_DC = 8;

template <typename T>
__global__ void __launch_bounds__(256)
ncc_kernel(const T* __restrict__ ref, int64_t ref_pitch,
           const float* __restrict__ tarw, int W, int H, int D, int r,
           const float* __restrict__ muX, const float* __restrict__ isdX,
           const float* __restrict__ muY, const float* __restrict__ isdY,
           float* __restrict__ C, int out_w, int64_t out_pitch,
           int64_t out_slice, int anchor) {
  extern __shared__ float sm[];
  const int k = 2 * r + 1;
  const int tw = NC_TX + 2 * r + NC_DC - 1;     // tile width (both images)
  const int th = NC_TY + 2 * r;
  const int vw = NC_TX + 2 * r;                 // vertical-sum row width
  float* Xs = sm;
  float* Ys = Xs + th * tw;
  float* Vs = Ys + th * tw;                     // [NC_DC][NC_TY][vw]
  const int x0 = blockIdx.x * NC_TX;
  const int y0 = blockIdx.y * NC_TY;
  const int d0 = blockIdx.z * NC_DC;
  const int SW = W + 2 * r;
  // column origins (image coordinates) of the two tiles
  //   anchor 0: X at x + j - r,      Y at x - d + j - r
  //   anchor 1: X at x + d + j - r,  Y at x + j - r
  const int xoX = anchor ? x0 - r + d0 : x0 - r;
  const int xoY = anchor ? x0 - r : x0 - r - d0 - (NC_DC - 1);
  for (int i = threadIdx.x; i < th * tw; i += blockDim.x) {
    const int yy = i / tw, xx = i - yy * tw;
    const int gy = min(max(y0 - r + yy, 0), H - 1);
    const int gxX = min(max(xoX + xx, 0), W - 1);
    const int gxY = min(max(xoY + xx, 0), W - 1);
    Xs[i] = ld(ref + (int64_t)gy * ref_pitch + gxX) - kOffset;
    Ys[i] = tarw[(int64_t)gy * W + gxY] - kOffset;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < NC_DC * NC_TY * vw; i += blockDim.x) {
    const int dc = i / (NC_TY * vw);
    const int rem = i - dc * NC_TY * vw;
    const int y = rem / vw, xx = rem - y * vw;
    const int cx = anchor ? xx + dc : xx;
    const int cy = anchor ? xx : xx + (NC_DC - 1 - dc);
    float s = 0.0f;
    for (int a = 0; a < k; ++a) s = fmaf(Xs[(y + a) * tw + cx], Ys[(y + a) * tw + cy], s);
    Vs[i] = s;
  }
  __syncthreads();
  const float inv_n = 1.0f / (float)(k * k);
  for (int i = threadIdx.x; i < NC_DC * NC_TY * NC_TX; i += blockDim.x) {
    const int dc = i / (NC_TY * NC_TX);
    const int rem = i - dc * NC_TY * NC_TX;
    const int y = rem / NC_TX, xo = rem - y * NC_TX;
    const int d = d0 + dc, gy = y0 + y, gx = x0 + xo;
    if (d >= D || gy >= H || gx >= out_w) continue;
    const float* vrow = Vs + (dc * NC_TY + y) * vw + xo;
    float S = 0.0f;
    for (int a = 0; a < k; ++a) S += vrow[a];
    // statistics at the block centres, clamped to the map's column range
    const int cxX = min(max(anchor ? gx + d : gx, -r), W - 1 + r) + r;
    const int cxY = min(max(anchor ? gx : gx - d, -r), W - 1 + r) + r;
    const float ix = isdX[(int64_t)gy * SW + cxX];
    const float iy = isdY[(int64_t)gy * SW + cxY];
    float c = 1.0f;
    if (ix != 0.0f && iy != 0.0f) {
      const float cov = fmaf(S, inv_n, -muX[(int64_t)gy * SW + cxX] * muY[(int64_t)gy * SW + cxY]);
      c = 1.0f - cov * ix * iy;
    }
    C[(int64_t)d * out_slice + (int64_t)gy * out_pitch + gx] = c;
  }
}

}  // namespace

hipError_t launch_warp(const Plan& P, const void* tar, float* tar_w, hipStream_t s) {
  dim3 grid((P.W + 255) / 256, P.H);
  const stereo_params& p = P.p;
  const double dp = p.perspective ? (double)p.delta_p : 0.0;
  if (p.dtype == STEREO_U8)
    hipLaunchKernelGGL(warp_kernel<uint8_t>, grid, dim3(256), 0, s,
                       (const uint8_t*)tar, p.pitch_tar, P.W, P.H, dp, p.plane[0],
                       p.plane[1], p.plane[2], p.perspective, tar_w);
  else
    hipLaunchKernelGGL(warp_kernel<float>, grid, dim3(256), 0, s,
                       (const float*)tar, p.pitch_tar, P.W, P.H, dp, p.plane[0],
                       p.plane[1], p.plane[2], p.perspective, tar_w);
  return hipGetLastError();
}

hipError_t launch_block_stats(const Plan& P, const void* img, stereo_dtype dt,
                              int64_t pitch, float* mu, float* isd, hipStream_t s) {
  const int SW = P.W + 2 * P.r;
  dim3 grid((SW + ST_TX - 1) / ST_TX, (P.H + ST_TY - 1) / ST_TY);
  const size_t lds = sizeof(float) * (ST_TX + 2 * P.r) * (ST_TY + 2 * P.r);
  if (dt == STEREO_U8)
    hipLaunchKernelGGL(block_stats_kernel<uint8_t>, grid, dim3(256), lds, s,
                       (const uint8_t*)img, pitch, P.W, P.H, P.r, mu, isd);
  else
    hipLaunchKernelGGL(block_stats_kernel<float>, grid, dim3(256), lds, s,
                       (const float*)img, pitch, P.W, P.H, P.r, mu, isd);
  return hipGetLastError();
}

hipError_t launch_ncc(const Plan& P, const void* ref, const float* tar_w,
                      const float* muX, const float* isdX, const float* muY,
                      const float* isdY, float* C, int out_w, int64_t out_pitch,
                      int64_t out_slice, int anchor, hipStream_t s) {
  dim3 grid((out_w + NC_TX - 1) / NC_TX, (P.H + NC_TY - 1) / NC_TY,
            (P.D + NC_DC - 1) / NC_DC);
  const int r = P.r;
  const size_t tile = (size_t)(NC_TY + 2 * r) * (NC_TX + 2 * r + NC_DC - 1);
  const size_t lds = sizeof(float) * (2 * tile + (size_t)NC_DC * NC_TY * (NC_TX + 2 * r));
  if (P.p.dtype == STEREO_U8)
    hipLaunchKernelGGL(ncc_kernel<uint8_t>, grid, dim3(256), lds, s,
                       (const uint8_t*)ref, P.p.pitch_ref, tar_w, P.W, P.H, P.D, r,
                       muX, isdX, muY, isdY, C, out_w, out_pitch, out_slice, anchor);
  else
    hipLaunchKernelGGL(ncc_kernel<float>, grid, dim3(256), lds, s,
                       (const float*)ref, P.p.pitch_ref, tar_w, P.W, P.H, P.D, r,
                       muX, isdX, muY, isdY, C, out_w, out_pitch, out_slice, anchor);
  return hipGetLastError();
}

}  // namespace stereo
