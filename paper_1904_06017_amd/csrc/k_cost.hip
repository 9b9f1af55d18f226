// Perspective transformation (Sec. 3.1, Eq. 4), block statistics (Sec. 4.3:
// means and deviations precomputed once) and the NCC matching cost of Eq. (8).
//
// Layout: images row-major with an element pitch; statistics maps [H][W+2r]
// over block centres x in [-r, W + r) (block reads are clamped, so centres
// further out repeat the edge values); cost slices [D][H][pitch].
#include "ncc_impl.h"

namespace stereo {
namespace {

// tar_w(x, v) = lerp of target row v at X = x + s(x, v), where
// s = delta_p - d_road(x + delta_p, v).  The shift is evaluated in FP64 apart
// from x so that the fractional position stays exact at large x.
template <typename T>
__device__ __forceinline__ void warp_body(const T* __restrict__ tar, int64_t pitch, int W,
                                          double delta_p, double c0, double c1, double c2,
                                          int persp, float* __restrict__ out, int bx, int v) {
  const int x = bx * 256 + threadIdx.x;
  if (x >= W) return;
  const T* row = tar + (int64_t)v * pitch;
  float val;
  if (!persp) {
    val = ld(row + x);
  } else {
    // explicit fused multiply-adds: the rounding does not depend on how the
    // compiler contracts the expression where this body is inlined
    const double ux = (double)x + delta_p;
    const double X = ux - fma(c2, (double)v, fma(c1, ux, c0));
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
    val = fmaf(f, ld(row + i1), (1.0f - f) * ld(row + i0));
  }
  out[(int64_t)v * W + x] = val;
}

// Eq. (3) in full: tar_w(x, v) = target at H (x + delta_p, v, 1)^T, read
// bilinearly with both coordinates clamped; positions in FP64.
template <typename T>
__device__ __forceinline__ void warp_h_body(const T* __restrict__ tar, int64_t pitch, int W,
                                            int H, double delta_p, const Homog& M,
                                            float* __restrict__ out, int bx, int v) {
  const int x = bx * 256 + threadIdx.x;
  if (x >= W) return;
  const double* h = M.h;
  const double u = (double)x + delta_p, vv = (double)v;
  const double z = fma(h[6], u, fma(h[7], vv, h[8]));
  double X = fma(h[0], u, fma(h[1], vv, h[2])) / z;
  double Y = fma(h[3], u, fma(h[4], vv, h[5])) / z;
  X = fmin(fmax(X, 0.0), (double)(W - 1));
  Y = fmin(fmax(Y, 0.0), (double)(H - 1));
  const double fx0 = floor(X), fy0 = floor(Y);
  const int i0 = (int)fx0, j0 = (int)fy0;
  const int i1 = min(i0 + 1, W - 1), j1 = min(j0 + 1, H - 1);
  const float fx = (float)(X - fx0), fy = (float)(Y - fy0);
  const T* r0 = tar + (int64_t)j0 * pitch;
  const T* r1 = tar + (int64_t)j1 * pitch;
  const float top = fmaf(fx, ld(r0 + i1), (1.0f - fx) * ld(r0 + i0));
  const float bot = fmaf(fx, ld(r1 + i1), (1.0f - fx) * ld(r1 + i0));
  out[(int64_t)v * W + x] = fmaf(fy, bot, (1.0f - fy) * top);
}

template <typename T>
__global__ void __launch_bounds__(256)
warp_h_kernel(const T* __restrict__ tar, int64_t pitch, int W, int H, double delta_p, Homog M,
              float* __restrict__ out) {
  warp_h_body<T>(tar, pitch, W, H, delta_p, M, out, blockIdx.x, blockIdx.y);
}

template <typename T>
__global__ void __launch_bounds__(256)
warp_kernel(const T* __restrict__ tar, int64_t pitch, int W, int H,
            double delta_p, double c0, double c1, double c2, int persp,
            float* __restrict__ out) {
  warp_body<T>(tar, pitch, W, delta_p, c0, c1, c2, persp, out, blockIdx.x, blockIdx.y);
}

template <typename T>
__global__ void __launch_bounds__(256)
warp_tracked_kernel(const T* __restrict__ tar, int64_t pitch, int W, double delta_p,
                    const stereo_plane_state* __restrict__ st, float* __restrict__ out) {
  warp_body<T>(tar, pitch, W, delta_p, st->plane[0], st->plane[1], st->plane[2], 1, out,
               blockIdx.x, blockIdx.y);
}

// Block statistics.  One workgroup covers 64 block centres x 16 rows; the
// clamped input tile (16 + 2r rows x 64 + 2r columns, offset by -128) is
// staged in LDS.  The block sums of x and x^2 are separable: a vertical pass
// sums 2r + 1 rows per tile column, a horizontal pass 2r + 1 of those column
// sums per block.  Both run in FP64 (the vector FP64 rate equals the FP32
// one here): x^2 of an FP32 value is exact in FP64 and sums of at most 289
// of them lose nothing that matters, so the one-pass variance
// q / n - (s / n)^2 carries no cancellation error.  Stored as z = mu / sigma
// and isd = 1 / sigma (rounded to FP32 once), so that the cost is
// 1 + zX zY - (S / n) isdX isdY; a flat block (variance below kFlatVar)
// stores z = isd = 0, which makes its cost exactly 1 without a branch.
constexpr int ST_TX = 64, ST_TY = 16;

__host__ __device__ constexpr size_t stats_lds_bytes(int r) {
  return sizeof(float) * (size_t)(ST_TX + 2 * r) * (ST_TY + 2 * r) +
         2 * sizeof(double) * (size_t)ST_TY * (ST_TX + 2 * r);
}

template <typename T>
__device__ __forceinline__ void block_stats_body(const T* __restrict__ img, int64_t pitch,
                                                 int W, int H, int r, float* __restrict__ zmap,
                                                 float* __restrict__ isd, float* tile, int bx,
                                                 int by) {
  const int SW = W + 2 * r;
  const int tw = ST_TX + 2 * r, th = ST_TY + 2 * r;
  const int xc0 = bx * ST_TX - r;            // first block centre (image col)
  const int y0 = by * ST_TY;
  // staged in chunks: four loads of a thread in flight before their stores
  for (int i0 = threadIdx.x; i0 < tw * th; i0 += 4 * (int)blockDim.x) {
    float v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = min(i0 + k * (int)blockDim.x, tw * th - 1);
      const int yy = i / tw, xx = i - yy * tw;
      const int gy = min(max(y0 - r + yy, 0), H - 1);
      const int gx = min(max(xc0 - r + xx, 0), W - 1);
      v[k] = ld(img + (int64_t)gy * pitch + gx);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = i0 + k * (int)blockDim.x;
      if (i < tw * th) tile[i] = v[k] - kOffset;
    }
  }
  // column sums of the block rows of each output row: [ST_TY][tw], x and x^2
  double* cs = reinterpret_cast<double*>(tile + tw * th);
  double* cq = cs + ST_TY * tw;
  __syncthreads();
  const int k = 2 * r + 1;
  for (int o = threadIdx.x; o < ST_TY * tw; o += blockDim.x) {
    const int ty = o / tw, c = o - ty * tw;
    double sx = 0.0, sq = 0.0;
    for (int i = 0; i < k; ++i) {
      const double v = (double)tile[(ty + i) * tw + c];
      sx += v;
      sq = fma(v, v, sq);
    }
    cs[o] = sx;
    cq[o] = sq;
  }
  __syncthreads();
  const double inv_n = 1.0 / (double)(k * k);
  for (int o = threadIdx.x; o < ST_TX * ST_TY; o += blockDim.x) {
    const int ty = o / ST_TX, tx = o - ty * ST_TX;
    const int xi = bx * ST_TX + tx;               // map column index
    const int y = y0 + ty;
    if (xi >= SW || y >= H) continue;
    double sx = 0.0, sq = 0.0;
    for (int j = 0; j < k; ++j) {
      sx += cs[ty * tw + tx + j];
      sq += cq[ty * tw + tx + j];
    }
    const double m = sx * inv_n;
    const double var = fma(-m, m, sq * inv_n);
    const double is = (var < (double)kFlatVar) ? 0.0 : 1.0 / sqrt(var);
    zmap[(int64_t)y * SW + xi] = (float)(m * is);
    isd[(int64_t)y * SW + xi] = (float)is;
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
block_stats_kernel(const T* __restrict__ img, int64_t pitch, int W, int H, int r,
                   float* __restrict__ zmap, float* __restrict__ isd) {
  extern __shared__ float tile[];   // (ST_TY + 2r) x (ST_TX + 2r)
  block_stats_body<T>(img, pitch, W, H, r, zmap, isd, tile, blockIdx.x, blockIdx.y);
}

// Both images of a pair in one launch: blockIdx.z = 0 the reference (T),
// 1 the warped target (FP32).
template <typename T>
__global__ void __launch_bounds__(256)
block_stats2_kernel(const T* __restrict__ ref, int64_t ref_pitch, const float* __restrict__ tarw,
                    int W, int H, int r, float* __restrict__ zX, float* __restrict__ isdX,
                    float* __restrict__ zY, float* __restrict__ isdY) {
  extern __shared__ float tile[];
  if (blockIdx.z == 0)
    block_stats_body<T>(ref, ref_pitch, W, H, r, zX, isdX, tile, blockIdx.x, blockIdx.y);
  else
    block_stats_body<float>(tarw, W, W, H, r, zY, isdY, tile, blockIdx.x, blockIdx.y);
}

template <typename T>
__global__ void __launch_bounds__(256)
warp_jobs_kernel(const WarpJob* __restrict__ jobs, const int* __restrict__ first, int n) {
  const int j = job_of(first, n, blockIdx.x);
  const WarpJob& J = jobs[j];
  const int l = blockIdx.x - first[j];
  if (J.homog)
    warp_h_body<T>(static_cast<const T*>(J.tar), J.pitch, J.W, J.H, J.dp, J.Hm, J.out,
                   l % J.gx, l / J.gx);
  else
    warp_body<T>(static_cast<const T*>(J.tar), J.pitch, J.W, J.dp, J.c0, J.c1, J.c2, J.persp,
                 J.out, l % J.gx, l / J.gx);
}

template <typename T>
__global__ void __launch_bounds__(256)
stats_jobs_kernel(const StatsJob* __restrict__ jobs, const int* __restrict__ first, int n) {
  extern __shared__ float tile[];
  const int j = job_of(first, n, blockIdx.x);
  const StatsJob& J = jobs[j];
  const int l = blockIdx.x - first[j];
  block_stats_body<T>(static_cast<const T*>(J.img), J.pitch, J.W, J.H, J.r, J.z, J.isd, tile,
                      l % J.gx, l / J.gx);
}

hipError_t launch_ncc_any(const Plan& P, const void* ref, const float* tar_w, const float* zX,
                          const float* isdX, const float* zY, const float* isdY, float* C,
                          int out_w, int64_t out_pitch, int64_t out_slice, int anchor,
                          int d_first, int d_end, int quad, int pad, hipStream_t s, float* C2) {
#define NCC_CASE(R_) \
  case R_: return launch_ncc_r##R_(P, ref, tar_w, zX, isdX, zY, isdY, C, out_w, out_pitch, \
                                   out_slice, anchor, d_first, d_end, quad, pad, s, C2);
  switch (P.r) {
    NCC_CASE(1) NCC_CASE(2) NCC_CASE(3) NCC_CASE(4)
    NCC_CASE(5) NCC_CASE(6) NCC_CASE(7) NCC_CASE(8)
    default: return hipErrorInvalidValue;
  }
#undef NCC_CASE
}

}  // namespace

int warp_job_blocks(const Plan& P) { return ((P.W + 255) / 256) * P.H; }
int stats_job_blocks(int W, int H, int r) {
  return ((W + 2 * r + ST_TX - 1) / ST_TX) * ((H + ST_TY - 1) / ST_TY);
}
int ncc_job_blocks(const Plan& P, int out_w, int d_first, int d_end, int dc, int quad) {
  const int tx = quad == 4 ? NC_TX4 : NC_TX;
  return ((out_w + tx - 1) / tx) * ((P.H + NC_TY - 1) / NC_TY) *
         ((d_end - d_first + dc - 1) / dc);
}
int ncc_both_extent(int out_pitch, int d_first, int d_end) {
  return out_pitch + (((d_end - d_first) + 15) & ~15);
}

WarpJob warp_job(const Plan& P, const void* tar, float* tar_w) {
  const stereo_params& p = P.p;
  WarpJob J{};
  J.tar = tar; J.pitch = p.pitch_tar; J.out = tar_w;
  J.dp = p.perspective ? (double)p.delta_p : 0.0;
  J.c0 = p.plane[0]; J.c1 = p.plane[1]; J.c2 = p.plane[2];
  J.W = P.W; J.H = P.H; J.persp = p.perspective; J.gx = (P.W + 255) / 256;
  J.homog = P.homog;
  for (int k = 0; k < 9; ++k) J.Hm.h[k] = P.Hm[k];
  return J;
}

StatsJob stats_job(const Plan& P, const void* img, int64_t pitch, float* z, float* isd) {
  StatsJob J{};
  J.img = img; J.pitch = pitch; J.z = z; J.isd = isd;
  J.W = P.W; J.H = P.H; J.r = P.r; J.gx = (P.W + 2 * P.r + ST_TX - 1) / ST_TX;
  return J;
}

NccJob ncc_job(const Plan& P, const void* ref, const float* tar_w, const float* zX,
               const float* isdX, const float* zY, const float* isdY, float* C, int out_w,
               int64_t out_pitch, int64_t out_slice, int anchor, int d_first, int d_end,
               int quad, float* C2, const void* base) {
  NccJob J{};
  J.C2 = C2;
  J.c_off = reinterpret_cast<const char*>(C) - static_cast<const char*>(base);
  J.c2_off = C2 ? reinterpret_cast<const char*>(C2) - static_cast<const char*>(base) : -1;
  J.ref = ref; J.ref_pitch = P.p.pitch_ref; J.tarw = tar_w;
  J.zX = zX; J.isdX = isdX; J.zY = zY; J.isdY = isdY;
  J.C = C; J.out_pitch = out_pitch; J.out_slice = out_slice;
  J.W = P.W; J.H = P.H; J.d_first = d_first; J.d_end = d_end < 0 ? P.D : d_end;
  J.out_w = out_w; J.anchor = anchor;
  const int tx = quad == 4 ? NC_TX4 : NC_TX;
  J.gx = (out_w + tx - 1) / tx; J.gy = (P.H + NC_TY - 1) / NC_TY;
  return J;
}

hipError_t launch_warp_jobs(stereo_dtype dt, const WarpJob* jobs, const int* first, int n,
                            int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  if (dt == STEREO_U8)
    hipLaunchKernelGGL(warp_jobs_kernel<uint8_t>, dim3(blocks), dim3(256), 0, s, jobs, first, n);
  else
    hipLaunchKernelGGL(warp_jobs_kernel<float>, dim3(blocks), dim3(256), 0, s, jobs, first, n);
  return hipGetLastError();
}

hipError_t launch_stats_jobs(stereo_dtype dt, const StatsJob* jobs, const int* first, int n,
                             int blocks, int max_r, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  const size_t lds = stats_lds_bytes(max_r);
  if (dt == STEREO_U8)
    hipLaunchKernelGGL(stats_jobs_kernel<uint8_t>, dim3(blocks), dim3(256), lds, s, jobs, first,
                       n);
  else
    hipLaunchKernelGGL(stats_jobs_kernel<float>, dim3(blocks), dim3(256), lds, s, jobs, first, n);
  return hipGetLastError();
}


hipError_t launch_ncc_jobs(int r, stereo_dtype dt, int quad, int dc, const NccJob* jobs,
                           const int* first, int n, int blocks, char* base, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  switch (r) {
    case 1: return launch_ncc_jobs_r1(dt, quad, dc, jobs, first, n, blocks, base, s);
    case 2: return launch_ncc_jobs_r2(dt, quad, dc, jobs, first, n, blocks, base, s);
    case 3: return launch_ncc_jobs_r3(dt, quad, dc, jobs, first, n, blocks, base, s);
    case 4: return launch_ncc_jobs_r4(dt, quad, dc, jobs, first, n, blocks, base, s);
    case 5: return launch_ncc_jobs_r5(dt, quad, dc, jobs, first, n, blocks, base, s);
    case 6: return launch_ncc_jobs_r6(dt, quad, dc, jobs, first, n, blocks, base, s);
    case 7: return launch_ncc_jobs_r7(dt, quad, dc, jobs, first, n, blocks, base, s);
    case 8: return launch_ncc_jobs_r8(dt, quad, dc, jobs, first, n, blocks, base, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_warp(const Plan& P, const void* tar, float* tar_w, hipStream_t s) {
  dim3 grid((P.W + 255) / 256, P.H);
  const stereo_params& p = P.p;
  if (P.homog) {
    Homog M;
    for (int k = 0; k < 9; ++k) M.h[k] = P.Hm[k];
    if (p.dtype == STEREO_U8)
      hipLaunchKernelGGL(warp_h_kernel<uint8_t>, grid, dim3(256), 0, s, (const uint8_t*)tar,
                         p.pitch_tar, P.W, P.H, (double)p.delta_p, M, tar_w);
    else
      hipLaunchKernelGGL(warp_h_kernel<float>, grid, dim3(256), 0, s, (const float*)tar,
                         p.pitch_tar, P.W, P.H, (double)p.delta_p, M, tar_w);
    return hipGetLastError();
  }
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

hipError_t launch_warp_tracked(const Plan& P, const void* tar, const stereo_plane_state* st,
                               float* tar_w, hipStream_t s) {
  dim3 grid((P.W + 255) / 256, P.H);
  const double dp = (double)P.p.delta_p;
  if (P.p.dtype == STEREO_U8)
    hipLaunchKernelGGL(warp_tracked_kernel<uint8_t>, grid, dim3(256), 0, s,
                       (const uint8_t*)tar, P.p.pitch_tar, P.W, dp, st, tar_w);
  else
    hipLaunchKernelGGL(warp_tracked_kernel<float>, grid, dim3(256), 0, s,
                       (const float*)tar, P.p.pitch_tar, P.W, dp, st, tar_w);
  return hipGetLastError();
}

hipError_t launch_block_stats2(const Plan& P, const void* ref, stereo_dtype dt,
                               int64_t ref_pitch, const float* tarw, float* zX, float* isdX,
                               float* zY, float* isdY, hipStream_t s) {
  const int SW = P.W + 2 * P.r;
  dim3 grid((SW + ST_TX - 1) / ST_TX, (P.H + ST_TY - 1) / ST_TY, 2);
  const size_t lds = stats_lds_bytes(P.r);
  if (dt == STEREO_U8)
    hipLaunchKernelGGL(block_stats2_kernel<uint8_t>, grid, dim3(256), lds, s,
                       (const uint8_t*)ref, ref_pitch, tarw, P.W, P.H, P.r, zX, isdX, zY, isdY);
  else
    hipLaunchKernelGGL(block_stats2_kernel<float>, grid, dim3(256), lds, s, (const float*)ref,
                       ref_pitch, tarw, P.W, P.H, P.r, zX, isdX, zY, isdY);
  return hipGetLastError();
}

hipError_t launch_block_stats(const Plan& P, const void* img, stereo_dtype dt,
                              int64_t pitch, float* z, float* isd, hipStream_t s) {
  const int SW = P.W + 2 * P.r;
  dim3 grid((SW + ST_TX - 1) / ST_TX, (P.H + ST_TY - 1) / ST_TY);
  const size_t lds = stats_lds_bytes(P.r);
  if (dt == STEREO_U8)
    hipLaunchKernelGGL(block_stats_kernel<uint8_t>, grid, dim3(256), lds, s,
                       (const uint8_t*)img, pitch, P.W, P.H, P.r, z, isd);
  else
    hipLaunchKernelGGL(block_stats_kernel<float>, grid, dim3(256), lds, s,
                       (const float*)img, pitch, P.W, P.H, P.r, z, isd);
  return hipGetLastError();
}

hipError_t launch_ncc(const Plan& P, const void* ref, const float* tar_w,
                      const float* zX, const float* isdX, const float* zY,
                      const float* isdY, float* C, int out_w, int64_t out_pitch,
                      int64_t out_slice, int anchor, hipStream_t s, int d_first, int d_end,
                      int quad, int pad, float* C2) {
  if (d_end < 0) d_end = P.D;
  if (quad == 1 && (d_first & 3)) return hipErrorInvalidValue;
  if (quad >= 2 && (d_first & 15 || pad < 0 || (out_pitch & 7) || out_w < out_pitch))
    return hipErrorInvalidValue;
  if (quad == 4 && out_w < ncc_both_extent((int)out_pitch, d_first, d_end))
    return hipErrorInvalidValue;
  if (quad == 3 && (!C2 || P.p.dtype != STEREO_F32)) return hipErrorInvalidValue;
  return launch_ncc_any(P, ref, tar_w, zX, isdX, zY, isdY, C, out_w, out_pitch, out_slice,
                        anchor, d_first, d_end, quad, pad, s, C2);
}

}  // namespace stereo
