// Perspective transformation (Sec. 3.1, Eq. 4), block statistics (Sec. 4.3:
// means and deviations precomputed once) and the NCC matching cost of Eq. (8).
//
// Layout: images row-major with an element pitch; statistics maps [H][W+2r]
// over block centres x in [-r, W + r) (block reads are clamped, so centres
// further out repeat the edge values); cost slices [D][H][pitch].
#include <type_traits>

#include "internal.h"

namespace stereo {
namespace {

template <typename T>
__device__ __forceinline__ float ld(const T* p) { return static_cast<float>(*p); }

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
  for (int i = threadIdx.x; i < tw * th; i += blockDim.x) {
    const int yy = i / tw, xx = i - yy * tw;
    const int gy = min(max(y0 - r + yy, 0), H - 1);
    const int gx = min(max(xc0 - r + xx, 0), W - 1);
    tile[i] = ld(img + (int64_t)gy * pitch + gx) - kOffset;
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

// NCC cost, Eq. (8), in its equivalent 1 - NCC form on offset intensities:
//   C = 1 - (S/n - muX muY) / (sdX sdY) = 1 + zX zY - (S/n) isdX isdY,
// S = sum over the block of X' Y', z = mu / sd, isd = 1 / sd.
// A workgroup covers NC_TX = 64 output columns (one per lane, conflict-free
// LDS rows) x NC_TY rows x NC_DC levels (NC_DW per wave).  Each lane walks
// down its column: for every input row it forms the horizontal sum of the
// 2r+1 products (fixed order j = -r..r) and keeps the last 2r+1 row sums in a
// register ring; the block sum is the fixed-order sum of that ring
// (i = -r..r).  Every output is the same expression whatever the tiling.
//
// The unshifted operand A (X' for anchor 0, Y' for anchor 1), the
// level-shifted operand B and the B side's statistics of the workgroup's
// output rows (z and 1/sd at the shifted block centres: one contiguous column
// range per row) are staged in LDS with clamped reads.  A wave's NC_DW
// levels read overlapping windows of the same B row: one window of
// K + NC_DW - 1 values serves them all.
constexpr int NC_TX = 64, NC_TY = 32, NC_DC = 16, NC_DW = 4;
// NC_DC is the default level block; a workgroup of DC levels has DC / 4 waves.

template <int r, int DC = NC_DC>
struct NccGeom {
  static constexpr int K = 2 * r + 1;
  static constexpr int ROWS = NC_TY + 2 * r;
  static constexpr int AW = NC_TX + 2 * r;
  static constexpr int BW = NC_TX + 2 * r + DC - 1;
  static constexpr int ZW = NC_TX + DC - 1;         // B-side statistics per output row
  static constexpr size_t lds_bytes =
      sizeof(float) * ((size_t)ROWS * (AW + BW) + 2 * (size_t)NC_TY * ZW);
};

// QUAD = 1 writes the level-quad-interleaved layout [levels/4][H][pitch]
// float4 (out_slice and out_pitch in float4 units; levels at or past d_end
// inside the last quad are written as 0), QUAD = 0 the planar layout
// [levels][H][pitch].  QUAD = 2 writes the split-FP16 volumes of the
// FP16-operand matrix-core aggregation (anchor 0 over the extended columns,
// d_first = 0): blocks of 16 levels, each [part][H][pitch / 4 column quads]
// [16 levels][4 columns] halves, i.e. level d of stored column s = x + pad at
// ((2 (d >> 4) + part) H + y) 16 pitch + 64 (s >> 2) + 4 (d & 15) + (s & 3),
// out_slice = 16 H pitch, out_pitch = pitch; part 0 = FP16 rounding of the
// cost, part 1 = FP16 rounding of the remainder; the anchor decides which
// volume (0: reference-anchored, 1: target-anchored).  The tiles start pad
// columns left of their 64-column boundary, so a lane quad is a stored column
// quad and, after a transpose within the quad, each lane writes 4 columns of
// one level as 8 bytes; the grid's columns cover the stored row
// (out_w >= out_pitch), columns outside [0, W) and the last block's levels at
// or past d_end are written as zeros.  QUAD = 4 writes both anchors' split
// volumes from one pass (the target-anchored one to C2 when non-NULL): the
// cost of reference column x at level d is also the target-anchored cost of
// column m = x - d, the same two blocks and the same products.  Tiles step
// by NC_TX4 = 60 columns; lane x + k holds level d + k of target column m,
// so three lane shifts (level k from k lanes to the right) line a quad of
// lanes up with a stored column quad of that volume, after which the same
// transpose gives 8-byte stores.  The last quad of lanes only feeds the
// shifts.  The grid covers x < out_w = stored row + the 16-rounded levels,
// so that every target column, pads included, is written at every level.
constexpr int NC_TX4 = 60;
// 4x4 transpose within each quad of lanes (lane c of a quad holds v[0..3];
// afterwards v[k] holds what lane k held in element c): two butterfly stages
// of DPP quad permutations, swapping the off-diagonal 2x2 blocks.
__device__ __forceinline__ float dpp_quad_xor1(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ float dpp_quad_xor2(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0x4E, 0xF, 0xF, false));
}
__device__ __forceinline__ void quad_transpose4(float (&v)[4], int lane) {
  const bool b0 = lane & 1, b1 = lane & 2;
  float t[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) t[k] = dpp_quad_xor1(v[k ^ 1]);
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = (b0 != (bool)(k & 1)) ? t[k] : v[k];
#pragma unroll
  for (int k = 0; k < 4; ++k) t[k] = dpp_quad_xor2(v[k ^ 2]);
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = (b1 != (bool)(k & 2)) ? t[k] : v[k];
}

// v = hi + lo in FP16 (round to nearest; lo rounds the exact remainder),
// four values packed two per register.
__device__ __forceinline__ void split4_f16(const float (&v)[4], uint2& hi, uint2& lo) {
  typedef _Float16 h2 __attribute__((ext_vector_type(2)));
  typedef float f2 __attribute__((ext_vector_type(2)));
  const h2 h01 = __builtin_convertvector((f2){v[0], v[1]}, h2);
  const h2 h23 = __builtin_convertvector((f2){v[2], v[3]}, h2);
  const h2 l01 = __builtin_convertvector((f2){v[0] - (float)h01.x, v[1] - (float)h01.y}, h2);
  const h2 l23 = __builtin_convertvector((f2){v[2] - (float)h23.x, v[3] - (float)h23.y}, h2);
  hi = make_uint2(__builtin_bit_cast(unsigned, h01), __builtin_bit_cast(unsigned, h23));
  lo = make_uint2(__builtin_bit_cast(unsigned, l01), __builtin_bit_cast(unsigned, l23));
}

template <int r, typename T, int QUAD, int DC>
__device__ __forceinline__ void ncc_body(const T* __restrict__ ref, int64_t ref_pitch,
                                         const float* __restrict__ tarw, int W, int H,
                                         int d_first, int d_end,
                                         const float* __restrict__ zX,
                                         const float* __restrict__ isdX,
                                         const float* __restrict__ zY,
                                         const float* __restrict__ isdY,
                                         float* __restrict__ C, int out_w, int64_t out_pitch,
                                         int64_t out_slice, int anchor, int pad, float* sm, int bx,
                                         int by, int bz, float* __restrict__ C2 = nullptr) {
  using G = NccGeom<r, DC>;
  constexpr int K = G::K;
  float* As = sm;                         // [ROWS][AW]
  float* Bs = sm + G::ROWS * G::AW;       // [ROWS][BW]
  float* Zs = Bs + G::ROWS * G::BW;       // [NC_TY][ZW]: z of the B side
  float* Is = Zs + NC_TY * G::ZW;         // [NC_TY][ZW]: 1/sd of the B side
  // split-FP16 output: the tile starts pad columns left of 64 bx, so that
  // lane l writes stored column 64 bx + l and a lane quad is a column quad
  const int x0 = QUAD == 4 ? bx * NC_TX4 - pad : bx * NC_TX - (QUAD >= 2 ? pad : 0);
  const int y0 = by * NC_TY;
  const int d0 = d_first + bz * DC;
  const int SW = W + 2 * r;
  // image column of A[.][0] and B[.][0]
  //   anchor 0: A = X' at x + j - r, B = Y' at x - d + j - r
  //   anchor 1: A = Y' at x + j - r, B = X' at x + d + j - r
  const int axo = x0 - r;
  const int bxo = anchor ? x0 - r + d0 : x0 - r - d0 - (DC - 1);
  for (int i = threadIdx.x; i < G::ROWS * G::BW; i += blockDim.x) {
    const int yy = i / G::BW, xx = i - yy * G::BW;
    const int gy = min(max(y0 - r + yy, 0), H - 1);
    const int gxb = min(max(bxo + xx, 0), W - 1);
    Bs[i] = anchor ? ld(ref + (int64_t)gy * ref_pitch + gxb) - kOffset
                   : tarw[(int64_t)gy * W + gxb] - kOffset;
    if (xx < G::AW) {
      const int gxa = min(max(axo + xx, 0), W - 1);
      As[yy * G::AW + xx] = anchor ? tarw[(int64_t)gy * W + gxa] - kOffset
                                   : ld(ref + (int64_t)gy * ref_pitch + gxa) - kOffset;
    }
  }
  // B-side statistics: entry c of output row t is the block centred at image
  // column zxo + c (clamped to the map's [-r, W - 1 + r]), the centre that
  // level offset boff reads for lane c - boff
  {
    const int zxo = anchor ? x0 + d0 : x0 - d0 - (DC - 1);
    const float* zm = anchor ? zX : zY;
    const float* im = anchor ? isdX : isdY;
    for (int i = threadIdx.x; i < NC_TY * G::ZW; i += blockDim.x) {
      const int t = i / G::ZW, c = i - t * G::ZW;
      const int64_t rowo = (int64_t)min(y0 + t, H - 1) * SW;
      const int cb = min(max(zxo + c, -r), W - 1 + r) + r;
      Zs[i] = zm[rowo + cb];
      Is[i] = im[rowo + cb];
    }
  }
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int x = x0 + lane;
  int boff[NC_DW];
#pragma unroll
  for (int k = 0; k < NC_DW; ++k) {
    const int dc = wave * NC_DW + k;
    boff[k] = anchor ? dc : (DC - 1 - dc);
  }
  const int bmin = anchor ? boff[0] : boff[NC_DW - 1];
  const float inv_n = 1.0f / (float)(K * K);
  float ring[NC_DW][K];
#pragma unroll
  for (int k = 0; k < NC_DW; ++k)
#pragma unroll
    for (int i = 0; i < K; ++i) ring[k][i] = 0.0f;
  const int cx = min(max(x, -r), W - 1 + r) + r;   // centre of the A block in the maps

  for (int yb = 0; yb < G::ROWS; yb += K) {
#pragma unroll
    for (int s = 0; s < K; ++s) {
      const int yy = yb + s;
      if (yy < G::ROWS) {
        float a[K];
#pragma unroll
        for (int j = 0; j < K; ++j) a[j] = As[yy * G::AW + lane + j];
        // window of the wave's levels: level k reads bw[boff[k] - bmin + j]
        float bw[K + NC_DW - 1];
        const float* bw0 = Bs + yy * G::BW + lane + bmin;
#pragma unroll
        for (int j = 0; j < K + NC_DW - 1; ++j) bw[j] = bw0[j];
#pragma unroll
        for (int k = 0; k < NC_DW; ++k) {
          const int o = anchor ? k : NC_DW - 1 - k;       // boff[k] - bmin
          float h = a[0] * bw[o];
#pragma unroll
          for (int j = 1; j < K; ++j) h = fmaf(a[j], bw[o + j], h);
          ring[k][s] = h;
        }
        const int y = y0 + yy - 2 * r;        // output row completed by this input row
        if (yy >= 2 * r && y < H &&
            (QUAD == 4 ? true : QUAD >= 2 ? x + pad < out_pitch : x < out_w)) {
          const int64_t rowo = (int64_t)y * SW;
          const float zA = anchor ? zY[rowo + cx] : zX[rowo + cx];
          const float iA = (anchor ? isdY[rowo + cx] : isdX[rowo + cx]) * inv_n;
          float cq[NC_DW];
#pragma unroll
          for (int k = 0; k < NC_DW; ++k) {
            const int d = d0 + wave * NC_DW + k;
            cq[k] = 0.0f;
            if (d >= d_end) continue;
            // rows y-r .. y+r sit in ring slots (s+1) .. (s+K) mod K, in order
            float S = ring[k][(s + 1) % K];
#pragma unroll
            for (int i = 2; i <= K; ++i) S += ring[k][(s + i) % K];
            const int zi = (yy - 2 * r) * G::ZW + lane + boff[k];
            const float zB = Zs[zi];
            const float iB = Is[zi];
            cq[k] = fmaf(-S * iA, iB, fmaf(zA, zB, 1.0f));
            if (!QUAD)
              C[(int64_t)(d - d_first) * out_slice + (int64_t)y * out_pitch + x] = cq[k];
            if (QUAD == 3 && x >= 0 && x < W)      // and the planar copy [level][H][W]
              C2[((int64_t)(d - d_first) * H + y) * W + x] = cq[k];
          }
          if (QUAD == 1) {
            const int q = (d0 + wave * NC_DW - d_first) >> 2;
            if (d0 + wave * NC_DW < d_end)
              reinterpret_cast<float4*>(C)[(int64_t)q * out_slice + (int64_t)y * out_pitch + x] =
                  make_float4(cq[0], cq[1], cq[2], cq[3]);
          }
          if (QUAD >= 2) {
            // this wave's 4 levels of the lane quad's 4 columns, transposed so
            // that lane c of the quad holds level 4 wave + c of all 4 columns;
            // columns outside the image and levels past d_end are zeros
            float v[NC_DW];
#pragma unroll
            for (int k = 0; k < NC_DW; ++k) v[k] = (x >= 0 && x < W) ? cq[k] : 0.0f;
            // the target-anchored copy (QUAD 4): level k from lane + k, all
            // for target column m = x - (first level of the wave)
            const int db = d0 + wave * NC_DW;
            float u[NC_DW];
            if (QUAD == 4 && C2) {
#pragma unroll
              for (int k = 0; k < NC_DW; ++k) u[k] = k ? __shfl_down(cq[k], k, 64) : cq[k];
              const int m = x - db;
#pragma unroll
              for (int k = 0; k < NC_DW; ++k) u[k] = (m >= 0 && m < W) ? u[k] : 0.0f;
            }
            quad_transpose4(v, lane);
            const int dl = db + (lane & 3);
            const bool full = QUAD != 4 || lane < NC_TX4;
            if (dl < ((d_end + 15) & ~15) && full) {
              // stored column quad of row y, level dl
              const int sq = (QUAD == 4 ? NC_TX4 / 4 : 16) * bx + (lane >> 2);
              if (QUAD != 4 || 4 * sq < out_pitch) {
                uint2 hi, lo;
                split4_f16(v, hi, lo);
                const int64_t off = (int64_t)(2 * ((dl - d_first) >> 4)) * out_slice +
                                    (int64_t)y * 16 * out_pitch + 64 * sq + 4 * (dl & 15);
                *reinterpret_cast<uint2*>(reinterpret_cast<_Float16*>(C) + off) = hi;
                *reinterpret_cast<uint2*>(reinterpret_cast<_Float16*>(C) + out_slice + off) = lo;
              }
            }
            if (QUAD == 4 && C2) {
              quad_transpose4(u, lane);
              // target-anchored stored column quad: x0 + pad = 60 bx and the
              // wave's first level are multiples of 4
              const int s1 = NC_TX4 * bx + 4 * (lane >> 2) - db;
              if (dl < ((d_end + 15) & ~15) && full && s1 >= 0 && s1 + 4 <= out_pitch) {
                uint2 hi, lo;
                split4_f16(u, hi, lo);
                const int64_t off = (int64_t)(2 * ((dl - d_first) >> 4)) * out_slice +
                                    (int64_t)y * 16 * out_pitch + 16 * s1 + 4 * (dl & 15);
                *reinterpret_cast<uint2*>(reinterpret_cast<_Float16*>(C2) + off) = hi;
                *reinterpret_cast<uint2*>(reinterpret_cast<_Float16*>(C2) + out_slice + off) = lo;
              }
            }
          }
        }
      }
    }
  }
}

template <int r, typename T, int QUAD, int DC>
__global__ void __launch_bounds__(16 * DC)
ncc_kernel(const T* __restrict__ ref, int64_t ref_pitch,
           const float* __restrict__ tarw, int W, int H, int d_first, int d_end,
           const float* __restrict__ zX, const float* __restrict__ isdX,
           const float* __restrict__ zY, const float* __restrict__ isdY,
           float* __restrict__ C, int out_w, int64_t out_pitch,
           int64_t out_slice, int anchor, int pad, float* __restrict__ C2) {
  extern __shared__ float sm[];
  ncc_body<r, T, QUAD, DC>(ref, ref_pitch, tarw, W, H, d_first, d_end, zX, isdX, zY, isdY, C,
                       out_w, out_pitch, out_slice, anchor, pad, sm, blockIdx.x, blockIdx.y,
                       blockIdx.z, C2);
}


// Job index of a block of a batched launch (binary search of the prefix).
__device__ __forceinline__ int job_of(const int* __restrict__ first, int n, int b) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (first[mid] <= b) lo = mid; else hi = mid;
  }
  return lo;
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

template <int r, typename T, int QUAD, int DC>
__global__ void __launch_bounds__(16 * DC)
ncc_jobs_kernel(const NccJob* __restrict__ jobs, const int* __restrict__ first, int n) {
  extern __shared__ float sm[];
  const int j = job_of(first, n, blockIdx.x);
  const NccJob& J = jobs[j];
  const int l = blockIdx.x - first[j];
  const int gxy = J.gx * J.gy;
  const int bz = l / gxy, rem = l - bz * gxy;
  ncc_body<r, T, QUAD, DC>(static_cast<const T*>(J.ref), J.ref_pitch, J.tarw, J.W, J.H, J.d_first,
                       J.d_end, J.zX, J.isdX, J.zY, J.isdY, J.C, J.out_w, J.out_pitch,
                       J.out_slice, J.anchor, J.pad, sm, rem % J.gx, rem / J.gx, bz, J.C2);
}

// Dynamic LDS above the 64 KB default (large radii at 64 levels), set once
// per kernel instantiation.
template <int r, typename T, int QUAD, int DC, int JOBS>
hipError_t ncc_allow_lds() {
  static bool done = false;
  constexpr size_t bytes = NccGeom<r, DC>::lds_bytes;
  if (!done && bytes > 64 * 1024) {
    const void* k = JOBS ? (const void*)ncc_jobs_kernel<r, T, QUAD, DC>
                         : (const void*)ncc_kernel<r, T, QUAD, DC>;
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
  }
  done = true;
  return hipSuccess;
}

template <int r, typename T, int DC>
hipError_t launch_ncc_rdc(const Plan& P, const T* ref, const float* tar_w, const float* zX,
                          const float* isdX, const float* zY, const float* isdY, float* C,
                          int out_w, int64_t out_pitch, int64_t out_slice, int anchor,
                          int d_first, int d_end, int quad, int pad,
                          hipStream_t s, float* C2) {
  dim3 grid((out_w + NC_TX - 1) / NC_TX, (P.H + NC_TY - 1) / NC_TY,
            (d_end - d_first + DC - 1) / DC);
  if (quad == 4) {
    // both anchors' split volumes (C, and C2 when non-NULL)
    grid.x = (out_w + NC_TX4 - 1) / NC_TX4;
    hipError_t e = ncc_allow_lds<r, T, 4, DC, 0>();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((ncc_kernel<r, T, 4, DC>), grid, dim3(16 * DC),
                       (NccGeom<r, DC>::lds_bytes), s, ref, P.p.pitch_ref, tar_w, P.W, P.H,
                       d_first, d_end, zX, isdX, zY, isdY, C, out_w, out_pitch, out_slice,
                       0, pad, C2);
    return hipGetLastError();
  }
  if (quad == 3) {
    // split-FP16 and planar FP32 outputs in one pass (FP32 images only)
    if constexpr (std::is_same<T, float>::value) {
      hipError_t e = ncc_allow_lds<r, T, 3, DC, 0>();
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((ncc_kernel<r, T, 3, DC>), grid, dim3(16 * DC),
                         (NccGeom<r, DC>::lds_bytes), s, ref, P.p.pitch_ref, tar_w, P.W, P.H,
                         d_first, d_end, zX, isdX, zY, isdY, C, out_w, out_pitch, out_slice,
                         anchor, pad, C2);
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }
  hipError_t e = quad == 2 ? ncc_allow_lds<r, T, 2, DC, 0>()
                 : quad ? ncc_allow_lds<r, T, 1, DC, 0>() : ncc_allow_lds<r, T, 0, DC, 0>();
  if (e != hipSuccess) return e;
  if (quad == 2)
    hipLaunchKernelGGL((ncc_kernel<r, T, 2, DC>), grid, dim3(16 * DC),
                       (NccGeom<r, DC>::lds_bytes), s, ref, P.p.pitch_ref, tar_w, P.W, P.H,
                       d_first, d_end, zX, isdX, zY, isdY, C, out_w, out_pitch, out_slice,
                       anchor, pad, (float*)nullptr);
  else if (quad)
    hipLaunchKernelGGL((ncc_kernel<r, T, 1, DC>), grid, dim3(16 * DC),
                       (NccGeom<r, DC>::lds_bytes), s, ref, P.p.pitch_ref, tar_w, P.W, P.H,
                       d_first, d_end, zX, isdX, zY, isdY, C, out_w, out_pitch, out_slice,
                       anchor, 0, (float*)nullptr);
  else
    hipLaunchKernelGGL((ncc_kernel<r, T, 0, DC>), grid, dim3(16 * DC),
                       (NccGeom<r, DC>::lds_bytes), s, ref, P.p.pitch_ref, tar_w, P.W, P.H,
                       d_first, d_end, zX, isdX, zY, isdY, C, out_w, out_pitch, out_slice,
                       anchor, 0, (float*)nullptr);
  return hipGetLastError();
}

template <int r, typename T>
hipError_t launch_ncc_r(const Plan& P, const T* ref, const float* tar_w, const float* zX,
                        const float* isdX, const float* zY, const float* isdY, float* C,
                        int out_w, int64_t out_pitch, int64_t out_slice, int anchor,
                        int d_first, int d_end, int quad, int pad,
                        hipStream_t s, float* C2) {
  int dc = P.ncc_levels;
  if (dc == 0) {
    // automatic: the smallest block that holds every level, at most 64 (a
    // larger block spreads the staging of the unshifted operand over more
    // levels, which pays even when its last levels are idle)
    const int nl = d_end - d_first;
    dc = nl > 32 ? 64 : nl > 16 ? 32 : 16;
    // the both-anchors form needs more registers (70 at r = 3): a 64-level
    // workgroup (16 waves) then fits once per CU, two 32-level ones twice
    // (1280x720, D = 64: 0.167 against 0.181 ms)
    if (quad == 4 && dc == 64) dc = 32;
  }
  switch (dc) {
    case 32:
      return launch_ncc_rdc<r, T, 32>(P, ref, tar_w, zX, isdX, zY, isdY, C, out_w, out_pitch,
                                      out_slice, anchor, d_first, d_end, quad, pad, s, C2);
    case 64:
      return launch_ncc_rdc<r, T, 64>(P, ref, tar_w, zX, isdX, zY, isdY, C, out_w, out_pitch,
                                      out_slice, anchor, d_first, d_end, quad, pad, s, C2);
    default:
      return launch_ncc_rdc<r, T, 16>(P, ref, tar_w, zX, isdX, zY, isdY, C, out_w, out_pitch,
                                      out_slice, anchor, d_first, d_end, quad, pad, s, C2);
  }
}

template <typename T>
hipError_t launch_ncc_t(const Plan& P, const T* ref, const float* tar_w, const float* zX,
                        const float* isdX, const float* zY, const float* isdY, float* C,
                        int out_w, int64_t out_pitch, int64_t out_slice, int anchor,
                        int d_first, int d_end, int quad, int pad,
                        hipStream_t s, float* C2) {
#define NCC_CASE(R_) \
  case R_: return launch_ncc_r<R_, T>(P, ref, tar_w, zX, isdX, zY, isdY, C, out_w, \
                                      out_pitch, out_slice, anchor, d_first, d_end, quad, pad, \
                                      s, C2);
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
               int quad, float* C2) {
  NccJob J{};
  J.C2 = C2;
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

namespace {
template <int r, typename T, int DC>
hipError_t ncc_jobs_rdc(int quad, const NccJob* jobs, const int* first, int n, int blocks,
                        hipStream_t s) {
  hipError_t e = quad == 4 ? ncc_allow_lds<r, T, 4, DC, 1>()
                 : quad == 2 ? ncc_allow_lds<r, T, 2, DC, 1>()
                 : quad ? ncc_allow_lds<r, T, 1, DC, 1>() : ncc_allow_lds<r, T, 0, DC, 1>();
  if (e != hipSuccess) return e;
  if (quad == 4)
    hipLaunchKernelGGL((ncc_jobs_kernel<r, T, 4, DC>), dim3(blocks), dim3(16 * DC),
                       (NccGeom<r, DC>::lds_bytes), s, jobs, first, n);
  else if (quad == 2)
    hipLaunchKernelGGL((ncc_jobs_kernel<r, T, 2, DC>), dim3(blocks), dim3(16 * DC),
                       (NccGeom<r, DC>::lds_bytes), s, jobs, first, n);
  else if (quad)
    hipLaunchKernelGGL((ncc_jobs_kernel<r, T, 1, DC>), dim3(blocks), dim3(16 * DC),
                       (NccGeom<r, DC>::lds_bytes), s, jobs, first, n);
  else
    hipLaunchKernelGGL((ncc_jobs_kernel<r, T, 0, DC>), dim3(blocks), dim3(16 * DC),
                       (NccGeom<r, DC>::lds_bytes), s, jobs, first, n);
  return hipGetLastError();
}
template <int r, typename T>
hipError_t ncc_jobs_r(int quad, int dc, const NccJob* jobs, const int* first, int n, int blocks,
                      hipStream_t s) {
  switch (dc) {
    case 64: return ncc_jobs_rdc<r, T, 64>(quad, jobs, first, n, blocks, s);
    case 32: return ncc_jobs_rdc<r, T, 32>(quad, jobs, first, n, blocks, s);
    default: return ncc_jobs_rdc<r, T, 16>(quad, jobs, first, n, blocks, s);
  }
}
template <typename T>
hipError_t ncc_jobs_t(int r, int quad, int dc, const NccJob* jobs, const int* first, int n,
                      int blocks, hipStream_t s) {
  switch (r) {
    case 1: return ncc_jobs_r<1, T>(quad, dc, jobs, first, n, blocks, s);
    case 2: return ncc_jobs_r<2, T>(quad, dc, jobs, first, n, blocks, s);
    case 3: return ncc_jobs_r<3, T>(quad, dc, jobs, first, n, blocks, s);
    case 4: return ncc_jobs_r<4, T>(quad, dc, jobs, first, n, blocks, s);
    case 5: return ncc_jobs_r<5, T>(quad, dc, jobs, first, n, blocks, s);
    case 6: return ncc_jobs_r<6, T>(quad, dc, jobs, first, n, blocks, s);
    case 7: return ncc_jobs_r<7, T>(quad, dc, jobs, first, n, blocks, s);
    case 8: return ncc_jobs_r<8, T>(quad, dc, jobs, first, n, blocks, s);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace

hipError_t launch_ncc_jobs(int r, stereo_dtype dt, int quad, int dc, const NccJob* jobs,
                           const int* first, int n, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  if (dt == STEREO_U8) return ncc_jobs_t<uint8_t>(r, quad, dc, jobs, first, n, blocks, s);
  return ncc_jobs_t<float>(r, quad, dc, jobs, first, n, blocks, s);
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
  if (P.p.dtype == STEREO_U8)
    return launch_ncc_t(P, (const uint8_t*)ref, tar_w, zX, isdX, zY, isdY, C, out_w,
                        out_pitch, out_slice, anchor, d_first, d_end, quad, pad, s, C2);
  return launch_ncc_t(P, (const float*)ref, tar_w, zX, isdX, zY, isdY, C, out_w, out_pitch,
                      out_slice, anchor, d_first, d_end, quad, pad, s, C2);
}

}  // namespace stereo
