// NCC matching cost of Eq. (8) over a level block: the kernel body, its
// single-image and batched launches and their host launchers, shared by the
// per-radius instantiation units (k_ncc_r1 .. r8) and the dispatch in
// k_cost.hip (which instantiates none of them).
#pragma once
#include <type_traits>

#include "internal.h"

namespace stereo {
namespace {

template <typename T>
__device__ __forceinline__ float ld(const T* p) { return static_cast<float>(*p); }

// Staging loads of the NCC body through the global address space: its
// pointers may come from a job descriptor in memory, which the compiler
// would reach with flat instructions (flat operations also count against
// the LDS wait counter).  The batched kernel forms its output pointers from
// a kernel argument, which the compiler knows to be global.
#define NCC_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ float gld(const T* p) {
  return static_cast<float>(*(const NCC_GLOBAL T*)p);
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
// level-shifted operand B, the B side's statistics of the workgroup's output
// rows (z and 1/sd at the shifted block centres: one contiguous column range
// per row) and the A side's at the lanes' own columns are staged in LDS with
// clamped reads.  A wave's NC_DW levels read overlapping windows of the same
// B row: one window of K + NC_DW - 1 values serves them all.  8-row tiles
// redo 2r of every 8 + 2r input rows but need a quarter of the LDS of
// 32-row ones, so more workgroups stay resident to overlap the stores
// (1280x720, 64 levels, r = 3, both split volumes: 0.111 ms against 0.113 /
// 0.114 / 0.131 ms with 12- / 16- / 32-row tiles).
constexpr int NC_TX = 64, NC_TY = 8, NC_DC = 16, NC_DW = 4;
// NC_DC is the default level block; a workgroup of DC levels has DC / 4 waves.

template <int r, int DC = NC_DC>
struct NccGeom {
  static constexpr int K = 2 * r + 1;
  static constexpr int ROWS = NC_TY + 2 * r;
  static constexpr int AW = NC_TX + 2 * r;
  static constexpr int BW = NC_TX + 2 * r + DC - 1;
  static constexpr int ZW = NC_TX + DC - 1;         // B-side statistics per output row
  // A, B, the B side's and the A side's statistics of the output rows
  static constexpr size_t lds_bytes =
      sizeof(float) * ((size_t)ROWS * (AW + BW) + 2 * (size_t)NC_TY * (ZW + NC_TX));
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
// that swap the off-diagonal 2x2 blocks.  Each element of a stage is one
// v_cndmask_b32 whose first source is read through a DPP quad permutation:
// lanes whose bit (0, then 1) equals that of k keep v[k], the others take
// the partner lane's v[k ^ 1] (v[k ^ 2]).  The condition is a constant lane
// pattern in VCC.  The compiler cannot see the DPP reads inside the asm, so
// each stage opens with s_nop 4: the five wait states a DPP read needs after
// a VALU write of EXEC, which also covers the two it needs after a VALU
// write of its source.  Every lane of a quad must be active.
__device__ __forceinline__ void quad_transpose4(float (&v)[4]) {
  float t[4];
  // lanes c and c ^ 1: (0, 1) and (2, 3); outputs 0, 2 keep where bit 0 is clear
  asm volatile("s_nop 4\n\t"
               "s_mov_b32 vcc_lo, 0x55555555\n\t"
               "s_mov_b32 vcc_hi, 0x55555555\n\t"
               "v_cndmask_b32_dpp %0, %5, %4, vcc quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf\n\t"
               "v_cndmask_b32_dpp %2, %7, %6, vcc quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf\n\t"
               "s_mov_b32 vcc_lo, 0xaaaaaaaa\n\t"
               "s_mov_b32 vcc_hi, 0xaaaaaaaa\n\t"
               "v_cndmask_b32_dpp %1, %4, %5, vcc quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf\n\t"
               "v_cndmask_b32_dpp %3, %6, %7, vcc quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf"
               : "=&v"(t[0]), "=&v"(t[1]), "=&v"(t[2]), "=&v"(t[3])
               : "v"(v[0]), "v"(v[1]), "v"(v[2]), "v"(v[3])
               : "vcc");
  // lanes c and c ^ 2: (0, 2) and (1, 3); outputs 0, 1 keep where bit 1 is clear
  asm volatile("s_nop 4\n\t"
               "s_mov_b32 vcc_lo, 0x33333333\n\t"
               "s_mov_b32 vcc_hi, 0x33333333\n\t"
               "v_cndmask_b32_dpp %0, %6, %4, vcc quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf\n\t"
               "v_cndmask_b32_dpp %1, %7, %5, vcc quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf\n\t"
               "s_mov_b32 vcc_lo, 0xcccccccc\n\t"
               "s_mov_b32 vcc_hi, 0xcccccccc\n\t"
               "v_cndmask_b32_dpp %2, %4, %6, vcc quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf\n\t"
               "v_cndmask_b32_dpp %3, %5, %7, vcc quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf"
               : "=&v"(v[0]), "=&v"(v[1]), "=&v"(v[2]), "=&v"(v[3])
               : "v"(t[0]), "v"(t[1]), "v"(t[2]), "v"(t[3])
               : "vcc");
}

// v = hi + lo in FP16 (round to nearest; lo rounds the remainder v - hi,
// which is exact in FP32 and formed by one mixed-precision FMA reading hi
// from its half of the packed register), four values packed two per register.
__device__ __forceinline__ void split4_f16(const float (&v)[4], uint2& hi, uint2& lo) {
  unsigned h[2], l[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    float r0, r1;
    asm volatile("v_cvt_pk_f16_f32 %0, %1, %2" : "=v"(h[j]) : "v"(v[2 * j]), "v"(v[2 * j + 1]));
    asm volatile("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0]"
                 : "=v"(r0) : "v"(h[j]), "v"(v[2 * j]));
    asm volatile("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]"
                 : "=v"(r1) : "v"(h[j]), "v"(v[2 * j + 1]));
    asm volatile("v_cvt_pk_f16_f32 %0, %1, %2" : "=v"(l[j]) : "v"(r0), "v"(r1));
  }
  hi = make_uint2(h[0], h[1]);
  lo = make_uint2(l[0], l[1]);
}

// Copy N elements (two floats each) into LDS with NT threads: element i =
// tid + k NT is read by get(i) and written by put(i, v); NC_SCH reads of a
// thread are issued before their writes.
constexpr int NC_SCH = 6;
template <int N, int NT, class Get, class Put>
__device__ __forceinline__ void ncc_stage(int tid, Get get, Put put) {
  constexpr int KK = (N + NT - 1) / NT;
#pragma unroll
  for (int k0 = 0; k0 < KK; k0 += NC_SCH) {
    float2 v[NC_SCH];
#pragma unroll
    for (int k = 0; k < NC_SCH; ++k)
      if (k0 + k < KK) v[k] = get(min(tid + (k0 + k) * NT, N - 1));
#pragma unroll
    for (int k = 0; k < NC_SCH; ++k)
      if (k0 + k < KK && tid + (k0 + k) * NT < N) put(tid + (k0 + k) * NT, v[k]);
  }
}

// The anchor is a template parameter: it fixes which register of the B
// window each level's products read, so the window stays in plain registers
// (a run-time choice turns every read into an indexed register move).
template <int r, typename T, int QUAD, int DC, int anchor>
__device__ __forceinline__ void ncc_body_a(const T* __restrict__ ref, int64_t ref_pitch,
                                           const float* __restrict__ tarw, int W, int H,
                                           int d_first, int d_end,
                                           const float* __restrict__ zX,
                                           const float* __restrict__ isdX,
                                           const float* __restrict__ zY,
                                           const float* __restrict__ isdY,
                                           float* __restrict__ C, int out_w, int64_t out_pitch,
                                           int64_t out_slice, int pad, float* sm, int bx,
                                           int by, int bz, float* __restrict__ C2) {
  using G = NccGeom<r, DC>;
  constexpr int K = G::K;
  float* As = sm;                         // [ROWS][AW]
  float* Bs = sm + G::ROWS * G::AW;       // [ROWS][BW]
  float* Zs = Bs + G::ROWS * G::BW;       // [NC_TY][ZW]: z of the B side
  float* Is = Zs + NC_TY * G::ZW;         // [NC_TY][ZW]: 1/sd of the B side
  float* ZA = Is + NC_TY * G::ZW;         // [NC_TY][NC_TX]: z of the A side at the lanes
  float* IA = ZA + NC_TY * NC_TX;         // [NC_TY][NC_TX]: 1/sd of the A side / K^2
  const float inv_n = 1.0f / (float)(K * K);
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
  // Staging in chunks: NC_SCH loads of each thread are in flight before
  // their LDS stores (one wait per chunk instead of one per element).
  constexpr int NT = 16 * DC;                        // threads per workgroup
  const int tid = threadIdx.x;
  const int zxo = anchor ? x0 + d0 : x0 - d0 - (DC - 1);
  const float* zm = anchor ? zX : zY;
  const float* im = anchor ? isdX : isdY;
  const float* za = anchor ? zY : zX;
  const float* ia = anchor ? isdY : isdX;
  // A and B rows (clamped reads, offset-centred values)
  ncc_stage<G::ROWS * G::BW, NT>(tid, [&](int i) {
    const int yy = i / G::BW, xx = i - yy * G::BW;
    const int gy = min(max(y0 - r + yy, 0), H - 1);
    const int gxb = min(max(bxo + xx, 0), W - 1);
    const int gxa = min(max(axo + min(xx, G::AW - 1), 0), W - 1);
    return anchor ? make_float2(gld(ref + (int64_t)gy * ref_pitch + gxb), gld(tarw + (int64_t)gy * W + gxa))
                  : make_float2(gld(tarw + (int64_t)gy * W + gxb), gld(ref + (int64_t)gy * ref_pitch + gxa));
  }, [&](int i, float2 v) {
    const int yy = i / G::BW, xx = i - yy * G::BW;
    Bs[i] = v.x - kOffset;
    if (xx < G::AW) As[yy * G::AW + xx] = v.y - kOffset;
  });
  // B-side statistics: entry c of output row t is the block centred at image
  // column zxo + c (clamped to the map's [-r, W - 1 + r]), the centre that
  // level offset boff reads for lane c - boff
  ncc_stage<NC_TY * G::ZW, NT>(tid, [&](int i) {
    const int t = i / G::ZW, c = i - t * G::ZW;
    const int64_t rowo = (int64_t)min(y0 + t, H - 1) * SW;
    const int cb = min(max(zxo + c, -r), W - 1 + r) + r;
    return make_float2(gld(zm + rowo + cb), gld(im + rowo + cb));
  }, [&](int i, float2 v) { Zs[i] = v.x; Is[i] = v.y; });
  // A-side statistics of each lane's own column (in LDS, so that the row
  // loop issues no global loads: their wait would also wait for the previous
  // rows' stores)
  ncc_stage<NC_TY * NC_TX, NT>(tid, [&](int i) {
    const int t = i / NC_TX, c = i - t * NC_TX;
    const int64_t rowo = (int64_t)min(y0 + t, H - 1) * SW;
    const int cb = min(max(x0 + c, -r), W - 1 + r) + r;
    return make_float2(gld(za + rowo + cb), gld(ia + rowo + cb));
  }, [&](int i, float2 v) { ZA[i] = v.x; IA[i] = v.y * inv_n; });
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int x = x0 + lane;
  int boff[NC_DW];
#pragma unroll
  for (int k = 0; k < NC_DW; ++k) {
    const int dc = wave * NC_DW + k;
    boff[k] = anchor ? dc : (DC - 1 - dc);
  }
  const int bmin = anchor ? boff[0] : boff[NC_DW - 1];
  float ring[NC_DW][K];
#pragma unroll
  for (int k = 0; k < NC_DW; ++k)
#pragma unroll
    for (int i = 0; i < K; ++i) ring[k][i] = 0.0f;

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
          const float zA = ZA[(yy - 2 * r) * NC_TX + lane];
          const float iA = IA[(yy - 2 * r) * NC_TX + lane];
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
            quad_transpose4(v);
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
              quad_transpose4(u);
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
  // the both-anchors form always runs from the reference anchor
  if (QUAD != 4 && anchor)
    ncc_body_a<r, T, QUAD, DC, 1>(ref, ref_pitch, tarw, W, H, d_first, d_end, zX, isdX, zY,
                                  isdY, C, out_w, out_pitch, out_slice, pad, sm, bx, by, bz, C2);
  else
    ncc_body_a<r, T, QUAD, DC, 0>(ref, ref_pitch, tarw, W, H, d_first, d_end, zX, isdX, zY,
                                  isdY, C, out_w, out_pitch, out_slice, pad, sm, bx, by, bz, C2);
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


// Job index of a block of a batched launch: the jobs whose first block is at
// or before b, counted 64 at a time by one load per lane and a ballot (every
// lane of the wave calls it; first[] is the ascending block prefix).
__device__ __forceinline__ int job_of(const int* __restrict__ first, int n, int b) {
  int cnt = 0;
  for (int c = 0; c < n; c += 64) {
    const int k = c + (int)(threadIdx.x & 63);
    const bool le = k < n && first[min(k, n - 1)] <= b;
    const int add = __popcll(__ballot(le));
    cnt += add;
    if (add < 64) break;
  }
  return cnt - 1;
}

template <int r, typename T, int QUAD, int DC>
__global__ void __launch_bounds__(16 * DC)
ncc_jobs_kernel(const NccJob* __restrict__ jobs, const int* __restrict__ first, int n,
                char* __restrict__ base) {
  extern __shared__ float sm[];
  const int j = job_of(first, n, blockIdx.x);
  const NccJob& J = jobs[j];
  const int l = blockIdx.x - first[j];
  const int gxy = J.gx * J.gy;
  const int bz = l / gxy, rem = l - bz * gxy;
  float* C = reinterpret_cast<float*>(base + J.c_off);
  float* C2 = J.c2_off >= 0 ? reinterpret_cast<float*>(base + J.c2_off) : nullptr;
  ncc_body<r, T, QUAD, DC>(static_cast<const T*>(J.ref), J.ref_pitch, J.tarw, J.W, J.H, J.d_first,
                       J.d_end, J.zX, J.isdX, J.zY, J.isdY, C, J.out_w, J.out_pitch,
                       J.out_slice, J.anchor, J.pad, sm, rem % J.gx, rem / J.gx, bz, C2);
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
    // the split-FP16 forms: 16-level workgroups (1280x720, D = 64, both
    // anchors: 0.114 against 0.121 / 0.125 ms at 32 / 64 levels)
    if (quad >= 2) dc = 16;
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


template <int r, typename T, int DC>
hipError_t ncc_jobs_rdc(int quad, const NccJob* jobs, const int* first, int n, int blocks,
                        char* base, hipStream_t s) {
  hipError_t e = quad == 4 ? ncc_allow_lds<r, T, 4, DC, 1>()
                 : quad == 2 ? ncc_allow_lds<r, T, 2, DC, 1>()
                 : quad ? ncc_allow_lds<r, T, 1, DC, 1>() : ncc_allow_lds<r, T, 0, DC, 1>();
  if (e != hipSuccess) return e;
  if (quad == 4)
    hipLaunchKernelGGL((ncc_jobs_kernel<r, T, 4, DC>), dim3(blocks), dim3(16 * DC),
                       (NccGeom<r, DC>::lds_bytes), s, jobs, first, n, base);
  else if (quad == 2)
    hipLaunchKernelGGL((ncc_jobs_kernel<r, T, 2, DC>), dim3(blocks), dim3(16 * DC),
                       (NccGeom<r, DC>::lds_bytes), s, jobs, first, n, base);
  else if (quad)
    hipLaunchKernelGGL((ncc_jobs_kernel<r, T, 1, DC>), dim3(blocks), dim3(16 * DC),
                       (NccGeom<r, DC>::lds_bytes), s, jobs, first, n, base);
  else
    hipLaunchKernelGGL((ncc_jobs_kernel<r, T, 0, DC>), dim3(blocks), dim3(16 * DC),
                       (NccGeom<r, DC>::lds_bytes), s, jobs, first, n, base);
  return hipGetLastError();
}
template <int r, typename T>
hipError_t ncc_jobs_r(int quad, int dc, const NccJob* jobs, const int* first, int n, int blocks,
                      char* base, hipStream_t s) {
  switch (dc) {
    case 64: return ncc_jobs_rdc<r, T, 64>(quad, jobs, first, n, blocks, base, s);
    case 32: return ncc_jobs_rdc<r, T, 32>(quad, jobs, first, n, blocks, base, s);
    default: return ncc_jobs_rdc<r, T, 16>(quad, jobs, first, n, blocks, base, s);
  }
}

}  // namespace
}  // namespace stereo
