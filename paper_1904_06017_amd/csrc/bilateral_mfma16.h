// Bilateral cost aggregation, Eqs. (10)-(11), fused with winner-take-all
// selection and sub-pixel refinement (Sec. 3.2.2, Eq. 13) or the soft-argmin
// head, on the matrix cores with FP16 operands split in two.
//
// As in the FP32 matrix-core kernel, the aggregated costs of a 4x4 block of
// pixels p and 16 levels d are the product E[p][d] = sum_q w(p, q) C(q, d)
// over the block's window union, with zero weights outside a pixel's own
// window.  Here every operand is carried as two FP16 numbers, x = x_hi + x_lo
// (x_hi the FP16 rounding of x, x_lo that of the remainder), and the product
// takes the three terms w_hi C_hi + w_hi C_lo + w_lo C_hi on
// v_mfma_f32_16x16x32_f16 with FP32 accumulation.  Each operand keeps about
// 22 significant bits and the dropped w_lo C_lo term is below 2^-22 of the
// product, so the sums are as accurate as FP32 products; the three FP16
// products take about a third of the matrix-core time of the FP32 ones.
// Weights are scaled by 2^12 before the split (the selection and the
// normalised soft-argmin are scale-free), which keeps the low parts of small
// weights out of the FP16 subnormal range.
//
// Operand layout.  The K index of one product runs over 32 union positions:
// lane (m, g) (m = lane & 15, g = lane >> 4) holds 8 of them, a 2-row x
// 4-column patch of the union, for pixel m (A, weights) or level m (B,
// costs).  Patch 4 i + g of product i; the union ((4 + 2R) rows, 4 + 2R
// columns rounded up to whole column quads) has (R + 2) x ceil((4+2R)/4)
// patches, padded to a multiple of 4 with zero-weight patches.
//
// Costs.  The NCC writes two split-FP16 volumes, reference-anchored and
// target-anchored, so both volumes stage the same way.  Each is stored in
// blocks of 16 levels, [block][part][row][column quad][16 levels][4 columns]
// (columns shifted by R so that a tile's halo starts at a column quad): one
// operand read (16 levels x 4 columns of a row) is 128 contiguous bytes, and
// one halo row of a block part is HXP / 4 x 128 contiguous bytes.  A
// workgroup (12 waves) owns a 16 x 12 pixel tile; each pass of 16 levels
// copies the halo slab (2 parts x (12 + 2R) rows x HXP columns x 16 levels)
// global -> LDS with direct-to-LDS loads into one of two buffers while the
// other is being multiplied, one barrier per pass.  Rows outside the image
// read clamped (finite) data, and the levels of the last block past D are
// zeros; their weights are zero or their outputs unused.
//
// Per pixel the result depends on the pixel's block and the levels only, so
// per-pair and queued launches are bitwise equal.  The summation order
// differs from the other engines': the three agree to rounding.
#pragma once
#include "bilateral_mfma.h"

namespace stereo {
namespace bilh {

using bil::BilPair;
typedef float f4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

constexpr int kBR = 3;                  // block rows per tile
constexpr int kWaves = 4 * kBR;         // one 4x4 block per wave
constexpr int kThreads = 64 * kWaves;
constexpr int kTW = 16, kTH = 4 * kBR;  // tile in pixels
static_assert(kTW == kMfmaTileW && kTH == kMfmaTileH, "tile size shared with the batch tables");
constexpr float kFar = 1e30f;           // guide outside the image: zero weight
constexpr float kLog2WScale = 12.0f;    // weights scaled by 2^12 before the split

// Row pitch (halves) of the split-FP16 volumes for image width W at radius R.
template <int R>
struct HGeom {
  static constexpr int UH = 4 + 2 * R;                  // union rows of a 4x4 block
  static constexpr int UW = (4 + 2 * R + 3) & ~3;       // union columns, whole quads
  static constexpr int NRP = UH / 2;                    // row pairs
  static constexpr int NCQ = UW / 4;                    // column quads
  static constexpr int NP = NRP * NCQ;                  // 2x4 patches
  static constexpr int NI = (NP + 3) / 4;               // products (x3) per pass
  static constexpr int HY = kTH + 2 * R;                // halo rows
  static constexpr int HXP = (4 * (kTW / 4 - 1) + UW + 7) & ~7;   // halo columns
  static constexpr int NQH = HXP / 4;                   // column quads per halo row
  static constexpr int ROWB = NQH * 128;                // bytes per halo row of a part
  static constexpr int PARTB = HY * ROWB;               // bytes per part of a slab
  static constexpr int CPR = NQH * 8;                   // 16-byte chunks per row
  static constexpr int NCH = 2 * HY * CPR;              // chunks per slab
  static constexpr int NWC = (NCH + 63) / 64;           // wave copies per slab
  static constexpr int KPW = (NWC + kWaves - 1) / kWaves;
  static constexpr int BUF = 2 * PARTB / 4;             // dwords per slab
  // guide row stride (floats) = 4 NQH: a patch's guide offset (floats) is
  // 4 x its offset in 128-byte units
  static constexpr int GS = HXP;
  static constexpr int GUIDE = HY * GS;
  static constexpr int GPT = (GUIDE + kThreads - 1) / kThreads;
  static constexpr int SCR = kWaves * 16 * 20;          // per-wave [pixel][20] scratch
  static constexpr int STAB = NI * 64 * 8;              // spatial terms [i][lane][slot]
  static constexpr size_t base_bytes = sizeof(float) * (2 * (size_t)BUF + 2 * GUIDE + SCR);
  // the spatial terms are tabulated in LDS where it has room
  static constexpr bool kTable = base_bytes + sizeof(float) * STAB <= 160 * 1024;
  static constexpr size_t lds_bytes = base_bytes + (kTable ? sizeof(float) * STAB : 0);
  static_assert(kTW + 2 * R <= GS && 4 * (kTW / 4 - 1) + UW <= GS, "guide rows");
  static_assert(HY * NQH < 256, "patch offsets are packed in 8 bits");
  static_assert(lds_bytes <= 160 * 1024, "LDS budget");
  static_assert(PARTB < 65536, "lo-part offset must fit a DS immediate");
};

template <int R>
inline int h2_pitch_for(int W) {
  return ((W + kTW - 1) / kTW) * kTW - kTW + HGeom<R>::HXP;
}

// The fields one tile needs; uniform across the workgroup.
struct View {
  const uint16_t* V;              // split-FP16 volume
  int64_t plane;                  // halves per block part: 16 H pitch
  int pitch;                      // columns per row (a multiple of 8)
  const void* guide;
  int64_t g_pitch;
  int W, H, D;
  float ks2, kr2;
  int16_t* dint;                  // selection (mode 1)
  float* dsub;
  float* sm_m;                    // soft-argmin (mode 2)
  float* sm_logZ;
  float* sm_dh;
  float* disp;
  float invT;
  double delta_p, c0, c1, c2;
};

__host__ __device__ inline View view_of(const BilPair& a) {
  View v;
  v.V = a.h2;
  v.plane = a.h2_plane;
  v.pitch = a.h2_pitch;
  v.guide = a.guide;
  v.g_pitch = a.g_pitch;
  v.W = a.W; v.H = a.H; v.D = a.D;
  v.ks2 = a.ks2;
  v.kr2 = a.kr2;
  v.dint = a.o.dint;
  v.dsub = a.o.dsub;
  v.sm_m = a.o.sm_m;
  v.sm_logZ = a.o.sm_logZ;
  v.sm_dh = a.o.sm_dh;
  v.disp = a.o.disp;
  v.invT = a.o.invT;
  v.delta_p = a.o.delta_p;
  v.c0 = a.o.c0; v.c1 = a.o.c1; v.c2 = a.o.c2;
  return v;
}

// Slab of levels [d0, d0 + 16) (one stored block) of the tile at (x0, y0)
// into buf: [part][row][column quad][16 levels][4 columns] halves.  Chunk c
// (16 bytes) is part c / (HY CPR), row (c / CPR) % HY, bytes 16 (c % CPR) of
// the row, the same bytes as in the stored block row.  Rows clamp to the
// image.
template <int R>
__device__ __forceinline__ void stage(const View& v, int x0, int y0, int d0, float* buf,
                                      int wave, int lane, const int (&coff)[HGeom<R>::KPW],
                                      bool fast) {
  using G = HGeom<R>;
  const int64_t rows = 16 * (int64_t)v.pitch;          // halves per stored row
  if (fast && y0 >= R && y0 + kTH + R <= v.H) {
    const uint16_t* base = v.V + (int64_t)(2 * (d0 >> 4)) * v.plane + (int64_t)(y0 - R) * rows +
                           16 * x0;
    if constexpr (G::CPR == 64) {
      // one wave copy = one halo row of one part: (part, row) = (k / HY, k % HY)
#pragma unroll
      for (int m = 0; m < G::KPW; ++m) {
        const int k = wave + kWaves * m;
        if (k < G::NWC) {
          const int pr = k / G::HY, row = k - pr * G::HY;
          __builtin_amdgcn_global_load_lds(
              (BILM_GLOBAL void*)(base + pr * v.plane + row * rows + 8 * lane),
              (BILM_LOCAL void*)(buf + k * 256), 16, 0, 0);
        }
      }
    } else {
      // interior rows: the lane's chunk offsets relative to the slab origin
      // were formed once per kernel
#pragma unroll
      for (int m = 0; m < G::KPW; ++m) {
        const int k = wave + kWaves * m;
        if (k < G::NWC && coff[m] >= 0)
          __builtin_amdgcn_global_load_lds((BILM_GLOBAL void*)(base + coff[m]),
                                           (BILM_LOCAL void*)(buf + k * 256), 16, 0, 0);
      }
    }
    return;
  }
  // border tiles: rows clamped; recomputed per call so that nothing of it
  // stays live
  int ln = lane;
  asm volatile("" : "+v"(ln));
#pragma unroll
  for (int m = 0; m < G::KPW; ++m) {
    const int k = wave + kWaves * m;
    if (k < G::NWC) {
      const int c = k * 64 + ln;
      if (c < G::NCH) {
        const int pr = c / (G::HY * G::CPR);
        const int w = c - pr * (G::HY * G::CPR);
        const int row = w / G::CPR;
        const int cr = w - row * G::CPR;
        int gy = y0 - R + row;
        gy = gy < 0 ? 0 : (gy >= v.H ? v.H - 1 : gy);
        const int64_t off = (int64_t)(2 * (d0 >> 4) + pr) * v.plane + (int64_t)gy * rows +
                            16 * x0 + 8 * cr;
        __builtin_amdgcn_global_load_lds((BILM_GLOBAL void*)(v.V + off),
                                         (BILM_LOCAL void*)(buf + k * 256), 16, 0, 0);
      }
    }
  }
}

// Guide of a tile's halo: the raw values are loaded into registers
// (unconditionally, clamped addresses) and turned into the scaled guide
// (sqrt(kr2) g, kFar outside the image) only when stored to LDS.  A value
// used right after its load waits at once, and that wait also covers the
// slab copies in flight; this way the loads of the next tile's guide overlap
// the last pass's products.
template <int R, typename GT>
struct GuideRaw {
  GT raw[HGeom<R>::GPT];
};

template <int R, typename GT>
__device__ __forceinline__ void guide_load(const View& v, int x0, int y0, GuideRaw<R, GT>& g) {
  using G = HGeom<R>;
  const GT* __restrict__ src = static_cast<const GT*>(v.guide);
#pragma unroll
  for (int k = 0; k < G::GPT; ++k) {
    const int i = threadIdx.x + k * kThreads;
    const int yy = i / G::GS, xx = i % G::GS;
    const int cy = min(max(y0 - R + yy, 0), v.H - 1), cx = min(max(x0 - R + xx, 0), v.W - 1);
    g.raw[k] = src[(int64_t)cy * v.g_pitch + cx];
  }
}

__device__ __forceinline__ float guide_value(uint8_t raw, unsigned z) {
  return (float)((unsigned)raw ^ z);
}
__device__ __forceinline__ float guide_value(float raw, unsigned z) {
  return __builtin_bit_cast(float, __builtin_bit_cast(unsigned, raw) ^ z);
}

// (v, x0, y0): the tile the guide was loaded for
template <int R, typename GT>
__device__ __forceinline__ void guide_store(float* gs, const GuideRaw<R, GT>& g, const View& v,
                                            int x0, int y0) {
  using G = HGeom<R>;
  // an opaque zero: the conversion cannot move up into the load's branch
  unsigned z = 0u;
  asm volatile("" : "+s"(z));
  const float kr = sqrtf(v.kr2);
#pragma unroll
  for (int k = 0; k < G::GPT; ++k) {
    const int i = threadIdx.x + k * kThreads;
    const int yy = i / G::GS, xx = i % G::GS;
    const int gy = y0 - R + yy, gx = x0 - R + xx;
    const bool in = xx < kTW + 2 * R && gy >= 0 && gy < v.H && gx >= 0 && gx < v.W;
    if (i < G::GUIDE) gs[i] = in ? guide_value(g.raw[k], z) * kr : kFar;
  }
}

// x = hi + lo in FP16 (round to nearest); lo is the rounding of the
// remainder x - hi, which is exact in FP32 and formed by one mixed-precision
// FMA per value (the FP16 hi read from its half of the packed register).
// Written out so that each pair is packed where it is formed: left to the
// compiler, the FP32 remainders of a whole tile's weights stay live until
// the end of the weight loop and spill.
__device__ __forceinline__ void split8(const float (&w)[8], u4& hi, u4& lo) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    unsigned hb, lb;
    float r0, r1;
    asm volatile("v_cvt_pk_f16_f32 %0, %1, %2" : "=v"(hb) : "v"(w[2 * j]), "v"(w[2 * j + 1]));
    asm volatile("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0]"
                 : "=v"(r0) : "v"(hb), "v"(w[2 * j]));
    asm volatile("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]"
                 : "=v"(r1) : "v"(hb), "v"(w[2 * j + 1]));
    asm volatile("v_cvt_pk_f16_f32 %0, %1, %2" : "=v"(lb) : "v"(r0), "v"(r1));
    hi[j] = hb;
    lo[j] = lb;
  }
}

// MODE 1: winner-take-all and the parabola (Eq. 13) -> dint, dsub.  MODE 2:
// the soft-argmin head over the normalised costs (P = softmax_d(-E/T)) -> the
// soft level, its state (max, log Z) and the shifted disparity.
template <int R, typename GT, int QUEUE, int MODE>
__global__ void __launch_bounds__(kThreads, 1)
agg_mfma16_kernel(View one, const BilPair* __restrict__ pairs, const int* __restrict__ tiles,
                  int n_tiles, unsigned int* __restrict__ counter) {
  using G = HGeom<R>;
  constexpr int NI = G::NI;
  extern __shared__ float lds[];
  float* const buf0 = lds;
  float* const buf1 = lds + G::BUF;
  float* const gbuf0 = lds + 2 * G::BUF;
  float* const gbuf1 = gbuf0 + G::GUIDE;
  float* const scr = gbuf1 + G::GUIDE;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int by = wave >> 2, bx = wave & 3;
  const int li = lane & 15, lk = lane >> 4;      // MFMA roles: row/column 16, k-group 4
  const int pr = li >> 2, pc = li & 3;
  const int P = lane >> 2, Q = lane & 3;         // selection roles: pixel, level quarter
  float* sc = scr + wave * (16 * 20);
  const float* prow = sc + P * 20;

  // offset (128-byte units: one row of a column quad) of this lane's patch
  // 4 i + lk for every product i, four per register (zero-weight padding
  // patches read patch 0); the operand of level li is 128 poff + 8 li bytes
  // into a slab part, the patch's guide 4 poff floats into the guide tile
  unsigned poff[(NI + 3) / 4];
#pragma unroll
  for (int i = 0; i < NI; i += 4) {
    unsigned v4 = 0;
#pragma unroll
    for (int h = 0; h < 4 && i + h < NI; ++h) {
      int p = 4 * (i + h) + lk;
      p = p < G::NP ? p : 0;
      const int rp = p / G::NCQ, cq = p - rp * G::NCQ;
      v4 |= (unsigned)((4 * by + 2 * rp) * G::NQH + bx + cq) << (8 * h);
    }
    poff[i / 4] = v4;
  }
  const int lbase = 8 * li;
  // unpacked at every use (opaque to the compiler): hoisted, the twelve
  // unpacked offsets would stay live across the tile loop and spill
  auto patch_off = [&](int i) -> int {
    unsigned pk = poff[i >> 2];
    asm volatile("" : "+v"(pk));
    return (int)((pk >> (8 * (i & 3))) & 0xFFu);
  };
  // chunk offsets (halves) of this lane's slab copies relative to the slab
  // origin (interior tiles; -1: the chunk is past the slab)
  int coff[G::KPW];
  if constexpr (G::CPR != 64) {
    const int64_t vplane = QUEUE ? 0 : one.plane;
    const int64_t rows = QUEUE ? 0 : 16 * (int64_t)one.pitch;
#pragma unroll
    for (int m = 0; m < G::KPW; ++m) {
      const int c = (wave + kWaves * m) * 64 + lane;
      const int pr = c / (G::HY * G::CPR);
      const int w = c - pr * (G::HY * G::CPR);
      const int row = w / G::CPR;
      const int cr = w - row * G::CPR;
      coff[m] = c < G::NCH ? (int)(pr * vplane + row * rows) + 8 * cr : -1;
    }
  }
  // spatial terms of this lane's slots, tabulated once per launch in LDS
  // (where it has room): per-pair launches keep the exponent
  // 12 - |p - q|^2 log2(e) / sigma_s^2, queued launches (whose pairs may
  // differ in sigma_s) the squared distance |p - q|^2; -inf / +inf outside
  // the pixel's window and for padding patches
  float* const stab = scr + G::SCR;
  auto dist2 = [&](int i, int s) -> float {
    const int p = 4 * i + lk;
    const int rp = p / G::NCQ, cq = p - rp * G::NCQ;
    const int ty = 2 * rp + (s >> 2) - pr - R, tx = 4 * cq + (s & 3) - pc - R;
    return (p < G::NP && ty >= -R && ty <= R && tx >= -R && tx <= R) ? (float)(ty * ty + tx * tx)
                                                                     : __builtin_inff();
  };
  constexpr bool kTab = G::kTable;
  if constexpr (kTab) {
    if (wave == 0) {
#pragma unroll 1
      for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const float d2 = dist2(i, s);
          stab[(i * 64 + lane) * 8 + s] = QUEUE ? d2 : fmaf(-d2, one.ks2, kLog2WScale);
        }
    }
  }

  // tiles of this workgroup.  QUEUE = 1: (pair, x0, y0) triples of a list
  // sorted longest first, dealt one per workgroup and round (below), so that
  // every workgroup's share costs nearly the same.  A shared counter would balance at run time, but an atomic that
  // returns its value waits behind the direct-to-LDS copies in flight and
  // stalls the whole workgroup once per tile.  QUEUE = 0, the tiles of one
  // pair: XCD x walks the tile columns of band x row by row.
  int tx = 1, n1 = n_tiles, per = 0, c0 = 0, bc = 1, nb = 0;
  if (!QUEUE) {
    tx = __builtin_amdgcn_readfirstlane((one.W + kTW - 1) / kTW);
    n1 = __builtin_amdgcn_readfirstlane(tx * ((one.H + kTH - 1) / kTH));
    if (gridDim.x % 8 == 0) {
      per = gridDim.x / 8;
      const int bw = (tx + 7) / 8;
      c0 = (blockIdx.x % 8) * bw;
      bc = tx - c0 < bw ? (tx - c0 > 0 ? tx - c0 : 0) : bw;
      nb = bc * (n1 / tx);
    }
  }
  auto arith_tile = [&](int k) -> int {
    if (QUEUE) {
      // round k of G workgroups covers entries [k G, (k + 1) G); workgroup b
      // (XCD b % 8) takes entry k G + (b % 8) G / 8 + b / 8, so that each XCD
      // works on a contiguous run of the list: the host orders a pair's tiles
      // in bands of a few tile columns walked row by row, so a run is a 2-D
      // patch of tiles whose halos meet in that XCD's L2
      const int G = (int)gridDim.x;
      if (G % 8 == 0) return k * G + ((int)blockIdx.x % 8) * (G / 8) + (int)blockIdx.x / 8;
      return (int)blockIdx.x + G * k;
    }
    if (per) {
      const int idx = (int)blockIdx.x / 8 + per * k;
      if (idx >= nb) return n1;
      const int row = __builtin_amdgcn_readfirstlane(idx / bc);
      return row * tx + c0 + (idx - row * bc);
    }
    return (int)blockIdx.x + (int)gridDim.x * k;
  };
  auto resolve = [&](int t, View& v, int& x0, int& y0) {
    if (QUEUE) {
      const int* e = tiles + 3 * t;
      v = view_of(pairs[e[0]]);
      x0 = e[1]; y0 = e[2];
    } else {
      v = one;
      const int ty = __builtin_amdgcn_readfirstlane(t / tx);
      x0 = (t - ty * tx) * kTW;
      y0 = ty * kTH;
    }
  };

  int cur = arith_tile(0);
  if (cur >= n1) return;                         // uniform
  {
    View cv;
    int cx0, cy0;
    resolve(cur, cv, cx0, cy0);
    GuideRaw<R, GT> g;
    stage<R>(cv, cx0, cy0, 0, buf0, wave, lane, coff, !QUEUE || G::CPR == 64);
    guide_load<R, GT>(cv, cx0, cy0, g);
    guide_store<R, GT>(gbuf0, g, cv, cx0, cy0);
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();

  int par = 0, gpar = 0;
  for (int k = 0;; ++k) {
    // weights of this wave's block, split in FP16 halves: lane (li, lk)
    // holds w(pixel li, slot s of patch 4 i + lk) in ahi[i][s], alo[i][s]
    u4 ahi[NI], alo[NI];
    float wsum = 0.0f;
    // queued launches read this tile's descriptor once, keeping scalar loads
    // out of the pass loop, where they would hold up the operand reads that
    // share their wait counter; per-pair launches take the kernel argument
    View tv;
    int tx0, ty0;
    resolve(cur, tv, tx0, ty0);
    {
      View cv;
      int cx0, cy0;
      if (QUEUE) cv = tv; else resolve(cur, cv, cx0, cy0);
      const float* gs = gpar ? gbuf1 : gbuf0;
      const float Gp = gs[(4 * by + pr + R) * G::GS + 4 * bx + pc + R];
      float ks2 = cv.ks2;
      asm volatile("" : "+v"(ks2));
#pragma unroll
      for (int i = 0; i < NI; ++i) {
        // opaque per product: keeps the guide and table reads next to their use
        const float* gp = gs + 4 * patch_off(i);
        const float4 g0 = *reinterpret_cast<const float4*>(gp);
        const float4 g1 = *reinterpret_cast<const float4*>(gp + G::GS);
        float sv[8];
        if constexpr (kTab) {
          int to = (i * 64 + lane) * 8;
          asm volatile("" : "+v"(to));
          const float* tp = stab + to;
          const float4 s0 = *reinterpret_cast<const float4*>(tp);
          const float4 s1 = *reinterpret_cast<const float4*>(tp + 4);
          sv[0] = s0.x; sv[1] = s0.y; sv[2] = s0.z; sv[3] = s0.w;
          sv[4] = s1.x; sv[5] = s1.y; sv[6] = s1.z; sv[7] = s1.w;
          if constexpr (QUEUE) {
#pragma unroll
            for (int q = 0; q < 8; ++q) sv[q] = fmaf(-sv[q], ks2, kLog2WScale);
          }
        } else {
#pragma unroll
          for (int q = 0; q < 8; ++q) sv[q] = fmaf(-dist2(i, q), ks2, kLog2WScale);
        }
        const float gq[8] = {g0.x, g0.y, g0.z, g0.w, g1.x, g1.y, g1.z, g1.w};
        float w[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const float g = Gp - gq[q];
          w[q] = __builtin_amdgcn_exp2f(fmaf(-g, g, sv[q]));
        }
        split8(w, ahi[i], alo[i]);
        if constexpr (MODE == 2) {
          const h8 wh = __builtin_bit_cast(h8, ahi[i]), wl = __builtin_bit_cast(h8, alo[i]);
#pragma unroll
          for (int q = 0; q < 8; ++q) wsum += (float)wh[q] + (float)wl[q];
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    // soft-argmin: 1 / W_p of selection pixel P (W_p = sum of its weights:
    // a lane's slots, then the four lanes of pixel li)
    float rinvP = 1.0f, zscale = 0.0f;
    if constexpr (MODE == 2) {
      View cv;
      int cx0, cy0;
      if (QUEUE) cv = tv; else resolve(cur, cv, cx0, cy0);
      zscale = -cv.invT * 1.4426950408889634f;
      float ws = wsum;
      ws += __shfl_xor(ws, 16);
      ws += __shfl_xor(ws, 32);
      rinvP = 1.0f / __shfl(ws, P);
    }
    // no barrier here: the weights read only this tile's guide (complete since
    // the last pass's barrier) and the spatial table
    const int nxt = arith_tile(k + 1);
    const bool has_next = nxt < n1;
    View nv = tv;
    int nx0 = 0, ny0 = 0;
    if (QUEUE && has_next) resolve(nxt, nv, nx0, ny0);

    float bestE = 3.402823466e38f, Em = 0.f, Ep = 0.f, lastE = 0.f;
    int bestD = 0;
    bool pending = false;
    constexpr float kNeg = -3.402823466e38f;
    float mr = kNeg, Zr = 0.0f, Sr = 0.0f;
    int D, passes;
    {
      View cv;
      int cx0, cy0;
      if (QUEUE) cv = tv; else resolve(cur, cv, cx0, cy0);
      D = cv.D;
      passes = (D + 15) / 16;
    }
    for (int p = 0; p < passes; ++p) {
      // the pass reads one buffer while the copies fill the other; as
      // __restrict__ parameters the compiler knows that they do not alias
      // and does not wait for the copies before the pass's first LDS read
      // (1280x720, D = 64, R = 7: 0.272 -> 0.257 ms per launch)
      auto pass_body = [&](float* __restrict__ cbuf, float* __restrict__ obuf) {
      const int d0 = 16 * p;
      const bool last = p + 1 == passes;
      GuideRaw<R, GT> gq;
      if (!last || has_next) {
        View sv;
        int sx0, sy0;
        if (QUEUE) {
          sv = last ? nv : tv;
          sx0 = last ? nx0 : tx0;
          sy0 = last ? ny0 : ty0;
        } else {
          resolve(last ? nxt : cur, sv, sx0, sy0);
        }
        stage<R>(sv, sx0, sy0, last ? 0 : d0 + 16, obuf, wave, lane, coff, !QUEUE || G::CPR == 64);
        if (last) guide_load<R, GT>(sv, sx0, sy0, gq);
      }
      const char* cb = reinterpret_cast<const char*>(cbuf);
      // two accumulators (products i even / odd): halves the dependent chain
      f4 acc = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
      // operands of product i + 1 are read while product i is multiplied
      u4 bh[2], bl[2];
      auto load_b = [&](int i, u4& h, u4& l) {
        const char* a = cb + lbase + 128 * patch_off(i);
        const uint2 h0 = *reinterpret_cast<const uint2*>(a);
        const uint2 h1 = *reinterpret_cast<const uint2*>(a + G::ROWB);
        const uint2 l0 = *reinterpret_cast<const uint2*>(a + G::PARTB);
        const uint2 l1 = *reinterpret_cast<const uint2*>(a + G::PARTB + G::ROWB);
        h = u4{h0.x, h0.y, h1.x, h1.y};
        l = u4{l0.x, l0.y, l1.x, l1.y};
      };
      __builtin_amdgcn_sched_barrier(0);
      load_b(0, bh[0], bl[0]);
#pragma unroll
      for (int i = 0; i < NI; ++i) {
        if (i + 1 < NI) load_b(i + 1, bh[(i + 1) & 1], bl[(i + 1) & 1]);
        __builtin_amdgcn_sched_barrier(0);
        const h8 bH = __builtin_bit_cast(h8, bh[i & 1]);
        const h8 bL = __builtin_bit_cast(h8, bl[i & 1]);
        const h8 aH = __builtin_bit_cast(h8, ahi[i]);
        const h8 aL = __builtin_bit_cast(h8, alo[i]);
        f4& ac = (i & 1) ? acc1 : acc;
        ac = __builtin_amdgcn_mfma_f32_16x16x32_f16(aH, bH, ac, 0, 0, 0);
        ac = __builtin_amdgcn_mfma_f32_16x16x32_f16(aH, bL, ac, 0, 0, 0);
        ac = __builtin_amdgcn_mfma_f32_16x16x32_f16(aL, bH, ac, 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
      }
      acc += acc1;
      // lane holds pixel 4 lk + v, level d0 + li
#pragma unroll
      for (int v = 0; v < 4; ++v) sc[(4 * lk + v) * 20 + li] = acc[v];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if constexpr (MODE == 1) {
        // first minimum over the pass: a quad of lanes per pixel, four levels
        // per lane, then merged across the quad (lower level wins ties)
        const float4 e4 = *reinterpret_cast<const float4*>(prow + 4 * Q);
        const int nvl = D - d0 - 4 * Q;
        const float inf = __builtin_inff();
        const float e0 = nvl > 0 ? e4.x : inf, e1 = nvl > 1 ? e4.y : inf;
        const float e2 = nvl > 2 ? e4.z : inf, e3 = nvl > 3 ? e4.w : inf;
        float m = fminf(fminf(e0, e1), fminf(e2, e3));
        int idx = 4 * Q + (e0 == m ? 0 : (e1 == m ? 1 : (e2 == m ? 2 : 3)));
        {
          const float om = bilm::dpp_f<0xB1>(m);
          const int oi = __builtin_amdgcn_mov_dpp(idx, 0xB1, 0xF, 0xF, false);
          const bool take = om < m || (om == m && oi < idx);
          m = take ? om : m;
          idx = take ? oi : idx;
        }
        {
          const float om = bilm::dpp_f<0x4E>(m);
          const int oi = __builtin_amdgcn_mov_dpp(idx, 0x4E, 0xF, 0xF, false);
          const bool take = om < m || (om == m && oi < idx);
          m = take ? om : m;
          idx = take ? oi : idx;
        }
        if (pending) Ep = prow[0];               // level after a best at the previous pass's end
        if (m < bestE) {
          Em = idx > 0 ? prow[idx > 0 ? idx - 1 : 0] : lastE;
          Ep = prow[idx < 15 ? idx + 1 : 15];
          bestE = m;
          bestD = d0 + idx;
          pending = idx == 15;
        } else {
          pending = false;
        }
        lastE = prow[D - d0 < 16 ? D - d0 - 1 : 15];
      } else {
        // soft-argmin: each lane keeps the running state (max, Z, S) of its
        // quarter of every pass's levels; the quad is merged once per tile
        const float4 e4 = *reinterpret_cast<const float4*>(prow + 4 * Q);
        const int nvl = D - d0 - 4 * Q;
        const float zv[4] = {nvl > 0 ? e4.x * rinvP * zscale : kNeg, nvl > 1 ? e4.y * rinvP * zscale : kNeg,
                             nvl > 2 ? e4.z * rinvP * zscale : kNeg, nvl > 3 ? e4.w * rinvP * zscale : kNeg};
        const float M = fmaxf(mr, fmaxf(fmaxf(zv[0], zv[1]), fmaxf(zv[2], zv[3])));
        const float a = __builtin_amdgcn_exp2f(mr - M);
        Zr *= a;
        Sr *= a;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float e = nvl > j ? __builtin_amdgcn_exp2f(zv[j] - M) : 0.0f;
          Zr += e;
          Sr = fmaf((float)(d0 + 4 * Q + j), e, Sr);
        }
        mr = M;
      }
      if (last && has_next) {
        View gv = nv;
        int gx0 = nx0, gy0 = ny0;
        if (!QUEUE) resolve(nxt, gv, gx0, gy0);
        guide_store<R, GT>(gpar ? gbuf0 : gbuf1, gq, gv, gx0, gy0);
      }
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
      };
      pass_body(par ? buf1 : buf0, par ? buf0 : buf1);
      par ^= 1;
    }
    if constexpr (MODE == 2) {
      auto merge = [&](float om, float oZ, float oS) {
        const float M = fmaxf(mr, om);
        const float a = __builtin_amdgcn_exp2f(mr - M), b = __builtin_amdgcn_exp2f(om - M);
        Zr = fmaf(Zr, a, oZ * b);
        Sr = fmaf(Sr, a, oS * b);
        mr = M;
      };
      merge(bilm::dpp_f<0xB1>(mr), bilm::dpp_f<0xB1>(Zr), bilm::dpp_f<0xB1>(Sr));
      merge(bilm::dpp_f<0x4E>(mr), bilm::dpp_f<0x4E>(Zr), bilm::dpp_f<0x4E>(Sr));
    }
    if (MODE == 2 && Q == 0) {
      View cv;
      int cx0, cy0;
      resolve(cur, cv, cx0, cy0);
      const int py = cy0 + 4 * by + (P >> 2), px = cx0 + 4 * bx + (P & 3);
      if (py < cv.H && px < cv.W) {
        const int64_t pix = (int64_t)py * cv.W + px;
        const float ln2 = 0.6931471805599453f;
        const float dh = Sr / Zr;
        cv.sm_m[pix] = mr * ln2;
        cv.sm_logZ[pix] = __builtin_amdgcn_logf(Zr) * ln2;
        cv.sm_dh[pix] = dh;
        const double dd = dh;
        cv.disp[pix] = (float)(dd - cv.delta_p + (cv.c0 + cv.c1 * ((double)px - dd + cv.delta_p) +
                                                  cv.c2 * (double)py));
      }
    }
    if (MODE == 1 && Q == 0) {
      View cv;
      int cx0, cy0;
      resolve(cur, cv, cx0, cy0);
      const int py = cy0 + 4 * by + (P >> 2), px = cx0 + 4 * bx + (P & 3);
      if (py < cv.H && px < cv.W) {
        cv.dint[(int64_t)py * cv.W + px] = (int16_t)bestD;
        if (cv.dsub) {
          float off = 0.0f;
          if (bestD > 0 && bestD < D - 1) {
            const float den = 2.0f * Em + 2.0f * Ep - 4.0f * bestE;
            if (den > 0.0f) off = (Em - Ep) / den;
          }
          cv.dsub[(int64_t)py * cv.W + px] = (float)bestD + off;
        }
      }
    }
    if (!has_next) break;
    cur = nxt;
    gpar ^= 1;
  }
}

template <int R, typename GT, int QUEUE, int MODE>
hipError_t set_lds_attr() {
  static bool done = false;
  if (!done) {
    hipError_t e = hipFuncSetAttribute((const void*)agg_mfma16_kernel<R, GT, QUEUE, MODE>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)HGeom<R>::lds_bytes);
    if (e != hipSuccess) return e;
    done = true;
  }
  return hipSuccess;
}

// One pair: persistent, one workgroup per CU.
template <int R, typename GT, int MODE>
hipError_t launch_pair(const BilPair& a, hipStream_t s) {
  if (!a.h2 || a.h2_pitch < h2_pitch_for<R>(a.W) || (a.h2_pitch & 7) ||
      a.h2_plane < 16 * (int64_t)a.H * a.h2_pitch)
    return hipErrorInvalidValue;
  hipError_t e = set_lds_attr<R, GT, 0, MODE>();
  if (e != hipSuccess) return e;
  const int n = ((a.W + kTW - 1) / kTW) * ((a.H + kTH - 1) / kTH);
  const int cus = bilm::cu_count_of_current_device();
  int grid = std::min(n, cus > 0 ? cus : 256);
  if (grid >= 8) grid -= grid % 8;               // whole XCD bands
  hipLaunchKernelGGL((agg_mfma16_kernel<R, GT, 0, MODE>), dim3(grid), dim3(kThreads),
                     HGeom<R>::lds_bytes, s, view_of(a), (const BilPair*)nullptr,
                     (const int*)nullptr, 0, (unsigned int*)nullptr);
  return hipGetLastError();
}

// Queue of (pair, x0, y0) tiles over many pairs (x0 a multiple of kTW, y0 of kTH).
template <int R, typename GT>
hipError_t launch_queue(const BilPair* pairs, const int* tiles, int n_tiles, unsigned int* counter,
                        int n_groups, hipStream_t s) {
  hipError_t e = set_lds_attr<R, GT, 1, 1>();
  if (e != hipSuccess) return e;
  View none{};
  hipLaunchKernelGGL((agg_mfma16_kernel<R, GT, 1, 1>), dim3(n_groups), dim3(kThreads),
                     HGeom<R>::lds_bytes, s, none, pairs, tiles, n_tiles, counter);
  return hipGetLastError();
}

template <int R>
hipError_t launch_args(const Plan& P, const BilArgs& a, int mode, hipStream_t s) {
  const BilPair b = bil::make_pair(P, a);
  if (mode == 2)
    return a.guide_dt == STEREO_U8 ? launch_pair<R, uint8_t, 2>(b, s) : launch_pair<R, float, 2>(b, s);
  return a.guide_dt == STEREO_U8 ? launch_pair<R, uint8_t, 1>(b, s) : launch_pair<R, float, 1>(b, s);
}

template <int R>
hipError_t launch_queue_r(stereo_dtype gdt, const BilPair* pairs, const int* tiles, int n_tiles,
                          unsigned int* counter, int n_groups, hipStream_t s) {
  return gdt == STEREO_U8 ? launch_queue<R, uint8_t>(pairs, tiles, n_tiles, counter, n_groups, s)
                          : launch_queue<R, float>(pairs, tiles, n_tiles, counter, n_groups, s);
}

}  // namespace bilh
}  // namespace stereo
