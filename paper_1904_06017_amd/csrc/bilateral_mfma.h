// Bilateral cost aggregation, Eqs. (10)-(11), fused with winner-take-all
// selection and sub-pixel refinement (Sec. 3.2.2, Eq. 13), on the matrix cores.
//
// For one 4x4 block of pixels p and 16 levels d, the aggregated costs are the
// matrix product E[p][d] = sum_q w(p, q) C(q, d) over the positions q of the
// block's window union ((2R + 4) x (2R + 4) halo positions).  One wave owns one
// block: the contraction runs on v_mfma_f32_16x16x4f32 with M = the 16 pixels,
// N = 16 levels and K = 2x2 positions of the union, so a block takes
// (R + 2)^2 products per 16 levels.  Weights outside a pixel's own window are
// zero, which keeps the sum equal to the windowed one.  The weights w depend on
// the guide only: each wave evaluates its (R + 2)^2 operand registers once per
// tile and reuses them for every level.
//
// A workgroup (12 waves) owns a 16 x 12 pixel tile and walks the levels in
// passes of 16.  Each pass's halo slab (4 level quads x halo rows x 36 float4
// slots) is copied global -> LDS by direct-to-LDS loads into one of two
// buffers while the other is being multiplied, one barrier per pass (a last
// pass with fewer than 16 levels copies the quads that hold a level below D).
// Tiles at the image border stage through registers with every bound checked
// instead.  The kernel is persistent: one workgroup per CU
// takes tiles in turn and prefetches the next tile's first slab and guide
// during its current tile's last pass.
//
// Per pixel the result depends on the pixel's block and the levels only (the
// block grid is aligned to the image origin and the products run in a fixed
// order), so the per-pair and the queued batch launches give bitwise equal
// results.  The summation order differs from the vector-ALU kernel's raster
// order: the two engines agree to rounding, not bit for bit.
#pragma once
#include "bilateral_impl.h"

#define BILM_GLOBAL __attribute__((address_space(1)))
#define BILM_LOCAL __attribute__((address_space(3)))

namespace stereo {
namespace bilm {

using bil::BilPair;
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kBR = 3;                  // block rows per tile
constexpr int kWaves = 4 * kBR;         // one 4x4 block per wave
constexpr int kThreads = 64 * kWaves;
constexpr int kTW = 16, kTH = 4 * kBR;  // tile in pixels
static_assert(kTW == kMfmaTileW && kTH == kMfmaTileH, "tile size shared with the batch tables");
constexpr int kRS = 36;                 // float4 slots per staged halo row
constexpr float kFar = 1e30f;           // guide outside the image: zero weight

template <int R>
struct MGeom {
  static constexpr int NB = R + 2;                              // 2x2 K-blocks per side
  static constexpr int HY = kTH + 2 * R, HX = kTW + 2 * R;
  // quad plane stride = 8 (mod 64) floats: with the 36-slot rows the operand
  // reads of one MFMA spread over the LDS banks
  static constexpr int QS0 = HY * kRS * 4;
  static constexpr int QS = QS0 + ((8 - QS0 % 64) + 64) % 64;
  static constexpr int BUF = 4 * QS;                            // floats per slab
  static constexpr int NCH = (HY * kRS + 63) / 64;              // 64-slot copies per quad plane
  static constexpr int NK = 4 * NCH;                            // copies per slab
  static constexpr int KPW = (NK + kWaves - 1) / kWaves;
  static constexpr int GS = 32;                                 // guide row stride
  static constexpr int GUIDE = HY * GS;
  static constexpr int GPT = (GUIDE + kThreads - 1) / kThreads;
  static constexpr int SCR = kWaves * 16 * 20;                  // per-wave [pixel][20] scratch
  static constexpr size_t lds_bytes = sizeof(float) * (2 * BUF + 2 * GUIDE + SCR);
  static_assert(HX + 3 <= kRS && HX <= GS, "halo wider than its slots");
  // row = (s * 1821) >> 16 equals s / 36 for s < 1080
  static_assert(HY * kRS <= 1080, "slot split by multiplication out of range");
  static_assert(lds_bytes <= 160 * 1024, "LDS budget");
};

// The fields one tile needs; uniform across the workgroup.
struct View {
  const float4* C;
  uint32_t slice, pitch;
  int shift;
  const void* guide;
  int64_t g_pitch;
  int W, H, D;
  float ks2, kr2;
  int16_t* dint;                  // selection (mode 1)
  float* dsub;
  float* sm_m;                    // soft-argmin (mode 2): max_d(-E/T), log Z,
  float* sm_logZ;                 // soft level and the shifted disparity
  float* sm_dh;
  float* disp;
  float invT;
  double delta_p, c0, c1, c2;
};

__host__ __device__ inline View view_of(const BilPair& a) {
  View v;
  v.C = reinterpret_cast<const float4*>(a.C);
  v.slice = (uint32_t)a.c_slice;
  v.pitch = (uint32_t)a.c_pitch;
  v.shift = a.shift;
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

// Slab of levels [d0, d0 + 16) of the tile at (x0, y0) into buf:
// buf[q][row][slot] float4.  Reference volume: slot c holds the quad of halo
// column c.  Target volume (level d of column x is read at column x + d):
// slot c holds the quad at extended column x0 - R + c + d0 + 4q, whose
// component j is level 4q + j of halo column c - j.
// In a last pass with fewer than 16 levels only the quads holding a level
// below D are copied; the slab's other levels keep stale values, which stay in
// their own output columns of the product and are never selected.  A target
// slot whose column passes the volume's pitch holds levels >= D or columns
// >= W only (x + d >= W + D - 1), so its column is clamped.
template <int R>
__device__ __forceinline__ void stage(const View& v, int x0, int y0, int d0, float* buf,
                                      int wave, int lane) {
  using G = MGeom<R>;
  const bool inner = x0 >= R && x0 + kTW + R <= v.W && y0 >= R && y0 + kTH + R <= v.H;
  if (inner) {
    const uint32_t base = (uint32_t)(d0 >> 2) * v.slice + (uint32_t)(y0 - R) * v.pitch +
                          (uint32_t)(x0 - R + (v.shift ? d0 : 0));
    const uint32_t qstep = v.slice + (v.shift ? 4u : 0u);
    const int cmax = v.shift ? G::HX + 2 : G::HX - 1;
    const int nq = (v.D - d0 + 3) >> 2;          // quads with a level below D (>= 1)
    // recomputed per pass: hoisted out of the pass loop, the per-lane offsets
    // would stay live across the products and crowd out the operand prefetch
    int ln = lane;
    asm volatile("" : "+v"(ln));
    // last column of the volume row relative to the slab's first column
    const int emax = (int)v.pitch - 1 - (x0 - R + (v.shift ? d0 : 0));
#pragma unroll
    for (int m = 0; m < G::KPW; ++m) {
      const int k = wave + kWaves * m;
      if (k < G::NK) {
        const int q = k / G::NCH, ch = k - q * G::NCH;
        const int s = ch * 64 + ln;
        if (q < nq && s < G::HY * kRS) {
          const int row = (s * 1821) >> 16, col = s - row * kRS;
          int cc = col < cmax ? col : cmax;
          if (v.shift) cc = cc + 4 * q <= emax ? cc : emax - 4 * q;
          const uint32_t off = (uint32_t)q * qstep + (uint32_t)row * v.pitch + (uint32_t)cc;
          __builtin_amdgcn_global_load_lds((BILM_GLOBAL void*)(v.C + base + off),
                                           (BILM_LOCAL void*)(buf + q * G::QS + ch * 256), 16, 0, 0);
        }
      }
    }
    return;
  }
  const int ncol = v.shift ? G::HX + 3 : G::HX;
  const int n = 4 * G::HY * ncol;
  for (int i = threadIdx.x; i < n; i += kThreads) {
    const int q = i / (G::HY * ncol);
    const int rem = i - q * (G::HY * ncol);
    const int row = rem / ncol, c = rem - row * ncol;
    const int gy = y0 - R + row, dq = d0 + 4 * q;
    const int e = v.shift ? x0 - R + c + dq : x0 - R + c;
    float4 val = make_float4(0.f, 0.f, 0.f, 0.f);
    if (gy >= 0 && gy < v.H && dq < v.D && e >= 0 && e < (int)v.pitch)
      val = v.C[(uint32_t)(dq >> 2) * v.slice + (uint32_t)gy * v.pitch + (uint32_t)e];
    float comp[4] = {val.x, val.y, val.z, val.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int x = v.shift ? x0 - R + c - j : x0 - R + c;
      comp[j] = (x >= 0 && x < v.W && dq + j < v.D) ? comp[j] : 0.0f;
    }
    *reinterpret_cast<float4*>(buf + q * G::QS + (row * kRS + c) * 4) =
        make_float4(comp[0], comp[1], comp[2], comp[3]);
  }
}

// Guide of the tile's halo, scaled by sqrt(kr2), into registers (kFar outside).
template <int R, typename GT>
__device__ __forceinline__ void guide_load(const View& v, int x0, int y0, float (&g)[MGeom<R>::GPT]) {
  using G = MGeom<R>;
  const GT* __restrict__ src = static_cast<const GT*>(v.guide);
  const float kr = sqrtf(v.kr2);
#pragma unroll
  for (int k = 0; k < G::GPT; ++k) {
    const int i = threadIdx.x + k * kThreads;
    const int yy = i / G::GS, xx = i % G::GS;
    const int gy = y0 - R + yy, gx = x0 - R + xx;
    const bool in = i < G::GUIDE && xx < G::HX && gy >= 0 && gy < v.H && gx >= 0 && gx < v.W;
    g[k] = in ? (float)src[(int64_t)gy * v.g_pitch + gx] * kr : kFar;
  }
}

template <int R>
__device__ __forceinline__ void guide_store(float* gs, const float (&g)[MGeom<R>::GPT]) {
  using G = MGeom<R>;
#pragma unroll
  for (int k = 0; k < G::GPT; ++k) {
    const int i = threadIdx.x + k * kThreads;
    if (i < G::GUIDE) gs[i] = g[k];
  }
}

// A float from another lane of the quad (DPP quad permutation CTL).
template <int CTL>
__device__ __forceinline__ float dpp_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTL, 0xF, 0xF, false));
}

// MODE 1: winner-take-all and the parabola (Eq. 13) -> dint, dsub.  MODE 2:
// the soft-argmin head over the normalised costs (P = softmax_d(-E/T)) -> the
// soft level, its state (max, log Z) and the shifted disparity.
template <int R, typename GT, int QUEUE, int MODE>
__global__ void __launch_bounds__(kThreads, 1)
agg_wta_mfma_kernel(View one, const BilPair* __restrict__ pairs, const int* __restrict__ tiles,
                    int n_tiles, unsigned int* __restrict__ counter) {
  using G = MGeom<R>;
  constexpr int NB = G::NB;
  extern __shared__ float lds[];
  __shared__ int s_next;
  float* const buf0 = lds;
  float* const buf1 = lds + G::BUF;
  float* const gbuf0 = lds + 2 * G::BUF;
  float* const gbuf1 = gbuf0 + G::GUIDE;
  float* const scr = gbuf1 + G::GUIDE;
  const int lane = threadIdx.x & 63;
  // From R = 7 on the weights fill most vector registers; there the wave
  // index is read into a scalar register, so that the values derived from it
  // (block position, copy chunks, scratch base) stay scalar instead of being
  // spilled to scratch and reloaded in every pass (measured 6 % faster at
  // R = 7, 17 % at R = 8).  At R <= 6 the vector form measured 0-3 % faster.
  const int wave = R >= 7 ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : (threadIdx.x >> 6);
  const int by = wave >> 2, bx = wave & 3;
  const int li = lane & 15, lk = lane >> 4;      // MFMA roles: row/column 16, k-group 4
  const int pr = li >> 2, pc = li & 3, dy0 = lk >> 1, dx0 = lk & 1;
  const int P = lane >> 2, Q = lane & 3;         // selection roles: pixel, level quarter
  float* sc = scr + wave * (16 * 20);
  const float* prow = sc + P * 20;

  // tiles of this workgroup.  QUEUE = 1: (pair, x0, y0) triples taken from a
  // counter.  QUEUE = 0, the tiles of one pair: workgroup b runs on XCD b % 8
  // (round-robin dispatch), so XCD x walks the tile columns of band x (ceil of
  // a eighth of them) row by row with its workgroups in turn: the tiles in
  // flight on one XCD are neighbours and share their halos in its L2.
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
    if (per) {
      const int idx = (int)blockIdx.x / 8 + per * k;
      if (idx >= nb) return n1;
      const int row = __builtin_amdgcn_readfirstlane(idx / bc);
      return row * tx + c0 + (idx - row * bc);
    }
    return (int)blockIdx.x + (int)gridDim.x * k;
  };
  // descriptors are re-read where needed (scalar loads) rather than kept live
  auto resolve = [&](int t, View& v, int& x0, int& y0) {
    if (QUEUE) {
      const int* e = tiles + 3 * t;
      v = view_of(pairs[e[0]]);
      x0 = e[1]; y0 = e[2];
    } else {
      v = one;
      // the division expands to vector ALU code: bring the (uniform) result back
      // to scalar registers so that everything derived from it stays scalar
      const int ty = __builtin_amdgcn_readfirstlane(t / tx);
      x0 = (t - ty * tx) * kTW;
      y0 = ty * kTH;
    }
  };

  int cur;
  if (QUEUE) {
    if (threadIdx.x == 0) s_next = (int)atomicAdd(counter, 1u);
    __syncthreads();
    cur = __builtin_amdgcn_readfirstlane(s_next);
  } else {
    cur = arith_tile(0);
  }
  if (cur >= n1) return;                         // uniform
  {
    View cv;
    int cx0, cy0;
    resolve(cur, cv, cx0, cy0);
    float g[G::GPT];
    stage<R>(cv, cx0, cy0, 0, buf0, wave, lane);
    guide_load<R, GT>(cv, cx0, cy0, g);
    guide_store<R>(gbuf0, g);
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();

  int par = 0, gpar = 0;
  for (int k = 0;; ++k) {
    if (QUEUE && threadIdx.x == 0) s_next = (int)atomicAdd(counter, 1u);
    // weights of this wave's block: lane (li, lk) holds w(pixel li, position
    // (2i + dy0, 2j + dx0) of the union) for K-block (i, j)
    float wv[NB * NB];
    {
      View cv;
      int cx0, cy0;
      resolve(cur, cv, cx0, cy0);
      const float* gs = gpar ? gbuf1 : gbuf0;
      const float Gp = gs[(4 * by + pr + R) * G::GS + 4 * bx + pc + R];
      const float* gb = gs + (4 * by + dy0) * G::GS + 4 * bx + dx0;
      // opaque per tile: otherwise the spatial terms of all (R + 2)^2 K-blocks
      // are hoisted out of the tile loop and spilled
      float ks2 = cv.ks2;
      asm volatile("" : "+v"(ks2));
      float sy[NB], sx[NB];
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const int ty = 2 * i + dy0 - pr - R, tx2 = 2 * i + dx0 - pc - R;
        sy[i] = (ty >= -R && ty <= R) ? -(float)(ty * ty) * ks2 : -__builtin_inff();
        sx[i] = (tx2 >= -R && tx2 <= R) ? -(float)(tx2 * tx2) * ks2 : -__builtin_inff();
      }
      // one union row at a time: keeps the guide reads from piling up in registers
#pragma unroll
      for (int i = 0; i < NB; ++i) {
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          const float g = Gp - gb[2 * i * G::GS + 2 * j];
          wv[i * NB + j] = __builtin_amdgcn_exp2f(fmaf(-g, g, sy[i] + sx[j]));
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    // soft-argmin: 1 / W_p of selection pixel P (W_p = sum of its weights:
    // a lane's K-groups, then the four lanes of pixel li)
    float rinvP = 1.0f, zscale = 0.0f;
    if constexpr (MODE == 2) {
      View cv;
      int cx0, cy0;
      resolve(cur, cv, cx0, cy0);
      zscale = -cv.invT * 1.4426950408889634f;
      float ws = 0.0f;
#pragma unroll
      for (int kb = 0; kb < NB * NB; ++kb) ws += wv[kb];
      ws += __shfl_xor(ws, 16);
      ws += __shfl_xor(ws, 32);
      rinvP = 1.0f / __shfl(ws, P);
    }
    __syncthreads();                             // publishes s_next
    const int nxt = QUEUE ? __builtin_amdgcn_readfirstlane(s_next) : arith_tile(k + 1);
    const bool has_next = nxt < n1;

    float bestE = 3.402823466e38f, Em = 0.f, Ep = 0.f, lastE = 0.f;
    int bestD = 0;
    bool pending = false;
    // soft-argmin state in base-2 exponents z = -E log2(e) / T: running max,
    // Z = sum_d 2^(z - max), S = sum_d d 2^(z - max)
    constexpr float kNeg = -3.402823466e38f;
    float mr = kNeg, Zr = 0.0f, Sr = 0.0f;
    int D, passes;
    {
      View cv;
      int cx0, cy0;
      resolve(cur, cv, cx0, cy0);
      D = cv.D;
      passes = (D + 15) / 16;
    }
    for (int p = 0; p < passes; ++p) {
      // the two slab buffers as __restrict__ parameters: the products need
      // not wait for the copies into the other buffer
      auto pass_body = [&](float* __restrict__ cbuf, float* __restrict__ obuf) {
      const int d0 = 16 * p;
      const bool last = p + 1 == passes;
      float gq[G::GPT];
      int shift;
      {
        View cv;
        int cx0, cy0;
        resolve(cur, cv, cx0, cy0);
        shift = cv.shift;
      }
      // one staging site: the next slab of this tile, or the first of the next
      if (!last || has_next) {
        View sv;
        int sx0, sy0;
        resolve(last ? nxt : cur, sv, sx0, sy0);
        stage<R>(sv, sx0, sy0, last ? 0 : d0 + 16, obuf, wave, lane);
        if (last) guide_load<R, GT>(sv, sx0, sy0, gq);
      }
      const int lq = li >> 2, lj = li & 3;
      const int boff = lq * G::QS + ((4 * by + dy0) * kRS + 4 * bx + dx0) * 4 + (shift ? 5 * lj : lj);
      const float* cb = cbuf + boff;
      f4 acc = {0.f, 0.f, 0.f, 0.f};
      // operands of union row i + 1 are read while row i is multiplied
      float bb[2][NB];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int j = 0; j < NB; ++j) bb[0][j] = cb[2 * j * 4];
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        if (i + 1 < NB) {
#pragma unroll
          for (int j = 0; j < NB; ++j) bb[(i + 1) & 1][j] = cb[(2 * (i + 1) * kRS + 2 * j) * 4];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 0; j < NB; ++j)
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wv[i * NB + j], bb[i & 1][j], acc, 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
      }
      // lane holds pixel 4 lk + v, level d0 + li
#pragma unroll
      for (int v = 0; v < 4; ++v) sc[(4 * lk + v) * 20 + li] = acc[v];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // first minimum over the pass: a quad of lanes per pixel, four levels
      // per lane, then merged across the quad (lower level wins ties)
      if constexpr (MODE == 1) {
        const float4 e4 = *reinterpret_cast<const float4*>(prow + 4 * Q);
        const int nvl = D - d0 - 4 * Q;
        const float inf = __builtin_inff();
        const float e0 = nvl > 0 ? e4.x : inf, e1 = nvl > 1 ? e4.y : inf;
        const float e2 = nvl > 2 ? e4.z : inf, e3 = nvl > 3 ? e4.w : inf;
        float m = fminf(fminf(e0, e1), fminf(e2, e3));
        int idx = 4 * Q + (e0 == m ? 0 : (e1 == m ? 1 : (e2 == m ? 2 : 3)));
        {
          const float om = __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, m), 0xB1, 0xF, 0xF, false));
          const int oi = __builtin_amdgcn_mov_dpp(idx, 0xB1, 0xF, 0xF, false);
          const bool take = om < m || (om == m && oi < idx);
          m = take ? om : m;
          idx = take ? oi : idx;
        }
        {
          const float om = __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, m), 0x4E, 0xF, 0xF, false));
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
        // soft-argmin: each lane keeps the running state of its quarter of
        // every pass's levels (rescaled when its maximum grows); the quad is
        // merged once per tile, below
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
      if (last && has_next) guide_store<R>(gpar ? gbuf0 : gbuf1, gq);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
      };
      pass_body(par ? buf1 : buf0, par ? buf0 : buf1);
      par ^= 1;
    }
    if constexpr (MODE == 2) {
      // the quad's four running states into one (every lane takes part)
      auto merge = [&](float om, float oZ, float oS) {
        const float M = fmaxf(mr, om);
        const float a = __builtin_amdgcn_exp2f(mr - M), b = __builtin_amdgcn_exp2f(om - M);
        Zr = fmaf(Zr, a, oZ * b);
        Sr = fmaf(Sr, a, oS * b);
        mr = M;
      };
      merge(dpp_f<0xB1>(mr), dpp_f<0xB1>(Zr), dpp_f<0xB1>(Sr));
      merge(dpp_f<0x4E>(mr), dpp_f<0x4E>(Zr), dpp_f<0x4E>(Sr));
    }
    if (MODE == 2 && Q == 0) {
      // soft level, the saved state (m, log Z) in natural units, and the
      // shift back D = dh - delta_p + d_road(u - dh + delta_p, v)
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

inline int cu_count_of_current_device() {
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (cache[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    cache[dev] = n;
  }
  return cache[dev];
}

template <int R, typename GT, int QUEUE, int MODE>
hipError_t set_lds_attr() {
  static bool done = false;
  if (!done) {
    hipError_t e = hipFuncSetAttribute((const void*)agg_wta_mfma_kernel<R, GT, QUEUE, MODE>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)MGeom<R>::lds_bytes);
    if (e != hipSuccess) return e;
    done = true;
  }
  return hipSuccess;
}

// One pair (quad-layout volume): persistent, one workgroup per CU.
template <int R, typename GT, int MODE>
hipError_t launch_pair(const BilPair& a, hipStream_t s) {
  if (!a.quad) return hipErrorInvalidValue;
  hipError_t e = set_lds_attr<R, GT, 0, MODE>();
  if (e != hipSuccess) return e;
  const int n = ((a.W + kTW - 1) / kTW) * ((a.H + kTH - 1) / kTH);
  const int cus = cu_count_of_current_device();
  int grid = std::min(n, cus > 0 ? cus : 256);
  if (grid >= 8) grid -= grid % 8;               // whole XCD bands
  hipLaunchKernelGGL((agg_wta_mfma_kernel<R, GT, 0, MODE>), dim3(grid), dim3(kThreads), MGeom<R>::lds_bytes, s,
                     view_of(a), (const BilPair*)nullptr, (const int*)nullptr, 0, (unsigned int*)nullptr);
  return hipGetLastError();
}

// Queue of (pair, x0, y0) tiles over many pairs (x0 a multiple of kTW, y0 of kTH).
template <int R, typename GT>
hipError_t launch_queue(const BilPair* pairs, const int* tiles, int n_tiles, unsigned int* counter,
                        int n_groups, hipStream_t s) {
  hipError_t e = set_lds_attr<R, GT, 1, 1>();
  if (e != hipSuccess) return e;
  View none{};
  hipLaunchKernelGGL((agg_wta_mfma_kernel<R, GT, 1, 1>), dim3(n_groups), dim3(kThreads), MGeom<R>::lds_bytes, s,
                     none, pairs, tiles, n_tiles, counter);
  return hipGetLastError();
}

// Entry points of one radius: the plan's pair (guide type from the args);
// mode 1 selection, mode 2 soft-argmin.
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

}  // namespace bilm
}  // namespace stereo
