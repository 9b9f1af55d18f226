// Backward of the soft-argmin head through the bilateral aggregation
// (Eqs. 10-11 differentiated) on the FP16 matrix cores with split operands.
//
// The two passes of the vector-ALU backward (one level tile of the
// recomputed cost volume at a time) become two product chains per 4x4 pixel
// block and 16 levels, both over the block's window union as in the forward
// kernel, with the same costs (B) and two weight operands (A):
//   w(p, q)                       (Eq. 11's weight)
//   w(p, q) (G'(p) - G'(q))       (its derivative in the guide, up to the
//                                  factor -2 kr2, applied by the caller)
// Pass 1 (B = the tile's costs C) forms E = sum_q w C / W_p, the softmax
// adjoint dE = g' (-1/T) P (d - dh), writes C' = dE / W_p and accumulates
//   aP += sum_d dE E,  A1 += sum_d dE sum_q w (G'(p) - G'(q)) C(q, d) / kr.
// Pass 2 (B = C', scaled into the FP16 range) forms dC = sum_q w C' (the
// weights are symmetric, so this is the adjoint of Eq. 11's sum over the
// window) and accumulates
//   A2 += -sum_d C(p, d) sum_q w (G'(p) - G'(q)) C'(q, d) / kr.
// Both operands are split (x = x_hi + x_lo, three FP16 products per term,
// FP32 accumulation), so the sums are as accurate as FP32 products; the
// weights carry the 2^12 scale of the forward kernel and C' a power-of-two
// scale S (the gradient's magnitude is arbitrary) chosen from a bound on
// |C'|: P <= 1, |d - dh| <= D - 1 and W_p >= 1 (the pixel's own weight) give
// |C'| <= max |g'| |1 - c1| (D - 1) / T; both scales are removed exactly at
// the end.  Pass 1 writes C' in the split layout pass 2 stages.  Results sit in the matrix-core output layout
// (lane: level, block row, four columns), so the epilogues need no LDS: the
// per-pixel sums over levels are reduced across the 16 level lanes once per
// tile.
#pragma once
#include "bilateral_mfma16.h"

namespace stereo {
namespace bilh {

// Per-launch arguments of a backward pass; v describes the split-FP16
// input volume (v.D = levels of the tile) and the FP32 guide.
struct BView {
  View v;
  float* out;             // pass 2: dC planar [D][H][W]
  uint16_t* h2out;        // pass 1: C' S, split-FP16 volume (pitch and plane of v)
  const float* cpix;      // pass 2: C planar [D][H][W]
  const unsigned int* gmax;  // max |g'| over the image (float bits), for the scale S
  const float* sm_m;
  const float* sm_logZ;
  const float* sm_dh;
  const float* gD;
  float* aP;
  float* A1;
  float* A2;
  float* Wp;              // pass 1, nullable: sum_q w(p, q)
  float invT, one_minus_c1;
  int d_first;            // level of the tile's first slice
  int d_all;              // levels of the whole range (the bound on |d - dh|)
};

// Power-of-two scale that puts a bound m on |C'| in [2^13, 2^14) (bits: m
// as a float): FP16 keeps its range for every value up to the bound.
__host__ __device__ inline float cprime_scale(unsigned int bits) {
  const int ex = (int)((bits >> 23) & 0xFF);
  if (ex == 0xFF || bits == 0) return 1.0f;          // non-finite or zero: no scaling
  int e = ex - 126;                                   // max = f 2^e, f in [0.5, 1)
  if (e < -80) e = -80;
  int k = 14 - e;                                     // scale 2^k, |k| <= 94
  float s = 1.0f;
  const float step = k >= 0 ? 2.0f : 0.5f;
  for (int n = k >= 0 ? k : -k; n > 0; --n) s *= step;
  return s;
}

// One level block of a tile, [16 levels][kTH rows][kTW columns] floats: pass
// 2 stages the costs at the tile's pixels in it and collects its outputs in
// two more, so that both move between HBM and LDS in whole 64-byte rows.
constexpr int kTileBlk = 16 * kTH * kTW;
template <int R, int PASS>
constexpr size_t bwd_lds_bytes() {
  return HGeom<R>::lds_bytes + (PASS == 2 ? sizeof(float) * 2 * kTileBlk : 0);
}

template <int R, int PASS>
__global__ void __launch_bounds__(kThreads, 1) agg_mfma16_bwd_kernel(BView b) {
  using G = HGeom<R>;
  constexpr int NI = G::NI;
  extern __shared__ float lds[];
  const View& one = b.v;
  float* const buf0 = lds;
  float* const buf1 = lds + G::BUF;
  float* const gbuf0 = lds + 2 * G::BUF;
  float* const gbuf1 = gbuf0 + G::GUIDE;
  float* const scr = gbuf1 + G::GUIDE;
  float* const stab = scr + G::SCR;
  float* const tout = stab + G::STAB;             // pass 2: two output blocks
  static_assert(G::kTable, "the backward keeps the spatial terms in LDS");
  static_assert(bwd_lds_bytes<R, PASS>() <= 160 * 1024, "LDS budget");
  static_assert(kTileBlk + kWaves * 32 <= G::SCR, "pass 2's cost block and sums fit the scratch");
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int by = wave >> 2, bx = wave & 3;
  const int li = lane & 15, lk = lane >> 4;
  const int pr = li >> 2, pc = li & 3;

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
  auto patch_off = [&](int i) -> int {
    unsigned pk = poff[i >> 2];
    asm volatile("" : "+v"(pk));
    return (int)((pk >> (8 * (i & 3))) & 0xFFu);
  };
  int coff[G::KPW];
  if constexpr (G::CPR != 64) {
#pragma unroll
    for (int m = 0; m < G::KPW; ++m) {
      const int c = (wave + kWaves * m) * 64 + lane;
      const int pr2 = c / (G::HY * G::CPR);
      const int w = c - pr2 * (G::HY * G::CPR);
      const int row = w / G::CPR;
      const int cr = w - row * G::CPR;
      coff[m] = c < G::NCH ? (int)(pr2 * one.plane + row * 16 * (int64_t)one.pitch) + 8 * cr : -1;
    }
  }
  if (wave == 0) {
#pragma unroll 1
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int p = 4 * i + lk;
        const int rp = p / G::NCQ, cq = p - rp * G::NCQ;
        const int ty = 2 * rp + (s >> 2) - pr - R, tx = 4 * cq + (s & 3) - pc - R;
        const bool in = p < G::NP && ty >= -R && ty <= R && tx >= -R && tx <= R;
        stab[(i * 64 + lane) * 8 + s] =
            in ? fmaf(-(float)(ty * ty + tx * tx), one.ks2, kLog2WScale) : -__builtin_inff();
      }
  }

  // tiles: XCD x walks the tile columns of band x row by row (as the forward)
  const int tx = __builtin_amdgcn_readfirstlane((one.W + kTW - 1) / kTW);
  const int n1 = __builtin_amdgcn_readfirstlane(tx * ((one.H + kTH - 1) / kTH));
  int per = 0, c0 = 0, bc = 1, nb = 0;
  if (gridDim.x % 8 == 0) {
    per = gridDim.x / 8;
    const int bw = (tx + 7) / 8;
    c0 = (blockIdx.x % 8) * bw;
    bc = tx - c0 < bw ? (tx - c0 > 0 ? tx - c0 : 0) : bw;
    nb = bc * (n1 / tx);
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
  auto origin = [&](int t, int& x0, int& y0) {
    const int ty = __builtin_amdgcn_readfirstlane(t / tx);
    x0 = (t - ty * tx) * kTW;
    y0 = ty * kTH;
  };

  const int nl = one.D;
  const int passes = (nl + 15) / 16;
  // C' scale (pass 2: removed from both sums with the weights' 2^12)
  const float bound = __uint_as_float(*b.gmax) * fabsf(b.one_minus_c1) * b.invT *
                      (float)(b.d_all > 1 ? b.d_all - 1 : 1);
  const float cscale = cprime_scale(__float_as_uint(bound));
  const float unscale = PASS == 2 ? 1.0f / (4096.0f * cscale) : 1.0f / 4096.0f;
  const float inv_kr = 1.0f / sqrtf(one.kr2);

  int cur = arith_tile(0);
  if (cur >= n1) return;                         // uniform
  {
    int cx0, cy0;
    origin(cur, cx0, cy0);
    GuideRaw<R, float> g;
    stage<R>(one, cx0, cy0, 0, buf0, wave, lane, coff, true);
    guide_load<R, float>(one, cx0, cy0, g);
    guide_store<R, float>(gbuf0, g, one, cx0, cy0);
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();

  int par = 0, gpar = 0, gpass = 0;
  for (int k = 0;; ++k) {
    int x0, y0;
    origin(cur, x0, y0);
    // the two weight operands of this wave's block, split in FP16 halves
    u4 wh[NI], wl[NI], gh[NI], gl[NI];
    float wsum = 0.0f;
    {
      const float* gs = gpar ? gbuf1 : gbuf0;
      const float Gp = gs[(4 * by + pr + R) * G::GS + 4 * bx + pc + R];
#pragma unroll
      for (int i = 0; i < NI; ++i) {
        const float* gp = gs + 4 * patch_off(i);
        const float4 g0 = *reinterpret_cast<const float4*>(gp);
        const float4 g1 = *reinterpret_cast<const float4*>(gp + G::GS);
        int to = (i * 64 + lane) * 8;
        asm volatile("" : "+v"(to));
        const float4 s0 = *reinterpret_cast<const float4*>(stab + to);
        const float4 s1 = *reinterpret_cast<const float4*>(stab + to + 4);
        const float sv[8] = {s0.x, s0.y, s0.z, s0.w, s1.x, s1.y, s1.z, s1.w};
        const float gq[8] = {g0.x, g0.y, g0.z, g0.w, g1.x, g1.y, g1.z, g1.w};
        float w[8], wg[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const float g = Gp - gq[q];
          w[q] = __builtin_amdgcn_exp2f(fmaf(-g, g, sv[q]));
          wg[q] = w[q] * g;
        }
        split8(w, wh[i], wl[i]);
        split8(wg, gh[i], gl[i]);
        if constexpr (PASS == 1) {
          const h8 a = __builtin_bit_cast(h8, wh[i]), c = __builtin_bit_cast(h8, wl[i]);
#pragma unroll
          for (int q = 0; q < 8; ++q) wsum += (float)a[q] + (float)c[q];
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    // this lane's four output pixels: row lk, columns 0..3 of the block
    const int py = y0 + 4 * by + lk;
    const int px0 = x0 + 4 * bx;
    // The wave's LDS scratch.  Pass 1: [value][pixel] = m, log Z, g', dh (one
    // direct-to-LDS copy, lane j: value j / 16 of pixel j % 16), 1 / W_p,
    // W_p, then the two per-pixel sums over levels.  Pass 2: the pass's costs
    // at the wave's 16 pixels, [block row][level][column], then the sum.
    float* const sc = scr + wave * (16 * 20);
    float* const sums = PASS == 1 ? sc + 96 : sc + 256;
    if constexpr (PASS == 1) {
      {
        const int m = lane & 15, which = lane >> 4;
        int qy = y0 + 4 * by + (m >> 2), qx = x0 + 4 * bx + (m & 3);
        qy = qy < one.H ? qy : one.H - 1;                // clamped; masked in the epilogue
        qx = qx < one.W ? qx : one.W - 1;
        const float* src = which == 0 ? b.sm_m : which == 1 ? b.sm_logZ : which == 2 ? b.gD : b.sm_dh;
        __builtin_amdgcn_global_load_lds((BILM_GLOBAL void*)(src + (int64_t)qy * one.W + qx),
                                         (BILM_LOCAL void*)sc, 4, 0, 0);
      }
      // W_p of pixel li: its slots are spread over the lanes lk
      float wsP = wsum;
      wsP += __shfl_xor(wsP, 16);
      wsP += __shfl_xor(wsP, 32);
      if (lk == 0) {
        sc[64 + li] = 1.0f / wsP;
        sc[80 + li] = wsP;
      }
    }
    if (lane < 32) sums[lane] = 0.0f;
    // no barrier here: the weights read only this tile's guide (complete since
    // the last pass's barrier) and the spatial table
    const int nxt = arith_tile(k + 1);
    const bool has_next = nxt < n1;
    int nx0 = 0, ny0 = 0;
    if (has_next) origin(nxt, nx0, ny0);

    // the flat element f = 64 t + lane of this wave's share of a level block
    // (4 per lane): level, tile row, tile column
    auto blk_elem = [&](int t, int& l, int& row, int& col) {
      int ln = lane;
      asm volatile("" : "+v"(ln));                // recomputed per use, not kept live
      const int f = (wave * 4 + t) * 64 + ln;
      l = f / (kTH * kTW);
      const int rem = f - l * (kTH * kTW);
      row = rem / kTW;
      col = rem - row * kTW;
    };
    // a pass's outputs leave at the start of the next pass (or after the
    // last): issued before the copies, they have a pass to complete before
    // the wait at its end instead of holding it up
    float ov[4] = {0.f, 0.f, 0.f, 0.f};
    int oaddr = -1;                               // pass 1: the lane's (level, row) in C' S
    int opass = -1;                               // pass 2: level block held in tout
    int obuf_sel = 0;                             //   and which of the two
    auto flush = [&]() {
      if constexpr (PASS == 1) {
        // level li of stored columns x + R (x = px0 + v), both halves; a
        // column quad of the layout straddles two of the block's columns
        // unless R is a multiple of 4, so the halves go out one by one
        if (oaddr >= 0) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            if (px0 + v < one.W) {
              const int sc = px0 + v + R;
              const int o = oaddr + 64 * (sc >> 2) + (sc & 3);
              const _Float16 hi = (_Float16)ov[v];
              const _Float16 lo = (_Float16)(ov[v] - (float)hi);
              b.h2out[o] = __builtin_bit_cast(uint16_t, hi);
              b.h2out[o + (int)one.plane] = __builtin_bit_cast(uint16_t, lo);
            }
          }
        }
      } else {
        if (opass >= 0) {
          const float* to = tout + obuf_sel * kTileBlk;
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            int l, row, col;
            blk_elem(t, l, row, col);
            const int d = 16 * opass + l, gy = y0 + row, gx = x0 + col;
            if (d < nl && gy < one.H && gx < one.W)
              b.out[((int64_t)d * one.H + gy) * one.W + gx] = to[(l * kTH + row) * kTW + col];
          }
        }
      }
    };
    for (int p = 0; p < passes; ++p) {
      // the two slab buffers as __restrict__ parameters: the products need
      // not wait for the copies into the other buffer
      auto pass_body = [&](float* __restrict__ cbuf, float* __restrict__ obuf) {
      const int d0 = 16 * p;
      const bool last = p + 1 == passes;
      flush();
      GuideRaw<R, float> gq;
      if (!last || has_next) {
        stage<R>(one, last ? nx0 : x0, last ? ny0 : y0, last ? 0 : d0 + 16, obuf, wave, lane,
                 coff, true);
        if (last) guide_load<R, float>(one, nx0, ny0, gq);
      }
      if constexpr (PASS == 2) {
        // this pass's costs at the wave's pixels into its scratch: copy t is
        // block row t, lane j level j / 4, column j % 4 (runs of 16 bytes);
        // clamped addresses, values outside the tile's range are unused
        int ln = lane;
        asm volatile("" : "+v"(ln));
        int d = d0 + (ln >> 2), gx = px0 + (ln & 3);
        d = d < nl ? d : nl - 1;
        gx = gx < one.W ? gx : one.W - 1;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          int gy = y0 + 4 * by + t;
          gy = gy < one.H ? gy : one.H - 1;
          __builtin_amdgcn_global_load_lds(
              (BILM_GLOBAL void*)(b.cpix + ((int64_t)d * one.H + gy) * one.W + gx),
              (BILM_LOCAL void*)(sc + 64 * t), 4, 0, 0);
        }
      }
      const char* cb = reinterpret_cast<const char*>(cbuf);
      f4 aw = {0.f, 0.f, 0.f, 0.f}, ag = {0.f, 0.f, 0.f, 0.f};
      // one operand buffer per part: the low part's two products run first,
      // so the next low part is read while the high part's four run
      u4 bh, bl;
      auto load_h = [&](int i) {
        const char* a = cb + lbase + 128 * patch_off(i);
        const uint2 h0 = *reinterpret_cast<const uint2*>(a);
        const uint2 h1 = *reinterpret_cast<const uint2*>(a + G::ROWB);
        bh = u4{h0.x, h0.y, h1.x, h1.y};
      };
      auto load_l = [&](int i) {
        const char* a = cb + lbase + 128 * patch_off(i) + G::PARTB;
        const uint2 l0 = *reinterpret_cast<const uint2*>(a);
        const uint2 l1 = *reinterpret_cast<const uint2*>(a + G::ROWB);
        bl = u4{l0.x, l0.y, l1.x, l1.y};
      };
      __builtin_amdgcn_sched_barrier(0);
      load_l(0);
      load_h(0);
#pragma unroll
      for (int i = 0; i < NI; ++i) {
        const h8 aH = __builtin_bit_cast(h8, wh[i]), aL = __builtin_bit_cast(h8, wl[i]);
        const h8 cH = __builtin_bit_cast(h8, gh[i]), cL = __builtin_bit_cast(h8, gl[i]);
        const h8 bL = __builtin_bit_cast(h8, bl);
        aw = __builtin_amdgcn_mfma_f32_16x16x32_f16(aH, bL, aw, 0, 0, 0);
        ag = __builtin_amdgcn_mfma_f32_16x16x32_f16(cH, bL, ag, 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
        if (i + 1 < NI) load_l(i + 1);
        __builtin_amdgcn_sched_barrier(0);
        const h8 bH = __builtin_bit_cast(h8, bh);
        aw = __builtin_amdgcn_mfma_f32_16x16x32_f16(aH, bH, aw, 0, 0, 0);
        ag = __builtin_amdgcn_mfma_f32_16x16x32_f16(cH, bH, ag, 0, 0, 0);
        aw = __builtin_amdgcn_mfma_f32_16x16x32_f16(aL, bH, aw, 0, 0, 0);
        ag = __builtin_amdgcn_mfma_f32_16x16x32_f16(cL, bH, ag, 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
        if (i + 1 < NI) load_h(i + 1);
        __builtin_amdgcn_sched_barrier(0);
      }
      // the copies into the scratch (issued before the products) are complete
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      // lane: level d0 + li of pixels (row lk, columns v)
      const int d = d0 + li;
      const bool dv = d < nl;
      const bool rowin = py < one.H;
      int so = 4 * lk;
      asm volatile("" : "+v"(so));                 // read here, not hoisted
      float ca[4], cb2[4];
      if constexpr (PASS == 1) {
        const float gscale = b.one_minus_c1 * (-b.invT);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const bool in = dv && rowin && px0 + v < one.W;
          const float rinv = sc[64 + so + v];
          const float e = aw[v] * rinv;
          const float P = __builtin_amdgcn_exp2f(
              fmaf(-e, b.invT, -(sc[so + v] + sc[16 + so + v])) * 1.4426950408889634f);
          const float dE =
              in ? sc[32 + so + v] * gscale * P * ((float)(b.d_first + d) - sc[48 + so + v]) : 0.0f;
          ov[v] = dE * rinv * (4096.0f * cscale);   // S dE / W_p (rinv carries the 2^-12)
          ca[v] = dE * e;
          cb2[v] = dE * ag[v];
        }
        // offsets below 2^31: at most 64 levels (4 blocks) of one tile
        oaddr = rowin && px0 < one.W ? (int)((2 * p) * one.plane) + py * 16 * one.pitch + 4 * li
                                     : -1;
      } else {
        // the costs at (level li, block row lk, columns v); the outputs into
        // the tile's output block at (level li, tile row 4 by + lk, columns 4 bx + v)
        int co = 64 * lk + 4 * li;
        asm volatile("" : "+v"(co));
        const float4 c4 = *reinterpret_cast<const float4*>(sc + co);
        const int bo = (li * kTH + 4 * by + lk) * kTW + 4 * bx;
        const float cv[4] = {c4.x, c4.y, c4.z, c4.w};
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const bool in = dv && rowin && px0 + v < one.W;
          ov[v] = aw[v] * unscale;
          ca[v] = 0.0f;
          cb2[v] = in ? cv[v] * ag[v] : 0.0f;
        }
        // output blocks alternate with every pass of the launch (not of the
        // tile), so a block is rewritten only after the barrier that follows
        // its last read
        *reinterpret_cast<float4*>(tout + (gpass & 1) * kTileBlk + bo) =
            make_float4(ov[0], ov[1], ov[2], ov[3]);
        opass = p;
        obuf_sel = gpass & 1;
      }
      // this pass's per-pixel sums over its 16 levels (lanes li), added to the
      // wave's running sums by the lanes li = 0
#pragma unroll
      for (int v = 0; v < 4; ++v) {
#pragma unroll
        for (int m = 1; m < 16; m <<= 1) {
          if constexpr (PASS == 1) ca[v] += __shfl_xor(ca[v], m);
          cb2[v] += __shfl_xor(cb2[v], m);
        }
      }
      if (li == 0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if constexpr (PASS == 1) sums[so + v] += ca[v];
          sums[16 + so + v] += cb2[v];
        }
      }
      if (last && has_next) guide_store<R, float>(gpar ? gbuf0 : gbuf1, gq, one, nx0, ny0);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
      };
      pass_body(par ? buf1 : buf0, par ? buf0 : buf1);
      par ^= 1;
      ++gpass;
    }
    flush();
    // one lane per pixel adds this launch's sum (atomic adds without a return
    // value: no wait; one add per pixel and launch, so the order is fixed)
    if (li == 0 && py < one.H) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int px = px0 + v;
        if (px < one.W) {
          const int64_t pix = (int64_t)py * one.W + px;
          const float sbv = sums[16 + 4 * lk + v];
          if constexpr (PASS == 1) {
            atomicAdd(b.aP + pix, sums[4 * lk + v]);
            atomicAdd(b.A1 + pix, sbv * unscale * inv_kr);
            if (b.Wp) b.Wp[pix] = sc[80 + 4 * lk + v] * (1.0f / 4096.0f);
          } else {
            atomicAdd(b.A2 + pix, -sbv * unscale * inv_kr);
          }
        }
      }
    }
    if (!has_next) break;
    cur = nxt;
    gpar ^= 1;
  }
}

inline BView make_bview(const bil::BilPair& bp, const BilArgs& a) {
  BView b{};
  b.v = view_of(bp);
  b.out = a.E;
  b.cpix = a.cpix;
  b.gmax = a.gmax;
  b.h2out = a.h2_out;
  b.sm_m = a.sm_m;
  b.sm_logZ = a.sm_logZ;
  b.sm_dh = a.sm_dh;
  b.gD = a.gD;
  b.aP = a.aP;
  b.A1 = a.A1;
  b.A2 = a.A2;
  b.Wp = a.Wp;
  b.invT = bp.o.invT;
  b.one_minus_c1 = bp.o.one_minus_c1;
  b.d_first = a.d_first;
  return b;
}

template <int R, int PASS>
hipError_t launch_bwd_pass(const BView& b, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)agg_mfma16_bwd_kernel<R, PASS>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)bwd_lds_bytes<R, PASS>());
    if (e != hipSuccess) return e;
    attr = true;
  }
  const int n = ((b.v.W + kTW - 1) / kTW) * ((b.v.H + kTH - 1) / kTH);
  const int cus = bilm::cu_count_of_current_device();
  int grid = std::min(n, cus > 0 ? cus : 256);
  if (grid >= 8) grid -= grid % 8;
  constexpr size_t lds = bwd_lds_bytes<R, PASS>();
  hipLaunchKernelGGL((agg_mfma16_bwd_kernel<R, PASS>), dim3(grid), dim3(kThreads), lds, s, b);
  return hipGetLastError();
}

// Pass 1 or 2 of the backward for one level tile at radius R (float guide).
template <int R>
hipError_t launch_bwd_args(const Plan& P, const BilArgs& a, int pass, hipStream_t s) {
  const bil::BilPair bp = bil::make_pair(P, a);
  if (!a.h2 || a.h2_pitch < h2_pitch_for<R>(bp.W) || (a.h2_pitch & 7) || !a.gmax ||
      (pass == 1 && !a.h2_out) || (pass == 2 && (!a.cpix || !a.E)))
    return hipErrorInvalidValue;
  BView b = make_bview(bp, a);
  b.d_all = P.D;
  return pass == 1 ? launch_bwd_pass<R, 1>(b, s) : launch_bwd_pass<R, 2>(b, s);
}

}  // namespace bilh
}  // namespace stereo
