// Adjoint kernels of the differentiable form: soft-argmin head, bilateral
// aggregation (Eqs. 10-11), NCC cost (Eq. 8), perspective warp (Eq. 4), and
// the photometric L1 loss.
//
// Determinism: every gradient is either a gather in a fixed order or a sum of
// fixed-point integers (for the two true scatters, the warp and the loss
// sampling of the target image), so results do not depend on scheduling.
//
// Domains (x = column, y = row, all row-major):
//   image            [H][W]
//   virtual X domain [H + 2r][W + 2r], position (y + r, x + r) for y, x in
//                    [-r, H + r) x [-r, W + r): every place a reference block
//                    element can be read from before clamping
//   virtual Y domain [H + 2r][W + D - 1 + 2r], columns [-(D-1) - r, W + r):
//                    every place a warped-target block element can be read
//                    from (blocks centred down to column -(D-1))
// Block reads clamp, so a gradient that lands on a virtual position belongs
// to the clamped image pixel; the fold kernel adds it there.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace stereo {
namespace grad {

constexpr double kFix = 17592186044416.0;   // 2^44: fixed-point scale
constexpr int kT = 256;

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

template <typename T>
__device__ __forceinline__ float ldf(const T* p) { return static_cast<float>(*p); }

__device__ __forceinline__ void fix_add(unsigned long long* dst, double v) {
  atomicAdd(dst, (unsigned long long)(long long)llrint(v * kFix));
}

// After all tiles: B1(x) = sum_q w (G(x) - G(q)), B2(x) = sum_q w (G(q) - G(x)) a_q / W_q,
// dG(x) = 2/sigma_r^2 [ -(A1 - a_x B1) / W_x + (A2 - B2) ];  out = gX + dG.
// A workgroup covers GF_TX x GF_TY pixels; the guide and a_q / W_q of the
// tile and its R-halo (R <= 8) are staged in LDS once, the taps read them
// there (same expressions, same tap order as a per-pixel gather).
constexpr int GF_TX = 32, GF_TY = 8, GF_RMAX = 8;
template <typename GT>
__global__ void __launch_bounds__(kT)
guide_finish_kernel(const GT* __restrict__ g, int64_t gpitch, const float* __restrict__ Wp,
                    const float* __restrict__ aP, const float* __restrict__ A1,
                    const float* __restrict__ A2, const float* __restrict__ gX, int W, int H,
                    int R, float ks2, float kr2, float two_over_sr2,
                    float* __restrict__ out) {
  __shared__ float gs[(GF_TY + 2 * GF_RMAX) * (GF_TX + 2 * GF_RMAX)];
  __shared__ float rs[(GF_TY + 2 * GF_RMAX) * (GF_TX + 2 * GF_RMAX)];
  const int HWD = GF_TX + 2 * R, HHT = GF_TY + 2 * R;
  const int x0 = blockIdx.x * GF_TX, y0 = blockIdx.y * GF_TY;
  for (int i = threadIdx.x; i < HWD * HHT; i += kT) {
    const int yy = i / HWD, xx = i - yy * HWD;
    const int qy = y0 - R + yy, qx = x0 - R + xx;
    const bool in = qy >= 0 && qy < H && qx >= 0 && qx < W;
    const int64_t q = (int64_t)qy * W + qx;
    gs[i] = in ? ldf(g + (int64_t)qy * gpitch + qx) : 0.0f;
    rs[i] = in ? aP[q] / Wp[q] : 0.0f;
  }
  __syncthreads();
  const int tx = threadIdx.x % GF_TX, ty = threadIdx.x / GF_TX;
  const int x = x0 + tx, y = y0 + ty;
  if (x >= W || y >= H) return;
  const int64_t p = (int64_t)y * W + x;
  const float gx = gs[(ty + R) * HWD + tx + R];
  float b1 = 0.0f, b2 = 0.0f;
  for (int dy = -R; dy <= R; ++dy) {
    const int qy = y + dy;
    if (qy < 0 || qy >= H) continue;
    const int rowo = (ty + R + dy) * HWD + tx + R;
    for (int dx = -R; dx <= R; ++dx) {
      const int qx = x + dx;
      if (qx < 0 || qx >= W) continue;
      const float dg = gx - gs[rowo + dx];
      const float w = __builtin_amdgcn_exp2f(-(float)(dx * dx + dy * dy) * ks2 - dg * dg * kr2);
      b1 = fmaf(w, dg, b1);
      b2 = fmaf(-w * dg, rs[rowo + dx], b2);
    }
  }
  const float dG = two_over_sr2 * (-(A1[p] - aP[p] * b1) / Wp[p] + (A2[p] - b2));
  out[p] = gX[p] + dG;
}

// ---------------------------------------------------------------------------
// NCC adjoint coefficients for one level tile.  With A = -dC/n (0 for flat
// blocks), rho = 1 - C, offset intensities (I - 128) and their block means:
//   alpha = A isX isY, beta = A rho isX^2, gamma = A rho isY^2,
// the gradient of the reference block element i is
//   alpha (Y_i - muY) - beta (X_i - muX),
// and of the target block element  alpha (X_i - muX) - gamma (Y_i - muY).
// Per level map: alpha; per reference pixel sums over levels (all tiles):
// beta, beta muX, alpha muY.
// Target side: the target block of pixel x at level d is centred at column
// m = x - d, so its level sums are maps over m in [-(D-1), W):
//   SaX(m) += sum_d alpha(m+d, d) muX(m+d),  Sg(m) += sum_d gamma(m+d, d),
//   SgY(m) += sum_d gamma(m+d, d) muY(m),
// maps [H][W + D - 1] at column index m + D - 1.
// Two passes per tile: the coefficients and reference-side sums by pixel,
// then the target-side sums along the diagonals (the second pass re-reads C
// and dC; one fused pass with the diagonals exchanged through LDS, or read
// through the caches, measured slower).
// max |g| over n values into *out (float bits; non-negative floats order as
// their bits), one atomic per workgroup (atomics on one address serialise);
// *out is zeroed before the launch.  Four independent loads per thread and
// round.
__global__ void __launch_bounds__(256) absmax_kernel(const float* __restrict__ g, int64_t n,
                                                     unsigned int* __restrict__ out) {
  __shared__ float wm[4];
  float m = 0.0f;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i0 = (int64_t)blockIdx.x * 256 + threadIdx.x; i0 < n; i0 += 4 * stride) {
    float v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t i = i0 + k * stride;
      v[k] = i < n ? fabsf(g[i]) : 0.0f;
    }
    m = fmaxf(m, fmaxf(fmaxf(v[0], v[1]), fmaxf(v[2], v[3])));
  }
#pragma unroll
  for (int k = 1; k < 64; k <<= 1) m = fmaxf(m, __shfl_xor(m, k));
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = fmaxf(fmaxf(wm[0], wm[1]), fmaxf(wm[2], wm[3]));
    if (m > 0.0f) atomicMax(out, __float_as_uint(m));
  }
}

// Both passes read the levels of a thread in chunks of NA_CH: every load of
// a chunk is issued (unconditionally; the flat-block rule selects after the
// load) before the first use, so a thread waits once per chunk.
constexpr int NA_CH = 8;

__global__ void __launch_bounds__(kT)
ncc_coef_kernel(const float* __restrict__ Ct, const float* __restrict__ gCt,
                const float* __restrict__ muX, const float* __restrict__ isdX,
                const float* __restrict__ muY, const float* __restrict__ isdY, int W, int H,
                int r, int d_first, int nlev, float inv_n, float* __restrict__ Fa,
                float* __restrict__ Sb, float* __restrict__ SbmX, float* __restrict__ SamY) {
  const int x = blockIdx.x * kT + threadIdx.x, y = blockIdx.y;
  if (x >= W) return;
  const int64_t HW = (int64_t)W * H;
  const int64_t p = (int64_t)y * W + x;
  const int SW = W + 2 * r;
  const int64_t ro = (int64_t)y * SW;
  const float iX = isdX[ro + x + r];
  const float mX = muX[ro + x + r];
  float sb = Sb[p], sbm = SbmX[p], sam = SamY[p];
  for (int t0 = 0; t0 < nlev; t0 += NA_CH) {
    float iY[NA_CH], mY[NA_CH], g[NA_CH], c[NA_CH];
#pragma unroll
    for (int k = 0; k < NA_CH; ++k) {
      const int t = min(t0 + k, nlev - 1);
      const int cy = max(x - (d_first + t), -r) + r;
      iY[k] = isdY[ro + cy];
      mY[k] = muY[ro + cy];
      g[k] = gCt[t * HW + p];
      c[k] = Ct[t * HW + p];
    }
#pragma unroll
    for (int k = 0; k < NA_CH; ++k) {
      const int t = t0 + k;
      const bool ok = t < nlev;
      const bool flat = (iX == 0.0f) || (iY[k] == 0.0f);
      const float A = flat ? 0.0f : -g[k] * inv_n;
      const float rho = 1.0f - c[k];
      const float al = A * iX * iY[k];
      const float be = A * rho * iX * iX;
      sb = ok ? sb + be : sb;
      sbm = ok ? fmaf(be, mX, sbm) : sbm;
      sam = ok ? fmaf(al, mY[k], sam) : sam;
      if (ok) Fa[t * HW + p] = al;
    }
  }
  Sb[p] = sb;
  SbmX[p] = sbm;
  SamY[p] = sam;
}

__global__ void __launch_bounds__(kT)
ncc_shear_kernel(const float* __restrict__ Ct, const float* __restrict__ gCt,
                 const float* __restrict__ muX, const float* __restrict__ isdX,
                 const float* __restrict__ muY, const float* __restrict__ isdY, int W, int H,
                 int D, int r, int d_first, int nlev, float inv_n, float* __restrict__ SaX,
                 float* __restrict__ Sg, float* __restrict__ SgY) {
  const int WY = W + D - 1;
  const int mi = blockIdx.x * kT + threadIdx.x, y = blockIdx.y;
  if (mi >= WY) return;
  const int m = mi - (D - 1);
  const int64_t HW = (int64_t)W * H;
  const int SW = W + 2 * r;
  const int64_t ro = (int64_t)y * SW;
  const int cy = max(m, -r) + r;
  const float iY = isdY[ro + cy];
  const float mY = muY[ro + cy];
  const int64_t q = (int64_t)y * WY + mi;
  float sax = SaX[q], sg = Sg[q];
  // clamped columns, results selected
  for (int t0 = 0; t0 < nlev; t0 += NA_CH) {
    float iX[NA_CH], mX[NA_CH], g[NA_CH], c[NA_CH];
#pragma unroll
    for (int k = 0; k < NA_CH; ++k) {
      const int t = min(t0 + k, nlev - 1);
      const int xc = min(max(m + d_first + t, 0), W - 1);
      const int64_t p = (int64_t)y * W + xc;
      iX[k] = isdX[ro + xc + r];
      mX[k] = muX[ro + xc + r];
      g[k] = gCt[t * HW + p];
      c[k] = Ct[t * HW + p];
    }
#pragma unroll
    for (int k = 0; k < NA_CH; ++k) {
      const int t = t0 + k;
      const int x = m + d_first + t;
      const bool ok = t < nlev && x >= 0 && x < W;
      const bool flat = (iX[k] == 0.0f) || (iY == 0.0f);
      const float A = flat ? 0.0f : -g[k] * inv_n;
      const float rho = 1.0f - c[k];
      sax = ok ? fmaf(A * iX[k] * iY, mX[k], sax) : sax;
      sg = ok ? fmaf(A * rho, iY * iY, sg) : sg;
    }
  }
  SaX[q] = sax;
  Sg[q] = sg;
  SgY[q] = sg * mY;
}

// ncc_coef and ncc_shear in one pass (level tiles of at most 64 levels): a
// wave covers pixels x = 64 bx + lane of row y, reads C and dC once, writes
// alpha and the per-pixel sums as ncc_coef does, and forms the target-side
// sums of column m = x - d along the diagonals: the partial sums of SaX and Sg
// move one lane up per level (DPP wave shift; the one leaving lane 63 is
// complete), so that local index U holds column m = 64 bx - d_first -
// (nlev - 1) + U.  U >= nlev - 1 are this wave's own columns (added to the
// maps); U < nlev - 1 also take levels of the next wave's pixels and go to
// spill[y][bx][U][2] for ncc_adjoint_merge_kernel (one spill per column,
// fixed order).  Products and their order per term are those of the two
// separate passes.
__device__ __forceinline__ float wave_shr1(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
      0, __builtin_bit_cast(int, v), 0x138 /* wave_shr:1 */, 0xF, 0xF, false));
}

__global__ void __launch_bounds__(64)
ncc_adjoint_kernel(const float* __restrict__ Ct, const float* __restrict__ gCt,
                   const float* __restrict__ muX, const float* __restrict__ isdX,
                   const float* __restrict__ muY, const float* __restrict__ isdY, int W, int H,
                   int D, int r, int d_first, int nlev, float inv_n, float* __restrict__ Fa,
                   float* __restrict__ Sb, float* __restrict__ SbmX, float* __restrict__ SamY,
                   float* __restrict__ SaX, float* __restrict__ Sg,
                   float* __restrict__ spill) {
  __shared__ float fin[2][128];
  const int lane = threadIdx.x, bx = blockIdx.x, y = blockIdx.y;
  const int x = 64 * bx + lane;
  const bool in = x < W;
  const int xc = min(x, W - 1);
  const int64_t HW = (int64_t)W * H;
  const int64_t p = (int64_t)y * W + xc;
  const int SW = W + 2 * r, WY = W + D - 1;
  const int64_t ro = (int64_t)y * SW;
  const float iX = isdX[ro + xc + r];
  const float mX = muX[ro + xc + r];
  float sb = Sb[p], sbm = SbmX[p], sam = SamY[p];
  float dax = 0.0f, dg = 0.0f;                      // diagonal partial sums
  for (int t0 = 0; t0 < nlev; t0 += NA_CH) {
    float iY[NA_CH], mY[NA_CH], g[NA_CH], c[NA_CH];
#pragma unroll
    for (int k = 0; k < NA_CH; ++k) {
      const int t = min(t0 + k, nlev - 1);
      const int cy = max(xc - (d_first + t), -r) + r;
      iY[k] = isdY[ro + cy];
      mY[k] = muY[ro + cy];
      g[k] = gCt[t * HW + p];
      c[k] = Ct[t * HW + p];
    }
#pragma unroll
    for (int k = 0; k < NA_CH; ++k) {
      const int t = t0 + k;
      if (t >= nlev) break;                         // uniform
      const bool flat = (iX == 0.0f) || (iY[k] == 0.0f);
      const float A = flat ? 0.0f : -g[k] * inv_n;
      const float rho = 1.0f - c[k];
      const float al = A * iX * iY[k];
      const float Ar = A * rho;
      const float be = Ar * iX * iX;
      sb = in ? sb + be : sb;
      sbm = in ? fmaf(be, mX, sbm) : sbm;
      sam = in ? fmaf(al, mY[k], sam) : sam;
      if (in) Fa[t * HW + p] = al;
      if (t > 0) {
        if (lane == 63) {                           // complete: no later level reaches it
          fin[0][63 + nlev - t] = dax;
          fin[1][63 + nlev - t] = dg;
        }
        dax = wave_shr1(dax);
        dg = wave_shr1(dg);
      }
      dax = in ? fmaf(al, mX, dax) : dax;
      dg = in ? fmaf(Ar, iY[k] * iY[k], dg) : dg;
    }
  }
  if (in) {
    Sb[p] = sb;
    SbmX[p] = sbm;
    SamY[p] = sam;
  }
  fin[0][lane] = dax;
  fin[1][lane] = dg;
  __syncthreads();
  const int mi = 64 * bx + lane - d_first + D - 1;  // own index U = lane + nlev - 1
  if (mi < WY) {
    const int64_t q = (int64_t)y * WY + mi;
    SaX[q] += fin[0][lane + nlev - 1];
    Sg[q] += fin[1][lane + nlev - 1];
  }
  if (lane < nlev - 1) {
    float* sp = spill + (((int64_t)y * gridDim.x + bx) * 64 + lane) * 2;
    sp[0] = fin[0][lane];
    sp[1] = fin[1][lane];
  }
}

// Adds the spills of ncc_adjoint_kernel (column m of local index U < nlev - 1
// of wave bx) and sets SgY = Sg muY for every column.
__global__ void __launch_bounds__(kT)
ncc_adjoint_merge_kernel(const float* __restrict__ spill, int nbx, int W, int D, int r,
                         int d_first, int nlev, const float* __restrict__ muY,
                         float* __restrict__ SaX, float* __restrict__ Sg,
                         float* __restrict__ SgY) {
  const int WY = W + D - 1;
  const int mi = blockIdx.x * kT + threadIdx.x, y = blockIdx.y;
  if (mi >= WY) return;
  const int m = mi - (D - 1);
  const int64_t q = (int64_t)y * WY + mi;
  float sg = Sg[q];
  const int u64 = m + d_first + nlev - 1;           // 64 bx + U
  if (u64 >= 0) {
    const int bx = u64 >> 6, u = u64 & 63;
    if (u < nlev - 1 && bx < nbx) {
      const float* sp = spill + (((int64_t)y * nbx + bx) * 64 + u) * 2;
      SaX[q] += sp[0];
      sg += sp[1];
      Sg[q] = sg;
    }
  }
  SgY[q] = sg * muY[(int64_t)y * (W + 2 * r) + max(m, -r) + r];
}

// Box sums onto a virtual domain: B(j) = sum_{o in [-r,r]^2} F(j - o) over
// image pixels j - o (F is [H][W], B is [H + 2r][W + 2r], virtual position j
// at index j + r).  A workgroup (BX_TX / 64 waves) covers BX_TX virtual
// columns x BX_TY virtual rows of one map: the (BX_TY + 2r) x (BX_TX + 2r)
// input tile, zero outside the image, is staged in LDS (clamped loads, all
// issued before the first LDS store); each lane walks down its column with
// a ring of 2r+1 horizontal sums (fixed order: horizontal j = -r..r, then
// vertical i = -r..r).  grid.z indexes the maps.
constexpr int BX_TX = 256, BX_TY = 32;

template <int r>
__global__ void __launch_bounds__(BX_TX)
box_kernel(const float* __restrict__ F, int W, int H, float* __restrict__ B) {
  constexpr int K = 2 * r + 1;
  constexpr int TWI = BX_TX + 2 * r, THI = BX_TY + 2 * r;
  __shared__ float tile[THI * TWI];
  const int WV = W + 2 * r, HV = H + 2 * r;
  const int64_t HW = (int64_t)W * H;
  const float* f = F + blockIdx.z * HW;
  float* b = B + (int64_t)blockIdx.z * HV * WV;
  const int vx0 = blockIdx.x * BX_TX - r;          // first virtual column (image coords)
  const int vy0 = blockIdx.y * BX_TY - r;          // first virtual row (image coords)
  const int ix0 = vx0 - r, iy0 = vy0 - r;          // first input column / row
  constexpr int NL = (THI * TWI + BX_TX - 1) / BX_TX;
  float v[NL];
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int i = min((int)threadIdx.x + BX_TX * k, THI * TWI - 1);
    const int yy = i / TWI, xx = i - yy * TWI;
    const int iy = iy0 + yy, ix = ix0 + xx;
    const bool in = iy >= 0 && iy < H && ix >= 0 && ix < W;
    const float val = f[(int64_t)clampi(iy, 0, H - 1) * W + clampi(ix, 0, W - 1)];
    v[k] = in ? val : 0.0f;
  }
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int i = threadIdx.x + BX_TX * k;
    if (i < THI * TWI) tile[i] = v[k];
  }
  __syncthreads();
  const int c = threadIdx.x;
  const int jx = vx0 + c;                          // this lane's virtual column
  float ring[K];
#pragma unroll
  for (int i = 0; i < K; ++i) ring[i] = 0.0f;
  for (int yb = 0; yb < THI; yb += K) {
#pragma unroll
    for (int s = 0; s < K; ++s) {
      const int yy = yb + s;
      if (yy >= THI) break;
      const float* trow = tile + yy * TWI + c;
      float h = trow[0];
#pragma unroll
      for (int j = 1; j < K; ++j) h += trow[j];
      ring[s] = h;
      const int oy = vy0 + yy - 2 * r;             // virtual row completed (image coords)
      if (yy >= 2 * r && oy < H + r && jx < W + r) {
        float S = ring[(s + 1) % K];
#pragma unroll
        for (int i = 2; i <= K; ++i) S += ring[(s + i) % K];
        b[(int64_t)(oy + r) * WV + (jx + r)] = S;
      }
    }
  }
}

// gXv(j) += sum_{d in tile} Yv(j - d) B_alpha,d(j)     (virtual X domain)
__global__ void __launch_bounds__(kT)
assemble_x_kernel(const float* __restrict__ Ba, const float* __restrict__ tarw, int W, int H,
                  int r, int d_first, int nlev, float* __restrict__ gXv) {
  const int WV = W + 2 * r, HV = H + 2 * r;
  const int vx = blockIdx.x * kT + threadIdx.x, vy = blockIdx.y;
  if (vx >= WV) return;
  const int y = clampi(vy - r, 0, H - 1);
  const int64_t jv = (int64_t)vy * WV + vx;
  const int64_t HVWV = (int64_t)HV * WV;
  float acc = 0.0f;
  #pragma unroll 4
  for (int t = 0; t < nlev; ++t) {
    const int xs = clampi(vx - r - (d_first + t), 0, W - 1);
    acc = fmaf(tarw[(int64_t)y * W + xs] - kOffset, Ba[t * HVWV + jv], acc);
  }
  gXv[jv] += acc;
}

// gYv(k) += sum_{d in tile} Xv(k+d) B_alpha,d(k+d) on the virtual Y domain;
// B at virtual X column k + d (zero outside it).
template <typename T>
__global__ void __launch_bounds__(kT)
assemble_y_kernel(const float* __restrict__ Ba, const T* __restrict__ ref, int64_t rpitch,
                  int W, int H, int D, int r, int d_first, int nlev, float* __restrict__ gYv) {
  const int WVX = W + 2 * r, HV = H + 2 * r, WVY = W + D - 1 + 2 * r;
  const int ky = blockIdx.x * kT + threadIdx.x, vy = blockIdx.y;   // ky: Y-domain column index
  if (ky >= WVY) return;
  const int kx = ky - (D - 1) - r;                                  // image column of k
  const int y = clampi(vy - r, 0, H - 1);
  const int64_t HVWV = (int64_t)HV * WVX;
  float acc = 0.0f;
  #pragma unroll 4
  for (int t = 0; t < nlev; ++t) {
    const int jx = kx + d_first + t;                                // virtual X column
    if (jx < -r || jx >= W + r) continue;
    const int64_t j = (int64_t)t * HVWV + (int64_t)vy * WVX + (jx + r);
    const float xv = ldf(ref + (int64_t)y * rpitch + clampi(jx, 0, W - 1)) - kOffset;
    acc = fmaf(xv, Ba[j], acc);
  }
  gYv[(int64_t)vy * WVY + ky] += acc;
}

// Both sides from one read of the boxes of alpha (levels d = d_first + t of
// one level tile, t < nlev <= 64):
//   gXv(j) += sum_t Yv(j - d) B_alpha,t(j)            (per virtual X column)
//   gYv(k) += sum_t Xv(k + d) B_alpha,t(k + d)        (along the diagonals)
// with the products and their order those of assemble_x / assemble_y.  A
// wave covers the virtual X columns j = 64 bx + lane of virtual row vy.  The
// target sum of local index U (Y-domain column 64 bx + D - 1 - d_first -
// (nlev - 1) + U) takes lane U - (nlev - 1 - t) at level t: the partial sums
// move one lane up per level (DPP wave shift), and the one leaving lane 63 is
// complete (kept in LDS).  Indices U >= nlev - 1 are this wave's own columns
// (added to gYv); U < nlev - 1 also take levels of the next wave's columns:
// they go to spill[vy][bx][U], which assemble_merge_kernel adds afterwards
// (one spill per column: deterministic).
constexpr int AS_CH = 8;

template <typename T>
__global__ void __launch_bounds__(64)
assemble_kernel(const float* __restrict__ Ba, const float* __restrict__ tarw,
                const T* __restrict__ ref, int64_t rpitch, int W, int H, int D, int r,
                int d_first, int nlev, float* __restrict__ gXv, float* __restrict__ gYv,
                float* __restrict__ spill) {
  __shared__ float fin[128];
  const int WV = W + 2 * r, HV = H + 2 * r, WVY = W + D - 1 + 2 * r;
  const int lane = threadIdx.x, bx = blockIdx.x, vy = blockIdx.y;
  const int vx = 64 * bx + lane;
  const bool in = vx < WV;
  const int64_t HVWV = (int64_t)HV * WV;
  const int y = clampi(vy - r, 0, H - 1);
  const float* trow = tarw + (int64_t)y * W;
  const float* brow = Ba + (int64_t)vy * WV + min(vx, WV - 1);
  const float xv = ldf(ref + (int64_t)y * rpitch + clampi(vx - r, 0, W - 1)) - kOffset;
  float ax = 0.0f, ay = 0.0f;
  for (int t0 = 0; t0 < nlev; t0 += AS_CH) {
    float b[AS_CH], yv[AS_CH];
#pragma unroll
    for (int k = 0; k < AS_CH; ++k) {
      const int t = min(t0 + k, nlev - 1);
      b[k] = brow[t * HVWV];
      yv[k] = trow[clampi(vx - r - (d_first + t), 0, W - 1)];
    }
#pragma unroll
    for (int k = 0; k < AS_CH; ++k) {
      const int t = t0 + k;
      if (t >= nlev) break;                         // uniform
      const float bb = in ? b[k] : 0.0f;
      ax = fmaf(yv[k] - kOffset, bb, ax);
      if (t > 0) {
        if (lane == 63) fin[63 + nlev - t] = ay;    // complete: no later level reaches it
        ay = __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
                 0, __builtin_bit_cast(int, ay), 0x138 /* wave_shr:1 */, 0xF, 0xF, false));
      }
      ay = fmaf(xv, bb, ay);
    }
  }
  fin[lane] = ay;
  __syncthreads();
  if (in) gXv[(int64_t)vy * WV + vx] += ax;
  const int ky = 64 * bx + lane + D - 1 - d_first;  // own index U = lane + nlev - 1
  if (ky < WVY) gYv[(int64_t)vy * WVY + ky] += fin[lane + nlev - 1];
  if (lane < nlev - 1) spill[((int64_t)vy * gridDim.x + bx) * 64 + lane] = fin[lane];
}

// gYv(k) += the spill of the wave whose local index U < nlev - 1 is k.
__global__ void __launch_bounds__(kT)
assemble_merge_kernel(const float* __restrict__ spill, int nbx, int W, int D, int r,
                      int d_first, int nlev, float* __restrict__ gYv) {
  const int WVY = W + D - 1 + 2 * r;
  const int ky = blockIdx.x * kT + threadIdx.x, vy = blockIdx.y;
  if (ky >= WVY) return;
  const int q = ky - (D - 1) + d_first + (nlev - 1);    // 64 bx + U
  if (q < 0) return;
  const int bx = q >> 6, u = q & 63;
  if (u >= nlev - 1 || bx >= nbx) return;
  gYv[(int64_t)vy * WVY + ky] += spill[((int64_t)vy * nbx + bx) * 64 + u];
}

// Target side terms summed over all levels (virtual Y domain):
//   gYv(k) += -B(SaX)(k) - Yv(k) B(Sg)(k) + B(SgY)(k)
__global__ void __launch_bounds__(kT)
y_complete_kernel(const float* __restrict__ BSaX, const float* __restrict__ BSg,
                  const float* __restrict__ BSgY, const float* __restrict__ tarw, int W, int H,
                  int D, int r, float* __restrict__ gYv) {
  const int WVY = W + D - 1 + 2 * r;
  const int ky = blockIdx.x * kT + threadIdx.x, vy = blockIdx.y;
  if (ky >= WVY) return;
  const int64_t k = (int64_t)vy * WVY + ky;
  const int kx = ky - (D - 1) - r;
  const float yv = tarw[(int64_t)clampi(vy - r, 0, H - 1) * W + clampi(kx, 0, W - 1)] - kOffset;
  gYv[k] += -BSaX[k] - yv * BSg[k] + BSgY[k];
}

// X side terms summed over all levels:
//   gXv(j) += -B(S alpha muY)(j) - Xv(j) B(S beta)(j) + B(S beta muX)(j)
template <typename T>
__global__ void __launch_bounds__(kT)
x_complete_kernel(const float* __restrict__ BSamY, const float* __restrict__ BSb,
                  const float* __restrict__ BSbmX, const T* __restrict__ ref, int64_t rpitch,
                  int W, int H, int r, float* __restrict__ gXv) {
  const int WV = W + 2 * r;
  const int vx = blockIdx.x * kT + threadIdx.x, vy = blockIdx.y;
  if (vx >= WV) return;
  const int64_t j = (int64_t)vy * WV + vx;
  const float xv = ldf(ref + (int64_t)clampi(vy - r, 0, H - 1) * rpitch + clampi(vx - r, 0, W - 1)) - kOffset;
  gXv[j] += -BSamY[j] - xv * BSb[j] + BSbmX[j];
}

// Fold a virtual domain back onto the image (clamped reads): pixel (x, y)
// receives every virtual position that clamps to it.  left = columns of
// padding on the left of the domain (r for X, D - 1 + r for Y).
__global__ void __launch_bounds__(kT)
fold_kernel(const float* __restrict__ gv, int W, int H, int r, int left,
            float* __restrict__ out) {
  const int x = blockIdx.x * kT + threadIdx.x, y = blockIdx.y;
  if (x >= W) return;
  const int WV = W + left + r;
  const int ylo = (y == 0) ? -r : y, yhi = (y == H - 1) ? H - 1 + r : y;
  const int xlo = (x == 0) ? -left : x, xhi = (x == W - 1) ? W - 1 + r : x;
  float s = 0.0f;
  for (int vy = ylo; vy <= yhi; ++vy)
    for (int vx = xlo; vx <= xhi; ++vx) s += gv[(int64_t)(vy + r) * WV + (vx + left)];
  out[(int64_t)y * W + x] = s;
}

// ---------------------------------------------------------------------------
// FP64 block reduction of three sums into partials[block][3].
__device__ void reduce3(double a, double b, double c, double* __restrict__ partials) {
  __shared__ double red[3][kT];
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  red[2][threadIdx.x] = c;
  __syncthreads();
  for (int s = kT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
      red[2][threadIdx.x] += red[2][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x < 3) {
    const int64_t b0 = (int64_t)(blockIdx.y * gridDim.x + blockIdx.x) * 3;
    partials[b0 + threadIdx.x] = red[threadIdx.x][0];
  }
}

// Warp adjoint: tar_w = (1-f) tar(i0) + f tar(i1) at X = x + dp - d_road(x + dp, v).
// dtar scatters through fixed-point atomics; dX feeds the plane gradient:
// dc -= dX (1, x + dp, v).
template <typename T>
__global__ void __launch_bounds__(kT)
warp_adjoint_kernel(const T* __restrict__ tar, int64_t pitch, const float* __restrict__ gw,
                    int W, int H, double dp, double c0, double c1, double c2,
                    unsigned long long* __restrict__ gtar_fix, double* __restrict__ partials) {
  const int x = blockIdx.x * kT + threadIdx.x, v = blockIdx.y;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  if (x < W) {
    const double ux = (double)x + dp;             // as the forward warp
    const double X = ux - fma(c2, (double)v, fma(c1, ux, c0));
    int i0;
    double f;
    bool inside = false;
    if (X <= 0.0) { i0 = 0; f = 0.0; }
    else if (X >= (double)(W - 1)) { i0 = W - 1; f = 0.0; }
    else { const double fl = floor(X); i0 = (int)fl; f = X - fl; inside = true; }
    const int i1 = min(i0 + 1, W - 1);
    const double g = gw[(int64_t)v * W + x];
    const int64_t row = (int64_t)v * W;
    fix_add(gtar_fix + row + i0, (1.0 - (double)(float)f) * g);
    fix_add(gtar_fix + row + i1, (double)(float)f * g);
    if (inside) {
      const double gX = g * ((double)ldf(tar + (int64_t)v * pitch + i1) -
                             (double)ldf(tar + (int64_t)v * pitch + i0));
      s0 = gX; s1 = gX * ((double)x + dp); s2 = gX * (double)v;
    }
  }
  reduce3(s0, s1, s2, partials);
}

// Direct plane terms of the shift back D = dh (1 - c1) + c0 + c1 (u + dp) + c2 v - dp.
__global__ void __launch_bounds__(kT)
plane_direct_kernel(const float* __restrict__ gD, const float* __restrict__ dh, int W, int H,
                    double dp, double* __restrict__ partials) {
  const int x = blockIdx.x * kT + threadIdx.x, v = blockIdx.y;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  if (x < W) {
    const int64_t p = (int64_t)v * W + x;
    const double g = gD[p];
    s0 = g; s1 = g * ((double)x - (double)dh[p] + dp); s2 = g * (double)v;
  }
  reduce3(s0, s1, s2, partials);
}

// out[k] = sum of (sign_a * A[b][k]) + (sign_b * B[b][k]) over blocks, fixed tree.
__global__ void __launch_bounds__(kT)
plane_finish_kernel(const double* __restrict__ pa, int na, double sa,
                    const double* __restrict__ pb, int nb, double sb,
                    double* __restrict__ out) {
  __shared__ double red[3][kT];
  double a[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < na; b += kT)
    for (int k = 0; k < 3; ++k) a[k] += sa * pa[(int64_t)b * 3 + k];
  for (int b = threadIdx.x; b < nb; b += kT)
    for (int k = 0; k < 3; ++k) a[k] += sb * pb[(int64_t)b * 3 + k];
  for (int k = 0; k < 3; ++k) red[k][threadIdx.x] = a[k];
  __syncthreads();
  for (int s = kT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < 3) out[threadIdx.x] = red[threadIdx.x][0];
}

__global__ void __launch_bounds__(kT)
fix_to_float_kernel(const unsigned long long* __restrict__ fx, int64_t n, const float* __restrict__ add,
                    float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  const double v = (double)(long long)fx[i] / kFix;
  out[i] = (float)v + (add ? add[i] : 0.0f);
}

// Several regions cleared by one launch: grid.y picks the region.
constexpr int kZeroMax = 9;
struct ZeroList {
  float* p[kZeroMax];
  int64_t n[kZeroMax];
};

// Four floats per thread (the regions start 256-byte aligned).
__global__ void __launch_bounds__(kT)
zero_many_kernel(ZeroList z) {
  const int k = blockIdx.y;
  const int64_t i = 4 * ((int64_t)blockIdx.x * kT + threadIdx.x);
  const int64_t n = z.n[k];
  if (i + 4 <= n) {
    *reinterpret_cast<float4*>(z.p[k] + i) = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  } else {
    for (int64_t j = i; j < n; ++j) z.p[k][j] = 0.0f;
  }
}

// Block means mu = z / (1/sd) of both statistics maps (0 for flat blocks),
// once per backward: the level loops of the NCC adjoint read them.
__global__ void __launch_bounds__(256)
mean_maps_kernel(const float* __restrict__ zX, const float* __restrict__ isdX,
                 const float* __restrict__ zY, const float* __restrict__ isdY, int64_t n,
                 float* __restrict__ muX, float* __restrict__ muY) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float iX = isdX[i], iY = isdY[i];
  muX[i] = iX != 0.0f ? zX[i] / iX : 0.0f;
  muY[i] = iY != 0.0f ? zY[i] / iY : 0.0f;
}

__global__ void __launch_bounds__(kT)
zero_u64_kernel(unsigned long long* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

// ---------------------------------------------------------------------------
// Photometric L1: s = lerp(tar, v, u - D) clamped; L = mean |ref - s|.
template <typename T>
__device__ __forceinline__ void sample(const T* tar, int64_t pitch, int W, int v, double X,
                                       int& i0, int& i1, double& f, bool& inside) {
  inside = false;
  if (X <= 0.0) { i0 = 0; f = 0.0; }
  else if (X >= (double)(W - 1)) { i0 = W - 1; f = 0.0; }
  else { const double fl = floor(X); i0 = (int)fl; f = X - fl; inside = true; }
  i1 = min(i0 + 1, W - 1);
}

template <typename T>
__global__ void __launch_bounds__(kT)
l1_forward_kernel(const T* __restrict__ ref, const T* __restrict__ tar, int64_t pr, int64_t pt,
                  const float* __restrict__ disp, int W, int H, double* __restrict__ partials) {
  const int x = blockIdx.x * kT + threadIdx.x, v = blockIdx.y;
  double s = 0.0;
  if (x < W) {
    int i0, i1; double f; bool in;
    sample(tar, pt, W, v, (double)x - (double)disp[(int64_t)v * W + x], i0, i1, f, in);
    const double sv = (1.0 - f) * ldf(tar + (int64_t)v * pt + i0) + f * ldf(tar + (int64_t)v * pt + i1);
    s = fabs((double)ldf(ref + (int64_t)v * pr + x) - sv);
  }
  reduce3(s, 0.0, 0.0, partials);
}

template <typename T>
__global__ void __launch_bounds__(kT)
l1_backward_kernel(const T* __restrict__ ref, const T* __restrict__ tar, int64_t pr, int64_t pt,
                   const float* __restrict__ disp, int W, int H, double scale,
                   float* __restrict__ g_ref, float* __restrict__ g_disp,
                   unsigned long long* __restrict__ gtar_fix) {
  const int x = blockIdx.x * kT + threadIdx.x, v = blockIdx.y;
  if (x >= W) return;
  const int64_t p = (int64_t)v * W + x;
  int i0, i1; double f; bool in;
  sample(tar, pt, W, v, (double)x - (double)disp[p], i0, i1, f, in);
  const double t0 = ldf(tar + (int64_t)v * pt + i0), t1 = ldf(tar + (int64_t)v * pt + i1);
  const double sv = (1.0 - f) * t0 + f * t1;
  const double a = (double)ldf(ref + (int64_t)v * pr + x);
  const double sg = (a > sv ? 1.0 : (a < sv ? -1.0 : 0.0)) * scale;
  if (g_ref) g_ref[p] = (float)sg;
  if (g_disp) g_disp[p] = (float)(in ? sg * (t1 - t0) : 0.0);
  if (gtar_fix) {
    fix_add(gtar_fix + (int64_t)v * W + i0, -(1.0 - f) * sg);
    fix_add(gtar_fix + (int64_t)v * W + i1, -f * sg);
  }
}

}  // namespace grad
}  // namespace stereo

// ===========================================================================
// Entry points: soft-argmin forward, its backward with per-level-tile
// recompute of the cost volume, and the photometric L1 loss.
namespace stereo {

size_t grad_layout(Plan& P, size_t o) {
  P.g_end = o;
  if (P.p.dtype != STEREO_F32) return o;
  const size_t HW = (size_t)P.W * P.H, DT = (size_t)P.grad_levels;
  const size_t HV = P.H + 2 * P.r, WVX = P.W + 2 * P.r, WVY = P.W + P.D - 1 + 2 * P.r;
  const size_t nb = (size_t)((P.W + 255) / 256) * P.H;
  const size_t f4 = sizeof(float);
  size_t sz[GR_COUNT];
  for (int i = GR_WP; i <= GR_GTARW; ++i) sz[i] = f4 * HW;
  sz[GR_SUMS] = 3 * f4 * HW;
  for (int i = GR_CT; i <= GR_GCT; ++i) sz[i] = f4 * DT * HW;
  // alpha maps, then the assemble pass's spills [HV][WVX / 64][64]
  sz[GR_FA] = f4 * std::max((size_t)DT * HW, HV * ((WVX + 63) / 64) * 64);
  // boxes of alpha; before them the NCC adjoint pass's spills [H][W / 64][64][2]
  sz[GR_BA] = f4 * std::max((size_t)DT * HV * WVX, (size_t)P.H * ((P.W + 63) / 64) * 128);
  sz[GR_BS] = 3 * f4 * HV * WVX;
  sz[GR_SY] = 3 * f4 * (size_t)P.H * (P.W + P.D - 1);
  sz[GR_BSY] = 3 * f4 * HV * WVY;
  sz[GR_MU] = 2 * f4 * (size_t)P.H * (P.W + 2 * P.r);
  sz[GR_GXV] = f4 * HV * WVX;
  sz[GR_GYV] = f4 * HV * WVY;
  sz[GR_GTARFIX] = sizeof(unsigned long long) * HW;
  sz[GR_PART_A] = sizeof(double) * 3 * nb;
  sz[GR_PART_B] = sizeof(double) * 3 * nb;
  sz[GR_SCRATCH] = sizeof(double) * 4;
  sz[GR_GMAX] = sizeof(float);
  for (int i = 0; i < GR_COUNT; ++i) {
    P.g_off[i] = o;
    o = align256(o + sz[i]);
  }
  P.g_end = o;
  return o;
}

}  // namespace stereo

using namespace stereo;
using namespace stereo::grad;

namespace {

template <typename T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

#define REQ(cond, ...) \
  do { if (!(cond)) return fail(STEREO_ERR_INVALID_ARGUMENT, __VA_ARGS__); } while (0)
#define HIPC(expr, what) \
  do { stereo_status s_ = hip_check((expr), (what)); if (s_ != STEREO_OK) return s_; } while (0)
#define LAUNCH(what, ...) \
  do { hipLaunchKernelGGL(__VA_ARGS__); HIPC(hipGetLastError(), what); } while (0)

stereo_status check_grad(const Plan& P, void* ws, size_t bytes) {
  REQ(P.p.dtype == STEREO_F32, "the differentiable form needs an F32 plan");
  REQ(P.p.perspective == 1, "the differentiable form needs perspective = 1");
  REQ(!P.homog, "the differentiable form differentiates the plane, not a homography");
  REQ(ws != nullptr, "workspace is NULL");
  if (bytes < P.ws_bytes)
    return fail(STEREO_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes < required %zu", bytes,
                P.ws_bytes);
  REQ((reinterpret_cast<uintptr_t>(ws) & 255) == 0, "workspace must be 256-byte aligned");
  return STEREO_OK;
}

// Plan copy whose warp / shift-back plane is the call's plane.
Plan with_plane(const Plan& P, const double plane[3]) {
  Plan Q = P;
  Q.p.plane[0] = plane[0];
  Q.p.plane[1] = plane[1];
  Q.p.plane[2] = plane[2];
  return Q;
}

struct Maps {
  float *zX, *isdX, *zY, *isdY;
};
Maps maps_of(const Plan& P, void* ws) {
  float* b = at<float>(ws, P.off_stats);
  const size_t n = (size_t)P.stats_w * P.H;
  return {b, b + n, b + 2 * n, b + 3 * n};
}

template <int r>
stereo_status box_r(int W, int H, const float* F, int nmaps, float* B, hipStream_t s) {
  dim3 grid((W + 2 * r + BX_TX - 1) / BX_TX, (H + 2 * r + BX_TY - 1) / BX_TY, nmaps);
  LAUNCH("box sums", (box_kernel<r>), grid, dim3(BX_TX), 0, s, F, W, H, B);
  return STEREO_OK;
}

// Box sums of nmaps [H][width] maps onto [H + 2r][width + 2r].
stereo_status box(const Plan& P, int width, const float* F, int nmaps, float* B,
                  hipStream_t s) {
  switch (P.r) {
#define BOX_CASE(R_) case R_: return box_r<R_>(width, P.H, F, nmaps, B, s);
    BOX_CASE(1) BOX_CASE(2) BOX_CASE(3) BOX_CASE(4) BOX_CASE(5) BOX_CASE(6) BOX_CASE(7) BOX_CASE(8)
#undef BOX_CASE
    default: return fail(STEREO_ERR_UNSUPPORTED, "ncc_radius");
  }
}

}  // namespace

extern "C" {

stereo_status stereo_soft_forward(stereo_plan_t plan, const float* ref, const float* tar,
                                  const double plane[3], float* disp_soft, float* saved,
                                  void* ws, size_t ws_bytes, hipStream_t stream) {
  REQ(plan && ref && tar && plane && disp_soft && saved,
      "plan, ref, tar, plane, disp_soft and saved must be non-NULL");
  stereo_status st = check_grad(plan->P, ws, ws_bytes);
  if (st != STEREO_OK) return st;
  REQ(std::isfinite(plane[0]) && std::isfinite(plane[1]) && std::isfinite(plane[2]) &&
          std::fabs(plane[1]) < 0.5, "plane must be finite with |c1| < 0.5");
  const Plan P = with_plane(plan->P, plane);
  const size_t HW = (size_t)P.W * P.H;
  float* tarw = at<float>(ws, P.off_tarw);
  Maps m = maps_of(P, ws);
  float* cvol = at<float>(ws, P.off_cvol);
  HIPC(launch_warp(P, tar, tarw, stream), "warp");
  HIPC(launch_block_stats2(P, ref, STEREO_F32, P.p.pitch_ref, tarw, m.zX, m.isdX, m.zY, m.isdY,
                           stream), "stats");
  BilArgs a{};
  if (P.agg_engine == 2) {
    // split-FP16 reference-anchored volume for the FP16-operand matrix cores
    uint16_t* vR = at<uint16_t>(ws, P.off_cvol);
    const int64_t plane = 16 * (int64_t)P.H * P.h2_pitch;
    HIPC(launch_ncc(P, ref, tarw, m.zX, m.isdX, m.zY, m.isdY, reinterpret_cast<float*>(vR),
                    P.h2_pitch, P.h2_pitch, plane, 0, stream, 0, -1, 2, P.R), "ncc");
    a.h2 = vR;
    a.h2_plane = plane;
    a.h2_pitch = P.h2_pitch;
  } else {
    HIPC(launch_ncc(P, ref, tarw, m.zX, m.isdX, m.zY, m.isdY, cvol, P.W, P.W, (int64_t)HW, 0,
                    stream, 0, -1, 1), "ncc");
    a.C = cvol;                     // float4 quads of levels: [ceil(D/4)][H][W]
    a.c_slice = (int64_t)HW;
    a.c_pitch = P.W;
    a.quad = 1;
  }
  a.guide = ref;
  a.guide_dt = STEREO_F32;
  a.guide_pitch = P.p.pitch_ref;
  a.sm_m = saved;
  a.sm_logZ = saved + HW;
  a.sm_dh = saved + 2 * HW;
  a.disp = disp_soft;
  a.plane[0] = plane[0]; a.plane[1] = plane[1]; a.plane[2] = plane[2];
  HIPC(launch_bilateral(P, a, 2, stream), "aggregation + soft-argmin");
  return STEREO_OK;
}

stereo_status stereo_backward(stereo_plan_t plan, const float* ref, const float* tar,
                              const double plane[3], const float* saved, const float* grad_disp,
                              float* grad_ref, float* grad_tar, double* grad_plane, void* ws,
                              size_t ws_bytes, hipStream_t stream) {
  return stereo_backward_profiled(plan, ref, tar, plane, saved, grad_disp, grad_ref, grad_tar,
                                  grad_plane, ws, ws_bytes, nullptr, stream);
}

stereo_status stereo_backward_profiled(stereo_plan_t plan, const float* ref, const float* tar,
                                       const double plane[3], const float* saved,
                                       const float* grad_disp, float* grad_ref, float* grad_tar,
                                       double* grad_plane, void* ws, size_t ws_bytes,
                                       hipEvent_t* ev, hipStream_t stream) {
  REQ(plan && ref && tar && plane && saved && grad_disp && grad_ref && grad_tar && grad_plane,
      "all arguments must be non-NULL");
  auto mark = [&](int i) -> hipError_t {
    return ev ? hipEventRecord(ev[i], stream) : hipSuccess;
  };
  stereo_status st = check_grad(plan->P, ws, ws_bytes);
  if (st != STEREO_OK) return st;
  REQ(std::isfinite(plane[0]) && std::isfinite(plane[1]) && std::isfinite(plane[2]) &&
          std::fabs(plane[1]) < 0.5, "plane must be finite with |c1| < 0.5");
  const Plan P = with_plane(plan->P, plane);
  const int W = P.W, H = P.H, D = P.D, r = P.r, DT = P.grad_levels;
  const int64_t HW = (int64_t)W * H;
  const int HV = H + 2 * r, WVX = W + 2 * r, WVY = W + D - 1 + 2 * r;
  const int64_t HVWV = (int64_t)HV * WVX;
  const Consts c = consts_of(P);
  const double dp = (double)P.p.delta_p;
  auto R_ = [&](int i) { return at<float>(ws, P.g_off[i]); };
  float* tarw = at<float>(ws, P.off_tarw);
  Maps m = maps_of(P, ws);
  float *Wp = R_(GR_WP), *aP = R_(GR_AP), *A1 = R_(GR_A1), *A2 = R_(GR_A2);
  // the three level sums are one [3][H][W] region: one box launch covers them
  float *SamY = R_(GR_SUMS), *Sb = SamY + HW, *SbmX = SamY + 2 * HW;
  float *gX = R_(GR_GX), *gtarw = R_(GR_GTARW);
  float *Ct = R_(GR_CT), *Gt = R_(GR_GT), *gCt = R_(GR_GCT);
  float* Fa = R_(GR_FA);
  float* Ba = R_(GR_BA);
  float* BS = R_(GR_BS);
  const int WY = W + D - 1;
  const int64_t HWY = (int64_t)H * WY, HVWVY = (int64_t)HV * WVY;
  float *SaX = R_(GR_SY), *Sg = SaX + HWY, *SgY = SaX + 2 * HWY;
  float* BSY = R_(GR_BSY);
  float *gXv = R_(GR_GXV), *gYv = R_(GR_GYV);
  auto* gfix = at<unsigned long long>(ws, P.g_off[GR_GTARFIX]);
  double* partA = at<double>(ws, P.g_off[GR_PART_A]);
  double* partB = at<double>(ws, P.g_off[GR_PART_B]);
  const float* sm_m = saved;
  const float* sm_logZ = saved + HW;
  const float* sm_dh = saved + 2 * HW;
  const dim3 rows((W + 255) / 256, H);
  const dim3 flat((unsigned)((HW + 255) / 256));
  const int nb = (int)rows.x * H;

  HIPC(mark(0), "event record");
  // accumulators, cleared by one kernel launch (graph-safe; the fixed-point
  // target accumulator is cleared as two floats per element, all bits zero)
  {
    ZeroList z{};
    float* const reg[kZeroMax] = {aP, A1, A2, SamY, SaX, gXv, gYv,
                                  reinterpret_cast<float*>(gfix), R_(GR_GMAX)};
    const int64_t len[kZeroMax] = {HW, HW, HW, 3 * HW, 2 * HWY, HVWV, (int64_t)HV * WVY,
                                   2 * HW, 1};
    int64_t nmax = 0;
    for (int k = 0; k < kZeroMax; ++k) {
      z.p[k] = reg[k];
      z.n[k] = len[k];
      nmax = std::max(nmax, len[k]);
    }
    LAUNCH("zero", zero_many_kernel, dim3((unsigned)((nmax + 4 * kT - 1) / (4 * kT)), kZeroMax),
           dim3(kT), 0, stream, z);
  }

  // forward state that is cheap to rebuild: warp, block statistics
  HIPC(launch_warp(P, tar, tarw, stream), "warp");
  HIPC(launch_block_stats2(P, ref, STEREO_F32, P.p.pitch_ref, tarw, m.zX, m.isdX, m.zY, m.isdY,
                           stream), "stats");
  float* muX = R_(GR_MU);
  float* muY = muX + (int64_t)H * (W + 2 * r);
  {
    const int64_t nmu = (int64_t)H * (W + 2 * r);
    LAUNCH("block means", mean_maps_kernel, dim3((unsigned)((nmu + 255) / 256)), dim3(256), 0,
           stream, m.zX, m.isdX, m.zY, m.isdY, nmu, muX, muY);
  }

  const int n = (2 * r + 1) * (2 * r + 1);
  // the aggregation passes on the split-FP16 matrix cores where they fit
  // (small radii: two weight operands per lane) and the level tiles start on
  // 16-level blocks; elsewhere on the vector ALU
  const bool mc = P.agg_engine == 2 && P.R <= kBwd16MaxR && (D <= DT || DT % 16 == 0);
  if (mc) {
    // max |g'| (the scale of C' in pass 1) and zeros in the pad columns of
    // the C' volume, which the passes never write
    LAUNCH("max |g'|", absmax_kernel,
           dim3((unsigned)std::min<int64_t>(256, (HW + 1023) / 1024)), dim3(256), 0, stream,
           grad_disp, HW,
           reinterpret_cast<unsigned int*>(R_(GR_GMAX)));
    HIPC(launch_h2_pad_zero(at<uint16_t>(ws, P.off_cvol + P.h2_tar_off),
                            16 * (int64_t)H * P.h2_pitch, P.h2_pitch, W, H, P.R, (DT + 15) / 16,
                            stream), "pad columns of C'");
  }
  for (int d0 = 0; d0 < D; d0 += DT) {
    const int nl = std::min(DT, D - d0);
    // pass 1: aggregated costs E, the softmax adjoint dE, dE / W_p, aP, A1 (and W_p)
    if (mc) {
      // matrix cores: the tile's costs recomputed once into both the split
      // volume the passes stage and the planar one the NCC adjoint reads;
      // pass 1 writes C' split for pass 2
      uint16_t* hC = at<uint16_t>(ws, P.off_cvol);
      uint16_t* hG = at<uint16_t>(ws, P.off_cvol + P.h2_tar_off);
      const int64_t hplane = 16 * (int64_t)H * P.h2_pitch;
      HIPC(launch_ncc(P, ref, tarw, m.zX, m.isdX, m.zY, m.isdY, reinterpret_cast<float*>(hC),
                      P.h2_pitch, P.h2_pitch, hplane, 0, stream, d0, d0 + nl, 3, P.R, Ct),
           "ncc tile (split and planar)");
      BilArgs a{};
      a.h2 = hC; a.h2_plane = hplane; a.h2_pitch = P.h2_pitch;
      a.guide = ref; a.guide_dt = STEREO_F32; a.guide_pitch = P.p.pitch_ref;
      a.levels = nl;
      a.E = Gt;
      a.sm_m = const_cast<float*>(sm_m);
      a.sm_logZ = const_cast<float*>(sm_logZ);
      a.sm_dh = const_cast<float*>(sm_dh);
      a.gD = grad_disp;
      a.aP = aP; a.A1 = A1; a.A2 = A2;
      a.Wp = d0 == 0 ? Wp : nullptr;
      a.d_first = d0;
      a.gmax = reinterpret_cast<const unsigned int*>(R_(GR_GMAX));
      a.h2_out = hG;
      a.plane[0] = plane[0]; a.plane[1] = plane[1]; a.plane[2] = plane[2];
      if (d0 == 0) HIPC(mark(1), "event record");
      HIPC(launch_bilateral_bwd16(P, a, 1, stream), "aggregation + softmax adjoint");
      if (d0 == 0) HIPC(mark(2), "event record");
      if (d0 == 0) HIPC(mark(3), "event record");
      a.h2 = hG;
      a.h2_out = nullptr;
      a.E = gCt;
      a.cpix = Ct;
      HIPC(launch_bilateral_bwd16(P, a, 2, stream), "aggregation adjoint");
      if (d0 == 0) HIPC(mark(4), "event record");
    } else {
    // recompute this tile of the cost volume
    HIPC(launch_ncc(P, ref, tarw, m.zX, m.isdX, m.zY, m.isdY, Ct, W, W, HW, 0, stream, d0,
                    d0 + nl), "ncc tile");
    BilArgs a{};
    a.C = Ct; a.c_slice = HW; a.c_pitch = W;
    a.guide = ref; a.guide_dt = STEREO_F32; a.guide_pitch = P.p.pitch_ref;
    a.levels = nl;
    a.E = Gt;
    a.sm_m = const_cast<float*>(sm_m);
    a.sm_logZ = const_cast<float*>(sm_logZ);
    a.sm_dh = const_cast<float*>(sm_dh);
    a.gD = grad_disp;
    a.aP = aP; a.A1 = A1; a.A2 = A2;
    a.Wp = d0 == 0 ? Wp : nullptr;
    a.d_first = d0;
    a.plane[0] = plane[0]; a.plane[1] = plane[1]; a.plane[2] = plane[2];
    if (d0 == 0) HIPC(mark(1), "event record");
    HIPC(launch_bilateral(P, a, 5, stream), "aggregation + softmax adjoint");
    if (d0 == 0) HIPC(mark(2), "event record");
    if (d0 == 0) HIPC(mark(3), "event record");
    // pass 2: dC(q, d) = sum_p w(q, p) dE(p, d) / W_p (weights are symmetric), A2
    a.C = Gt;
    a.E = gCt;
    a.cpix = Ct;
    HIPC(launch_bilateral(P, a, 6, stream), "aggregation adjoint");
    if (d0 == 0) HIPC(mark(4), "event record");
    }
    if (nl <= 64) {
      // both passes over C and dC in one; the boxes of alpha (written later)
      // hold the spills until the merge
      const int nbx = (W + 63) / 64;
      LAUNCH("ncc adjoint (coefficients, diagonal sums)", ncc_adjoint_kernel, dim3(nbx, H),
             dim3(64), 0, stream, Ct, gCt, muX, m.isdX, muY, m.isdY, W, H, D, r, d0, nl,
             1.0f / (float)n, Fa, Sb, SbmX, SamY, SaX, Sg, Ba);
      LAUNCH("ncc adjoint (diagonal spills)", ncc_adjoint_merge_kernel,
             dim3((WY + kT - 1) / kT, H), dim3(kT), 0, stream, Ba, nbx, W, D, r, d0, nl, muY,
             SaX, Sg, SgY);
    } else {
      LAUNCH("ncc adjoint coefficients", ncc_coef_kernel, rows, dim3(kT), 0, stream, Ct, gCt,
             muX, m.isdX, muY, m.isdY, W, H, r, d0, nl, 1.0f / (float)n, Fa, Sb, SbmX, SamY);
      LAUNCH("ncc adjoint target sums", ncc_shear_kernel, dim3((WY + kT - 1) / kT, H), dim3(kT),
             0, stream, Ct, gCt, muX, m.isdX, muY, m.isdY, W, H, D, r, d0, nl,
             1.0f / (float)n, SaX, Sg, SgY);
    }
    if ((st = box(P, W, Fa, nl, Ba, stream)) != STEREO_OK) return st;
    if (nl <= 64) {
      // both sides in one pass over the boxes; the alpha maps are consumed,
      // their region holds the spills
      const int nbx = (WVX + 63) / 64;
      LAUNCH("ncc adjoint (both sides)", assemble_kernel<float>, dim3(nbx, HV), dim3(64), 0,
             stream, Ba, tarw, ref, P.p.pitch_ref, W, H, D, r, d0, nl, gXv, gYv, Fa);
      LAUNCH("ncc adjoint (target spills)", assemble_merge_kernel,
             dim3((WVY + kT - 1) / kT, HV), dim3(kT), 0, stream, Fa, nbx, W, D, r, d0, nl, gYv);
    } else {
      LAUNCH("ncc adjoint (reference side)", assemble_x_kernel, dim3((WVX + 255) / 256, HV),
             dim3(256), 0, stream, Ba, tarw, W, H, r, d0, nl, gXv);
      LAUNCH("ncc adjoint (target side)", assemble_y_kernel<float>, dim3((WVY + 255) / 256, HV),
             dim3(256), 0, stream, Ba, ref, P.p.pitch_ref, W, H, D, r, d0, nl, gYv);
    }
  }
  if ((st = box(P, W, SamY, 3, BS, stream)) != STEREO_OK) return st;
  LAUNCH("ncc adjoint (level sums)", x_complete_kernel<float>, dim3((WVX + 255) / 256, HV),
         dim3(256), 0, stream, BS, BS + HVWV, BS + 2 * HVWV, ref, P.p.pitch_ref, W, H, r, gXv);
  if ((st = box(P, WY, SaX, 3, BSY, stream)) != STEREO_OK) return st;
  LAUNCH("ncc adjoint (target level sums)", y_complete_kernel, dim3((WVY + 255) / 256, HV),
         dim3(256), 0, stream, BSY, BSY + HVWVY, BSY + 2 * HVWVY, tarw, W, H, D, r, gYv);
  LAUNCH("fold", fold_kernel, rows, dim3(256), 0, stream, gXv, W, H, r, r, gX);
  LAUNCH("fold", fold_kernel, rows, dim3(256), 0, stream, gYv, W, H, r, D - 1 + r, gtarw);
  LAUNCH("guide gradient", guide_finish_kernel<float>,
         dim3((W + GF_TX - 1) / GF_TX, (H + GF_TY - 1) / GF_TY), dim3(256), 0, stream, ref,
         P.p.pitch_ref, Wp, aP, A1, A2, gX, W, H, P.R, c.ks2, c.kr2,
         (float)(2.0 / ((double)P.p.sigma_r * P.p.sigma_r)), grad_ref);
  LAUNCH("warp adjoint", warp_adjoint_kernel<float>, rows, dim3(256), 0, stream, tar,
         P.p.pitch_tar, gtarw, W, H, dp, plane[0], plane[1], plane[2], gfix, partB);
  LAUNCH("fixed point", fix_to_float_kernel, flat, dim3(256), 0, stream, gfix, HW,
         (const float*)nullptr, grad_tar);
  LAUNCH("plane (shift back)", plane_direct_kernel, rows, dim3(256), 0, stream, grad_disp,
         sm_dh, W, H, dp, partA);
  LAUNCH("plane", plane_finish_kernel, dim3(1), dim3(256), 0, stream, partA, nb, 1.0, partB, nb,
         -1.0, grad_plane);
  HIPC(mark(5), "event record");
  return STEREO_OK;
}

stereo_status stereo_photometric_l1(stereo_plan_t plan, const float* ref, const float* tar,
                                    const float* disp_soft, double* loss_dev, void* ws,
                                    size_t ws_bytes, hipStream_t stream) {
  REQ(plan && ref && tar && disp_soft && loss_dev, "all arguments must be non-NULL");
  stereo_status st = check_grad(plan->P, ws, ws_bytes);
  if (st != STEREO_OK) return st;
  const Plan& P = plan->P;
  const dim3 rows((P.W + 255) / 256, P.H);
  const int nb = (int)rows.x * P.H;
  double* part = at<double>(ws, P.g_off[GR_PART_A]);
  double* scratch = at<double>(ws, P.g_off[GR_SCRATCH]);
  LAUNCH("l1", l1_forward_kernel<float>, rows, dim3(256), 0, stream, ref, tar, P.p.pitch_ref,
         P.p.pitch_tar, disp_soft, P.W, P.H, part);
  LAUNCH("l1", plane_finish_kernel, dim3(1), dim3(256), 0, stream, part, nb,
         1.0 / ((double)P.W * P.H), (const double*)nullptr, 0, 0.0, scratch);
  HIPC(hipMemcpyAsync(loss_dev, scratch, sizeof(double), hipMemcpyDeviceToDevice, stream),
       "copy loss");
  return STEREO_OK;
}

stereo_status stereo_photometric_l1_bwd(stereo_plan_t plan, const float* ref, const float* tar,
                                        const float* disp_soft, double grad_loss, float* g_ref,
                                        float* g_tar, float* g_disp, void* ws, size_t ws_bytes,
                                        hipStream_t stream) {
  REQ(plan && ref && tar && disp_soft, "plan, ref, tar and disp_soft must be non-NULL");
  REQ(g_ref || g_tar || g_disp, "no gradient requested");
  stereo_status st = check_grad(plan->P, ws, ws_bytes);
  if (st != STEREO_OK) return st;
  const Plan& P = plan->P;
  const int64_t HW = (int64_t)P.W * P.H;
  const dim3 rows((P.W + 255) / 256, P.H);
  const dim3 flat((unsigned)((HW + 255) / 256));
  auto* gfix = at<unsigned long long>(ws, P.g_off[GR_GTARFIX]);
  if (g_tar) LAUNCH("zero", zero_u64_kernel, flat, dim3(256), 0, stream, gfix, HW);
  LAUNCH("l1 adjoint", l1_backward_kernel<float>, rows, dim3(256), 0, stream, ref, tar,
         P.p.pitch_ref, P.p.pitch_tar, disp_soft, P.W, P.H, grad_loss / (double)HW, g_ref, g_disp,
         g_tar ? gfix : nullptr);
  if (g_tar)
    LAUNCH("fixed point", fix_to_float_kernel, flat, dim3(256), 0, stream, gfix, HW,
           (const float*)nullptr, g_tar);
  return STEREO_OK;
}

}  // extern "C"
