// Disparity selection on a materialised aggregated volume (Sec. 3.2.2):
// winner-take-all with the sub-pixel parabola of Eq. (13), and the
// left-right check of Eq. (12) followed by the shift back to the full
// disparity domain.
#include "internal.h"

namespace stereo {
namespace {

// One thread per pixel walks the levels in order; volume reads are
// coalesced across the threads of a slice.
__global__ void __launch_bounds__(256)
wta_kernel(const float* __restrict__ E, int W, int H, int D,
           int16_t* __restrict__ dint, float* __restrict__ dsub) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t HW = (int64_t)W * H;
  if (p >= HW) return;
  float bestE = 3.402823466e38f, Em = 0.0f, Ep = 0.0f, prev = 0.0f;
  int bestD = 0;
  for (int d = 0; d < D; ++d) {
    const float e = E[(int64_t)d * HW + p];
    if (d == bestD + 1) Ep = e;
    if (e < bestE) { Em = prev; bestE = e; bestD = d; }
    prev = e;
  }
  dint[p] = (int16_t)bestD;
  if (dsub) {
    float off = 0.0f;
    if (bestD > 0 && bestD < D - 1) {
      const float den = 2.0f * Em + 2.0f * Ep - 4.0f * bestE;
      if (den > 0.0f) off = (Em - Ep) / den;
    }
    dsub[p] = (float)bestD + off;
  }
}

// valid = (u - dR >= 0) && (dR - dT(u - dR))^2 <= delta_r;
// disp = l - delta_p + d_road(u - l + delta_p, v), evaluated in FP64.
__device__ __forceinline__ void lr_body(const int16_t* __restrict__ dR,
                                        const int16_t* __restrict__ dT,
                                        const float* __restrict__ dsub, int W, float lr_delta,
                                        int use_lr, int persp, double delta_p, double c0,
                                        double c1, double c2, uint8_t* __restrict__ valid,
                                        float* __restrict__ disp, int bx, int v) {
  const int u = bx * 256 + threadIdx.x;
  if (u >= W) return;
  const int64_t p = (int64_t)v * W + u;
  const int d = dR[p];
  const int x = u - d;
  bool ok = x >= 0;
  if (ok && use_lr) {
    const float diff = (float)(d - (int)dT[(int64_t)v * W + x]);
    ok = diff * diff <= lr_delta;
  }
  if (valid) valid[p] = ok ? 1 : 0;
  if (disp) {
    const double ell = dsub ? (double)dsub[p] : (double)d;
    double out = ell;
    if (persp) out = ell - delta_p + fma(c2, (double)v, fma(c1, (double)u - ell + delta_p, c0));
    disp[p] = ok ? (float)out : __builtin_nanf("");
  }
}

// The same check; the shift back by the homography: disp = u - X with
// (X, Y) = H (u - l + delta_p, v, 1) (Eq. 3), in FP64.
__device__ __forceinline__ void lr_h_body(const int16_t* __restrict__ dR,
                                          const int16_t* __restrict__ dT,
                                          const float* __restrict__ dsub, int W, float lr_delta,
                                          int use_lr, double delta_p, const Homog& M,
                                          uint8_t* __restrict__ valid, float* __restrict__ disp,
                                          int bx, int v) {
  const int u = bx * 256 + threadIdx.x;
  if (u >= W) return;
  const int64_t p = (int64_t)v * W + u;
  const int d = dR[p];
  const int x = u - d;
  bool ok = x >= 0;
  if (ok && use_lr) {
    const float diff = (float)(d - (int)dT[(int64_t)v * W + x]);
    ok = diff * diff <= lr_delta;
  }
  if (valid) valid[p] = ok ? 1 : 0;
  if (disp) {
    const double ell = dsub ? (double)dsub[p] : (double)d;
    const double* h = M.h;
    const double uu = (double)u - ell + delta_p, vv = (double)v;
    const double X = fma(h[0], uu, fma(h[1], vv, h[2])) / fma(h[6], uu, fma(h[7], vv, h[8]));
    disp[p] = ok ? (float)((double)u - X) : __builtin_nanf("");
  }
}

__global__ void __launch_bounds__(256)
lr_h_kernel(const int16_t* __restrict__ dR, const int16_t* __restrict__ dT,
            const float* __restrict__ dsub, int W, float lr_delta, int use_lr, double delta_p,
            Homog M, uint8_t* __restrict__ valid, float* __restrict__ disp) {
  lr_h_body(dR, dT, dsub, W, lr_delta, use_lr, delta_p, M, valid, disp, blockIdx.x, blockIdx.y);
}

__global__ void __launch_bounds__(256)
lr_kernel(const int16_t* __restrict__ dR, const int16_t* __restrict__ dT,
          const float* __restrict__ dsub, int W, int H, float lr_delta,
          int use_lr, int persp, double delta_p, double c0, double c1, double c2,
          uint8_t* __restrict__ valid, float* __restrict__ disp) {
  lr_body(dR, dT, dsub, W, lr_delta, use_lr, persp, delta_p, c0, c1, c2, valid, disp,
          blockIdx.x, blockIdx.y);
}

__global__ void __launch_bounds__(256)
lr_tracked_kernel(const int16_t* __restrict__ dR, const int16_t* __restrict__ dT,
                  const float* __restrict__ dsub, int W, float lr_delta, int use_lr,
                  double delta_p, const stereo_plane_state* __restrict__ st,
                  uint8_t* __restrict__ valid, float* __restrict__ disp) {
  lr_body(dR, dT, dsub, W, lr_delta, use_lr, 1, delta_p, st->plane[0], st->plane[1],
          st->plane[2], valid, disp, blockIdx.x, blockIdx.y);
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

__global__ void __launch_bounds__(256)
lr_jobs_kernel(const LrJob* __restrict__ jobs, const int* __restrict__ first, int n) {
  const int j = job_of(first, n, blockIdx.x);
  const LrJob& J = jobs[j];
  const int l = blockIdx.x - first[j];
  if (J.homog)
    lr_h_body(J.dR, J.dT, J.dsub, J.W, J.lr_delta, J.use_lr, J.dp, J.Hm, J.valid, J.disp,
              l % J.gx, l / J.gx);
  else
    lr_body(J.dR, J.dT, J.dsub, J.W, J.lr_delta, J.use_lr, J.persp, J.dp, J.c0, J.c1, J.c2,
            J.valid, J.disp, l % J.gx, l / J.gx);
}

}  // namespace

hipError_t launch_wta(const Plan& P, const float* E, int16_t* dint, float* dsub,
                      hipStream_t s) {
  const int64_t HW = (int64_t)P.W * P.H;
  hipLaunchKernelGGL(wta_kernel, dim3((unsigned)((HW + 255) / 256)), dim3(256), 0, s,
                     E, P.W, P.H, P.D, dint, dsub);
  return hipGetLastError();
}

int lr_job_blocks(const Plan& P) { return ((P.W + 255) / 256) * P.H; }

LrJob lr_job(const Plan& P, const int16_t* dR, const int16_t* dT, const float* dsub,
             uint8_t* valid, float* disp) {
  const stereo_params& p = P.p;
  LrJob J{};
  J.dR = dR; J.dT = dT; J.dsub = dsub; J.valid = valid; J.disp = disp;
  J.dp = p.perspective ? (double)p.delta_p : 0.0;
  J.c0 = p.plane[0]; J.c1 = p.plane[1]; J.c2 = p.plane[2];
  J.lr_delta = p.lr_delta;
  J.W = P.W; J.H = P.H; J.use_lr = (p.lr_check && dT) ? 1 : 0; J.persp = p.perspective;
  J.gx = (P.W + 255) / 256;
  J.homog = P.homog;
  for (int k = 0; k < 9; ++k) J.Hm.h[k] = P.Hm[k];
  return J;
}

hipError_t launch_lr_jobs(const LrJob* jobs, const int* first, int n, int blocks,
                          hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(lr_jobs_kernel, dim3(blocks), dim3(256), 0, s, jobs, first, n);
  return hipGetLastError();
}

hipError_t launch_lr_check_tracked(const Plan& P, const int16_t* dR, const int16_t* dT,
                                   const float* dsub, const stereo_plane_state* st,
                                   uint8_t* valid, float* disp, hipStream_t s) {
  const stereo_params& p = P.p;
  hipLaunchKernelGGL(lr_tracked_kernel, dim3((P.W + 255) / 256, P.H), dim3(256), 0, s, dR, dT,
                     dsub, P.W, p.lr_delta, (p.lr_check && dT) ? 1 : 0, (double)p.delta_p, st,
                     valid, disp);
  return hipGetLastError();
}

hipError_t launch_lr_check(const Plan& P, const int16_t* dR, const int16_t* dT,
                           const float* dsub, uint8_t* valid, float* disp,
                           hipStream_t s) {
  const stereo_params& p = P.p;
  if (P.homog) {
    Homog M;
    for (int k = 0; k < 9; ++k) M.h[k] = P.Hm[k];
    hipLaunchKernelGGL(lr_h_kernel, dim3((P.W + 255) / 256, P.H), dim3(256), 0, s, dR, dT,
                       dsub, P.W, p.lr_delta, (p.lr_check && dT) ? 1 : 0, (double)p.delta_p,
                       M, valid, disp);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(lr_kernel, dim3((P.W + 255) / 256, P.H), dim3(256), 0, s, dR, dT,
                     dsub, P.W, P.H, p.lr_delta, (p.lr_check && dT) ? 1 : 0,
                     p.perspective, p.perspective ? (double)p.delta_p : 0.0,
                     p.plane[0], p.plane[1], p.plane[2], valid, disp);
  return hipGetLastError();
}

}  // namespace stereo
