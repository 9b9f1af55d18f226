// Disparity transformation, Sec. 3.3: roll-angle fit (Eqs. 14-28) and the
// transformation of Eq. (29), entirely on the device so that the call can be
// captured into a graph (no device-to-host copy).
//
// The energy of Eq. (23) and its gradient (Eq. 26) depend on the data only
// through ten sums over the selected pixels:
//   n, Su, Sv, Suu, Suv, Svv, Sd, Sdd, Sdu, Sdv.
// With y = v cos psi - u sin psi and y' = dy/dpsi:
//   alpha = A^-1 b,  A = [[n, Sy], [Sy, Syy]],  b = [Sd, Sdy]      (Eq. 21)
//   E(psi) = Sdd - alpha . b                                       (Eq. 23)
//   dE/dpsi = -2 alpha1 (Sdy' - alpha0 Sy' - alpha1 Syy')          (Eq. 26)
// The sums are accumulated in FP64 in a fixed order (per-thread grid-stride
// sums, a fixed tree per block, then a fixed tree over the block partials),
// so the fit is deterministic.
#include <mutex>

#include "internal.h"

namespace stereo {
namespace {

constexpr int kRoadThreads = 256;
constexpr int kMom = 10;

struct Mom {
  double n, su, sv, suu, suv, svv, sd, sdd, sdu, sdv;
};

__global__ void __launch_bounds__(kRoadThreads)
road_moments_kernel(const float* __restrict__ disp, const uint8_t* __restrict__ mask,
                    int W, int H, double* __restrict__ partials) {
  __shared__ double red[kMom][kRoadThreads];
  double a[kMom];
#pragma unroll
  for (int j = 0; j < kMom; ++j) a[j] = 0.0;
  // rows by block, columns by thread: no division per pixel
  for (int y = blockIdx.x; y < H; y += gridDim.x) {
    const float* drow = disp + (int64_t)y * W;
    const uint8_t* mrow = mask ? mask + (int64_t)y * W : nullptr;
    const double v = (double)y;
    for (int x = threadIdx.x; x < W; x += kRoadThreads) {
      const float df = drow[x];
      if (!(df == df) || isinf(df)) continue;        // NaN / inf: not a disparity
      if (mrow && !mrow[x]) continue;
      const double d = df;
      const double u = (double)x;
      a[0] += 1.0; a[1] += u; a[2] += v; a[3] += u * u; a[4] += u * v;
      a[5] += v * v; a[6] += d; a[7] += d * d; a[8] += d * u; a[9] += d * v;
    }
  }
#pragma unroll
  for (int j = 0; j < kMom; ++j) red[j][threadIdx.x] = a[j];
  __syncthreads();
  for (int s = kRoadThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
#pragma unroll
      for (int j = 0; j < kMom; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x < kMom) partials[(int64_t)blockIdx.x * kMom + threadIdx.x] = red[threadIdx.x][0];
}

struct Fit {
  double a0, a1, sdy, sy;
};

__device__ Fit alpha_cs(const Mom& m, double c, double s) {
  Fit f;
  f.sy = c * m.sv - s * m.su;
  const double syy = c * c * m.svv - 2.0 * s * c * m.suv + s * s * m.suu;
  f.sdy = c * m.sdv - s * m.sdu;
  const double det = m.n * syy - f.sy * f.sy;
  f.a0 = (syy * m.sd - f.sy * f.sdy) / det;
  f.a1 = (m.n * f.sdy - f.sy * m.sd) / det;
  return f;
}

__device__ Fit alpha_at(const Mom& m, double psi) {
  double s, c;
  sincos(psi, &s, &c);
  return alpha_cs(m, c, s);
}

__device__ double energy_at(const Mom& m, double psi) {
  const Fit f = alpha_at(m, psi);
  return m.sdd - (f.a0 * m.sd + f.a1 * f.sdy);
}

__device__ double gradient_at(const Mom& m, double psi) {
  double s, c;
  sincos(psi, &s, &c);
  const Fit f = alpha_cs(m, c, s);
  const double syp = -s * m.sv - c * m.su;
  const double syyp = s * c * (m.suu - m.svv) + (s * s - c * c) * m.suv;
  const double sdyp = -s * m.sdv - c * m.sdu;
  return -2.0 * f.a1 * (sdyp - f.a0 * syp - f.a1 * syyp);
}

__device__ double wrap_half_pi(double psi) {
  const double pi = 3.14159265358979323846;
  double w = fmod(psi + pi / 2.0, pi);
  if (w <= 0.0) w += pi;
  return w - pi / 2.0;
}

// One block: thread b loads the partial sums of block b, then a fixed tree
// combines them (deterministic); one lane then runs the descent.  Rate:
// Eq. (28), lambda_k+1 = lambda_k g_k / (g_k - g_k+1); a step is halved while
// it raises the normalised energy or exceeds pi/4; a non-positive rate
// restarts at lambda0.
__global__ void __launch_bounds__(kRoadThreads)
road_fit_kernel(const double* __restrict__ partials, int nblocks, int W, int H,
                double psi0, double lambda0, double delta_psi, int max_iter,
                stereo_road_fit* __restrict__ out, stereo_plane_state* __restrict__ state) {
  __shared__ double red[kMom][kRoadThreads];
  double a[kMom];
#pragma unroll
  for (int j = 0; j < kMom; ++j) a[j] = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kRoadThreads) {
#pragma unroll
    for (int j = 0; j < kMom; ++j) a[j] += partials[(int64_t)b * kMom + j];
  }
#pragma unroll
  for (int j = 0; j < kMom; ++j) red[j][threadIdx.x] = a[j];
  __syncthreads();
  for (int s = kRoadThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
#pragma unroll
      for (int j = 0; j < kMom; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  if (state) psi0 = state->psi;            // warm start from the previous frame
  double mom[kMom];
#pragma unroll
  for (int j = 0; j < kMom; ++j) mom[j] = red[j][0];
  Mom m{mom[0], mom[1], mom[2], mom[3], mom[4], mom[5], mom[6], mom[7], mom[8], mom[9]};
  stereo_road_fit r;
  r.n_points = m.n;
  r.pad_ = 0;
  double psi = psi0;
  int iters = 0, converged = 0, flat = 0;
  Fit f0;
  if (m.n < 3.0) {
    flat = 1; converged = 1;
    f0.a0 = m.n > 0.0 ? m.sd / m.n : 0.0;
    f0.a1 = 0.0;
  } else {
    f0 = alpha_at(m, psi0);
    if (!(fabs(f0.a1) >= 1e-6)) { flat = 1; converged = 1; }
  }
  if (!flat) {
    const double s = (double)max(W, H);
    const double scale = 1.0 / (m.n * s * s * f0.a1 * f0.a1);
    double lam = lambda0;
    double E = energy_at(m, psi) * scale;
    double g = gradient_at(m, psi) * scale;
    const double pi = 3.14159265358979323846;
    for (iters = 1; iters <= max_iter; ++iters) {
      double step = -lam * g;
      for (int h = 0; h < 64; ++h) {
        if (fabs(step) <= pi / 4.0 &&
            energy_at(m, wrap_half_pi(psi + step)) * scale <= E * (1.0 + 1e-9))
          break;
        lam *= 0.5;
        step = -lam * g;
      }
      const double psi_new = wrap_half_pi(psi + step);
      const double g_new = gradient_at(m, psi_new) * scale;
      const bool done = fabs(step) < delta_psi;
      if (g_new == g) {
        psi = psi_new; converged = 1;
        break;
      }
      lam = lam * g / (g - g_new);
      if (!(lam > 0.0) || isinf(lam)) lam = lambda0;
      psi = psi_new;
      E = energy_at(m, psi) * scale;
      g = g_new;
      if (done) { converged = 1; break; }
    }
    if (iters > max_iter) iters = max_iter;
    f0 = alpha_at(m, psi);
  }
  r.psi = psi;
  r.alpha0 = f0.a0;
  r.alpha1 = f0.a1;
  r.e_min = (m.n >= 3.0) ? energy_at(m, psi) : 0.0;
  r.plane[0] = f0.a0;
  r.plane[1] = -f0.a1 * sin(psi);
  r.plane[2] = f0.a1 * cos(psi);
  r.iters = iters;
  r.converged = converged;
  r.flat = flat;
  *out = r;
  if (state && !flat) {                    // the next frame's plane
    state->plane[0] = r.plane[0];
    state->plane[1] = r.plane[1];
    state->plane[2] = r.plane[2];
    state->psi = psi;
    state->frames += 1;
  }
}

// Eq. (29): l' = l - a0 + a1 (u sin psi - v cos psi) + delta_t.
__global__ void __launch_bounds__(256)
road_apply_kernel(const float* __restrict__ disp, int W, int H,
                  const stereo_road_fit* __restrict__ fit, float delta_t,
                  float* __restrict__ out) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  if (u >= W) return;
  const double psi = fit->psi, a0 = fit->alpha0, a1 = fit->alpha1;
  const int64_t p = (int64_t)v * W + u;
  out[p] = (float)((double)disp[p] - a0 + a1 * ((double)u * sin(psi) - (double)v * cos(psi)) +
                   (double)delta_t);
}

// Damage below the flattened road: mask = finite(l') && l' < delta_t - tau.
__global__ void __launch_bounds__(256)
damage_mask_kernel(const float* __restrict__ disp_t, int64_t n, float level,
                   uint8_t* __restrict__ mask) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float d = disp_t[i];
  mask[i] = (isfinite(d) && d < level) ? 1 : 0;
}

}  // namespace

hipError_t launch_damage_mask(const Plan& P, const float* disp_t, float delta_t, float tau,
                              uint8_t* mask, hipStream_t s) {
  const int64_t n = (int64_t)P.W * P.H;
  const float level = delta_t - tau;
  hipLaunchKernelGGL(damage_mask_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     disp_t, n, level, mask);
  return hipGetLastError();
}

// Fixed device buffer of the allocation-free road transform: room for the
// ten FP64 moment partials of up to kRoadScratchDoubles / 10 reduction
// blocks.  Every device the library runs on holds one copy for the life of
// the process; calls on one device share it.
static __device__ __align__(256) double scratch[kRoadScratchDoubles];

hipError_t road_scratch(double** out, size_t* bytes) {
  static std::mutex mu;
  static double* ptr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    // the array's name is a host-side stand-in: the device address of this
    // device's copy comes from the runtime, once per device
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    ptr[dev] = static_cast<double*>(p);
  }
  *out = ptr[dev];
  *bytes = sizeof(double) * (size_t)kRoadScratchDoubles;
  return hipSuccess;
}

hipError_t launch_road(const Plan& P, const float* disp, const uint8_t* mask,
                       double psi0, double lambda0, double delta_psi, int max_iter,
                       float delta_t, stereo_road_fit* fit, float* disp_t,
                       double* partials, hipStream_t s, stereo_plane_state* state) {
  hipLaunchKernelGGL(road_moments_kernel, dim3(P.road_blocks), dim3(kRoadThreads), 0, s,
                     disp, mask, P.W, P.H, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(road_fit_kernel, dim3(1), dim3(kRoadThreads), 0, s, partials, P.road_blocks,
                     P.W, P.H, psi0, lambda0, delta_psi, max_iter, fit, state);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (disp_t) {
    hipLaunchKernelGGL(road_apply_kernel, dim3((P.W + 255) / 256, P.H), dim3(256), 0, s,
                       disp, P.W, P.H, fit, delta_t, disp_t);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace stereo
