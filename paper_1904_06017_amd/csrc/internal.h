// Internal declarations shared by the library's host and device sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/stereo.h"

namespace stereo {

// Set the thread-local error message and return the status.
stereo_status fail(stereo_status s, const char* fmt, ...);
// Map a HIP error (after a launch) to a status; hipSuccess -> STEREO_OK.
stereo_status hip_check(hipError_t e, const char* what);

constexpr float kOffset = 128.0f;   // NCC is offset invariant; centring the
                                    // intensities keeps FP32 block sums exact
constexpr float kFlatVar = 1e-6f;   // block variance (gray^2) below which the
                                    // NCC is undefined and the cost is 1
constexpr float kFarGuide = 1e30f;  // guide value outside the image: weight 0

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Derived sizes and the workspace layout of a plan.
struct Plan {
  stereo_params p;
  int W, H, D, r, R;
  int stats_w;        // block-statistics map width: columns [-r, W + r)
  int cw;             // row pitch of the internal cost volume (>= W + D - 1),
                      // stored level-quad-interleaved: [ceil(D/4)][H][cw] float4
  size_t off_tarw, off_stats, off_cvol, off_dT, off_dsub, off_road;
  size_t ws_bytes;
  int road_blocks;    // partial-sum blocks of the road moments
  // tuning (stereo_plan_set_tuning): levels per aggregation pass by guide type
  int agg_levels_u8 = 8;
  int agg_levels_f32 = 8;
  int homog = 0;        // 1: warp / shift back by the homography Hm (Eq. 3)
  double Hm[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  int ncc_levels = 0;   // levels per NCC workgroup (16, 32 or 64; DC / 4 waves);
                        // 0: 64 / 32 / 16 by the levels of the launch
  int agg_engine = 2;   // fused aggregation + selection: 2 matrix cores with split
                        // FP16 operands, 1 matrix cores with FP32 operands, 0 vector ALU
  int h2_pitch = 0;     // row pitch (halves) of the split-FP16 volumes
  size_t h2_tar_off = 0;  // byte offset of the target-anchored one in the volume region
  // differentiable form (F32 plans): levels recomputed per backward tile and
  // the workspace regions it uses (offsets from the workspace base)
  int grad_levels = 16;  // set from D at plan creation
  size_t g_off[32];
  size_t g_end;
};

// Workspace regions of the backward (indices into Plan::g_off).
enum GradRegion {
  GR_WP, GR_AP, GR_A1, GR_A2,
  GR_SUMS,                                      // [3][H][W]: alpha muY, beta, beta muX
  GR_GX, GR_GTARW,
  GR_CT, GR_GT, GR_GCT, GR_FA,                 // GR_FA: [DT][H][W] alpha maps
  GR_BA,                                        // [DT][HV][WVX] boxes of alpha
  GR_BS,                                        // [3][HV][WVX] boxes of the X sums
  GR_SY,                                        // [3][H][W+D-1] target-side sums
  GR_BSY,                                       // [3][HV][WVY] their boxes
  GR_MU,                                        // [2][H][W+2r] block means of X, Y
  GR_GXV, GR_GYV, GR_GTARFIX, GR_PART_A, GR_PART_B, GR_SCRATCH,
  GR_GMAX,                                      // max |C'| of the matrix-core backward
  GR_COUNT
};

// Float view of a few plan parameters, precomputed on the host.
struct Consts {
  float ks2;          // log2(e) / sigma_s^2
  float kr2;          // log2(e) / sigma_r^2
};
Consts consts_of(const Plan& P);

// ---- kernel launchers (each returns hipGetLastError after the launch) ----
hipError_t launch_warp(const Plan& P, const void* tar, float* tar_w,
                       hipStream_t s);
// the same with the plane read from device memory (perspective plans)
hipError_t launch_warp_tracked(const Plan& P, const void* tar, const stereo_plane_state* st,
                               float* tar_w, hipStream_t s);

// z = mu / sigma and isd = 1 / sigma of (I - 128) over the clamped (2r+1)^2
// block centred at every column x in [-r, W + r) and row y; a flat block
// stores z = isd = 0.
// Statistics of the reference (dt) and the warped target (FP32) in one launch.
hipError_t launch_block_stats2(const Plan& P, const void* ref, stereo_dtype dt,
                               int64_t ref_pitch, const float* tarw, float* zX, float* isdX,
                               float* zY, float* isdY, hipStream_t s);
hipError_t launch_block_stats(const Plan& P, const void* img, stereo_dtype dt,
                              int64_t pitch, float* z, float* isd,
                              hipStream_t s);

// C[d][y][x], x in [0, out_w): anchor 0 compares the ref block at x with the
// tar_w block at x - d; anchor 1 the ref block at x + d with tar_w at x.
// ref statistics in (zX, isdX), tar_w statistics in (zY, isdY).
// Levels [d_first, d_end) (d_end < 0: all D), written to slice d - d_first.
// quad = 1: level-quad-interleaved float4 layout [levels/4][H][out_pitch]
// (out_slice, out_pitch in float4 units; d_first a multiple of 4).  quad = 2:
// split-FP16 volume of the anchor (see BilArgs::h2), out_pitch = stored
// columns (a multiple of 8), out_slice = 16 H out_pitch, out_w >= out_pitch,
// pad = column shift (the window radius R), d_first a multiple of 16.
// quad = 3 (FP32 images): both the split-FP16 volume in C (as quad 2) and
// the planar FP32 volume [levels][H][W] in C2, from one pass.  quad = 4:
// the reference-anchored split volume in C and the target-anchored one in
// C2 (nullable) from one pass; out_w = ncc_both_extent(out_pitch, ...).
hipError_t launch_ncc(const Plan& P, const void* ref, const float* tar_w,
                      const float* zX, const float* isdX, const float* zY,
                      const float* isdY, float* C, int out_w, int64_t out_pitch,
                      int64_t out_slice, int anchor, hipStream_t s, int d_first = 0,
                      int d_end = -1, int quad = 0, int pad = 0, float* C2 = nullptr);

struct BilArgs {
  const float* C;     // planar: C[d * c_slice + y * c_pitch + x + d*shift]
  int64_t c_slice;    // quad: component d % 4 of float4
  int64_t c_pitch;    //   C4[(d / 4) * c_slice + y * c_pitch + x + d*shift]
  int shift;          // 1: slice d is read from column x + d (target volume)
  int quad;           // 1: level-quad-interleaved layout (c_* in float4 units)
  const void* guide;  // guide image
  stereo_dtype guide_dt;
  int64_t guide_pitch;
  float* E;           // modes 0, 4: output volume [levels][H][W]
  int16_t* dint;      // mode 1: WTA level [H][W]
  float* dsub;        // mode 1: sub-pixel level [H][W] (nullable)
  float* sm_m;        // mode 2: softmax state and outputs [H][W]
  float* sm_logZ;
  float* sm_dh;
  float* disp;
  double plane[3];    // mode 2: plane of the shift back
  int levels;         // number of levels in C (0: plan D)
  // modes 5, 6 (backward of the soft-argmin head over one level tile):
  const float* gD;    // mode 5: gradient of the shifted soft disparity [H][W]
  const float* cpix;  // mode 6: the tile's cost volume (planar, as C of mode 5)
  float* aP;          // mode 5: += sum_d dE E            [H][W]
  float* A1;          // mode 5: += sum_q w (G(p)-G(q)) sum_d dE(p,d) C(q,d)
  float* A2;          // mode 6: += sum_q w (G(q)-G(p)) sum_d dE(q,d)/W_q C(p,d)
  float* Wp;          // mode 5 (nullable): sum_q w(p, q)
  int d_first;        // modes 5, 6: level of the tile's first slice
  // split-FP16 volume of the matrix-core engine with FP16 operands (modes 1,
  // 2; used when non-NULL), in blocks of 16 levels: level d of column x at
  // h2[(2 (d >> 4) + part) * h2_plane + 16 y h2_pitch + 64 (s >> 2) +
  // 4 (d & 15) + (s & 3)], s = x + R; part 0 = FP16 value c_hi of the cost,
  // part 1 = FP16 value of c - c_hi; columns outside [0, W) and the last
  // block's levels past D hold zeros
  const uint16_t* h2;
  int64_t h2_plane;   // halves per block part (>= 16 H h2_pitch)
  int h2_pitch;       // columns per stored row (a multiple of 8)
  // backward passes on the split-FP16 matrix cores: max |g'| (float bits),
  // and pass 1's output volume (C' scaled, split; pitch and plane of h2)
  const unsigned int* gmax;
  uint16_t* h2_out;
};
// mode 0: write the normalised aggregated volume; mode 1: fused WTA and
// sub-pixel refinement (the volume never leaves the chip); mode 2: fused
// soft-argmin (soft level, softmax state, shifted disparity); mode 4: the
// unnormalised weighted sum sum_q w(p, q) C(q, d) (adjoint gather); modes 5
// and 6: the two passes of the soft-argmin backward per level tile (mode 5:
// E, the softmax adjoint dE, E out = dE / W_p, aP and A1; mode 6 on C = dE/W:
// E out = dC = sum_q w C, and A2), float guides only.
hipError_t launch_bilateral(const Plan& P, const BilArgs& a, int mode,
                            hipStream_t s);

// Backward of the soft-argmin head on the split-FP16 matrix cores, for one
// level tile (radius R <= kBwd16MaxR, float guide, d_first a multiple of 16):
// pass 1 reads the tile's split costs (a.h2) and writes C' = dE / W_p, times
// a power of two set by the bound max |g'| |1 - c1| (D - 1) / T (*a.gmax =
// max |g'| as float bits), split into a.h2_out (same layout), with aP, A1,
// Wp as mode 5; pass 2 reads that volume (a.h2) and writes dC planar
// [levels][H][W] to a.E and A2 as mode 6 (a.cpix: the tile's costs, planar).
// The stored columns of a.h2_out outside the image are not written: zero
// them first (launch_h2_pad_zero).
constexpr int kBwd16MaxR = 5;
hipError_t launch_bilateral_bwd16(const Plan& P, const BilArgs& a, int pass, hipStream_t s);
// Zeros in the stored columns outside [0, W) (all levels, both halves) of
// the first nblk 16-level blocks of a split-FP16 volume at radius R.
hipError_t launch_h2_pad_zero(uint16_t* h2, int64_t plane, int pitch, int W, int H, int R,
                              int nblk, hipStream_t s);

// Row pitch (halves, a multiple of 8) of the split-FP16 volumes at window
// radius R for width W: covers the halo columns of every 16-pixel tile.
int h2_pitch(int R, int W);
// Columns (and so blocks) of a batched NCC job: the extended range
// [0, W + D - 1) of the quad volume or the stored row of a split-FP16 volume.
inline int ncc_out_w(const Plan& P) {
  const int ext = P.W + P.D - 1;
  return ext > P.h2_pitch ? ext : P.h2_pitch;
}

// Persistent aggregation (mode 1, fused WTA) over a queue of tiles of many
// pairs: pairs = device array of per-pair descriptors (bilateral_pair), tiles
// = device int triples (pair, x0, y0), counter = device uint zeroed before the
// launch.  All pairs of one launch share R, the guide type and `levels`.
// engine 1 (matrix cores): tiles of kMfmaTileW x kMfmaTileH, one workgroup
// per CU; engine 0 (vector ALU): tiles of kBilTileW x kBilTileH.
hipError_t launch_bilateral_persistent(int engine, int R, stereo_dtype gdt, int levels, const void* pairs,
                                       const int* tiles, int n_tiles, unsigned int* counter,
                                       int n_groups, hipStream_t s);
size_t bilateral_pair_bytes();
void* bilateral_pair(const Plan& P, const BilArgs& a, void* out);
constexpr int kBilTileW = 32, kBilTileH = 32;   // pixels per aggregation tile
constexpr int kMfmaTileW = 16, kMfmaTileH = 12; // the same on the matrix cores

hipError_t launch_wta(const Plan& P, const float* E, int16_t* dint,
                      float* dsub, hipStream_t s);
hipError_t launch_lr_check(const Plan& P, const int16_t* dR, const int16_t* dT,
                           const float* dsub, uint8_t* valid, float* disp,
                           hipStream_t s);
hipError_t launch_lr_check_tracked(const Plan& P, const int16_t* dR, const int16_t* dT,
                                   const float* dsub, const stereo_plane_state* st,
                                   uint8_t* valid, float* disp, hipStream_t s);

// ---- batched stages: one launch covers every job of a list.  Job j owns
// blocks [first[j], first[j+1]) of the launch (first[0] = 0, first[n] = the
// launch's block count) and runs exactly the per-pair kernel's code on its own
// block grid, so a batched result is bitwise the per-pair one.
struct Homog {              // row-major 3x3, by value in kernel arguments
  double h[9];
};
struct WarpJob {            // grid: gx = ceil(W / 256) x H rows
  const void* tar; int64_t pitch; float* out;
  double dp, c0, c1, c2;
  int W, H, persp, gx;
  int homog;                // 1: by Hm (Eq. 3) instead of the plane
  Homog Hm;
};
struct StatsJob {           // grid: gx = ceil((W + 2r) / 64) x ceil(H / 16)
  const void* img; int64_t pitch; float* z; float* isd;
  int W, H, r, gx;
};
struct NccJob {             // grid: gx = ceil(out_w / 64) x gy = ceil(H / 32) x level blocks
  const void* ref; int64_t ref_pitch; const float* tarw;
  const float *zX, *isdX, *zY, *isdY;
  float* C; int64_t out_pitch, out_slice;
  int W, H, d_first, d_end, out_w, anchor, gx, gy;
  int pad;                    // split-FP16 output (quad = 2, 4): column shift
  float* C2;                  // quad = 4: the target-anchored volume (nullable)
  // the kernel reaches C and C2 as byte offsets from the launch's base (a
  // kernel argument, so the compiler knows the stores are global); c2_off
  // < 0: no C2
  int64_t c_off, c2_off;
};
struct LrJob {              // grid: gx = ceil(W / 256) x H rows
  const int16_t* dR; const int16_t* dT; const float* dsub; uint8_t* valid; float* disp;
  double dp, c0, c1, c2;
  float lr_delta;
  int W, H, use_lr, persp, gx;
  int homog;
  Homog Hm;
};
int warp_job_blocks(const Plan& P);
int stats_job_blocks(int W, int H, int r);
int ncc_job_blocks(const Plan& P, int out_w, int d_first, int d_end, int dc, int quad);
// Columns a quad = 4 launch covers (its out_w): the stored row plus the
// levels rounded up to 16, so that every target-anchored column is reached.
int ncc_both_extent(int out_pitch, int d_first, int d_end);
int lr_job_blocks(const Plan& P);
WarpJob warp_job(const Plan& P, const void* tar, float* tar_w);
StatsJob stats_job(const Plan& P, const void* img, int64_t pitch, float* z, float* isd);
NccJob ncc_job(const Plan& P, const void* ref, const float* tar_w, const float* zX,
               const float* isdX, const float* zY, const float* isdY, float* C, int out_w,
               int64_t out_pitch, int64_t out_slice, int anchor, int d_first, int d_end,
               int quad, float* C2, const void* base);
LrJob lr_job(const Plan& P, const int16_t* dR, const int16_t* dT, const float* dsub,
             uint8_t* valid, float* disp);
// jobs / first are device arrays; dt is the element type of the job images
// (ref for the NCC); stats LDS is sized for max_r; quad as in launch_ncc.
hipError_t launch_warp_jobs(stereo_dtype dt, const WarpJob* jobs, const int* first, int n,
                            int blocks, hipStream_t s);
hipError_t launch_stats_jobs(stereo_dtype dt, const StatsJob* jobs, const int* first, int n,
                             int blocks, int max_r, hipStream_t s);
// dc: levels per workgroup (16, 32 or 64), the same for every job of the list
// base: the allocation holding every job's C and C2 (their offsets)
hipError_t launch_ncc_jobs(int r, stereo_dtype dt, int quad, int dc, const NccJob* jobs,
                           const int* first, int n, int blocks, char* base, hipStream_t s);
hipError_t launch_lr_jobs(const LrJob* jobs, const int* first, int n, int blocks,
                          hipStream_t s);
// Per-radius NCC instantiation units (k_ncc_rN.hip): launch_ncc and
// launch_ncc_jobs dispatch on the plan's radius to these.
#define STEREO_NCC_UNIT(N)                                                                     \
  hipError_t launch_ncc_r##N(const Plan& P, const void* ref, const float* tar_w,              \
                             const float* zX, const float* isdX, const float* zY,            \
                             const float* isdY, float* C, int out_w, int64_t out_pitch,      \
                             int64_t out_slice, int anchor, int d_first, int d_end,          \
                             int quad, int pad, hipStream_t s, float* C2);                   \
  hipError_t launch_ncc_jobs_r##N(stereo_dtype dt, int quad, int dc, const NccJob* jobs,     \
                                  const int* first, int n, int blocks, char* base,          \
                                  hipStream_t s);
STEREO_NCC_UNIT(1) STEREO_NCC_UNIT(2) STEREO_NCC_UNIT(3) STEREO_NCC_UNIT(4)
STEREO_NCC_UNIT(5) STEREO_NCC_UNIT(6) STEREO_NCC_UNIT(7) STEREO_NCC_UNIT(8)
#undef STEREO_NCC_UNIT

// Grad workspace layout for the plan (sets g_off / g_end); 0 for U8 plans.
size_t grad_layout(Plan& P, size_t base);

hipError_t launch_damage_mask(const Plan& P, const float* disp_t, float delta_t, float tau,
                              uint8_t* mask, hipStream_t s);

// Device address and size of this device's fixed road-transform buffer
// (allocation-free entry point); looked up once per device.
constexpr int kMaxDevices = 64;
constexpr int kRoadScratchDoubles = 10 * 1024;
hipError_t road_scratch(double** out, size_t* bytes);

hipError_t launch_road(const Plan& P, const float* disp, const uint8_t* mask,
                       double psi0, double lambda0, double delta_psi,
                       int max_iter, float delta_t, stereo_road_fit* fit,
                       float* disp_t, double* partials, hipStream_t s,
                       stereo_plane_state* state = nullptr);

}  // namespace stereo

namespace stereo {
// Batch introspection for the autotuner: pair count and (W, H, D, r, R, dtype).
int batch_pair_count(stereo_batch_t b);
void batch_pair_shape(stereo_batch_t b, int i, int32_t* shape6);
}  // namespace stereo

// The opaque plan handle of the C ABI.
struct stereo_plan_s {
  stereo::Plan P;
};
