/*
 * stereo.h -- C ABI of the MI355X (gfx950) road-stereo library.
 *
 * The library implements the dense road stereo method of Fan et al.,
 * "Real-Time Dense Stereo Embedded in A UAV for Road Inspection"
 * (arXiv 1904.06017):
 *   perspective transformation of the target image   (Sec. 3.1, Eq. 4)
 *   NCC matching costs for two cost volumes          (Sec. 3.2.1, Eq. 8)
 *   bilateral cost aggregation                       (Sec. 3.2.1, Eqs. 10-11)
 *   winner-take-all, left-right check, sub-pixel     (Sec. 3.2.2, Eqs. 12-13)
 *   roll-angle fit and disparity transformation      (Sec. 3.3, Eqs. 14-29)
 * plus a differentiable soft-argmin head with its adjoint and a batched
 * persistent launch over many pairs.
 *
 * Conventions (apply to every call unless stated otherwise)
 *   - Every call returns a stereo_status; nothing throws across the ABI.
 *     stereo_last_error() returns a thread-local message for the last failure.
 *   - The caller owns every buffer.  Device buffers are plain device pointers
 *     (e.g. from hipMalloc or a framework allocator).  Inputs are const and
 *     never written; outputs are fully overwritten.
 *   - Images are row-major [H][W] with an element pitch >= W.  Disparity maps
 *     and other per-pixel outputs are dense [H][W] (pitch W).  Cost volumes
 *     are dense FP32 [D][H][W], slice d at offset d*H*W.
 *   - Enqueue calls are asynchronous on the given stream, allocate nothing and
 *     never synchronise the host, so they can be captured into a hipGraph.
 *     Device faults surface at the next synchronisation of that stream.
 *   - A plan is immutable host state; one plan may be used from several
 *     streams at once provided each stream uses its own workspace.
 *   - Coordinates: u (column) grows to the right, v (row) downwards, origin at
 *     the top-left pixel.  Disparity levels d' = 0..D-1 are searched after the
 *     perspective transformation; the residual disparity is d' - delta_p.
 */
#ifndef MI355X_ROAD_STEREO_H
#define MI355X_ROAD_STEREO_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  STEREO_OK = 0,
  STEREO_ERR_INVALID_ARGUMENT = 1,   /* null pointer, bad size, bad parameter */
  STEREO_ERR_UNSUPPORTED = 2,        /* radius / D above the compiled limits  */
  STEREO_ERR_WORKSPACE_TOO_SMALL = 3,
  STEREO_ERR_HIP = 4,                /* a HIP runtime call or launch failed   */
  STEREO_ERR_NOT_CONVERGED = 5       /* road fit hit max_iter; outputs written */
} stereo_status;

typedef enum { STEREO_U8 = 0, STEREO_F32 = 1 } stereo_dtype;

/* Compiled limits. */
#define STEREO_MAX_NCC_RADIUS 8      /* r: NCC block (2r+1)^2                */
#define STEREO_MIN_BIL_RADIUS 1
#define STEREO_MAX_BIL_RADIUS 8      /* R: bilateral window (2R+1)^2          */
#define STEREO_MAX_DISP 256          /* D                                     */

typedef struct {
  int32_t width, height;          /* W, H >= 1                               */
  int64_t pitch_ref, pitch_tar;   /* elements per image row, >= width        */
  stereo_dtype dtype;             /* pixel type of ref and tar               */
  int32_t num_disp;               /* D >= 3 disparity levels                 */
  float delta_p;                  /* delta_p of Sec. 3.1 (0 without warp)    */
  int32_t perspective;            /* 1: warp the target by the road plane    */
  double plane[3];                /* d_road(u,v) = c0 + c1 u + c2 v, pixels  */
  int32_t ncc_radius;             /* r, 1..STEREO_MAX_NCC_RADIUS             */
  int32_t bil_radius;             /* R, 1..STEREO_MAX_BIL_RADIUS             */
  float sigma_s, sigma_r;         /* sigma_0, sigma_1 of Eq. (10), > 0       */
  float lr_delta;                 /* delta_r of Eq. (12) (paper: 1)          */
  int32_t lr_check;               /* 1: build the target volume and check    */
  float softargmin_T;             /* temperature of the soft-argmin head > 0 */
} stereo_params;

typedef struct stereo_plan_s* stereo_plan_t;

/* Result of the road fit (Sec. 3.3); written to device memory. */
typedef struct {
  double psi;        /* roll angle, (-pi/2, pi/2]                            */
  double alpha0;     /* Eq. (21) at psi                                      */
  double alpha1;
  double e_min;      /* Eq. (23) at psi (unnormalised)                       */
  double plane[3];   /* (alpha0, -alpha1 sin psi, alpha1 cos psi)            */
  double n_points;   /* pixels used by the fit                               */
  int32_t iters;
  int32_t converged; /* 1 converged, 0 hit max_iter                          */
  int32_t flat;      /* 1 if |alpha1(psi0)| < 1e-6: psi returned unchanged    */
  int32_t pad_;
} stereo_road_fit;

/* ---- status ------------------------------------------------------------ */
const char* stereo_status_string(stereo_status s);
/* Message for the last failing call on this thread ("" if none). */
const char* stereo_last_error(void);
/* Library version string. */
const char* stereo_version(void);

/* ---- plans (host only; no device calls) ---------------------------------
 * stereo_plan_create validates *params (copied) and returns a plan, or
 * INVALID_ARGUMENT / UNSUPPORTED.  stereo_plan_workspace_bytes reports the
 * device workspace every enqueue call of this plan needs (one size for all).
 * stereo_plan_destroy accepts NULL. */
stereo_status stereo_plan_create(const stereo_params* params, stereo_plan_t* out);
stereo_status stereo_plan_destroy(stereo_plan_t plan);
stereo_status stereo_plan_workspace_bytes(stereo_plan_t plan, size_t* bytes);
stereo_status stereo_plan_get_params(stereo_plan_t plan, stereo_params* out);

/* ---- general homography warp, Eq. (3) (host only) ----------------------------
 * Replaces the row shift of the plan's plane by the full homography H
 * (row-major 3x3, reference pixel -> target pixel, Eq. 3): the warped target
 * at (x, v) is the target read bilinearly (clamped) at H (x + delta_p, v, 1),
 * and the shift back gives disp(u, v) = u - X with (X, Y) = H (u - l +
 * delta_p, v, 1), the column of the correspondence in the target.  For rigs
 * outside the rectified hypotheses of Sec. 3.1.  The plan must have
 * perspective = 1; H must be finite with a positive third row over the
 * reference columns [delta_p - D + 1, W - 1 + delta_p] x rows [0, H - 1]
 * (checked at the corners).  H = NULL restores the plane's row shift.  Plans
 * with a homography work with stereo_warp, stereo_match (plain and batched);
 * the tracked and differentiable entry points reject them. */
stereo_status stereo_plan_set_homography(stereo_plan_t plan, const double* H);

/* ---- tuning knobs (host only) ---------------------------------------------
 * Launch-shape choices.  Keys:
 *   "agg_engine": the kernel of the fused aggregation and selection
 *   (stereo_match, Eq. 9-11 and 13) and of the soft-argmin forward
 *   (stereo_soft_forward): 2 (default) the matrix cores with FP16 operands
 *   split in two (each cost and weight carried as the sum of two FP16
 *   numbers, three FP16 products per term, FP32 accumulation: as accurate
 *   as FP32 products), 1 the matrix cores with FP32 operands, 0 the vector
 *   ALU.  With 2 the NCC stage writes the reference- and target-anchored
 *   volumes in that split form; with 0 and 1 one FP32 volume.  The engines
 *   sum in different orders, so they agree to FP32 rounding (a disparity
 *   can differ at a near tie), not bit for bit;
 *   "agg_levels_u8", "agg_levels_f32": disparity levels staged per pass of
 *   the vector-ALU aggregation kernel for 8-bit / float guides, 8 or 16
 *   (default 8); results are bitwise identical for every value;
 *   "ncc_levels": disparity levels per workgroup of the NCC cost kernel, 16,
 *   32 or 64, or 0 (default: the smallest of 16, 32, 64 that holds the
 *   launch's levels, else 64); results are bitwise identical for every value;
 *   "grad_levels": levels recomputed per tile by stereo_backward, a multiple
 *   of 4 in 4..64 (default: num_disp rounded up to a multiple of 4, at most
 *   64); changes the workspace size and the FP32 summation order of the
 *   gradients (not their value beyond rounding).
 * Unknown keys and values give INVALID_ARGUMENT.  Not thread-safe against
 * concurrent enqueues on the same plan. */
stereo_status stereo_plan_set_tuning(stereo_plan_t plan, const char* key, int32_t value);
stereo_status stereo_plan_get_tuning(stereo_plan_t plan, const char* key, int32_t* value);

/* ---- perspective transformation, Sec. 3.1, Eq. (4) ----------------------
 * tar: [H][pitch_tar] of params.dtype.  tar_w: [H][W] FP32.
 * tar_w(x,v) = lerp of row v at X = x + delta_p - d_road(x + delta_p, v),
 * X clamped to [0, W-1].  Without perspective, tar_w = tar (converted). */
stereo_status stereo_warp(stereo_plan_t plan, const void* tar, float* tar_w,
                          hipStream_t stream);

/* ---- NCC cost volumes, Sec. 3.2.1, Eq. (8) ------------------------------
 * ref: [H][pitch_ref] of params.dtype; tar_w: [H][W] FP32 (stereo_warp).
 * cost_R[d][v][u] = 1 - NCC(ref block at (u,v), tar_w block at (u-d,v));
 * cost_T[d][v][x] = 1 - NCC(ref block at (x+d,v), tar_w block at (x,v))
 * (nullable).  Blocks are (2r+1)^2 with clamped reads; population
 * statistics; a block with variance < 1e-6 has cost 1. */
stereo_status stereo_cost_volume(stereo_plan_t plan, const void* ref,
                                 const float* tar_w, float* cost_R,
                                 float* cost_T, void* ws, size_t ws_bytes,
                                 hipStream_t stream);

/* ---- bilateral aggregation, Eqs. (10)-(11) ------------------------------
 * cost_out[d][p] = sum_q w(p,q) cost_in[d][q] / sum_q w(p,q) over the
 * (2R+1)^2 window truncated to the image, w = exp(-|p-q|^2/sigma_s^2
 * - (G(p)-G(q))^2/sigma_r^2).  guide: [H][guide_pitch] of guide_dtype (the
 * reference image for the reference volume, tar_w for the target volume). */
stereo_status stereo_bilateral_aggregate(stereo_plan_t plan, const void* guide,
                                         stereo_dtype guide_dtype,
                                         int64_t guide_pitch,
                                         const float* cost_in, float* cost_out,
                                         hipStream_t stream);

/* ---- winner-take-all + sub-pixel, Sec. 3.2.2, Eq. (13) ------------------
 * dint[p] = first argmin_d agg[d][p] (int16).  dsub (nullable, FP32):
 * dint + (E(d-1) - E(d+1)) / (2E(d-1) + 2E(d+1) - 4E(d)) where 0 < d < D-1
 * and the denominator is > 0, else dint. */
stereo_status stereo_wta_subpixel(stereo_plan_t plan, const float* agg,
                                  int16_t* dint, float* dsub,
                                  hipStream_t stream);

/* ---- left-right check + shift back, Eq. (12), Sec. 3.2.2 ----------------
 * valid[p] = (u - dR >= 0) && (dR - dT(u - dR, v))^2 <= lr_delta (uint8 0/1).
 * disp[p] = dsub - delta_p + d_road(u - dsub + delta_p, v) where valid, NaN
 * elsewhere (dsub itself when perspective = 0).  dint_T may be NULL only
 * when params.lr_check = 0 (then valid = (u - dR >= 0)). */
stereo_status stereo_lr_check(stereo_plan_t plan, const int16_t* dint_R,
                              const int16_t* dint_T, const float* dsub_R,
                              uint8_t* valid, float* disp, hipStream_t stream);

/* ---- whole plain forward (warp .. shift back), fused where it pays ------
 * Same results as stereo_warp, stereo_cost_volume, stereo_bilateral_aggregate
 * (twice), stereo_wta_subpixel and stereo_lr_check in sequence, without
 * materialising the aggregated volumes.  dint_T and dsub may be NULL. */
stereo_status stereo_match(stereo_plan_t plan, const void* ref, const void* tar,
                           int16_t* dint_R, int16_t* dint_T, float* dsub,
                           uint8_t* valid, float* disp, void* ws,
                           size_t ws_bytes, hipStream_t stream);

/* ---- the same, recording caller-owned events at the stage boundaries ---
 * ev: 7 events created by the caller (hipEventCreate), recorded on `stream`:
 * [0] start, [1] after the warp, [2] after the block statistics, [3] after
 * the NCC volume, [4] after aggregation + WTA of the reference volume, [5]
 * after that of the target volume, [6] after the left-right check.  For
 * profiling; results are identical to stereo_match. */
#define STEREO_MATCH_EVENTS 7
stereo_status stereo_match_profiled(stereo_plan_t plan, const void* ref, const void* tar,
                                    int16_t* dint_R, int16_t* dint_T, float* dsub,
                                    uint8_t* valid, float* disp, void* ws,
                                    size_t ws_bytes, hipEvent_t* ev, hipStream_t stream);

/* ---- road fit + disparity transformation, Sec. 3.3, Eqs. (14)-(29) ------
 * disp: [H][W] FP32 (NaN = invalid); mask: [H][W] uint8 (nullable: all).
 * Fits the roll psi by gradient descent (Eq. 25) with the adaptive rate of
 * Eq. (28) from psi_init, on the energy normalised by n*max(W,H)^2*a1(psi0)^2;
 * stops when |dpsi| < delta_psi or after max_iter steps.  Writes *fit_dev
 * (device memory) and disp_t = disp - a0 + a1 (u sin psi - v cos psi)
 * + delta_t (NaN stays NaN).  Returns OK even when the fit did not converge;
 * read fit_dev->converged.  No host synchronisation. */
stereo_status stereo_road_transform(stereo_plan_t plan, const float* disp,
                                    const uint8_t* mask, double psi_init,
                                    double lambda0, double delta_psi,
                                    int32_t max_iter, float delta_t,
                                    stereo_road_fit* fit_dev, float* disp_t,
                                    void* ws, size_t ws_bytes,
                                    hipStream_t stream);

/* ---- the road transform without a workspace -------------------------------
 * For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): stereo_road_transform
 * with its reduction partials (10 FP64 per reduction block, 240 blocks,
 * 19200 bytes) in a fixed device buffer of 80 KiB that the library holds on
 * every device it runs on until the process ends.  Allocates nothing and
 * never synchronises; same arguments, semantics and bitwise results as
 * stereo_road_transform.  Returns UNSUPPORTED if the plan's partials exceed
 * the buffer.  Calls that overlap on one device (several streams or host
 * threads at once) share the buffer and race: serialise them. */
stereo_status stereo_road_transform_noalloc(stereo_plan_t plan, const float* disp,
                                            const uint8_t* mask, double psi_init,
                                            double lambda0, double delta_psi,
                                            int32_t max_iter, float delta_t,
                                            stereo_road_fit* fit_dev, float* disp_t,
                                            hipStream_t stream);

/* ---- closed-loop plane tracking over a frame sequence ----------------------
 * The road fit of frame t (Sec. 3.3) gives the plane c = (alpha0,
 * -alpha1 sin psi, alpha1 cos psi) that frame t+1's perspective
 * transformation (Sec. 3.1) and shift back use, and its psi warm-starts frame
 * t+1's fit (the paper seeds each fit from the previous estimate).  The state
 * lives in device memory, so a tracked frame needs no host synchronisation
 * and can be captured in a graph.  The caller initialises it (for instance
 * from a fit of a full-range pass without the perspective transformation:
 * copy stereo_road_fit.plane and .psi, frames = 0). */
typedef struct {
  double plane[3];   /* (c0, c1, c2): the plane the next frame is matched with  */
  double psi;        /* warm start of the next roll fit                        */
  int32_t frames;    /* fits folded into the state so far                      */
  int32_t pad_;
} stereo_plane_state;   /* 40 bytes */

/* stereo_match with the plane of *state_dev (device memory) in place of the
 * plan's; the plan must have perspective = 1 (its delta_p, ranges and radii
 * apply).  Outputs and workspace as stereo_match. */
stereo_status stereo_match_tracked(stereo_plan_t plan, const void* ref, const void* tar,
                                   const stereo_plane_state* state_dev, int16_t* dint_R,
                                   int16_t* dint_T, float* dsub, uint8_t* valid, float* disp,
                                   void* ws, size_t ws_bytes, hipStream_t stream);

/* stereo_road_transform with psi_init = state_dev->psi; afterwards, if the
 * fit is not flat (>= 3 points and |alpha1| >= 1e-6), the state takes the
 * fitted plane and psi and frames += 1; otherwise it is left unchanged. */
stereo_status stereo_road_transform_tracked(stereo_plan_t plan, const float* disp,
                                            const uint8_t* mask, double lambda0,
                                            double delta_psi, int32_t max_iter,
                                            float delta_t, stereo_plane_state* state_dev,
                                            stereo_road_fit* fit_dev, float* disp_t,
                                            void* ws, size_t ws_bytes, hipStream_t stream);

/* ---- road damage on the transformed map, Sec. 4.4.3 -----------------------
 * After Eq. (29) the road surface is flat at delta_t and damage (potholes,
 * cracks: farther away, smaller disparity) lies below it.  Writes
 * mask[p] = 1 where disp_t[p] is finite and disp_t[p] < delta_t - tau, else 0
 * (the comparison in FP32, with delta_t - tau rounded to FP32 once).
 * disp_t: [H][W] FP32 as written by stereo_road_transform; mask: [H][W]
 * uint8, caller-owned.  tau > 0 is the depth threshold in pixels of
 * disparity.  No workspace, no host synchronisation. */
stereo_status stereo_damage_mask(stereo_plan_t plan, const float* disp_t, float delta_t,
                                 float tau, uint8_t* mask, hipStream_t stream);

/* ---- batched form ----------------------------------------------------------
 * Many pairs of uneven size and disparity range (each with its own plan) in
 * one workspace and one captured graph.  Per pair, results are bitwise those
 * of stereo_match with the same plan.  The aggregation + WTA of both volumes
 * of all pairs runs as one persistent launch per (R, guide type) group that
 * takes 32x32 tiles of all pairs from a work queue, largest range first. */
typedef struct stereo_batch_s* stereo_batch_t;
typedef struct {
  stereo_plan_t plan;      /* the pair's plan (copied at create)                */
  const void* ref;         /* device images as described by the plan           */
  const void* tar;
  int16_t* dint_R;         /* device outputs [H][W]; valid / disp nullable      */
  uint8_t* valid;
  float* disp;
} stereo_batch_item;

/* Host only: copies the items, groups the tiles, sizes the workspace. */
stereo_status stereo_batch_create(const stereo_batch_item* items, int32_t n,
                                  stereo_batch_t* out);
stereo_status stereo_batch_workspace_bytes(stereo_batch_t b, size_t* bytes);
/* Tuning keys: "agg_engine" (as for a plan: 2, default, 1 or 0; a batch
 * gives the same bits as its pairs' stereo_match when both use the same
 * engine), "wg_per_cu" (persistent workgroups per CU of
 * the vector-ALU engine, 1..8, default 2), "agg_levels_u8", "agg_levels_f32"
 * (8 or 16), "tile_band" (matrix-core engines: the tile list of a pair runs
 * in bands of this many 16-pixel tile columns, row by row; 1, 2, 4, 8, 16
 * or 32, default 4; changes only the order of independent tiles, never the
 * results), "ncc_levels" (levels per workgroup of the batch's NCC launches:
 * 0 = automatic, default, or 16, 32, 64; never changes the results),
 * "group_overlap" (split-FP16 engine: 1, default, runs the aggregation of
 * the radii below the largest on a second stream, a graph branch when
 * captured, beside the NCC of the largest radius; 0 runs every stage in
 * order; never changes the results).  Drops an instantiated graph. */
stereo_status stereo_batch_set_tuning(stereo_batch_t b, const char* key, int32_t value);
stereo_status stereo_batch_get_tuning(stereo_batch_t b, const char* key, int32_t* value);
/* Enqueue the whole batch on `stream` (no graph).  The first call with a given
 * workspace uploads the per-pair descriptors and synchronises the stream. */
stereo_status stereo_submit_batch(stereo_batch_t b, void* ws, size_t ws_bytes,
                                  hipStream_t stream);
/* The same, recording caller-owned events on `stream` around the persistent
 * aggregation launches (Eqs. 10-11 with the fused selection of Eq. 13, all
 * groups): ev[0] before the first, ev[1] after the last.  For profiling. */
stereo_status stereo_submit_batch_profiled(stereo_batch_t b, void* ws, size_t ws_bytes,
                                           hipEvent_t* ev, hipStream_t stream);
/* Upload the descriptors (synchronising `stream`) and capture the batch into a
 * graph bound to `ws`; stereo_batch_launch replays it on any stream. */
stereo_status stereo_batch_instantiate(stereo_batch_t b, void* ws, size_t ws_bytes,
                                       hipStream_t stream);
stereo_status stereo_batch_launch(stereo_batch_t b, hipStream_t stream);
stereo_status stereo_batch_destroy(stereo_batch_t b);

/* ---- autotuner ---------------------------------------------------------------
 * Times the launch-shape variants on the caller's inputs (HIP events, median
 * of `reps` runs, synchronous), applies the fastest and stores it in the JSON
 * file cache_path (nullable: no cache) keyed by GPU architecture, problem
 * shape and aggregation engine; a cached choice is applied without timing.
 * Plans: "ncc_levels" (16, 32, 64), and with agg_engine = 0 also
 * "agg_levels_u8" / "agg_levels_f32"; batches: with agg_engine = 0
 * "wg_per_cu" and the levels per pass, with the matrix-core engines
 * "tile_band" (2, 4, 8, 16), "ncc_levels" (16, 32, 64) and, with the
 * split-FP16 engine, "group_overlap" (0, 1).  best_ms (nullable) receives
 * the time of the chosen variant.  Results never depend on the variant.
 * stereo_plan_autotune allocates temporary outputs (hipMalloc). */
stereo_status stereo_plan_autotune(stereo_plan_t plan, const void* ref, const void* tar,
                                   void* ws, size_t ws_bytes, hipStream_t stream,
                                   const char* cache_path, int32_t reps, double* best_ms);
stereo_status stereo_batch_autotune(stereo_batch_t b, void* ws, size_t ws_bytes,
                                    hipStream_t stream, const char* cache_path, int32_t reps,
                                    double* best_ms);

/* ---- differentiable form (F32 plans, perspective = 1) --------------------
 * Soft-argmin head over the aggregated reference volume E_R (Eqs. 8-11):
 *   P(p,d) = softmax_d(-E_R(p,d) / T),  dh(p) = sum_d d P(p,d),
 *   disp_soft(p) = dh - delta_p + d_road(u - dh + delta_p, v).
 * plane: host double[3], the road plane of the warp and of the shift back for
 * this call (the parameter being learned; params.plane is not used).
 * disp_soft: [H][W] FP32.  saved: [3][H][W] FP32 = (max_d(-E/T), log of the
 * softmax normaliser, dh) -- everything the backward needs; the cost volume
 * itself is not kept. */
stereo_status stereo_soft_forward(stereo_plan_t plan, const float* ref, const float* tar,
                                  const double plane[3], float* disp_soft, float* saved,
                                  void* ws, size_t ws_bytes, hipStream_t stream);

/* Vector-Jacobian product of disp_soft with grad_disp ([H][W] FP32): writes
 * grad_ref, grad_tar ([H][W] FP32) and grad_plane (device double[3]).  The cost
 * and aggregated volumes are recomputed per tile of "grad_levels" levels (a
 * tuning key; by default all levels up to 64 form one tile).  Gradients flow through the aggregation weights
 * (guide = ref), the NCC cost of both images, the warp and the shift back.
 * Deterministic: gathers in a fixed order, and fixed-point integer sums
 * (scale 2^44) where the warp scatters into the target image, so per-pixel
 * contributions must stay below 2^19 in magnitude. */
stereo_status stereo_backward(stereo_plan_t plan, const float* ref, const float* tar,
                              const double plane[3], const float* saved,
                              const float* grad_disp, float* grad_ref, float* grad_tar,
                              double* grad_plane, void* ws, size_t ws_bytes,
                              hipStream_t stream);
/* The same, recording caller-owned events on `stream` (for profiling;
 * results identical): ev[0] start, ev[1] before the first level tile's first
 * aggregation pass (Eq. 11 and the softmax adjoint), ev[2] after it, ev[3]
 * before its second pass (the adjoint of Eq. 11's sum), ev[4] after it, ev[5]
 * end.  With one level tile (D <= 64 by default) [1, 2] and [3, 4] time the
 * two aggregation passes of the whole backward. */
#define STEREO_BACKWARD_EVENTS 6
stereo_status stereo_backward_profiled(stereo_plan_t plan, const float* ref, const float* tar,
                                       const double plane[3], const float* saved,
                                       const float* grad_disp, float* grad_ref, float* grad_tar,
                                       double* grad_plane, void* ws, size_t ws_bytes,
                                       hipEvent_t* ev, hipStream_t stream);

/* Photometric L1 loss L = mean_p |ref(p) - lerp(tar, v, u - disp_soft(p))|
 * (row lerp, clamped), written to *loss_dev (device double).  The _bwd call
 * writes dL/dref, dL/dtar, dL/ddisp times grad_loss (each nullable). */
stereo_status stereo_photometric_l1(stereo_plan_t plan, const float* ref, const float* tar,
                                    const float* disp_soft, double* loss_dev, void* ws,
                                    size_t ws_bytes, hipStream_t stream);
stereo_status stereo_photometric_l1_bwd(stereo_plan_t plan, const float* ref,
                                        const float* tar, const float* disp_soft,
                                        double grad_loss, float* g_ref, float* g_tar,
                                        float* g_disp, void* ws, size_t ws_bytes,
                                        hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* MI355X_ROAD_STEREO_H */
