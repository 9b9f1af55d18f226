// C ABI: plans (pure host state), parameter validation, workspace layout and
// the enqueue entry points declared in include/stereo.h.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <new>

#include "internal.h"

namespace stereo {

namespace {
thread_local std::string g_last_error;
}

stereo_status fail(stereo_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

stereo_status hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return STEREO_OK;
  return fail(STEREO_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

Consts consts_of(const Plan& P) {
  const double log2e = 1.4426950408889634;
  Consts c;
  c.ks2 = (float)(log2e / ((double)P.p.sigma_s * P.p.sigma_s));
  c.kr2 = (float)(log2e / ((double)P.p.sigma_r * P.p.sigma_r));
  return c;
}

}  // namespace stereo

using namespace stereo;

namespace {

stereo_status validate(const stereo_params* p) {
  if (!p) return fail(STEREO_ERR_INVALID_ARGUMENT, "params is NULL");
  if (p->width < 1 || p->height < 1)
    return fail(STEREO_ERR_INVALID_ARGUMENT, "width/height must be >= 1 (got %d x %d)",
                p->width, p->height);
  if ((int64_t)p->width * p->height > (int64_t)1 << 30)
    return fail(STEREO_ERR_UNSUPPORTED, "image too large");
  if (p->pitch_ref < p->width || p->pitch_tar < p->width)
    return fail(STEREO_ERR_INVALID_ARGUMENT, "pitch (%lld, %lld) < width %d",
                (long long)p->pitch_ref, (long long)p->pitch_tar, p->width);
  if (p->dtype != STEREO_U8 && p->dtype != STEREO_F32)
    return fail(STEREO_ERR_INVALID_ARGUMENT, "unknown dtype %d", (int)p->dtype);
  if (p->num_disp < 3)
    return fail(STEREO_ERR_INVALID_ARGUMENT, "num_disp must be >= 3 (got %d)", p->num_disp);
  if (p->num_disp > STEREO_MAX_DISP)
    return fail(STEREO_ERR_UNSUPPORTED, "num_disp %d above %d", p->num_disp, STEREO_MAX_DISP);
  if (p->ncc_radius < 1 || p->ncc_radius > STEREO_MAX_NCC_RADIUS)
    return fail(p->ncc_radius < 1 ? STEREO_ERR_INVALID_ARGUMENT : STEREO_ERR_UNSUPPORTED,
                "ncc_radius %d outside 1..%d", p->ncc_radius, STEREO_MAX_NCC_RADIUS);
  if (p->bil_radius < STEREO_MIN_BIL_RADIUS || p->bil_radius > STEREO_MAX_BIL_RADIUS)
    return fail(p->bil_radius < 1 ? STEREO_ERR_INVALID_ARGUMENT : STEREO_ERR_UNSUPPORTED,
                "bil_radius %d outside %d..%d", p->bil_radius, STEREO_MIN_BIL_RADIUS,
                STEREO_MAX_BIL_RADIUS);
  if (!(p->sigma_s > 0.0f) || !(p->sigma_r > 0.0f) || !std::isfinite(p->sigma_s) ||
      !std::isfinite(p->sigma_r))
    return fail(STEREO_ERR_INVALID_ARGUMENT, "sigma_s, sigma_r must be finite and > 0");
  if (!(p->lr_delta >= 0.0f))
    return fail(STEREO_ERR_INVALID_ARGUMENT, "lr_delta must be >= 0");
  if (!(p->softargmin_T > 0.0f))
    return fail(STEREO_ERR_INVALID_ARGUMENT, "softargmin_T must be > 0");
  if (p->perspective != 0 && p->perspective != 1)
    return fail(STEREO_ERR_INVALID_ARGUMENT, "perspective must be 0 or 1");
  if (!p->perspective && p->delta_p != 0.0f)
    return fail(STEREO_ERR_INVALID_ARGUMENT, "delta_p must be 0 without the perspective step");
  if (!std::isfinite(p->delta_p) || !std::isfinite(p->plane[0]) ||
      !std::isfinite(p->plane[1]) || !std::isfinite(p->plane[2]))
    return fail(STEREO_ERR_INVALID_ARGUMENT, "delta_p and plane must be finite");
  if ((int64_t)p->num_disp * p->height * ((int64_t)p->width + p->num_disp + 4) >= ((int64_t)1 << 31))
    return fail(STEREO_ERR_UNSUPPORTED, "cost volume above 2^31 elements");
  if (p->perspective && !(std::fabs(p->plane[1]) < 0.5))
    return fail(STEREO_ERR_INVALID_ARGUMENT, "|plane c1| must be < 0.5 px/column");
  return STEREO_OK;
}

void layout(Plan& P) {
  const int W = P.W, H = P.H, D = P.D, r = P.r;
  P.stats_w = W + 2 * r;
  P.cw = ((W + D - 1) + 3) & ~3;
  P.road_blocks = 240;
  size_t o = 0;
  P.off_tarw = o;  o = align256(o + sizeof(float) * (size_t)W * H);
  P.off_stats = o; o = align256(o + sizeof(float) * 4 * (size_t)P.stats_w * H);
  // the cost volume region holds either the quad-interleaved FP32 volume
  // (engines 0 and 1) or the two split-FP16 volumes (engine 2)
  P.h2_pitch = h2_pitch(P.R, W);
  P.h2_tar_off = align256(sizeof(uint16_t) * 2 * 16 * (size_t)((D + 15) / 16) * H * P.h2_pitch);
  const size_t quad_bytes = sizeof(float) * 4 * (size_t)((D + 3) / 4) * H * P.cw;
  const size_t h2_bytes = 2 * P.h2_tar_off;
  P.off_cvol = o;  o = align256(o + (quad_bytes > h2_bytes ? quad_bytes : h2_bytes));
  P.off_dT = o;    o = align256(o + sizeof(int16_t) * (size_t)W * H);
  P.off_dsub = o;  o = align256(o + sizeof(float) * (size_t)W * H);
  P.off_road = o;  o = align256(o + sizeof(double) * 10 * (size_t)P.road_blocks);
  P.ws_bytes = grad_layout(P, o);
}

template <typename T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

stereo_status check_ws(const Plan& P, void* ws, size_t bytes) {
  if (!ws) return fail(STEREO_ERR_INVALID_ARGUMENT, "workspace is NULL");
  if (bytes < P.ws_bytes)
    return fail(STEREO_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes < required %zu", bytes,
                P.ws_bytes);
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0)
    return fail(STEREO_ERR_INVALID_ARGUMENT, "workspace must be 256-byte aligned");
  return STEREO_OK;
}

#define STEREO_REQUIRE(cond, ...) \
  do { if (!(cond)) return fail(STEREO_ERR_INVALID_ARGUMENT, __VA_ARGS__); } while (0)
#define STEREO_HIP(expr, what) \
  do { stereo_status s_ = hip_check((expr), (what)); if (s_ != STEREO_OK) return s_; } while (0)

// Statistics maps inside the workspace.
struct StatMaps {
  float *zX, *isdX, *zY, *isdY;
};
StatMaps stat_maps(const Plan& P, void* ws) {
  float* b = at<float>(ws, P.off_stats);
  const size_t n = (size_t)P.stats_w * P.H;
  return {b, b + n, b + 2 * n, b + 3 * n};
}

}  // namespace

extern "C" {

const char* stereo_status_string(stereo_status s) {
  switch (s) {
    case STEREO_OK: return "ok";
    case STEREO_ERR_INVALID_ARGUMENT: return "invalid argument";
    case STEREO_ERR_UNSUPPORTED: return "unsupported";
    case STEREO_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case STEREO_ERR_HIP: return "HIP error";
    case STEREO_ERR_NOT_CONVERGED: return "not converged";
  }
  return "unknown status";
}

const char* stereo_last_error(void) { return g_last_error.c_str(); }

const char* stereo_version(void) { return "mi355x-road-stereo 0.1 (gfx950)"; }

stereo_status stereo_plan_create(const stereo_params* params, stereo_plan_t* out) {
  if (!out) return fail(STEREO_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  stereo_status s = validate(params);
  if (s != STEREO_OK) return s;
  stereo_plan_s* pl = new (std::nothrow) stereo_plan_s;
  if (!pl) return fail(STEREO_ERR_INVALID_ARGUMENT, "out of host memory");
  Plan& P = pl->P;
  P.p = *params;
  P.W = params->width;
  P.H = params->height;
  P.D = params->num_disp;
  P.r = params->ncc_radius;
  P.R = params->bil_radius;
  // backward tile: every level at once up to 64 (a few hundred MB of
  // workspace at 1280x720); larger ranges are recomputed in 64-level tiles
  P.grad_levels = std::min(64, (P.D + 3) / 4 * 4);
  layout(P);
  *out = pl;
  return STEREO_OK;
}

stereo_status stereo_plan_destroy(stereo_plan_t plan) {
  delete plan;
  return STEREO_OK;
}

stereo_status stereo_plan_workspace_bytes(stereo_plan_t plan, size_t* bytes) {
  STEREO_REQUIRE(plan && bytes, "plan and bytes must be non-NULL");
  *bytes = plan->P.ws_bytes;
  return STEREO_OK;
}

stereo_status stereo_plan_set_homography(stereo_plan_t plan, const double* H) {
  STEREO_REQUIRE(plan, "plan is NULL");
  Plan& P = plan->P;
  if (!H) {
    P.homog = 0;
    return STEREO_OK;
  }
  STEREO_REQUIRE(P.p.perspective == 1, "a homography needs a plan with perspective = 1");
  for (int k = 0; k < 9; ++k) STEREO_REQUIRE(std::isfinite(H[k]), "H[%d] is not finite", k);
  const double dp = (double)P.p.delta_p;
  const double us[2] = {dp - P.D + 1, P.W - 1 + dp}, vs[2] = {0.0, (double)(P.H - 1)};
  for (double u : us)
    for (double v : vs)
      STEREO_REQUIRE(H[6] * u + H[7] * v + H[8] > 0.0,
                     "H maps (%g, %g) to or behind the plane at infinity", u, v);
  for (int k = 0; k < 9; ++k) P.Hm[k] = H[k];
  P.homog = 1;
  return STEREO_OK;
}

stereo_status stereo_plan_set_tuning(stereo_plan_t plan, const char* key, int32_t value) {
  STEREO_REQUIRE(plan && key, "plan and key must be non-NULL");
  const std::string k(key);
  if (k == "grad_levels") {
    STEREO_REQUIRE(value >= 4 && value <= 64 && value % 4 == 0,
                   "grad_levels must be a multiple of 4 in 4..64");
    plan->P.grad_levels = value;
    plan->P.ws_bytes = grad_layout(plan->P, plan->P.off_road +
                                   align256(sizeof(double) * 10 * (size_t)plan->P.road_blocks));
    return STEREO_OK;
  }
  if (k == "agg_levels_u8" || k == "agg_levels_f32") {
    STEREO_REQUIRE(value == 8 || value == 16, "%s must be 8 or 16", key);
    (k == "agg_levels_u8" ? plan->P.agg_levels_u8 : plan->P.agg_levels_f32) = value;
    return STEREO_OK;
  }
  if (k == "agg_engine") {
    STEREO_REQUIRE(value >= 0 && value <= 2,
                   "agg_engine must be 0 (vector ALU), 1 (matrix cores, FP32 operands) or 2 "
                   "(matrix cores, split-FP16 operands)");
    plan->P.agg_engine = value;
    return STEREO_OK;
  }
  if (k == "ncc_levels") {
    STEREO_REQUIRE(value == 0 || value == 16 || value == 32 || value == 64,
                   "ncc_levels must be 0 (automatic), 16, 32 or 64");
    plan->P.ncc_levels = value;
    return STEREO_OK;
  }
  return fail(STEREO_ERR_INVALID_ARGUMENT, "unknown tuning key '%s'", key);
}

stereo_status stereo_plan_get_tuning(stereo_plan_t plan, const char* key, int32_t* value) {
  STEREO_REQUIRE(plan && key && value, "plan, key and value must be non-NULL");
  const std::string k(key);
  if (k == "agg_levels_u8") { *value = plan->P.agg_levels_u8; return STEREO_OK; }
  if (k == "agg_levels_f32") { *value = plan->P.agg_levels_f32; return STEREO_OK; }
  if (k == "grad_levels") { *value = plan->P.grad_levels; return STEREO_OK; }
  if (k == "ncc_levels") { *value = plan->P.ncc_levels; return STEREO_OK; }
  if (k == "agg_engine") { *value = plan->P.agg_engine; return STEREO_OK; }
  return fail(STEREO_ERR_INVALID_ARGUMENT, "unknown tuning key '%s'", key);
}

stereo_status stereo_plan_get_params(stereo_plan_t plan, stereo_params* out) {
  STEREO_REQUIRE(plan && out, "plan and out must be non-NULL");
  *out = plan->P.p;
  return STEREO_OK;
}

stereo_status stereo_warp(stereo_plan_t plan, const void* tar, float* tar_w,
                          hipStream_t stream) {
  STEREO_REQUIRE(plan && tar && tar_w, "plan, tar and tar_w must be non-NULL");
  STEREO_HIP(launch_warp(plan->P, tar, tar_w, stream), "warp");
  return STEREO_OK;
}

stereo_status stereo_cost_volume(stereo_plan_t plan, const void* ref, const float* tar_w,
                                 float* cost_R, float* cost_T, void* ws, size_t ws_bytes,
                                 hipStream_t stream) {
  STEREO_REQUIRE(plan && ref && tar_w && cost_R, "plan, ref, tar_w and cost_R must be non-NULL");
  const Plan& P = plan->P;
  stereo_status s = check_ws(P, ws, ws_bytes);
  if (s != STEREO_OK) return s;
  StatMaps m = stat_maps(P, ws);
  STEREO_HIP(launch_block_stats2(P, ref, P.p.dtype, P.p.pitch_ref, tar_w, m.zX, m.isdX, m.zY,
                                 m.isdY, stream), "block statistics");
  const int64_t slice = (int64_t)P.W * P.H;
  STEREO_HIP(launch_ncc(P, ref, tar_w, m.zX, m.isdX, m.zY, m.isdY, cost_R, P.W, P.W, slice,
                        0, stream), "ncc (reference volume)");
  if (cost_T)
    STEREO_HIP(launch_ncc(P, ref, tar_w, m.zX, m.isdX, m.zY, m.isdY, cost_T, P.W, P.W, slice,
                          1, stream), "ncc (target volume)");
  return STEREO_OK;
}

stereo_status stereo_bilateral_aggregate(stereo_plan_t plan, const void* guide,
                                         stereo_dtype guide_dtype, int64_t guide_pitch,
                                         const float* cost_in, float* cost_out,
                                         hipStream_t stream) {
  STEREO_REQUIRE(plan && guide && cost_in && cost_out,
                 "plan, guide, cost_in and cost_out must be non-NULL");
  STEREO_REQUIRE(guide_dtype == STEREO_U8 || guide_dtype == STEREO_F32, "bad guide dtype");
  const Plan& P = plan->P;
  STEREO_REQUIRE(guide_pitch >= P.W, "guide_pitch < width");
  STEREO_REQUIRE(cost_in != cost_out, "cost_in and cost_out must not alias");
  BilArgs a{};
  a.C = cost_in;
  a.c_slice = (int64_t)P.W * P.H;
  a.c_pitch = P.W;
  a.shift = 0;
  a.guide = guide;
  a.guide_dt = guide_dtype;
  a.guide_pitch = guide_pitch;
  a.E = cost_out;
  STEREO_HIP(launch_bilateral(P, a, 0, stream), "bilateral aggregation");
  return STEREO_OK;
}

stereo_status stereo_wta_subpixel(stereo_plan_t plan, const float* agg, int16_t* dint,
                                  float* dsub, hipStream_t stream) {
  STEREO_REQUIRE(plan && agg && dint, "plan, agg and dint must be non-NULL");
  STEREO_HIP(launch_wta(plan->P, agg, dint, dsub, stream), "winner-take-all");
  return STEREO_OK;
}

stereo_status stereo_lr_check(stereo_plan_t plan, const int16_t* dint_R,
                              const int16_t* dint_T, const float* dsub_R, uint8_t* valid,
                              float* disp, hipStream_t stream) {
  STEREO_REQUIRE(plan && dint_R, "plan and dint_R must be non-NULL");
  STEREO_REQUIRE(valid || disp, "valid and disp are both NULL");
  STEREO_REQUIRE(dint_T || !plan->P.p.lr_check, "dint_T is NULL but lr_check = 1");
  STEREO_HIP(launch_lr_check(plan->P, dint_R, dint_T, dsub_R, valid, disp, stream),
             "left-right check");
  return STEREO_OK;
}

stereo_status stereo_match(stereo_plan_t plan, const void* ref, const void* tar,
                           int16_t* dint_R, int16_t* dint_T, float* dsub, uint8_t* valid,
                           float* disp, void* ws, size_t ws_bytes, hipStream_t stream) {
  return stereo_match_profiled(plan, ref, tar, dint_R, dint_T, dsub, valid, disp, ws, ws_bytes,
                               nullptr, stream);
}

}  // extern "C"

namespace {

// The plain forward; st (nullable) supplies the plane from device memory.
stereo_status match_impl(stereo_plan_t plan, const void* ref, const void* tar,
                         const stereo_plane_state* st, int16_t* dint_R, int16_t* dint_T,
                         float* dsub, uint8_t* valid, float* disp, void* ws, size_t ws_bytes,
                         hipEvent_t* ev, hipStream_t stream) {
  STEREO_REQUIRE(plan && ref && tar && dint_R, "plan, ref, tar and dint_R must be non-NULL");
  const Plan& P = plan->P;
  stereo_status s = check_ws(P, ws, ws_bytes);
  if (s != STEREO_OK) return s;
  float* tarw = at<float>(ws, P.off_tarw);
  StatMaps m = stat_maps(P, ws);
  float* cvol = at<float>(ws, P.off_cvol);
  int16_t* dT = dint_T ? dint_T : at<int16_t>(ws, P.off_dT);
  float* ds = dsub ? dsub : at<float>(ws, P.off_dsub);
  auto mark = [&](int i) -> hipError_t {
    return ev ? hipEventRecord(ev[i], stream) : hipSuccess;
  };

  STEREO_HIP(mark(0), "event record");
  STEREO_HIP(st ? launch_warp_tracked(P, tar, st, tarw, stream)
                : launch_warp(P, tar, tarw, stream), "warp");
  STEREO_HIP(mark(1), "event record");
  STEREO_HIP(launch_block_stats2(P, ref, P.p.dtype, P.p.pitch_ref, tarw, m.zX, m.isdX, m.zY,
                                 m.isdY, stream), "block statistics");
  STEREO_HIP(mark(2), "event record");
  const bool lr = P.p.lr_check != 0;
  BilArgs a{};
  if (P.agg_engine == 2) {
    // Split-FP16 volumes for the FP16-operand matrix cores from one NCC
    // pass: the reference-anchored volume and, for the LR check, the
    // target-anchored one (each stored by the column it is aggregated at).
    uint16_t* vR = at<uint16_t>(ws, P.off_cvol);
    uint16_t* vT = at<uint16_t>(ws, P.off_cvol + P.h2_tar_off);
    const int64_t plane = 16 * (int64_t)P.H * P.h2_pitch;
    STEREO_HIP(launch_ncc(P, ref, tarw, m.zX, m.isdX, m.zY, m.isdY, reinterpret_cast<float*>(vR),
                          ncc_both_extent(P.h2_pitch, 0, P.D), P.h2_pitch, plane, 0, stream, 0,
                          -1, 4, P.R, lr ? reinterpret_cast<float*>(vT) : nullptr),
               "ncc (both anchors)");
    a.h2 = vR;
    a.h2_plane = plane;
    a.h2_pitch = P.h2_pitch;
  } else {
    // One reference-anchored volume over the extended columns [0, W + D - 1):
    // the target volume is its re-indexing C_T(x, d) = C_R(x + d, d).  Stored
    // as float4 quads of consecutive levels (slice and pitch in float4 units).
    const int64_t slice = (int64_t)P.H * P.cw;
    const int ext_w = P.W + P.D - 1;
    STEREO_HIP(launch_ncc(P, ref, tarw, m.zX, m.isdX, m.zY, m.isdY, cvol, ext_w, P.cw, slice,
                          0, stream, 0, -1, 1), "ncc");
    a.C = cvol;
    a.c_slice = slice;
    a.c_pitch = P.cw;
    a.shift = 0;
    a.quad = 1;
  }
  STEREO_HIP(mark(3), "event record");
  a.guide = ref;
  a.guide_dt = P.p.dtype;
  a.guide_pitch = P.p.pitch_ref;
  a.dint = dint_R;
  a.dsub = ds;
  STEREO_HIP(launch_bilateral(P, a, 1, stream), "bilateral + WTA (reference)");
  STEREO_HIP(mark(4), "event record");
  if (lr) {
    BilArgs b = a;
    if (a.h2) b.h2 = at<uint16_t>(ws, P.off_cvol + P.h2_tar_off);
    else b.shift = 1;
    b.guide = tarw;
    b.guide_dt = STEREO_F32;
    b.guide_pitch = P.W;
    b.dint = dT;
    b.dsub = nullptr;
    STEREO_HIP(launch_bilateral(P, b, 1, stream), "bilateral + WTA (target)");
  }
  STEREO_HIP(mark(5), "event record");
  if (valid || disp)
    STEREO_HIP(st ? launch_lr_check_tracked(P, dint_R, lr ? dT : nullptr, ds, st, valid, disp,
                                            stream)
                  : launch_lr_check(P, dint_R, lr ? dT : nullptr, ds, valid, disp, stream),
               "left-right check");
  STEREO_HIP(mark(6), "event record");
  return STEREO_OK;
}

}  // namespace

extern "C" {

stereo_status stereo_match_profiled(stereo_plan_t plan, const void* ref, const void* tar,
                                    int16_t* dint_R, int16_t* dint_T, float* dsub,
                                    uint8_t* valid, float* disp, void* ws, size_t ws_bytes,
                                    hipEvent_t* ev, hipStream_t stream) {
  return match_impl(plan, ref, tar, nullptr, dint_R, dint_T, dsub, valid, disp, ws, ws_bytes,
                    ev, stream);
}

stereo_status stereo_match_tracked(stereo_plan_t plan, const void* ref, const void* tar,
                                   const stereo_plane_state* state_dev, int16_t* dint_R,
                                   int16_t* dint_T, float* dsub, uint8_t* valid, float* disp,
                                   void* ws, size_t ws_bytes, hipStream_t stream) {
  STEREO_REQUIRE(plan && state_dev, "plan and state_dev must be non-NULL");
  STEREO_REQUIRE(plan->P.p.perspective == 1, "tracking needs a plan with perspective = 1");
  STEREO_REQUIRE(!plan->P.homog, "tracking follows the plane model; the plan has a homography");
  return match_impl(plan, ref, tar, state_dev, dint_R, dint_T, dsub, valid, disp, ws, ws_bytes,
                    nullptr, stream);
}

stereo_status stereo_road_transform(stereo_plan_t plan, const float* disp,
                                    const uint8_t* mask, double psi_init, double lambda0,
                                    double delta_psi, int32_t max_iter, float delta_t,
                                    stereo_road_fit* fit_dev, float* disp_t, void* ws,
                                    size_t ws_bytes, hipStream_t stream) {
  STEREO_REQUIRE(plan && disp && fit_dev, "plan, disp and fit_dev must be non-NULL");
  STEREO_REQUIRE(max_iter >= 1, "max_iter must be >= 1");
  STEREO_REQUIRE(lambda0 > 0.0 && std::isfinite(lambda0), "lambda0 must be finite and > 0");
  STEREO_REQUIRE(delta_psi > 0.0, "delta_psi must be > 0");
  STEREO_REQUIRE(std::isfinite(psi_init), "psi_init must be finite");
  const Plan& P = plan->P;
  stereo_status s = check_ws(P, ws, ws_bytes);
  if (s != STEREO_OK) return s;
  STEREO_HIP(launch_road(P, disp, mask, psi_init, lambda0, delta_psi, max_iter, delta_t,
                         fit_dev, disp_t, at<double>(ws, P.off_road), stream),
             "road transform");
  return STEREO_OK;
}

stereo_status stereo_road_transform_noalloc(stereo_plan_t plan, const float* disp,
                                            const uint8_t* mask, double psi_init,
                                            double lambda0, double delta_psi,
                                            int32_t max_iter, float delta_t,
                                            stereo_road_fit* fit_dev, float* disp_t,
                                            hipStream_t stream) {
  STEREO_REQUIRE(plan && disp && fit_dev, "plan, disp and fit_dev must be non-NULL");
  STEREO_REQUIRE(max_iter >= 1, "max_iter must be >= 1");
  STEREO_REQUIRE(lambda0 > 0.0 && std::isfinite(lambda0), "lambda0 must be finite and > 0");
  STEREO_REQUIRE(delta_psi > 0.0, "delta_psi must be > 0");
  STEREO_REQUIRE(std::isfinite(psi_init), "psi_init must be finite");
  const Plan& P = plan->P;
  double* partials = nullptr;
  size_t cap = 0;
  STEREO_HIP(road_scratch(&partials, &cap), "road transform (fixed buffer address)");
  const size_t need = sizeof(double) * 10 * (size_t)P.road_blocks;
  if (need > cap)
    return fail(STEREO_ERR_UNSUPPORTED,
                "road transform needs %zu bytes of partials, the fixed buffer holds %zu", need,
                cap);
  STEREO_HIP(launch_road(P, disp, mask, psi_init, lambda0, delta_psi, max_iter, delta_t,
                         fit_dev, disp_t, partials, stream),
             "road transform (fixed buffer)");
  return STEREO_OK;
}

stereo_status stereo_road_transform_tracked(stereo_plan_t plan, const float* disp,
                                            const uint8_t* mask, double lambda0,
                                            double delta_psi, int32_t max_iter,
                                            float delta_t, stereo_plane_state* state_dev,
                                            stereo_road_fit* fit_dev, float* disp_t,
                                            void* ws, size_t ws_bytes, hipStream_t stream) {
  STEREO_REQUIRE(plan && disp && fit_dev && state_dev,
                 "plan, disp, fit_dev and state_dev must be non-NULL");
  STEREO_REQUIRE(max_iter >= 1, "max_iter must be >= 1");
  STEREO_REQUIRE(lambda0 > 0.0 && std::isfinite(lambda0), "lambda0 must be finite and > 0");
  STEREO_REQUIRE(delta_psi > 0.0, "delta_psi must be > 0");
  const Plan& P = plan->P;
  stereo_status s = check_ws(P, ws, ws_bytes);
  if (s != STEREO_OK) return s;
  STEREO_HIP(launch_road(P, disp, mask, 0.0, lambda0, delta_psi, max_iter, delta_t, fit_dev,
                         disp_t, at<double>(ws, P.off_road), stream, state_dev),
             "road transform (tracked)");
  return STEREO_OK;
}

stereo_status stereo_damage_mask(stereo_plan_t plan, const float* disp_t, float delta_t,
                                 float tau, uint8_t* mask, hipStream_t stream) {
  STEREO_REQUIRE(plan && disp_t && mask, "plan, disp_t and mask must be non-NULL");
  STEREO_REQUIRE(std::isfinite(delta_t) && std::isfinite(tau) && tau > 0.0f,
                 "delta_t must be finite and tau finite and > 0");
  STEREO_HIP(launch_damage_mask(plan->P, disp_t, delta_t, tau, mask, stream), "damage mask");
  return STEREO_OK;
}

}  // extern "C"
