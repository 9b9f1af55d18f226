// Autotuner: times the launch-shape variants of a plan (levels staged per
// aggregation pass, by guide type) or of a batch (persistent workgroups per
// CU, levels per pass) on the caller's own inputs with HIP events, keeps the
// fastest, and caches the choice in a small JSON file keyed by the GPU
// architecture and the problem shape, so that later runs skip the timing.
// Variants never change results (same per-pixel arithmetic), only speed.
#include <algorithm>
#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "internal.h"

using namespace stereo;

namespace {

#define AREQ(cond, ...) \
  do { if (!(cond)) return fail(STEREO_ERR_INVALID_ARGUMENT, __VA_ARGS__); } while (0)
#define AHIP(expr, what) \
  do { stereo_status s_ = hip_check((expr), (what)); if (s_ != STEREO_OK) return s_; } while (0)

using Entry = std::map<std::string, double>;

// The cache is a flat JSON object of objects: {"key": {"name": number, ...}, ...}.
std::map<std::string, Entry> load_cache(const char* path) {
  std::map<std::string, Entry> out;
  if (!path) return out;
  std::ifstream f(path);
  if (!f) return out;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  size_t i = 0;
  auto skip = [&]() { while (i < s.size() && isspace((unsigned char)s[i])) ++i; };
  auto str = [&](std::string& o) {
    skip();
    if (i >= s.size() || s[i] != '"') return false;
    const size_t j = s.find('"', i + 1);
    if (j == std::string::npos) return false;
    o = s.substr(i + 1, j - i - 1);
    i = j + 1;
    return true;
  };
  skip();
  if (i >= s.size() || s[i] != '{') return out;
  ++i;
  for (;;) {
    std::string key;
    if (!str(key)) break;
    skip();
    if (i >= s.size() || s[i] != ':') break;
    ++i;
    skip();
    if (i >= s.size() || s[i] != '{') break;
    ++i;
    Entry e;
    for (;;) {
      std::string name;
      if (!str(name)) break;
      skip();
      if (i >= s.size() || s[i] != ':') break;
      ++i;
      char* end = nullptr;
      const double v = strtod(s.c_str() + i, &end);
      i = end - s.c_str();
      e[name] = v;
      skip();
      if (i < s.size() && s[i] == ',') ++i;
    }
    skip();
    if (i < s.size() && s[i] == '}') ++i;
    out[key] = e;
    skip();
    if (i < s.size() && s[i] == ',') ++i;
  }
  return out;
}

void save_cache(const char* path, const std::map<std::string, Entry>& c) {
  if (!path) return;
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return;
  fprintf(f, "{\n");
  size_t k = 0;
  for (const auto& kv : c) {
    fprintf(f, "  \"%s\": {", kv.first.c_str());
    size_t j = 0;
    for (const auto& nv : kv.second)
      fprintf(f, "%s\"%s\": %.6g", j++ ? ", " : "", nv.first.c_str(), nv.second);
    fprintf(f, "}%s\n", ++k < c.size() ? "," : "");
  }
  fprintf(f, "}\n");
  fclose(f);
  rename(tmp.c_str(), path);
}

std::string arch_name() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return "unknown";
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

std::string plan_key(const Plan& P) {
  char buf[256];
  snprintf(buf, sizeof(buf), "%s:plan:W=%d,H=%d,D=%d,r=%d,R=%d,dtype=%s,persp=%d,lr=%d,engine=%d",
           arch_name().c_str(), P.W, P.H, P.D, P.r, P.R, P.p.dtype == STEREO_U8 ? "u8" : "f32",
           P.p.perspective, P.p.lr_check, P.agg_engine);
  return buf;
}

// Median of `reps` timed runs of fn() on the stream.
template <typename F>
stereo_status time_ms(hipStream_t s, int reps, F fn, double* ms) {
  hipEvent_t a, b;
  AHIP(hipEventCreate(&a), "event");
  AHIP(hipEventCreate(&b), "event");
  std::vector<float> t;
  stereo_status st = fn();                       // warm-up
  for (int i = 0; i < reps && st == STEREO_OK; ++i) {
    hipEventRecord(a, s);
    st = fn();
    hipEventRecord(b, s);
    hipEventSynchronize(b);
    float x = 0.0f;
    hipEventElapsedTime(&x, a, b);
    t.push_back(x);
  }
  hipEventDestroy(a);
  hipEventDestroy(b);
  if (st != STEREO_OK) return st;
  std::sort(t.begin(), t.end());
  *ms = t.empty() ? 0.0 : t[t.size() / 2];
  return STEREO_OK;
}

}  // namespace

extern "C" {

stereo_status stereo_plan_autotune(stereo_plan_t plan, const void* ref, const void* tar,
                                   void* ws, size_t ws_bytes, hipStream_t stream,
                                   const char* cache_path, int32_t reps, double* best_ms) {
  AREQ(plan && ref && tar && ws, "plan, ref, tar and ws must be non-NULL");
  AREQ(reps >= 1, "reps must be >= 1");
  Plan& P = plan->P;
  const std::string key = plan_key(P);
  auto cache = load_cache(cache_path);
  auto it = cache.find(key);
  if (it != cache.end() && it->second.count("agg_levels_u8") && it->second.count("agg_levels_f32")) {
    P.agg_levels_u8 = (int)it->second["agg_levels_u8"];
    P.agg_levels_f32 = (int)it->second["agg_levels_f32"];
    if (it->second.count("ncc_levels")) P.ncc_levels = (int)it->second["ncc_levels"];
    if (best_ms) *best_ms = it->second.count("ms") ? it->second["ms"] : 0.0;
    return STEREO_OK;
  }
  const size_t HW = (size_t)P.W * P.H;
  void* buf = nullptr;
  AHIP(hipMalloc(&buf, HW * (2 + 2 + 4 + 1 + 4) + 1024), "temporary outputs");
  int16_t* dR = static_cast<int16_t*>(buf);
  int16_t* dT = dR + HW;
  float* dsub = reinterpret_cast<float*>(dT + HW);
  float* disp = dsub + HW;
  uint8_t* valid = reinterpret_cast<uint8_t*>(disp + HW);
  // the knobs of the plan's aggregation engine (levels per pass of the vector
  // kernel; the matrix-core kernel has none) and the NCC level block: none
  // changes a result
  double best = 1e30;
  int bu = P.agg_levels_u8, bf = P.agg_levels_f32, bn = P.ncc_levels;
  stereo_status st = STEREO_OK;
  const std::vector<int> lvs = P.agg_engine == 0 ? std::vector<int>{8, 16}
                                                 : std::vector<int>{P.agg_levels_u8};
  const std::vector<int> lfs = P.agg_engine == 0 ? std::vector<int>{8, 16}
                                                 : std::vector<int>{P.agg_levels_f32};
  for (int nl : {16, 32, 64}) {
    for (int lu : lvs) {
      for (int lf : lfs) {
        P.agg_levels_u8 = lu;
        P.agg_levels_f32 = lf;
        P.ncc_levels = nl;
        double ms = 0.0;
        st = time_ms(stream, reps, [&]() {
          return stereo_match(plan, ref, tar, dR, dT, dsub, valid, disp, ws, ws_bytes, stream);
        }, &ms);
        if (st != STEREO_OK) break;
        if (ms < best) { best = ms; bu = lu; bf = lf; bn = nl; }
      }
      if (st != STEREO_OK) break;
    }
    if (st != STEREO_OK) break;
  }
  hipFree(buf);
  P.agg_levels_u8 = bu;
  P.agg_levels_f32 = bf;
  P.ncc_levels = bn;
  if (st != STEREO_OK) return st;
  cache[key] = Entry{{"agg_levels_u8", (double)bu}, {"agg_levels_f32", (double)bf},
                     {"ncc_levels", (double)bn}, {"ms", best}};
  save_cache(cache_path, cache);
  if (best_ms) *best_ms = best;
  return STEREO_OK;
}

stereo_status stereo_batch_autotune(stereo_batch_t b, void* ws, size_t ws_bytes,
                                    hipStream_t stream, const char* cache_path, int32_t reps,
                                    double* best_ms) {
  AREQ(b && ws, "batch and ws must be non-NULL");
  AREQ(reps >= 1, "reps must be >= 1");
  // key: architecture + FNV-1a hash of every pair's shape
  uint64_t h = 1469598103934665603ull;
  int32_t n = 0;
  constexpr int NK = 6;
  const char* keys[NK] = {"wg_per_cu", "agg_levels_u8", "agg_levels_f32", "tile_band",
                          "ncc_levels", "group_overlap"};
  int32_t cur[NK];
  for (int k = 0; k < NK; ++k) stereo_batch_get_tuning(b, keys[k], &cur[k]);
  // shapes are hashed through the workspace size and the plan shapes
  size_t wsb = 0;
  stereo_batch_workspace_bytes(b, &wsb);
  auto mix = [&](uint64_t x) {
    for (int i = 0; i < 8; ++i) { h ^= (x >> (8 * i)) & 0xff; h *= 1099511628211ull; }
  };
  mix(wsb);
  n = batch_pair_count(b);
  mix((uint64_t)n);
  for (int i = 0; i < n; ++i) {
    int32_t shape[6];
    batch_pair_shape(b, i, shape);
    for (int k = 0; k < 6; ++k) mix((uint64_t)(uint32_t)shape[k]);
  }
  int32_t engine = 1;
  stereo_batch_get_tuning(b, "agg_engine", &engine);
  char kb[128];
  snprintf(kb, sizeof(kb), "%s:batch:n=%d:engine=%d:%016llx", arch_name().c_str(), n, (int)engine,
           (unsigned long long)h);
  const std::string key = kb;
  auto cache = load_cache(cache_path);
  auto it = cache.find(key);
  if (it != cache.end() && it->second.count("wg_per_cu")) {
    for (int k = 0; k < NK; ++k)
      if (it->second.count(keys[k])) stereo_batch_set_tuning(b, keys[k], (int)it->second[keys[k]]);
    if (best_ms) *best_ms = it->second.count("ms") ? it->second["ms"] : 0.0;
    return STEREO_OK;
  }
  // the vector-ALU engine's knobs are its workgroups per CU and levels per
  // pass; the matrix-core engines' are the band width of their tile list (the
  // 2-D patch of tiles an XCD works on at a time: L2 reuse of the halos) and
  // the NCC level block of the batch's job lists, and with the split-FP16
  // engine whether the smaller radii's aggregation overlaps the largest
  // radius's NCC
  double best = 1e30;
  int32_t bestv[NK] = {cur[0], cur[1], cur[2], cur[3], cur[4], cur[5]};
  stereo_status st = STEREO_OK;
  const std::vector<int> wgs = engine == 0 ? std::vector<int>{1, 2, 3, 4} : std::vector<int>{cur[0]};
  const std::vector<int> lvls = engine == 0 ? std::vector<int>{8, 16} : std::vector<int>{cur[1]};
  const std::vector<int> bands = engine == 0 ? std::vector<int>{cur[3]}
                                             : std::vector<int>{2, 4, 8, 16};
  const std::vector<int> nccs = engine == 0 ? std::vector<int>{cur[4]}
                                            : std::vector<int>{16, 32, 64};
  const std::vector<int> ovs = engine == 2 ? std::vector<int>{0, 1} : std::vector<int>{cur[5]};
  for (size_t v = 0; v < wgs.size() * lvls.size() * bands.size() * nccs.size() * ovs.size();
       ++v) {
    size_t q = v;
    const int ov = ovs[q % ovs.size()]; q /= ovs.size();
    const int nv = nccs[q % nccs.size()]; q /= nccs.size();
    const int bd = bands[q % bands.size()]; q /= bands.size();
    const int lv = lvls[q % lvls.size()]; q /= lvls.size();
    const int wg = wgs[q];
    stereo_batch_set_tuning(b, "wg_per_cu", wg);
    stereo_batch_set_tuning(b, "agg_levels_u8", lv);
    stereo_batch_set_tuning(b, "agg_levels_f32", lv);
    stereo_batch_set_tuning(b, "tile_band", bd);
    stereo_batch_set_tuning(b, "ncc_levels", nv);
    stereo_batch_set_tuning(b, "group_overlap", ov);
    double ms = 0.0;
    st = time_ms(stream, reps,
                 [&]() { return stereo_submit_batch(b, ws, ws_bytes, stream); }, &ms);
    if (st != STEREO_OK) break;
    if (ms < best) {
      best = ms;
      bestv[0] = wg; bestv[1] = lv; bestv[2] = lv; bestv[3] = bd; bestv[4] = nv; bestv[5] = ov;
    }
  }
  for (int k = 0; k < NK; ++k) stereo_batch_set_tuning(b, keys[k], bestv[k]);
  if (st != STEREO_OK) return st;
  cache[key] = Entry{{"wg_per_cu", (double)bestv[0]}, {"agg_levels_u8", (double)bestv[1]},
                     {"agg_levels_f32", (double)bestv[2]}, {"tile_band", (double)bestv[3]},
                     {"ncc_levels", (double)bestv[4]}, {"group_overlap", (double)bestv[5]},
                     {"ms", best}};
  save_cache(cache_path, cache);
  if (best_ms) *best_ms = best;
  return STEREO_OK;
}

}  // extern "C"
