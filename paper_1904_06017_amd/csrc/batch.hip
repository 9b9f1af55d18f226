// Batched form: many stereo pairs of uneven size and disparity range in one
// captured graph of a dozen launches.  The cheap stages (warp, block
// statistics, NCC volume, left-right check) run as one launch per stage and
// element type (per NCC radius) over the blocks of every pair; the dominant
// stage, the aggregation + WTA of both cost volumes of every pair, runs as
// one persistent launch per (radius, guide type) group that takes tiles of
// all pairs of the group from a work queue, largest disparity range first.
// Every block and tile runs the same code as the per-pair path, so each
// pair's result is bitwise the plain path's.
#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

using namespace stereo;

namespace {

struct Group {
  int R;
  stereo_dtype gdt;
  int levels;
  std::vector<int> tiles;     // (pair descriptor index, x0, y0) triples, vector-ALU tiles
  std::vector<int> tiles_m;   // the same over the matrix-core tiles
  size_t tiles_off;           // in the workspace
  size_t tiles_m_off;
};

// One batched launch of a cheap stage: its jobs (pair, and for statistics
// which image), the block prefix, and where both live in the workspace.
enum JobKind { JK_WARP = 0, JK_STATS = 1, JK_NCC = 2, JK_LR = 3 };
struct JobList {
  JobKind kind;
  stereo_dtype dt;
  int r;                      // NCC radius; statistics: largest radius
  int dc = 16;                // NCC: levels per workgroup
  std::vector<int> pair;
  std::vector<int> which;     // statistics: 0 = reference, 1 = warped target
  std::vector<int> first;     // block prefix, size jobs + 1
  size_t job_bytes;
  size_t jobs_off, first_off;
};

__global__ void zero_u32_kernel(unsigned int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

}  // namespace

struct stereo_batch_s {
  std::vector<stereo_batch_item> items;
  std::vector<Plan> plans;             // copies of the pairs' plans
  std::vector<size_t> pair_ws;         // offset of each pair's plan workspace
  std::vector<Group> groups;
  std::vector<JobList> lists;
  size_t desc_off = 0, desc_bytes = 0; // per-volume descriptors (2 per pair)
  size_t counter_off = 0;
  size_t ws_bytes = 0;
  std::vector<char> host_desc;         // descriptors bound to the last workspace
  void* bound_ws = nullptr;
  int wg_per_cu = 2;
  int tile_band = 4;                   // tile columns per band of the matrix-core tile list
  int ncc_levels = 0;                  // NCC levels per workgroup (0: automatic)
  int overlap = 1;                     // split-FP16 engine: the aggregation of the
                                       // smaller radii beside the largest radius's NCC
  int levels_u8 = 8, levels_f32 = 8;
  int engine = 2;                      // aggregation engine: 2 / 1 matrix cores with split-FP16
                                       // / FP32 operands, 0 vector ALU
  int cu_count = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t capture = nullptr;
  hipStream_t side = nullptr;          // second branch of the overlapped schedule
  hipEvent_t fork = nullptr, join = nullptr;
};

namespace {

#define BREQ(cond, ...) \
  do { if (!(cond)) return fail(STEREO_ERR_INVALID_ARGUMENT, __VA_ARGS__); } while (0)
#define BHIP(expr, what) \
  do { stereo_status s_ = hip_check((expr), (what)); if (s_ != STEREO_OK) return s_; } while (0)

template <typename T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

// Block prefix of the NCC job lists for the batch's engine: the quad volume
// covers the extended columns (anchor 0 only); the split-FP16 engine writes
// both anchors' volumes (the target-anchored one when the pair has an LR
// check) from one job over the stored row plus the levels.
// Levels per NCC workgroup of a job list: the both-anchors form of the
// split-FP16 engine runs at most 32 (its register count fits two 16-wave
// workgroups per CU only below that).
int ncc_dc(const stereo_batch_s& b, const JobList& L) {
  if (b.ncc_levels) return b.ncc_levels;
  return b.engine == 2 ? std::min(L.dc, 32) : L.dc;
}

void ncc_blocks(stereo_batch_s& b) {
  for (JobList& L : b.lists) {
    if (L.kind != JK_NCC) continue;
    for (size_t k = 0; k < L.pair.size(); ++k) {
      const Plan& P = b.plans[L.pair[k]];
      int blocks = 0;
      if (b.engine == 2) {
        if (L.which[k] == 0)
          blocks = ncc_job_blocks(P, ncc_both_extent(P.h2_pitch, 0, P.D), 0, P.D,
                                  ncc_dc(b, L), 4);
      } else if (L.which[k] == 0) {
        blocks = ncc_job_blocks(P, P.W + P.D - 1, 0, P.D, L.dc, 1);
      }
      L.first[k + 1] = L.first[k] + blocks;
    }
  }
}

void build_layout(stereo_batch_s& b) {
  const int n = (int)b.items.size();
  size_t o = 0;
  b.desc_off = o;
  b.desc_bytes = bilateral_pair_bytes() * 2 * n;
  o = align256(o + b.desc_bytes);
  // groups: (R, guide type); tiles sorted by cost = D (largest first) so the
  // queue drains with the long tiles taken first
  b.groups.clear();
  struct T { int cost, pair, vol, x0, y0; };
  std::vector<std::vector<T>> per, per_m;
  auto find_group = [&](int R, stereo_dtype g) {
    for (size_t i = 0; i < b.groups.size(); ++i)
      if (b.groups[i].R == R && b.groups[i].gdt == g) return (int)i;
    Group G;
    G.R = R; G.gdt = g;
    G.levels = g == STEREO_U8 ? b.levels_u8 : b.levels_f32;
    b.groups.push_back(G);
    per.emplace_back();
    per_m.emplace_back();
    return (int)b.groups.size() - 1;
  };
  for (int i = 0; i < n; ++i) {
    const Plan& P = b.plans[i];
    for (int vol = 0; vol < (P.p.lr_check ? 2 : 1); ++vol) {
      const stereo_dtype g = vol == 0 ? P.p.dtype : STEREO_F32;
      const int gi = find_group(P.R, g);
      for (int y = 0; y < P.H; y += kBilTileH)
        for (int x = 0; x < P.W; x += kBilTileW) per[gi].push_back({P.D, i, vol, x, y});
      // matrix-core tiles in bands of tile_band tile columns walked row by
      // row: a run of the list is a 2-D patch of the image (shared halos)
      const int bandw = b.tile_band * kMfmaTileW;
      for (int xb = 0; xb < P.W; xb += bandw)
        for (int y = 0; y < P.H; y += kMfmaTileH)
          for (int x = xb; x < std::min(P.W, xb + bandw); x += kMfmaTileW)
            per_m[gi].push_back({P.D, i, vol, x, y});
    }
  }
  auto table = [&](std::vector<T>& src, std::vector<int>& tl, size_t& off) {
    std::stable_sort(src.begin(), src.end(), [](const T& a, const T& c) { return a.cost > c.cost; });
    tl.clear();
    for (const T& t : src) {
      tl.push_back(2 * t.pair + t.vol);
      tl.push_back(t.x0);
      tl.push_back(t.y0);
    }
    off = o;
    o = align256(o + sizeof(int) * tl.size());
  };
  for (size_t gi = 0; gi < b.groups.size(); ++gi) {
    table(per[gi], b.groups[gi].tiles, b.groups[gi].tiles_off);
    table(per_m[gi], b.groups[gi].tiles_m, b.groups[gi].tiles_m_off);
  }
  b.counter_off = o;
  o = align256(o + sizeof(unsigned int) * std::max<size_t>(1, b.groups.size()));
  // job lists of the cheap stages, in launch order
  b.lists.clear();
  auto list_of = [&](JobKind k, stereo_dtype dt, int r) -> JobList& {
    for (JobList& L : b.lists)
      if (L.kind == k && L.dt == dt && (k != JK_NCC || L.r == r)) return L;
    JobList L;
    L.kind = k; L.dt = dt; L.r = r;
    L.job_bytes = k == JK_WARP ? sizeof(WarpJob) : k == JK_STATS ? sizeof(StatsJob)
                : k == JK_NCC ? sizeof(NccJob) : sizeof(LrJob);
    L.first.push_back(0);
    b.lists.push_back(L);
    return b.lists.back();
  };
  auto push = [](JobList& L, int pair, int which, int blocks) {
    L.pair.push_back(pair);
    L.which.push_back(which);
    L.first.push_back(L.first.back() + blocks);
  };
  for (int i = 0; i < n; ++i) {
    const Plan& P = b.plans[i];
    push(list_of(JK_WARP, P.p.dtype, 0), i, 0, warp_job_blocks(P));
  }
  for (int i = 0; i < n; ++i) {
    const Plan& P = b.plans[i];
    JobList& Lr = list_of(JK_STATS, P.p.dtype, 0);
    push(Lr, i, 0, stats_job_blocks(P.W, P.H, P.r));
    Lr.r = std::max(Lr.r, P.r);
    JobList& Lt = list_of(JK_STATS, STEREO_F32, 0);
    push(Lt, i, 1, stats_job_blocks(P.W, P.H, P.r));
    Lt.r = std::max(Lt.r, P.r);
  }
  // NCC: the level block of the list's smallest pair (the smallest block that
  // holds its levels, at most 64); two job slots per pair (which = 0: the
  // job, covering both anchors with the split-FP16 engine; which = 1 has no
  // blocks), their blocks set per engine by ncc_blocks
  for (int i = 0; i < n; ++i) {
    const Plan& P = b.plans[i];
    JobList& L = list_of(JK_NCC, P.p.dtype, P.r);
    const int dc = P.D > 32 ? 64 : P.D > 16 ? 32 : 16;
    L.dc = L.pair.empty() ? dc : std::min(L.dc, dc);
    push(L, i, 0, 0);
    push(L, i, 1, 0);
  }
  ncc_blocks(b);
  for (int i = 0; i < n; ++i)
    if (b.items[i].valid || b.items[i].disp)
      push(list_of(JK_LR, STEREO_F32, 0), i, 0, lr_job_blocks(b.plans[i]));
  for (JobList& L : b.lists) {
    L.jobs_off = o;
    o = align256(o + L.job_bytes * L.pair.size());
    L.first_off = o;
    o = align256(o + sizeof(int) * L.first.size());
  }
  b.pair_ws.resize(n);
  for (int i = 0; i < n; ++i) {
    b.pair_ws[i] = o;
    o = align256(o + b.plans[i].ws_bytes);
  }
  b.ws_bytes = o;
}

// Descriptors depend on the workspace address; rebuilt and uploaded on bind.
stereo_status bind(stereo_batch_s& b, void* ws, size_t bytes, hipStream_t s) {
  BREQ(ws, "workspace is NULL");
  if (bytes < b.ws_bytes)
    return fail(STEREO_ERR_WORKSPACE_TOO_SMALL, "batch workspace %zu < %zu", bytes, b.ws_bytes);
  BREQ((reinterpret_cast<uintptr_t>(ws) & 255) == 0, "workspace must be 256-byte aligned");
  if (b.bound_ws == ws) return STEREO_OK;
  const int n = (int)b.items.size();
  const size_t pb = bilateral_pair_bytes();
  b.host_desc.assign(b.desc_bytes, 0);
  for (int i = 0; i < n; ++i) {
    const Plan& P = b.plans[i];
    void* pws = at<char>(ws, b.pair_ws[i]);
    BilArgs a{};
    if (b.engine == 2) {
      a.h2 = at<uint16_t>(pws, P.off_cvol);
      a.h2_plane = 16 * (int64_t)P.H * P.h2_pitch;
      a.h2_pitch = P.h2_pitch;
    } else {
      a.C = at<float>(pws, P.off_cvol);
      a.c_slice = (int64_t)P.H * P.cw;
      a.c_pitch = P.cw;
      a.shift = 0;
      a.quad = 1;
    }
    a.guide = b.items[i].ref;
    a.guide_dt = P.p.dtype;
    a.guide_pitch = P.p.pitch_ref;
    a.dint = b.items[i].dint_R;
    a.dsub = at<float>(pws, P.off_dsub);
    bilateral_pair(P, a, b.host_desc.data() + (2 * i) * pb);
    BilArgs t = a;
    if (b.engine == 2) t.h2 = at<uint16_t>(pws, P.off_cvol + P.h2_tar_off);
    else t.shift = 1;
    t.guide = at<float>(pws, P.off_tarw);
    t.guide_dt = STEREO_F32;
    t.guide_pitch = P.W;
    t.dint = at<int16_t>(pws, P.off_dT);
    t.dsub = nullptr;
    bilateral_pair(P, t, b.host_desc.data() + (2 * i + 1) * pb);
  }
  BHIP(hipMemcpyAsync(at<char>(ws, b.desc_off), b.host_desc.data(), b.desc_bytes,
                      hipMemcpyHostToDevice, s), "upload descriptors");
  // job descriptors of the cheap stages
  ncc_blocks(b);
  std::vector<std::vector<char>> host_jobs(b.lists.size());
  for (size_t li = 0; li < b.lists.size(); ++li) {
    const JobList& L = b.lists[li];
    std::vector<char>& hj = host_jobs[li];
    hj.assign(L.job_bytes * L.pair.size(), 0);
    for (size_t k = 0; k < L.pair.size(); ++k) {
      const int i = L.pair[k];
      const Plan& P = b.plans[i];
      void* pws = at<char>(ws, b.pair_ws[i]);
      float* tarw = at<float>(pws, P.off_tarw);
      float* st = at<float>(pws, P.off_stats);
      const size_t sn = (size_t)P.stats_w * P.H;
      char* dst = hj.data() + k * L.job_bytes;
      if (L.kind == JK_WARP) {
        const WarpJob J = warp_job(P, b.items[i].tar, tarw);
        memcpy(dst, &J, sizeof(J));
      } else if (L.kind == JK_STATS) {
        const StatsJob J = L.which[k] == 0
            ? stats_job(P, b.items[i].ref, P.p.pitch_ref, st, st + sn)
            : stats_job(P, tarw, P.W, st + 2 * sn, st + 3 * sn);
        memcpy(dst, &J, sizeof(J));
      } else if (L.kind == JK_NCC) {
        NccJob J;
        if (b.engine == 2) {
          // both anchored split volumes from one job (which = 0; the second
          // job of the pair has no blocks)
          J = ncc_job(P, b.items[i].ref, tarw, st, st + sn, st + 2 * sn, st + 3 * sn,
                      at<float>(pws, P.off_cvol), ncc_both_extent(P.h2_pitch, 0, P.D),
                      P.h2_pitch, 16 * (int64_t)P.H * P.h2_pitch, 0, 0, P.D, 4,
                      P.p.lr_check ? at<float>(pws, P.off_cvol + P.h2_tar_off) : nullptr, ws);
          J.pad = P.R;
        } else {
          J = ncc_job(P, b.items[i].ref, tarw, st, st + sn, st + 2 * sn, st + 3 * sn,
                      at<float>(pws, P.off_cvol), P.W + P.D - 1, P.cw, (int64_t)P.H * P.cw, 0,
                      0, P.D, 1, nullptr, ws);
        }
        memcpy(dst, &J, sizeof(J));
      } else {
        const LrJob J = lr_job(P, b.items[i].dint_R,
                               P.p.lr_check ? at<int16_t>(pws, P.off_dT) : nullptr,
                               at<float>(pws, P.off_dsub), b.items[i].valid, b.items[i].disp);
        memcpy(dst, &J, sizeof(J));
      }
    }
    BHIP(hipMemcpyAsync(at<char>(ws, L.jobs_off), hj.data(), hj.size(), hipMemcpyHostToDevice,
                        s), "upload jobs");
    BHIP(hipMemcpyAsync(at<char>(ws, L.first_off), L.first.data(), sizeof(int) * L.first.size(),
                        hipMemcpyHostToDevice, s), "upload job prefix");
  }
  for (const Group& G : b.groups) {
    BHIP(hipMemcpyAsync(at<char>(ws, G.tiles_off), G.tiles.data(), sizeof(int) * G.tiles.size(),
                        hipMemcpyHostToDevice, s), "upload tiles");
    BHIP(hipMemcpyAsync(at<char>(ws, G.tiles_m_off), G.tiles_m.data(),
                        sizeof(int) * G.tiles_m.size(), hipMemcpyHostToDevice, s),
         "upload matrix-core tiles");
  }
  BHIP(hipStreamSynchronize(s), "synchronise after upload");
  b.bound_ws = ws;
  return STEREO_OK;
}

stereo_status enqueue(stereo_batch_s& b, hipStream_t s, hipEvent_t* ev = nullptr) {
  void* ws = b.bound_ws;
  BREQ(ws, "batch not bound to a workspace");
  // the split-FP16 NCC of pair i (both anchored volumes), one launch
  auto ncc_pair = [&](int i) -> stereo_status {
    Plan P = b.plans[i];
    if (b.ncc_levels) P.ncc_levels = b.ncc_levels;
    void* pws = at<char>(ws, b.pair_ws[i]);
    const float* tarw = at<float>(pws, P.off_tarw);
    const float* st = at<float>(pws, P.off_stats);
    const size_t sn = (size_t)P.stats_w * P.H;
    BHIP(launch_ncc(P, b.items[i].ref, tarw, st, st + sn, st + 2 * sn, st + 3 * sn,
                    at<float>(pws, P.off_cvol), ncc_both_extent(P.h2_pitch, 0, P.D), P.h2_pitch,
                    16 * (int64_t)P.H * P.h2_pitch, 0, s, 0, -1, 4, P.R,
                    P.p.lr_check ? at<float>(pws, P.off_cvol + P.h2_tar_off) : nullptr),
         "batch ncc (per pair)");
    return STEREO_OK;
  };
  auto run_list = [&](const JobList& L) -> stereo_status {
    const int nj = (int)L.pair.size();
    const int blocks = L.first.back();
    const int* first = at<int>(ws, L.first_off);
    const void* jobs = at<char>(ws, L.jobs_off);
    switch (L.kind) {
      case JK_WARP:
        BHIP(launch_warp_jobs(L.dt, static_cast<const WarpJob*>(jobs), first, nj, blocks, s),
             "batch warp");
        break;
      case JK_STATS:
        BHIP(launch_stats_jobs(L.dt, static_cast<const StatsJob*>(jobs), first, nj, blocks, L.r,
                               s), "batch statistics");
        break;
      case JK_NCC:
        if (b.engine == 2) {
          // the split-FP16 engine: one single-image launch per pair (both
          // anchors), as the per-pair path makes it.  Its arguments arrive
          // preloaded, whereas every workgroup of a batched launch first
          // looks up its job and reads the descriptor: with 8-row tiles that
          // start-up outweighs the launches it saves (64 mixed pairs: 6.4
          // against 8.9 ms)
          for (size_t k = 0; k < L.pair.size(); ++k) {
            if (L.which[k] != 0) continue;
            stereo_status st = ncc_pair(L.pair[k]);
            if (st != STEREO_OK) return st;
          }
          break;
        }
        BHIP(launch_ncc_jobs(L.r, L.dt, 1, ncc_dc(b, L), static_cast<const NccJob*>(jobs), first,
                             nj, blocks, static_cast<char*>(ws), s),
             "batch ncc");
        break;
      case JK_LR:
        BHIP(launch_lr_jobs(static_cast<const LrJob*>(jobs), first, nj, blocks, s),
             "batch lr check");
        break;
    }
    return STEREO_OK;
  };
  // warp first (the target statistics read its output), then statistics, NCC
  unsigned int* ctr = at<unsigned int>(ws, b.counter_off);
  const int ng = (int)b.groups.size();
  const void* desc = at<char>(ws, b.desc_off);
  auto run_group = [&](int g, hipStream_t st) -> stereo_status {
    const Group& G = b.groups[g];
    if (b.engine >= 1) {                 // one workgroup per CU holds the whole LDS
      const int nt = (int)G.tiles_m.size() / 3;
      const int groups = std::max(1, std::min(nt, b.cu_count));
      BHIP(launch_bilateral_persistent(b.engine, G.R, G.gdt, G.levels, desc,
                                       at<int>(ws, G.tiles_m_off), nt, ctr + g, groups, st),
           "batch aggregation");
    } else {
      const int nt = (int)G.tiles.size() / 3;
      const int groups = std::max(1, std::min(nt, b.cu_count * b.wg_per_cu));
      BHIP(launch_bilateral_persistent(0, G.R, G.gdt, G.levels, desc, at<int>(ws, G.tiles_off), nt,
                                       ctr + g, groups, st), "batch aggregation");
    }
    return STEREO_OK;
  };
  int rmax = 0, rmin = 1 << 30;
  for (const Group& G : b.groups) {
    rmax = std::max(rmax, G.R);
    rmin = std::min(rmin, G.R);
  }
  if (b.engine == 2 && b.overlap && !ev && b.side && rmin < rmax) {
    // overlapped schedule: the NCC of the pairs below the largest radius
    // first; their aggregation groups then run on a second branch (graph
    // branch when captured) while the main one computes the NCC of the
    // largest radius and aggregates it; the LR check joins both
    for (JobKind k : {JK_WARP, JK_STATS})
      for (const JobList& L : b.lists)
        if (L.kind == k) {
          stereo_status st = run_list(L);
          if (st != STEREO_OK) return st;
        }
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(64), 0, s, ctr, ng);
    BHIP(hipGetLastError(), "zero counters");
    auto ncc_pairs = [&](bool small) -> stereo_status {
      for (const JobList& L : b.lists) {
        if (L.kind != JK_NCC) continue;
        for (size_t k = 0; k < L.pair.size(); ++k) {
          if (L.which[k] != 0) continue;
          const int i = L.pair[k];
          if ((b.plans[i].R < rmax) != small) continue;
          stereo_status st = ncc_pair(i);
          if (st != STEREO_OK) return st;
        }
      }
      return STEREO_OK;
    };
    stereo_status st = ncc_pairs(true);
    if (st != STEREO_OK) return st;
    BHIP(hipEventRecord(b.fork, s), "event record");
    BHIP(hipStreamWaitEvent(b.side, b.fork, 0), "stream wait");
    for (int g = 0; g < ng; ++g)
      if (b.groups[g].R < rmax && (st = run_group(g, b.side)) != STEREO_OK) return st;
    BHIP(hipEventRecord(b.join, b.side), "event record");
    if ((st = ncc_pairs(false)) != STEREO_OK) return st;
    for (int g = 0; g < ng; ++g)
      if (b.groups[g].R == rmax && (st = run_group(g, s)) != STEREO_OK) return st;
    BHIP(hipStreamWaitEvent(s, b.join, 0), "stream wait");
  } else {
    for (JobKind k : {JK_WARP, JK_STATS, JK_NCC})
      for (const JobList& L : b.lists)
        if (L.kind == k) {
          stereo_status st = run_list(L);
          if (st != STEREO_OK) return st;
        }
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(64), 0, s, ctr, ng);
    BHIP(hipGetLastError(), "zero counters");
    if (ev) BHIP(hipEventRecord(ev[0], s), "event record");
    for (int g = 0; g < ng; ++g) {
      stereo_status st = run_group(g, s);
      if (st != STEREO_OK) return st;
    }
    if (ev) BHIP(hipEventRecord(ev[1], s), "event record");
  }
  for (const JobList& L : b.lists)
    if (L.kind == JK_LR) {
      stereo_status st = run_list(L);
      if (st != STEREO_OK) return st;
    }
  return STEREO_OK;
}

// The second stream and the two events of the overlapped schedule (created
// outside any capture; default priority).
stereo_status ensure_side(stereo_batch_s& b) {
  if (b.engine != 2 || !b.overlap) return STEREO_OK;
  if (!b.side) BHIP(hipStreamCreateWithFlags(&b.side, hipStreamNonBlocking), "stream");
  if (!b.fork) BHIP(hipEventCreateWithFlags(&b.fork, hipEventDisableTiming), "event");
  if (!b.join) BHIP(hipEventCreateWithFlags(&b.join, hipEventDisableTiming), "event");
  return STEREO_OK;
}

void drop_graph(stereo_batch_s& b) {
  if (b.exec) hipGraphExecDestroy(b.exec);
  if (b.graph) hipGraphDestroy(b.graph);
  b.exec = nullptr;
  b.graph = nullptr;
}

}  // namespace

namespace stereo {
int batch_pair_count(stereo_batch_t b) { return b ? (int)b->items.size() : 0; }
void batch_pair_shape(stereo_batch_t b, int i, int32_t* s) {
  const Plan& P = b->plans[i];
  s[0] = P.W; s[1] = P.H; s[2] = P.D; s[3] = P.r; s[4] = P.R; s[5] = (int32_t)P.p.dtype;
}
}  // namespace stereo

extern "C" {

stereo_status stereo_batch_create(const stereo_batch_item* items, int32_t n,
                                  stereo_batch_t* out) {
  BREQ(out, "out is NULL");
  *out = nullptr;
  BREQ(items && n >= 1, "need at least one item");
  stereo_batch_s* b = new (std::nothrow) stereo_batch_s;
  if (!b) return fail(STEREO_ERR_INVALID_ARGUMENT, "out of host memory");
  for (int i = 0; i < n; ++i) {
    const stereo_batch_item& it = items[i];
    if (!it.plan || !it.ref || !it.tar || !it.dint_R) {
      delete b;
      return fail(STEREO_ERR_INVALID_ARGUMENT, "item %d: plan, ref, tar and dint_R must be set", i);
    }
    b->items.push_back(it);
    b->plans.push_back(it.plan->P);
  }
  build_layout(*b);
  *out = b;
  return STEREO_OK;
}

stereo_status stereo_batch_workspace_bytes(stereo_batch_t b, size_t* bytes) {
  BREQ(b && bytes, "batch and bytes must be non-NULL");
  *bytes = b->ws_bytes;
  return STEREO_OK;
}

stereo_status stereo_batch_set_tuning(stereo_batch_t b, const char* key, int32_t value) {
  BREQ(b && key, "batch and key must be non-NULL");
  const std::string k(key);
  if (k == "wg_per_cu") {
    BREQ(value >= 1 && value <= 8, "wg_per_cu must be 1..8");
    b->wg_per_cu = value;
  } else if (k == "agg_levels_u8" || k == "agg_levels_f32") {
    BREQ(value == 8 || value == 16, "%s must be 8 or 16", key);
    (k == "agg_levels_u8" ? b->levels_u8 : b->levels_f32) = value;
    for (Group& G : b->groups) G.levels = G.gdt == STEREO_U8 ? b->levels_u8 : b->levels_f32;
  } else if (k == "tile_band") {
    BREQ(value == 1 || value == 2 || value == 4 || value == 8 || value == 16 || value == 32,
         "tile_band must be 1, 2, 4, 8, 16 or 32");
    if (value != b->tile_band) {
      b->tile_band = value;
      build_layout(*b);                 // the same sizes and offsets, another tile order
      b->bound_ws = nullptr;            // tables are uploaded again
    }
  } else if (k == "ncc_levels") {
    BREQ(value == 0 || value == 16 || value == 32 || value == 64,
         "ncc_levels must be 0 (automatic), 16, 32 or 64");
    if (value != b->ncc_levels) {
      b->ncc_levels = value;
      ncc_blocks(*b);                   // block counts of the NCC job lists
      b->bound_ws = nullptr;            // tables are uploaded again
    }
  } else if (k == "group_overlap") {
    BREQ(value == 0 || value == 1, "group_overlap must be 0 or 1");
    b->overlap = value;
  } else if (k == "agg_engine") {
    BREQ(value >= 0 && value <= 2,
         "agg_engine must be 0 (vector ALU), 1 (matrix cores, FP32 operands) or 2 (matrix "
         "cores, split-FP16 operands)");
    b->engine = value;
    b->bound_ws = nullptr;              // descriptors and NCC jobs depend on the engine
  } else {
    return fail(STEREO_ERR_INVALID_ARGUMENT, "unknown batch tuning key '%s'", key);
  }
  drop_graph(*b);
  return STEREO_OK;
}

stereo_status stereo_batch_get_tuning(stereo_batch_t b, const char* key, int32_t* value) {
  BREQ(b && key && value, "batch, key and value must be non-NULL");
  const std::string k(key);
  if (k == "wg_per_cu") *value = b->wg_per_cu;
  else if (k == "tile_band") *value = b->tile_band;
  else if (k == "ncc_levels") *value = b->ncc_levels;
  else if (k == "group_overlap") *value = b->overlap;
  else if (k == "agg_levels_u8") *value = b->levels_u8;
  else if (k == "agg_levels_f32") *value = b->levels_f32;
  else if (k == "agg_engine") *value = b->engine;
  else return fail(STEREO_ERR_INVALID_ARGUMENT, "unknown batch tuning key '%s'", key);
  return STEREO_OK;
}

stereo_status stereo_submit_batch(stereo_batch_t b, void* ws, size_t ws_bytes,
                                  hipStream_t stream) {
  return stereo_submit_batch_profiled(b, ws, ws_bytes, nullptr, stream);
}

stereo_status stereo_submit_batch_profiled(stereo_batch_t b, void* ws, size_t ws_bytes,
                                           hipEvent_t* ev, hipStream_t stream) {
  BREQ(b, "batch is NULL");
  if (b->cu_count == 0) {
    int dev = 0;
    BHIP(hipGetDevice(&dev), "hipGetDevice");
    BHIP(hipDeviceGetAttribute(&b->cu_count, hipDeviceAttributeMultiprocessorCount, dev),
         "CU count");
  }
  stereo_status s = bind(*b, ws, ws_bytes, stream);
  if (s != STEREO_OK) return s;
  if ((s = ensure_side(*b)) != STEREO_OK) return s;
  return enqueue(*b, stream, ev);
}

stereo_status stereo_batch_instantiate(stereo_batch_t b, void* ws, size_t ws_bytes,
                                       hipStream_t stream) {
  BREQ(b, "batch is NULL");
  if (b->cu_count == 0) {
    int dev = 0;
    BHIP(hipGetDevice(&dev), "hipGetDevice");
    BHIP(hipDeviceGetAttribute(&b->cu_count, hipDeviceAttributeMultiprocessorCount, dev),
         "CU count");
  }
  stereo_status s = bind(*b, ws, ws_bytes, stream);
  if (s != STEREO_OK) return s;
  drop_graph(*b);
  if ((s = ensure_side(*b)) != STEREO_OK) return s;
  if (!b->capture) BHIP(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking), "stream");
  BHIP(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal), "begin capture");
  s = enqueue(*b, b->capture);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->capture, &g);
  if (s != STEREO_OK) {
    if (g) hipGraphDestroy(g);
    return s;
  }
  BHIP(e, "end capture");
  b->graph = g;
  BHIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0), "instantiate graph");
  return STEREO_OK;
}

stereo_status stereo_batch_launch(stereo_batch_t b, hipStream_t stream) {
  BREQ(b && b->exec, "batch has no instantiated graph");
  BHIP(hipGraphLaunch(b->exec, stream), "graph launch");
  return STEREO_OK;
}

stereo_status stereo_batch_destroy(stereo_batch_t b) {
  if (!b) return STEREO_OK;
  drop_graph(*b);
  if (b->capture) hipStreamDestroy(b->capture);
  if (b->side) hipStreamDestroy(b->side);
  if (b->fork) hipEventDestroy(b->fork);
  if (b->join) hipEventDestroy(b->join);
  delete b;
  return STEREO_OK;
}

}  // extern "C"
