// Batched executor: many keyframe contexts, each fused with one new frame, by
// one staging, one stereo and one persistent solver launch per call. The
// per-keyframe solver arguments live in a static device table; each call
// uploads (from double-buffered pinned host memory, in one copy) the
// per-frame part: the active member count, their stereo arguments (image
// pointer and epipolar constants) and the solver's per-workgroup team queues.
// The launches read all of it from device memory, so they are captured once
// as HIP graphs and replayed for any subset of the members.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "kf_internal.h"

using namespace kf;

namespace {

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Per-call region of the batch workspace (uploaded as a whole).
struct DynLayout {
  size_t hdr, st, queue, qoff, total;
};

DynLayout dyn_layout(int n, int members_total) {
  DynLayout L;
  size_t off = 0;
  L.hdr = off; off += 256;
  L.st = off; off += align256((size_t)n * sizeof(StereoArgs));
  L.queue = off; off += align256((size_t)members_total * 4);
  L.qoff = off; off += align256((size_t)(members_total + 1) * 4);
  L.total = off;
  return L;
}

}  // namespace

struct kf_batch {
  std::vector<kf_ctx*> m;
  hipStream_t stream = nullptr;
  hipStream_t capture = nullptr;   // private stream the graphs are captured on
  int device = 0;
  int prec = 0, pattern = 0, ns = 0, threads = 0, ppt = 0;
  bool pipelined = false;
  int kind = 0;                 // solve_kind of the launch: pipelined bit | any member's variant bit
  size_t smem = 0;
  int grid = 0;                    // solver workgroups
  int max_queue = 0;               // longest per-workgroup queue of the last schedule
  int capacity = 0;                // co-resident workgroups of the batched solver
  int cus = 256;   // compute units of the device (stereo grid)
  bool use_graph = true;
  DynLayout dl{};
  char* d_dyn = nullptr;           // device: per-call region
  SolveArgs* d_so = nullptr;       // device: static solver table
  char* h_pin[2] = {nullptr, nullptr};
  hipEvent_t ev[2] = {nullptr, nullptr};
  bool ev_used[2] = {false, false};
  int parity = 0;
  // captured launch sequences: 0 = stereo + solve, 1 = stereo, 2 = solve
  hipGraphExec_t exec[3] = {nullptr, nullptr, nullptr};
  std::vector<int32_t> queue, qoff;
  std::string err;

  ~kf_batch() {
    for (hipGraphExec_t g : exec)
      if (g) (void)hipGraphExecDestroy(g);
    for (int i = 0; i < 2; ++i) {
      if (ev[i]) {
        (void)hipEventSynchronize(ev[i]);
        (void)hipEventDestroy(ev[i]);
      }
      if (h_pin[i]) (void)hipHostFree(h_pin[i]);
    }
    if (capture) (void)hipStreamDestroy(capture);
  }

  const int32_t* d_n() const { return reinterpret_cast<const int32_t*>(d_dyn + dl.hdr); }
  const StereoArgs* d_st() const { return reinterpret_cast<const StereoArgs*>(d_dyn + dl.st); }
  const int32_t* d_queue() const { return reinterpret_cast<const int32_t*>(d_dyn + dl.queue); }
  const int32_t* d_qoff() const { return reinterpret_cast<const int32_t*>(d_dyn + dl.qoff); }
};

namespace {

kf_status bfail(kf_batch* b, kf_status s, const std::string& msg) {
  if (b) b->err = msg;
  return s;
}

kf_status bhip(kf_batch* b, hipError_t e, const std::string& where) {
  return bfail(b, KF_ERR_HIP, where + ": " + hipGetErrorString(e));
}

int total_members(kf_ctx* const* m, int n) {
  int s = 0;
  for (int i = 0; i < n; ++i) s += m[i]->tiling.blocks;
  return s;
}

size_t static_bytes(int n) { return align256((size_t)n * sizeof(SolveArgs)); }

// Estimated duration of one keyframe's solve (microseconds): the latency
// model of the single-keyframe tiling choice times the synchronisations.
double team_cost(const kf_ctx* c) {
  const kf_config& g = c->cfg;
  const double cg = g.cg_rtol > 0.0 ? (double)g.cg_max : (double)g.n_cg;
  return g.n_gn * (cg + 2.0) * iteration_us(c->tiling);
}

// List schedule of the active teams over the `grid` workgroups. A team runs
// on the B workgroups that become free first (ties to the lower workgroup
// index, which spreads a team evenly over the XCDs because consecutive
// workgroups of a launch are dispatched to consecutive XCDs) and starts when
// the last of them is free. The next team placed is the one that can start
// earliest (ties: the most work, cost x B, then the lower member index), so
// small teams fill the workgroups that larger ones would leave waiting. On the
// 64-keyframe mix the cost model's makespan is 1.04 times its busy-time bound,
// against 1.17 with the teams placed in order of decreasing cost (measured:
// 7.4 against 8.3 ms per batched solve). Every workgroup's queue follows the
// one global team order, which keeps the launch free of deadlock.
void schedule(kf_batch* b, const std::vector<int>& active) {
  std::vector<double> cost(b->m.size(), 0.0);
  for (int c : active) cost[c] = team_cost(b->m[c]);
  std::vector<double> avail(b->grid, 0.0);
  std::vector<std::vector<int32_t>> q(b->grid);
  std::vector<int> idx(b->grid);
  std::vector<double> sorted_avail(b->grid);
  std::vector<int> rest(active);
  while (!rest.empty()) {
    sorted_avail = avail;
    std::sort(sorted_avail.begin(), sorted_avail.end());
    size_t pick = 0;
    for (size_t r = 1; r < rest.size(); ++r) {
      const int x = rest[r], y = rest[pick];
      const double sx = sorted_avail[b->m[x]->tiling.blocks - 1], sy = sorted_avail[b->m[y]->tiling.blocks - 1];
      const double wx = cost[x] * b->m[x]->tiling.blocks, wy = cost[y] * b->m[y]->tiling.blocks;
      if (sx < sy || (sx == sy && (wx > wy || (wx == wy && x < y)))) pick = r;
    }
    const int c = rest[pick];
    rest.erase(rest.begin() + (std::ptrdiff_t)pick);
    const int B = b->m[c]->tiling.blocks;
    for (int g = 0; g < b->grid; ++g) idx[g] = g;
    std::partial_sort(idx.begin(), idx.begin() + B, idx.end(), [&](int x, int y) {
      return avail[x] < avail[y] || (avail[x] == avail[y] && x < y);
    });
    std::sort(idx.begin(), idx.begin() + B);
    double start = 0.0;
    for (int k = 0; k < B; ++k) start = std::max(start, avail[idx[k]]);
    for (int k = 0; k < B; ++k) {
      avail[idx[k]] = start + cost[c];
      q[idx[k]].push_back((int32_t)((c << 8) | k));
    }
  }
  b->queue.clear();
  b->qoff.assign(1, 0);
  b->max_queue = 0;
  for (int g = 0; g < b->grid; ++g) {
    b->queue.insert(b->queue.end(), q[g].begin(), q[g].end());
    b->qoff.push_back((int32_t)b->queue.size());
    b->max_queue = std::max(b->max_queue, (int)q[g].size());
  }
}

hipError_t enqueue(kf_batch* b, int which, hipStream_t s) {
  hipError_t e = hipSuccess;
  if (which != 2)
    e = launch_stereo_batch(b->prec, b->pattern, b->ns, b->d_st(), b->d_n(), (int)b->m.size(), b->cus, s);
  if (e == hipSuccess && which != 1)
    e = launch_solve_batch(b->prec, b->threads, b->ppt, b->kind, b->d_so, b->d_queue(), b->d_qoff(), b->grid,
                           b->smem, s);
  return e;
}

// Captures launch sequence `which` once on the private stream.
hipError_t graph_for(kf_batch* b, int which) {
  if (b->exec[which]) return hipSuccess;
  hipError_t e = hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  const hipError_t el = enqueue(b, which, b->capture);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(b->capture, &g);
  if (el != hipSuccess || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return el != hipSuccess ? el : e;
  }
  e = hipGraphInstantiate(&b->exec[which], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  return e;
}

// One call: validates, fills the free pinned buffer (active count, stereo
// arguments, team queues), uploads it, launches sequence `which` (0 fuse,
// 1 stereo, 2 solve) and advances the members' frame / epoch counters.
kf_status run_call(kf_batch* b, int which, const std::vector<int>& active, const uint8_t* const* images,
                   const double* poses, const char* who) {
  const bool stereo = which != 2, solve = which != 1;
  for (size_t k = 0; k < active.size(); ++k) {
    const int i = active[k];
    if (!b->m[i]->has_prior)
      return bfail(b, KF_ERR_STATE, std::string(who) + ": member " + std::to_string(i) + " has no prior (kf_set_prior)");
    if (stereo) {
      if (!images[k]) return bfail(b, KF_ERR_ARG, std::string(who) + ": NULL image for member " + std::to_string(i));
      if (!pose_ok(poses + 16 * k))
        return bfail(b, KF_ERR_ARG, std::string(who) + ": pose of member " + std::to_string(i) +
                                    " must be finite with last row 0 0 0 1");
    }
  }
  // the pinned buffer of this parity was last read by the upload two calls ago
  const int p = b->parity;
  hipError_t e = hipSuccess;
  if (b->ev_used[p]) {
    e = hipEventSynchronize(b->ev[p]);
    if (e != hipSuccess) return bhip(b, e, who);
  }
  char* h = b->h_pin[p];
  int32_t* hn = reinterpret_cast<int32_t*>(h + b->dl.hdr);
  StereoArgs* hst = reinterpret_cast<StereoArgs*>(h + b->dl.st);
  *hn = stereo ? (int32_t)active.size() : 0;
  if (stereo)
    for (size_t k = 0; k < active.size(); ++k)
      if (!stereo_args(b->m[active[k]], images[k], poses + 16 * k, &hst[k]))
        return bfail(b, KF_ERR_ARG, std::string(who) + ": singular pose for member " + std::to_string(active[k]));
  if (solve) {
    schedule(b, active);
    std::memcpy(h + b->dl.queue, b->queue.data(), b->queue.size() * 4);
    std::memcpy(h + b->dl.qoff, b->qoff.data(), b->qoff.size() * 4);
    for (int i : active) {
      e = epoch_wrap_if_needed(b->m[i], solve_epoch_bound(b->m[i]->cfg));
      if (e != hipSuccess) return bhip(b, e, std::string(who) + " (epoch wrap)");
    }
  } else {
    std::memset(h + b->dl.qoff, 0, (size_t)(b->grid + 1) * 4);
  }
  e = hipMemcpyAsync(b->d_dyn, h, b->dl.total, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipEventRecord(b->ev[p], b->stream);
  if (e != hipSuccess) return bhip(b, e, std::string(who) + " (descriptor upload)");
  b->ev_used[p] = true;
  b->parity ^= 1;
  if (b->use_graph) {
    e = graph_for(b, which);
    if (e == hipSuccess) e = hipGraphLaunch(b->exec[which], b->stream);
  } else {
    e = enqueue(b, which, b->stream);
  }
  if (e != hipSuccess) return bhip(b, e, who);
  for (int i : active) {
    if (stereo) ++b->m[i]->frame;
    if (solve) b->m[i]->epoch += solve_epoch_bound(b->m[i]->cfg);
  }
  return KF_OK;
}

std::vector<int> all_members(const kf_batch* b) {
  std::vector<int> v(b->m.size());
  for (size_t i = 0; i < v.size(); ++i) v[i] = (int)i;
  return v;
}

}  // namespace

extern "C" {

void kf_batch_config_default(kf_batch_config* cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->use_graph = 1;
}

size_t kf_batch_workspace_bytes(kf_ctx* const* members, int32_t n) {
  if (!members || n < 1 || n > KF_BATCH_MAX) return 0;
  for (int i = 0; i < n; ++i)
    if (!members[i]) return 0;
  return static_bytes(n) + dyn_layout(n, total_members(members, n)).total;
}

kf_status kf_batch_create(kf_ctx* const* members, int32_t n, const kf_batch_config* cfg, kf_batch** out) {
  if (!out) return KF_ERR_ARG;
  *out = nullptr;
  if (!members || !cfg || n < 1 || n > KF_BATCH_MAX) return KF_ERR_ARG;
  if (cfg->use_graph != 0 && cfg->use_graph != 1) return KF_ERR_ARG;
  for (int i = 0; i < n; ++i) {
    if (!members[i]) return KF_ERR_ARG;
    for (int j = 0; j < i; ++j)
      if (members[j] == members[i]) return KF_ERR_ARG;
  }
  const kf_ctx* c0 = members[0];
  for (int i = 0; i < n; ++i) {
    const kf_ctx* c = members[i];
    if (c->cfg.pipeline_frames || c->cfg.precision != c0->cfg.precision || c->cfg.pattern != c0->cfg.pattern ||
        c->cfg.n_samples != c0->cfg.n_samples || c->tiling.threads != c0->tiling.threads ||
        solve_pipelined(c->cfg) != solve_pipelined(c0->cfg) || c->device != c0->device ||
        c->stream != reinterpret_cast<hipStream_t>(cfg->stream))
      return KF_ERR_ARG;
  }
  const int members_total = total_members(members, n);
  const DynLayout dl = dyn_layout(n, members_total);
  if (!cfg->workspace) return KF_ERR_ARG;
  if (cfg->workspace_bytes < static_bytes(n) + dl.total) return KF_ERR_OOM;
  if (reinterpret_cast<uintptr_t>(cfg->workspace) % 256 != 0) return KF_ERR_ARG;

  kf_batch* b = new (std::nothrow) kf_batch();
  if (!b) return KF_ERR_OOM;
  b->m.assign(members, members + n);
  b->stream = reinterpret_cast<hipStream_t>(cfg->stream);
  b->device = c0->device;
  b->prec = c0->cfg.precision;
  b->pattern = c0->cfg.pattern;
  b->ns = c0->cfg.n_samples;
  b->threads = c0->tiling.threads;
  b->pipelined = solve_pipelined(c0->cfg);
  b->kind = b->pipelined ? 1 : 0;
  for (int i = 0; i < n; ++i) b->kind |= solve_kind(members[i]->cfg) & 2;
  b->use_graph = cfg->use_graph != 0;
  b->cus = device_cus(c0->device);
  b->dl = dl;
  char* ws = reinterpret_cast<char*>(cfg->workspace);
  b->d_so = reinterpret_cast<SolveArgs*>(ws);
  b->d_dyn = ws + static_bytes(n);

  int maxB = 0;
  size_t smem = 0;
  for (kf_ctx* c : b->m) {
    b->ppt = std::max(b->ppt, c->tiling.ppt);
    maxB = std::max(maxB, c->tiling.blocks);
    smem = std::max(smem, solve_smem_bytes(b->prec, c->tiling));
  }
  if (!solve_batch_supported(b->prec, b->threads, b->ppt)) {
    delete b;
    return KF_ERR_ARG;
  }
  // LDS: the largest member's need (team partials + the three rings of its tile)
  b->smem = smem;
  b->capacity = solve_batch_coresident(b->prec, b->threads, b->ppt, b->kind, b->smem, b->device);
  if (b->capacity < maxB) {
    delete b;
    return KF_ERR_ARG;
  }
  b->grid = std::min(b->capacity, members_total);
  schedule(b, all_members(b));
  const int full_queue = b->max_queue;

  std::vector<SolveArgs> so(n);
  for (int i = 0; i < n; ++i) {
    solve_args(b->m[i], &so[i]);
    // a member may wait for its team while the team's other members finish
    // the teams queued before it
    so[i].timeout_ticks = b->m[i]->timeout_ticks * (uint64_t)full_queue;
  }
  hipError_t e = hipMemcpy(b->d_so, so.data(), n * sizeof(SolveArgs), hipMemcpyHostToDevice);
  for (int i = 0; i < 2 && e == hipSuccess; ++i) {
    e = hipHostMalloc(reinterpret_cast<void**>(&b->h_pin[i]), dl.total, hipHostMallocDefault);
    if (e == hipSuccess) {
      std::memset(b->h_pin[i], 0, dl.total);
      e = hipEventCreateWithFlags(&b->ev[i], hipEventDisableTiming);
    }
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
  if (e == hipSuccess && b->use_graph) e = graph_for(b, 0);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    delete b;
    return KF_ERR_HIP;
  }
  *out = b;
  return KF_OK;
}

void kf_batch_destroy(kf_batch* b) { delete b; }

const char* kf_batch_last_error(const kf_batch* b) {
  if (!b) return "no batch";
  return b->err.c_str();
}

kf_status kf_batch_layout(const kf_batch* b, int32_t out[4]) {
  if (!b || !out) return KF_ERR_ARG;
  out[0] = b->grid;
  out[1] = b->threads;
  out[2] = b->ppt;
  out[3] = b->max_queue;
  return KF_OK;
}

kf_status kf_batch_fuse(kf_batch* b, const uint8_t* const* images, const double* poses) {
  if (!b) return KF_ERR_ARG;
  if (!images || !poses) return bfail(b, KF_ERR_ARG, "kf_batch_fuse: NULL images or poses");
  return run_call(b, 0, all_members(b), images, poses, "kf_batch_fuse");
}

kf_status kf_batch_fuse_subset(kf_batch* b, int32_t n_active, const int32_t* members, const uint8_t* const* images,
                               const double* poses) {
  if (!b) return KF_ERR_ARG;
  if (n_active < 0 || n_active > (int32_t)b->m.size())
    return bfail(b, KF_ERR_ARG, "kf_batch_fuse_subset: n_active out of range");
  if (n_active == 0) return KF_OK;
  if (!members || !images || !poses) return bfail(b, KF_ERR_ARG, "kf_batch_fuse_subset: NULL argument");
  std::vector<int> active(members, members + n_active);
  std::vector<char> seen(b->m.size(), 0);
  for (int i : active) {
    if (i < 0 || i >= (int)b->m.size() || seen[i])
      return bfail(b, KF_ERR_ARG, "kf_batch_fuse_subset: member indices must be distinct and in range");
    seen[i] = 1;
  }
  return run_call(b, 0, active, images, poses, "kf_batch_fuse_subset");
}

kf_status kf_batch_stereo_update(kf_batch* b, const uint8_t* const* images, const double* poses) {
  if (!b) return KF_ERR_ARG;
  if (!images || !poses) return bfail(b, KF_ERR_ARG, "kf_batch_stereo_update: NULL images or poses");
  return run_call(b, 1, all_members(b), images, poses, "kf_batch_stereo_update");
}

kf_status kf_batch_solve(kf_batch* b) {
  if (!b) return KF_ERR_ARG;
  return run_call(b, 2, all_members(b), nullptr, nullptr, "kf_batch_solve");
}

}  // extern "C"
