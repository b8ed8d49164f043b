// Batched scoring of size groups (sections 3-4: the files are split into
// size groups and each group is classified by its own two-class model; a
// group without a model borrows the next trained group's).
//
// All groups of a call are scored by ONE persistent launch over the
// concatenation of every group's blocks (a block is the two-class kernel's
// unit: R row-steps of 64/LPR files).  Two schedules:
//   * static ranges (the default): workgroup w takes the w-th of grid equal
//     contiguous runs of blocks.  A run crosses few group boundaries (a group
//     averages hundreds of blocks); at each one the workgroup stages the new
//     group's scoring rows in LDS and goes on.  The four waves of a
//     workgroup take every fourth block of the run, with the single-model
//     kernel's pipeline.  Balanced by construction, no atomics.
//   * dynamic items: the host cuts every group into items of at most `tile`
//     blocks, sorted largest first; each workgroup takes the next item from
//     a device counter (longest-processing-time order: at most one small
//     item of imbalance per workgroup at the end).  The counter pair (next
//     item, finished workgroups) is zero between launches: the last
//     workgroup to finish re-arms it, so a captured graph replays the launch
//     with no memset node.  Launches that share a counter must not overlap.
// A plan times both (and several tiles) and keeps the fastest.
//
// Each file's summation order is that of the single-model kernel for the
// same (F, xtype): results are identical to scoring each group alone with
// nb_score, whatever the schedule, the tile, the grid or the order in which
// work runs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "nb_score2.hpp"

namespace nb {
namespace {

struct GroupItem {
  int64_t block0;     // first block of the item, in its group's rows
  int32_t group;      // descriptor index
  int32_t nblocks;
};
static_assert(sizeof(GroupItem) == 16, "item layout");
static_assert(sizeof(Score2Args) <= kGroupDescBound, "descriptor bound used by serving");

struct GroupsArgs {
  const Score2Args* descs;   // [n_groups]
  const GroupItem* items;    // dynamic: [n_items], largest first
  const int64_t* gstart;     // static: [n_groups + 1] first block of each group
  int32_t* counter;          // dynamic: [2] next item, finished workgroups
  int32_t n_items;
  int32_t n_groups;
  int64_t total_blocks;
};

template <int XT, int LPR, int NS, bool BIN, bool MULTI>
__global__ __launch_bounds__(kThreads) void score2_groups_static_kernel(GroupsArgs g) {
  extern __shared__ float tbl[];        // [NS][Fp] of the current group
  __shared__ float stage[kWaves][NS][(64 / LPR) * kRowSteps];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t B = g.total_blocks;
  int64_t b = B * blockIdx.x / gridDim.x;
  const int64_t b1 = B * (blockIdx.x + 1) / gridDim.x;
  if (b >= b1) return;
  // the group holding block b: the last gi with gstart[gi] <= b
  int lo = 0, hi = g.n_groups - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (g.gstart[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  for (int gi = lo; b < b1; ++gi) {
    const int64_t gs = g.gstart[gi];
    const int64_t seg_end = min(b1, g.gstart[gi + 1]);
    if (seg_end <= b) continue;                 // empty group
    const Score2Args a = g.descs[gi];
    __syncthreads();                            // the previous group's table is no longer read
    stage_table<NS>(a, tbl);
    __syncthreads();
    score_blocks<XT, LPR, NS, BIN, MULTI>(a, tbl, (b - gs) + wave, kWaves, seg_end - gs, stage);
    b = seg_end;
  }
}

template <int XT, int LPR, int NS, bool BIN, bool MULTI>
__global__ __launch_bounds__(kThreads) void score2_groups_kernel(GroupsArgs g) {
  extern __shared__ float tbl[];        // [NS][Fp] of the current item's group
  __shared__ float stage[kWaves][NS][(64 / LPR) * kRowSteps];
  __shared__ int32_t s_item;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(g.counter, 1);
    // the barrier also ends every read of the previous item's table
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    if (it >= g.n_items) break;
    const GroupItem item = g.items[it];
    const Score2Args a = g.descs[item.group];
    stage_table<NS>(a, tbl);
    __syncthreads();
    score_blocks<XT, LPR, NS, BIN, MULTI>(a, tbl, item.block0 + wave, kWaves, item.block0 + item.nblocks, stage);
  }
  // every workgroup has taken its last item when the finished count reaches
  // the grid size: the last one re-arms the counters for the next launch
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(g.counter + 1, 1) == (int32_t)gridDim.x - 1) {
      __threadfence();
      atomicExch(g.counter, 0);
      atomicExch(g.counter + 1, 0);
    }
  }
}

struct Grouped {
  template <int XT, int LPR, int NS, bool BIN, bool MULTI>
  static const void* fn() {
    return reinterpret_cast<const void*>(score2_groups_kernel<XT, LPR, NS, BIN, MULTI>);
  }
};

struct GroupedStatic {
  template <int XT, int LPR, int NS, bool BIN, bool MULTI>
  static const void* fn() {
    return reinterpret_cast<const void*>(score2_groups_static_kernel<XT, LPR, NS, BIN, MULTI>);
  }
};

constexpr size_t kCounterBytes = 256;

// Everything the host knows about one grouped call, before any device work.
struct GroupSetup {
  std::vector<Score2Args> descs;
  std::vector<int64_t> blocks;     // blocks per group
  int64_t n_files = 0;
  int F = 0, lpr = 0, ns = 1, nch = 1;
  bool bin = false;
  int xtype = 0, wtype = 0;
  size_t lds = 0;
  const void* fn = nullptr;        // dynamic-item kernel
  const void* fn_static = nullptr; // static-range kernel
  int grid_cap = 1;                // resident workgroups on the device
  int64_t total_blocks = 0;
};

int setup_groups(const nb_model* models, int32_t n_models, const nb_group* groups, int32_t n_groups, int32_t xtype,
                 int32_t wtype, GroupSetup* S) {
  if (!models || n_models < 1) return fail(NB_EINVAL, "models: need at least one");
  if (!groups || n_groups < 1) return fail(NB_EINVAL, "groups: need at least one");
  if (elem_bytes(xtype) == 0) return fail(NB_EINVAL, "unknown feature type");
  if (wtype != NB_W_F32 && wtype != NB_W_BF16) return fail(NB_EINVAL, "unknown table type");
  std::vector<char> has(n_groups);
  for (int32_t g = 0; g < n_groups; ++g) {
    const int32_t mi = groups[g].model;
    if (mi < -1 || mi >= n_models) return fail(NB_EINVAL, "group " + std::to_string(g) + ": model index out of range");
    if (groups[g].reserved != 0) return fail(NB_EINVAL, "nb_group.reserved must be 0");
    has[g] = mi >= 0;
  }
  std::vector<int32_t> route(n_groups);
  route_trained(has.data(), n_groups, route.data());
  if (route[0] < 0) return fail(NB_ENOMODEL, "no group has a model to fall back on");
  // every model in use: two classes, one kind, one feature count
  const nb_model* ref = &models[groups[route[0]].model];
  S->F = ref->n_features;
  S->bin = ref->kind == NB_BERNOULLI;
  S->ns = 1;
  for (int32_t g = 0; g < n_groups; ++g)
    if (groups[g].scores && groups[g].n > 0) S->ns = 2;
  S->descs.resize(n_groups);
  S->blocks.assign(n_groups, 0);
  S->lpr = lanes_per_row(S->F);
  const int64_t br = (int64_t)(64 / S->lpr) * kRowSteps;
  for (int32_t g = 0; g < n_groups; ++g) {
    const nb_group& G = groups[g];
    const nb_model* m = &models[groups[route[g]].model];
    if (m->n_classes != 2)
      return fail(NB_EINVAL, "group scoring takes two-class models (benign / malware per size group)");
    if (m->n_features != S->F || (m->kind == NB_BERNOULLI) != S->bin)
      return fail(NB_EINVAL, "all group models must share the kind and the feature count");
    if (G.n < 0) return fail(NB_EINVAL, "group " + std::to_string(g) + ": n must be >= 0");
    Score2Args a{};
    if (G.n > 0) {
      nb_layout L;
      int rc = check_score_args(m, &L, G.x, xtype, G.n, G.ld, wtype, G.labels, G.log_post, G.scores);
      if (rc) return fail(rc, "group " + std::to_string(g) + ": " + nb_last_error());
      rc = make_score2_args(m, L, G.x, xtype, G.n, G.ld, wtype, G.labels, G.log_post, G.scores, S->ns, &a);
      if (rc) return rc;
      S->blocks[g] = (G.n + br - 1) / br;
      S->n_files += G.n;
      S->nch = a.nch;
    } else {
      nb_layout L;
      int rc = check_model(m, &L);
      if (rc) return rc;
    }
    S->descs[g] = a;
  }
  S->xtype = xtype;
  S->wtype = wtype;
  nb_layout L;
  compute_layout(2, S->F, &L);
  S->lds = (size_t)S->ns * L.padded_features * sizeof(float);
  if (S->lds > kMaxTableLds) return fail(NB_EINVAL, "two-class scoring supports F up to 16384 (table staged in LDS)");
  const int cw = 16 * S->lpr;
  S->nch = (S->F + cw - 1) / cw;
  S->fn = pick_score2<Grouped>(xtype, S->lpr, S->nch > 1, S->ns, S->bin);
  S->fn_static = pick_score2<GroupedStatic>(xtype, S->lpr, S->nch > 1, S->ns, S->bin);
  if (S->lds > 64 * 1024) {
    NB_HIP_CHECK(hipFuncSetAttribute(S->fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)S->lds));
    NB_HIP_CHECK(hipFuncSetAttribute(S->fn_static, hipFuncAttributeMaxDynamicSharedMemorySize, (int)S->lds));
  }
  S->grid_cap = resident_per_cu(S->fn, kThreads, S->lds) * device_cu_count();
  for (int64_t b : S->blocks) S->total_blocks += b;
  return NB_OK;
}

// Blocks per item: whole multiples of the four waves, about four items per
// resident workgroup over the whole call, within [4, 256] blocks.
int default_tile_blocks(const GroupSetup& S) {
  int64_t total = 0;
  for (int64_t b : S.blocks) total += b;
  int64_t t = total / (4 * (int64_t)std::max(1, S.grid_cap));
  t = std::max<int64_t>(kWaves, std::min<int64_t>(256, t));
  return (int)((t + kWaves - 1) / kWaves * kWaves);
}

int tile_blocks_from_rows(const GroupSetup& S, int32_t tile_rows) {
  const int br = (64 / S.lpr) * kRowSteps;
  const int64_t b = ((int64_t)tile_rows + br - 1) / br;
  return (int)std::max<int64_t>(kWaves, (b + kWaves - 1) / kWaves * kWaves);
}

std::vector<GroupItem> make_items(const GroupSetup& S, int tile_blocks) {
  std::vector<GroupItem> items;
  for (size_t g = 0; g < S.blocks.size(); ++g)
    for (int64_t b0 = 0; b0 < S.blocks[g]; b0 += tile_blocks)
      items.push_back(GroupItem{b0, (int32_t)g, (int32_t)std::min<int64_t>(tile_blocks, S.blocks[g] - b0)});
  // largest first; equal sizes keep group and row order
  std::stable_sort(items.begin(), items.end(),
                   [](const GroupItem& a, const GroupItem& b) { return a.nblocks > b.nblocks; });
  return items;
}

// A schedule is a tile size in blocks: 0 = static ranges, > 0 = dynamic
// items of at most that many blocks.  Its device image (the work list):
//   [256-byte header: two zeroed int32 counters]
//   [descriptors, one per group]
//   [payload: items (dynamic) or the first block of each group plus the
//    total (static: n_groups + 1 int64)]
struct WorkList {
  int tile_blocks = 0;
  std::vector<GroupItem> items;
  std::vector<int64_t> gstart;
  int32_t n_items() const { return (int32_t)items.size(); }
};

WorkList make_work_list(const GroupSetup& S, int tile_blocks) {
  WorkList w;
  w.tile_blocks = tile_blocks;
  if (tile_blocks == 0) {
    w.gstart.resize(S.blocks.size() + 1);
    int64_t acc = 0;
    for (size_t g = 0; g < S.blocks.size(); ++g) {
      w.gstart[g] = acc;
      acc += S.blocks[g];
    }
    w.gstart[S.blocks.size()] = acc;
  } else {
    w.items = make_items(S, tile_blocks);
  }
  return w;
}

size_t payload_bytes(const WorkList& w) {
  return w.tile_blocks == 0 ? w.gstart.size() * sizeof(int64_t) : w.items.size() * sizeof(GroupItem);
}

size_t work_list_bytes(size_t n_groups, size_t payload) {
  return kCounterBytes + align_up(n_groups * sizeof(Score2Args), kAlign) + align_up(payload, kAlign);
}

struct DevLists {
  int32_t* counter;
  Score2Args* descs;
  void* payload;
};

DevLists carve(void* ws, size_t n_groups) {
  uint8_t* p = static_cast<uint8_t*>(ws);
  DevLists d;
  d.counter = reinterpret_cast<int32_t*>(p);
  d.descs = reinterpret_cast<Score2Args*>(p + kCounterBytes);
  d.payload = p + kCounterBytes + align_up(n_groups * sizeof(Score2Args), kAlign);
  return d;
}

// The device image of a work list (counters zeroed).
void serialise(const GroupSetup& S, const WorkList& w, std::vector<uint8_t>* blob) {
  const size_t ng = S.descs.size();
  blob->assign(work_list_bytes(ng, payload_bytes(w)), 0);
  std::memcpy(blob->data() + kCounterBytes, S.descs.data(), ng * sizeof(Score2Args));
  uint8_t* pay = blob->data() + kCounterBytes + align_up(ng * sizeof(Score2Args), kAlign);
  if (w.tile_blocks == 0) std::memcpy(pay, w.gstart.data(), payload_bytes(w));
  else std::memcpy(pay, w.items.data(), payload_bytes(w));
}

// Launch geometry of a schedule: the kernel and the number of workgroups.
struct Geometry {
  const void* fn = nullptr;
  int grid = 0;
};

Geometry geometry(const GroupSetup& S, const WorkList& w) {
  Geometry G;
  if (w.tile_blocks == 0) {
    G.fn = S.fn_static;
    // every workgroup gets at least a few blocks per wave
    const int64_t most = std::max<int64_t>(1, S.total_blocks / (2 * kWaves));
    G.grid = (int)std::max<int64_t>(1, std::min<int64_t>(S.grid_cap, most));
  } else {
    G.fn = S.fn;
    G.grid = std::max(1, std::min(S.grid_cap, w.n_items()));
  }
  return G;
}

int launch_grouped(const void* fn, size_t lds, int grid, const DevLists& d, int32_t n_groups, int32_t n_items,
                   int64_t total_blocks, bool is_static, hipStream_t s) {
  if (total_blocks == 0) return NB_OK;
  GroupsArgs g;
  g.descs = d.descs;
  g.items = is_static ? nullptr : static_cast<const GroupItem*>(d.payload);
  g.gstart = is_static ? static_cast<const int64_t*>(d.payload) : nullptr;
  g.counter = d.counter;
  g.n_items = n_items;
  g.n_groups = n_groups;
  g.total_blocks = total_blocks;
  void* args[] = {&g};
  NB_HIP_CHECK(hipLaunchKernel(fn, dim3(grid), dim3(kThreads), args, lds, s));
  NB_HIP_CHECK(hipGetLastError());
  return NB_OK;
}

int launch_grouped(const GroupSetup& S, const WorkList& w, const DevLists& d, hipStream_t s) {
  const Geometry G = geometry(S, w);
  return launch_grouped(G.fn, S.lds, G.grid, d, (int32_t)S.descs.size(), w.n_items(), S.total_blocks,
                        w.tile_blocks == 0, s);
}

// ------------------------------------------------------------ tile cache
// Tuned schedules persist in a flat JSON object {"key": tile_blocks, ...}
// (0 = static ranges) at the path named by NB_TUNE_CACHE (when set); always
// kept in memory.
std::mutex g_tune_mu;
std::map<std::string, int> g_tune;
bool g_tune_loaded = false;

std::string tune_key(const GroupSetup& S, int32_t n_groups) {
  char buf[160];
  std::snprintf(buf, sizeof buf, "score2_groups/F%d/x%d/w%d/ns%d/%s/g%d/n%lld/cu%d", S.F, S.xtype, S.wtype, S.ns,
                S.bin ? "bern" : "mult", n_groups, (long long)S.n_files, device_cu_count());
  return buf;
}

void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("NB_TUNE_CACHE");
  if (!path) return;
  std::ifstream f(path);
  if (!f) return;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string t = ss.str();
  size_t i = 0;
  while ((i = t.find('"', i)) != std::string::npos) {
    const size_t j = t.find('"', i + 1);
    if (j == std::string::npos) break;
    const std::string key = t.substr(i + 1, j - i - 1);
    size_t k = t.find(':', j);
    if (k == std::string::npos) break;
    const int v = std::atoi(t.c_str() + k + 1);
    if (v >= 0) g_tune[key] = v;
    i = t.find_first_of(",}", k);
    if (i == std::string::npos) break;
  }
}

void tune_store_locked() {
  const char* path = std::getenv("NB_TUNE_CACHE");
  if (!path) return;
  std::ofstream f(path, std::ios::trunc);
  if (!f) return;
  f << "{";
  bool first = true;
  for (const auto& kv : g_tune) {
    f << (first ? "\n  \"" : ",\n  \"") << kv.first << "\": " << kv.second;
    first = false;
  }
  f << "\n}\n";
}

// tile in blocks (0 = static ranges), or -1 when the shape was never tuned
int tune_lookup(const std::string& key) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  auto it = g_tune.find(key);
  return it == g_tune.end() ? -1 : it->second;
}

void tune_record(const std::string& key, int tile_blocks) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  g_tune[key] = tile_blocks;
  tune_store_locked();
}

}  // namespace

int prepare_group_launch(const nb_model* models, int32_t n_models, const nb_group* groups, int32_t n_groups,
                         int32_t xtype, int32_t wtype, int32_t tile_rows, std::vector<uint8_t>* blob,
                         GroupLaunch* out) {
  GroupSetup S;
  int rc = setup_groups(models, n_models, groups, n_groups, xtype, wtype, &S);
  if (rc) return rc;
  if (tile_rows < 0) return fail(NB_EINVAL, "tile_rows must be >= 0");
  const WorkList w = make_work_list(S, tile_rows > 0 ? tile_blocks_from_rows(S, tile_rows) : 0);
  serialise(S, w, blob);
  const Geometry G = geometry(S, w);
  out->fn = G.fn;
  out->lds = S.lds;
  out->grid = G.grid;
  out->n_items = w.n_items();
  out->n_groups = n_groups;
  out->is_static = w.tile_blocks == 0;
  out->total_blocks = S.total_blocks;
  out->blob_bytes = blob->size();
  return NB_OK;
}

int enqueue_group_launch(const GroupLaunch& L, void* dev_blob, hipStream_t s) {
  return launch_grouped(L.fn, L.lds, L.grid, carve(dev_blob, L.n_groups), L.n_groups, L.n_items, L.total_blocks,
                        L.is_static, s);
}

}  // namespace nb

using namespace nb;

// ------------------------------------------------------------------ plan
struct nb_group_plan {
  GroupSetup S;
  void* dev = nullptr;            // work list: counters, descriptors, payload
  size_t dev_bytes = 0;
  int32_t n_groups = 0;
  WorkList w;
  int tuned = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

int upload(nb_group_plan* p, const WorkList& w) {
  std::vector<uint8_t> blob;
  serialise(p->S, w, &blob);
  if (blob.size() > p->dev_bytes) return fail(NB_EHIP, "internal: work list larger than its buffer");
  NB_HIP_CHECK(hipMemcpy(p->dev, blob.data(), blob.size(), hipMemcpyHostToDevice));
  p->w = w;
  return NB_OK;
}

// Time the static schedule and several dynamic tiles on the caller's data;
// keep the fastest.
int autotune(nb_group_plan* p, hipStream_t s) {
  std::vector<int> cand = {0};
  const int def = default_tile_blocks(p->S);
  for (int t : {8, 16, 32, 64, 128, def}) cand.push_back(t);
  std::sort(cand.begin() + 1, cand.end());
  cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
  hipEvent_t e0, e1;
  NB_HIP_CHECK(hipEventCreate(&e0));
  NB_HIP_CHECK(hipEventCreate(&e1));
  float best = 1e30f;
  int best_t = 0;
  int rc = NB_OK;
  const DevLists d = carve(p->dev, p->n_groups);
  for (int t : cand) {
    const WorkList w = make_work_list(p->S, t);
    if ((rc = upload(p, w))) break;
    if ((rc = launch_grouped(p->S, w, d, s))) break;   // warm
    float tot = 0.0f;
    for (int r = 0; r < 3 && rc == NB_OK; ++r) {
      if (hipEventRecord(e0, s) != hipSuccess) rc = fail(NB_EHIP, "hipEventRecord");
      if (!rc) rc = launch_grouped(p->S, w, d, s);
      if (!rc && hipEventRecord(e1, s) != hipSuccess) rc = fail(NB_EHIP, "hipEventRecord");
      if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = fail(NB_EHIP, "hipEventSynchronize");
      float ms = 0.0f;
      if (!rc) hipEventElapsedTime(&ms, e0, e1);
      tot += ms;
    }
    if (rc) break;
    if (tot < best) {
      best = tot;
      best_t = t;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc) return rc;
  p->w.tile_blocks = best_t;
  p->tuned = 1;
  return NB_OK;
}

void plan_free(nb_group_plan* p) {
  if (!p) return;
  if (p->exec) hipGraphExecDestroy(p->exec);
  if (p->graph) hipGraphDestroy(p->graph);
  if (p->dev) hipFree(p->dev);
  delete p;
}

int plan_build(nb_group_plan* p, const nb_model* models, int32_t n_models, const nb_group* groups, int32_t n_groups,
               int32_t xtype, int32_t wtype, int32_t tile_rows, int32_t flags, hipStream_t s) {
  int rc = setup_groups(models, n_models, groups, n_groups, xtype, wtype, &p->S);
  if (rc) return rc;
  p->n_groups = n_groups;
  // room for the largest work list any schedule makes (the smallest tile)
  const WorkList smallest = make_work_list(p->S, kWaves);
  p->dev_bytes = std::max(work_list_bytes(n_groups, payload_bytes(smallest)),
                          work_list_bytes(n_groups, (n_groups + 1) * sizeof(int64_t)));
  NB_HIP_CHECK(hipStreamSynchronize(s));
  NB_HIP_CHECK(hipMalloc(&p->dev, p->dev_bytes));
  const std::string key = tune_key(p->S, n_groups);
  int tile = 0;
  if (tile_rows > 0) {
    tile = tile_blocks_from_rows(p->S, tile_rows);
  } else if ((tile = tune_lookup(key)) >= 0) {
    p->tuned = 2;
  } else if (flags & NB_PLAN_TUNE) {
    if ((rc = autotune(p, s))) return rc;
    tile = p->w.tile_blocks;
    tune_record(key, tile);
  } else {
    tile = 0;
  }
  if ((rc = upload(p, make_work_list(p->S, tile)))) return rc;
  // capture the launch into a graph on a private stream
  hipStream_t cs;
  NB_HIP_CHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    hipStreamDestroy(cs);
    return fail(NB_EHIP, "hipStreamBeginCapture failed");
  }
  rc = launch_grouped(p->S, p->w, carve(p->dev, n_groups), cs);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(cs, &graph);
  hipStreamDestroy(cs);
  if (rc) {
    if (graph) hipGraphDestroy(graph);
    return rc;
  }
  if (ec != hipSuccess) return hip_fail(ec, "hipStreamEndCapture");
  p->graph = graph;
  NB_HIP_CHECK(hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0));
  return NB_OK;
}

}  // namespace

extern "C" {

size_t nb_score_groups_workspace_bytes(const nb_model* models, int32_t n_models, const nb_group* groups,
                                       int32_t n_groups, int32_t xtype, int32_t wtype, int32_t tile_rows) {
  std::vector<uint8_t> blob;
  GroupLaunch L;
  if (prepare_group_launch(models, n_models, groups, n_groups, xtype, wtype, tile_rows, &blob, &L)) return 0;
  return blob.size();
}

int nb_score_groups(const nb_model* models, int32_t n_models, const nb_group* groups, int32_t n_groups,
                    int32_t xtype, int32_t wtype, int32_t tile_rows, void* workspace, size_t workspace_bytes_,
                    void* stream) {
  std::vector<uint8_t> blob;
  GroupLaunch L;
  int rc = prepare_group_launch(models, n_models, groups, n_groups, xtype, wtype, tile_rows, &blob, &L);
  if (rc) return rc;
  if (L.total_blocks == 0) return NB_OK;
  if (!workspace) return fail(NB_EINVAL, "workspace is NULL");
  if ((reinterpret_cast<uintptr_t>(workspace) & (kAlign - 1)) != 0)
    return fail(NB_EINVAL, "workspace must be 256-byte aligned");
  if (workspace_bytes_ < blob.size()) return fail(NB_ENOMEM, "workspace smaller than nb_score_groups_workspace_bytes()");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  NB_HIP_CHECK(hipMemcpyAsync(workspace, blob.data(), blob.size(), hipMemcpyHostToDevice, s));
  if ((rc = enqueue_group_launch(L, workspace, s))) return rc;
  // the work list is staged from host memory released on return
  NB_HIP_CHECK(hipStreamSynchronize(s));
  return NB_OK;
}

int nb_group_plan_create(const nb_model* models, int32_t n_models, const nb_group* groups, int32_t n_groups,
                         int32_t xtype, int32_t wtype, int32_t tile_rows, int32_t flags, void* stream,
                         nb_group_plan** out) {
  if (!out) return fail(NB_EINVAL, "out is NULL");
  *out = nullptr;
  if (tile_rows < 0) return fail(NB_EINVAL, "tile_rows must be >= 0");
  if (flags & ~NB_PLAN_TUNE) return fail(NB_EINVAL, "unknown plan flags");
  nb_group_plan* p = new (std::nothrow) nb_group_plan();
  if (!p) return fail(NB_ENOMEM, "out of host memory");
  const int rc = plan_build(p, models, n_models, groups, n_groups, xtype, wtype, tile_rows, flags,
                            reinterpret_cast<hipStream_t>(stream));
  if (rc) {
    (void)hipDeviceSynchronize();
    plan_free(p);
    return rc;
  }
  *out = p;
  return NB_OK;
}

int nb_group_plan_launch(nb_group_plan* plan, void* stream) {
  if (!plan) return fail(NB_EINVAL, "plan is NULL");
  if (plan->S.total_blocks == 0) return NB_OK;
  NB_HIP_CHECK(hipGraphLaunch(plan->exec, reinterpret_cast<hipStream_t>(stream)));
  return NB_OK;
}

int nb_group_plan_query(const nb_group_plan* plan, nb_group_plan_info* out) {
  if (!plan || !out) return fail(NB_EINVAL, "NULL argument");
  const int br = (64 / plan->S.lpr) * kRowSteps;
  const Geometry G = geometry(plan->S, plan->w);
  out->schedule = plan->w.tile_blocks == 0 ? NB_SCHEDULE_STATIC : NB_SCHEDULE_DYNAMIC;
  out->tile_rows = plan->w.tile_blocks == 0
                       ? (int32_t)std::min<int64_t>(INT32_MAX, (plan->S.total_blocks + G.grid - 1) / G.grid * br)
                       : plan->w.tile_blocks * br;
  out->n_items = plan->w.tile_blocks == 0 ? G.grid : plan->w.n_items();
  out->grid = G.grid;
  out->tuned = plan->tuned;
  out->n_files = plan->S.n_files;
  out->rows_per_block = br;
  out->lds_bytes = (int32_t)plan->S.lds;
  return NB_OK;
}

int nb_group_plan_destroy(nb_group_plan* plan) {
  if (!plan) return NB_OK;
  NB_HIP_CHECK(hipDeviceSynchronize());
  plan_free(plan);
  return NB_OK;
}

}  // extern "C"
