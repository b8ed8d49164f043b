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
#include <memory>
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

// Counts of a work list, in its device header right after the two dynamic
// counters: kernels read them at launch, so a captured launch picks up a
// work list rewritten in place (nb_group_plan_update).
struct ListCounts {
  int32_t n_items;
  int32_t n_tails;
  int32_t n_groups;
  int32_t kind;              // 0 static, 1 dynamic, 2 stream, 3 sweep
  int64_t total_blocks;      // every block (static), or the sweep's blocks (sweep)
};
static_assert(sizeof(ListCounts) == 24, "work-list header layout");

struct GroupsArgs {
  const Score2Args* descs;   // [n_groups]
  const void* payload;       // the work list's payload (see make_work_list)
  const ListCounts* counts;  // in the work list's header
  int32_t* counter;          // dynamic: [2] next item, finished workgroups
  int32_t Fp;                // padded feature count (every group's model has the same F)
  int32_t nch;               // feature chunks per row
  int32_t F;                 // features (sweep)
  int32_t wt;                // table type (sweep)
  // resolved from the header by each kernel (resolve_list)
  const GroupItem* items;    // dynamic: [n_items], largest first; stream: fast items in memory order
  const GroupItem* tails;    // stream, sweep: [n_tails] blocks scored after the items
  const int64_t* gstart;     // static: [n_groups + 1] first block of each group
  const int64_t* sstart;     // sweep: [n_groups + 1] first sweep block of each group
  int32_t n_items;
  int32_t n_tails;
  int32_t n_groups;
  int64_t total_blocks;      // every block (static), or the sweep's blocks (sweep)
};

__device__ __forceinline__ GroupsArgs resolve_list(GroupsArgs g) {
  const ListCounts c = dev::load_uniform(g.counts);
  const uint8_t* pay = static_cast<const uint8_t*>(g.payload);
  g.n_items = c.n_items;
  g.n_tails = c.n_tails;
  g.n_groups = c.n_groups;
  g.total_blocks = c.total_blocks;
  g.items = reinterpret_cast<const GroupItem*>(pay);
  g.gstart = reinterpret_cast<const int64_t*>(pay);
  g.sstart = reinterpret_cast<const int64_t*>(pay);
  g.tails = (c.kind == 3) ? reinterpret_cast<const GroupItem*>(pay + (((size_t)c.n_groups + 1) * 8 + 15) / 16 * 16)
                          : g.items + c.n_items;
  return g;
}

// ---- stream schedule (tables of at most kStreamTable floats: NS * Fp)
// Workgroup w takes the fast items w, w + grid, ... in memory order, so the
// whole machine sweeps one window of the concatenated files, as the
// single-model kernel does.  Every item holds at least four blocks, so each
// wave has work in every item.  A wave's (item, block, chunk) units form ONE
// pipelined sequence across items: the loads of the next unit are in flight
// while the current one is accumulated, item boundaries included.  The next
// item's scoring rows ride along: when a wave issues an item's first unit it
// also loads its eighth of that item's table (kStreamTPL floats per lane);
// when it consumes that unit it writes them to one of two LDS table buffers
// and meets the other waves at an LDS-only barrier (no wait on the feature
// loads in flight).  Buffer k % 2 is free again because every wave passed
// item k - 1's barrier after finishing item k - 2.  The blocks that need
// guarded loads (each group's ragged end) are scored after the stream.
constexpr int kStreamTable = 2048;
constexpr int kStreamTPL = kStreamTable / kThreads;     // 8 floats per lane

// Workgroup barrier for LDS data only: the wavefront-scope fences keep the
// compiler from moving memory accesses across it without emitting waits,
// lgkmcnt(0) completes this wave's LDS writes, and nothing waits for the
// global loads in flight (a workgroup-scope fence would).
__device__ __forceinline__ void lds_only_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0); vmcnt and expcnt untouched
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int XT, int LPR, int NS, bool BIN, bool MULTI>
__global__ __launch_bounds__(kThreads) void score2_groups_stream_kernel(GroupsArgs g_in) {
  const GroupsArgs g = resolve_list(g_in);
  constexpr int EB = (XT == NB_X_I32) ? 4 : 1;
  constexpr int NV = EB;
  constexpr int G = 64 / LPR;
  constexpr int R = row_steps<XT, false>();
  constexpr int BR = G * R;
  constexpr int CW = 16 * LPR;
  constexpr int TPL = kStreamTPL;
  using LM = LaneMap<XT, LPR>;
  __shared__ __attribute__((aligned(16))) float tbl2[2][kStreamTable];
  __shared__ __attribute__((aligned(16))) float tbl_sink[kStreamTable];
  __shared__ float stage[kWaves][NS][BR];

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int sub = lane / LPR, j = lane % LPR;
  const int nch = MULTI ? g.nch : 1;
  const int Fp = g.Fp;
  const int grid = (int)gridDim.x;
  const int my_items = (g.n_items > (int)blockIdx.x) ? (g.n_items - (int)blockIdx.x + grid - 1) / grid : 0;

  float acc[R][NS];
  auto zero_acc = [&]() {
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
      for (int s = 0; s < NS; ++s) acc[i][s] = 0.0f;
  };
  zero_acc();
  float w[NS][16];
  uint32_t keep[4] = {~0u, ~0u, ~0u, ~0u};

  if (my_items > 0) {
    // ---- issue side: the item whose unit is being loaded
    int ik = 0, ib = 0, ich = 0;
    bool at_end = false;
    GroupItem iit = dev::load_uniform(g.items + blockIdx.x);
    Score2Args ia = dev::load_uniform(g.descs + iit.group);
    int i_nbw = (iit.nblocks - wave + kWaves - 1) / kWaves;
    uint32_t voff[R];
    auto set_voff = [&](int64_t ld) {
#pragma unroll
      for (int i = 0; i < R; ++i)
        voff[i] = (uint32_t)((i * G + sub) * ld) + (uint32_t)((XT == NB_X_I32) ? 16 * j : 16 * j * EB);
    };
    set_voff(ia.ld_bytes);
    auto advance = [&]() {
      if (at_end) return;
      if (++ich < nch) return;
      ich = 0;
      if (++ib < i_nbw) return;
      if (ik + 1 >= my_items) {            // stay on the last unit: it is re-issued (an L2 hit)
        ib = i_nbw - 1;
        ich = nch - 1;
        at_end = true;
        return;
      }
      ++ik;
      ib = 0;
      iit = dev::load_uniform(g.items + blockIdx.x + ik * grid);
      ia = dev::load_uniform(g.descs + iit.group);
      i_nbw = (iit.nblocks - wave + kWaves - 1) / kWaves;
      set_voff(ia.ld_bytes);
    };
    auto issue = [&](dev::u32x4 (&dst)[R][NV], dev::u32x4 (&tdst)[2]) {
      const int64_t blk = iit.block0 + wave + (int64_t)ib * kWaves;
      const int64_t off = blk * BR * ia.ld_bytes + (int64_t)ich * CW * EB;
      const auto rsrc = dev::make_rsrc(dev::uniform_ptr(ia.x + off), dev::uniform64(ia.total_bytes - off));
      // this lane's share of the item's table: floats [TPL*tid, +TPL) of
      // the [NS][Fp] rows (FP32: 32 bytes; BF16: 16 bytes, second load
      // empty).  Units other than an item's first load from an empty range:
      // no memory access, the same number of loads in flight.
      const bool bf = __builtin_amdgcn_readfirstlane(ia.wt) == NB_W_BF16;
      const int tbytes = __builtin_amdgcn_readfirstlane((ib == 0 && ich == 0) ? NS * Fp * (bf ? 2 : 4) : 0);
      const auto trs =
          dev::make_rsrc(dev::uniform_ptr(bf ? (const void*)ia.rows16 : (const void*)ia.rows32), tbytes);
      const uint32_t toff = (uint32_t)threadIdx.x * TPL * (bf ? 2u : 4u);
      tdst[0] = dev::buffer_load16(trs, toff);
      tdst[1] = dev::buffer_load16(trs, bf ? (uint32_t)tbytes : toff + 16u);
      // loads whose features of this chunk lie past F read nothing
      if constexpr (XT == NB_X_I32) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
          const bool live = ich * CW + LM::feat0(j) + q * LM::kWStep < ia.F;
#pragma unroll
          for (int i = 0; i < R; ++i)
            dst[i][q] = dev::buffer_load16(rsrc, live ? voff[i] + q * LM::kLoadStep : dev::kNoAccess);
        }
      } else {
        const bool live = ich * CW + 16 * j < ia.F;
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
          for (int q = 0; q < NV; ++q) dst[i][q] = dev::buffer_load16(rsrc, live ? voff[i] + 16 * q : dev::kNoAccess);
      }
      __builtin_amdgcn_sched_barrier(0);
      advance();
    };

    // ---- consume side
    int ck = 0, cb = 0, cch = 0;
    GroupItem cit = iit;
    Score2Args ca = ia;
    int c_nbw = i_nbw;
    float rb[NS];
    bool done = false;
    auto consume = [&](dev::u32x4 (&src)[R][NV], const dev::u32x4 (&tsrc)[2]) {
      float* tb = tbl2[ck & 1];
      // every unit consumes its table registers the same way (the first unit
      // of an item into the item's buffer, the others into a sink), so the
      // registers are free after the write on every path
      const bool first = cb == 0 && cch == 0;
      const bool bf = __builtin_amdgcn_readfirstlane(ca.wt) == NB_W_BF16;
      float tv[TPL];
#pragma unroll
      for (int e = 0; e < TPL; ++e) {
        const uint32_t word = tsrc[0][e >> 1];
        const float from16 = __uint_as_float((e & 1) ? (word & 0xFFFF0000u) : (word << 16));
        const float from32 = __uint_as_float(tsrc[e >> 2][e & 3]);
        tv[e] = bf ? from16 : from32;
      }
      float4* t4 = reinterpret_cast<float4*>((first ? tb : tbl_sink) + threadIdx.x * TPL);
      t4[0] = make_float4(tv[0], tv[1], tv[2], tv[3]);
      t4[1] = make_float4(tv[4], tv[5], tv[6], tv[7]);
      if (first) {                                       // first unit of item ck
        lds_only_barrier();
#pragma unroll
        for (int s = 0; s < NS; ++s) rb[s] = dev::load_uniform(ca.row_bias + s);
        if (!MULTI) {
          load_table<XT, NS, LM::kWStep>(tb, Fp, (XT == NB_X_I32) ? LM::feat0(j) : 16 * j, w);
          if (XT == NB_X_FP8) fp8_keep_mask(ca.F, 16 * j, keep);
        }
      }
      if (MULTI) {
        const int fc = cch * CW + ((XT == NB_X_I32) ? LM::feat0(j) : 16 * j);
        load_table<XT, NS, LM::kWStep>(tb, Fp, fc, w);
        if (XT == NB_X_FP8) fp8_keep_mask(ca.F, fc, keep);
      }
      accumulate_rows<XT, NS, BIN, NV>(src, w, keep, true, acc);
      if (++cch == nch) {
        const int64_t row0 = (cit.block0 + wave + (int64_t)cb * kWaves) * BR;
        finish_block<LPR, NS, true>(ca, acc, lane, wave, sub, rb, row0, BR, stage);
        zero_acc();
        cch = 0;
        if (++cb == c_nbw) {
          cb = 0;
          if (++ck >= my_items) {
            done = true;
          } else {
            cit = dev::load_uniform(g.items + blockIdx.x + ck * grid);
            ca = dev::load_uniform(g.descs + cit.group);
            c_nbw = (cit.nblocks - wave + kWaves - 1) / kWaves;
          }
        }
      }
    };

    dev::u32x4 b0[R][NV], b1[R][NV];
    dev::u32x4 t0[2], t1[2];
    issue(b0, t0);
    for (;;) {
      issue(b1, t1);
      consume(b0, t0);
      if (done) break;
      issue(b0, t0);
      consume(b1, t1);
      if (done) break;
    }
  }

  // ---- blocks needing guarded loads
  for (int t = blockIdx.x; t < g.n_tails; t += grid) {
    const GroupItem it = dev::load_uniform(g.tails + t);
    const Score2Args a = dev::load_uniform(g.descs + it.group);
    __syncthreads();
    stage_table<NS>(a, tbl2[0]);
    __syncthreads();
    score_blocks<XT, LPR, NS, BIN, MULTI>(a, tbl2[0], it.block0 + wave, kWaves, it.block0 + it.nblocks, stage);
  }
}

// The stream schedule with flat staging (two-chunk byte rows; see
// score_blocks): a sweep, the single-model kernel's order over the
// concatenation of every group's blocks.  The blocks form runs of
// kSweepRun consecutive blocks; wave w of the grid takes runs w, w + W,
// w + 2W, ... (W waves) and the blocks past the last whole round one at a
// time, so the machine reads one window of memory at a time and the waves'
// block counts differ by at most kSweepRun.  Each
// block is fetched as ONE aligned window of FL 1 KB pieces into the wave's
// LDS region and read back row by row with the lane mapping of the direct
// loads (identical arithmetic).  The groups' prefix block counts and a
// compact copy of their descriptors (with the row biases) sit in LDS, so
// finding the next block's group (a ballot over the prefix counts) and its
// window never waits on memory: it runs while the current block's window
// is in flight, and the next block's loads (window and each lane's table
// weights) go out as soon as the current window has landed.  No barrier in
// the sweep.  Groups smaller than a window are tails, scored afterwards
// with the table in LDS.
constexpr int kSweepMaxGroups = 320;
constexpr int kSweepRun = 4;

struct SweepDesc {                 // one group as the sweep reads it (LDS)
  const uint8_t* x;
  int64_t ld_bytes;
  int64_t total_bytes;
  int64_t n;
  const void* table;               // rows32 or rows16 (the call's table type)
  int32_t* labels;
  float* log_post;
  float* scores;
  float rb[2];
};
static_assert(sizeof(SweepDesc) == 72, "sweep descriptor layout");

template <int XT, int NS, bool BIN, bool MULTI, int FL, bool BF>
__global__ __launch_bounds__(kThreads) void score2_groups_sweep_kernel(GroupsArgs g_in) {
  const GroupsArgs g = resolve_list(g_in);
  constexpr int LPR = 64;
  constexpr int R = block_steps<XT, false, MULTI, FL>();
  constexpr int BR = R;                 // one row per row-step
  constexpr int CW = 16 * LPR;
  constexpr int NCH = 2;                // two chunks per row
  constexpr int kPiece = 64 * 16;
  static_assert(XT != NB_X_I32 && MULTI, "the sweep stages two-chunk byte rows");
  __shared__ __attribute__((aligned(16))) uint8_t flat_all[kWaves * flat_region_bytes(FL)];
  __shared__ float stage[kWaves][NS][BR];
  __shared__ int64_t s_start[kSweepMaxGroups + 1];
  __shared__ SweepDesc s_desc[kSweepMaxGroups];

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int j = lane;
  const int ng = g.n_groups;
  constexpr bool bf = BF;               // BF16 table (else FP32)
  constexpr int TW = BF ? 2 : 4;        // 16-byte table loads per lane, chunk and row
  const int F = g.F, Fp = g.Fp;
  for (int t = threadIdx.x; t <= ng; t += kThreads) s_start[t] = g.sstart[t];
  for (int t = threadIdx.x; t < ng; t += kThreads) {
    const Score2Args& a = g.descs[t];
    SweepDesc d;
    d.x = a.x;
    d.ld_bytes = a.ld_bytes;
    d.total_bytes = a.total_bytes;
    d.n = a.n;
    d.table = bf ? (const void*)a.rows16 : (const void*)a.rows32;
    d.labels = a.labels;
    d.log_post = a.log_post;
    d.scores = a.scores;
    d.rb[0] = a.n > 0 ? a.row_bias[0] : 0.0f;
    d.rb[1] = a.n > 0 ? a.row_bias[NS - 1] : 0.0f;
    s_desc[t] = d;
  }
  __syncthreads();

  // Order: rounds of kSweepRun consecutive blocks per wave (wave w takes
  // blocks w*RUN .. w*RUN + RUN-1 of each round of W*RUN), so a wave's next
  // block is usually in the same group and keeps its table registers; the
  // blocks after the last whole round go one per wave.
  const int64_t nwaves = (int64_t)gridDim.x * kWaves;
  const int64_t gw = (int64_t)blockIdx.x * kWaves + wave;
  const int64_t total = g.total_blocks;
  const int64_t round = nwaves * kSweepRun;
  const int64_t full = total / round;                 // whole rounds
  const int64_t rem = total - full * round;
  const int nb = (int)(full * kSweepRun + (rem > gw ? (rem - gw - 1) / nwaves + 1 : 0));
  auto sweep_block = [&](int k) -> int64_t {
    const int64_t kf = full * kSweepRun;
    if (k < kf) return (k / kSweepRun) * round + gw * kSweepRun + (k % kSweepRun);
    return full * round + gw + (int64_t)(k - kf) * nwaves;
  };
  uint8_t* mine = flat_all + wave * flat_region_bytes(FL);

  float acc[R][NS];
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int s = 0; s < NS; ++s) acc[i][s] = 0.0f;
  uint32_t keep[4] = {~0u, ~0u, ~0u, ~0u};

  if (nb > 0) {
    // ---- a block ready to launch: its group, place and outputs
    struct Next {
      const uint8_t* base;              // first byte of its window
      const void* table;
      int32_t* labels;
      float* log_post;
      float* scores;
      float rb[2];
      int64_t lb;                       // block index inside its group
      int32_t ld;
      uint32_t lead;
      int32_t nrows;
      int32_t group;
    };
    int gi = 0;                         // group of the block last prepared
    auto prep = [&](int k, Next& nx) {
      const int64_t sb = sweep_block(k);
      // the last group whose first sweep block is <= sb: the entries past
      // gi that are <= sb form a prefix (the counts never decrease)
      for (;;) {
        const int e = gi + 1 + lane;
        const bool le = e <= ng && s_start[e <= ng ? e : ng] <= sb;
        const int adv = __popcll(__ballot(le));
        gi += adv;
        if (adv < 64) break;
      }
      const SweepDesc& d = s_desc[gi];
      const uint8_t* x = dev::uniform_ptr(d.x);
      const int64_t ldb = d.ld_bytes;
      nx.group = gi;
      nx.lb = sb - s_start[gi];
      const int64_t s0 = nx.lb * BR * ldb;
      const int64_t mis = (int64_t)(reinterpret_cast<uintptr_t>(x + s0) & 127u);
      const int64_t w0 = s0 >= mis ? s0 - mis : 0;
      const int64_t last = d.total_bytes - (int64_t)FL * 1024;
      const int64_t ws = w0 < last ? w0 : last;
      nx.base = x + ws;
      nx.lead = (uint32_t)(s0 - ws);
      const int64_t left = d.n - nx.lb * BR;
      nx.nrows = left < BR ? (int)left : BR;
      nx.ld = (int32_t)ldb;
      nx.table = d.table;
      nx.labels = d.labels;
      nx.log_post = d.log_post;
      nx.scores = d.scores;
      nx.rb[0] = d.rb[0];
      nx.rb[1] = d.rb[1];
    };
    dev::u32x4 fb[FL];
    // live == false: the same instructions with every offset out of range
    // (no memory access), for the iteration that has no next block
    auto launch = [&](const Next& nx, bool live) {
      const uint32_t span = live ? nx.lead + (uint32_t)((nx.nrows - 1) * nx.ld + F) : 0u;
      // the window lies in bounds (the host stages only buffers holding a window)
      const auto rsrc = dev::make_rsrc(dev::uniform_ptr(nx.base), (int64_t)FL * 1024);
#pragma unroll
      for (int q = 0; q < FL; ++q) {
        const uint32_t off = (uint32_t)(q * kPiece + 16 * lane);
        fb[q] = dev::buffer_load16(rsrc, off < span ? off : dev::kNoAccess);
      }
      __builtin_amdgcn_sched_barrier(0);
    };
    // each lane's 16 weights of each chunk and row, as raw words (FP32: four
    // 16-byte loads; BF16: two)
    dev::u32x4 wt[NCH][NS][TW];
    auto load_table_regs = [&](const void* table) {
      const auto trs = dev::make_rsrc(dev::uniform_ptr(table), NS * Fp * (bf ? 2 : 4));
#pragma unroll
      for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int s2 = 0; s2 < NS; ++s2)
#pragma unroll
          for (int q = 0; q < TW; ++q)
            wt[c][s2][q] = dev::buffer_load16(trs, (uint32_t)(s2 * Fp + c * CW + 16 * j) * (bf ? 2u : 4u) + 16u * q);
    };

    Next cur, nxt;
    prep(0, cur);
    launch(cur, true);
    load_table_regs(cur.table);
    if (nb > 1) prep(1, nxt);
    for (int k = 0; k < nb; ++k) {
      // the launched block lands in LDS; the next one goes out
#pragma unroll
      for (int q = 0; q < FL; ++q) *reinterpret_cast<dev::u32x4*>(mine + q * kPiece + 16 * lane) = fb[q];
      // every iteration issues the window loads (the last one with no
      // memory access), so the compiler's wait counts for the window stay
      // exact; issued only when a next block exists, they made it wait for
      // every outstanding load before writing the window to LDS (measured:
      // 3-4% slower)
      const bool more = k + 1 < nb;
      launch(more ? nxt : cur, more);

#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        float w[NS][16];
#pragma unroll
        for (int s2 = 0; s2 < NS; ++s2)
#pragma unroll
          for (int e = 0; e < 16; ++e) {
            if constexpr (BF) {
              const uint32_t word16 = wt[c][s2][e >> 3][(e >> 1) & 3];
              w[s2][e] = __uint_as_float((e & 1) ? (word16 & 0xFFFF0000u) : (word16 << 16));
            } else {
              w[s2][e] = __uint_as_float(wt[c][s2][(e >> 2) % TW][e & 3]);
            }
          }
        const int fc = c * CW + 16 * j;
        if (XT == NB_X_FP8) fp8_keep_mask(F, fc, keep);
        read_flat_rows<XT, NS, BIN, R>(mine + cur.lead + (uint32_t)fc, (uint32_t)cur.ld, fc < F, w, keep, acc);
      }
      Score2Args a{};
      a.labels = cur.labels;
      a.log_post = cur.log_post;
      a.scores = cur.scores;
      float rb[NS];
      rb[0] = cur.rb[0];
      rb[NS - 1] = cur.rb[NS - 1];
      // a group's last block may be partial: its rows past the end hold
      // stale bytes and are never stored
      if (cur.nrows == BR) finish_block<LPR, NS, true>(a, acc, lane, wave, 0, rb, cur.lb * BR, BR, stage);
      else finish_block<LPR, NS, false>(a, acc, lane, wave, 0, rb, cur.lb * BR, cur.nrows, stage);
#pragma unroll
      for (int i = 0; i < R; ++i)
#pragma unroll
        for (int s2 = 0; s2 < NS; ++s2) acc[i][s2] = 0.0f;
      // the next block's table weights, when its group differs (measured:
      // reloading them for every block, which would keep the wait counts
      // exact, costs 9% with FP32 tables of many groups)
      if (more && nxt.group != cur.group) load_table_regs(nxt.table);
      cur = nxt;
      if (k + 2 < nb) prep(k + 2, nxt);
    }
  }

  // ---- groups smaller than a window: the table in LDS (the staging regions
  // are free once every wave of the workgroup has left the sweep)
  float* tbl = reinterpret_cast<float*>(flat_all);
  for (int t = blockIdx.x; t < g.n_tails; t += (int)gridDim.x) {
    const GroupItem it = dev::load_uniform(g.tails + t);
    const Score2Args a = dev::load_uniform(g.descs + it.group);
    __syncthreads();
    stage_table<NS>(a, tbl);
    __syncthreads();
    score_blocks<XT, LPR, NS, BIN, MULTI>(a, tbl, it.block0 + wave, kWaves, it.block0 + it.nblocks, stage);
  }
}

template <int XT, int LPR, int NS, bool BIN, bool MULTI, int FL = 0>
__global__ __launch_bounds__(kThreads) void score2_groups_static_kernel(GroupsArgs g_in) {
  const GroupsArgs g = resolve_list(g_in);
  extern __shared__ float tbl[];        // [NS][Fp] of the current group, then the flat staging regions
  __shared__ float stage[kWaves][NS][(64 / LPR) * block_steps<XT, false, MULTI, FL>()];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t B = g.total_blocks;
  int64_t b = B * blockIdx.x / gridDim.x;
  const int64_t b1 = B * (blockIdx.x + 1) / gridDim.x;
  if (b >= b1) return;
  uint8_t* flat = FL ? reinterpret_cast<uint8_t*>(tbl) + (size_t)NS * g.Fp * sizeof(float) : nullptr;
  // the group holding block b: the last gi with gstart[gi] <= b
  int lo = 0, hi = g.n_groups - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (dev::load_uniform(g.gstart + mid) <= b) lo = mid;
    else hi = mid - 1;
  }
  for (int gi = lo; b < b1; ++gi) {
    const int64_t gs = dev::load_uniform(g.gstart + gi);
    const int64_t seg_end = min(b1, dev::load_uniform(g.gstart + gi + 1));
    if (seg_end <= b) continue;                 // empty group
    const Score2Args a = dev::load_uniform(g.descs + gi);
    __syncthreads();                            // the previous group's table is no longer read
    stage_table<NS>(a, tbl);
    __syncthreads();
    score_blocks<XT, LPR, NS, BIN, MULTI, false, FL>(a, tbl, (b - gs) + wave, kWaves, seg_end - gs, stage, flat);
    b = seg_end;
  }
}

template <int XT, int LPR, int NS, bool BIN, bool MULTI, int FL = 0>
__global__ __launch_bounds__(kThreads) void score2_groups_kernel(GroupsArgs g_in) {
  const GroupsArgs g = resolve_list(g_in);
  extern __shared__ float tbl[];        // [NS][Fp] of the current item's group, then the flat staging regions
  __shared__ float stage[kWaves][NS][(64 / LPR) * block_steps<XT, false, MULTI, FL>()];
  __shared__ int32_t s_item;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint8_t* flat = FL ? reinterpret_cast<uint8_t*>(tbl) + (size_t)NS * g.Fp * sizeof(float) : nullptr;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(g.counter, 1);
    // the barrier also ends every read of the previous item's table
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    if (it >= g.n_items) break;
    const GroupItem item = dev::load_uniform(g.items + it);
    const Score2Args a = dev::load_uniform(g.descs + item.group);
    stage_table<NS>(a, tbl);
    __syncthreads();
    score_blocks<XT, LPR, NS, BIN, MULTI, false, FL>(a, tbl, item.block0 + wave, kWaves, item.block0 + item.nblocks,
                                                     stage, flat);
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

// The dynamic and static schedules take direct loads only: with flat
// staging's one workgroup per CU, their per-item barriers and table
// stages stall the CU (measured slower than direct loads).
struct Grouped {
  template <int XT, int LPR, int NS, bool BIN, bool MULTI, int FL = 0>
  static const void* fn() {
    if constexpr (FL != 0) return nullptr;
    else return reinterpret_cast<const void*>(score2_groups_kernel<XT, LPR, NS, BIN, MULTI>);
  }
};

struct GroupedStream {
  template <int XT, int LPR, int NS, bool BIN, bool MULTI, int FL = 0>
  static const void* fn() {
    if constexpr (FL != 0) return nullptr;   // the stream schedule stages no rows
    else return reinterpret_cast<const void*>(score2_groups_stream_kernel<XT, LPR, NS, BIN, MULTI>);
  }
};

template <bool BF>
struct GroupedSweep {
  template <int XT, int LPR, int NS, bool BIN, bool MULTI, int FL = 0>
  static const void* fn() {
    if constexpr (FL == 0 || LPR != 64 || XT == NB_X_I32 || !MULTI) return nullptr;
    else return reinterpret_cast<const void*>(score2_groups_sweep_kernel<XT, NS, BIN, MULTI, FL, BF>);
  }
};

struct GroupedStatic {
  template <int XT, int LPR, int NS, bool BIN, bool MULTI, int FL = 0>
  static const void* fn() {
    if constexpr (FL != 0) return nullptr;
    else return reinterpret_cast<const void*>(score2_groups_static_kernel<XT, LPR, NS, BIN, MULTI>);
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
  size_t lds = 0;                  // table bytes in LDS
  int fl = 0;                      // flat staging pieces of the sweep (stream schedule), 0: none
  size_t lds_dyn = 0;              // dynamic LDS of the static and dynamic kernels
  const void* fn = nullptr;        // dynamic-item kernel
  const void* fn_static = nullptr; // static-range kernel
  const void* fn_stream = nullptr; // stream kernel (tables of at most kStreamTable floats)
  int Fp = 0;
  int grid_cap = 1;                // resident workgroups on the device (dynamic kernel)
  int grid_cap_static = 1;
  int grid_cap_stream = 1;
  bool stream_ok = false;
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
  // flat staging when every non-empty group qualifies (the largest window)
  S->fl = -1;
  for (int32_t g = 0; g < n_groups && S->fl != 0; ++g) {
    if (groups[g].n <= 0) continue;
    const int f = flat_pieces(xtype, S->F, groups[g].ld * (int64_t)elem_bytes(xtype), groups[g].x, false);
    S->fl = (f == 0) ? 0 : std::max(S->fl, f);
  }
  if (S->fl < 0) S->fl = 0;
  const int64_t br = (int64_t)(64 / S->lpr) * block_steps_of(xtype, false, (S->F + 16 * S->lpr - 1) / (16 * S->lpr), S->fl);
  for (int32_t g = 0; g < n_groups; ++g) {
    const nb_group& G = groups[g];
    const nb_model* m = &models[groups[route[g]].model];
    if (m->n_classes != 2)
      return fail(NB_EINVAL, "group scoring takes two-class models (benign / malware per size group)");
    if (m->kind == NB_GAUSSIAN)
      return fail(NB_EINVAL, "group scoring takes multinomial and Bernoulli models (Gaussian models: nb_score)");
    if (m->n_features != S->F || (m->kind == NB_BERNOULLI) != S->bin)
      return fail(NB_EINVAL, "all group models must share the kind and the feature count");
    if (G.n < 0) return fail(NB_EINVAL, "group " + std::to_string(g) + ": n must be >= 0");
    Score2Args a{};
    if (G.n > 0) {
      nb_layout L;
      int rc = check_score_args(m, &L, G.x, xtype, G.n, G.ld, wtype, G.labels, G.log_post, G.scores);
      if (rc) return fail(rc, "group " + std::to_string(g) + ": " + nb_last_error());
      rc = make_score2_args(m, L, G.x, xtype, G.n, G.ld, wtype, G.labels, G.log_post, G.scores, S->ns, &a, false,
                            S->fl);
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
  S->lds_dyn = S->lds;
  if (S->lds_dyn > 64 * 1024) {
    NB_HIP_CHECK(hipFuncSetAttribute(S->fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)S->lds_dyn));
    NB_HIP_CHECK(hipFuncSetAttribute(S->fn_static, hipFuncAttributeMaxDynamicSharedMemorySize, (int)S->lds_dyn));
  }
  S->Fp = L.padded_features;
  S->stream_ok = (size_t)S->ns * L.padded_features <= (size_t)kStreamTable;
  // with flat staging the stream schedule is a sweep: its tables ride in
  // registers (tails stage one group's rows in LDS), any NS
  if (S->fl > 0 && n_groups > kSweepMaxGroups) S->fl = 0;   // the sweep keeps every group's descriptor in LDS
  if (S->fl > 0) {
    S->stream_ok = true;
    S->fn_stream = wtype == NB_W_BF16 ? pick_score2<GroupedSweep<true>>(xtype, S->lpr, S->nch > 1, S->ns, S->bin, S->fl)
                                      : pick_score2<GroupedSweep<false>>(xtype, S->lpr, S->nch > 1, S->ns, S->bin, S->fl);
    S->grid_cap_stream = resident_per_cu(S->fn_stream, kThreads, 0) * device_cu_count();
  } else if (S->stream_ok) {
    S->fn_stream = pick_score2<GroupedStream>(xtype, S->lpr, S->nch > 1, S->ns, S->bin);
    S->grid_cap_stream = resident_per_cu(S->fn_stream, kThreads, 0) * device_cu_count();
  }
  S->grid_cap = resident_per_cu(S->fn, kThreads, S->lds_dyn) * device_cu_count();
  S->grid_cap_static = resident_per_cu(S->fn_static, kThreads, S->lds_dyn) * device_cu_count();
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
  const int br = (64 / S.lpr) * block_steps_of(S.xtype, false, S.nch, S.fl);
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

// A schedule code: 0 = static ranges, T > 0 = dynamic items of at most T
// blocks, -T < 0 = stream items of T blocks.  Its device image (the work
// list):
//   [256-byte header: two zeroed int32 counters]
//   [descriptors, one per group]
//   [payload: static: the first block of each group plus the total
//    (n_groups + 1 int64); dynamic: items; stream: items, then tails]
struct WorkList {
  int code = 0;
  bool sweep = false;              // stream code with flat staging: sstart + tails
  std::vector<GroupItem> items;
  std::vector<GroupItem> tails;
  std::vector<int64_t> gstart;
  std::vector<int64_t> sstart;     // sweep: first sweep block of each group, then the total
  bool is_static() const { return code == 0; }
  bool is_stream() const { return code < 0; }
  int32_t n_items() const { return (int32_t)items.size(); }
  int32_t n_tails() const { return (int32_t)tails.size(); }
};

// Stream items: each group's fast blocks cut into items of T blocks in
// memory order (a remainder below four blocks joins the item before it);
// groups with fewer than four fast blocks, and every group's blocks past
// its fast ones, become tails.
void make_stream_items(const GroupSetup& S, int T, WorkList* w) {
  for (size_t g = 0; g < S.blocks.size(); ++g) {
    const int64_t nb = S.blocks[g];
    if (nb == 0) continue;
    const int64_t nf = std::min<int64_t>(nb, S.descs[g].nfast);
    int64_t b0 = 0;
    if (nf >= kWaves) {
      while (b0 < nf) {
        int64_t len = std::min<int64_t>(T, nf - b0);
        if (nf - (b0 + len) < kWaves) len = nf - b0;       // fold a short remainder in
        w->items.push_back(GroupItem{b0, (int32_t)g, (int32_t)len});
        b0 += len;
      }
    }
    if (b0 < nb) w->tails.push_back(GroupItem{b0, (int32_t)g, (int32_t)(nb - b0)});
  }
}

// Sweep: each group's staged blocks (below its nflat) in memory order, as
// prefix counts over the groups; the blocks past them are tails.
void make_sweep_list(const GroupSetup& S, WorkList* w) {
  w->sweep = true;
  w->sstart.resize(S.blocks.size() + 1);
  int64_t acc = 0;
  for (size_t g = 0; g < S.blocks.size(); ++g) {
    w->sstart[g] = acc;
    const int64_t nb = S.blocks[g];
    const int64_t ns = std::min<int64_t>(nb, S.descs[g].nflat);
    acc += ns;
    if (ns < nb) w->tails.push_back(GroupItem{ns, (int32_t)g, (int32_t)(nb - ns)});
  }
  w->sstart[S.blocks.size()] = acc;
}

WorkList make_work_list(const GroupSetup& S, int code) {
  WorkList w;
  w.code = code;
  if (code < 0 && S.fl > 0) {
    make_sweep_list(S, &w);
  } else if (code == 0) {
    w.gstart.resize(S.blocks.size() + 1);
    int64_t acc = 0;
    for (size_t g = 0; g < S.blocks.size(); ++g) {
      w.gstart[g] = acc;
      acc += S.blocks[g];
    }
    w.gstart[S.blocks.size()] = acc;
  } else if (code > 0) {
    w.items = make_items(S, code);
  } else {
    make_stream_items(S, -code, &w);
  }
  return w;
}

size_t payload_bytes(const WorkList& w) {
  if (w.is_static()) return w.gstart.size() * sizeof(int64_t);
  if (w.sweep) return align_up(w.sstart.size() * sizeof(int64_t), 16) + w.tails.size() * sizeof(GroupItem);
  return (w.items.size() + w.tails.size()) * sizeof(GroupItem);
}

// A work list's device image:
//   [header, kCounterBytes: two int32 counters (zero), then ListCounts]
//   [descriptors: room for cap_groups, 256-byte aligned]
//   [payload]
// cap_groups is the call's group count, or a plan's capacity.
size_t work_list_bytes(size_t cap_groups, size_t payload) {
  return kCounterBytes + align_up(cap_groups * sizeof(Score2Args), kAlign) + align_up(payload, kAlign);
}

struct DevLists {
  int32_t* counter;
  const ListCounts* counts;
  Score2Args* descs;
  void* payload;
};

DevLists carve(void* ws, size_t cap_groups) {
  uint8_t* p = static_cast<uint8_t*>(ws);
  DevLists d;
  d.counter = reinterpret_cast<int32_t*>(p);
  d.counts = reinterpret_cast<const ListCounts*>(p + 2 * sizeof(int32_t));
  d.descs = reinterpret_cast<Score2Args*>(p + kCounterBytes);
  d.payload = p + kCounterBytes + align_up(cap_groups * sizeof(Score2Args), kAlign);
  return d;
}

int list_kind(const WorkList& w) { return w.is_static() ? 0 : (w.code > 0 ? 1 : (w.sweep ? 3 : 2)); }

// The device image of a work list (counters zeroed).
void serialise(const GroupSetup& S, const WorkList& w, std::vector<uint8_t>* blob, size_t cap_groups = 0) {
  const size_t ng = S.descs.size();
  if (cap_groups < ng) cap_groups = ng;
  blob->assign(work_list_bytes(cap_groups, payload_bytes(w)), 0);
  ListCounts c{};
  c.n_items = w.n_items();
  c.n_tails = w.n_tails();
  c.n_groups = (int32_t)ng;
  c.kind = list_kind(w);
  c.total_blocks = w.sweep ? w.sstart.back() : S.total_blocks;
  std::memcpy(blob->data() + 2 * sizeof(int32_t), &c, sizeof c);
  std::memcpy(blob->data() + kCounterBytes, S.descs.data(), ng * sizeof(Score2Args));
  uint8_t* pay = blob->data() + kCounterBytes + align_up(cap_groups * sizeof(Score2Args), kAlign);
  if (w.is_static()) {
    std::memcpy(pay, w.gstart.data(), w.gstart.size() * sizeof(int64_t));
  } else if (w.sweep) {
    std::memcpy(pay, w.sstart.data(), w.sstart.size() * sizeof(int64_t));
    std::memcpy(pay + align_up(w.sstart.size() * sizeof(int64_t), 16), w.tails.data(),
                w.tails.size() * sizeof(GroupItem));
  } else {
    std::memcpy(pay, w.items.data(), w.items.size() * sizeof(GroupItem));
    std::memcpy(pay + w.items.size() * sizeof(GroupItem), w.tails.data(), w.tails.size() * sizeof(GroupItem));
  }
}

// Launch of one work list: kernel, grid and the arguments it needs (the
// counts travel in the list's header).
struct LaunchDesc {
  const void* fn = nullptr;
  size_t lds = 0;
  int grid = 0;
  int kind = 0;                // 0 static, 1 dynamic, 2 stream, 3 sweep
  int32_t n_items = 0, n_tails = 0, n_groups = 0, Fp = 0, nch = 0, F = 0, wt = 0;
  int64_t total_blocks = 0;
  int64_t sweep_blocks = 0;
};

// fixed_grid: the resident grid of the schedule's kernel whatever the list
// (a plan's captured launch serves every work list written into it)
LaunchDesc describe(const GroupSetup& S, const WorkList& w, bool fixed_grid = false) {
  LaunchDesc L;
  L.n_items = w.n_items();
  L.n_tails = w.n_tails();
  L.n_groups = (int32_t)S.descs.size();
  L.Fp = S.Fp;
  L.nch = S.nch;
  L.F = S.F;
  L.wt = S.wtype;
  L.total_blocks = S.total_blocks;
  L.kind = list_kind(w);
  if (L.kind == 0) {
    L.fn = S.fn_static;
    L.lds = S.lds_dyn;
    // every workgroup gets at least a few blocks per wave
    const int64_t most = std::max<int64_t>(1, S.total_blocks / (2 * kWaves));
    L.grid = fixed_grid ? S.grid_cap_static : (int)std::max<int64_t>(1, std::min<int64_t>(S.grid_cap_static, most));
  } else if (L.kind == 1) {
    L.fn = S.fn;
    L.lds = S.lds_dyn;
    L.grid = fixed_grid ? S.grid_cap : std::max(1, std::min(S.grid_cap, L.n_items));
  } else if (L.kind == 3) {
    L.fn = S.fn_stream;
    L.lds = 0;
    L.sweep_blocks = w.sstart.back();
    const int64_t most = std::max<int64_t>({1, (L.sweep_blocks + kWaves - 1) / kWaves, (int64_t)L.n_tails});
    L.grid = fixed_grid ? S.grid_cap_stream : (int)std::min<int64_t>(S.grid_cap_stream, most);
  } else {
    L.fn = S.fn_stream;
    L.lds = 0;
    L.grid = fixed_grid ? S.grid_cap_stream : std::max(1, std::min(S.grid_cap_stream, std::max(L.n_items, L.n_tails)));
  }
  return L;
}

int launch_grouped(const LaunchDesc& L, const DevLists& d, hipStream_t s) {
  GroupsArgs g{};
  g.descs = d.descs;
  g.payload = d.payload;
  g.counts = d.counts;
  g.counter = d.counter;
  g.Fp = L.Fp;
  g.nch = L.nch;
  g.F = L.F;
  g.wt = L.wt;
  void* args[] = {&g};
  NB_HIP_CHECK(hipLaunchKernel(L.fn, dim3(L.grid), dim3(kThreads), args, L.lds, s));
  NB_HIP_CHECK(hipGetLastError());
  return NB_OK;
}

int launch_grouped(const GroupSetup& S, const WorkList& w, const DevLists& d, hipStream_t s) {
  if (S.total_blocks == 0) return NB_OK;
  return launch_grouped(describe(S, w), d, s);
}

// ---- pinned staging of work lists (nb_score_groups and plan updates
// return before the device has read the list): coherent host-pinned
// buffers, mapped into the device's address space, read by a small copy
// kernel on the caller's stream (a copy-engine transfer between two kernels
// of one stream costs tens of microseconds of queue hand-over, measured;
// a kernel costs none), each buffer reused once the copy that last read it
// has run (an event per buffer).
__global__ __launch_bounds__(256) void copy_list_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                       int n16) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n16; i += gridDim.x * 256) dst[i] = src[i];
}

int host_buffer(size_t bytes, void** host, void** dev_view) {
  NB_HIP_CHECK(hipHostMalloc(host, bytes, hipHostMallocCoherent | hipHostMallocMapped));
  NB_HIP_CHECK(hipHostGetDevicePointer(dev_view, *host, 0));
  return NB_OK;
}

// Enqueue the copy of `bytes` (a multiple of 16) from a mapped pinned
// buffer to device memory.
int enqueue_list_copy(const void* src_view, void* dst, size_t bytes, hipStream_t s) {
  const int n16 = (int)(bytes / 16);
  const int grid = std::max(1, std::min(64, (n16 + 255) / 256));
  hipLaunchKernelGGL(copy_list_kernel, dim3(grid), dim3(256), 0, s, static_cast<const uint4*>(src_view),
                     static_cast<uint4*>(dst), n16);
  NB_HIP_CHECK(hipGetLastError());
  return NB_OK;
}

struct PinnedSlot {
  void* host = nullptr;
  void* view = nullptr;            // the device's address of host
  size_t bytes = 0;
  hipEvent_t done = nullptr;
  int device = -1;
};
constexpr int kMaxPinnedSlots = 16;
std::mutex g_pin_mu;
std::vector<std::unique_ptr<PinnedSlot>> g_pin;

// Copy `blob` to device memory `dst` on stream s through a pinned buffer.
int stage_to_device(const std::vector<uint8_t>& blob, void* dst, hipStream_t s) {
  int dev = -1;
  NB_HIP_CHECK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_pin_mu);
  PinnedSlot* use = nullptr;
  for (auto& sl : g_pin)
    if (sl->device == dev && sl->bytes >= blob.size() && hipEventQuery(sl->done) == hipSuccess) {
      use = sl.get();
      break;
    }
  if (!use) {
    int mine = 0;
    for (auto& sl : g_pin) mine += sl->device == dev;
    if (mine < kMaxPinnedSlots) {
      auto sl = std::make_unique<PinnedSlot>();
      sl->device = dev;
      sl->bytes = std::max<size_t>(blob.size(), (size_t)1 << 20);
      if (int rc = host_buffer(sl->bytes, &sl->host, &sl->view)) return rc;
      NB_HIP_CHECK(hipEventCreateWithFlags(&sl->done, hipEventDisableTiming));
      use = sl.get();
      g_pin.push_back(std::move(sl));
    } else {
      // every buffer of this device is still being read: wait for the first
      // one and grow it if needed
      for (auto& sl : g_pin)
        if (sl->device == dev) {
          use = sl.get();
          break;
        }
      NB_HIP_CHECK(hipEventSynchronize(use->done));
      if (use->bytes < blob.size()) {
        NB_HIP_CHECK(hipHostFree(use->host));
        use->host = nullptr;
        use->bytes = blob.size();
        if (int rc = host_buffer(use->bytes, &use->host, &use->view)) return rc;
      }
    }
  }
  std::memcpy(use->host, blob.data(), blob.size());
  if (int rc = enqueue_list_copy(use->view, dst, blob.size(), s)) return rc;
  NB_HIP_CHECK(hipEventRecord(use->done, s));
  return NB_OK;
}

// Default schedule: the stream when the table fits, else static ranges.
int default_code(const GroupSetup& S) { return S.stream_ok ? -16 : 0; }

// ------------------------------------------------------------ tile cache
// Tuned schedules persist in a flat JSON object {"key": code, ...} (the
// schedule code above) at the path named by NB_TUNE_CACHE (when set);
// always kept in memory.
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
    g_tune[key] = std::atoi(t.c_str() + k + 1);
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

// schedule code recorded for the shape, if any
bool tune_lookup(const std::string& key, int* code) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  auto it = g_tune.find(key);
  if (it == g_tune.end()) return false;
  *code = it->second;
  return true;
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
  const WorkList w = make_work_list(S, tile_rows > 0 ? tile_blocks_from_rows(S, tile_rows) : default_code(S));
  serialise(S, w, blob);
  const LaunchDesc L = describe(S, w);
  out->fn = L.fn;
  out->lds = L.lds;
  out->grid = L.grid;
  out->kind = L.kind;
  out->n_items = L.n_items;
  out->n_tails = L.n_tails;
  out->n_groups = L.n_groups;
  out->Fp = L.Fp;
  out->nch = L.nch;
  out->F = L.F;
  out->wt = L.wt;
  out->total_blocks = L.total_blocks;
  out->sweep_blocks = L.sweep_blocks;
  out->blob_bytes = blob->size();
  return NB_OK;
}

int enqueue_group_launch(const GroupLaunch& G, void* dev_blob, hipStream_t s) {
  if (G.total_blocks == 0) return NB_OK;
  LaunchDesc L;
  L.fn = G.fn;
  L.lds = G.lds;
  L.grid = G.grid;
  L.kind = G.kind;
  L.n_items = G.n_items;
  L.n_tails = G.n_tails;
  L.n_groups = G.n_groups;
  L.Fp = G.Fp;
  L.nch = G.nch;
  L.F = G.F;
  L.wt = G.wt;
  L.total_blocks = G.total_blocks;
  L.sweep_blocks = G.sweep_blocks;
  return launch_grouped(L, carve(dev_blob, G.n_groups), s);
}

}  // namespace nb

using namespace nb;

// ------------------------------------------------------------------ plan
struct nb_group_plan {
  GroupSetup S;
  void* dev = nullptr;            // work list: header, descriptors, payload
  size_t dev_bytes = 0;
  int32_t n_groups = 0;           // groups of the current work list
  int32_t cap_groups = 0;         // room for descriptors (the creation call's count)
  WorkList w;
  int tuned = 0;
  LaunchDesc launch;              // the captured launch (kernel, fixed grid)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* pinned[2] = {nullptr, nullptr};     // staging of updated work lists
  void* pinned_view[2] = {nullptr, nullptr};
  hipEvent_t staged[2] = {nullptr, nullptr};
  int slot = 0;
};

namespace {

int upload(nb_group_plan* p, const WorkList& w) {
  std::vector<uint8_t> blob;
  serialise(p->S, w, &blob, (size_t)p->cap_groups);
  if (blob.size() > p->dev_bytes) return fail(NB_EHIP, "internal: work list larger than its buffer");
  NB_HIP_CHECK(hipMemcpy(p->dev, blob.data(), blob.size(), hipMemcpyHostToDevice));
  p->w = w;
  return NB_OK;
}

// Time the stream schedule at a few item sizes, static ranges and a few
// dynamic tiles on the caller's data; keep the fastest.
int autotune(nb_group_plan* p, hipStream_t s) {
  std::vector<int> cand;
  if (p->S.stream_ok)
    for (int t : {8, 16, 32, 64}) cand.push_back(-t);
  cand.push_back(0);
  const int def = default_tile_blocks(p->S);
  for (int t : {16, 32, 64, 128}) cand.push_back(t);
  if (std::find(cand.begin(), cand.end(), def) == cand.end()) cand.push_back(def);
  hipEvent_t e0, e1;
  NB_HIP_CHECK(hipEventCreate(&e0));
  NB_HIP_CHECK(hipEventCreate(&e1));
  float best = 1e30f;
  int best_t = default_code(p->S);
  int rc = NB_OK;
  const DevLists d = carve(p->dev, (size_t)p->cap_groups);
  for (int t : cand) {
    const WorkList w = make_work_list(p->S, t);
    if ((rc = upload(p, w))) break;
    const LaunchDesc L = describe(p->S, w, true);
    if ((rc = launch_grouped(L, d, s))) break;   // warm
    // the median of a few single launches: robust to an occasional slow one
    constexpr int kReps = 7;
    float ms_r[kReps];
    for (int r = 0; r < kReps && rc == NB_OK; ++r) {
      if (hipEventRecord(e0, s) != hipSuccess) rc = fail(NB_EHIP, "hipEventRecord");
      if (!rc) rc = launch_grouped(L, d, s);
      if (!rc && hipEventRecord(e1, s) != hipSuccess) rc = fail(NB_EHIP, "hipEventRecord");
      if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = fail(NB_EHIP, "hipEventSynchronize");
      ms_r[r] = 0.0f;
      if (!rc && hipEventElapsedTime(&ms_r[r], e0, e1) != hipSuccess) rc = fail(NB_EHIP, "hipEventElapsedTime");
    }
    if (rc) break;
    std::sort(ms_r, ms_r + kReps);
    const float tot = ms_r[kReps / 2];
    if (tot < best) {
      best = tot;
      best_t = t;
    }
  }
  // releases on a path that reports its own status
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  p->w.code = best_t;
  p->tuned = 1;
  return NB_OK;
}

void plan_free(nb_group_plan* p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->dev) (void)hipFree(p->dev);
  for (int i = 0; i < 2; ++i) {
    if (p->staged[i]) (void)hipEventDestroy(p->staged[i]);
    if (p->pinned[i]) (void)hipHostFree(p->pinned[i]);
  }
  delete p;
}

// Room of a plan's work-list buffer: updated work lists may carry up to this
// many times the payload of the largest list the creation call could make,
// and at least kPlanMinPayload bytes (65,536 items), for up to the creation
// call's number of groups.
constexpr size_t kPlanHeadroom = 4;
constexpr size_t kPlanMinPayload = (size_t)1 << 20;

int plan_build(nb_group_plan* p, const nb_model* models, int32_t n_models, const nb_group* groups, int32_t n_groups,
               int32_t xtype, int32_t wtype, int32_t tile_rows, int32_t flags, hipStream_t s) {
  int rc = setup_groups(models, n_models, groups, n_groups, xtype, wtype, &p->S);
  if (rc) return rc;
  p->n_groups = n_groups;
  p->cap_groups = n_groups;
  // room for the largest work list any schedule makes (the smallest tiles),
  // times the headroom for later steps
  const size_t pay = std::max({payload_bytes(make_work_list(p->S, kWaves)),
                               payload_bytes(make_work_list(p->S, -kWaves)),
                               ((size_t)n_groups + 1) * sizeof(int64_t) + 16});
  p->dev_bytes = work_list_bytes((size_t)n_groups, std::max(kPlanHeadroom * pay, kPlanMinPayload));
  NB_HIP_CHECK(hipStreamSynchronize(s));
  NB_HIP_CHECK(hipMalloc(&p->dev, p->dev_bytes));
  for (int i = 0; i < 2; ++i) {
    if ((rc = host_buffer(p->dev_bytes, &p->pinned[i], &p->pinned_view[i]))) return rc;
    NB_HIP_CHECK(hipEventCreateWithFlags(&p->staged[i], hipEventDisableTiming));
  }
  const std::string key = tune_key(p->S, n_groups);
  int tile = 0;
  int cached = 0;
  if (flags & NB_PLAN_STATIC) {
    tile = 0;
  } else if (flags & NB_PLAN_STREAM) {
    if (!p->S.stream_ok) return fail(NB_EINVAL, "stream schedule: the scoring rows exceed 2048 floats");
    tile = tile_rows > 0 ? -tile_blocks_from_rows(p->S, tile_rows) : default_code(p->S);
  } else if (tile_rows > 0) {
    tile = tile_blocks_from_rows(p->S, tile_rows);
  } else if (tune_lookup(key, &cached)) {
    tile = cached;
    p->tuned = 2;
  } else if (flags & NB_PLAN_TUNE) {
    if ((rc = autotune(p, s))) return rc;
    tile = p->w.code;
    tune_record(key, tile);
  } else {
    tile = default_code(p->S);
  }
  if ((rc = upload(p, make_work_list(p->S, tile)))) return rc;
  p->launch = describe(p->S, p->w, true);
  // capture the launch into a graph on a private stream
  hipStream_t cs;
  NB_HIP_CHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return fail(NB_EHIP, "hipStreamBeginCapture failed");
  }
  rc = launch_grouped(p->launch, carve(p->dev, (size_t)p->cap_groups), cs);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(cs, &graph);
  (void)hipStreamDestroy(cs);
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (ec != hipSuccess) return hip_fail(ec, "hipStreamEndCapture");
  p->graph = graph;
  NB_HIP_CHECK(hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0));
  return NB_OK;
}

// A new step's groups for an existing plan: same kernel, new work list.
int plan_update(nb_group_plan* p, const nb_model* models, int32_t n_models, const nb_group* groups, int32_t n_groups,
                hipStream_t s) {
  if (n_groups > p->cap_groups)
    return fail(NB_EINVAL, "more groups (" + std::to_string(n_groups) + ") than the plan was created with (" +
                               std::to_string(p->cap_groups) + ")");
  GroupSetup S;
  int rc = setup_groups(models, n_models, groups, n_groups, p->S.xtype, p->S.wtype, &S);
  if (rc) return rc;
  const WorkList w = make_work_list(S, p->w.code);
  const LaunchDesc L = describe(S, w, true);
  // the captured kernel, its launch shape and its fixed arguments must serve
  if (L.fn != p->launch.fn || L.lds != p->launch.lds || L.grid != p->launch.grid || S.F != p->S.F ||
      S.Fp != p->S.Fp || S.nch != p->S.nch)
    return fail(NB_EINVAL, "the new groups need another kernel than the plan's (models must share the plan's "
                           "feature count and kind, the same outputs must be requested, and rows must stay "
                           "eligible for the plan's row staging)");
  std::vector<uint8_t> blob;
  serialise(S, w, &blob, (size_t)p->cap_groups);
  if (blob.size() > p->dev_bytes)
    return fail(NB_ENOMEM, "the new work list (" + std::to_string(blob.size()) + " bytes) exceeds the plan's room (" +
                               std::to_string(p->dev_bytes) + " bytes): create a plan for the larger step");
  // the pinned buffer is free once the copy that last read it has run
  const int k = p->slot;
  NB_HIP_CHECK(hipEventSynchronize(p->staged[k]));
  std::memcpy(p->pinned[k], blob.data(), blob.size());
  if ((rc = enqueue_list_copy(p->pinned_view[k], p->dev, blob.size(), s))) return rc;
  NB_HIP_CHECK(hipEventRecord(p->staged[k], s));
  p->slot ^= 1;
  p->S = std::move(S);
  p->w = w;
  p->n_groups = n_groups;
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
  // the work list goes through pinned host memory: the call returns once
  // the copy and the launch are enqueued
  if ((rc = stage_to_device(blob, workspace, s))) return rc;
  return enqueue_group_launch(L, workspace, s);
}

int nb_group_plan_create(const nb_model* models, int32_t n_models, const nb_group* groups, int32_t n_groups,
                         int32_t xtype, int32_t wtype, int32_t tile_rows, int32_t flags, void* stream,
                         nb_group_plan** out) {
  if (!out) return fail(NB_EINVAL, "out is NULL");
  *out = nullptr;
  if (tile_rows < 0) return fail(NB_EINVAL, "tile_rows must be >= 0");
  if (flags & ~(NB_PLAN_TUNE | NB_PLAN_STATIC | NB_PLAN_STREAM)) return fail(NB_EINVAL, "unknown plan flags");
  if ((flags & NB_PLAN_STATIC) && (flags & NB_PLAN_STREAM)) return fail(NB_EINVAL, "pick one schedule");
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

int nb_group_plan_update(nb_group_plan* plan, const nb_model* models, int32_t n_models, const nb_group* groups,
                         int32_t n_groups, void* stream) {
  if (!plan) return fail(NB_EINVAL, "plan is NULL");
  return plan_update(plan, models, n_models, groups, n_groups, reinterpret_cast<hipStream_t>(stream));
}

int nb_group_plan_launch(nb_group_plan* plan, void* stream) {
  if (!plan) return fail(NB_EINVAL, "plan is NULL");
  if (plan->S.total_blocks == 0) return NB_OK;
  NB_HIP_CHECK(hipGraphLaunch(plan->exec, reinterpret_cast<hipStream_t>(stream)));
  return NB_OK;
}

int nb_group_plan_query(const nb_group_plan* plan, nb_group_plan_info* out) {
  if (!plan || !out) return fail(NB_EINVAL, "NULL argument");
  const int br = (64 / plan->S.lpr) * block_steps_of(plan->S.xtype, false, plan->S.nch, plan->S.fl);
  const LaunchDesc L = describe(plan->S, plan->w, true);
  const int code = plan->w.code;
  out->schedule = code == 0 ? NB_SCHEDULE_STATIC : (code > 0 ? NB_SCHEDULE_DYNAMIC : NB_SCHEDULE_STREAM);
  out->tile_rows = code == 0 ? (int32_t)std::min<int64_t>(INT32_MAX, (plan->S.total_blocks + L.grid - 1) / L.grid * br)
                             : (plan->w.sweep ? br : std::abs(code) * br);
  out->n_items = code == 0 ? L.grid
                           : (int32_t)std::min<int64_t>(INT32_MAX, (plan->w.sweep ? L.sweep_blocks : L.n_items) + L.n_tails);
  out->grid = L.grid;
  out->tuned = plan->tuned;
  out->n_files = plan->S.n_files;
  out->rows_per_block = br;
  out->lds_bytes = (int32_t)plan->S.lds;
  out->staged = plan->w.sweep ? 1 : 0;
  return NB_OK;
}

int nb_group_plan_destroy(nb_group_plan* plan) {
  if (!plan) return NB_OK;
  NB_HIP_CHECK(hipDeviceSynchronize());
  plan_free(plan);
  return NB_OK;
}

}  // extern "C"
