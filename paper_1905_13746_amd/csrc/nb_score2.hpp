// Two-class scoring building blocks shared by the single-model kernel
// (nb_score.hip) and the grouped persistent kernel (nb_groups.hip).
//
// A row (file) is split across LPR lanes of a wave (LPR = the smallest power
// of two >= F/16, at most 64), each lane owning 16 consecutive features per
// chunk of 16*LPR features.  A wave processes blocks of R row-steps of
// 64/LPR rows; the table rows sit in LDS as FP32.  See nb_score.hip for the
// full description of the mapping and of the summation order.
#pragma once

#include <algorithm>
#include <cstdlib>

#include "nb_device.hpp"
#include "nb_internal.hpp"

namespace nb {
namespace {


constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
// Row-steps per block (a block is R row-steps of 64/LPR rows): 16 for the
// linear kernels on byte features (multinomial, Bernoulli; uint8 or FP8), 8
// for int32 features (four 16-byte vectors per lane and row: 16 row-steps,
// double-buffered, would not fit the register file) and for the Gaussian
// kernel (four table rows and a longer chain per feature); measured on
// gfx950 at every lanes-per-file width.  And whether a wave double-buffers
// its loads (the next unit's loads in flight while the current one is
// accumulated).
#ifndef NB_ROW_STEPS
#define NB_ROW_STEPS 16
#endif
#ifndef NB_ROW_STEPS_HEAVY
#define NB_ROW_STEPS_HEAVY 8
#endif
#ifndef NB_PIPELINE
#define NB_PIPELINE 1
#endif
template <int XT, bool QUAD>
constexpr int row_steps() { return (QUAD || XT == NB_X_I32) ? NB_ROW_STEPS_HEAVY : NB_ROW_STEPS; }
inline int row_steps_of(int xtype, bool quad) {
  return (quad || xtype == NB_X_I32) ? NB_ROW_STEPS_HEAVY : NB_ROW_STEPS;
}
// Row-steps per block of a two-class kernel (one name for the block size of
// every variant, direct loads or flat staging).
template <int XT, bool QUAD, bool MULTI, int FL>
constexpr int block_steps() { return row_steps<XT, QUAD>(); }
inline int block_steps_of(int xtype, bool quad, int nch, int fl) { return row_steps_of(xtype, quad); }
// the transposed butterfly of finish_block halves R x NS values per step
static_assert((NB_ROW_STEPS & (NB_ROW_STEPS - 1)) == 0 && (NB_ROW_STEPS_HEAVY & (NB_ROW_STEPS_HEAVY - 1)) == 0,
              "row steps per block must be powers of two");
constexpr bool kPipeline = NB_PIPELINE != 0;

struct Score2Args {
  const uint8_t* x;
  int64_t ld_bytes;
  int64_t n;
  int64_t total_bytes;
  const float* rows32;      // [2][Fp] log-odds row, aux row
  const uint16_t* rows16;   // same rows in BF16
  const float* rows32_q;    // Gaussian: [2][Fp] rows of the x^2 weights
  const uint16_t* rows16_q; //   (log-odds, aux), FP32 / BF16
  const float* row_bias;    // [2]
  int32_t* labels;
  float* log_post;
  float* scores;
  int64_t nfast;            // leading blocks with every row present and in bounds
  int64_t nflat;            // leading blocks scored through flat staging (all or none)
  int32_t F, Fp, nch, wt;
};

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Convert the 16 features of one lane's segment and accumulate them into
// acc[s] against the 16 table values w[s][*].
template <int XT, int NS, bool BIN>
__device__ __forceinline__ void accumulate_seg(const dev::u32x4 (&v)[(XT == NB_X_I32) ? 4 : 1],
                                               const float (&w)[NS][16], float (&acc)[NS]) {
  float xf[16];
  if (XT == NB_X_I32) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int d = 0; d < 4; ++d) xf[4 * q + d] = (float)(int32_t)v[q][d];
  } else if (XT == NB_X_U8) {
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const uint32_t u = v[0][d];
      xf[4 * d + 0] = (float)(u & 0xFFu);
      xf[4 * d + 1] = (float)((u >> 8) & 0xFFu);
      xf[4 * d + 2] = (float)((u >> 16) & 0xFFu);
      xf[4 * d + 3] = (float)(u >> 24);
    }
  } else {  // FP8 e4m3
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const uint32_t u = v[0][d];
      const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8(u, false);
      const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8(u, true);
      xf[4 * d + 0] = lo[0];
      xf[4 * d + 1] = lo[1];
      xf[4 * d + 2] = hi[0];
      xf[4 * d + 3] = hi[1];
    }
  }
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    // presence: for integer counts, clamping to [0, 1] is 1[x > 0], and the
    // clamp folds into the conversion's output modifier (no extra
    // instruction); FP8 values may be fractional, so compare
    const float g = !BIN ? xf[e]
                         : (XT == NB_X_FP8 ? (xf[e] > 0.0f ? 1.0f : 0.0f) : __builtin_amdgcn_fmed3f(xf[e], 0.0f, 1.0f));
#pragma unroll
    for (int s = 0; s < NS; ++s) acc[s] = fmaf(g, w[s][e], acc[s]);
  }
}

// Output stores through global-address-space pointers.  Outputs always live
// in device memory; a pointer whose origin the compiler cannot see (read
// from LDS, as the grouped sweep's descriptors are) would otherwise become a
// flat store, which the hardware counts on both the vector-memory and the
// LDS counters, and the compiler then waits for every outstanding load
// before the loop's next LDS access.
template <class T>
__device__ __forceinline__ void store_out(T* p, const T& v) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "4- or 8-byte outputs");
  if constexpr (sizeof(T) == 4) {
    uint32_t u;
    __builtin_memcpy(&u, &v, 4);
    *(__attribute__((address_space(1))) uint32_t*)p = u;
  } else {
    uint64_t u;
    __builtin_memcpy(&u, &v, 8);
    *(__attribute__((address_space(1))) uint64_t*)p = u;
  }
}

// Destination of outputs the caller did not request: the fast path stores
// every output unconditionally so the number of memory operations in flight
// is known at compile time (loads of the next unit stay in flight).
__device__ int32_t g_sink_label[64];
__device__ float2 g_sink_pair[64];

// Reduce acc[R][NS] across the LPR lanes of each row group (transposed
// butterfly), stage the per-row totals in LDS and run the fused epilogue for
// the block's rows [row0, row0 + nrows).  FAST: nrows == BR and no branches
// around the stores (lanes beyond BR repeat a row: same value, same address).
template <int LPR, int NS, bool FAST, int R>
__device__ __forceinline__ void finish_block(const Score2Args& a, float (&acc)[R][NS], int lane, int wave,
                                             int sub, const float (&rb)[NS], int64_t row0, int nrows,
                                             float (*stage)[NS][(64 / LPR) * R]) {
  constexpr int G = 64 / LPR;
  constexpr int BR = G * R;
  constexpr int V = R * NS;
  float val[V];
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int s = 0; s < NS; ++s) val[i * NS + s] = acc[i][s];
  int offset = 0;
  bool owner = true;
  int cnt = V;
#pragma unroll
  for (int m = LPR / 2; m >= 1; m >>= 1) {
    const bool up = (lane & m) != 0;
    if (cnt > 1) {
      const int h = cnt / 2;
#pragma unroll
      for (int k = 0; k < h; ++k) {
        // both values loaded first: a conditional over the array elements
        // themselves selects an address, i.e. a runtime index into val,
        // which the compiler expands into a compare/select chain over all V
        const float lo = val[k], hi = val[k + h];
        const float send = up ? lo : hi;
        const float keep = up ? hi : lo;
        val[k] = keep + __shfl_xor(send, m);
      }
      if (up) offset += h;
      cnt = h;
    } else {
      val[0] += __shfl_xor(val[0], m);
      if (up) owner = false;
    }
  }
  // cnt values remain per lane, value indices offset .. offset + cnt - 1
  if (owner) {
#pragma unroll
    for (int k = 0; k < cnt; ++k) {
      const int idx = offset + k;
      stage[wave][idx % NS][(idx / NS) * G + sub] = val[k];
    }
  }
  wave_lds_sync();
  const bool want_lab = a.labels != nullptr, want_lp = a.log_post != nullptr, want_sc = a.scores != nullptr;
#pragma unroll
  for (int L0 = 0; L0 < BR; L0 += 64) {
    const int L = (BR >= 64) ? L0 + lane : lane % BR;
    if (FAST || L < nrows) {
      const int64_t row = row0 + L;
      const float delta = stage[wave][0][L] + rb[0];
      // log(1 + e^-|delta|) with the hardware exp/log: absolute error ~1e-7
      const float t = __logf(1.0f + __expf(-fabsf(delta)));
      float2 lp;
      lp.x = fminf(-delta, 0.0f) - t;
      lp.y = fminf(delta, 0.0f) - t;
      if (FAST) {
        int32_t* pl = want_lab ? a.labels + row : g_sink_label + lane;
        float2* pp = want_lp ? reinterpret_cast<float2*>(a.log_post) + row : g_sink_pair + lane;
        store_out(pl, delta > 0.0f ? 1 : 0);
        store_out(pp, lp);
        if (NS == 2) {
          float2 sc;
          sc.x = stage[wave][NS - 1][L] + rb[NS - 1];
          sc.y = sc.x + delta;
          float2* ps = want_sc ? reinterpret_cast<float2*>(a.scores) + row : g_sink_pair + lane;
          store_out(ps, sc);
        }
      } else {
        if (want_lab) store_out(a.labels + row, delta > 0.0f ? 1 : 0);
        if (want_lp) store_out(reinterpret_cast<float2*>(a.log_post) + row, lp);
        if (NS == 2 && want_sc) {
          float2 sc;
          sc.x = stage[wave][NS - 1][L] + rb[NS - 1];
          sc.y = sc.x + delta;
          store_out(reinterpret_cast<float2*>(a.scores) + row, sc);
        }
      }
    }
  }
  wave_lds_sync();
}

// Where a lane's features sit inside a chunk of 16*LPR features.  Byte
// features: 16 consecutive features from byte 16j, one 16-byte load.  int32
// features: four 16-byte loads 16*LPR bytes apart, so load q of the wave
// reads one contiguous 16*LPR-byte stretch of the chunk (whole cache lines
// per instruction); lane j holds features 4*LPR*q + 4j .. 4*LPR*q + 4j + 3.
template <int XT, int LPR>
struct LaneMap {
  static constexpr int kLoadStep = (XT == NB_X_I32) ? 16 * LPR : 16;   // bytes between a lane's loads
  static constexpr int kWStep = (XT == NB_X_I32) ? 4 * LPR : 4;        // features between its groups of four
  static __device__ __forceinline__ int feat0(int j) { return (XT == NB_X_I32) ? 4 * j : 16 * j; }
};

// The lane's 16 weights per row: four groups of four features, WSTEP apart.
template <int XT, int NS, int WSTEP = 4>
__device__ __forceinline__ void load_table(const float* tbl, int Fp, int fc, float (&w)[NS][16]) {
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const float4* t4 = reinterpret_cast<const float4*>(tbl + s * Fp + fc);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 t = t4[q * (WSTEP / 4)];
      w[s][4 * q + 0] = t.x;
      w[s][4 * q + 1] = t.y;
      w[s][4 * q + 2] = t.z;
      w[s][4 * q + 3] = t.w;
    }
  }
}

// FP8 bytes past the last feature may hold NaN encodings: mask them.
__device__ __forceinline__ void fp8_keep_mask(int F, int fc, uint32_t (&keep)[4]) {
  const int nv = max(0, F - fc);
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const int nb = min(4, max(0, nv - 4 * d));
    keep[d] = (nb >= 4) ? ~0u : ((1u << (8 * nb)) - 1u);
  }
}

template <int XT, int NS, bool BIN, int NV, int R>
__device__ __forceinline__ void accumulate_rows(dev::u32x4 (&v)[R][NV], const float (&w)[NS][16],
                                                const uint32_t (&keep)[4], bool masked, float (&acc)[R][NS]) {
#pragma unroll
  for (int i = 0; i < R; ++i) {
    if (XT == NB_X_FP8 && masked) {
#pragma unroll
      for (int d = 0; d < 4; ++d) v[i][0][d] &= keep[d];
    }
    accumulate_seg<XT, NS, BIN>(v[i], w, acc[i]);
  }
}


// Gaussian models: s_c = b_c + sum_f h_cf (x_f - mean_cf)^2 (the density's
// own form).  Two classes: the LDS table holds four rows, mean_0, mean_1,
// h_0, h_1; acc[0] gathers the log-odds terms h_1 d_1^2 - h_0 d_0^2 and,
// with raw scores, acc[1] the terms h_0 d_0^2 of s_0, so the reduction and
// the epilogue are those of the linear kinds.
template <int XT, int WSTEP = 4>
__device__ __forceinline__ void load_table_q(const float* tbl, int Fp, int fc, float (&mu)[2][16],
                                             float (&h)[2][16]) {
  load_table<XT, 2, WSTEP>(tbl, Fp, fc, mu);
  load_table<XT, 2, WSTEP>(tbl + 2 * Fp, Fp, fc, h);
}

template <int XT, int NS>
__device__ __forceinline__ void accumulate_seg_q(const dev::u32x4 (&v)[(XT == NB_X_I32) ? 4 : 1],
                                                 const float (&mu)[2][16], const float (&h)[2][16],
                                                 float (&acc)[NS]) {
  float xf[16];
  if (XT == NB_X_I32) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int d = 0; d < 4; ++d) xf[4 * q + d] = (float)(int32_t)v[q][d];
  } else {
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const uint32_t u = v[0][d];
      xf[4 * d + 0] = (float)(u & 0xFFu);
      xf[4 * d + 1] = (float)((u >> 8) & 0xFFu);
      xf[4 * d + 2] = (float)((u >> 16) & 0xFFu);
      xf[4 * d + 3] = (float)(u >> 24);
    }
  }
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const float d0 = xf[e] - mu[0][e], d1 = xf[e] - mu[1][e];
    const float t0 = h[0][e] * d0, t1 = h[1][e] * d1;
    acc[0] = fmaf(t1, d1, fmaf(-t0, d0, acc[0]));
    if (NS == 2) acc[NS - 1] = fmaf(t0, d0, acc[NS - 1]);
  }
}

template <int XT, int NS, int NV, int R>
__device__ __forceinline__ void accumulate_rows_q(dev::u32x4 (&v)[R][NV], const float (&mu)[2][16],
                                                  const float (&h)[2][16], float (&acc)[R][NS]) {
#pragma unroll
  for (int i = 0; i < R; ++i) accumulate_seg_q<XT, NS>(v[i], mu, h, acc[i]);
}

// Copy the NS scoring rows (FP32, or BF16 widened: exact) into LDS.  The
// caller synchronises the workgroup afterwards.
template <int NS>
__device__ __forceinline__ void stage_table(const Score2Args& a, float* tbl) {
  for (int i = threadIdx.x; i < NS * a.Fp; i += kThreads)
    tbl[i] = (a.wt == NB_W_BF16) ? dev::bf16_to_f32(a.rows16[i]) : a.rows32[i];
}

// Gaussian (two classes): the two mean rows, then the two h rows.
__device__ __forceinline__ void stage_table_q(const Score2Args& a, float* tbl) {
  stage_table<2>(a, tbl);
  for (int i = threadIdx.x; i < 2 * a.Fp; i += kThreads)
    tbl[2 * a.Fp + i] = (a.wt == NB_W_BF16) ? dev::bf16_to_f32(a.rows16_q[i]) : a.rows32_q[i];
}

// ---- flat staging helpers (see score_blocks)
// LDS bytes of one wave's staging region: the window, then 16 bytes that
// catch the reads of a row's last 16-byte piece past the window's end.
__host__ __device__ constexpr int flat_region_bytes(int fl) { return fl * 1024 + 16; }

// Start of a block's window, relative to a.x: the cache line holding the
// block's first byte (x itself when that line begins before the buffer),
// moved back so that the window ends inside the buffer (the host stages a
// block only when the buffer holds at least a window).
__device__ __forceinline__ int64_t flat_window_start(const Score2Args& a, int64_t s0, int fl) {
  const int64_t mis = (int64_t)(reinterpret_cast<uintptr_t>(a.x + s0) & 127u);
  const int64_t w0 = s0 >= mis ? s0 - mis : 0;
  const int64_t last = a.total_bytes - (int64_t)fl * 1024;
  return w0 < last ? w0 : last;
}

// Rows of block blk (all BR but for a buffer's partial last block).
template <int BR>
__device__ __forceinline__ int flat_block_rows(const Score2Args& a, int64_t blk) {
  const int64_t left = a.n - blk * BR;
  return left < BR ? (int)left : BR;
}

// Accumulate the R rows of one chunk from a staged window: lane j reads its
// 16 bytes of each row (rows 8-byte aligned in LDS, the host's condition:
// two 8-byte reads); a lane whose features all lie past F reads nothing
// (its weights are zero: the same sums).
// Rows are read four at a time (the scheduler would otherwise hoist every
// row's LDS read ahead of the arithmetic: 64 registers).
template <int XT, int NS, bool BIN, int R>
__device__ __forceinline__ void read_flat_rows(const uint8_t* p, uint32_t ld, bool live, const float (&w)[NS][16],
                                               const uint32_t (&keep)[4], float (&acc)[R][NS]) {
  constexpr int kBatch = R < 4 ? R : 4;
#pragma unroll
  for (int i0 = 0; i0 < R; i0 += kBatch) {
    dev::u32x4 v[kBatch][1];
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      v[b][0] = dev::u32x4{0u, 0u, 0u, 0u};
      if (live) {
        const uint2* q2 = reinterpret_cast<const uint2*>(p + (uint32_t)(i0 + b) * ld);
        const uint2 lo = q2[0], hi = q2[1];
        v[b][0] = dev::u32x4{lo.x, lo.y, hi.x, hi.y};
      }
    }
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      if (XT == NB_X_FP8) {
#pragma unroll
        for (int d = 0; d < 4; ++d) v[b][0][d] &= keep[d];
      }
      accumulate_seg<XT, NS, BIN>(v[b], w, acc[i0 + b]);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// One wave scores the blocks first, first + stride, ... below `end` of the
// files described by `a` (a block is R row-steps of 64/LPR rows; rows are
// relative to a.x and to the output pointers).  Blocks below a.nfast take
// the pipelined path: every row present and every load in bounds, the loads
// of the next unit (block, chunk) in flight while the current one is
// accumulated.  The rest take guarded loads.  tbl: the rows in LDS.
// MULTI: F spans more than one chunk of 16*LPR features (only with LPR = 64).
// QUAD: a Gaussian model (x and x^2 rows, see accumulate_seg_q).
// FL > 0: byte features with one row per row-step: the blocks below a.nflat
// are fetched as ONE aligned byte range (FL pieces of 1 KB per wave: whole
// cache lines per load instruction, however the rows fall on lines) into the
// wave's region of `flat` (LDS, kWaves * FL KB), and each row is then read
// from LDS with the same lane mapping, so the arithmetic is unchanged.
template <int XT, int LPR, int NS, bool BIN, bool MULTI, bool QUAD = false, int FL = 0>
__device__ __forceinline__ void score_blocks(const Score2Args& a, const float* tbl, int64_t first, int64_t stride,
                                             int64_t end,
                                             float (*stage)[NS][(64 / LPR) * block_steps<XT, QUAD, MULTI, FL>()],
                                             uint8_t* flat = nullptr) {
  constexpr int EB = (XT == NB_X_I32) ? 4 : 1;
  constexpr int NV = EB;
  constexpr int G = 64 / LPR;           // rows per row-step
  constexpr int R = block_steps<XT, QUAD, MULTI, FL>();
  constexpr int BR = G * R;             // rows per block
  constexpr int CW = 16 * LPR;          // features per chunk
  using LM = LaneMap<XT, LPR>;

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int sub = lane / LPR, j = lane % LPR;
  const int nch = MULTI ? a.nch : 1;
  const int64_t ld = a.ld_bytes;
  // this lane's first byte offsets inside a block: row (i*G + sub), byte 16*j
  uint32_t voff[R];
#pragma unroll
  for (int i = 0; i < R; ++i)
    voff[i] = (uint32_t)((i * G + sub) * ld) + (uint32_t)((XT == NB_X_I32) ? 16 * j : 16 * j * EB);

  float rb[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) rb[s] = a.row_bias[s];

  float w[QUAD ? 2 : NS][16];        // Gaussian: the means
  float w2[QUAD ? 2 : 1][16];        // Gaussian: h
  uint32_t keep[4] = {~0u, ~0u, ~0u, ~0u};
  auto load_w = [&](int fc) {
    if constexpr (QUAD) load_table_q<XT, LM::kWStep>(tbl, a.Fp, fc, w, w2);
    else load_table<XT, NS, LM::kWStep>(tbl, a.Fp, fc, w);
  };
  if (!MULTI) {
    load_w((XT == NB_X_I32) ? LM::feat0(j) : 16 * j);
    if (XT == NB_X_FP8) fp8_keep_mask(a.F, 16 * j, keep);
  }

  float acc[R][NS];
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int s = 0; s < NS; ++s) acc[i][s] = 0.0f;
  auto accumulate = [&](dev::u32x4 (&v)[R][NV]) {
    if constexpr (QUAD) accumulate_rows_q<XT, NS, NV>(v, w, w2, acc);
    else accumulate_rows<XT, NS, BIN, NV>(v, w, keep, true, acc);
  };

  // ---- flat blocks: first + k*stride < min(end, nflat)
  if constexpr (FL > 0) {
    static_assert(XT != NB_X_I32 && LPR == 64 && !QUAD, "flat staging: byte features, one row per row-step");
    constexpr int kPiece = 64 * 16;     // bytes of one wave load instruction
    uint8_t* mine = flat + (size_t)wave * flat_region_bytes(FL);
    const int64_t flat_end = a.nflat < end ? a.nflat : end;
    const int nb = (flat_end > first) ? (int)((flat_end - first + stride - 1) / stride) : 0;
    dev::u32x4 fb[FL];
    uint32_t lead_next = 0;
    auto issue_flat = [&](int k) {
      const int64_t blk = first + (int64_t)k * stride;
      const int64_t s0 = blk * BR * ld;
      const int64_t w0 = flat_window_start(a, s0, FL);
      lead_next = (uint32_t)(s0 - w0);
      const uint32_t span = lead_next + (uint32_t)((flat_block_rows<BR>(a, blk) - 1) * ld + a.F);
      const auto rsrc = dev::make_rsrc(dev::uniform_ptr(a.x + w0), dev::uniform64(a.total_bytes - w0));
#pragma unroll
      for (int q = 0; q < FL; ++q) {
        const uint32_t off = (uint32_t)(q * kPiece + 16 * lane);
        fb[q] = dev::buffer_load16(rsrc, off < span ? off : dev::kNoAccess);
      }
      __builtin_amdgcn_sched_barrier(0);
    };
    auto consume_flat = [&](uint32_t lead, int64_t blk) {
      for (int ch = 0; ch < nch; ++ch) {
        const int fc = ch * CW + 16 * j;
        if (MULTI) {
          load_w(fc);
          if (XT == NB_X_FP8) fp8_keep_mask(a.F, fc, keep);
        }
        read_flat_rows<XT, NS, BIN, R>(mine + lead + (uint32_t)fc, (uint32_t)ld, fc < a.F, w, keep, acc);
      }
      // a buffer's last block may be partial (its window moved back from
      // the end): rows past it hold stale bytes and are never stored
      const int nrows = flat_block_rows<BR>(a, blk);
      if (nrows == BR) finish_block<LPR, NS, true>(a, acc, lane, wave, sub, rb, blk * BR, BR, stage);
      else finish_block<LPR, NS, false>(a, acc, lane, wave, sub, rb, blk * BR, nrows, stage);
#pragma unroll
      for (int i = 0; i < R; ++i)
#pragma unroll
        for (int s = 0; s < NS; ++s) acc[i][s] = 0.0f;
    };
    if (nb > 0) {
      issue_flat(0);
      for (int k = 0; k < nb; ++k) {
#pragma unroll
        for (int q = 0; q < FL; ++q) *reinterpret_cast<dev::u32x4*>(mine + q * kPiece + 16 * lane) = fb[q];
        const uint32_t lead = lead_next;
        if (k + 1 < nb) issue_flat(k + 1);
        consume_flat(lead, first + (int64_t)k * stride);
      }
    }
    first += (int64_t)nb * stride;
  }

  // ---- fast blocks: first + i*stride < min(end, nfast).  Per-wave counters
  // are 32-bit so loop control stays on the scalar unit.  (Flat kernels
  // leave the few blocks past nflat to the guarded loop: the double buffer
  // of their block size would not fit the register file.)
  const int64_t fast_end = FL > 0 ? first : (a.nfast < end ? a.nfast : end);
  const int my_blocks = (fast_end > first) ? (int)((fast_end - first + stride - 1) / stride) : 0;
  const int units = my_blocks * nch;
  dev::u32x4 buf0[R][NV], buf1[R][NV];
  int ib = 0;       // index of the block being issued, among this wave's blocks
  int ich = 0;      // chunk being issued
  // point the issue cursor back at the last issued unit; written as value
  // selects: a branch that decrements one of two counters becomes a store
  // to a selected address, which moves both counters to scratch memory
  auto rewind = [&]() {
    const bool wrap = ich == 0;
    ib = wrap ? ib - 1 : ib;
    ich = wrap ? nch - 1 : ich - 1;
  };
  auto issue = [&](dev::u32x4 (&dst)[R][NV]) {
    const int64_t blk = first + (int64_t)ib * stride;
    const int64_t off = blk * BR * ld + (int64_t)ich * CW * EB;
    const auto rsrc = dev::make_rsrc(a.x + off, a.total_bytes - off);
    // a load whose features of this chunk all lie past F reads nothing:
    // those bytes belong to the next row, which its own loads fetch
    if constexpr (XT == NB_X_I32) {
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        const bool live = ich * CW + LM::feat0(j) + q * LM::kWStep < a.F;
#pragma unroll
        for (int i = 0; i < R; ++i)
          dst[i][q] = dev::buffer_load16(rsrc, live ? voff[i] + q * LM::kLoadStep : dev::kNoAccess);
      }
    } else {
      const bool live = ich * CW + 16 * j < a.F;
#pragma unroll
      for (int i = 0; i < R; ++i)
#pragma unroll
        for (int q = 0; q < NV; ++q) dst[i][q] = dev::buffer_load16(rsrc, live ? voff[i] + 16 * q : dev::kNoAccess);
    }
    // keep the loads here: the scheduler would otherwise sink them into the
    // arithmetic of the unit being consumed and shrink the overlap
    __builtin_amdgcn_sched_barrier(0);
    if (++ich == nch) {
      ich = 0;
      ++ib;
    }
  };
  int cb = 0;       // block being computed
  int cch = 0;      // chunk being computed
  auto consume = [&](dev::u32x4 (&src)[R][NV]) {
    if (MULTI) {
      const int fc = cch * CW + ((XT == NB_X_I32) ? LM::feat0(j) : 16 * j);
      load_w(fc);
      if (XT == NB_X_FP8) fp8_keep_mask(a.F, fc, keep);
    }
    accumulate(src);
    if (++cch == nch) {
      finish_block<LPR, NS, true>(a, acc, lane, wave, sub, rb, (first + (int64_t)cb * stride) * BR, BR, stage);
#pragma unroll
      for (int i = 0; i < R; ++i)
#pragma unroll
        for (int s = 0; s < NS; ++s) acc[i][s] = 0.0f;
      cch = 0;
      ++cb;
    }
  };
  // The prefetch of the unit after the last one re-reads the last unit (an L2
  // hit) so that every iteration issues the same loads unconditionally.
  if (units > 0 && !kPipeline) {
    for (int u = 0; u < units; ++u) {
      issue(buf0);
      consume(buf0);
    }
  } else if (units > 0) {
    issue(buf0);
    for (int u = 0;; u += 2) {
      if (u + 1 >= units) rewind();
      issue(buf1);
      consume(buf0);
      if (u + 1 >= units) break;
      if (u + 2 >= units) rewind();
      issue(buf0);
      consume(buf1);
      if (u + 2 >= units) break;
    }
  }

  // ---- the wave's remaining blocks: guarded loads, partial rows
  const int64_t nrows_total = a.n;
  for (int64_t blk = first + (int64_t)my_blocks * stride; blk < end; blk += stride) {
    const int64_t row0 = blk * BR;
    const int nrows = (int)min((int64_t)BR, nrows_total - row0);
    for (int ch = 0; ch < nch; ++ch) {
      const int fc = ch * CW + ((XT == NB_X_I32) ? LM::feat0(j) : 16 * j);
      if (MULTI) {
        load_w(fc);
        if (XT == NB_X_FP8) fp8_keep_mask(a.F, fc, keep);
      }
      dev::u32x4 v[R][NV];
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int L = i * G + sub;
#pragma unroll
        for (int q = 0; q < NV; ++q) v[i][q] = dev::u32x4{0u, 0u, 0u, 0u};
        if (L < nrows) {
          if constexpr (XT == NB_X_I32) {
            const int64_t off = (row0 + L) * ld + (int64_t)ch * CW * EB + 16 * j;
#pragma unroll
            for (int q = 0; q < NV; ++q)
              v[i][q] = dev::load16_guarded(a.x + off + q * LM::kLoadStep, a.total_bytes - off - q * LM::kLoadStep);
          } else {
            const int64_t off = (row0 + L) * ld + (int64_t)fc * EB;
#pragma unroll
            for (int q = 0; q < NV; ++q)
              v[i][q] = dev::load16_guarded(a.x + off + 16 * q, a.total_bytes - off - 16 * q);
          }
        }
      }
      accumulate(v);
    }
    finish_block<LPR, NS, false>(a, acc, lane, wave, sub, rb, row0, nrows, stage);
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
      for (int s = 0; s < NS; ++s) acc[i][s] = 0.0f;
  }
}

// ------------------------------------------------------------ host helpers
int lanes_per_row(int F) {
  const int need = (F + 15) / 16;
  int l = 4;
  while (l < need && l < 64) l <<= 1;
  return l;
}

constexpr size_t kMaxTableLds = 128 * 1024;

// Flat staging (score_blocks with FL > 0): 1 KB pieces per wave (32), or 0
// when the call does not qualify.  It needs byte features in two chunks per
// row (1024 < F), rows 8-byte aligned (x, the stride and F), little padding
// between rows (the window fetches it), and a block's window (up to 127
// bytes before its first row, its rows, each lane's last chunk) within
// 32 KB.  NB_FLAT_ROWS=0 in the environment turns it off.
constexpr int64_t kFlatMinBlock = 28 * 1024;
inline int flat_pieces(int xtype, int F, int64_t ld_bytes, const void* x, bool quad) {
  static const bool off = [] {
    const char* e = std::getenv("NB_FLAT_ROWS");
    return e && e[0] == '0';
  }();
  if (off || quad || xtype == NB_X_I32 || lanes_per_row(F) != 64) return 0;
  // 8-byte aligned rows and buffer end: windows (including those moved
  // back from the end) keep every row 8-byte aligned in LDS
  if (((reinterpret_cast<uintptr_t>(x) | (uintptr_t)ld_bytes | (uintptr_t)F) & 7u) != 0) return 0;
  if (ld_bytes * 16 > (int64_t)F * 17) return 0;
  const int nch = (F + 1023) / 1024;
  const int64_t rows = block_steps_of(xtype, false, nch, 32);
  const int64_t need = 127 + (rows - 1) * ld_bytes + (int64_t)nch * 1024;
  // two-chunk rows only, a window within 32 KB that carries enough bytes to
  // keep the wave's loads in flight (measured on gfx950: one-chunk rows and
  // smaller blocks run no faster, or slower, than direct loads)
  return (nch == 2 && need <= 32 * 1024 && rows * ld_bytes >= kFlatMinBlock) ? 32 : 0;
}

// Launch arguments of the two-class kernels for one model and one feature
// matrix (arguments already validated).  Returns NB_OK or NB_EINVAL.
int make_score2_args(const nb_model* m, const nb_layout& L, const void* x, int32_t xtype, int64_t n, int64_t ld,
                     int32_t wtype, int32_t* labels, float* log_post, float* scores, int ns, Score2Args* out,
                     bool quad = false, int fl = 0) {
  const int F = m->n_features;
  const int eb = elem_bytes(xtype);
  const int lpr = lanes_per_row(F);
  const int cw = 16 * lpr;
  const int nch = (F + cw - 1) / cw;
  if ((size_t)(quad ? 4 : ns) * L.padded_features * sizeof(float) > kMaxTableLds)
    return fail(NB_EINVAL, quad ? "two-class Gaussian scoring supports F up to 8192 (tables staged in LDS)"
                                : "two-class scoring supports F up to 16384 (table staged in LDS)");
  const uint8_t* base = static_cast<const uint8_t*>(m->dev);
  Score2Args a;
  a.x = static_cast<const uint8_t*>(x);
  a.ld_bytes = ld * eb;
  a.n = n;
  a.total_bytes = ((n - 1) * ld + F) * (int64_t)eb;
  a.rows32 = reinterpret_cast<const float*>(base + L.off_form_f32);
  a.rows16 = reinterpret_cast<const uint16_t*>(base + L.off_form_bf16);
  a.row_bias = reinterpret_cast<const float*>(base + L.off_form_bias);
  a.rows32_q = reinterpret_cast<const float*>(base + L.off_form2_f32);
  a.rows16_q = reinterpret_cast<const uint16_t*>(base + L.off_form2_bf16);
  a.labels = labels;
  a.log_post = log_post;
  a.scores = scores;
  a.F = F;
  a.Fp = L.padded_features;
  a.nch = nch;
  a.wt = wtype;
  const int64_t rows_per_blk = (int64_t)(64 / lpr) * block_steps_of(xtype, quad, nch, fl);
  if (rows_per_blk * a.ld_bytes >= (int64_t)1 << 31)
    return fail(NB_EINVAL, "row stride too large (a block of rows must span < 2 GiB)");
  // leading blocks whose rows all exist and whose loads stay inside the buffer
  const int64_t span = (int64_t)nch * cw * eb;
  const int64_t full = n / rows_per_blk;
  const int64_t rmax = (a.total_bytes >= span) ? (a.total_bytes - span) / a.ld_bytes : -1;
  a.nfast = std::max<int64_t>(0, std::min(full, (rmax + 1) / rows_per_blk));
  // flat staging: every block, the partial last one included, once the
  // buffer holds a whole window (windows near the end are moved back
  // inside the buffer)
  a.nflat = (fl > 0 && a.total_bytes >= (int64_t)fl * 1024) ? (n + rows_per_blk - 1) / rows_per_blk : 0;
  *out = a;
  return NB_OK;
}

// Kernel pointer of a two-class kernel family: Fam::fn<XT, LPR, NS, BIN,
// MULTI, FL>() (FL: flat staging pieces, byte features with LPR = 64 only).
template <class Fam, int XT, int NS, bool BIN>
const void* pick_lpr(int lpr, bool multi, int fl) {
  switch (lpr) {
    case 4: return Fam::template fn<XT, 4, NS, BIN, false>();
    case 8: return Fam::template fn<XT, 8, NS, BIN, false>();
    case 16: return Fam::template fn<XT, 16, NS, BIN, false>();
    case 32: return Fam::template fn<XT, 32, NS, BIN, false>();
    default:
      if constexpr (XT != NB_X_I32) {
        if (fl == 32 && multi) return Fam::template fn<XT, 64, NS, BIN, true, 32>();
      }
      return multi ? Fam::template fn<XT, 64, NS, BIN, true>() : Fam::template fn<XT, 64, NS, BIN, false>();
  }
}

template <class Fam, int XT>
const void* pick_ns_bin(int lpr, bool multi, int ns, bool bin, int fl) {
  if (ns == 1) return bin ? pick_lpr<Fam, XT, 1, true>(lpr, multi, fl) : pick_lpr<Fam, XT, 1, false>(lpr, multi, fl);
  return bin ? pick_lpr<Fam, XT, 2, true>(lpr, multi, fl) : pick_lpr<Fam, XT, 2, false>(lpr, multi, fl);
}

template <class Fam>
const void* pick_score2(int xtype, int lpr, bool multi, int ns, bool bin, int fl = 0) {
  switch (xtype) {
    case NB_X_U8: return pick_ns_bin<Fam, NB_X_U8>(lpr, multi, ns, bin, fl);
    case NB_X_I32: return pick_ns_bin<Fam, NB_X_I32>(lpr, multi, ns, bin, 0);
    default: return pick_ns_bin<Fam, NB_X_FP8>(lpr, multi, ns, bin, fl);
  }
}

}  // namespace
}  // namespace nb
