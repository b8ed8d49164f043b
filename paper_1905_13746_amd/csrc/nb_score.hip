// Naive Bayes scoring on gfx950: per-file joint log-likelihoods, the label
// and the log posteriors (paper, section 4: posterior of each class given the
// file's opcode occurrences; malware iff its posterior is the higher one).
//
// Two-class path (score2_kernel).  The posterior of a two-class model depends
// on the log-odds only,
//   Delta = s_1 - s_0 = (b_1 - b_0) + sum_f g(x_f) (W_1f - W_0f),
// so the kernel contracts each file against ONE row (the log-odds row, built
// in FP64 and rounded once) and performs one FMA per feature; the raw scores,
// when requested, add a second row (W_0) for s_0 and take s_1 = s_0 + Delta.
// This is HBM-bound streaming (about 2 VALU operations per feature byte), not
// a GEMM, so it stays on the vector ALUs.
//
// Mapping.  A row (file) is split across LPR lanes of a wave (LPR = the
// smallest power of two >= F/16, at most 64), each lane owning 16 consecutive
// features per chunk of 16*LPR features: its loads are 16 contiguous bytes,
// so a wave instruction reads 64/LPR whole rows (or one 16*LPR-feature
// stretch of a row) contiguously.  A wave processes R = 8 row-steps of
// 64/LPR rows per block and strides over blocks (persistent grid sized to the
// resident capacity).  The table row(s) sit in LDS as FP32 (BF16 tables are
// widened on load: exact).  Lane partial sums are reduced across the LPR
// lanes with a transposed butterfly (each exchange step halves the number of
// values per lane), staged in LDS and handed to one lane per file for the
// fused epilogue: label, log-sum-exp, log posteriors, raw scores.
//
// Summation order of a file depends only on (F, xtype): lanes sum their 16
// features in order, chunks in order, then the fixed butterfly.  It never
// depends on n, on the block a file lands in, or on other files.
#include <algorithm>
#include <map>
#include <mutex>

#include "nb_device.hpp"
#include "nb_internal.hpp"

namespace nb {
namespace {

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
// Rows per lane group per block, and whether a wave double-buffers its loads
// (the next unit's loads in flight while the current one is accumulated).
#ifndef NB_ROW_STEPS
#define NB_ROW_STEPS 8
#endif
#ifndef NB_PIPELINE
#define NB_PIPELINE 1
#endif
constexpr int kRowSteps = NB_ROW_STEPS;
constexpr bool kPipeline = NB_PIPELINE != 0;

struct Score2Args {
  const uint8_t* x;
  int64_t ld_bytes;
  int64_t n;
  int64_t total_bytes;
  const float* rows32;      // [2][Fp] log-odds row, aux row
  const uint16_t* rows16;   // same rows in BF16
  const float* row_bias;    // [2]
  int32_t* labels;
  float* log_post;
  float* scores;
  int64_t nfast;            // leading blocks with every row present and in bounds
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
    // presence: byte/int counts are integers >= 0, so min(x, 1) is 1[x > 0];
    // FP8 values may be fractional, so compare
    const float g = !BIN ? xf[e] : (XT == NB_X_FP8 ? (xf[e] > 0.0f ? 1.0f : 0.0f) : fminf(xf[e], 1.0f));
#pragma unroll
    for (int s = 0; s < NS; ++s) acc[s] = fmaf(g, w[s][e], acc[s]);
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
template <int LPR, int NS, bool FAST>
__device__ __forceinline__ void finish_block(const Score2Args& a, float (&acc)[kRowSteps][NS], int lane, int wave,
                                             int sub, const float (&rb)[NS], int64_t row0, int nrows,
                                             float (*stage)[NS][(64 / LPR) * kRowSteps]) {
  constexpr int G = 64 / LPR;
  constexpr int R = kRowSteps;
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
        const float send = up ? val[k] : val[k + h];
        const float keep = up ? val[k + h] : val[k];
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
        *pl = delta > 0.0f ? 1 : 0;
        *pp = lp;
        if (NS == 2) {
          float2 sc;
          sc.x = stage[wave][NS - 1][L] + rb[NS - 1];
          sc.y = sc.x + delta;
          float2* ps = want_sc ? reinterpret_cast<float2*>(a.scores) + row : g_sink_pair + lane;
          *ps = sc;
        }
      } else {
        if (want_lab) a.labels[row] = delta > 0.0f ? 1 : 0;
        if (want_lp) reinterpret_cast<float2*>(a.log_post)[row] = lp;
        if (NS == 2 && want_sc) {
          float2 sc;
          sc.x = stage[wave][NS - 1][L] + rb[NS - 1];
          sc.y = sc.x + delta;
          reinterpret_cast<float2*>(a.scores)[row] = sc;
        }
      }
    }
  }
  wave_lds_sync();
}

template <int XT, int NS>
__device__ __forceinline__ void load_table(const float* tbl, int Fp, int fc, float (&w)[NS][16]) {
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const float4* t4 = reinterpret_cast<const float4*>(tbl + s * Fp + fc);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 t = t4[q];
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

template <int XT, int NS, bool BIN, int NV>
__device__ __forceinline__ void accumulate_rows(dev::u32x4 (&v)[kRowSteps][NV], const float (&w)[NS][16],
                                                const uint32_t (&keep)[4], bool masked,
                                                float (&acc)[kRowSteps][NS]) {
#pragma unroll
  for (int i = 0; i < kRowSteps; ++i) {
    if (XT == NB_X_FP8 && masked) {
#pragma unroll
      for (int d = 0; d < 4; ++d) v[i][0][d] &= keep[d];
    }
    accumulate_seg<XT, NS, BIN>(v[i], w, acc[i]);
  }
}

// MULTI: F spans more than one chunk of 16*LPR features (only with LPR = 64).
template <int XT, int LPR, int NS, bool BIN, bool MULTI>
__global__ __launch_bounds__(kThreads) void score2_kernel(Score2Args a) {
  constexpr int EB = (XT == NB_X_I32) ? 4 : 1;
  constexpr int NV = EB;
  constexpr int G = 64 / LPR;           // rows per row-step
  constexpr int R = kRowSteps;
  constexpr int BR = G * R;             // rows per block
  constexpr int CW = 16 * LPR;          // features per chunk

  extern __shared__ float tbl[];        // [NS][Fp]
  __shared__ float stage[kWaves][NS][BR];

  for (int i = threadIdx.x; i < NS * a.Fp; i += kThreads)
    tbl[i] = (a.wt == NB_W_BF16) ? dev::bf16_to_f32(a.rows16[i]) : a.rows32[i];
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int sub = lane / LPR, j = lane % LPR;
  const int64_t wave_id = (int64_t)blockIdx.x * kWaves + wave;
  const int64_t nwaves = (int64_t)gridDim.x * kWaves;
  const int nch = MULTI ? a.nch : 1;
  const int64_t ld = a.ld_bytes;
  // this lane's byte offsets inside a block: row (i*G + sub), feature 16*j
  uint32_t voff[R];
#pragma unroll
  for (int i = 0; i < R; ++i) voff[i] = (uint32_t)((i * G + sub) * ld) + (uint32_t)(16 * j * EB);

  float rb[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) rb[s] = a.row_bias[s];

  float w[NS][16];
  uint32_t keep[4] = {~0u, ~0u, ~0u, ~0u};
  if (!MULTI) {
    load_table<XT, NS>(tbl, a.Fp, 16 * j, w);
    if (XT == NB_X_FP8) fp8_keep_mask(a.F, 16 * j, keep);
  }

  float acc[R][NS];
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int s = 0; s < NS; ++s) acc[i][s] = 0.0f;

  // ---- fast blocks [0, nfast): every row present and every load in bounds.
  // Units (block, chunk) are visited in order; the loads of the next unit are
  // in flight while the current one is accumulated (two register buffers).
  // per-wave counters are 32-bit so loop control stays on the scalar unit
  const int my_blocks = (a.nfast > wave_id) ? (int)((a.nfast - wave_id + nwaves - 1) / nwaves) : 0;
  const int units = my_blocks * nch;
  dev::u32x4 buf0[R][NV], buf1[R][NV];
  int ib = 0;       // index of the block being issued, among this wave's blocks
  int ich = 0;      // chunk being issued
  auto rewind = [&]() {          // point the issue cursor back at the last issued unit
    if (ich == 0) {
      ich = nch - 1;
      --ib;
    } else {
      --ich;
    }
  };
  auto issue = [&](dev::u32x4 (&dst)[R][NV]) {
    const int64_t blk = wave_id + (int64_t)ib * nwaves;
    const int64_t off = blk * BR * ld + (int64_t)ich * CW * EB;
    const auto rsrc = dev::make_rsrc(a.x + off, a.total_bytes - off);
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
      for (int q = 0; q < NV; ++q) dst[i][q] = dev::buffer_load16(rsrc, voff[i] + 16 * q);
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
      const int fc = cch * CW + 16 * j;
      load_table<XT, NS>(tbl, a.Fp, fc, w);
      if (XT == NB_X_FP8) fp8_keep_mask(a.F, fc, keep);
    }
    accumulate_rows<XT, NS, BIN, NV>(src, w, keep, true, acc);
    if (++cch == nch) {
      finish_block<LPR, NS, true>(a, acc, lane, wave, sub, rb, (wave_id + (int64_t)cb * nwaves) * BR, BR, stage);
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

  // ---- remaining blocks [nfast, nblk): guarded loads, partial rows
  const int64_t nblk = (a.n + BR - 1) / BR;
  for (int64_t blk = a.nfast + wave_id; blk < nblk; blk += nwaves) {
    const int64_t row0 = blk * BR;
    const int nrows = (int)min((int64_t)BR, a.n - row0);
    for (int ch = 0; ch < nch; ++ch) {
      const int fc = ch * CW + 16 * j;
      if (MULTI) {
        load_table<XT, NS>(tbl, a.Fp, fc, w);
        if (XT == NB_X_FP8) fp8_keep_mask(a.F, fc, keep);
      }
      dev::u32x4 v[R][NV];
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int L = i * G + sub;
#pragma unroll
        for (int q = 0; q < NV; ++q) v[i][q] = dev::u32x4{0u, 0u, 0u, 0u};
        if (L < nrows) {
          const int64_t off = (row0 + L) * ld + (int64_t)fc * EB;
#pragma unroll
          for (int q = 0; q < NV; ++q)
            v[i][q] = dev::load16_guarded(a.x + off + 16 * q, a.total_bytes - off - 16 * q);
        }
      }
      accumulate_rows<XT, NS, BIN, NV>(v, w, keep, true, acc);
    }
    finish_block<LPR, NS, false>(a, acc, lane, wave, sub, rb, row0, nrows, stage);
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
      for (int s = 0; s < NS; ++s) acc[i][s] = 0.0f;
  }
}

// ---------------------------------------------------------------- dispatch
using KernelFn = void (*)(Score2Args);

template <int XT, int NS, bool BIN>
KernelFn pick_lpr(int lpr, bool multi) {
  switch (lpr) {
    case 4: return score2_kernel<XT, 4, NS, BIN, false>;
    case 8: return score2_kernel<XT, 8, NS, BIN, false>;
    case 16: return score2_kernel<XT, 16, NS, BIN, false>;
    case 32: return score2_kernel<XT, 32, NS, BIN, false>;
    default: return multi ? score2_kernel<XT, 64, NS, BIN, true> : score2_kernel<XT, 64, NS, BIN, false>;
  }
}

template <int XT>
KernelFn pick2(int lpr, bool multi, int ns, bool bin) {
  if (ns == 1) return bin ? pick_lpr<XT, 1, true>(lpr, multi) : pick_lpr<XT, 1, false>(lpr, multi);
  return bin ? pick_lpr<XT, 2, true>(lpr, multi) : pick_lpr<XT, 2, false>(lpr, multi);
}

KernelFn pick_score2(int xtype, int lpr, bool multi, int ns, bool bin) {
  switch (xtype) {
    case NB_X_U8: return pick2<NB_X_U8>(lpr, multi, ns, bin);
    case NB_X_I32: return pick2<NB_X_I32>(lpr, multi, ns, bin);
    default: return pick2<NB_X_FP8>(lpr, multi, ns, bin);
  }
}

int lanes_per_row(int F) {
  const int need = (F + 15) / 16;
  int l = 4;
  while (l < need && l < 64) l <<= 1;
  return l;
}

// Resident workgroups per CU for a kernel and its dynamic LDS (cached).
int resident_per_cu(const void* fn, size_t lds) {
  static std::mutex mu;
  static std::map<std::pair<const void*, size_t>, int> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto key = std::make_pair(fn, lds);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int per = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, kThreads, lds) != hipSuccess || per < 1) per = 1;
  cache[key] = per;
  return per;
}

constexpr size_t kMaxTableLds = 128 * 1024;

int launch_score2(const nb_model* m, const nb_layout& L, const void* x, int32_t xtype, int64_t n, int64_t ld,
                  int32_t wtype, int32_t* labels, float* log_post, float* scores, hipStream_t s) {
  const int F = m->n_features;
  const int eb = elem_bytes(xtype);
  const int lpr = lanes_per_row(F);
  const int cw = 16 * lpr;
  const int nch = (F + cw - 1) / cw;
  const int ns = scores ? 2 : 1;
  const size_t lds = (size_t)ns * L.padded_features * sizeof(float);
  if (lds > kMaxTableLds)
    return fail(NB_EINVAL, "two-class scoring supports F up to 16384 (table staged in LDS)");
  const uint8_t* base = static_cast<const uint8_t*>(m->dev);
  Score2Args a;
  a.x = static_cast<const uint8_t*>(x);
  a.ld_bytes = ld * eb;
  a.n = n;
  a.total_bytes = ((n - 1) * ld + F) * (int64_t)eb;
  a.rows32 = reinterpret_cast<const float*>(base + L.off_form_f32);
  a.rows16 = reinterpret_cast<const uint16_t*>(base + L.off_form_bf16);
  a.row_bias = reinterpret_cast<const float*>(base + L.off_form_bias);
  a.labels = labels;
  a.log_post = log_post;
  a.scores = scores;
  a.F = F;
  a.Fp = L.padded_features;
  a.nch = nch;
  a.wt = wtype;
  const int64_t rows_per_blk = (int64_t)(64 / lpr) * kRowSteps;
  if (rows_per_blk * a.ld_bytes >= (int64_t)1 << 31)
    return fail(NB_EINVAL, "row stride too large (a block of rows must span < 2 GiB)");
  // leading blocks whose rows all exist and whose loads stay inside the buffer
  {
    const int64_t span = (int64_t)nch * cw * eb;
    const int64_t full = n / rows_per_blk;
    const int64_t rmax = (a.total_bytes >= span) ? (a.total_bytes - span) / a.ld_bytes : -1;
    a.nfast = std::max<int64_t>(0, std::min(full, (rmax + 1) / rows_per_blk));
  }
  KernelFn fn = pick_score2(xtype, lpr, nch > 1, ns, m->kind == NB_BERNOULLI);
  if (lds > 64 * 1024) NB_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  const int64_t nblk = (n + rows_per_blk - 1) / rows_per_blk;
  const int64_t want = (nblk + kWaves - 1) / kWaves;
  const int64_t cap = (int64_t)resident_per_cu(reinterpret_cast<const void*>(fn), lds) * device_cu_count();
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min(want, cap));
  hipLaunchKernelGGL(fn, dim3(grid), dim3(kThreads), lds, s, a);
  NB_HIP_CHECK(hipGetLastError());
  return NB_OK;
}

}  // namespace
}  // namespace nb

using namespace nb;

extern "C" int nb_score(const nb_model* m, const void* x, int32_t xtype, int64_t n, int64_t ld, int32_t wtype,
                        int32_t* labels, float* log_post, float* scores, void* stream) {
  nb_layout L;
  int rc = check_model(m, &L);
  if (rc) return rc;
  if (elem_bytes(xtype) == 0) return fail(NB_EINVAL, "unknown feature type");
  if (wtype != NB_W_F32 && wtype != NB_W_BF16) return fail(NB_EINVAL, "unknown table type");
  if (n < 0) return fail(NB_EINVAL, "n must be >= 0");
  if (!labels && !log_post && !scores) return fail(NB_EINVAL, "at least one output must be non-NULL");
  if (n == 0) return NB_OK;
  if (!x) return fail(NB_EINVAL, "x is NULL");
  if (ld < m->n_features) return fail(NB_EINVAL, "ld must be >= n_features");
  const int eb = elem_bytes(xtype);
  if ((ld * eb) % 4 != 0) return fail(NB_EINVAL, "row stride must be a multiple of 4 bytes");
  if ((reinterpret_cast<uintptr_t>(x) & 3) != 0) return fail(NB_EINVAL, "x must be 4-byte aligned");
  if ((log_post && (reinterpret_cast<uintptr_t>(log_post) & 7)) || (scores && (reinterpret_cast<uintptr_t>(scores) & 7)))
    return fail(NB_EINVAL, "log_post and scores must be 8-byte aligned");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (m->n_classes == 2) return launch_score2(m, L, x, xtype, n, ld, wtype, labels, log_post, scores, s);
  // BF16 tables with a full column tile of classes go to the matrix cores;
  // everything else (the FP32 plain path, fewer classes, int32 features) to
  // the vector ALUs
  if (wtype == NB_W_BF16 && m->n_classes >= 16 && xtype != NB_X_I32)
    return launch_scoreC_mfma(m, L, x, xtype, n, ld, labels, log_post, scores, s);
  return launch_scoreC_valu(m, L, x, xtype, n, ld, wtype, labels, log_post, scores, s);
}
