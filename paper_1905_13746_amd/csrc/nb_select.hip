// Per-group feature selection and feature gather on gfx950.
//
// Paper, section 3: each size group keeps its top-k opcodes, ranked by the
// difference between the malware and benign programs' normalised opcode
// occurrences; section 4: each group's model is trained and applied on those
// k features.
//
//   select_kernel  one workgroup per model.  Feature f's key is the exact
//                  integer |T_1f S_0 - T_0f S_1| (d_f scaled by S_0 S_1, at
//                  most 94 bits) shifted up 32 bits, with F - 1 - f in the
//                  low word: keys are distinct and a larger key is a better
//                  feature, an exact tie going to the lower index.  A radix
//                  select (16 passes of 8-bit digits, one LDS histogram per
//                  pass, the digit found by a wave scan) yields the k-th
//                  largest key; the features at or above it are written in
//                  ascending order by a ballot compaction.  Keys are
//                  recomputed from the counts (L2-resident) in every pass,
//                  so any F works with 1 KB of LDS.
//   expand_rows    the k-feature model widened to the full feature vector
//                  (its tables and rows at the selected features, zero
//                  elsewhere; a binary search of the ascending index list
//                  per feature), so a group's files are scored on their
//                  full rows in one pass.
//   gather_kernel  out[i][j] = x[i][idx[j]], HBM-bound: every row is read
//                  once with 16-byte loads and k elements are written.  Each
//                  wave stages units of consecutive rows, each loaded as one
//                  contiguous span from a 16-byte boundary, in its own LDS
//                  slice (the loads of its next two units in flight while
//                  the current one is gathered);
//                  each lane keeps the indices of its output positions
//                  (j = 256 q + 4 lane + e) in registers for the whole
//                  kernel, reads its four elements from LDS and writes them
//                  with one packed store; every load and store is issued
//                  unconditionally (absent lanes go out of the buffer
//                  range), so waiting for one unit never waits for the two
//                  behind it.  Rows longer than 8 KB, rows or outputs that
//                  are not dword aligned, and more than 2048 indices are
//                  gathered straight from global memory.
#include <algorithm>

#include "nb_device.hpp"
#include "nb_internal.hpp"

namespace nb {
namespace {

typedef unsigned __int128 u128;

// ------------------------------------------------------------------ select

constexpr int kSelectBatch = 64;  // models per launch (descriptors by value)

struct SelectDesc {
  const int32_t* counts;  // [2][F]
  const int64_t* sums;    // [2]
  int32_t* idx;           // [k] output
  int32_t F;
  int32_t pad;
};

struct SelectArgs {
  SelectDesc d[kSelectBatch];
  int32_t n;
  int32_t k;
};

__device__ __forceinline__ u128 select_key(const int32_t* __restrict__ counts, int F, int f, int64_t S0,
                                           int64_t S1) {
  const uint64_t t0 = (uint32_t)counts[f], t1 = (uint32_t)counts[F + f];
  u128 d;
  if (S0 == 0) {
    d = t1;
  } else if (S1 == 0) {
    d = t0;
  } else {
    const u128 a = (u128)t1 * (uint64_t)S0;
    const u128 b = (u128)t0 * (uint64_t)S1;
    d = a > b ? a - b : b - a;
  }
  return (d << 32) | (uint32_t)(F - 1 - f);
}

__global__ __launch_bounds__(256) void select_kernel(SelectArgs a) {
  const SelectDesc d = a.d[blockIdx.x];
  const int F = d.F, t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t S0 = d.sums[0], S1 = d.sums[1];
  __shared__ uint32_t hist[256];
  __shared__ uint32_t found[2];
  __shared__ uint32_t wcount[4];

  u128 prefix = 0, mask = 0;
  uint32_t rem = (uint32_t)a.k;  // rank of the wanted key among those matching prefix (1 = largest)
  for (int shift = 120; shift >= 0; shift -= 8) {
    hist[t] = 0;
    __syncthreads();
    for (int f = t; f < F; f += 256) {
      const u128 c = select_key(d.counts, F, f, S0, S1);
      if ((c & mask) == prefix) atomicAdd(&hist[(uint32_t)(c >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (w == 0) {
      // lane l holds digits 255 - 4l .. 252 - 4l (descending); an inclusive
      // scan from the top digit finds the bucket holding rank rem
      uint32_t h[4], s = 0;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        h[e] = hist[255 - 4 * lane - e];
        s += h[e];
      }
      uint32_t inc = s;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t v = __shfl_up(inc, o);
        if (lane >= o) inc += v;
      }
      const uint32_t exc = inc - s;
      if (exc < rem && rem <= inc) {
        uint32_t run = exc;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (run < rem && rem <= run + h[e]) {
            found[0] = (uint32_t)(255 - 4 * lane - e);
            found[1] = rem - run;
          }
          run += h[e];
        }
      }
    }
    __syncthreads();
    const uint32_t digit = found[0];
    rem = found[1];
    prefix |= (u128)digit << shift;
    mask |= (u128)255u << shift;
    __syncthreads();
  }

  // prefix is now the k-th largest key: exactly k features are >= it
  uint32_t base = 0;
  for (int f0 = 0; f0 < F; f0 += 256) {
    const int f = f0 + t;
    const bool sel = (f < F) && select_key(d.counts, F, f, S0, S1) >= prefix;
    const uint64_t bal = __ballot(sel);
    const uint32_t before = (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wcount[w] = (uint32_t)__popcll(bal);
    __syncthreads();
    uint32_t off = base;
    for (int i = 0; i < w; ++i) off += wcount[i];
    if (sel && off + before < (uint32_t)a.k) d.idx[off + before] = f;   // exactly k are selected
    base += wcount[0] + wcount[1] + wcount[2] + wcount[3];
    __syncthreads();
  }
}

// ------------------------------------------------------------------ gather

constexpr int kGatherWaves = 4;
constexpr int kGatherThreads = 64 * kGatherWaves;
constexpr int kRegQ = 8;               // indices held in registers: 4 * 64 * kRegQ = 2048
constexpr int kMaxStagedRow = 8192;    // bytes of the longest staged row (plus its lead)
// Bytes of a unit: the contiguous span of rows a wave stages at once (two
// units' loads in flight per wave; 8 KB measured faster than 4 KB for rows
// of 1000 to 5000 bytes); 8 KB for rows too long for a smaller unit.
#ifndef NB_GATHER_UNIT_KB
#define NB_GATHER_UNIT_KB 8
#endif
constexpr int kGatherUnitKB = NB_GATHER_UNIT_KB;
constexpr uint32_t kOutOfRange = 0x80000000u;  // buffer offset past any range: no access

struct GatherArgs {
  const uint8_t* x;
  int64_t ld_bytes;
  int64_t n;
  int64_t total_bytes;   // bytes the input buffer holds
  const int32_t* idx;
  uint8_t* out;
  int64_t ld_out_bytes;
  int32_t* status;
  int64_t nfast;         // leading units whose whole span lies inside the buffer
  int32_t F, k, row_bytes;
  int32_t out_vec;       // packed stores allowed (alignment)
};

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Index of output position j: idx[j] if in [0, F), else -1 (and bad).
__device__ __forceinline__ int32_t checked_index(const GatherArgs& a, int j, bool& bad) {
  if (j >= a.k) return -1;
  const int32_t v = a.idx[j];
  if (v < 0 || v >= a.F) {
    bad = true;
    return -1;
  }
  return v;
}

// ---- global-memory gather (rows longer than 8 KB, rows or outputs that are
// not dword aligned, more than 2048 indices): plain loads and stores.

template <int ES>
__device__ __forceinline__ void store4(const GatherArgs& a, int64_t r, int j0, const uint32_t (&v)[4]) {
  uint8_t* orow = a.out + r * a.ld_out_bytes;
  if (j0 + 3 < a.k && a.out_vec) {
    if (ES == 1) {
      const uint32_t w = v[0] | (v[1] << 8) | (v[2] << 16) | (v[3] << 24);
      __builtin_nontemporal_store(w, reinterpret_cast<uint32_t*>(orow + j0));
    } else {
      reinterpret_cast<dev::u32x4_a4*>(orow + 4 * (int64_t)j0)->v = dev::u32x4{v[0], v[1], v[2], v[3]};
    }
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if (j0 + e < a.k) {
        if (ES == 1) orow[j0 + e] = (uint8_t)v[e];
        else reinterpret_cast<uint32_t*>(orow)[j0 + e] = v[e];
      }
    }
  }
}

template <int ES>
__global__ __launch_bounds__(kGatherThreads) void gather_global_kernel(GatherArgs a) {
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  bool bad = false;
  const int64_t nw = (int64_t)gridDim.x * kGatherWaves;
  const int qn = (a.k + 255) >> 8;
  for (int64_t r = (int64_t)blockIdx.x * kGatherWaves + w; r < a.n; r += nw) {
    const uint8_t* row = a.x + r * a.ld_bytes;
    for (int q = 0; q < qn; ++q) {
      const int j0 = 256 * q + 4 * lane;
      uint32_t v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int32_t f = checked_index(a, j0 + e, bad);
        v[e] = f < 0 ? 0u : (ES == 1 ? (uint32_t)row[f] : reinterpret_cast<const uint32_t*>(row)[f]);
      }
      store4<ES>(a, r, j0, v);
    }
  }
  if (a.status && __ballot(bad) != 0ull && lane == 0) atomicOr(a.status, 1);
}

// ---- staged gather.  Every memory operation of a unit is issued
// unconditionally (absent lanes and rows use out-of-range buffer offsets or
// empty buffer ranges, which access nothing), so the number of operations
// in flight is known at compile time and waiting for one unit's loads does
// not wait for the units behind it.  The one exception is a uniform one:
// the single-element stores of a row's last partial group of outputs,
// issued only when k is not a multiple of 4.

// The four outputs j0 .. j0+3 of one lane for the row staged at `row`:
// one packed store where all four are present, three single-element stores
// for the row's last partial group when k is not a multiple of 4 (absent
// elements go out of range).
template <int ES>
__device__ __forceinline__ void emit4(__amdgpu_buffer_rsrc_t orsrc, const uint8_t* row, const int32_t (&o)[4],
                                      int j0, int k) {
  uint32_t v[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int32_t oe = o[e] < 0 ? 0 : o[e];
    const uint32_t x = (ES == 1) ? (uint32_t)row[oe] : *reinterpret_cast<const uint32_t*>(row + oe);
    v[e] = o[e] < 0 ? 0u : x;
  }
  const bool full = j0 + 3 < k;
  const uint32_t vo = full ? (uint32_t)(j0 * ES) : kOutOfRange;
  if (ES == 1) {
    __builtin_amdgcn_raw_buffer_store_b32(v[0] | (v[1] << 8) | (v[2] << 16) | (v[3] << 24), orsrc, (int)vo, 0,
                                          NB_STREAM_CPOL);
  } else {
    const dev::u32x4 q = {v[0], v[1], v[2], v[3]};
    __builtin_amdgcn_raw_buffer_store_b128(q, orsrc, (int)vo, 0, NB_STREAM_CPOL);
  }
  // a last group of one to three outputs exists only when k is not a
  // multiple of 4 (k is the same for every lane: a uniform branch); the
  // paper's k values are all multiples of 4
  if (k & 3) {
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      const uint32_t to = (!full && j0 + e < k) ? (uint32_t)((j0 + e) * ES) : kOutOfRange;
      if (ES == 1) __builtin_amdgcn_raw_buffer_store_b8((uint8_t)v[e], orsrc, (int)to, 0, NB_STREAM_CPOL);
      else __builtin_amdgcn_raw_buffer_store_b32(v[e], orsrc, (int)to, 0, NB_STREAM_CPOL);
    }
  }
}

// NL: 1 KB loads per unit; RW: rows per unit; Q: 256-index groups per lane.
// A unit is RW consecutive rows, loaded as one contiguous span from a
// 16-byte boundary (relative to x) with 16-byte loads; row s of unit u
// starts at byte (u RW ld) mod 16 + s ld of the stage.  Wave w takes the
// units w, w + nw, ... below nfast with the loads of its next two units in
// flight (three register buffers), then the last units (whose span reaches
// the end of the buffer) with bytewise guarded loads.
template <int ES, int NL, int RW, int Q>
__global__ __launch_bounds__(kGatherThreads) void gather_kernel(GatherArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  bool bad = false;

  // byte offsets (in a row) of this lane's outputs, -1 = none
  int32_t off[Q][4];
#pragma unroll
  for (int q = 0; q < Q; ++q)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int32_t f = checked_index(a, 256 * q + 4 * lane + e, bad);
      off[q][e] = f < 0 ? -1 : f * ES;
    }

  const int64_t gw = (int64_t)blockIdx.x * kGatherWaves + w;
  const int64_t nw = (int64_t)gridDim.x * kGatherWaves;
  uint8_t* buf = lds + w * (NL * 1024);
  const int64_t nunits = (a.n + RW - 1) / RW;
  const int64_t mine = gw < a.nfast ? (a.nfast - 1 - gw) / nw + 1 : 0;

  struct Unit {
    int64_t r0, arel;
    int32_t lead, span;
  };
  auto unit = [&](int64_t u) {
    Unit v;
    v.r0 = u * RW;
    const int64_t rows = min((int64_t)RW, a.n - v.r0);
    const int64_t rel = v.r0 * a.ld_bytes;
    v.arel = rel & ~(int64_t)15;
    v.lead = (int32_t)(rel - v.arel);
    v.span = v.lead + (int32_t)((rows - 1) * a.ld_bytes) + a.row_bytes;
    return v;
  };
  // loads of this wave's t-th fast unit (none when t >= mine)
  auto issue = [&](int64_t t, dev::u32x4 (&dst)[NL]) {
    const bool valid = t < mine;
    const Unit u = unit(gw + (valid ? t : 0) * nw);
    const auto rsrc = dev::make_rsrc(a.x + u.arel, valid ? a.total_bytes - u.arel : 0);
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const uint32_t p = (uint32_t)(i * 64 + lane) * 16u;
      dst[i] = dev::buffer_load16(rsrc, p < (uint32_t)u.span ? p : kOutOfRange);
    }
    __builtin_amdgcn_sched_barrier(0);
  };
  auto consume = [&](int64_t ui, const dev::u32x4 (&src)[NL]) {
    const Unit u = unit(ui);
    wave_lds_sync();  // the previous unit's LDS reads are done
#pragma unroll
    for (int i = 0; i < NL; ++i) *reinterpret_cast<dev::u32x4*>(buf + (i * 64 + lane) * 16) = src[i];
    wave_lds_sync();
#pragma unroll
    for (int s = 0; s < RW; ++s) {
      const int64_t r = u.r0 + s;
      const auto orsrc = dev::make_rsrc(a.out + r * a.ld_out_bytes, r < a.n ? (int64_t)a.k * ES : 0);
      const uint8_t* row = buf + u.lead + s * (int32_t)a.ld_bytes;
#pragma unroll
      for (int q = 0; q < Q; ++q) emit4<ES>(orsrc, row, off[q], 256 * q + 4 * lane, a.k);
    }
  };
  if (mine > 0) {
    dev::u32x4 b0[NL], b1[NL], b2[NL];
    issue(0, b0);
    issue(1, b1);
    for (int64_t t = 0;; t += 3) {
      issue(t + 2, b2);
      consume(gw + t * nw, b0);
      if (t + 1 >= mine) break;
      issue(t + 3, b0);
      consume(gw + (t + 1) * nw, b1);
      if (t + 2 >= mine) break;
      issue(t + 4, b1);
      consume(gw + (t + 2) * nw, b2);
      if (t + 3 >= mine) break;
    }
  }
  // the last units: bytes past the end of the buffer read as 0
  for (int64_t ui = a.nfast + gw; ui < nunits; ui += nw) {
    const Unit u = unit(ui);
    const int64_t avail = a.total_bytes - u.arel;
    dev::u32x4 b[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const int p = (i * 64 + lane) * 16;
      b[i] = (p < u.span) ? dev::load16_guarded(a.x + u.arel + p, avail - p) : dev::u32x4{0u, 0u, 0u, 0u};
    }
    consume(ui, b);
  }
  if (a.status && __ballot(bad) != 0ull && lane == 0) atomicOr(a.status, 1);
}

// Index groups held in registers for k outputs: 1, 2 or 8 (0: more than
// 2048, gathered from global memory).
int gather_q(int32_t k) { return k <= 256 ? 1 : (k <= 512 ? 2 : (k <= 4 * 64 * kRegQ ? 8 : 0)); }

template <int ES, int NL, int RW>
const void* pick_q(int q) {
  switch (q) {
    case 1: return reinterpret_cast<const void*>(gather_kernel<ES, NL, RW, 1>);
    case 2: return reinterpret_cast<const void*>(gather_kernel<ES, NL, RW, 2>);
    default: return reinterpret_cast<const void*>(gather_kernel<ES, NL, RW, 8>);
  }
}

// Staged variants: (unit KB, rows per unit) = (kGatherUnitKB, 1/2/4/8) or (8, 1).
template <int ES>
const void* pick_gather(int nl, int rw, int q) {
  if (nl == 8 && kGatherUnitKB != 8) return pick_q<ES, 8, 1>(q);
  switch (rw) {
    case 8: return pick_q<ES, kGatherUnitKB, 8>(q);
    case 4: return pick_q<ES, kGatherUnitKB, 4>(q);
    case 2: return pick_q<ES, kGatherUnitKB, 2>(q);
    default: return pick_q<ES, kGatherUnitKB, 1>(q);
  }
}

// Span of unit u (rows u*rw ..) from its 16-byte boundary, rounded up to
// whole 16-byte loads: end offset relative to x.
int64_t unit_end(int64_t u, int64_t rw, int64_t n, int64_t ld_bytes, int64_t row_bytes) {
  const int64_t r0 = u * rw;
  const int64_t rows = std::min(rw, n - r0);
  const int64_t rel = r0 * ld_bytes;
  const int64_t arel = rel & ~(int64_t)15;
  const int64_t span = (rel - arel) + (rows - 1) * ld_bytes + row_bytes;
  return arel + ((span + 15) & ~(int64_t)15);
}

}  // namespace
}  // namespace nb

using namespace nb;

extern "C" {

int nb_select_features(const nb_model* models, int32_t n_models, int32_t k, int32_t* idx, int64_t ld_idx,
                       void* stream) {
  if (n_models < 1 || !models) return fail(NB_EINVAL, "need at least one model");
  if (!idx) return fail(NB_EINVAL, "idx must be non-NULL");
  if (k < 1) return fail(NB_EINVAL, "k must be >= 1");
  if (ld_idx < k) return fail(NB_EINVAL, "ld_idx must be >= k");
  std::vector<SelectDesc> desc((size_t)n_models);
  for (int32_t m = 0; m < n_models; ++m) {
    nb_layout L;
    const int rc = check_model(&models[m], &L);
    if (rc) return rc;
    if (models[m].n_classes != 2)
      return fail(NB_EINVAL, "model " + std::to_string(m) + ": selection needs a two-class model");
    if (!models[m].trained) return fail(NB_EINVAL, "model " + std::to_string(m) + " is not trained");
    if (k > models[m].n_features)
      return fail(NB_EINVAL, "k exceeds the feature count of model " + std::to_string(m));
    const uint8_t* base = static_cast<const uint8_t*>(models[m].dev);
    desc[m].counts = reinterpret_cast<const int32_t*>(base + L.off_counts);
    desc[m].sums = reinterpret_cast<const int64_t*>(base + L.off_class_sums);
    desc[m].idx = idx + (int64_t)m * ld_idx;
    desc[m].F = models[m].n_features;
    desc[m].pad = 0;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  for (int32_t m0 = 0; m0 < n_models; m0 += kSelectBatch) {
    SelectArgs a;
    a.n = std::min<int32_t>(kSelectBatch, n_models - m0);
    a.k = k;
    for (int i = 0; i < kSelectBatch; ++i) a.d[i] = desc[(size_t)std::min<int32_t>(m0 + i, n_models - 1)];
    hipLaunchKernelGGL(select_kernel, dim3((unsigned)a.n), dim3(256), 0, s, a);
    NB_HIP_CHECK(hipGetLastError());
  }
  return NB_OK;
}

int nb_gather_features(const void* x, int32_t xtype, int64_t n, int32_t F, int64_t ld, const int32_t* idx,
                       int32_t k, void* out, int64_t ld_out, int32_t* status, void* stream) {
  const int es = elem_bytes(xtype);
  if (es == 0) return fail(NB_EINVAL, "unknown feature type");
  if (F < 1 || F > kMaxFeatures) return fail(NB_EINVAL, "n_features out of range [1, 2^20]");
  if (k < 1 || k > kMaxFeatures) return fail(NB_EINVAL, "k out of range [1, 2^20]");
  if (n < 0) return fail(NB_EINVAL, "n must be >= 0");
  if (ld < F) return fail(NB_EINVAL, "ld must be >= n_features");
  if (ld_out < k) return fail(NB_EINVAL, "ld_out must be >= k");
  if (n == 0) return NB_OK;
  if (!x || !idx || !out) return fail(NB_EINVAL, "x, idx and out must be non-NULL");
  if (es == 4 && (((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(out)) & 3) != 0))
    return fail(NB_EINVAL, "int32 features must be 4-byte aligned");
  if ((reinterpret_cast<uintptr_t>(idx) & 3) != 0) return fail(NB_EINVAL, "idx must be 4-byte aligned");

  GatherArgs a;
  a.x = static_cast<const uint8_t*>(x);
  a.ld_bytes = ld * es;
  a.n = n;
  a.total_bytes = ((n - 1) * ld + F) * (int64_t)es;
  a.idx = idx;
  a.out = static_cast<uint8_t*>(out);
  a.ld_out_bytes = ld_out * es;
  a.status = status;
  a.F = F;
  a.k = k;
  a.row_bytes = F * es;
  a.out_vec = ((reinterpret_cast<uintptr_t>(out) & 3) == 0 && (a.ld_out_bytes & 3) == 0) ? 1 : 0;
  a.nfast = 0;

  // Staged when rows (plus up to 15 lead bytes) fit 8 KB, input rows and
  // outputs are dword aligned and the indices fit in registers; units of
  // kGatherUnitKB KB (8 KB for longer rows) holding 1, 2, 4 or 8 rows.
  const bool aligned = ((reinterpret_cast<uintptr_t>(x) & 3) == 0) && ((a.ld_bytes & 3) == 0) && a.out_vec;
  const int q = gather_q(k);
  int nl = 0;
  if (aligned && q > 0 && a.row_bytes + 15 <= kMaxStagedRow)
    nl = (a.row_bytes + 15 <= kGatherUnitKB * 1024) ? kGatherUnitKB : 8;
  const void* fn;
  size_t lds = 0;
  int64_t rw = 1;
  if (nl) {
    const int64_t pad = a.ld_bytes - a.row_bytes;
    if (nl == kGatherUnitKB && pad * 8 <= a.ld_bytes) {
      // the most rows whose span fits the unit
      for (int64_t c = 8; c > 1; c /= 2)
        if ((c - 1) * a.ld_bytes + a.row_bytes + 15 <= (int64_t)nl * 1024) {
          rw = c;
          break;
        }
    }
    lds = (size_t)kGatherWaves * nl * 1024;
    // no fewer units than resident waves
    const void* f1 = (es == 1) ? pick_gather<1>(nl, (int)rw, q) : pick_gather<4>(nl, (int)rw, q);
    const int64_t waves = (int64_t)resident_per_cu(f1, kGatherThreads, lds) * device_cu_count() * kGatherWaves;
    while (rw > 1 && (n + rw - 1) / rw < waves) rw /= 2;
    fn = (es == 1) ? pick_gather<1>(nl, (int)rw, q) : pick_gather<4>(nl, (int)rw, q);
    // units whose whole rounded span lies inside the buffer (all but the last few)
    const int64_t nunits = (n + rw - 1) / rw;
    int64_t nf = nunits;
    while (nf > 0 && nunits - nf < 64 && unit_end(nf - 1, rw, n, a.ld_bytes, a.row_bytes) > a.total_bytes) --nf;
    if (nf > 0 && unit_end(nf - 1, rw, n, a.ld_bytes, a.row_bytes) > a.total_bytes) nf = 0;
    a.nfast = nf;
  } else {
    fn = (es == 1) ? reinterpret_cast<const void*>(gather_global_kernel<1>)
                   : reinterpret_cast<const void*>(gather_global_kernel<4>);
  }
  const int64_t cap_wg = (int64_t)resident_per_cu(fn, kGatherThreads, lds) * device_cu_count();
  const int64_t units = (n + rw - 1) / rw;
  const int64_t need = (units + kGatherWaves - 1) / kGatherWaves;
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min(need, cap_wg));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  void* args[] = {&a};
  NB_HIP_CHECK(hipLaunchKernel(fn, dim3(grid), dim3(kGatherThreads), args, lds, s));
  return NB_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ expand
namespace nb {
namespace {

struct ExpandArgs {
  const uint8_t* kb;    // the k-feature model's buffer
  uint8_t* ob;          // the full model's buffer
  const int32_t* idx;
  nb_layout LK, LO;
  int32_t C, k, F, kind;
};

// Position of feature f in the ascending list idx[0..k) (or -1).
__device__ __forceinline__ int find_selected(const int32_t* __restrict__ idx, int k, int f) {
  int lo = 0, hi = k - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const int v = idx[mid];
    if (v == f) return mid;
    if (v < f) lo = mid + 1;
    else hi = mid - 1;
  }
  return -1;
}

// Every feature f of the full model: km's tables and scoring rows at its
// selected position, zero elsewhere.  grid Fp / 256.
__global__ __launch_bounds__(256) void expand_rows(ExpandArgs a) {
  const int f = blockIdx.x * 256 + threadIdx.x;
  const int Fp = a.LO.padded_features, Fk = a.LK.padded_features;
  if (f >= Fp) return;
  const int j = (f < a.F) ? find_selected(a.idx, a.k, f) : -1;
  const int P = a.LO.form_rows;
  for (int r = 0; r <= P; ++r) {
    reinterpret_cast<float*>(a.ob + a.LO.off_form_f32)[(int64_t)r * Fp + f] =
        j >= 0 ? reinterpret_cast<const float*>(a.kb + a.LK.off_form_f32)[(int64_t)r * Fk + j] : 0.0f;
    reinterpret_cast<uint16_t*>(a.ob + a.LO.off_form_bf16)[(int64_t)r * Fp + f] =
        j >= 0 ? reinterpret_cast<const uint16_t*>(a.kb + a.LK.off_form_bf16)[(int64_t)r * Fk + j] : (uint16_t)0;
  }
  if (f < a.F) {
    for (int c = 0; c < a.C; ++c) {
      const int64_t o = (int64_t)c * a.F + f, i = (int64_t)c * a.k + j;
      reinterpret_cast<int32_t*>(a.ob + a.LO.off_counts)[o] =
          j >= 0 ? reinterpret_cast<const int32_t*>(a.kb + a.LK.off_counts)[i] : 0;
      reinterpret_cast<double*>(a.ob + a.LO.off_log_theta)[o] =
          j >= 0 ? reinterpret_cast<const double*>(a.kb + a.LK.off_log_theta)[i] : 0.0;
      reinterpret_cast<double*>(a.ob + a.LO.off_log_1m_theta)[o] =
          j >= 0 ? reinterpret_cast<const double*>(a.kb + a.LK.off_log_1m_theta)[i] : 0.0;
      reinterpret_cast<double*>(a.ob + a.LO.off_weight)[o] =
          j >= 0 ? reinterpret_cast<const double*>(a.kb + a.LK.off_weight)[i] : 0.0;
    }
  }
}

// Class totals, sums and biases copied; the index list checked (strictly
// ascending, inside [0, F)); the status word.  One workgroup.
__global__ __launch_bounds__(256) void expand_finish(ExpandArgs a) {
  bool bad = false;
  for (int j = threadIdx.x; j < a.k; j += 256) {
    const int32_t v = a.idx[j];
    if (v < 0 || v >= a.F || (j + 1 < a.k && a.idx[j + 1] <= v)) bad = true;
  }
  const int any_bad = __syncthreads_or(bad);
  const int t = threadIdx.x;
  if (t < a.C) {
    reinterpret_cast<int64_t*>(a.ob + a.LO.off_class_totals)[t] =
        reinterpret_cast<const int64_t*>(a.kb + a.LK.off_class_totals)[t];
    reinterpret_cast<int64_t*>(a.ob + a.LO.off_class_sums)[t] =
        reinterpret_cast<const int64_t*>(a.kb + a.LK.off_class_sums)[t];
    reinterpret_cast<double*>(a.ob + a.LO.off_bias)[t] = reinterpret_cast<const double*>(a.kb + a.LK.off_bias)[t];
  }
  for (int r = t; r <= a.LO.form_rows; r += 256)
    reinterpret_cast<float*>(a.ob + a.LO.off_form_bias)[r] =
        reinterpret_cast<const float*>(a.kb + a.LK.off_form_bias)[r];
  if (t == 0) {
    int32_t* st = reinterpret_cast<int32_t*>(a.ob + a.LO.off_status);
    st[kStatusFlags] = any_bad ? kFlagBadIndex : 0;
    st[kStatusTrained] = any_bad ? 0 : 1;
    st[2] = 0;
    st[3] = 0;
  }
}

}  // namespace
}  // namespace nb

extern "C" int nb_model_expand(const nb_model* km, const int32_t* idx, nb_model* out, int32_t flags, void* stream) {
  nb_layout LK, LO;
  int rc = check_model(km, &LK);
  if (rc) return rc;
  if (!km->trained) return fail(NB_EINVAL, "the k-feature model is not trained");
  if (km->kind == NB_GAUSSIAN) return fail(NB_EINVAL, "expansion takes multinomial and Bernoulli models");
  if (!out) return fail(NB_EINVAL, "out is NULL");
  if (out->kind != km->kind || out->n_classes != km->n_classes)
    return fail(NB_EINVAL, "out must have the kind and class count of the k-feature model");
  rc = check_model(out, &LO);
  if (rc) return rc;
  if (out->n_features < km->n_features) return fail(NB_EINVAL, "out->n_features must be >= k");
  if (out->dev == km->dev) return fail(NB_EINVAL, "out must have its own buffer");
  if (!idx) return fail(NB_EINVAL, "idx must be non-NULL");
  out->trained = 0;
  ExpandArgs a;
  a.kb = static_cast<const uint8_t*>(km->dev);
  a.ob = static_cast<uint8_t*>(out->dev);
  a.idx = idx;
  a.LK = LK;
  a.LO = LO;
  a.C = km->n_classes;
  a.k = km->n_features;
  a.F = out->n_features;
  a.kind = km->kind;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(expand_rows, dim3((unsigned)(LO.padded_features / 256)), dim3(256), 0, s, a);
  NB_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(expand_finish, dim3(1), dim3(256), 0, s, a);
  NB_HIP_CHECK(hipGetLastError());
  if (flags & NB_TRAIN_ASYNC) return NB_OK;
  return nb_model_status(out, stream);
}
