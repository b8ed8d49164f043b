// Naive Bayes training on gfx950: exact per-class feature counts, the FP64
// Laplace-smoothed log table and the rounded scoring rows.
//
// Paper, section 4: a model is trained per size group on labelled opcode
// occurrence vectors.  The method's training is a pair of reductions,
//   N_c  = #{i : y_i = c},
//   T_cf = sum_{i : y_i = c} x_if      (multinomial)
//   D_cf = #{i : y_i = c, x_if > 0}    (Bernoulli),
// followed by C*F logarithms.  The reductions are HBM-bound (one pass over
// the training matrix); the logarithms are negligible.
//
// Kernel pipeline (one stream).  Error flags travel as plain per-workgroup
// words in the workspace and are OR-ed down the pipeline; form_rows writes
// the model's status word once, so no kernel has to clear it first.
//   count_kernel  grid (slot, class, chunk): each workgroup streams the rows
//                 of ONE class inside its slot of rows and ONE 1024-feature
//                 chunk.  Labels are read 64 at a time and compacted with a
//                 wave ballot, so a row is loaded only by the workgroup of its
//                 class; with three or more classes a wave first collects the
//                 matching rows of several 64-row windows in a list in LDS,
//                 so that its row loads still go out in full batches.  Byte counts accumulate in packed 16-bit register
//                 lanes (two features per 32-bit add), flushed to 32-bit every
//                 <= 256 rows; four waves then combine in LDS and write one
//                 int64 partial per (slot, class, feature) to the workspace.
//   reduce_counts first level of the partial sums, spread over
//                 (feature group, class, slot group) workgroups.
//   class_tables  one workgroup per class: the last level of the sums
//                 (integer: exact and order-free), the int32 range check,
//                 T/D, N_c, S_c, then the FP64 log theta /
//                 log(1 - theta) / weights and the bias, with a fixed-order
//                 tree reduction (deterministic).
//   form_rows     the scoring rows (log-odds / class-centred + aux) in FP64,
//                 rounded once to FP32 and to BF16.
#include <algorithm>
#include <cmath>

#include "nb_device.hpp"
#include "nb_internal.hpp"

namespace nb {
namespace {

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kSeg = 16;                  // features per lane per chunk
constexpr int kChunk = 64 * kSeg;         // features per chunk (one wave)
// rows loaded together by a wave: sixteen 16-byte loads in flight for byte
// features, eight rows of four loads for int32 features
template <int XT>
constexpr int batch_rows() { return XT == NB_X_I32 ? 8 : 16; }
constexpr int64_t kMinRowsPerSlot = 512;

struct CountArgs {
  const uint8_t* x;
  int64_t ld_bytes;
  int64_t n;
  int64_t total_bytes;     // bytes the caller's buffer is known to hold
  const int32_t* y;
  int64_t rows_per_slot;
  int64_t* part;           // [S][C][Fp]
  int64_t* nc_part;        // [S][C]
  int32_t* flag_part;      // [S][C][chunks] error flags of each workgroup
  int64_t* zero_words;     // n_zero words cleared by workgroup (0, 0, 0), or NULL
  int32_t F, C, Fp, n_zero;
};

// SQ: sums of squares x^2 instead of counts (the Gaussian variant's second
// moment): 32-bit per-feature lane sums for byte features (flushed to int64
// before they can wrap), int64 for int32 features (values of 65536 or more
// are flagged: their squares could overflow the exact int64 sums).
//
// WIN: 64-row label windows whose matching rows are loaded together.  With
// WIN = 1 the rows of a batch come straight from the window's ballot mask;
// with more windows (many classes: a 64-row window holds about 64 / C rows of
// one class) each wave writes the relative indices of its matching rows to a
// list in LDS and loads them kBatch at a time, so a batch is short only at the
// end of a list instead of in every window.
template <int XT, bool BIN, bool SQ = false, int WIN = 1>
__global__ __launch_bounds__(kThreads) void count_kernel(CountArgs a) {
  constexpr int EB = (XT == NB_X_I32) ? 4 : 1;   // bytes per feature
  constexpr int NV = EB;                          // 16-byte vectors per lane per row
  constexpr int kBatch = batch_rows<XT>();
  const int slot = blockIdx.x, cls = blockIdx.y, ch = blockIdx.z;
  // wave-uniform (readfirstlane): row ranges and buffer descriptors derived
  // from it then live in scalar registers
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

  // the class sums reduce_counts accumulates start from zero (the kernels
  // run in stream order)
  if (a.zero_words && slot == 0 && cls == 0 && ch == 0 && (int)threadIdx.x < a.n_zero) a.zero_words[threadIdx.x] = 0;
  const int64_t r_begin = (int64_t)slot * a.rows_per_slot;
  const int64_t r_end = min(a.n, r_begin + a.rows_per_slot);
  // four contiguous sub-ranges, 64-row aligned
  const int64_t per = ((r_end - r_begin + kWaves - 1) / kWaves + 63) / 64 * 64;
  const int64_t w_begin = min(r_end, r_begin + wave * per);
  const int64_t w_end = min(r_end, w_begin + per);

  const int f0 = ch * kChunk + lane * kSeg;       // this lane's first feature
  const int64_t col = (int64_t)f0 * EB;
  const int64_t chunk_end = (int64_t)min(a.Fp, (ch + 1) * kChunk) * EB;

  // byte features: packed 16-bit lanes (lo: bytes 0,2; hi: bytes 1,3 of each dword)
  uint32_t lo[4] = {0, 0, 0, 0}, hi[4] = {0, 0, 0, 0};
  uint32_t sq32[SQ ? kSeg : 1];
#pragma unroll
  for (int e = 0; e < (SQ ? kSeg : 1); ++e) sq32[e] = 0;
  int64_t acc[kSeg];
#pragma unroll
  for (int e = 0; e < kSeg; ++e) acc[e] = 0;
  int packed_rows = 0;
  int64_t matched = 0;
  bool bad_label = false, negative = false, too_large = false;

  auto flush = [&]() {
    if (SQ) {
#pragma unroll
      for (int e = 0; e < (SQ ? kSeg : 1); ++e) {
        acc[e] += sq32[e];
        sq32[e] = 0;
      }
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        acc[4 * k + 0] += lo[k] & 0xFFFFu;
        acc[4 * k + 2] += lo[k] >> 16;
        acc[4 * k + 1] += hi[k] & 0xFFFFu;
        acc[4 * k + 3] += hi[k] >> 16;
        lo[k] = 0;
        hi[k] = 0;
      }
    }
    packed_rows = 0;
  };

  // Cache policy of the window loads.  Two classes (WIN = 1): default, so
  // that a cache line shared by neighbouring rows of different classes, which
  // the two classes' workgroups load, is fetched from HBM once (their
  // workgroups sit on the same XCD) -- 1000-byte rows share a line at every
  // row boundary; non-temporal (nothing to share) with more classes, where
  // default caching was slower.
  constexpr int kCpol = (WIN == 1) ? 0 : NB_STREAM_CPOL;
  auto load_window = [&](__amdgpu_buffer_rsrc_t r, uint32_t off) {
    const auto q = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, kCpol);
    return dev::u32x4{(uint32_t)q[0], (uint32_t)q[1], (uint32_t)q[2], (uint32_t)q[3]};
  };
  // the combine buffer of the four waves (after the row loop) and the
  // per-wave row lists (inside it) share one LDS allocation
  constexpr int kListRows = 64 * WIN;
  static_assert(kWaves * kListRows * 4 <= (kWaves - 1) * kSeg * 64 * 8, "row lists exceed the shared buffer");
  __shared__ __align__(16) int64_t red[kWaves - 1][kSeg][64];
  uint32_t* const lst = reinterpret_cast<uint32_t*>(&red[0][0][0]) + wave * kListRows;

  for (int64_t base = w_begin; base < w_end; base += kListRows) {
    uint64_t mask = 0;   // WIN == 1: the window's matching rows
    int total = 0;       // WIN > 1: rows in this wave's list
#pragma unroll
    for (int j = 0; j < WIN; ++j) {
      const int64_t r = base + 64 * j + lane;
      const int lab = (r < w_end) ? a.y[r] : -1;
      if (r < w_end && (lab < 0 || lab >= a.C)) bad_label = true;
      const uint64_t m = __ballot(lab == cls);
      matched += __popcll(m);
      if (WIN == 1) {
        mask = m;
      } else {
        const int pos = total + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                               __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        if (lab == cls) lst[pos] = (uint32_t)(64 * j + lane);
        total += __popcll(m);
      }
    }
    // the list is written and read by the same wave, in order
    if (WIN > 1) __builtin_amdgcn_wave_barrier();
    // every row of the windows (their chunk) lies inside the buffer
    const int64_t last = min(base + kListRows, w_end) - 1;
    const bool window_fast =
        last * a.ld_bytes + chunk_end <= a.total_bytes && kListRows * a.ld_bytes < ((int64_t)1 << 31);
    const auto wrsrc = dev::make_rsrc(a.x + base * a.ld_bytes, a.total_bytes - base * a.ld_bytes);
    for (int b = 0; WIN == 1 ? mask != 0 : b < total; b += kBatch) {
      int64_t rows[kBatch];
      int cnt = 0;
      if (WIN == 1) {
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
          if (mask) {
            const int idx = __ffsll((unsigned long long)mask) - 1;
            mask &= mask - 1;
            rows[k] = base + idx;
            ++cnt;
          } else {
            rows[k] = -1;
          }
        }
      } else {
        // b is a multiple of kBatch: four aligned 16-byte reads per 16 rows
        cnt = min(kBatch, total - b);
        uint32_t rel[kBatch];
#pragma unroll
        for (int k = 0; k < kBatch; k += 4) {
          const uint4 q4 = *reinterpret_cast<const uint4*>(lst + b + k);
          rel[k] = q4.x;
          rel[k + 1] = q4.y;
          rel[k + 2] = q4.z;
          rel[k + 3] = q4.w;
        }
#pragma unroll
        for (int k = 0; k < kBatch; ++k) rows[k] = (k < cnt) ? base + rel[k] : -1;
      }
      dev::u32x4 v[kBatch][NV];
      if (window_fast) {
        // every row of the window is in bounds: one descriptor for the
        // window, all loads issued unconditionally (slots past cnt re-read
        // the batch's first row and are zeroed afterwards)
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
          const uint32_t ro = (uint32_t)((k < cnt ? rows[k] : rows[0]) - base) * (uint32_t)a.ld_bytes;
#pragma unroll
          for (int q = 0; q < NV; ++q) v[k][q] = load_window(wrsrc, ro + (uint32_t)col + 16 * q);
        }
#pragma unroll
        for (int k = 0; k < kBatch; ++k)
#pragma unroll
          for (int q = 0; q < NV; ++q)
            if (k >= cnt) v[k][q] = dev::u32x4{0u, 0u, 0u, 0u};
      } else {
#pragma unroll
      for (int k = 0; k < kBatch; ++k) {
#pragma unroll
        for (int q = 0; q < NV; ++q) v[k][q] = dev::u32x4{0u, 0u, 0u, 0u};
        if (rows[k] >= 0) {
          const int64_t row_off = rows[k] * a.ld_bytes;
          const uint8_t* p = a.x + row_off + col;
          if (row_off + chunk_end <= a.total_bytes) {
            // streaming, non-temporal loads through a per-row buffer resource
            const auto rsrc = dev::make_rsrc(a.x + row_off, a.total_bytes - row_off);
#pragma unroll
            for (int q = 0; q < NV; ++q) v[k][q] = dev::buffer_load16(rsrc, (uint32_t)col + 16 * q);
          } else {
#pragma unroll
            for (int q = 0; q < NV; ++q)
              v[k][q] = dev::load16_guarded(p + 16 * q, a.total_bytes - (row_off + col + 16 * q));
          }
        }
      }
      }
#pragma unroll
      for (int k = 0; k < kBatch; ++k) {
        if (XT == NB_X_I32) {
#pragma unroll
          for (int q = 0; q < NV; ++q) {
#pragma unroll
            for (int d = 0; d < 4; ++d) {
              const int e = 4 * q + d;
              const int32_t val = (int32_t)v[k][q][d];
              const bool valid = (f0 + e) < a.F;
              if (valid && val < 0) negative = true;
              if (SQ && valid && val >= 65536) too_large = true;
              if (valid) acc[e] += SQ ? (int64_t)val * val : (BIN ? (int64_t)(val > 0) : (int64_t)val);
            }
          }
        } else if (SQ) {
#pragma unroll
          for (int d = 0; d < 4; ++d) {
            const uint32_t w = v[k][0][d];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
              const uint32_t x = (w >> (8 * b)) & 0xFFu;
              sq32[(4 * d + b) % (SQ ? kSeg : 1)] += x * x;
            }
          }
        } else {
#pragma unroll
          for (int d = 0; d < 4; ++d) {
            const uint32_t w = v[k][0][d];
            uint32_t l = w & 0x00FF00FFu, h = (w >> 8) & 0x00FF00FFu;
            if (BIN) {   // presence: (b + 255) has bit 8 set iff b >= 1
              l = ((l + 0x00FF00FFu) >> 8) & 0x00010001u;
              h = ((h + 0x00FF00FFu) >> 8) & 0x00010001u;
            }
            lo[d] += l;
            hi[d] += h;
          }
        }
      }
      if (XT != NB_X_I32) {
        // packed 16-bit counts hold 256 rows; 32-bit square sums 66,051
        packed_rows += cnt;
        if (packed_rows > (SQ ? 65536 : 256) - kBatch) flush();
      }
    }
    // this list's reads are done before the next windows overwrite it
    if (WIN > 1) __builtin_amdgcn_wave_barrier();
  }
  if (XT != NB_X_I32) flush();

  {
    const int any_bad = __syncthreads_or(bad_label && cls == 0 && ch == 0);
    const int any_neg = __syncthreads_or(negative);
    const int any_big = __syncthreads_or(too_large);
    if (threadIdx.x == 0)
      a.flag_part[((int64_t)slot * a.C + cls) * gridDim.z + ch] =
          (any_bad ? kFlagBadLabel : 0) | (any_neg ? kFlagNegative : 0) | (any_big ? kFlagOverflow : 0);
  }

  // combine the four waves in LDS, then one partial row per workgroup (the
  // buffer held the row lists: the flag reductions above are workgroup
  // barriers, so every wave is past its loop)
  __shared__ int64_t red_m[kWaves];
  if (wave > 0) {
#pragma unroll
    for (int e = 0; e < kSeg; ++e) red[wave - 1][e][lane] = acc[e];
  }
  if (lane == 0) red_m[wave] = matched;
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int w = 0; w < kWaves - 1; ++w)
#pragma unroll
      for (int e = 0; e < kSeg; ++e) acc[e] += red[w][e][lane];
    int64_t* dst = a.part + ((int64_t)slot * a.C + cls) * a.Fp + f0;
#pragma unroll
    for (int e = 0; e < kSeg; ++e) dst[e] = acc[e];
    if (ch == 0 && lane == 0)
      a.nc_part[(int64_t)slot * a.C + cls] = red_m[0] + red_m[1] + red_m[2] + red_m[3];
  }
}

// First-level reduction of the per-slot partials: grid (ceil(F/64), C, RS),
// 4 slot lanes x 64 features per workgroup; writes RS second-level partials.
constexpr int kReduceSplit = 8;

// csum (or NULL): [RS][C] shares of S_c accumulated with integer atomics
// (exact, so the order of the additions does not matter; one word per split
// keeps the workgroups adding to one word few), then one word holding the OR
// of the count kernel's n_flags flag words (an atomic OR only where a flag is
// set); the count kernel cleared them.
__global__ __launch_bounds__(256) void reduce_counts(const int64_t* __restrict__ part,
                                                    const int64_t* __restrict__ nc_part, int S, int C,
                                                    int F, int Fp, int64_t* __restrict__ part2,
                                                    int64_t* __restrict__ nc2, int64_t* __restrict__ csum,
                                                    const int32_t* __restrict__ flag_part, int n_flags) {
  const int c = blockIdx.y, rs = blockIdx.z, RS = gridDim.z;
  const int fl = threadIdx.x & 63, sg = threadIdx.x >> 6;
  if (csum) {
    const int64_t nthreads = (int64_t)gridDim.x * gridDim.y * gridDim.z * 256;
    int32_t bits = 0;
    for (int64_t i = (((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x) * 256 + threadIdx.x;
         i < n_flags; i += nthreads)
      bits |= flag_part[i];
    if (bits) atomicOr(reinterpret_cast<int*>(csum + (int64_t)RS * C), bits);
  }
  const int f = blockIdx.x * 64 + fl;
  int64_t s = 0, m = 0;
  const int stride = 4 * RS;
  if (f < F) {
    int k = rs * 4 + sg;
    // sixteen partials in flight per lane, then their sum
    for (; k < S; k += 16 * stride) {
      int64_t v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int kk = k + u * stride;
        v[u] = (kk < S) ? part[((int64_t)kk * C + c) * Fp + f] : 0;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) s += v[u];
    }
  }
  if (blockIdx.x == 0) {     // class totals: spread over the 64 lanes, then a wave sum
    for (int k = rs * 4 + sg + fl * stride; k < S; k += 64 * stride) m += nc_part[(int64_t)k * C + c];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) m += __shfl_xor(m, o);
  }
  __shared__ int64_t red[4][64];
  __shared__ int64_t redm[4];
  red[sg][fl] = s;
  if (fl == 0) redm[sg] = m;
  __syncthreads();
  if (sg == 0) {
    const int64_t tot = (f < F) ? red[0][fl] + red[1][fl] + red[2][fl] + red[3][fl] : 0;
    if (f < F) part2[((int64_t)rs * C + c) * Fp + f] = tot;
    if (blockIdx.x == 0 && fl == 0) nc2[(int64_t)rs * C + c] = redm[0] + redm[1] + redm[2] + redm[3];
    if (csum) {
      int64_t w = tot;
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) w += __shfl_xor(w, o);
      if (fl == 0) atomicAdd(reinterpret_cast<unsigned long long*>(csum + (int64_t)rs * C + c), (unsigned long long)w);
    }
  }
}

struct TableArgs {
  const int64_t* part2;    // [RS][C][Fp] second-level partial counts
  const int64_t* nc2;      // [RS][C]
  int32_t* counts;
  int64_t* class_totals;
  int64_t* class_sums;
  double* log_theta;
  double* log_1m_theta;
  double* weight;
  double* bias;
  const int32_t* flag_part;  // [n_flags] the count kernel's per-workgroup flags
  int32_t* class_flags;      // [C] error flags gathered by each class's workgroup
  double alpha;
  int32_t F, C, Fp, RS, kind, min_files, n_flags;
};

// Sum over the 256 threads of a workgroup: wave shuffles, then the four
// wave totals in a fixed order (deterministic for floating point).
template <class T>
__device__ __forceinline__ T block_sum(T v, T* red4) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  if ((threadIdx.x & 63) == 0) red4[threadIdx.x >> 6] = v;
  __syncthreads();
  return red4[0] + red4[1] + red4[2] + red4[3];
}

// One workgroup per class: finish the counts (sum of the second-level
// partials, int32 range check), S_c, N_c, then the FP64 tables.
__global__ __launch_bounds__(256) void class_tables(TableArgs a) {
  const int c = blockIdx.x;
  const int t = threadIdx.x;
  int32_t* T = a.counts + (int64_t)c * a.F;

  // the count kernel's flags (every class workgroup gathers all of them),
  // loaded first: they do not depend on the sums below
  int32_t fl = 0;
  for (int i = t; i < a.n_flags; i += 256) fl |= a.flag_part[i];

  // Every partial is loaded before any is summed (the loads are independent;
  // summed one at a time they would form a chain of L2 round trips).  With
  // F <= 1024 a thread's counts stay in registers for the tables below.
  constexpr int kFeatPerPass = 4;
  const bool one_pass = a.F <= 256 * kFeatPerPass;
  int64_t s = 0;
  bool over = false;
  int32_t kept[kFeatPerPass];
  for (int f0 = t; f0 < a.F; f0 += 256 * kFeatPerPass) {
    int64_t v[kFeatPerPass][kReduceSplit];
#pragma unroll
    for (int q = 0; q < kFeatPerPass; ++q) {
      const int f = f0 + q * 256;
#pragma unroll
      for (int r = 0; r < kReduceSplit; ++r)
        v[q][r] = (f < a.F && r < a.RS) ? a.part2[((int64_t)r * a.C + c) * a.Fp + f] : 0;
    }
#pragma unroll
    for (int q = 0; q < kFeatPerPass; ++q) {
      const int f = f0 + q * 256;
      int64_t tot = 0;
#pragma unroll
      for (int r = 0; r < kReduceSplit; ++r) tot += v[q][r];
      if (tot > INT32_MAX) {
        over = true;
        tot = INT32_MAX;
      }
      kept[q] = (int32_t)tot;
      if (f < a.F) {
        T[f] = (int32_t)tot;
        s += tot;
      }
    }
  }
  // class totals: one partial per thread, summed in a fixed order
  __shared__ int64_t snc[kMaxClasses];
  if (t < a.C) {
    int64_t w[kReduceSplit];
#pragma unroll
    for (int r = 0; r < kReduceSplit; ++r) w[r] = (r < a.RS) ? a.nc2[(int64_t)r * a.C + t] : 0;
    int64_t tot = 0;
#pragma unroll
    for (int r = 0; r < kReduceSplit; ++r) tot += w[r];
    snc[t] = tot;
  }
  // S_c (wave sums, then the four wave totals in a fixed order) and the OR
  // of every thread's flags, behind one barrier
  int bits = (over ? kFlagOverflow : 0) | (fl & (kFlagOverflow | kFlagBadLabel | kFlagNegative | kFlagBadIndex));
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    s += __shfl_xor(s, m);
    bits |= __shfl_xor(bits, m);
  }
  __shared__ int64_t red_i[4];
  __shared__ int red_b[4];
  if ((t & 63) == 0) {
    red_i[t >> 6] = s;
    red_b[t >> 6] = bits;
  }
  __syncthreads();
  const int64_t Sc = red_i[0] + red_i[1] + red_i[2] + red_i[3];
  bits = red_b[0] | red_b[1] | red_b[2] | red_b[3];
  int64_t N = 0;
  for (int k = 0; k < a.C; ++k) N += snc[k];
  const int64_t Nc = snc[c];
  if (t == 0) {
    a.class_totals[c] = Nc;
    a.class_sums[c] = (a.kind == NB_BERNOULLI) ? Nc : Sc;
    a.class_flags[c] = bits | ((Nc < a.min_files || Nc < 1) ? kFlagMinFiles : 0);
  }

  if (a.kind == NB_GAUSSIAN) return;   // its tables follow from the moments (gauss_tables)
  const double al = a.alpha;
  double part = 0.0;
  const bool multi = (a.kind == NB_MULTINOMIAL);
  const double den = multi ? log((double)Sc + al * (double)a.F) : log((double)Nc + 2.0 * al);
  // feature f's tables from its count; Bernoulli terms log(1 - theta) are
  // added to `part` in increasing f, as the one-pass and the reloading
  // forms both visit a thread's features
  auto emit = [&](int f, int32_t Tf) {
    const double lt = log((double)Tf + al) - den;
    const int64_t i = (int64_t)c * a.F + f;
    a.log_theta[i] = lt;
    if (multi) {
      a.log_1m_theta[i] = 0.0;
      a.weight[i] = lt;
    } else {
      const double l1 = log((double)(Nc - Tf) + al) - den;
      a.log_1m_theta[i] = l1;
      a.weight[i] = lt - l1;
      part += l1;
    }
  };
  if (one_pass) {
#pragma unroll
    for (int q = 0; q < kFeatPerPass; ++q)
      if (t + q * 256 < a.F) emit(t + q * 256, kept[q]);
  } else {
    for (int f = t; f < a.F; f += 256) emit(f, T[f]);
  }
  __shared__ double red_d[4];
  const double sum_l1 = block_sum<double>(part, red_d);
  if (t == 0) {
    const double lp = log((double)Nc) - log((double)N);
    a.bias[c] = (a.kind == NB_MULTINOMIAL) ? lp : lp + sum_l1;
  }
}

__global__ __launch_bounds__(256) void form_rows(const double* __restrict__ W, const double* __restrict__ bias,
                                                int C, int F, int Fp, float* __restrict__ rows32,
                                                uint16_t* __restrict__ rows16, float* __restrict__ row_bias,
                                                const int32_t* __restrict__ class_flags,
                                                int32_t* __restrict__ status) {
  const int f = blockIdx.x * 256 + threadIdx.x;
  const int P = (C == 2) ? 1 : C;
  if (f < Fp) {
    if (f >= F) {
      for (int r = 0; r <= P; ++r) {
        rows32[(int64_t)r * Fp + f] = 0.0f;
        rows16[(int64_t)r * Fp + f] = 0;
      }
    } else if (C == 2) {
      const double w0 = W[f], w1 = W[(int64_t)F + f];
      const double d = w1 - w0;
      rows32[f] = (float)d;
      rows16[f] = dev::f64_to_bf16_rne(d);
      rows32[(int64_t)Fp + f] = (float)w0;
      rows16[(int64_t)Fp + f] = dev::f64_to_bf16_rne(w0);
    } else {
      double m = 0.0;
      for (int c = 0; c < C; ++c) m += W[(int64_t)c * F + f];
      m /= (double)C;
      for (int c = 0; c < C; ++c) {
        const double v = W[(int64_t)c * F + f] - m;
        rows32[(int64_t)c * Fp + f] = (float)v;
        rows16[(int64_t)c * Fp + f] = dev::f64_to_bf16_rne(v);
      }
      rows32[(int64_t)C * Fp + f] = (float)m;
      rows16[(int64_t)C * Fp + f] = dev::f64_to_bf16_rne(m);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && row_bias) {
    if (C == 2) {
      row_bias[0] = (float)(bias[1] - bias[0]);
      row_bias[1] = (float)bias[0];
    } else {
      double mb = 0.0;
      for (int c = 0; c < C; ++c) mb += bias[c];
      mb /= (double)C;
      for (int c = 0; c < C; ++c) row_bias[c] = (float)(bias[c] - mb);
      row_bias[C] = (float)mb;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && status) {
    int32_t flags = 0;
    for (int c = 0; c < C; ++c) flags |= class_flags[c];
    status[kStatusFlags] = flags;
    status[kStatusTrained] = (flags == 0) ? 1 : 0;
    status[2] = 0;
    status[3] = 0;
  }
}

// Two classes, multinomial, byte features: class_tables and form_rows as one
// launch, one thread per feature.  S_c comes from reduce_counts' exact sums,
// and no count can exceed INT32_MAX (nb_train refuses n * 255 > INT32_MAX),
// so a feature's tables need no other feature.  Counts, tables, bias, rows
// and status are the same expressions, in the same FP64 operations, as in
// class_tables followed by form_rows.  grid (Fp / 256).
__global__ __launch_bounds__(256) void tables_rows2(TableArgs a, const int64_t* __restrict__ csum,
                                                   float* __restrict__ rows32, uint16_t* __restrict__ rows16,
                                                   float* __restrict__ row_bias, int32_t* __restrict__ status) {
  const int t = threadIdx.x;
  const int f = blockIdx.x * 256 + t;
  const int F = a.F, Fp = a.Fp;
  // the OR of the count kernel's flags, gathered by reduce_counts
  const int32_t fl = (blockIdx.x == 0 && t == 0) ? *reinterpret_cast<const int32_t*>(csum + (int64_t)a.RS * 2) : 0;
  int64_t v[2][kReduceSplit], w[2][kReduceSplit], u[2][kReduceSplit];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int r = 0; r < kReduceSplit; ++r) {
      v[c][r] = (f < F && r < a.RS) ? a.part2[((int64_t)r * 2 + c) * Fp + f] : 0;
      w[c][r] = (r < a.RS) ? a.nc2[(int64_t)r * 2 + c] : 0;
      u[c][r] = (r < a.RS) ? csum[(int64_t)r * 2 + c] : 0;
    }
  int64_t Tc[2], Nc[2], Sc[2];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    Tc[c] = 0;
    Nc[c] = 0;
    Sc[c] = 0;
#pragma unroll
    for (int r = 0; r < kReduceSplit; ++r) {
      Tc[c] += v[c][r];
      Nc[c] += w[c][r];
      Sc[c] += u[c][r];
    }
  }
  const double al = a.alpha;
  if (f < F) {
    double lt[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      a.counts[(int64_t)c * F + f] = (int32_t)Tc[c];
      const double den = log((double)Sc[c] + al * (double)F);
      lt[c] = log((double)Tc[c] + al) - den;
      const int64_t i = (int64_t)c * F + f;
      a.log_theta[i] = lt[c];
      a.log_1m_theta[i] = 0.0;
      a.weight[i] = lt[c];
    }
    const double d = lt[1] - lt[0];
    rows32[f] = (float)d;
    rows16[f] = dev::f64_to_bf16_rne(d);
    rows32[(int64_t)Fp + f] = (float)lt[0];
    rows16[(int64_t)Fp + f] = dev::f64_to_bf16_rne(lt[0]);
  } else if (f < Fp) {
    for (int r = 0; r <= 1; ++r) {
      rows32[(int64_t)r * Fp + f] = 0.0f;
      rows16[(int64_t)r * Fp + f] = 0;
    }
  }
  if (blockIdx.x == 0) {
    if (t == 0) {
      const int32_t bits = fl & (kFlagOverflow | kFlagBadLabel | kFlagNegative | kFlagBadIndex);
      const int64_t N = Nc[0] + Nc[1];
      double bias[2];
      int32_t flags = 0;
      for (int c = 0; c < 2; ++c) {
        a.class_totals[c] = Nc[c];
        a.class_sums[c] = Sc[c];
        bias[c] = log((double)Nc[c]) - log((double)N);
        a.bias[c] = bias[c];
        const int32_t cf = bits | ((Nc[c] < a.min_files || Nc[c] < 1) ? kFlagMinFiles : 0);
        a.class_flags[c] = cf;
        flags |= cf;
      }
      row_bias[0] = (float)(bias[1] - bias[0]);
      row_bias[1] = (float)bias[0];
      status[kStatusFlags] = flags;
      status[kStatusTrained] = (flags == 0) ? 1 : 0;
      status[2] = 0;
      status[3] = 0;
    }
  }
}

// ------------------------------------------------------------ Gaussian
typedef unsigned __int128 u128;

// Nonnegative 128-bit integer to FP64 (at most two roundings).
__device__ __forceinline__ double u128_to_double(u128 v) {
  return (double)(uint64_t)(v >> 64) * 18446744073709551616.0 + (double)(uint64_t)v;
}

// n^2 times the population variance of n values with sum t and sum of
// squares q: n q - t^2 (>= 0), exact.
__device__ __forceinline__ u128 var_numerator(int64_t n, int64_t t, int64_t q) {
  return (u128)(uint64_t)n * (uint64_t)q - (u128)(uint64_t)t * (uint64_t)t;
}

// Q_cf: the last level of the square sums.  grid (ceil(F/256), C).
__global__ __launch_bounds__(256) void sumsq_finish(const int64_t* __restrict__ part2_sq, int RS, int C, int F,
                                                   int Fp, int64_t* __restrict__ sumsq) {
  const int c = blockIdx.y, f = blockIdx.x * 256 + threadIdx.x;
  if (f < F) {
    int64_t v[kReduceSplit];
#pragma unroll
    for (int r = 0; r < kReduceSplit; ++r) v[r] = (r < RS) ? part2_sq[((int64_t)r * C + c) * Fp + f] : 0;
    int64_t s = 0;
#pragma unroll
    for (int r = 0; r < kReduceSplit; ++r) s += v[r];
    sumsq[(int64_t)c * F + f] = s;
  }
}

// epsilon = 1e-9 x the largest variance of a feature over all training
// files (classes pooled).  One workgroup.
__global__ __launch_bounds__(256) void gauss_eps(const int32_t* __restrict__ counts,
                                                const int64_t* __restrict__ sumsq,
                                                const int64_t* __restrict__ class_totals, int C, int F,
                                                double* __restrict__ eps_out, int32_t* __restrict__ class_flags) {
  const int t = threadIdx.x;
  int64_t N = 0;
  for (int c = 0; c < C; ++c) N += class_totals[c];
  double m = 0.0;
  for (int f = t; f < F; f += 256) {
    int64_t tf = 0, qf = 0;
    for (int c = 0; c < C; ++c) {
      tf += counts[(int64_t)c * F + f];
      qf += sumsq[(int64_t)c * F + f];
    }
    const double v = u128_to_double(var_numerator(N, tf, qf)) / (double)N / (double)N;
    m = fmax(m, v);
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  __shared__ double red[4];
  if ((t & 63) == 0) red[t >> 6] = m;
  __syncthreads();
  if (t == 0) {
    const double top = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    *eps_out = 1e-9 * top;
    if (!(top > 0.0)) class_flags[0] |= kFlagZeroVariance;
  }
}

// Per class: mean, variance + epsilon, the weight h = -1 / (2 var) and the
// bias log prior - (1/2) sum_f log(2 pi var) (fixed-order reduction) of the
// score form s = bias + sum_f h (x - mean)^2.  grid C.
__global__ __launch_bounds__(256) void gauss_tables(const int32_t* __restrict__ counts,
                                                   const int64_t* __restrict__ sumsq,
                                                   const int64_t* __restrict__ class_totals,
                                                   const double* __restrict__ eps_in, int C, int F,
                                                   double* __restrict__ mean, double* __restrict__ var,
                                                   double* __restrict__ weight, double* __restrict__ bias) {
  const int c = blockIdx.x, t = threadIdx.x;
  const double eps = *eps_in;
  const int64_t Nc = class_totals[c];
  int64_t N = 0;
  for (int k = 0; k < C; ++k) N += class_totals[k];
  const double dn = (double)Nc;
  double part = 0.0;
  for (int f = t; f < F; f += 256) {
    const int64_t i = (int64_t)c * F + f;
    const int64_t tf = counts[i], qf = sumsq[i];
    const double mu = (double)tf / dn;
    const double v = u128_to_double(var_numerator(Nc, tf, qf)) / dn / dn + eps;
    mean[i] = mu;
    var[i] = v;
    weight[i] = -0.5 / v;
    part += log(2.0 * M_PI * v);
  }
  __shared__ double red_d[4];
  const double s = block_sum<double>(part, red_d);
  if (t == 0) bias[c] = log(dn) - log((double)N) - 0.5 * s;
}

// Gaussian scoring rows: row c of the first set is mean_c, row c of the
// second is h_c, each rounded once to FP32 and to BF16, zero padded; the
// row biases are b_1 - b_0 and b_0 for two classes (b_c otherwise); then
// the status word.  grid Fp / 256.
__global__ __launch_bounds__(256) void gauss_rows(const double* __restrict__ mean, const double* __restrict__ h,
                                                 const double* __restrict__ bias, int C, int F, int Fp,
                                                 float* __restrict__ mu32, uint16_t* __restrict__ mu16,
                                                 float* __restrict__ h32, uint16_t* __restrict__ h16,
                                                 float* __restrict__ row_bias,
                                                 const int32_t* __restrict__ class_flags,
                                                 int32_t* __restrict__ status) {
  const int f = blockIdx.x * 256 + threadIdx.x;
  if (f < Fp) {
    for (int c = 0; c < C; ++c) {
      const int64_t o = (int64_t)c * Fp + f;
      const double m = (f < F) ? mean[(int64_t)c * F + f] : 0.0;
      const double w = (f < F) ? h[(int64_t)c * F + f] : 0.0;
      mu32[o] = (float)m;
      mu16[o] = dev::f64_to_bf16_rne(m);
      h32[o] = (float)w;
      h16[o] = dev::f64_to_bf16_rne(w);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (C == 2) {
      row_bias[0] = (float)(bias[1] - bias[0]);
      row_bias[1] = (float)bias[0];
    } else {
      for (int c = 0; c < C; ++c) row_bias[c] = (float)bias[c];
      row_bias[C] = 0.0f;
    }
    int32_t flags = 0;
    for (int c = 0; c < C; ++c) flags |= class_flags[c];
    status[kStatusFlags] = flags;
    status[kStatusTrained] = (flags == 0) ? 1 : 0;
    status[2] = 0;
    status[3] = 0;
  }
}

// 64-row label windows per row list: at least about 32 matching rows per
// list (two full batches) for 2, 3 to 7 and 8 to 11 classes, about 64 from 12
// classes on.
int count_win(int32_t C) { return C <= 2 ? 1 : (C <= 7 ? 4 : (C <= 11 ? 8 : 16)); }

template <int XT, bool BIN, bool SQ>
const void* count_fn_win(int win) {
  switch (win) {
    case 1: return reinterpret_cast<const void*>(count_kernel<XT, BIN, SQ, 1>);
    case 4: return reinterpret_cast<const void*>(count_kernel<XT, BIN, SQ, 4>);
    case 16: return reinterpret_cast<const void*>(count_kernel<XT, BIN, SQ, 16>);
    default: return reinterpret_cast<const void*>(count_kernel<XT, BIN, SQ, 8>);
  }
}

// The count kernel for a feature type, kind and pass (SQ: square sums).
const void* count_fn(int32_t xtype, bool bin, bool sq, int win) {
  if (xtype == NB_X_I32)
    return sq ? count_fn_win<NB_X_I32, false, true>(win)
              : (bin ? count_fn_win<NB_X_I32, true, false>(win) : count_fn_win<NB_X_I32, false, false>(win));
  return sq ? count_fn_win<NB_X_U8, false, true>(win)
            : (bin ? count_fn_win<NB_X_U8, true, false>(win) : count_fn_win<NB_X_U8, false, false>(win));
}

// Workgroups of the count kernel resident on the device at once.
int count_capacity(int32_t xtype, int win) {
  return resident_per_cu(count_fn(xtype, false, false, win), kThreads, 0) * device_cu_count();
}

// Row slots of the count pass, with at least kMinRowsPerSlot rows per slot.
// Two classes: as many (slot, class, chunk) workgroups as fit on the device
// in one round (a few more would run as a second, nearly empty round).  With
// more classes a workgroup's work is the rows of its class in its slot, which
// differs between classes as much as their priors do; four rounds of smaller
// slots let the workgroups of the small classes finish and make room, so that
// the large classes' rows are spread over the whole device.
constexpr int64_t kManyClassRounds = 4;
int64_t train_slots(int32_t C, int32_t F, int64_t n, int32_t xtype) {
  const int64_t nch = (align_up((size_t)F, kFeaturePad)) / kChunk;
  const int64_t units = std::max<int64_t>(1, count_capacity(xtype, count_win(C)));
  const int64_t rounds = C > 2 ? kManyClassRounds : 1;
  const int64_t s = std::max<int64_t>(1, rounds * units / (C * nch));
  const int64_t by_rows = std::max<int64_t>(1, (n + kMinRowsPerSlot - 1) / kMinRowsPerSlot);
  return std::max<int64_t>(1, std::min(s, by_rows));
}

// Workspace: per-slot partials, per-slot class totals, and the RS
// second-level partials of each.
struct TrainWs {
  int64_t S, RS;
  size_t off_part, off_nc, off_part2, off_nc2, off_part_sq, off_part2_sq, off_flags, off_csum, total;
};

TrainWs train_ws(int32_t C, int32_t Fp, int64_t S) {
  TrainWs w;
  w.S = S;
  w.RS = std::min<int64_t>(kReduceSplit, S);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes, kAlign);
    return at;
  };
  w.off_part = take((size_t)S * C * Fp * 8);
  w.off_nc = take((size_t)S * C * 8);
  w.off_part2 = take((size_t)w.RS * C * Fp * 8);
  w.off_nc2 = take((size_t)w.RS * C * 8);
  // square sums of a Gaussian model (the workspace size does not depend on
  // the kind)
  w.off_part_sq = take((size_t)S * C * Fp * 8);
  w.off_part2_sq = take((size_t)w.RS * C * Fp * 8);
  // count-kernel flags [2][S][C][chunks] (counts, squares), then per-class flags
  w.off_flags = take(((size_t)2 * S * C * (Fp / kChunk) + C) * 4);
  // class-sum shares and the flag word of the one-launch two-class tables
  w.off_csum = take((size_t)(w.RS * C + 1) * 8);
  w.total = off;
  return w;
}

// A k-feature model from a trained model's counts (the model trained on the
// gathered columns): the selected columns become the single second-level
// partial of class_tables, the class totals are copied, and an index outside
// [0, F) is flagged (its column reads as 0).  grid (ceil(k/256), C).
__global__ __launch_bounds__(256) void subset_counts(const int32_t* __restrict__ counts,
                                                    const int64_t* __restrict__ totals,
                                                    const int32_t* __restrict__ idx, int F, int k, int Fp_out,
                                                    int64_t* __restrict__ part2, int64_t* __restrict__ nc2,
                                                    int32_t* __restrict__ flag_part) {
  const int c = blockIdx.y, t = threadIdx.x;
  const int j = blockIdx.x * 256 + t;
  bool bad = false;
  if (j < k) {
    const int32_t f = idx[j];
    int64_t v = 0;
    if (f < 0 || f >= F) bad = true;
    else v = counts[(int64_t)c * F + f];
    part2[(int64_t)c * Fp_out + j] = v;
  }
  const int any_bad = __syncthreads_or(bad);
  if (t == 0) {
    flag_part[(int64_t)c * gridDim.x + blockIdx.x] = any_bad ? kFlagBadIndex : 0;
    if (blockIdx.x == 0) nc2[c] = totals[c];
  }
}

// Workspace of nb_model_select: part2 [C][Fp], nc2 [C], flags.
struct SelectWs {
  int32_t n_flags;
  size_t off_part2, off_nc2, off_flags, total;
};

SelectWs select_ws(int32_t C, int32_t k, int32_t Fp) {
  SelectWs w;
  w.n_flags = C * ((k + 255) / 256);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes, kAlign);
    return at;
  };
  w.off_part2 = take((size_t)C * Fp * 8);
  w.off_nc2 = take((size_t)C * 8);
  w.off_flags = take(((size_t)w.n_flags + C) * 4);
  w.total = off;
  return w;
}

// Table build shared by nb_train and nb_model_select: class_tables over RS
// second-level partials, then the scoring rows and the status word.
// csum: the class sums from reduce_counts (two classes, multinomial, byte
// features): the tables and rows then take one launch.
int launch_tables(nb_model* m, const nb_layout& L, const int64_t* part2, const int64_t* nc2, int RS,
                  const int32_t* flag_part, int n_flags, int32_t* class_flags, double alpha, int min_files,
                  hipStream_t s, const int64_t* part2_sq = nullptr, const int64_t* csum = nullptr) {
  uint8_t* base = static_cast<uint8_t*>(m->dev);
  TableArgs ta;
  ta.part2 = part2;
  ta.nc2 = nc2;
  ta.counts = reinterpret_cast<int32_t*>(base + L.off_counts);
  ta.class_totals = reinterpret_cast<int64_t*>(base + L.off_class_totals);
  ta.class_sums = reinterpret_cast<int64_t*>(base + L.off_class_sums);
  ta.log_theta = reinterpret_cast<double*>(base + L.off_log_theta);
  ta.log_1m_theta = reinterpret_cast<double*>(base + L.off_log_1m_theta);
  ta.weight = reinterpret_cast<double*>(base + L.off_weight);
  ta.bias = reinterpret_cast<double*>(base + L.off_bias);
  ta.flag_part = flag_part;
  ta.class_flags = class_flags;
  ta.n_flags = n_flags;
  ta.alpha = alpha;
  ta.F = m->n_features;
  ta.C = m->n_classes;
  ta.Fp = L.padded_features;
  ta.RS = RS;
  ta.kind = m->kind;
  ta.min_files = min_files;
  if (csum) {
    hipLaunchKernelGGL(tables_rows2, dim3((unsigned)(ta.Fp / 256)), dim3(256), 0, s, ta, csum,
                       reinterpret_cast<float*>(base + L.off_form_f32),
                       reinterpret_cast<uint16_t*>(base + L.off_form_bf16),
                       reinterpret_cast<float*>(base + L.off_form_bias), reinterpret_cast<int32_t*>(base + L.off_status));
    NB_HIP_CHECK(hipGetLastError());
    return NB_OK;
  }
  hipLaunchKernelGGL(class_tables, dim3((unsigned)ta.C), dim3(256), 0, s, ta);
  NB_HIP_CHECK(hipGetLastError());
  if (m->kind == NB_GAUSSIAN) {
    int64_t* sumsq = reinterpret_cast<int64_t*>(base + L.off_sumsq);
    double* eps = reinterpret_cast<double*>(base + L.off_epsilon);
    hipLaunchKernelGGL(sumsq_finish, dim3((unsigned)((ta.F + 255) / 256), (unsigned)ta.C), dim3(256), 0, s,
                       part2_sq, RS, ta.C, ta.F, ta.Fp, sumsq);
    NB_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(gauss_eps, dim3(1), dim3(256), 0, s, ta.counts, sumsq, ta.class_totals, ta.C, ta.F, eps,
                       class_flags);
    NB_HIP_CHECK(hipGetLastError());
    double* mean = reinterpret_cast<double*>(base + L.off_mean);
    hipLaunchKernelGGL(gauss_tables, dim3((unsigned)ta.C), dim3(256), 0, s, ta.counts, sumsq, ta.class_totals, eps,
                       ta.C, ta.F, mean, reinterpret_cast<double*>(base + L.off_var), ta.weight, ta.bias);
    NB_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(gauss_rows, dim3((unsigned)(ta.Fp / 256)), dim3(256), 0, s, mean, ta.weight, ta.bias, ta.C,
                       ta.F, ta.Fp, reinterpret_cast<float*>(base + L.off_form_f32),
                       reinterpret_cast<uint16_t*>(base + L.off_form_bf16),
                       reinterpret_cast<float*>(base + L.off_form2_f32),
                       reinterpret_cast<uint16_t*>(base + L.off_form2_bf16),
                       reinterpret_cast<float*>(base + L.off_form_bias), class_flags,
                       reinterpret_cast<int32_t*>(base + L.off_status));
    NB_HIP_CHECK(hipGetLastError());
    return NB_OK;
  }
  hipLaunchKernelGGL(form_rows, dim3((unsigned)(ta.Fp / 256)), dim3(256), 0, s, ta.weight, ta.bias, ta.C, ta.F,
                     ta.Fp, reinterpret_cast<float*>(base + L.off_form_f32),
                     reinterpret_cast<uint16_t*>(base + L.off_form_bf16),
                     reinterpret_cast<float*>(base + L.off_form_bias), class_flags,
                     reinterpret_cast<int32_t*>(base + L.off_status));
  NB_HIP_CHECK(hipGetLastError());
  return NB_OK;
}

int flags_to_status(int32_t flags) {
  if (flags & kFlagBadIndex) return fail(NB_EDATA, "a selected feature index is outside [0, F)");
  if (flags & kFlagZeroVariance)
    return fail(NB_EDATA, "every training file is identical: the Gaussian variances are all zero");
  if (flags & (kFlagBadLabel | kFlagNegative))
    return fail(NB_EDATA, (flags & kFlagBadLabel) ? "a label is outside [0, C)" : "a feature value is negative");
  if (flags & kFlagOverflow)
    return fail(NB_EOVERFLOW, "a per-class count exceeds INT32_MAX (or, for a Gaussian model, an int32 feature "
                              "is 65536 or more)");
  if (flags & kFlagMinFiles) return fail(NB_EMINFILES, "a class has fewer training files than required");
  return NB_OK;
}

}  // namespace
}  // namespace nb

using namespace nb;

extern "C" {

size_t nb_train_workspace_bytes(int32_t n_classes, int32_t n_features, int64_t n, int32_t xtype) {
  nb_layout L;
  if (!compute_layout(n_classes, n_features, &L) || n < 0 || elem_bytes(xtype) == 0) return 0;
  return train_ws(n_classes, L.padded_features, train_slots(n_classes, n_features, n, xtype)).total;
}

int nb_train(nb_model* m, const void* x, int32_t xtype, int64_t n, int64_t ld, const int32_t* y,
             double alpha, int32_t min_files_per_class, void* workspace, size_t workspace_bytes,
             int32_t flags, void* stream) {
  nb_layout L;
  int rc = check_model(m, &L);
  if (rc) return rc;
  m->trained = 0;
  const int C = m->n_classes, F = m->n_features;
  if (xtype != NB_X_U8 && xtype != NB_X_I32)
    return fail(NB_EINVAL, "training features must be NB_X_U8 or NB_X_I32");
  if (n < 1) return fail(NB_EINVAL, "n must be >= 1");
  if (ld < F) return fail(NB_EINVAL, "ld must be >= n_features");
  const int eb = elem_bytes(xtype);
  if (((int64_t)ld * eb) % 4 != 0) return fail(NB_EINVAL, "row stride must be a multiple of 4 bytes");
  if (!x || !y) return fail(NB_EINVAL, "x and y must be non-NULL");
  if ((reinterpret_cast<uintptr_t>(x) & 3) != 0) return fail(NB_EINVAL, "x must be 4-byte aligned");
  if (!(alpha > 0.0) || !std::isfinite(alpha)) return fail(NB_EINVAL, "alpha must be finite and > 0");
  if (min_files_per_class < 1) return fail(NB_EINVAL, "min_files_per_class must be >= 1");
  if (xtype == NB_X_U8 && n > INT32_MAX / 255)
    return fail(NB_EOVERFLOW, "n * 255 exceeds INT32_MAX: byte counts could overflow int32");
  const size_t need = nb_train_workspace_bytes(C, F, n, xtype);
  if (!workspace || workspace_bytes < need)
    return fail(NB_ENOMEM, "workspace smaller than nb_train_workspace_bytes()");
  if ((reinterpret_cast<uintptr_t>(workspace) & 7) != 0) return fail(NB_EINVAL, "workspace must be 8-byte aligned");

  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  uint8_t* base = static_cast<uint8_t*>(m->dev);
  int32_t* status = reinterpret_cast<int32_t*>(base + L.off_status);
  const int Fp = L.padded_features;
  const int64_t S = train_slots(C, F, n, xtype);
  const TrainWs tw = train_ws(C, Fp, S);
  uint8_t* wsb = static_cast<uint8_t*>(workspace);
  int64_t* part = reinterpret_cast<int64_t*>(wsb + tw.off_part);
  int64_t* nc_part = reinterpret_cast<int64_t*>(wsb + tw.off_nc);
  int64_t* part2 = reinterpret_cast<int64_t*>(wsb + tw.off_part2);
  int64_t* nc2 = reinterpret_cast<int64_t*>(wsb + tw.off_nc2);
  const bool gauss = (m->kind == NB_GAUSSIAN);
  const int n_flags1 = (int)(S * C * (Fp / kChunk));
  const int n_flags = gauss ? 2 * n_flags1 : n_flags1;
  int32_t* flag_part = reinterpret_cast<int32_t*>(wsb + tw.off_flags);
  int32_t* class_flags = flag_part + 2 * n_flags1;
  int64_t* part_sq = reinterpret_cast<int64_t*>(wsb + tw.off_part_sq);
  int64_t* part2_sq = reinterpret_cast<int64_t*>(wsb + tw.off_part2_sq);

  CountArgs ca;
  ca.x = static_cast<const uint8_t*>(x);
  ca.ld_bytes = ld * eb;
  ca.n = n;
  ca.total_bytes = ((n - 1) * ld + F) * (int64_t)eb;
  ca.y = y;
  ca.rows_per_slot = (n + S - 1) / S;
  ca.part = part;
  ca.nc_part = nc_part;
  ca.flag_part = flag_part;
  ca.F = F;
  ca.C = C;
  ca.Fp = Fp;
  // two classes, multinomial, byte features: the class sums come from
  // reduce_counts and the tables and rows take one launch
  const bool fused = (C == 2 && m->kind == NB_MULTINOMIAL && xtype == NB_X_U8);
  int64_t* csum = fused ? reinterpret_cast<int64_t*>(wsb + tw.off_csum) : nullptr;
  ca.zero_words = csum;
  ca.n_zero = fused ? (int)(tw.RS * C + 1) : 0;
  const dim3 grid((unsigned)S, (unsigned)C, (unsigned)(Fp / kChunk));
  const bool bin = (m->kind == NB_BERNOULLI);
  const int win = count_win(C);
  {
    void* args[] = {&ca};
    NB_HIP_CHECK(hipLaunchKernel(count_fn(xtype, bin, false, win), grid, dim3(kThreads), args, 0, s));
  }
  if (gauss) {   // second pass: the sums of squares
    CountArgs cq = ca;
    cq.part = part_sq;
    cq.flag_part = flag_part + n_flags1;
    void* args[] = {&cq};
    NB_HIP_CHECK(hipLaunchKernel(count_fn(xtype, false, true, win), grid, dim3(kThreads), args, 0, s));
  }

  const dim3 rgrid((unsigned)((F + 63) / 64), (unsigned)C, (unsigned)tw.RS);
  hipLaunchKernelGGL(reduce_counts, rgrid, dim3(256), 0, s, part, nc_part, (int)S, C, F, Fp, part2, nc2, csum,
                     flag_part, n_flags);
  NB_HIP_CHECK(hipGetLastError());
  if (gauss) {   // (the class totals it writes again are the same values)
    hipLaunchKernelGGL(reduce_counts, rgrid, dim3(256), 0, s, part_sq, nc_part, (int)S, C, F, Fp, part2_sq, nc2,
                       nullptr, nullptr, 0);
    NB_HIP_CHECK(hipGetLastError());
  }

  rc = launch_tables(m, L, part2, nc2, (int)tw.RS, flag_part, n_flags, class_flags, alpha, min_files_per_class,
                     s, part2_sq, csum);
  if (rc) return rc;

  if (flags & NB_TRAIN_ASYNC) return NB_OK;
  return nb_model_status(m, stream);
}

size_t nb_model_select_workspace_bytes(int32_t n_classes, int32_t k) {
  nb_layout L;
  if (!compute_layout(n_classes, k, &L)) return 0;
  return select_ws(n_classes, k, L.padded_features).total;
}

int nb_model_select(const nb_model* full, const int32_t* idx, int32_t k, double alpha, nb_model* out,
                    void* workspace, size_t workspace_bytes, int32_t flags, void* stream) {
  nb_layout LF, L;
  int rc = check_model(full, &LF);
  if (rc) return rc;
  if (!full->trained) return fail(NB_EINVAL, "the full model is not trained");
  if (full->kind == NB_GAUSSIAN)
    return fail(NB_EINVAL, "k-feature models are built for multinomial and Bernoulli models");
  if (!out) return fail(NB_EINVAL, "out is NULL");
  if (out->n_features != k) return fail(NB_EINVAL, "out->n_features must equal k");
  if (out->kind != full->kind || out->n_classes != full->n_classes)
    return fail(NB_EINVAL, "out must have the kind and class count of the full model");
  rc = check_model(out, &L);
  if (rc) return rc;
  if (out->dev == full->dev) return fail(NB_EINVAL, "out must have its own buffer");
  out->trained = 0;
  if (!idx) return fail(NB_EINVAL, "idx must be non-NULL");
  if (!(alpha > 0.0) || !std::isfinite(alpha)) return fail(NB_EINVAL, "alpha must be finite and > 0");
  const int C = full->n_classes;
  const SelectWs w = select_ws(C, k, L.padded_features);
  if (!workspace || workspace_bytes < w.total)
    return fail(NB_ENOMEM, "workspace smaller than nb_model_select_workspace_bytes()");
  if ((reinterpret_cast<uintptr_t>(workspace) & 7) != 0) return fail(NB_EINVAL, "workspace must be 8-byte aligned");

  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  uint8_t* wsb = static_cast<uint8_t*>(workspace);
  int64_t* part2 = reinterpret_cast<int64_t*>(wsb + w.off_part2);
  int64_t* nc2 = reinterpret_cast<int64_t*>(wsb + w.off_nc2);
  int32_t* flag_part = reinterpret_cast<int32_t*>(wsb + w.off_flags);
  int32_t* class_flags = flag_part + w.n_flags;
  const uint8_t* fb = static_cast<const uint8_t*>(full->dev);
  hipLaunchKernelGGL(subset_counts, dim3((unsigned)((k + 255) / 256), (unsigned)C), dim3(256), 0, s,
                     reinterpret_cast<const int32_t*>(fb + LF.off_counts),
                     reinterpret_cast<const int64_t*>(fb + LF.off_class_totals), idx, full->n_features, k,
                     L.padded_features, part2, nc2, flag_part);
  NB_HIP_CHECK(hipGetLastError());
  rc = launch_tables(out, L, part2, nc2, 1, flag_part, w.n_flags, class_flags, alpha, 1, s);
  if (rc) return rc;
  if (flags & NB_TRAIN_ASYNC) return NB_OK;
  return nb_model_status(out, stream);
}

int nb_model_status(nb_model* m, void* stream) {
  nb_layout L;
  int rc = check_model(m, &L);
  if (rc) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int32_t st[4] = {0, 0, 0, 0};
  NB_HIP_CHECK(hipMemcpyAsync(st, static_cast<uint8_t*>(m->dev) + L.off_status, sizeof(st),
                              hipMemcpyDeviceToHost, s));
  NB_HIP_CHECK(hipStreamSynchronize(s));
  m->trained = st[kStatusTrained];
  return flags_to_status(st[kStatusFlags]);
}

}  // extern "C"
