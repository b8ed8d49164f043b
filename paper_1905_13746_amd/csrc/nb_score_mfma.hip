// Naive Bayes scoring with a BF16 table on the matrix cores (C >= 16):
// s~[file, class] = sum_f g(x_f) W~[class, f] is a skinny GEMM
// (M = files, N = classes, K = features) once the class count fills an MFMA
// column tile.  Feature bytes (uint8 counts or FP8-e4m3) convert exactly to
// BF16; products accumulate in FP32 (v_mfma_f32_16x16x32_bf16).
//
// Mapping.  A wave owns MT tiles of 16 files and all NT tiles of 16 classes.
// The K order inside a tile is free (the same permutation on A and B leaves
// the sum unchanged), so each lane streams 16 contiguous feature bytes of
// its file per 64-feature window (lane group q = lane / 16 takes bytes
// 16q .. 16q + 15) and feeds two MFMAs with them; the matching B fragment is
// 8 contiguous BF16 entries of one class row, read from a table slice staged
// in LDS (class-major, padded rows: conflict-free 16-byte reads).  The 4
// waves of a workgroup share each staged slice.  After the K loop the 16x16
// accumulator tiles (lane l holds rows 4*(l/16)..+3 of column l%16) are
// reduced across the 16 lanes of each column group for the max / log-sum-exp
// epilogue; labels take the lowest class index among maxima.
#include <algorithm>
#include <map>
#include <mutex>
#include <type_traits>

#include "nb_device.hpp"
#include "nb_internal.hpp"

namespace nb {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kWindow = 64;                 // features per window (one 16-byte load per lane)
constexpr int kSliceElems = 32768;          // BF16 table entries staged per slice (64 KiB)

struct ScoreMArgs {
  const uint8_t* x;
  int64_t ld_bytes;
  int64_t n;
  int64_t total_bytes;
  const uint16_t* rows16;   // [P+1][Fp] class-major BF16 rows (centred rows, aux row C)
  const float* row_bias;    // [P+1]
  int32_t* labels;
  float* log_post;
  float* scores;
  int32_t F, Fp, C, ns;     // ns: rows used (C, or C + 1 with the aux row)
  int64_t nfast;            // staged kernel: leading wave tiles with every row and load in bounds
};

__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
  // exact for the small integers and FP8 values converted here: keep the
  // upper halves of the two FP32 images
  return __builtin_amdgcn_perm(__float_as_uint(hi), __float_as_uint(lo), 0x07060302u);
}

// 16 feature bytes -> 16 BF16 values (two MFMA A operands).
template <int XT, bool BIN>
__device__ __forceinline__ void to_bf16(const dev::u32x4& v, dev::u32x4& a0, dev::u32x4& a1) {
  uint32_t o[8];
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const uint32_t u = v[d];
    float f0, f1, f2, f3;
    if (XT == NB_X_U8) {
      f0 = (float)(u & 0xFFu);
      f1 = (float)((u >> 8) & 0xFFu);
      f2 = (float)((u >> 16) & 0xFFu);
      f3 = (float)(u >> 24);
    } else {
      const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8(u, false);
      const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8(u, true);
      f0 = lo[0];
      f1 = lo[1];
      f2 = hi[0];
      f3 = hi[1];
    }
    if (BIN) {   // presence: a clamp to [0, 1] for byte counts (folds into the conversion), a compare for FP8
      if (XT == NB_X_U8) {
        f0 = __builtin_amdgcn_fmed3f(f0, 0.0f, 1.0f);
        f1 = __builtin_amdgcn_fmed3f(f1, 0.0f, 1.0f);
        f2 = __builtin_amdgcn_fmed3f(f2, 0.0f, 1.0f);
        f3 = __builtin_amdgcn_fmed3f(f3, 0.0f, 1.0f);
      } else {
        f0 = f0 > 0.0f ? 1.0f : 0.0f;
        f1 = f1 > 0.0f ? 1.0f : 0.0f;
        f2 = f2 > 0.0f ? 1.0f : 0.0f;
        f3 = f3 > 0.0f ? 1.0f : 0.0f;
      }
    }
    o[2 * d] = pack_bf16(f0, f1);
    o[2 * d + 1] = pack_bf16(f2, f3);
  }
  a0 = dev::u32x4{o[0], o[1], o[2], o[3]};
  a1 = dev::u32x4{o[4], o[5], o[6], o[7]};
}

__device__ __forceinline__ f32x4 mfma(const dev::u32x4& a, const dev::u32x4& b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                 0, 0, 0);
}

// Epilogue of a 16*MT-file tile: lane holds files 4q + i (i < 4) of each M
// tile for class 16 nt + col.  Max and lowest arg-max over the 16 lanes of a
// column group, log-sum-exp, then labels, log posteriors and raw scores.
template <int NT, int MT>
__device__ __forceinline__ void epilogue(const ScoreMArgs& a, f32x4 (&acc)[MT][NT], int lane, int64_t row0) {
  const int col = lane & 15, q = lane >> 4;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t row = row0 + 16 * mt + 4 * q + i;
      float s[NT];
      float m = -INFINITY;
      int best = 1 << 30;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int c = 16 * nt + col;
        s[nt] = acc[mt][nt][i] + ((c < a.ns) ? a.row_bias[c] : 0.0f);
        if (c < a.C && s[nt] > m) {
          m = s[nt];
          best = c;
        }
      }
      // max and lowest arg-max over the 16 lanes of this column group
#pragma unroll
      for (int sh = 1; sh < 16; sh <<= 1) {
        const float om = __shfl_xor(m, sh);
        const int ob = __shfl_xor(best, sh);
        if (om > m || (om == m && ob < best)) {
          m = om;
          best = ob;
        }
      }
      float z = 0.0f;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        if (16 * nt + col < a.C) z += __expf(s[nt] - m);
#pragma unroll
      for (int sh = 1; sh < 16; sh <<= 1) z += __shfl_xor(z, sh);
      const float lse = m + __logf(z);
      // aux row (raw-score offset) lives in column C
      float aux = 0.0f;
      if (a.ns > a.C) {
        float mine = 0.0f;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          if (16 * nt + col == a.C) mine = s[nt];
        aux = __shfl(mine, (lane & ~15) | (a.C & 15));
      }
      if (row < a.n) {
        if (a.labels && col == 0) a.labels[row] = best;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const int c = 16 * nt + col;
          if (c < a.C) {
            if (a.log_post) a.log_post[row * a.C + c] = s[nt] - lse;
            if (a.scores) a.scores[row * a.C + c] = s[nt] + aux;
          }
        }
      }
    }
  }
}

template <int XT, int NT, int MT, bool BIN>
__global__ __launch_bounds__(kThreads) void scoreM_kernel(ScoreMArgs a) {
  constexpr int NCOL = 16 * NT;
  constexpr int KT = kSliceElems / NCOL;            // features per staged slice
  constexpr int RS = KT + 8;                        // padded row stride (BF16 entries)
  constexpr int FILES = 16 * MT;                    // files per wave
  __shared__ __attribute__((aligned(16))) uint16_t tbl[NCOL * RS];

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int col = lane & 15, q = lane >> 4;
  const int64_t ld = a.ld_bytes;
  const int64_t per_tile = (int64_t)FILES * kWaves;
  const int64_t ntile = (a.n + per_tile - 1) / per_tile;

  for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const int64_t row0 = tile * per_tile + (int64_t)wave * FILES;   // first file of this wave
    f32x4 acc[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const bool wave_full = row0 + FILES <= a.n;

    for (int k0 = 0; k0 < a.F; k0 += KT) {
      const int kn = min(KT, a.Fp - k0);
      __syncthreads();
      // stage rows [0, NCOL) x features [k0, k0 + kn) (16-byte pieces; rows >= ns are zero)
      const int pieces_per_row = kn / 8;
      for (int i = threadIdx.x; i < NCOL * pieces_per_row; i += kThreads) {
        const int r = i / pieces_per_row, p = i - r * pieces_per_row;
        dev::u32x4 v = {0u, 0u, 0u, 0u};
        if (r < a.ns) v = *reinterpret_cast<const dev::u32x4*>(a.rows16 + (int64_t)r * a.Fp + k0 + 8 * p);
        *reinterpret_cast<dev::u32x4*>(tbl + r * RS + 8 * p) = v;
      }
      __syncthreads();
      const int kend = min(kn, a.F - k0);
      for (int w0 = 0; w0 < kend; w0 += kWindow) {
        // A: file (row0 + 16 mt + col), bytes [k0 + w0 + 16 q, +16)
        const int64_t wbase = row0 * ld + (int64_t)(k0 + w0);
        const auto rsrc = dev::make_rsrc(a.x + wbase, a.total_bytes - wbase);
        const bool safe = wave_full && (row0 + FILES - 1) * ld + k0 + w0 + kWindow <= a.total_bytes;
        dev::u32x4 xv[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const int r = 16 * mt + col;
          const uint32_t rel = (uint32_t)(r * ld) + 16 * q;
          if (safe) {
            xv[mt] = dev::buffer_load16(rsrc, rel);
          } else {
            xv[mt] = dev::u32x4{0u, 0u, 0u, 0u};
            if (row0 + r < a.n) xv[mt] = dev::load16_guarded(a.x + wbase + rel, a.total_bytes - (wbase + rel));
          }
          if (XT == NB_X_FP8 && k0 + w0 + 16 * q + 16 > a.F) {   // NaN encodings past the last feature
            const int nv = max(0, a.F - (k0 + w0 + 16 * q));
#pragma unroll
            for (int d = 0; d < 4; ++d) {
              const int nb = min(4, max(0, nv - 4 * d));
              xv[mt][d] &= (nb >= 4) ? ~0u : ((1u << (8 * nb)) - 1u);
            }
          }
        }
        dev::u32x4 av[MT][2];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) to_bf16<XT, BIN>(xv[mt], av[mt][0], av[mt][1]);
        // B: class (16 nt + col), features [w0 + 16 q + 8 t, +8)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const uint16_t* tb = tbl + (16 * nt + col) * RS + w0 + 16 * q;
          const dev::u32x4 b0 = *reinterpret_cast<const dev::u32x4*>(tb);
          const dev::u32x4 b1 = *reinterpret_cast<const dev::u32x4*>(tb + 8);
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            acc[mt][nt] = mfma(av[mt][0], b0, acc[mt][nt]);
            acc[mt][nt] = mfma(av[mt][1], b1, acc[mt][nt]);
          }
        }
      }
    }

    epilogue<NT, MT>(a, acc, lane, row0);
  }
}

// Whole-table variant: the BF16 rows of all NT column tiles fit in LDS, so a
// persistent workgroup of kWavesFull waves stages the table once and then
// streams files with no barriers: each wave walks its 16*MT-file tiles in
// groups of KU 64-feature windows, double-buffered (the loads of group g + 1
// are in flight while group g is converted and multiplied).
#ifndef NB_MFMA_WAVES
#define NB_MFMA_WAVES 8
#endif
#ifndef NB_MFMA_KU
#define NB_MFMA_KU 4
#endif
#ifndef NB_MFMA_MT
#define NB_MFMA_MT 2
#endif
constexpr int kWavesFull = NB_MFMA_WAVES;
constexpr int kThreadsFull = 64 * kWavesFull;
constexpr int kKU = NB_MFMA_KU;             // windows per group
constexpr int kMTFull = NB_MFMA_MT;         // 16-file tiles per wave (few column tiles)

template <int XT, int NT, int MT, bool BIN>
__global__ __launch_bounds__(kThreadsFull) void scoreM_full_kernel(ScoreMArgs a) {
  constexpr int NCOL = 16 * NT;
  constexpr int FILES = 16 * MT;
  constexpr int GB = kKU * kWindow;                 // features per group
  extern __shared__ __attribute__((aligned(16))) uint16_t tblf[];   // [NCOL][RS]
  const int RS = a.Fp + 8;

  // stage the whole table (rows >= ns are zero)
  const int pieces_per_row = a.Fp / 8;
  for (int i = threadIdx.x; i < NCOL * pieces_per_row; i += kThreadsFull) {
    const int r = i / pieces_per_row, p = i - r * pieces_per_row;
    dev::u32x4 v = {0u, 0u, 0u, 0u};
    if (r < a.ns) v = *reinterpret_cast<const dev::u32x4*>(a.rows16 + (int64_t)r * a.Fp + 8 * p);
    *reinterpret_cast<dev::u32x4*>(tblf + r * RS + 8 * p) = v;
  }
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int col = lane & 15, q = lane >> 4;
  const int64_t ld = a.ld_bytes;
  const int64_t nwtile = (a.n + FILES - 1) / FILES;                 // wave tiles
  const int64_t nwaves = (int64_t)gridDim.x * kWavesFull;
  const int ngroups = (a.F + GB - 1) / GB;
  uint32_t rel[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) rel[mt] = (uint32_t)((16 * mt + col) * ld) + 16 * q;

  // one wave tile of FILES files; FAST: all rows present and every load in bounds
  auto tile = [&](int64_t row0, auto fast_tag) {
    constexpr bool FAST = decltype(fast_tag)::value;
    f32x4 acc[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    auto load_group = [&](int g, dev::u32x4 (&dst)[kKU][MT]) {
      const int64_t wbase = row0 * ld + (int64_t)g * GB;
      if (FAST) {
        const auto rsrc = dev::make_rsrc(a.x + wbase, a.total_bytes - wbase);
#pragma unroll
        for (int u = 0; u < kKU; ++u)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) dst[u][mt] = dev::buffer_load16(rsrc, rel[mt] + u * kWindow);
        __builtin_amdgcn_sched_barrier(0);
      } else {
#pragma unroll
        for (int u = 0; u < kKU; ++u)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            dst[u][mt] = dev::u32x4{0u, 0u, 0u, 0u};
            const int64_t off = wbase + rel[mt] + u * kWindow;
            if (row0 + 16 * mt + col < a.n) dst[u][mt] = dev::load16_guarded(a.x + off, a.total_bytes - off);
          }
      }
    };
    auto compute_group = [&](int g, dev::u32x4 (&src)[kKU][MT]) {
#pragma unroll
      for (int u = 0; u < kKU; ++u) {
        const int f0 = g * GB + u * kWindow;         // first feature of the window
        dev::u32x4 av[MT][2];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          dev::u32x4 xv = src[u][mt];
          if (XT == NB_X_FP8 && f0 + 16 * q + 16 > a.F) {   // NaN encodings past the last feature
            const int nv = max(0, a.F - (f0 + 16 * q));
#pragma unroll
            for (int d = 0; d < 4; ++d) {
              const int nb = min(4, max(0, nv - 4 * d));
              xv[d] &= (nb >= 4) ? ~0u : ((1u << (8 * nb)) - 1u);
            }
          }
          to_bf16<XT, BIN>(xv, av[mt][0], av[mt][1]);
        }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const uint16_t* tb = tblf + (16 * nt + col) * RS + f0 + 16 * q;
          const dev::u32x4 b0 = *reinterpret_cast<const dev::u32x4*>(tb);
          const dev::u32x4 b1 = *reinterpret_cast<const dev::u32x4*>(tb + 8);
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            acc[mt][nt] = mfma(av[mt][0], b0, acc[mt][nt]);
            acc[mt][nt] = mfma(av[mt][1], b1, acc[mt][nt]);
          }
        }
      }
    };
    dev::u32x4 bufA[kKU][MT], bufB[kKU][MT];
    load_group(0, bufA);
    for (int g = 0; g < ngroups; g += 2) {
      // the prefetch past the last group re-reads the last one (an L2 hit),
      // so every iteration issues the same loads
      load_group(min(g + 1, ngroups - 1), bufB);
      compute_group(g, bufA);
      if (g + 1 >= ngroups) break;
      load_group(min(g + 2, ngroups - 1), bufA);
      compute_group(g + 1, bufB);
    }
    epilogue<NT, MT>(a, acc, lane, row0);
  };

  for (int64_t wt = (int64_t)blockIdx.x * kWavesFull + wave; wt < nwtile; wt += nwaves) {
    const int64_t row0 = wt * FILES;
    const bool full = row0 + FILES <= a.n && (row0 + FILES - 1) * ld + (int64_t)ngroups * GB <= a.total_bytes;
    if (full) tile(row0, std::true_type{});
    else tile(row0, std::false_type{});
  }
}

// Staged variant for one column tile (at most 16 score rows) and Fp <= 4096.
// A wave tile is 16 files; a group is 512 features.  Each group's loads
// read 512 contiguous bytes of each of the 16 files (a wave instruction
// covers 2 files x 512 bytes, eight instructions per group) instead of the
// A-operand layout's 16 files x 64 bytes, and the wave transposes them
// through a private 8 KB LDS stage into the operand layout.  The run length
// per file is what counts on HBM: with the same stage scheme, 128 contiguous
// bytes per file (32 files per tile) held the kernel at 69% of peak, 256
// bytes gave the same, 512 bytes 78%, whatever the waves per CU (8 or 16) or
// the groups in flight (2 to 5); 1024 bytes leave room for only two waves
// per CU.  LDS holds the whole BF16 table (16 rows x Fp, no padding: the
// 16-byte granules of row r are XOR-swizzled by r, so the 16 rows read by
// one B fragment fall in distinct banks) plus the four waves' stages; granule
// p of file r of a stage sits at p ^ (r & 15) (p ^ ((r >> 1) & 7) for
// 128-byte groups), which keeps both the line-shaped writes and the
// operand-shaped reads free of bank conflicts.  Loads run kStageDepth - 1
// groups ahead in registers, across tile boundaries.
constexpr int kStageWaves = 4;
constexpr int kStageThreads = 64 * kStageWaves;
constexpr int kStageMT = 1;                       // 16-file MFMA tiles per wave tile
constexpr int kStageFiles = 16 * kStageMT;        // files per wave tile
constexpr int kStageGB = 512;                     // features (bytes) per file per group
constexpr int kStageWin = kStageGB / kWindow;     // 64-feature windows per group
constexpr int kStageNG = kStageGB / 16;           // 16-byte granules per file per group
constexpr int kStageFPI = 1024 / kStageGB;        // files per wave load instruction
constexpr int kStageLoads = kStageFiles / kStageFPI;   // 16-byte loads per lane per group
constexpr int kStageBytes = kStageFiles * kStageGB;
static_assert(kStageGB >= 128 && kStageGB <= 1024 && kStageFiles % kStageFPI == 0, "stage shape");
constexpr int kStageDepth = 3;
#ifndef NB_USE_STAGE
#define NB_USE_STAGE 1
#endif
constexpr bool kUseStage = NB_USE_STAGE != 0;

__device__ __forceinline__ int stage_granule(int r, int p) {
  return kStageNG == 8 ? r * 8 + (p ^ ((r >> 1) & 7)) : r * kStageNG + (p ^ (r & 15));
}

// Destination of outputs the caller did not request (and of the lanes that
// hold no label): the fast path stores unconditionally so that the number of
// memory operations in flight stays known at compile time.
__device__ int32_t g_stage_sink_label[64];
__device__ float g_stage_sink_post[64 * 16];

template <int XT, bool BIN>
__global__ __launch_bounds__(kStageThreads) void scoreM_stage_kernel(ScoreMArgs a) {
  extern __shared__ __attribute__((aligned(16))) dev::u32x4 lds4[];
  dev::u32x4* tbl = lds4;                                    // [16][Fp / 8] granules, swizzled
  const int gpr = a.Fp / 8;                                  // granules per table row
  // stage the table (rows >= ns are zero)
  for (int i = threadIdx.x; i < 16 * gpr; i += kStageThreads) {
    const int r = i / gpr, g = i - r * gpr;
    dev::u32x4 v = {0u, 0u, 0u, 0u};
    if (r < a.ns) v = *reinterpret_cast<const dev::u32x4*>(a.rows16 + (int64_t)r * a.Fp + 8 * g);
    tbl[r * gpr + (g ^ r)] = v;
  }
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  dev::u32x4* stg = lds4 + 16 * gpr + wave * (kStageBytes / 16);
  const int col = lane & 15, q = lane >> 4;
  const int64_t ld = a.ld_bytes;
  const int64_t wave_id = (int64_t)blockIdx.x * kStageWaves + wave;
  const int64_t nwaves = (int64_t)gridDim.x * kStageWaves;
  const int ngroups = (a.F + kStageGB - 1) / kStageGB;
  const float bias = (col < a.ns) ? a.row_bias[col] : 0.0f;
  // load lane layout: instruction j covers files kStageFPI j + lane / kStageNG,
  // granule lane % kStageNG
  const int lr = lane / kStageNG, lp = lane % kStageNG;
  uint32_t rel[kStageLoads];
#pragma unroll
  for (int j = 0; j < kStageLoads; ++j) rel[j] = (uint32_t)((kStageFPI * j + lr) * ld) + 16 * lp;
  int wpos[kStageLoads];
#pragma unroll
  for (int j = 0; j < kStageLoads; ++j) wpos[j] = stage_granule(kStageFPI * j + lr, lp);
  // operand lane layout: tile mt, window u -> file 16 mt + col, granule 4 u + q
  int rpos[kStageMT][kStageWin];
#pragma unroll
  for (int mt = 0; mt < kStageMT; ++mt)
#pragma unroll
    for (int u = 0; u < kStageWin; ++u) rpos[mt][u] = stage_granule(16 * mt + col, 4 * u + q);

  f32x4 acc[kStageMT][1];
  auto zero_acc = [&]() {
#pragma unroll
    for (int mt = 0; mt < kStageMT; ++mt) acc[mt][0] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  };
  // transpose one group through the stage and multiply it into acc
  auto compute_group = [&](int g, const dev::u32x4 (&src)[kStageLoads]) {
    // the previous group's operand reads are done before the stage is
    // rewritten: LDS operations of a wave complete in order
#pragma unroll
    for (int j = 0; j < kStageLoads; ++j) stg[wpos[j]] = src[j];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int u = 0; u < kStageWin; ++u) {
      const int f0 = g * kStageGB + u * kWindow;         // first feature of the window
      dev::u32x4 av[kStageMT][2];
#pragma unroll
      for (int mt = 0; mt < kStageMT; ++mt) {
        dev::u32x4 xv = stg[rpos[mt][u]];
        if (XT == NB_X_FP8 && f0 + 16 * q + 16 > a.F) {   // NaN encodings past the last feature
          const int nv = max(0, a.F - (f0 + 16 * q));
#pragma unroll
          for (int d = 0; d < 4; ++d) {
            const int nb = min(4, max(0, nv - 4 * d));
            xv[d] &= (nb >= 4) ? ~0u : ((1u << (8 * nb)) - 1u);
          }
        }
        to_bf16<XT, BIN>(xv, av[mt][0], av[mt][1]);
      }
      const int G = (f0 + 16 * q) / 8;                    // table granule of this lane's k-group
      const dev::u32x4 b0 = tbl[col * gpr + (G ^ col)];
      const dev::u32x4 b1 = tbl[col * gpr + ((G + 1) ^ col)];
#pragma unroll
      for (int mt = 0; mt < kStageMT; ++mt) {
        acc[mt][0] = mfma(av[mt][0], b0, acc[mt][0]);
        acc[mt][0] = mfma(av[mt][1], b1, acc[mt][0]);
      }
    }
  };
  // Fast epilogue: 16 classes in the 16 columns, every row present, every
  // store issued (to a sink when the output was not requested).
  const bool want_lab = a.labels != nullptr, want_lp = a.log_post != nullptr;
  auto finish_fast = [&](int64_t row0) {
#pragma unroll
    for (int mt = 0; mt < kStageMT; ++mt) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t row = row0 + 16 * mt + 4 * q + i;
        const float sv = acc[mt][0][i] + bias;
        float m = sv;
        int best = col;
#pragma unroll
        for (int sh = 1; sh < 16; sh <<= 1) {
          const float om = __shfl_xor(m, sh);
          const int ob = __shfl_xor(best, sh);
          if (om > m || (om == m && ob < best)) {
            m = om;
            best = ob;
          }
        }
        float z = __expf(sv - m);
#pragma unroll
        for (int sh = 1; sh < 16; sh <<= 1) z += __shfl_xor(z, sh);
        const float lse = m + __logf(z);
        int32_t* pl = (want_lab && col == 0) ? a.labels + row : g_stage_sink_label + lane;
        float* pp = want_lp ? a.log_post + row * 16 + col : g_stage_sink_post + lane;
        *pl = best;
        *pp = sv - lse;
      }
    }
  };

  // ---- full tiles [0, a.nfast): one pipelined stream of (tile, group)
  // units; loads run kStageDepth - 1 units ahead and cross tile boundaries.
  // The prefetch past the last unit re-reads the last unit (an L2 hit).
  const int my_tiles = (a.nfast > wave_id) ? (int)((a.nfast - wave_id + nwaves - 1) / nwaves) : 0;
  const int units = my_tiles * ngroups;
  auto issue = [&](int k, dev::u32x4 (&dst)[kStageLoads]) {
    k = min(k, units - 1);
    const int it = k / ngroups, g = k - it * ngroups;
    const int64_t wbase = (wave_id + (int64_t)it * nwaves) * kStageFiles * ld + (int64_t)g * kStageGB;
    const auto rsrc = dev::make_rsrc(a.x + wbase, a.total_bytes - wbase);
#pragma unroll
    for (int j = 0; j < kStageLoads; ++j) dst[j] = dev::buffer_load16(rsrc, rel[j]);
    __builtin_amdgcn_sched_barrier(0);
  };
  int cg = 0, ct = 0;
  auto consume = [&](const dev::u32x4 (&src)[kStageLoads]) {
    compute_group(cg, src);
    if (++cg == ngroups) {
      finish_fast((wave_id + (int64_t)ct * nwaves) * kStageFiles);
      zero_acc();
      cg = 0;
      ++ct;
    }
  };
  zero_acc();
  if (units > 0) {
    // kStageDepth register buffers in rotation: unit k + kStageDepth - 1 is
    // issued just before unit k is consumed
    dev::u32x4 buf[kStageDepth][kStageLoads];
#pragma unroll
    for (int d = 0; d < kStageDepth - 1; ++d) issue(d, buf[d]);
    bool done = false;
    for (int k = 0; !done; k += kStageDepth) {
#pragma unroll
      for (int d = 0; d < kStageDepth; ++d) {
        if (!done) {
          issue(k + d + kStageDepth - 1, buf[(d + kStageDepth - 1) % kStageDepth]);
          consume(buf[d]);
          if (k + d + 1 >= units) done = true;
        }
      }
    }
  }

  // ---- remaining tiles: guarded loads, partial rows, generic epilogue
  const int64_t nwtile = (a.n + kStageFiles - 1) / kStageFiles;
  for (int64_t wt = a.nfast + wave_id; wt < nwtile; wt += nwaves) {
    const int64_t row0 = wt * kStageFiles;
    zero_acc();
    for (int g = 0; g < ngroups; ++g) {
      dev::u32x4 v[kStageLoads];
      const int64_t wbase = row0 * ld + (int64_t)g * kStageGB;
#pragma unroll
      for (int j = 0; j < kStageLoads; ++j) {
        v[j] = dev::u32x4{0u, 0u, 0u, 0u};
        const int64_t off = wbase + rel[j];
        if (row0 + kStageFPI * j + lr < a.n) v[j] = dev::load16_guarded(a.x + off, a.total_bytes - off);
      }
      compute_group(g, v);
    }
    epilogue<1, kStageMT>(a, acc, lane, row0);
  }
}

using KernelFn = void (*)(ScoreMArgs);

// column tiles rounded up to a compiled width (extra columns are zero rows)
int round_nt(int nt) { return nt <= 1 ? 1 : nt <= 2 ? 2 : nt <= 4 ? 4 : nt <= 8 ? 8 : nt <= 16 ? 16 : 0; }

template <int XT, int NT>
KernelFn pick_bin(bool bin, bool full) {
  constexpr int MT = (NT >= 8) ? 1 : 2;
  constexpr int MTF = (NT >= 8) ? 1 : (NT >= 4 ? 2 : kMTFull);
  if (full) return bin ? scoreM_full_kernel<XT, NT, MTF, true> : scoreM_full_kernel<XT, NT, MTF, false>;
  return bin ? scoreM_kernel<XT, NT, MT, true> : scoreM_kernel<XT, NT, MT, false>;
}

template <int XT>
KernelFn pick_nt(int ntr, bool bin, bool full) {
  switch (ntr) {
    case 1: return pick_bin<XT, 1>(bin, full);
    case 2: return pick_bin<XT, 2>(bin, full);
    case 4: return pick_bin<XT, 4>(bin, full);
    case 8: return pick_bin<XT, 8>(bin, full);
    case 16: return pick_bin<XT, 16>(bin, full);
    default: return nullptr;
  }
}

int max_lds_per_block() {
  static int v = 0;
  if (v == 0) {
    int dev = 0, b = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&b, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && b > 0)
      v = b;
    else
      v = 64 * 1024;
  }
  return v;
}

}  // namespace

int launch_scoreC_mfma(const nb_model* m, const nb_layout& L, const void* x, int32_t xtype, int64_t n, int64_t ld,
                       int32_t* labels, float* log_post, float* scores, hipStream_t s) {
  const int C = m->n_classes;
  const int ns = C + (scores ? 1 : 0);
  const int ntr = round_nt((ns + 15) / 16);
  if (ntr == 0) return fail(NB_EINVAL, "matrix-core scoring supports up to 256 score columns (255 classes with raw scores)");
  const bool bin = m->kind == NB_BERNOULLI;
  const size_t lds_full = (size_t)16 * ntr * (L.padded_features + 8) * sizeof(uint16_t);
  const bool full = lds_full <= (size_t)max_lds_per_block();
  const int mt = (ntr >= 8) ? 1 : (!full ? 2 : (ntr >= 4 ? 2 : kMTFull));
  KernelFn fn = (xtype == NB_X_U8) ? pick_nt<NB_X_U8>(ntr, bin, full) : pick_nt<NB_X_FP8>(ntr, bin, full);
  const uint8_t* base = static_cast<const uint8_t*>(m->dev);
  ScoreMArgs a;
  a.x = static_cast<const uint8_t*>(x);
  a.ld_bytes = ld;
  a.n = n;
  a.total_bytes = (n - 1) * ld + m->n_features;
  a.rows16 = reinterpret_cast<const uint16_t*>(base + L.off_form_bf16);
  a.row_bias = reinterpret_cast<const float*>(base + L.off_form_bias);
  a.labels = labels;
  a.log_post = log_post;
  a.scores = scores;
  a.F = m->n_features;
  a.Fp = L.padded_features;
  a.C = C;
  a.ns = ns;
  const int64_t files = (int64_t)16 * mt;
  if (files * kWavesFull * a.ld_bytes >= ((int64_t)1 << 31))
    return fail(NB_EINVAL, "row stride too large (a tile of rows must span < 2 GiB)");
  const size_t lds_stage = (size_t)16 * L.padded_features * sizeof(uint16_t) + (size_t)kStageWaves * kStageBytes;
  if (ntr == 1 && C == 16 && !scores && kUseStage && lds_stage <= (size_t)max_lds_per_block()) {
    if ((int64_t)kStageFiles * a.ld_bytes >= ((int64_t)1 << 31))
      return fail(NB_EINVAL, "row stride too large (a tile of rows must span < 2 GiB)");
    {
      // leading tiles whose rows all exist and whose group loads stay in the buffer
      const int64_t span = (int64_t)((a.F + kStageGB - 1) / kStageGB) * kStageGB;
      const int64_t full = n / kStageFiles;
      const int64_t rmax = (a.total_bytes >= span) ? (a.total_bytes - span) / a.ld_bytes : -1;
      a.nfast = std::max<int64_t>(0, std::min(full, (rmax + 1) / kStageFiles));
    }
    const void* sf = (xtype == NB_X_U8) ? (bin ? reinterpret_cast<const void*>(scoreM_stage_kernel<NB_X_U8, true>)
                                                : reinterpret_cast<const void*>(scoreM_stage_kernel<NB_X_U8, false>))
                                        : (bin ? reinterpret_cast<const void*>(scoreM_stage_kernel<NB_X_FP8, true>)
                                                : reinterpret_cast<const void*>(scoreM_stage_kernel<NB_X_FP8, false>));
    NB_HIP_CHECK(hipFuncSetAttribute(sf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_stage));
    const int64_t nwtile = (n + kStageFiles - 1) / kStageFiles;
    const int64_t want = (nwtile + kStageWaves - 1) / kStageWaves;
    const int64_t cap = (int64_t)resident_per_cu(sf, kStageThreads, lds_stage) * device_cu_count();
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min(want, cap));
    void* args[] = {&a};
    NB_HIP_CHECK(hipLaunchKernel(sf, dim3(grid), dim3(kStageThreads), args, lds_stage, s));
    NB_HIP_CHECK(hipGetLastError());
    return NB_OK;
  }
  if (full) {
    NB_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds_full));
    const int64_t nwtile = (n + files - 1) / files;
    const int64_t want = (nwtile + kWavesFull - 1) / kWavesFull;
    const int64_t cap =
        (int64_t)resident_per_cu(reinterpret_cast<const void*>(fn), kThreadsFull, lds_full) * device_cu_count();
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min(want, cap));
    hipLaunchKernelGGL(fn, dim3(grid), dim3(kThreadsFull), lds_full, s, a);
  } else {
    const int64_t per_tile = files * kWaves;
    const int64_t ntile = (n + per_tile - 1) / per_tile;
    const int64_t cap = (int64_t)resident_per_cu(reinterpret_cast<const void*>(fn), kThreads, 0) * device_cu_count();
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min(ntile, cap));
    hipLaunchKernelGGL(fn, dim3(grid), dim3(kThreads), 0, s, a);
  }
  NB_HIP_CHECK(hipGetLastError());
  return NB_OK;
}

}  // namespace nb
