// Naive Bayes scoring for more than two classes on the vector ALUs
// (paper, section 4: the class with the highest posterior wins; here C >= 3,
// e.g. malware families).  Used for the FP32 table (the plain path) and for
// BF16 tables with fewer than 16 classes.
//
// The kernel contracts each file against the P = C class-centred rows
// W_c - mean_c W (posteriors depend on score differences only; the centred
// rows are smaller, so FP32 sums lose less) and, when raw scores are
// requested, the aux row mean_c W that restores s_c.  Each lane owns ONE file:
// all lanes of a wave step through the same feature at the same time, so the
// table value of (feature, class) is the same for the whole wave and comes
// from LDS as a broadcast read, while the FMA count per feature byte is the
// number of rows.  Feature bytes are staged per wave through LDS: a coalesced
// load of 64 files x 64 bytes, then each lane reads its own file's 64 bytes.
// The table is staged in LDS in slices of kSlice features, transposed to
// feature-major.  Sums are two-level: 64-byte sub-steps accumulate into an
// inner partial that is added to the running total, so no term passes
// through more than 64 + F/64 roundings (the error depth used by the tests).
#include <algorithm>
#include <map>
#include <mutex>

#include "nb_device.hpp"
#include "nb_internal.hpp"

namespace nb {
namespace {

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kStepBytes = 64;      // bytes of each file per sub-step
constexpr int kSlice = 512;         // table features staged per slice
constexpr int kRowPad = 16;         // LDS row padding (bank spread)
constexpr int kXRow = kStepBytes + kRowPad;

struct ScoreCArgs {
  const uint8_t* x;
  int64_t ld_bytes;
  int64_t n;
  int64_t total_bytes;
  const float* rows32;       // [P+1][Fp] class-major scoring rows
  const uint16_t* rows16;    // same, BF16
  const float* row_bias;     // [P+1]
  int32_t* labels;
  float* log_post;
  float* scores;
  int32_t F, Fp, C, wt;
  int32_t ns;                // rows used: C, or C + 1 with the aux row (index C)
};

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// NS: sums per file, >= a.ns (C centred rows, plus the aux row when raw
// scores are requested; extra sums see zero rows); TS: LDS stride of a
// feature's table entries (NS rounded up to 4).
template <int XT, int NS, bool BIN>
__global__ __launch_bounds__(kThreads) void scoreC_kernel(ScoreCArgs a) {
  constexpr int EB = (XT == NB_X_I32) ? 4 : 1;
  constexpr int KS = kStepBytes / EB;          // features per sub-step
  constexpr int TS = (NS + 3) / 4 * 4;
  __shared__ float tbl[kSlice * TS];
  __shared__ __attribute__((aligned(16))) uint8_t xs[kWaves][64 * kXRow];

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int C = a.C;
  const int64_t ld = a.ld_bytes;
  const int64_t ntile = (a.n + kThreads - 1) / kThreads;

  for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const int64_t row0 = tile * kThreads + wave * 64;     // this wave's 64 files
    float acc[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) acc[s] = 0.0f;

    for (int k0 = 0; k0 < a.F; k0 += kSlice) {
      const int kn = min(kSlice, a.Fp - k0);
      __syncthreads();   // previous slice fully consumed
      for (int i = threadIdx.x; i < kn * NS; i += kThreads) {
        const int s = i / kn, f = i - s * kn;
        const int64_t src = (int64_t)s * a.Fp + k0 + f;
        tbl[f * TS + s] = (s >= a.ns) ? 0.0f : (a.wt == NB_W_BF16) ? dev::bf16_to_f32(a.rows16[src]) : a.rows32[src];
      }
      __syncthreads();
      const int kend = min(kn, a.F - k0);
      for (int ks = 0; ks < kend; ks += KS) {
        // stage 64 files x 64 bytes: piece p = lane + 64 t -> (row p/4, 16-byte column p%4);
        // one wave-uniform buffer resource per sub-step, per-lane 32-bit offsets
        const int64_t wbase = row0 * ld + (int64_t)(k0 + ks) * EB;
        const auto rsrc = dev::make_rsrc(a.x + wbase, a.total_bytes - wbase);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int p = lane + 64 * t;
          const int r = p >> 2, c16 = p & 3;
          const int64_t row = row0 + r;
          dev::u32x4 v = {0u, 0u, 0u, 0u};
          if (row < a.n) {
            const int64_t rel = (int64_t)r * ld + 16 * c16;
            if (wbase + rel + 16 <= a.total_bytes) {
              v = dev::buffer_load16(rsrc, (uint32_t)rel);
            } else {
              v = dev::load16_guarded(a.x + wbase + rel, a.total_bytes - (wbase + rel));
            }
          }
          *reinterpret_cast<dev::u32x4*>(&xs[wave][r * kXRow + 16 * c16]) = v;
        }
        wave_lds_sync();
        dev::u32x4 mine[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) mine[q] = *reinterpret_cast<const dev::u32x4*>(&xs[wave][lane * kXRow + 16 * q]);
        wave_lds_sync();
        // FP8 bytes past the last feature may encode NaN: clear them
        const int nvalid = min(KS, a.F - (k0 + ks));
        if (XT == NB_X_FP8 && nvalid < KS) {
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int d = 0; d < 4; ++d) {
              const int b0 = 16 * q + 4 * d;
              const int nb = min(4, max(0, nvalid - b0));
              mine[q][d] &= (nb >= 4) ? ~0u : ((1u << (8 * nb)) - 1u);
            }
        }
        float inner[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) inner[s] = 0.0f;
        const float* tb = tbl + ks * TS;
#pragma unroll
        for (int e = 0; e < KS; ++e) {
          float g;
          if (XT == NB_X_I32) {
            g = (float)(int32_t)mine[e >> 2][e & 3];
          } else if (XT == NB_X_U8) {
            g = (float)((mine[e >> 4][(e >> 2) & 3] >> (8 * (e & 3))) & 0xFFu);
          } else {
            const uint32_t w = mine[e >> 4][(e >> 2) & 3];
            g = ((e & 2) ? __builtin_amdgcn_cvt_pk_f32_fp8(w, true) : __builtin_amdgcn_cvt_pk_f32_fp8(w, false))[e & 1];
          }
          // presence: a clamp to [0, 1] for integer counts (folds into the
          // conversion), a compare for FP8 values
          if (BIN) g = (XT == NB_X_FP8) ? (g > 0.0f ? 1.0f : 0.0f) : __builtin_amdgcn_fmed3f(g, 0.0f, 1.0f);
          const float* te = tb + e * TS;
#pragma unroll
          for (int s4 = 0; s4 < TS; s4 += 4) {
            const float4 w4 = *reinterpret_cast<const float4*>(te + s4);
            if (s4 + 0 < NS) inner[s4 + 0] = fmaf(g, w4.x, inner[s4 + 0]);
            if (s4 + 1 < NS) inner[s4 + 1] = fmaf(g, w4.y, inner[s4 + 1]);
            if (s4 + 2 < NS) inner[s4 + 2] = fmaf(g, w4.z, inner[s4 + 2]);
            if (s4 + 3 < NS) inner[s4 + 3] = fmaf(g, w4.w, inner[s4 + 3]);
          }
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) acc[s] += inner[s];
      }
    }

    // epilogue: one file per lane
    const int64_t row = row0 + lane;
    if (row < a.n) {
      float sc[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) sc[s] = acc[s] + a.row_bias[s];
      float m = -INFINITY;
      int best = 0;
#pragma unroll
      for (int s = 0; s < NS; ++s)
        if (s < C && sc[s] > m) {
          m = sc[s];
          best = s;
        }
      float z = 0.0f;
#pragma unroll
      for (int s = 0; s < NS; ++s)
        if (s < C) z += __expf(sc[s] - m);
      const float lse = m + __logf(z);
      if (a.labels) a.labels[row] = best;
      if (a.log_post) {
#pragma unroll
        for (int s = 0; s < NS; ++s)
          if (s < C) a.log_post[row * C + s] = sc[s] - lse;
      }
      if (a.scores && a.ns > C) {
        float aux = 0.0f;
#pragma unroll
        for (int s = 0; s < NS; ++s)
          if (s == C) aux = sc[s];
#pragma unroll
        for (int s = 0; s < NS; ++s)
          if (s < C) a.scores[row * C + s] = sc[s] + aux;
      }
    }
  }
}

using KernelFn = void (*)(ScoreCArgs);

template <int XT, int NS>
KernelFn pick_bin(bool bin) {
  return bin ? scoreC_kernel<XT, NS, true> : scoreC_kernel<XT, NS, false>;
}

template <int XT>
KernelFn pick_ns(int ns, bool bin) {
  // sums per file rounded up to a compiled width (extra rows are zero)
  if (ns <= 4) return pick_bin<XT, 4>(bin);
  if (ns <= 8) return pick_bin<XT, 8>(bin);
  if (ns <= 12) return pick_bin<XT, 12>(bin);
  if (ns <= 16) return pick_bin<XT, 16>(bin);
  if (ns <= 17) return pick_bin<XT, 17>(bin);
  if (ns <= 20) return pick_bin<XT, 20>(bin);
  if (ns <= 24) return pick_bin<XT, 24>(bin);
  if (ns <= 32) return pick_bin<XT, 32>(bin);
  return nullptr;
}

}  // namespace

// Entry from nb_score for C >= 3 on the vector ALUs.  Arguments are validated
// by the caller.
int launch_scoreC_valu(const nb_model* m, const nb_layout& L, const void* x, int32_t xtype, int64_t n, int64_t ld,
                       int32_t wtype, int32_t* labels, float* log_post, float* scores, hipStream_t s) {
  const int C = m->n_classes;
  const int ns = C + (scores ? 1 : 0);
  KernelFn fn = nullptr;
  const bool bin = m->kind == NB_BERNOULLI;
  switch (xtype) {
    case NB_X_U8: fn = pick_ns<NB_X_U8>(ns, bin); break;
    case NB_X_I32: fn = pick_ns<NB_X_I32>(ns, bin); break;
    default: fn = pick_ns<NB_X_FP8>(ns, bin); break;
  }
  if (!fn)
    return fail(NB_EINVAL, "vector-ALU scoring supports up to 31 classes (32 with raw scores); "
                           "use the BF16 table (matrix cores) for more");
  const int eb = elem_bytes(xtype);
  const uint8_t* base = static_cast<const uint8_t*>(m->dev);
  ScoreCArgs a;
  a.x = static_cast<const uint8_t*>(x);
  a.ld_bytes = ld * eb;
  // a wave stages 64 rows through one buffer resource with 32-bit offsets
  if ((int64_t)64 * a.ld_bytes >= ((int64_t)1 << 31))
    return fail(NB_EINVAL, "row stride too large (64 rows must span < 2 GiB)");
  a.n = n;
  a.total_bytes = ((n - 1) * ld + m->n_features) * (int64_t)eb;
  a.rows32 = reinterpret_cast<const float*>(base + L.off_form_f32);
  a.rows16 = reinterpret_cast<const uint16_t*>(base + L.off_form_bf16);
  a.row_bias = reinterpret_cast<const float*>(base + L.off_form_bias);
  // with raw scores the aux row (index C) follows the C centred rows
  a.labels = labels;
  a.log_post = log_post;
  a.scores = scores;
  a.F = m->n_features;
  a.Fp = L.padded_features;
  a.C = C;
  a.wt = wtype;
  a.ns = ns;
  const int64_t ntile = (n + kThreads - 1) / kThreads;
  const int64_t cap = (int64_t)resident_per_cu(reinterpret_cast<const void*>(fn), kThreads, 0) * device_cu_count();
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min(ntile, cap));
  hipLaunchKernelGGL(fn, dim3(grid), dim3(kThreads), 0, s, a);
  NB_HIP_CHECK(hipGetLastError());
  return NB_OK;
}

}  // namespace nb
