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
// stretch of a row) contiguously.  A wave processes R row-steps of
// 64/LPR rows per block (R = 16 for byte features; 8 for int32 features and
// the Gaussian kernel) and strides over blocks (persistent grid sized to the
// resident capacity).  The table row(s) sit in LDS as FP32 (BF16 tables are
// widened on load: exact).  Lane partial sums are reduced across the LPR
// lanes with a transposed butterfly (each exchange step halves the number of
// values per lane), staged in LDS and handed to one lane per file for the
// fused epilogue: label, log-sum-exp, log posteriors, raw scores.
//
// Summation order of a file depends only on (F, xtype): lanes sum their 16
// features in order, chunks in order, then the fixed butterfly.  It never
// depends on n, on the block a file lands in, or on other files.
#include "nb_score2.hpp"

namespace nb {
namespace {

template <int XT, int LPR, int NS, bool BIN, bool MULTI, bool QUAD = false, int FL = 0>
__global__ __launch_bounds__(kThreads) void score2_kernel(Score2Args a) {
  // [NS][Fp] (Gaussian: [4][Fp], means then h); with flat staging, then the
  // waves' staging regions (kWaves x FL KB)
  extern __shared__ float tbl[];
  __shared__ float stage[kWaves][NS][(64 / LPR) * block_steps<XT, QUAD, MULTI, FL>()];
  if constexpr (QUAD) stage_table_q(a, tbl);
  else stage_table<NS>(a, tbl);
  __syncthreads();
  constexpr int BR = (64 / LPR) * block_steps<XT, QUAD, MULTI, FL>();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t wave_id = (int64_t)blockIdx.x * kWaves + wave;
  const int64_t nwaves = (int64_t)gridDim.x * kWaves;
  const int64_t nblk = (a.n + BR - 1) / BR;
  uint8_t* flat = FL ? reinterpret_cast<uint8_t*>(tbl) + (size_t)NS * a.Fp * sizeof(float) : nullptr;
  score_blocks<XT, LPR, NS, BIN, MULTI, QUAD, FL>(a, tbl, wave_id, nwaves, nblk, stage, flat);
}

struct Single {
  template <int XT, int LPR, int NS, bool BIN, bool MULTI, int FL = 0>
  static const void* fn() {
    return reinterpret_cast<const void*>(score2_kernel<XT, LPR, NS, BIN, MULTI, false, FL>);
  }
};

// Gaussian two-class kernels (uint8 and int32 features).
template <int XT, int NS>
const void* pick_quad_lpr(int lpr, bool multi) {
  switch (lpr) {
    case 4: return reinterpret_cast<const void*>(score2_kernel<XT, 4, NS, false, false, true>);
    case 8: return reinterpret_cast<const void*>(score2_kernel<XT, 8, NS, false, false, true>);
    case 16: return reinterpret_cast<const void*>(score2_kernel<XT, 16, NS, false, false, true>);
    case 32: return reinterpret_cast<const void*>(score2_kernel<XT, 32, NS, false, false, true>);
    default:
      return multi ? reinterpret_cast<const void*>(score2_kernel<XT, 64, NS, false, true, true>)
                   : reinterpret_cast<const void*>(score2_kernel<XT, 64, NS, false, false, true>);
  }
}

const void* pick_quad(int xtype, int lpr, bool multi, int ns) {
  if (xtype == NB_X_I32) return ns == 1 ? pick_quad_lpr<NB_X_I32, 1>(lpr, multi) : pick_quad_lpr<NB_X_I32, 2>(lpr, multi);
  return ns == 1 ? pick_quad_lpr<NB_X_U8, 1>(lpr, multi) : pick_quad_lpr<NB_X_U8, 2>(lpr, multi);
}

int launch_score2(const nb_model* m, const nb_layout& L, const void* x, int32_t xtype, int64_t n, int64_t ld,
                  int32_t wtype, int32_t* labels, float* log_post, float* scores, hipStream_t s) {
  const int ns = scores ? 2 : 1;
  const bool quad = (m->kind == NB_GAUSSIAN);
  Score2Args a;
  const int fl = quad ? 0 : flat_pieces(xtype, m->n_features, ld * elem_bytes(xtype), x, false);
  const int rc = make_score2_args(m, L, x, xtype, n, ld, wtype, labels, log_post, scores, ns, &a, quad, fl);
  if (rc) return rc;
  const int lpr = lanes_per_row(a.F);
  const size_t lds = (size_t)(quad ? 4 : ns) * a.Fp * sizeof(float) + (fl ? (size_t)kWaves * flat_region_bytes(fl) : 0);
  const void* fn = quad ? pick_quad(xtype, lpr, a.nch > 1, ns)
                        : pick_score2<Single>(xtype, lpr, a.nch > 1, ns, m->kind == NB_BERNOULLI, fl);
  if (lds > 64 * 1024) NB_HIP_CHECK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  const int64_t rows_per_blk = (int64_t)(64 / lpr) * block_steps_of(xtype, quad, a.nch, fl);
  const int64_t nblk = (n + rows_per_blk - 1) / rows_per_blk;
  const int64_t want = (nblk + kWaves - 1) / kWaves;
  const int64_t cap = (int64_t)resident_per_cu(fn, kThreads, lds) * device_cu_count();
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min(want, cap));
  void* args[] = {&a};
  NB_HIP_CHECK(hipLaunchKernel(fn, dim3(grid), dim3(kThreads), args, lds, s));
  NB_HIP_CHECK(hipGetLastError());
  return NB_OK;
}

}  // namespace

int check_score_args(const nb_model* m, nb_layout* L, const void* x, int32_t xtype, int64_t n, int64_t ld,
                     int32_t wtype, const int32_t* labels, const float* log_post, const float* scores) {
  int rc = check_model(m, L);
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
  return NB_OK;
}

}  // namespace nb

using namespace nb;

extern "C" int nb_score(const nb_model* m, const void* x, int32_t xtype, int64_t n, int64_t ld, int32_t wtype,
                        int32_t* labels, float* log_post, float* scores, void* stream) {
  nb_layout L;
  int rc = check_score_args(m, &L, x, xtype, n, ld, wtype, labels, log_post, scores);
  if (rc || n == 0) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (m->kind == NB_GAUSSIAN && (m->n_classes != 2 || xtype == NB_X_FP8))
    return fail(NB_EINVAL, "Gaussian models score two classes with uint8 or int32 features");
  if (m->n_classes == 2) return launch_score2(m, L, x, xtype, n, ld, wtype, labels, log_post, scores, s);
  // BF16 tables with a full column tile of classes go to the matrix cores;
  // everything else (the FP32 plain path, fewer classes, int32 features) to
  // the vector ALUs
  if (wtype == NB_W_BF16 && m->n_classes >= 16 && xtype != NB_X_I32)
    return launch_scoreC_mfma(m, L, x, xtype, n, ld, labels, log_post, scores, s);
  return launch_scoreC_valu(m, L, x, xtype, n, ld, wtype, labels, log_post, scores, s);
}
