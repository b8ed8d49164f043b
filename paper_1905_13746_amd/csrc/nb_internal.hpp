// Internal declarations shared by the libnbgpu translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "nb.h"

namespace nb {

// ------------------------------------------------------------------ errors
// Thread-local last-error message behind nb_last_error().
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define NB_HIP_CHECK(call)                                   \
  do {                                                       \
    hipError_t e_ = (call);                                  \
    if (e_ != hipSuccess) return ::nb::hip_fail(e_, #call);  \
  } while (0)

// ------------------------------------------------------------------ layout
constexpr int kMaxClasses = 256;
constexpr int kMaxFeatures = 1 << 20;
constexpr int kFeaturePad = 1024;    // scoring rows padded to this many features
constexpr size_t kAlign = 256;

// Status block (int32 words at off_status).
enum StatusWord { kStatusFlags = 0, kStatusTrained = 1 };
// Device-detected training errors, OR-ed into the status flags word.
enum StatusFlag : int32_t {
  kFlagBadLabel = 1,      // label outside [0, C)
  kFlagNegative = 2,      // negative feature value
  kFlagOverflow = 4,      // count above INT32_MAX
  kFlagMinFiles = 8,      // class below the minimum number of files
  kFlagBadIndex = 16,     // feature index outside [0, F) (nb_model_select)
  kFlagZeroVariance = 32, // Gaussian: every training file identical (all variances 0)
};

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

bool compute_layout(int32_t C, int32_t F, nb_layout* L);
int check_model(const nb_model* m, nb_layout* L);
int elem_bytes(int32_t xtype);

// Number of compute units of the current device (cached per device).
int device_cu_count();
// Size-group fallback (sections 3-4): route[g] = g if trained[g], else the
// first trained group above g, else the nearest trained group below; -1 if
// no group is trained.
void route_trained(const char* trained, int32_t n_groups, int32_t* route);

// Resident workgroups per CU of a kernel at a block size and dynamic LDS
// (at least 1; cached).
int resident_per_cu(const void* fn, int threads, size_t lds);

// Argument checks of nb_score (also applied to every group of
// nb_score_groups); fills *L.  NB_OK for n == 0 once the model and types are valid.
int check_score_args(const nb_model* m, nb_layout* L, const void* x, int32_t xtype, int64_t n, int64_t ld,
                     int32_t wtype, const int32_t* labels, const float* log_post, const float* scores);

// Scoring launchers for more than two classes (arguments validated by nb_score).
int launch_scoreC_valu(const nb_model* m, const nb_layout& L, const void* x, int32_t xtype, int64_t n, int64_t ld,
                       int32_t wtype, int32_t* labels, float* log_post, float* scores, hipStream_t s);
int launch_scoreC_mfma(const nb_model* m, const nb_layout& L, const void* x, int32_t xtype, int64_t n, int64_t ld,
                       int32_t* labels, float* log_post, float* scores, hipStream_t s);

// Bytes reserved per group descriptor when bounding work-list sizes.
constexpr size_t kGroupDescBound = 256;

// One grouped two-class launch prepared on the host (nb_groups.hip): the
// device image of its work list goes to a 256-byte aligned device buffer of
// blob_bytes, then enqueue_group_launch launches it (serving reuses this).
struct GroupLaunch {
  const void* fn = nullptr;
  size_t lds = 0;
  int32_t grid = 0;
  int32_t kind = 0;            // schedule: 0 static ranges, 1 dynamic items, 2 stream, 3 sweep
  int32_t n_items = 0;
  int32_t n_tails = 0;
  int32_t n_groups = 0;
  int32_t Fp = 0;
  int32_t nch = 0;
  int32_t F = 0;
  int32_t wt = 0;
  int64_t total_blocks = 0;
  int64_t sweep_blocks = 0;    // sweep: blocks of the sweep (the rest are tails)
  size_t blob_bytes = 0;
};
int prepare_group_launch(const nb_model* models, int32_t n_models, const nb_group* groups, int32_t n_groups,
                         int32_t xtype, int32_t wtype, int32_t tile_rows, std::vector<uint8_t>* blob,
                         GroupLaunch* out);
int enqueue_group_launch(const GroupLaunch& L, void* dev_blob, hipStream_t s);

}  // namespace nb
