// Internal declarations shared by the libnbgpu translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

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
};

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

bool compute_layout(int32_t C, int32_t F, nb_layout* L);
int check_model(const nb_model* m, nb_layout* L);
int elem_bytes(int32_t xtype);

// Number of compute units of the current device (cached per device).
int device_cu_count();

// Scoring launchers for more than two classes (arguments validated by nb_score).
int launch_scoreC_valu(const nb_model* m, const nb_layout& L, const void* x, int32_t xtype, int64_t n, int64_t ld,
                       int32_t wtype, int32_t* labels, float* log_post, float* scores, hipStream_t s);
int launch_scoreC_mfma(const nb_model* m, const nb_layout& L, const void* x, int32_t xtype, int64_t n, int64_t ld,
                       int32_t* labels, float* log_post, float* scores, hipStream_t s);

}  // namespace nb
