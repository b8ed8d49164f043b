// Grouped two-class scoring that allocates no device memory.
//
// nb_score_groups takes its work list (group descriptors, items, counters)
// in a caller workspace.  Callers that may not allocate device memory use
// nb_score_groups_static instead: the work list goes to `scratch`, a fixed
// array of this library in device memory (one copy per device, resident
// until the process ends).  The kernels are those of nb_score_groups; only
// the home of the work list differs, so outputs are bit-identical.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "nb_internal.hpp"

// Work list of the most recent nb_score_groups_static call on each device.
static __device__ __align__(256) uint8_t scratch[NB_SCORE_GROUPS_STATIC_MAX_BYTES];

namespace nb {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`.  The array's
// name in host code is only a handle for the runtime; every copy and launch
// uses the address resolved here, once per device.
int scratch_on_current_device(void** out) {
  int dev = -1;
  NB_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(NB_EINVAL, "device ordinal outside the library's device table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(NB_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return NB_OK;
}

}  // namespace
}  // namespace nb

using namespace nb;

extern "C" int nb_score_groups_static(const nb_model* models, int32_t n_models, const nb_group* groups,
                                      int32_t n_groups, int32_t xtype, int32_t wtype, int32_t tile_rows,
                                      void* stream) {
  // host staging of the work list, reused by later calls on this thread
  thread_local std::vector<uint8_t> blob;
  GroupLaunch L;
  int rc = prepare_group_launch(models, n_models, groups, n_groups, xtype, wtype, tile_rows, &blob, &L);
  if (rc) return rc;
  if (L.total_blocks == 0) return NB_OK;
  if (blob.size() > (size_t)NB_SCORE_GROUPS_STATIC_MAX_BYTES)
    return fail(NB_ENOMEM, "the work list (" + std::to_string(blob.size()) + " bytes) exceeds the " +
                               std::to_string((size_t)NB_SCORE_GROUPS_STATIC_MAX_BYTES) +
                               "-byte static array: use nb_score_groups with a workspace");
  void* dev = nullptr;
  if ((rc = scratch_on_current_device(&dev))) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // the copy also zeroes the dynamic schedule's counters (the image holds
  // them as zero), so the array's previous contents never matter
  NB_HIP_CHECK(hipMemcpyAsync(dev, blob.data(), blob.size(), hipMemcpyHostToDevice, s));
  if ((rc = enqueue_group_launch(L, dev, s))) return rc;
  // the array is reused by the next call and the image sits in pageable
  // host memory: return only once the launch has completed
  NB_HIP_CHECK(hipStreamSynchronize(s));
  return NB_OK;
}
