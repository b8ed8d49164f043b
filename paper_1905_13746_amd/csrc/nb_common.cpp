// Host-side helpers of libnbgpu: error reporting, model layout, size-group
// routing and the version string.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "nb_internal.hpp"

namespace nb {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return NB_EHIP;
}

int elem_bytes(int32_t xtype) {
  switch (xtype) {
    case NB_X_U8: return 1;
    case NB_X_FP8: return 1;
    case NB_X_I32: return 4;
    default: return 0;
  }
}

bool compute_layout(int32_t C, int32_t F, nb_layout* L) {
  if (C < 2 || C > kMaxClasses || F < 1 || F > kMaxFeatures) return false;
  std::memset(L, 0, sizeof(*L));
  const size_t Fp = align_up((size_t)F, kFeaturePad);
  const size_t P = (C == 2) ? 1 : (size_t)C;
  const size_t CF = (size_t)C * F;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off = align_up(off + bytes, kAlign);
    return at;
  };
  L->padded_features = (int32_t)Fp;
  L->form_rows = (int32_t)P;
  L->off_status = take(16);
  L->off_class_totals = take(8 * (size_t)C);
  L->off_class_sums = take(8 * (size_t)C);
  L->off_counts = take(4 * CF);
  L->off_log_theta = take(8 * CF);
  L->off_log_1m_theta = take(8 * CF);
  L->off_weight = take(8 * CF);
  L->off_bias = take(8 * (size_t)C);
  L->off_form_f32 = take(4 * (P + 1) * Fp);
  L->off_form_bf16 = take(2 * (P + 1) * Fp);
  L->off_form_bias = take(4 * (P + 1));
  L->off_sumsq = take(8 * CF);
  L->off_mean = take(8 * CF);
  L->off_var = take(8 * CF);
  L->off_form2_f32 = take(4 * (P + 1) * Fp);
  L->off_form2_bf16 = take(2 * (P + 1) * Fp);
  L->off_epsilon = take(8);
  L->total_bytes = off;
  return true;
}

int check_model(const nb_model* m, nb_layout* L) {
  if (!m) return fail(NB_EINVAL, "model is NULL");
  if (!m->dev) return fail(NB_EINVAL, "model->dev is NULL");
  if ((reinterpret_cast<uintptr_t>(m->dev) & (kAlign - 1)) != 0)
    return fail(NB_EINVAL, "model->dev must be 256-byte aligned");
  if (m->kind != NB_MULTINOMIAL && m->kind != NB_BERNOULLI && m->kind != NB_GAUSSIAN)
    return fail(NB_EINVAL, "model->kind must be NB_MULTINOMIAL, NB_BERNOULLI or NB_GAUSSIAN");
  if (!compute_layout(m->n_classes, m->n_features, L))
    return fail(NB_EINVAL, "model class/feature count out of range (C in [2,256], F in [1,2^20])");
  return NB_OK;
}

int device_cu_count() {
  static std::mutex mu;
  static std::vector<int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  std::lock_guard<std::mutex> lk(mu);
  if ((int)cache.size() <= dev) cache.resize(dev + 1, 0);
  if (cache[dev] == 0) {
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0)
      cu = 256;
    cache[dev] = cu;
  }
  return cache[dev];
}

void route_trained(const char* trained, int32_t n_groups, int32_t* route) {
  // next trained group above; scan from the top so each lookup is O(1)
  int32_t next = -1;
  for (int32_t g = n_groups - 1; g >= 0; --g) {
    if (trained[g]) next = g;
    route[g] = next;
  }
  int32_t prev = -1;
  for (int32_t g = 0; g < n_groups; ++g) {
    if (trained[g]) prev = g;
    if (route[g] < 0) route[g] = prev;   // none above: nearest below
  }
}

int resident_per_cu(const void* fn, int threads, size_t lds) {
  static std::mutex mu;
  static std::map<std::tuple<const void*, int, size_t>, int> cache;
  std::lock_guard<std::mutex> lk(mu);
  const auto key = std::make_tuple(fn, threads, lds);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int per = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, threads, lds) != hipSuccess || per < 1) per = 1;
  cache[key] = per;
  return per;
}

}  // namespace nb

extern "C" {

const char* nb_version(void) { return "libnbgpu 0.1 (gfx950)"; }

const char* nb_last_error(void) { return nb::g_last_error.c_str(); }

size_t nb_model_bytes(int32_t n_classes, int32_t n_features) {
  nb_layout L;
  if (!nb::compute_layout(n_classes, n_features, &L)) return 0;
  return L.total_bytes;
}

int nb_model_layout(int32_t n_classes, int32_t n_features, nb_layout* out) {
  if (!out) return nb::fail(NB_EINVAL, "out is NULL");
  if (!nb::compute_layout(n_classes, n_features, out))
    return nb::fail(NB_EINVAL, "class/feature count out of range (C in [2,256], F in [1,2^20])");
  return NB_OK;
}

int nb_route_groups(const int64_t* class_counts_host, int32_t n_groups, int32_t n_classes,
                    int32_t min_files, int32_t* route_host) {
  if (!class_counts_host || !route_host) return nb::fail(NB_EINVAL, "NULL argument");
  if (n_groups < 1 || n_classes < 1 || min_files < 0)
    return nb::fail(NB_EINVAL, "n_groups >= 1, n_classes >= 1, min_files >= 0 required");
  std::vector<char> trained(n_groups);
  bool any = false;
  for (int32_t g = 0; g < n_groups; ++g) {
    int64_t lo = INT64_MAX;
    for (int32_t c = 0; c < n_classes; ++c)
      lo = std::min(lo, class_counts_host[(size_t)g * n_classes + c]);
    trained[g] = lo >= min_files;
    any = any || trained[g];
  }
  if (!any) return nb::fail(NB_ENOMODEL, "no size group has enough files in every class");
  nb::route_trained(trained.data(), n_groups, route_host);
  return NB_OK;
}

}  // extern "C"
