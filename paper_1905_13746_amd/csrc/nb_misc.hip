// Feature quantiser (counts -> FP8-e4m3 bytes) and the HBM read-bandwidth
// probe used by the measurements.
#include <algorithm>

#include "nb_device.hpp"
#include "nb_internal.hpp"

namespace nb {
namespace {

// OCP FP8 E4M3 (e4m3fn) encoding of an integer count v in [0, 240], rounded
// to nearest, ties to even: exponent bias 7, three stored significand bits.
// Integers up to 16 are exact; above, the significand keeps 4 bits.
__device__ __forceinline__ uint32_t e4m3_from_count(uint32_t v) {
  if (v == 0) return 0;
  int e = 31 - __clz(v);                  // floor(log2 v), 0..7
  uint32_t q;
  if (e <= 3) {
    q = v << (3 - e);                     // exact
  } else {
    const int sh = e - 3;
    q = v >> sh;
    const uint32_t rem = v & ((1u << sh) - 1u), half = 1u << (sh - 1);
    if (rem > half || (rem == half && (q & 1u))) ++q;
    if (q == 16u) {
      q = 8u;
      ++e;
    }
  }
  return ((uint32_t)(e + 7) << 3) | (q & 7u);
}

__global__ __launch_bounds__(256) void quantize_fp8_kernel(const uint8_t* __restrict__ x, int64_t n, int F,
                                                          int64_t ld_x, uint8_t* __restrict__ out,
                                                          int64_t ld_out) {
  const int64_t total = n * (int64_t)F;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / F, f = i - r * F;
    const uint32_t v = min((uint32_t)x[r * ld_x + f], 240u);
    out[r * ld_out + f] = (uint8_t)e4m3_from_count(v);
  }
}

constexpr int kProbeBlocks = 4096;

__global__ __launch_bounds__(256) void probe_read_kernel(const dev::u32x4* __restrict__ src, int64_t n16,
                                                        uint32_t* __restrict__ sink) {
  uint32_t acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
       i += (int64_t)gridDim.x * blockDim.x) {
    const dev::u32x4 v = __builtin_nontemporal_load(src + i);
    acc ^= v[0] ^ v[1] ^ v[2] ^ v[3];
  }
  __shared__ uint32_t red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] ^= red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) sink[blockIdx.x] = red[0];
}

}  // namespace
}  // namespace nb

using namespace nb;

extern "C" {

int nb_quantize_fp8(const uint8_t* x, int64_t n, int32_t F, int64_t ld_x, uint8_t* out, int64_t ld_out,
                    void* stream) {
  if (n < 0 || F < 1) return fail(NB_EINVAL, "n >= 0 and n_features >= 1 required");
  if (n == 0) return NB_OK;
  if (!x || !out) return fail(NB_EINVAL, "NULL argument");
  if (ld_x < F || ld_out < F) return fail(NB_EINVAL, "strides must be >= n_features");
  const int64_t total = n * (int64_t)F;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(quantize_fp8_kernel, dim3((unsigned)blocks), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), x, n, F, ld_x, out, ld_out);
  NB_HIP_CHECK(hipGetLastError());
  return NB_OK;
}

int32_t nb_probe_sink_words(void) { return kProbeBlocks; }

int nb_probe_read(const void* src, int64_t bytes, uint32_t* sink, void* stream) {
  if (!src || !sink) return fail(NB_EINVAL, "NULL argument");
  if (bytes <= 0 || bytes % 16 != 0) return fail(NB_EINVAL, "bytes must be a positive multiple of 16");
  if ((reinterpret_cast<uintptr_t>(src) & 15) != 0) return fail(NB_EINVAL, "src must be 16-byte aligned");
  hipLaunchKernelGGL(probe_read_kernel, dim3(kProbeBlocks), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                     static_cast<const dev::u32x4*>(src), bytes / 16, sink);
  NB_HIP_CHECK(hipGetLastError());
  return NB_OK;
}

}  // extern "C"
