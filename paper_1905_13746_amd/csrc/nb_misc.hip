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

// The encoding is a byte-to-byte map: each workgroup builds its 256-entry
// table in LDS, then every lane maps 16 bytes of one row (one chunk) per
// step; chunks are numbered row by row so a wave covers 1 KB of a row.
// Rows whose pointers allow 4-byte access go through 16-byte loads and
// stores; the chunk holding a row's ragged end and every chunk of
// unaligned rows go byte by byte (never writing past F).
__global__ __launch_bounds__(256) void quantize_fp8_kernel(const uint8_t* __restrict__ x, int64_t n, int F,
                                                          int64_t ld_x, uint8_t* __restrict__ out,
                                                          int64_t ld_out, int vec) {
  __shared__ uint8_t lut[256];
  lut[threadIdx.x] = (uint8_t)e4m3_from_count(min((uint32_t)threadIdx.x, 240u));
  __syncthreads();
  const int64_t cpr = (F + 15) / 16;                  // chunks per row
  const int64_t total = n * cpr;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < total;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = c / cpr;
    const int f0 = (int)(c - r * cpr) * 16;
    const uint8_t* src = x + r * ld_x + f0;
    uint8_t* dst = out + r * ld_out + f0;
    if (vec && f0 + 16 <= F) {
      const dev::u32x4 v = dev::load16(src);
      dev::u32x4 o;
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        const uint32_t u = v[d];
        o[d] = (uint32_t)lut[u & 0xFFu] | ((uint32_t)lut[(u >> 8) & 0xFFu] << 8) |
               ((uint32_t)lut[(u >> 16) & 0xFFu] << 16) | ((uint32_t)lut[u >> 24] << 24);
      }
      reinterpret_cast<dev::u32x4_a4*>(dst)->v = o;
    } else {
      const int m = min(16, F - f0);
      for (int b = 0; b < m; ++b) dst[b] = lut[src[b]];
    }
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
  const int64_t chunks = n * ((F + 15) / 16);
  const int64_t blocks = std::min<int64_t>((chunks + 255) / 256, 8192);
  const int vec = ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(out)) & 3) == 0 &&
                  ld_x % 4 == 0 && ld_out % 4 == 0;
  hipLaunchKernelGGL(quantize_fp8_kernel, dim3((unsigned)blocks), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), x, n, F, ld_x, out, ld_out, vec);
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
