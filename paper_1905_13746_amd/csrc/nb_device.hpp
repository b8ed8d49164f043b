// Device helpers shared by the libnbgpu kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace nb {
namespace dev {

// 16-byte vector with 4-byte alignment: rows of byte features are only
// dword-aligned (row stride F bytes, F a multiple of 4), and gfx950 global
// loads need dword alignment only.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
struct __attribute__((packed, aligned(4))) u32x4_a4 {
  u32x4 v;
};

__device__ __forceinline__ u32x4 load16(const uint8_t* p) {
  return reinterpret_cast<const u32x4_a4*>(p)->v;
}

// Same 16 bytes, but every byte at or beyond `avail` bytes from p reads as 0
// (used only for the last rows of a buffer, where a full 16-byte access
// could leave the caller's allocation).
__device__ __forceinline__ u32x4 load16_guarded(const uint8_t* p, int64_t avail) {
  u32x4 out = {0u, 0u, 0u, 0u};
  if (avail >= 16) return load16(p);
#pragma unroll
  for (int b = 0; b < 16; ++b) {
    uint32_t v = (b < avail) ? (uint32_t)p[b] : 0u;
    out[b >> 2] |= v << (8 * (b & 3));
  }
  return out;
}

// Raw buffer resource over [base, base + bytes): loads at offsets beyond
// `bytes` return zero instead of touching memory.  Word 3 is the gfx9-family
// descriptor format for untyped dword access.
// `bytes` is clamped to [0, 2^31 - 1] (the descriptor field).
// The clamp uses 32-bit halves only: gfx9 has no 64-bit scalar ordered
// compare, and a 64-bit vector compare would need VGPRs (possibly ones with
// loads still in flight).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, int64_t bytes) {
  const uint32_t hi = (uint32_t)((uint64_t)bytes >> 32), lo = (uint32_t)bytes;
  const int32_t n = ((int32_t)hi < 0) ? 0 : ((hi != 0u || (lo >> 31) != 0u) ? 0x7FFFFFFF : (int32_t)lo);
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, n, 0x00020000);
}

// Values the compiler cannot prove wave-uniform (they pass through loop-
// carried state) but are: take lane 0's copy, so descriptors built from
// them live in scalar registers instead of forcing per-lane loops.
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  return reinterpret_cast<T*>(uniform64(reinterpret_cast<int64_t>(p)));
}

// Load of read-only data at a wave-uniform address through the constant
// address space: a scalar load (lgkmcnt), where a plain load could become a
// vector load (vmcnt, ordered behind the streaming loads in flight) when
// the compiler cannot rule out that the kernel's own stores alias it.
template <class T>
__device__ __forceinline__ T load_uniform(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "whole words");
  typedef const __attribute__((address_space(4))) uint32_t* ConstWords;
  const ConstWords q = (ConstWords)(p);
  uint32_t w[sizeof(T) / 4];
#pragma unroll
  for (unsigned i = 0; i < sizeof(T) / 4; ++i) w[i] = q[i];
  T out;
  __builtin_memcpy(&out, w, sizeof(T));
  return out;
}

// Cache policy of the streaming feature loads (gfx940+ bits: 1 sc0, 2 nt,
// 16 sc1); non-temporal by default: each feature byte is read once.
#ifndef NB_STREAM_CPOL
#define NB_STREAM_CPOL 2
#endif

// A buffer offset past every range make_rsrc builds: the load reads nothing
// and returns zeros (the instruction still issues, so counts of loads in
// flight stay fixed).
constexpr uint32_t kNoAccess = 0x80000000u;

__device__ __forceinline__ u32x4 buffer_load16(__amdgpu_buffer_rsrc_t r, uint32_t voff) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, 0, NB_STREAM_CPOL);
  return u32x4{(uint32_t)v[0], (uint32_t)v[1], (uint32_t)v[2], (uint32_t)v[3]};
}

// Round-to-nearest-even of an FP64 value to BF16, in one rounding: add the
// rounding increment below bit 45 of the FP64 significand (ties to even),
// truncate, and take the (then exact) FP32 image's upper half.  Valid for the
// normal BF16 range, which holds every table value.
__device__ __forceinline__ uint16_t f64_to_bf16_rne(double v) {
  uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint64_t lsb = (b >> 45) & 1ull;
  b += 0x00000FFFFFFFFFFFull + lsb;
  b &= ~((1ull << 45) - 1ull);
  const float f = (float)__longlong_as_double((long long)b);
  return (uint16_t)(__float_as_uint(f) >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
  return __uint_as_float(((uint32_t)h) << 16);
}

}  // namespace dev
}  // namespace nb
