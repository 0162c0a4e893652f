// Device-side helpers shared by the HIP kernels (gfx950 only).
//
// * Raw buffer resources: every global load and store goes through a buffer
//   descriptor whose range is the part of the array the caller may touch.
//   Loads past the range return zero and stores past it are dropped by the
//   hardware, so a tile that reaches beyond the grid can never fault.
// * Cross-lane moves: wave-wide DPP shifts by one lane (wave_shr:1 /
//   wave_shl:1), applied to 32-bit words.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stencil_dev {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Wait until every vector-memory operation this wave has issued is complete
// (gfx9 parts count loads and stores in one counter). A store written through
// to the point of device coherence (an agent-scope atomic store) is visible to
// every CU once it completes, so a flag stored after this wait never overtakes
// the data it announces. A compiler barrier as well.
__device__ __forceinline__ void wait_vmem_complete() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Buffer descriptor word 3 for gfx9-family parts: 32-bit data format, raw
// (untyped) addressing, range checking on num_records.
constexpr int kRsrcWord3 = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                           kRsrcWord3);
}

// Load N consecutive elements (N * sizeof(T) a multiple of 16 bytes).
template <typename T, int N>
__device__ __forceinline__ void load_vec(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff,
                                         T (&x)[N]) {
  static_assert((N * sizeof(T)) % 16 == 0, "row chunk must be whole 16-byte words");
  constexpr int NB = N * sizeof(T) / 16;
  constexpr int PER = 16 / sizeof(T);
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    u32x4 q = __builtin_amdgcn_raw_buffer_load_b128(rs, voff + 16 * b, soff, 0);
    T tmp[PER];
    __builtin_memcpy(tmp, &q, 16);
#pragma unroll
    for (int e = 0; e < PER; ++e) x[b * PER + e] = tmp[e];
  }
}

template <typename T, int N>
__device__ __forceinline__ void store_vec(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff,
                                          const T (&x)[N]) {
  static_assert((N * sizeof(T)) % 16 == 0, "row chunk must be whole 16-byte words");
  constexpr int NB = N * sizeof(T) / 16;
  constexpr int PER = 16 / sizeof(T);
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    T tmp[PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) tmp[e] = x[b * PER + e];
    u32x4 q;
    __builtin_memcpy(&q, tmp, 16);
    __builtin_amdgcn_raw_buffer_store_b128(q, rs, voff + 16 * b, soff, 0);
  }
}

// Single-element load/store (used where a lane's chunk is only partly inside).
template <typename T>
__device__ __forceinline__ T load_one(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff);
template <>
__device__ __forceinline__ double load_one<double>(__amdgpu_buffer_rsrc_t rs, uint32_t voff,
                                                   uint32_t soff) {
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  u32x2 q = __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0);
  return __builtin_bit_cast(double, q);
}
template <>
__device__ __forceinline__ float load_one<float>(__amdgpu_buffer_rsrc_t rs, uint32_t voff,
                                                 uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, voff, soff, 0));
}
__device__ __forceinline__ void store_one(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff,
                                          double v) {
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), rs, voff, soff, 0);
}
__device__ __forceinline__ void store_one(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff,
                                          float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rs, voff, soff, 0);
}

// DPP control words (gfx9 encoding).
constexpr int kDppWaveShr1 = 0x138;  // lane i receives lane i-1
constexpr int kDppWaveShl1 = 0x130;  // lane i receives lane i+1

template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffull), CTRL, 0xf, 0xf, true);
  int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, true);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

}  // namespace stencil_dev
