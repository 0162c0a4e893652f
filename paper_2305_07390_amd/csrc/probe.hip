// Microbenchmarks for the parameters of the attainable-performance model
// (paper Section 5.1: global and on-chip bandwidth; Section 5.2.2: the cost
// of a synchronisation; Section 6.1: latencies, from which Little's law gives
// the parallelism a kernel needs).
//
// * copy: a streaming device copy with 128-bit loads and stores, the
//   reachable HBM bandwidth B_gm (the best of a few unroll depths, cache
//   policies and grid sizes);
// * chase: dependent-load chains through HBM (a chain that jumps across a
//   buffer far larger than the last-level cache) and through LDS, and a chain
//   of dependent FP64 fused multiply-adds: one lane, time per link;
// * lds_bandwidth: every CU streams 128-bit LDS reads (B_sm);
// * neighbor_sync: one workgroup per CU on a 2D torus; in each round a
//   workgroup writes a payload, publishes a round counter, waits for its four
//   neighbours' counters and reads their payloads, counting every word that
//   does not carry the round's value (the check of the exchange protocol).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.hpp"
#include "launch.hpp"

namespace stencil_impl {
namespace {

using namespace stencil_dev;
typedef unsigned int u32x4v __attribute__((ext_vector_type(4)));

// U independent 16-byte loads per lane in flight, then their stores;
// non-temporal (NT) or ordinary accesses.
template <int U, bool NT>
__global__ __launch_bounds__(256) void copy_kernel(const u32x4v* __restrict__ src, u32x4v* __restrict__ dst,
                                                   int64_t n16) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + (U - 1) * stride < n16; i += U * stride) {
    u32x4v v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = NT ? __builtin_nontemporal_load(src + i + u * stride) : src[i + u * stride];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (NT) __builtin_nontemporal_store(v[u], dst + i + u * stride);
      else dst[i + u * stride] = v[u];
    }
  }
  for (; i < n16; i += stride) dst[i] = src[i];
}

// Chain over n nodes spaced `stride` 32-bit words apart: node i points to
// (a i + 1) mod n, a full-period linear congruential walk when n is a power of
// two and a = 1 mod 4, so consecutive links land far apart.
__global__ __launch_bounds__(256) void chain_init_kernel(uint32_t* buf, uint32_t n, uint32_t stride, uint32_t a) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    buf[(size_t)i * stride] = (uint32_t)(((uint64_t)a * i + 1u) & (uint64_t)(n - 1));
}

__global__ __launch_bounds__(64) void chase_hbm_kernel(const uint32_t* buf, uint32_t stride, int steps,
                                                       uint32_t* out) {
  if (threadIdx.x != 0) return;
  uint32_t j = 0;
  for (int k = 0; k < steps; ++k) j = __builtin_nontemporal_load(buf + (size_t)j * stride);
  out[0] = j;
}

constexpr int kLdsChain = 8192;  // 32 KB of links
__global__ __launch_bounds__(64) void chase_lds_kernel(int steps, uint32_t a, uint32_t* out) {
  __shared__ uint32_t lds[kLdsChain];
  for (int i = threadIdx.x; i < kLdsChain; i += 64) lds[i] = (uint32_t)((a * (uint32_t)i + 1u) & (kLdsChain - 1));
  __syncthreads();
  if (threadIdx.x != 0) return;
  uint32_t j = 0;
  for (int k = 0; k < steps; ++k) j = lds[j];
  out[0] = j;
}

__global__ __launch_bounds__(64) void chain_fma_kernel(int steps, double a, double b, double* out) {
  if (threadIdx.x != 0) return;
  double x = a;
  for (int k = 0; k < steps; k += 16) {
#pragma unroll
    for (int u = 0; u < 16; ++u) x = __builtin_fma(x, a, b);
  }
  out[0] = x;
}

constexpr int kLdsBwBytes = 64 * 1024;
__global__ __launch_bounds__(256) void lds_bw_kernel(int iters, uint32_t* out) {
  __shared__ u32x4v lds[kLdsBwBytes / 16];
  for (int i = threadIdx.x; i < kLdsBwBytes / 16; i += 256) lds[i] = u32x4v{(unsigned)i, 1u, 2u, 3u};
  __syncthreads();
  u32x4v acc = {0u, 0u, 0u, 0u};
  // consecutive lanes read consecutive 16-byte words: no bank conflicts
  unsigned idx = threadIdx.x;
  for (int k = 0; k < iters; ++k) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      acc ^= lds[(idx + u * 256) & (kLdsBwBytes / 16 - 1)];
    }
    idx += 2048 + (acc.x & 1u);  // the next addresses depend on the data read
  }
  if ((acc.x ^ acc.y ^ acc.z ^ acc.w) == 0x9e3779b9u) out[0] = acc.x;
}

// Neighbour synchronisation on a gx x gy torus of workgroups (one per CU).
// mode 0: plain stores, agent-scope release (writes back the L2) and an
//         acquire poll (invalidates it), plain loads;
// mode 1: payload written through to the coherence point (agent-scope relaxed
//         stores), a wait in every wave until those stores are complete
//         (without it the counter can become visible first: observed as
//         stale payload words), a relaxed counter store; relaxed
//         agent-scope polls and payload loads (they bypass the non-coherent
//         caches). No whole-cache write-back.
template <int MODE>
__global__ __launch_bounds__(256) void neighbor_sync_kernel(double* buf, unsigned* flags, unsigned* err,
                                                            unsigned long long* mismatches, int gx, int gy,
                                                            int rounds, int words, long long timeout) {
  __shared__ int s_ok;
  const int wg = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const bool wave0 = tid < 64;
  const int x = wg % gx, y = wg / gx;
  int nb[4];
  nb[0] = y * gx + (x + gx - 1) % gx;
  nb[1] = y * gx + (x + 1) % gx;
  nb[2] = ((y + gy - 1) % gy) * gx + x;
  nb[3] = ((y + 1) % gy) * gx + x;
  unsigned long long bad = 0;
  for (int k = 1; k <= rounds; ++k) {
    const int slot = k & 1;
    double* mine = buf + ((size_t)wg * 2 + slot) * words;
    for (int i = tid; i < words; i += 256) {
      if (MODE == 0) mine[i] = (double)k;
      else
        __hip_atomic_store((unsigned long long*)(mine + i), __builtin_bit_cast(unsigned long long, (double)k),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // mode 1: each wave waits until its own write-through stores are complete
    // before the barrier that precedes the counter store
    if (MODE == 1) wait_vmem_complete();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
    if (wave0) {
      if (MODE == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (lane == 0) __hip_atomic_store(flags + wg, (unsigned)k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else if (lane == 0) {
        __hip_atomic_store(flags + wg, (unsigned)k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      // lanes 0..3 poll one neighbour each
      const long long t0 = (long long)__builtin_amdgcn_s_memrealtime();
      int ok = 1;
      while (true) {
        unsigned v = (unsigned)k;
        if (lane < 4) {
          v = MODE == 0 ? __hip_atomic_load(flags + nb[lane], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)
                        : __hip_atomic_load(flags + nb[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        const unsigned long long behind = __builtin_amdgcn_ballot_w64(v < (unsigned)k);
        if (behind == 0ull) break;
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
            (long long)__builtin_amdgcn_s_memrealtime() - t0 > timeout) {
          if (lane == 0) __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      if (lane == 0) s_ok = ok;
    }
    __syncthreads();
    const int ok = __builtin_amdgcn_readfirstlane(s_ok);
    if (!ok) break;
    if (MODE == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    else __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    for (int q = 0; q < 4; ++q) {
      const double* theirs = buf + ((size_t)nb[q] * 2 + slot) * words;
      for (int i = tid; i < words; i += 256) {
        double v;
        if (MODE == 0) v = theirs[i];
        else
          v = __builtin_bit_cast(double, __hip_atomic_load((const unsigned long long*)(theirs + i), __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT));
        bad += v != (double)k;
      }
    }
    // every wave is done reading this round's slot before the next round's
    // counter can let a neighbour overwrite it (two rounds later)
    __syncthreads();
  }
  if (bad) atomicAdd(mismatches, bad);
}

}  // namespace

// variant: 0..3 = (4 loads, NT), (8, NT), (4, ordinary), (8, ordinary)
hipError_t probe_copy_launch(const void* src, void* dst, int64_t bytes, int grid, int variant, hipStream_t s) {
  const u32x4v* a = (const u32x4v*)src;
  u32x4v* b = (u32x4v*)dst;
  const int64_t n = bytes / 16;
  switch (variant) {
    case 0: hipLaunchKernelGGL((copy_kernel<4, true>), dim3(grid), dim3(256), 0, s, a, b, n); break;
    case 1: hipLaunchKernelGGL((copy_kernel<8, true>), dim3(grid), dim3(256), 0, s, a, b, n); break;
    case 2: hipLaunchKernelGGL((copy_kernel<4, false>), dim3(grid), dim3(256), 0, s, a, b, n); break;
    case 3: hipLaunchKernelGGL((copy_kernel<8, false>), dim3(grid), dim3(256), 0, s, a, b, n); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t probe_chain_init_launch(uint32_t* buf, uint32_t n, uint32_t stride, uint32_t a, hipStream_t s) {
  hipLaunchKernelGGL(chain_init_kernel, dim3(4096), dim3(256), 0, s, buf, n, stride, a);
  return hipGetLastError();
}

hipError_t probe_chase_hbm_launch(const uint32_t* buf, uint32_t stride, int steps, uint32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(chase_hbm_kernel, dim3(1), dim3(64), 0, s, buf, stride, steps, out);
  return hipGetLastError();
}

hipError_t probe_chase_lds_launch(int steps, uint32_t a, uint32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(chase_lds_kernel, dim3(1), dim3(64), 0, s, steps, a, out);
  return hipGetLastError();
}

hipError_t probe_chain_fma_launch(int steps, double a, double b, double* out, hipStream_t s) {
  hipLaunchKernelGGL(chain_fma_kernel, dim3(1), dim3(64), 0, s, steps, a, b, out);
  return hipGetLastError();
}

hipError_t probe_lds_bw_launch(int grid, int iters, uint32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(lds_bw_kernel, dim3(grid), dim3(256), 0, s, iters, out);
  return hipGetLastError();
}

hipError_t probe_neighbor_sync_launch(int mode, double* buf, unsigned* flags, unsigned* err,
                                      unsigned long long* mismatches, int gx, int gy, int rounds, int words,
                                      long long timeout, hipStream_t s) {
  const dim3 grid(gx * gy), block(256);
  if (mode == 0)
    hipLaunchKernelGGL(neighbor_sync_kernel<0>, grid, block, 0, s, buf, flags, err, mismatches, gx, gy, rounds,
                       words, timeout);
  else if (mode == 1)
    hipLaunchKernelGGL(neighbor_sync_kernel<1>, grid, block, 0, s, buf, flags, err, mismatches, gx, gy, rounds,
                       words, timeout);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace stencil_impl
