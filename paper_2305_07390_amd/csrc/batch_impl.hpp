// batch_impl.hpp -- persistent batch kernels over many independent grids.
//
// The decomposition of each grid is the single-grid one (tb2d / tb3d tiles);
// what changes is the schedule (the paper's tile-by-tile execution, Section
// 4.1, extended to a work list): one workgroup per CU pulls (job, pass, tiles)
// items of every grid and stencil variant of a dtype from one counter, waits
// until the job's previous pass is complete, runs the tiles and publishes
// their completion. Waits are bounded by a realtime-clock watchdog; an expired
// wait sets an error word, and every later item of the launch skips its work
// so the launch still drains.
#pragma once
#include "tb2d_impl.hpp"
#include "tb3d_impl.hpp"
#include "worklist.hpp"

// One translation unit per dtype instantiates the kernel; see batch_f*.hip.

namespace stencil_impl {
namespace batch {

// Job descriptors live in global memory; their fields are the same for every
// lane, so they are moved to scalar registers once per item (the kernel's own
// stores could alias the descriptor as far as the compiler knows, which would
// otherwise keep per-lane copies of every coefficient in VGPRs).
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni(int64_t v) {
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)((uint64_t)v & 0xffffffffull));
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double uni(double v) {
  return __builtin_bit_cast(double, uni(__builtin_bit_cast(int64_t, v)));
}
__device__ __forceinline__ float uni(float v) {
  return __builtin_bit_cast(float, uni(__builtin_bit_cast(int, v)));
}
template <typename T>
__device__ __forceinline__ T* uni_ptr(T* p) {
  return (T*)(uintptr_t)uni((int64_t)(uintptr_t)p);
}

// Memory operations and clock of the work-list waits on the device. Every
// value that steers a wait is made wave-uniform, so the compiler keeps the
// persistent item loop around it uniform too (a loop it believed divergent
// was restructured into a lane-masked one).
struct DeviceWait {
  __device__ static unsigned load_relaxed(const unsigned* p) {
    return __builtin_amdgcn_readfirstlane(__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  }
  __device__ static void acquire_fence() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
  __device__ static void raise(unsigned* p) {
    __hip_atomic_store(p, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __device__ static uint64_t now() { return __builtin_amdgcn_s_memrealtime(); }
  __device__ static void pause() { __builtin_amdgcn_s_sleep(4); }
};

// Pass k writes `out` when (npass - 1 - k) is even, else the workspace, so the
// last pass writes `out`; pass 0 reads `in`.
__device__ __forceinline__ void pass_buffers(const void* in, void* out, void* ws, int npass, int pass,
                                             const void** src, void** dst) {
  void* prev = ((npass - pass) & 1) == 0 ? out : ws;  // buffer of pass - 1
  *src = pass == 0 ? in : (const void*)prev;
  *dst = ((npass - 1 - pass) & 1) == 0 ? out : ws;
}

// 2D depths of the fused batch kernels: every variant shares one register
// allocation, so where the single-grid kernels go deeper into the AGPRs
// these stop at the depths measured and spill-checked for it: radius-2 stars
// 7 (FP64) / 6 (FP32), radius-3 stars 4, radius-1 and -2 boxes 8 and 5.
constexpr int batch_2d_depth_c(int dtype, int r, int shape) {
  if (shape == kStar) return r == 1 ? 12 : r == 2 ? (dtype == kF64 ? 7 : 6) : r == 3 ? 4 : 2;
  if (shape == kBox) return r == 1 ? 8 : r == 2 ? 5 : r == 3 ? 3 : 2;
  return max_depth_c(dtype == kF64, r, shape);
}

// Deepest compiled depth of a batched variant (0: not in the batch kernel;
// such jobs run with their single-grid kernels after it). All variants share
// one kernel, and so one register allocation: 2D tiles take the depths
// above, and FP64 3D radius-2 tiles (4 x 2 cells per lane) are left out.
constexpr int batch_depth_c(int dtype, int ndim, int r, int shape) {
  if (ndim == 2) return batch_2d_depth_c(dtype, r, shape);
  if (dtype == kF64 && r == 2) return 0;
  return tb3d::max_depth_c(dtype, r, shape);
}

// One wave tile of a 2D job (the tb2d strip/segment decomposition).
// SPLIT: interior strips take the tile body without halo reads (as in the
// single-grid kernel); the fused kernel keeps one body for all strips.
template <typename Real, int R, int SHAPE,
          int DEPTH = batch_depth_c(sizeof(Real) == 8 ? kF64 : kF32, 2, R, SHAPE), bool SPLIT = false>
__device__ __forceinline__ void run_2d(const BatchJob<Real>& J, int pass, int tile, Real* hq, int lane) {
  if constexpr (DEPTH > 0) {
    constexpr int V = tb2d_cols(sizeof(Real) == 8, R, SHAPE);
    constexpr int KB = (2 * R + 1) * (2 * R + 1);
    Real wl[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) wl[k] = uni(J.w[k]);
    const void* in = uni_ptr(J.in);
    const int npass = uni(J.npass);
    const void* src;
    void* dst;
    pass_buffers(in, uni_ptr(J.out), uni_ptr(J.ws), npass, pass, &src, &dst);
    const int d = pass == npass - 1 ? uni(J.depth_last) : uni(J.depth);
    const int P = (int)uni(J.P), Q = (int)uni(J.Qy);
    const int ns = uni(J.strips), HL = uni(J.hl);
    const Tile2D g = locate_2d(tile, ns, uni(J.seg_len), uni(J.seg_len_e), uni(J.edge_tiles), P, Q,
                               R, V, HL);
    const int edge = g.edge, X0 = g.X0, la = g.la, lb = g.lb, Y0 = g.Y0, Y1 = g.Y1;
    // Full-depth passes (all but a job's last) get the depth as a constant,
    // so the level loop unrolls without per-level checks, as in the
    // single-grid kernel; the remainder pass takes it at run time. One tile
    // body serves interior and edge strips here (the fused kernel's register
    // budget has no room for a second copy). The level rings keep 2r slots:
    // the work-list loop's state leaves no room for the wider ring (the
    // 25-point box's kernel would double its AGPR use).
    if (SPLIT && d == DEPTH)
      tb2d_tile<Real, R, SHAPE, DEPTH, V, false>(wl, src, dst, in, P, Q, hq, lane, edge, X0, la, lb, Y0, Y1,
                                                 DEPTH);
    else if (d == DEPTH)
      tb2d_tile_impl<Real, R, SHAPE, DEPTH, V, true, false>(wl, src, dst, in, P, Q, hq, lane, edge, X0, la,
                                                            lb, Y0, Y1, DEPTH);
    else
      tb2d_tile_impl<Real, R, SHAPE, DEPTH, V, true, false>(wl, src, dst, in, P, Q, hq, lane, edge, X0, la,
                                                            lb, Y0, Y1, d);
  }
}

// One workgroup tile of a 3D job (the tb3d xy-tile/z-segment decomposition).
template <typename Real, int R, int SHAPE,
          int DEPTH = batch_depth_c(sizeof(Real) == 8 ? kF64 : kF32, 3, R, SHAPE), int Z0 = 2>
__device__ __forceinline__ void run_3d(const BatchJob<Real>& J, int pass, int tile, char* lds) {
  if constexpr (DEPTH > 0) {
    using namespace tb3d;
    constexpr int BY = cells_y(sizeof(Real) == 8, R, SHAPE);
    using FL = FaceLayout<R, BY>;
    constexpr int KB = (2 * R + 1) * (2 * R + 1) * (2 * R + 1);
    Real* faces = (Real*)lds;
    Real* xchg = faces + kRing * FL::kPerPlane;
    Real wl[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) wl[k] = uni(J.w[k]);
    const int npass = uni(J.npass);
    const void* src;
    void* dst;
    pass_buffers(uni_ptr(J.in), uni_ptr(J.out), uni_ptr(J.ws), npass, pass, &src, &dst);
    const int d = pass == npass - 1 ? uni(J.depth_last) : uni(J.depth);
    const int P = (int)uni(J.P), Qy = (int)uni(J.Qy), Qz = (int)uni(J.Qz);
    const int sx = uni(J.sx), sy = uni(J.sy), seg_len = uni(J.seg_len);
    const int seg = tile / (sx * sy);
    const int rem = tile - seg * sx * sy;
    const int ty = rem / sx;
    const int tx = rem - ty * sx;
    const Tb3dGeom g = tb3d_geom<R, BY>(tx, ty, sx, sy, P, Qy, uni(J.hx), uni(J.hy));
    const int Zs0 = seg * seg_len;
    const int Zs1 = (Zs0 + seg_len < Qz) ? Zs0 + seg_len : Qz;
    if (d == DEPTH)
      tb3d_tile<Real, R, SHAPE, DEPTH, Z0>(wl, src, dst, P, Qy, Qz, g, Zs0, Zs1, DEPTH, faces, xchg);
    else
      tb3d_tile<Real, R, SHAPE, DEPTH, Z0>(wl, src, dst, P, Qy, Qz, g, Zs0, Zs1, d, faces, xchg);
  }
}

// Variants of the auxiliary batch kernel (SET 1): FP64 3D radius-2 stars,
// which the fused kernel leaves out (4 x 2 cells per lane at depth 2 spill in
// its shared register allocation). Alone in a kernel they fit, so their jobs
// are still fused among themselves instead of running one after another.
constexpr int aux_depth_c(int dtype, int ndim, int r, int shape) {
  return (dtype == kF64 && ndim == 3 && r == 2 && shape == kStar) ? tb3d::max_depth_c(kF64, 2, kStar) : 0;
}

// Single-variant persistent kernels (SET = kSingleBase + variant id) run one
// plan's passes in one launch (STENCIL_FLAG_PERSISTENT) with that variant's
// own register allocation, at its single-grid depth and plane ring.
constexpr int kSingleBase = 2;
constexpr int set_ndim(int set) { return 2 + (set - kSingleBase) / kBatch3DBase; }
constexpr int set_r(int set) { return ((set - kSingleBase) % kBatch3DBase) / 3 + 1; }
constexpr int set_shape(int set) { return (set - kSingleBase) % 3; }
// Depth and plane ring of a single-variant kernel: the single-grid ones,
// except where the job descriptor's extra registers would spill (2D radius-2
// stars stop at 7 / 6; the FP64 3D 7-point star keeps two planes in flight).
constexpr int single_depth_c(int dtype, int ndim, int r, int shape) {
  if (ndim == 2 && r == 2 && shape == kStar) return dtype == kF64 ? 7 : 6;
  return ndim == 2 ? max_depth_c(dtype == kF64, r, shape) : tb3d::max_depth_c(dtype, r, shape);
}
constexpr int single_ring_c(int dtype, int r, int shape, int depth) {
  return (dtype == kF64 && r == 1 && shape == kStar && depth == 4) ? 2
                                                                   : tb3d::plane_ring(dtype == kF64, r, shape, depth);
}

// The persistent batch kernel of one dtype: every compiled 2D and 3D variant
// behind one work list (SET 0), the auxiliary variants (SET 1), or one variant
// (SET >= kSingleBase). A workgroup claims an item (a 3D tile, or up to four
// 2D tiles of one pass, one per wave), waits for the job's previous pass, runs
// it and publishes the tiles done. Loop control is workgroup-uniform: wave 0
// claims and waits, the result travels through LDS behind a barrier, and no
// lane-dependent branch sits in the loop (the optimizer may thread a loop edge
// on such a predicate and skip the claim).
template <typename Real, int SET>
__global__ __launch_bounds__(256) void batch_kernel(const BatchParams<Real> p) {
  extern __shared__ char lds_raw[];
  __shared__ long long s_item;
  __shared__ int s_ok;
  const BatchQueue& q = p.q;
  const int lane = lane_id();
  const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const bool wave0 = wid == 0;
  while (true) {
    if (wave0) {
      const unsigned long long it = atomicAdd(q.cursor, lane == 0 ? 1ull : 0ull);
      const unsigned lo32 = __builtin_amdgcn_readlane((unsigned)(it & 0xffffffffull), 0);
      const unsigned hi32 = __builtin_amdgcn_readlane((unsigned)(it >> 32), 0);
      s_item = (long long)(((unsigned long long)hi32 << 32) | lo32);
    }
    __syncthreads();
    const int64_t item = uni((int64_t)s_item);
    if (item >= q.nitems) break;
    const int c = worklist::find_chunk(q.chunk_first, q.nchunks, item);
    const int job = uni(q.chunk_job[c]);
    const int pass = uni(q.chunk_pass[c]);
    const int sub = (int)(item - uni(q.chunk_first[c]));
    const BatchJob<Real>& J = p.jobs[job];
    const int variant = uni(J.variant);
    const int tiles = uni(J.tiles);
    if (wave0)
      s_ok = (pass == 0 || worklist::wait_count<DeviceWait>(q.done + job, worklist::need_before(pass, tiles),
                                                            q.err, q.timeout_ticks))
                 ? 1
                 : 0;
    __syncthreads();
    const bool ok = __builtin_amdgcn_readfirstlane(s_ok) != 0;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // every wave sees the previous pass
    unsigned ndone = worklist::tiles_per_item(3);  // 3D items: one tile
    constexpr int DT = sizeof(Real) == 8 ? kF64 : kF32;
    if constexpr (SET >= kSingleBase) {
      constexpr int ND = set_ndim(SET), RR = set_r(SET), SH = set_shape(SET);
      constexpr int D = single_depth_c(DT, ND, RR, SH);
      if constexpr (ND == 2) {
        ndone = worklist::item_tiles(2, tiles, sub);
        const int t = worklist::tiles_per_item(2) * sub + wid;
        if (ok && t < tiles) {
          Real* hq = (Real*)lds_raw + (size_t)wid * p.hq_stride;
          // (one body for the FP32 radius-3 star, whose registers overflow with two)
          run_2d<Real, RR, SH, D, !(DT == kF32 && RR == 3 && SH == kStar)>(J, pass, t, hq, lane);
        }
      } else if (ok) {
        run_3d<Real, RR, SH, D, single_ring_c(DT, RR, SH, D)>(J, pass, sub, lds_raw);
      }
      (void)variant;
    } else if constexpr (SET == 1) {
      if (ok && variant == batch_variant(3, 2, kStar))
        run_3d<Real, 2, kStar, aux_depth_c(DT, 3, 2, kStar)>(J, pass, sub, lds_raw);
    } else if (variant < kBatch3DBase) {
      ndone = worklist::item_tiles(2, tiles, sub);
      const int t = worklist::tiles_per_item(2) * sub + wid;
      if (ok && t < tiles) {
        Real* hq = (Real*)lds_raw + (size_t)wid * p.hq_stride;
        switch (variant) {
          case batch_variant(2, 1, kStar): run_2d<Real, 1, kStar>(J, pass, t, hq, lane); break;
          case batch_variant(2, 1, kBox): run_2d<Real, 1, kBox>(J, pass, t, hq, lane); break;
          case batch_variant(2, 1, kGeneral): run_2d<Real, 1, kGeneral>(J, pass, t, hq, lane); break;
          case batch_variant(2, 2, kStar): run_2d<Real, 2, kStar>(J, pass, t, hq, lane); break;
          case batch_variant(2, 2, kBox): run_2d<Real, 2, kBox>(J, pass, t, hq, lane); break;
          case batch_variant(2, 2, kGeneral): run_2d<Real, 2, kGeneral>(J, pass, t, hq, lane); break;
          case batch_variant(2, 3, kStar): run_2d<Real, 3, kStar>(J, pass, t, hq, lane); break;
          case batch_variant(2, 3, kBox): run_2d<Real, 3, kBox>(J, pass, t, hq, lane); break;
          case batch_variant(2, 4, kStar): run_2d<Real, 4, kStar>(J, pass, t, hq, lane); break;
          case batch_variant(2, 4, kBox): run_2d<Real, 4, kBox>(J, pass, t, hq, lane); break;
          default: break;
        }
      }
    } else if (ok) {
      switch (variant) {
        case batch_variant(3, 1, kStar): run_3d<Real, 1, kStar>(J, pass, sub, lds_raw); break;
        case batch_variant(3, 1, kBox): run_3d<Real, 1, kBox>(J, pass, sub, lds_raw); break;
        case batch_variant(3, 1, kGeneral): run_3d<Real, 1, kGeneral>(J, pass, sub, lds_raw); break;
        case batch_variant(3, 2, kStar): run_3d<Real, 2, kStar>(J, pass, sub, lds_raw); break;
        default: break;
      }
    }
    // Publish the tiles: every wave's stores reach this XCD's L2 (workgroup
    // release, ordered by the barrier), then wave 0 alone releases at agent
    // scope, which writes back the whole L2 once for the workgroup, and adds
    // the count.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
    if (wave0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_fetch_add(q.done + job, lane == 0 ? ndone : 0u, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

}  // namespace batch
}  // namespace stencil_impl

namespace stencil_impl {
namespace batch {

template <typename Real, int SET>
hipError_t launch(const BatchParams<Real>* p, int grid, size_t lds, hipStream_t s) {
  const void* fn = (const void*)&batch_kernel<Real, SET>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  void* args[] = {(void*)p};
  return hipLaunchKernel(fn, dim3(grid), dim3(256), args, lds, s);
}

// Variants with a single-variant persistent kernel: every variant with a
// blocked single-grid kernel.
constexpr bool single_supported(int dtype, int ndim, int r, int shape) {
  return r >= 1 && r <= (ndim == 2 ? kMaxR : 2) && single_depth_c(dtype, ndim, r, shape) > 0;
}

template <typename Real, int V>
hipError_t launch_single_from(int variant, const BatchParams<Real>* p, int grid, size_t lds,
                              hipStream_t s) {
  if constexpr (V >= 2 * kBatch3DBase) {
    return hipErrorInvalidValue;
  } else {
    constexpr int SET = kSingleBase + V;
    constexpr int DT = sizeof(Real) == 8 ? kF64 : kF32;
    if (variant == V) {
      if constexpr (single_supported(DT, set_ndim(SET), set_r(SET), set_shape(SET)))
        return launch<Real, SET>(p, grid, lds, s);
      return hipErrorInvalidValue;
    }
    return launch_single_from<Real, V + 1>(variant, p, grid, lds, s);
  }
}

}  // namespace batch
}  // namespace stencil_impl
