// tb3d_dev_impl.hpp -- 3D device tiling (kernel templates).
//
// The paper's device tiling (Section 4.1, "one tile at a time"; Section 5.2.2
// for its cost): the whole xy plane of the grid is one device-sized tile,
// split among workgroups without overlap, and every workgroup streams all of
// z through every time level of the pass. A tile computes no redundant
// margin; instead its neighbours' edges of every level are exchanged through
// global memory after each z-step, guarded by one progress counter per tile.
//
// Layout: workgroup (tx, ty) of a gx x gy grid owns the interior cells
// x in [R + 64 tx, R + 64 tx + 64), y in [R + TY ty, R + TY ty + TY),
// TY = 16 BY. The 256 lanes form a 16 x 16 grid; lane (lx, ly) holds a
// 4 x BY block of cells. Wave w holds lane rows 4w .. 4w + 3, so a 16-lane DPP
// row is one lane row of the tile.
//
// Time levels and the lag: in iteration i, level 1 takes input plane i and
// level s takes the output plane of level s-1 that was completed LAG
// iterations earlier (in plane terms, level s trails level s-1 by R + LAG
// planes; each level keeps the last LAG output planes of the level below in
// registers). Within one iteration the levels therefore do not depend on each
// other: all their y exchanges go through LDS behind one barrier, and the
// neighbours' edges a level needs were published LAG iterations ago, which
// leaves the exchange that much time (the paper's lazy streaming, Section
// 4.3.2: one synchronisation per z-step for all levels).
//
// Exchange protocol per iteration i:
//   * start: every wave waits until its own vector-memory operations of the
//     previous iteration are complete (gfx9 counts loads and stores together);
//     the edge strips were written through to the point of device coherence
//     (agent-scope stores), so after a barrier one lane publishes
//     progress = i;
//   * the faces of iteration i + 1 come from the neighbours' strips of
//     iteration i + 1 - LAG: wave 0 waits (bounded by the watchdog) until
//     every neighbour's progress is at least i + 2 - LAG, then, after a
//     barrier, they are loaded with agent-scope loads;
//   * the tile's own strips of iteration i go to ring slot i mod (2 LAG). A
//     slot is rewritten only after every neighbour has finished reading it,
//     which the wait above implies (2 LAG >= 2 LAG - 2).
// Faces outside the interior are the Dirichlet halo and come from `src`.
//
// Summation order: dense-box order (dz, dy, dx ascending), from +0.0, one fused
// multiply-add per term, so results equal an unblocked sweep bit for bit.
#pragma once
#include "tb3d_impl.hpp"

namespace stencil_impl {
namespace tb3dd {

using stencil_dev::wait_vmem_complete;
using tb3d::BX;
using tb3d::kThreads;
using tb3d::LX;
using tb3d::LY;
using tb3d::TX;

// Iterations between a level's output and its use by the next level: 3 for
// radius 1 and 4 for radius 2, so that the unrolled iteration period
// lcm(2R, LAG) stays short (6 and 4); the ring holds 2 LAG slots per tile.
constexpr int lag_of(int r) { return r == 1 ? 3 : 4; }
constexpr int ring_of(int r) { return 2 * lag_of(r); }

// LDS of one level (the level's input plane), per iteration:
//   side faces [2][R][H]: left (x = X0 - R + c) then right (x = X0 + TX + c),
//     y = Y0 - R + j, H = TY + 2R rows (the corner rows included);
//   rows [BY][BX][NL_] (element-major over "lane slots"): the lanes' own cells,
//     plus VR virtual lane rows above and below the tile that hold the top and
//     bottom faces, so the rows above and below a lane always sit at a fixed
//     distance from its own slot.
template <int R, int BY>
struct Lvl {
  static constexpr int TY = LY * BY;
  static constexpr int H = TY + 2 * R;
  static constexpr int VR = (R + BY - 1) / BY;       // virtual lane rows above / below
  static constexpr int NLS = (LY + 2 * VR) * LX;     // lane slots
  static constexpr int kSide = 2 * R * H;
  static constexpr int kRows = BY * BX * NLS;
  static constexpr int kStride = kSide + kRows;       // elements per level
  static constexpr int kPerPlane = 2 * R * H + 2 * R * TX;  // face entries per plane
  static constexpr int KF = (kPerPlane + kThreads - 1) / kThreads;
};

// One level's published edges of one plane, in the halo ring:
//   top [R][TX] (tile rows 0..R-1), bottom [R][TX] (rows TY-R..TY-1),
//   left [R][TY] (columns 0..R-1), right [R][TY] (columns TX-R..TX-1).
template <int R, int BY>
struct Strips {
  static constexpr int TY = LY * BY;
  static constexpr int kTop = 0;
  static constexpr int kBottom = R * TX;
  static constexpr int kLeft = 2 * R * TX;
  static constexpr int kRight = 2 * R * TX + R * TY;
  static constexpr int kPerLevel = 2 * R * (TX + TY);
};

// Published levels per ring slot (the ring's level stride).
constexpr int ring_levels(int depth) { return depth > 1 ? depth - 1 : 1; }

template <typename Real, int R, int BY, int DEPTH>
struct DevLds {
  static constexpr size_t kBytes = (size_t)DEPTH * Lvl<R, BY>::kStride * sizeof(Real);
};

// Ring elements per tile (all slots and levels).
template <int R, int BY>
constexpr int64_t ring_per_tile(int depth) {
  return (int64_t)ring_of(R) * ring_levels(depth) * Strips<R, BY>::kPerLevel;
}

// Cache policy of the ring's loads and stores: device scope (SC1). A store
// is written through to the point of device coherence; a load reads there.
constexpr int kDeviceScope = 16;

template <typename Real>
__device__ __forceinline__ void ring_store(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff, Real v);
template <>
__device__ __forceinline__ void ring_store<double>(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff,
                                                   double v) {
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), rs, voff, soff, kDeviceScope);
}
template <>
__device__ __forceinline__ void ring_store<float>(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff,
                                                  float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rs, voff, soff, kDeviceScope);
}
template <typename Real>
__device__ __forceinline__ Real ring_load(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff);
template <>
__device__ __forceinline__ double ring_load<double>(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff) {
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, kDeviceScope));
}
template <>
__device__ __forceinline__ float ring_load<float>(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, voff, soff, kDeviceScope));
}

enum FaceKind : int { kNone = 0, kSrc = 1, kRingFace = 2 };

template <typename Real, int R, int SHAPE, int DEPTH, int BY>
__global__ __launch_bounds__(kThreads) void tb3d_dev_kernel(const Tb3dDevParams<Real> a) {
  using LV = Lvl<R, BY>;
  using SL = Strips<R, BY>;
  constexpr int TY = LV::TY;
  constexpr int KF = LV::KF;
  constexpr int VR = LV::VR;
  constexpr int NLS = LV::NLS;
  constexpr int S = sizeof(Real);
  constexpr int NL = ring_levels(DEPTH);
  constexpr int kLag = lag_of(R);
  constexpr int kRing = ring_of(R);
  constexpr int UNROLL = tb3d::lcm_3d(2 * R, kLag);
  extern __shared__ char lds_raw[];
  Real* lds = (Real*)lds_raw;  // [DEPTH][kStride]
  __shared__ int s_ok;

  const int tid = threadIdx.x;
  const int lx = tid % LX;
  const int ly = tid / LX;
  const int lane = tid & 63;
  const int tile = blockIdx.x;
  const int gx = a.gx, gy = a.gy;
  const int tx = tile % gx, ty = tile / gx;
  const int P = (int)a.P, Qy = (int)a.Qy, Qz = (int)a.Qz;
  const int X0 = R + tx * TX, Y0 = R + ty * TY;
  const int d = a.depth;
  const Real* __restrict__ w = a.w;
  const uint32_t row_bytes = (uint32_t)(P * S);
  const uint32_t plane_bytes = (uint32_t)((int64_t)P * Qy * S);
  const uint32_t grid_bytes = (uint32_t)((int64_t)Qz * P * Qy * S);
  const __amdgpu_buffer_rsrc_t rs = stencil_dev::make_rsrc(a.src, grid_bytes);
  const __amdgpu_buffer_rsrc_t rd = stencil_dev::make_rsrc(a.dst, grid_bytes);
  const uint32_t ring_bytes = (uint32_t)((int64_t)gx * gy * ring_per_tile<R, BY>(DEPTH) * S);
  const __amdgpu_buffer_rsrc_t rr = stencil_dev::make_rsrc(a.ring, ring_bytes);
  const uint32_t blk_off = (uint32_t)(((Y0 + ly * BY) * P + X0 + lx * BX) * S);
  const int own_slot = (ly + VR) * LX + lx;  // the lane's slot in the rows area
  const uint32_t tile_ring = (uint32_t)(tile * ring_per_tile<R, BY>(DEPTH) * S);

  // face entries of this thread: entry e = tid + k * 256; f_lds is its place
  // in a level's LDS area
  int f_kind[KF];
  uint32_t f_src[KF], f_ring[KF];
  int f_lds[KF];
#pragma unroll
  for (int k = 0; k < KF; ++k) {
    const int e = tid + k * kThreads;
    f_kind[k] = kNone;
    f_src[k] = 0;
    f_ring[k] = 0;
    f_lds[k] = 0;
    if (e < LV::kPerPlane) {
      int fx, fy;
      bool corner = false;
      if (e < 2 * R * LV::H) {  // left then right side faces, [side][c][j]
        const int side = e / (R * LV::H), f = e % (R * LV::H);
        const int c = f / LV::H, j = f % LV::H;
        fx = side == 0 ? X0 - R + c : X0 + TX + c;
        fy = Y0 - R + j;
        corner = j < R || j >= TY + R;
        f_lds[k] = e;
      } else {  // top then bottom faces, [side][c][col]
        const int f = e - 2 * R * LV::H;
        const int side = f / (R * TX), g = f % (R * TX);
        const int c = g / TX, col = g % TX;
        const int yl = side == 0 ? c - R : TY + c;  // tile-local row
        fy = Y0 + yl;
        fx = X0 + col;
        const int lr = yl >= 0 ? yl / BY : -((-yl + BY - 1) / BY);  // lane row (virtual)
        const int j = yl - lr * BY;
        f_lds[k] = LV::kSide + (j * BX + col % BX) * NLS + (lr + VR) * LX + col / BX;
      }
      const int cx = fx < 0 ? 0 : (fx >= P ? P - 1 : fx);
      const int cy = fy < 0 ? 0 : (fy >= Qy ? Qy - 1 : fy);
      f_src[k] = (uint32_t)((cy * P + cx) * S);
      const bool interior = fx >= R && fx < P - R && fy >= R && fy < Qy - R;
      if (!interior) {
        f_kind[k] = kSrc;
      } else if (!(SHAPE == kStar && corner)) {
        // owner tile and the strip entry holding this cell
        const int otx = (fx - R) / TX, oty = (fy - R) / TY;
        const int xl = fx - R - otx * TX, yl = fy - R - oty * TY;
        int off;
        if (otx != tx) off = otx < tx ? SL::kRight + (xl - (TX - R)) * TY + yl : SL::kLeft + xl * TY + yl;
        else off = oty < ty ? SL::kBottom + (yl - (TY - R)) * TX + xl : SL::kTop + yl * TX + xl;
        f_kind[k] = kRingFace;
        f_ring[k] = (uint32_t)(((int64_t)(oty * gx + otx) * ring_per_tile<R, BY>(DEPTH) + off) * S);
      }
    }
  }
  // wave 0, lanes 0..7: the neighbour tiles whose progress this tile waits for
  int nb = -1;
  {
    const int ddx[8] = {-1, 1, 0, 0, -1, 1, -1, 1};
    const int ddy[8] = {0, 0, -1, 1, -1, -1, 1, 1};
    if (lane < 8 && (SHAPE != kStar || lane < 4)) {
      const int nx = tx + ddx[lane], ny = ty + ddy[lane];
      if (nx >= 0 && nx < gx && ny >= 0 && ny < gy) nb = ny * gx + nx;
    }
  }
  // own edge cells in the ring: per-lane byte offsets of the strips' first
  // cells (a cell (j, q) of the block adds a constant)
  const uint32_t o_top = (uint32_t)((SL::kTop + (ly * BY) * TX + lx * BX) * S);
  const uint32_t o_bot = (uint32_t)((SL::kBottom + (ly * BY - (TY - R)) * TX + lx * BX) * S);
  const uint32_t o_left = (uint32_t)((SL::kLeft + (lx * BX) * TY + ly * BY) * S);
  const uint32_t o_right = (uint32_t)((SL::kRight + (lx * BX - (TX - R)) * TY + ly * BY) * S);

  Real A[DEPTH][2 * R][BY][BX];
  Real lag[NL][kLag][BY][BX];
  Real L0[BY][BX];
  Real F0[KF];
  Real G[NL][KF];
#pragma unroll
  for (int s = 0; s < DEPTH; ++s)
#pragma unroll
    for (int sl = 0; sl < 2 * R; ++sl)
#pragma unroll
      for (int j = 0; j < BY; ++j)
#pragma unroll
        for (int q = 0; q < BX; ++q) A[s][sl][j][q] = Real(0);
#pragma unroll
  for (int s = 0; s < NL; ++s)
#pragma unroll
    for (int l = 0; l < kLag; ++l)
#pragma unroll
      for (int j = 0; j < BY; ++j)
#pragma unroll
        for (int q = 0; q < BX; ++q) lag[s][l][j][q] = Real(0);
#pragma unroll
  for (int s = 0; s < NL; ++s)
#pragma unroll
    for (int k = 0; k < KF; ++k) G[s][k] = Real(0);
  // plane 0 and its faces
#pragma unroll
  for (int j = 0; j < BY; ++j) stencil_dev::load_vec<Real, BX>(rs, blk_off + (uint32_t)j * row_bytes, 0, L0[j]);
#pragma unroll
  for (int k = 0; k < KF; ++k)
    F0[k] = (tid + k * kThreads) < LV::kPerPlane ? stencil_dev::load_one<Real>(rs, f_src[k], 0) : Real(0);

  const int n_iter = Qz + R + (d - 1) * (R + kLag);
  const unsigned base = a.flag_base;
  const int64_t t_limit = a.timeout_ticks;
  bool failed = false;

  for (int it0 = 0; it0 < n_iter && !failed; it0 += UNROLL) {
#pragma unroll
    for (int ph = 0; ph < UNROLL; ++ph) {
      const int i = it0 + ph;
      if (i >= n_iter || failed) break;

      // ---- 1. publish the previous iteration
      wait_vmem_complete();
      __syncthreads();
      if (tid == 0 && i > 0)
        __hip_atomic_store(a.flags + tile, base + (unsigned)i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

      // ---- 2. this iteration's faces and own rows into LDS
      Real x1[BY][BX];
#pragma unroll
      for (int j = 0; j < BY; ++j)
#pragma unroll
        for (int q = 0; q < BX; ++q) x1[j][q] = L0[j][q];
#pragma unroll
      for (int k = 0; k < KF; ++k) {
        if (tid + k * kThreads < LV::kPerPlane) {
          lds[f_lds[k]] = F0[k];
#pragma unroll
          for (int s = 2; s <= DEPTH; ++s)
            if (s <= d) lds[(s - 1) * LV::kStride + f_lds[k]] = G[s - 2][k];
        }
      }
#pragma unroll
      for (int s = 1; s <= DEPTH; ++s) {
        if (s > d) break;
        Real* xs = lds + (s - 1) * LV::kStride + LV::kSide + own_slot;
#pragma unroll
        for (int j = 0; j < BY; ++j)
#pragma unroll
          for (int q = 0; q < BX; ++q) xs[(j * BX + q) * NLS] = s == 1 ? x1[j][q] : lag[s - 2][ph % kLag][j][q];
      }

      // ---- 3. the neighbours' strips needed next iteration are published
      const int need = i + 2 - kLag;
      if (tid < 64) {
        int ok = 1;
        if (d >= 2 && need > 0) {
          const unsigned target = base + (unsigned)need;
          const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
          while (true) {
            unsigned v = target;
            if (nb >= 0) v = __hip_atomic_load(a.flags + nb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (__builtin_amdgcn_ballot_w64(v < target) == 0ull) break;
            const unsigned e = __builtin_amdgcn_readfirstlane(
                __hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            if (e != 0u) {
              ok = 0;
              break;
            }
            if ((int64_t)(__builtin_amdgcn_s_memrealtime() - t0) > t_limit) {
              if (lane == 0) __hip_atomic_store(a.err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              ok = 0;
              break;
            }
            __builtin_amdgcn_s_sleep(1);
          }
        }
        if (lane == 0) s_ok = ok;
      }
      __syncthreads();
      if (__builtin_amdgcn_readfirstlane(s_ok) == 0) {
        failed = true;
        break;
      }

      // ---- 4. loads for the next iteration: input plane i + 1 and its faces,
      // and the faces of levels 2..d
      {
        const int ip = i + 1;
        if (ip < Qz) {
          const uint32_t pb = (uint32_t)ip * plane_bytes;
#pragma unroll
          for (int j = 0; j < BY; ++j)
            stencil_dev::load_vec<Real, BX>(rs, blk_off + (uint32_t)j * row_bytes, pb, L0[j]);
#pragma unroll
          for (int k = 0; k < KF; ++k)
            if (tid + k * kThreads < LV::kPerPlane) F0[k] = stencil_dev::load_one<Real>(rs, f_src[k], pb);
        }
        const int slot_next = (ip - kLag) % kRing;  // ip - kLag >= 0 whenever a level >= 2 is valid
#pragma unroll
        for (int s = 2; s <= DEPTH; ++s) {
          if (s > d) break;
          const int u = ip - (s - 1) * (R + kLag);
          if (u >= 0 && u < Qz) {
            const uint32_t soff = (uint32_t)((slot_next * NL + (s - 2)) * SL::kPerLevel * S);
            const uint32_t pb = (uint32_t)u * plane_bytes;
#pragma unroll
            for (int k = 0; k < KF; ++k) {
              if (f_kind[k] == kRingFace) G[s - 2][k] = ring_load<Real>(rr, f_ring[k], soff);
              else if (f_kind[k] == kSrc) G[s - 2][k] = stencil_dev::load_one<Real>(rs, f_src[k], pb);
            }
          }
        }
      }

      // ---- 5. every level, top down (a level reads the lag slot before the
      // level below overwrites it)
      const int slot_now = i % kRing;
#pragma unroll
      for (int s = DEPTH; s >= 1; --s) {
        if (s > d) continue;
        const int u = i - (s - 1) * (R + kLag);
        const bool ok = u >= 0 && u < Qz;
        const Real* lv = lds + (s - 1) * LV::kStride;
        const Real* xs = lv + LV::kSide + own_slot;
        Real xin[BY][BX];
#pragma unroll
        for (int j = 0; j < BY; ++j)
#pragma unroll
          for (int q = 0; q < BX; ++q) xin[j][q] = s == 1 ? x1[j][q] : lag[s - 2][ph % kLag][j][q];

        Real ext[BY + 2 * R][BX + 2 * R];
#pragma unroll
        for (int jj = 0; jj < BY + 2 * R; ++jj) {
          if (jj >= R && jj < R + BY) {
#pragma unroll
            for (int q = 0; q < BX; ++q) ext[jj][R + q] = xin[jj - R][q];
          } else {
            // a row of the lane above / below (or of the top / bottom face)
            const int dl = (jj - R) >= 0 ? (jj - R) / BY : -((R - jj + BY - 1) / BY);
            const int j2 = (jj - R) - dl * BY;
#pragma unroll
            for (int q = 0; q < BX; ++q) ext[jj][R + q] = xs[(j2 * BX + q) * NLS + dl * LX];
          }
          // x extension (a star's off-row taps have dx = 0: only its own rows)
          if (SHAPE != kStar || (jj >= R && jj < R + BY)) {
#pragma unroll
            for (int c = 0; c < R; ++c) {
              const Real oldl = lv[c * LV::H + ly * BY + jj];
              const Real oldr = lv[(R + c) * LV::H + ly * BY + jj];
              ext[jj][c] = tb3d::dpp_keep<tb3d::kDppRowShr1>(oldl, ext[jj][BX + c]);
              ext[jj][BX + R + c] = tb3d::dpp_keep<tb3d::kDppRowShl1>(oldr, ext[jj][R + c]);
            }
          }
        }

        // push the arriving plane u into the outputs u-R .. u+R (halo planes
        // keep their input values)
        Real out[BY][BX];
        {
          const int o = u - R;
          const int sl = ph % (2 * R);
          const bool halo = (o < R) || (o >= Qz - R);
          if (ok && !halo) tb3d::add_plane<Real, R, SHAPE, BY>(A[s - 1][sl], ext, w, R);
#pragma unroll
          for (int j = 0; j < BY; ++j)
#pragma unroll
            for (int q = 0; q < BX; ++q) out[j][q] = A[s - 1][sl][j][q];
        }
        if (ok) {
#pragma unroll
          for (int dz = R - 1; dz >= -R; --dz) {
            const int o = u - dz;
            const int sl = tb3d::pmod(ph - dz - R, 2 * R);
            const bool halo = (o < R) || (o >= Qz - R);
            if (halo) {
              if (dz == 0) {
#pragma unroll
                for (int j = 0; j < BY; ++j)
#pragma unroll
                  for (int q = 0; q < BX; ++q) A[s - 1][sl][j][q] = xin[j][q];
              }
            } else {
              if (dz == -R) {
#pragma unroll
                for (int j = 0; j < BY; ++j)
#pragma unroll
                  for (int q = 0; q < BX; ++q) A[s - 1][sl][j][q] = Real(0);
              }
              tb3d::add_plane<Real, R, SHAPE, BY>(A[s - 1][sl], ext, w, dz);
            }
          }
        }

        const int o = u - R;  // the plane level s completed
        if (s < d) {
          // the next level takes it LAG iterations from now; its edges go to
          // the ring for the neighbours
#pragma unroll
          for (int j = 0; j < BY; ++j)
#pragma unroll
            for (int q = 0; q < BX; ++q) lag[s - 1 < NL ? s - 1 : 0][ph % kLag][j][q] = out[j][q];
          const uint32_t soff = tile_ring + (uint32_t)((slot_now * NL + (s - 1)) * SL::kPerLevel * S);
#pragma unroll
          for (int j = 0; j < BY; ++j) {
            const int yl = ly * BY + j;
#pragma unroll
            for (int q = 0; q < BX; ++q) {
              const int xl = lx * BX + q;
              if (yl < R) ring_store<Real>(rr, o_top + (uint32_t)((j * TX + q) * S), soff, out[j][q]);
              if (yl >= TY - R) ring_store<Real>(rr, o_bot + (uint32_t)((j * TX + q) * S), soff, out[j][q]);
              if (xl < R) ring_store<Real>(rr, o_left + (uint32_t)((q * TY + j) * S), soff, out[j][q]);
              if (xl >= TX - R) ring_store<Real>(rr, o_right + (uint32_t)((q * TY + j) * S), soff, out[j][q]);
            }
          }
        } else if (o >= 0 && o < Qz) {
          const uint32_t pb = (uint32_t)o * plane_bytes;
#pragma unroll
          for (int j = 0; j < BY; ++j)
            stencil_dev::store_vec<Real, BX>(rd, blk_off + (uint32_t)j * row_bytes, pb, out[j]);
        }
      }
    }
  }
}

// Deepest compiled depth of a device-tiled variant (0: none).
constexpr int dev_max_depth_c(int dtype, int r, int shape) {
  if (r == 1 && shape == kStar) return dtype == kF64 ? 8 : 9;
  if (r == 2 && shape == kStar) return dtype == kF64 ? 4 : 6;
  if (r == 1 && shape == kBox) return dtype == kF64 ? 6 : 8;
  return 0;
}

template <typename Real, int R, int SHAPE, int D>
hipError_t dev_launch_depth(int cdepth, const Tb3dDevParams<Real>* p, hipStream_t s) {
  if constexpr (D == 0) {
    return hipErrorInvalidValue;
  } else {
    if (cdepth == D) {
      constexpr int BY = 1;
      const void* fn = (const void*)&tb3d_dev_kernel<Real, R, SHAPE, D, BY>;
      constexpr size_t lds = DevLds<Real, R, BY, D>::kBytes;
      hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      void* args[] = {(void*)p};
      return hipLaunchKernel(fn, dim3(p->gx * p->gy), dim3(kThreads), args, lds, s);
    }
    return dev_launch_depth<Real, R, SHAPE, D - 1>(cdepth, p, s);
  }
}

}  // namespace tb3dd

template <typename Real, int R>
hipError_t tb3d_dev_launch_r(int shape, int cdepth, const Tb3dDevParams<Real>* p, hipStream_t s) {
  using namespace tb3dd;
  constexpr int dt = tb3d::dtype_code<Real>();
  if (shape == kStar) {
    if constexpr (dev_max_depth_c(dt, R, kStar) > 0)
      return dev_launch_depth<Real, R, kStar, dev_max_depth_c(dt, R, kStar)>(cdepth, p, s);
  } else if (shape == kBox) {
    if constexpr (dev_max_depth_c(dt, R, kBox) > 0)
      return dev_launch_depth<Real, R, kBox, dev_max_depth_c(dt, R, kBox)>(cdepth, p, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace stencil_impl
