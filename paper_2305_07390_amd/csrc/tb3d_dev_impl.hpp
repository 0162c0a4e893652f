// tb3d_dev_impl.hpp -- 3D device tiling (kernel templates).
//
// The paper's device tiling (Section 4.1, "one tile at a time"; Section 5.2.2
// for its cost): the whole xy plane of the grid is one device-sized tile,
// split among workgroups without overlap, and every workgroup streams all of
// z through every time level of the pass. A tile computes no redundant
// margin; instead its neighbours' edges of every level are exchanged through
// global memory after each z-step.
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
// Exchange protocol (tagged words, no counters): every 32-bit word of a
// published edge travels with the tag of its iteration in one 64-bit store
// (an FP64 value is two such words), written through to the point of device
// coherence; the edges of iteration i are staged in LDS and stored at the
// start of iteration i + 1. A reader loads the words it needs for iteration
// i + 1 during iteration i (device-scope loads) and, before using them,
// re-loads any word whose tag is not yet the expected one (bounded by the
// watchdog). A 64-bit store is single-copy atomic, so a word with the right
// tag carries the right value, and no store has to be waited for before
// another is published. Ring slot reuse: level 2 checks its words every
// iteration, so no tile runs more than LAG iterations ahead of a neighbour;
// a slot is rewritten 2 LAG iterations later, after every reader is done
// with it. The ring is zeroed before each execution and tags start at 1.
// Faces outside the interior are the Dirichlet halo and come from `src`.
//
// Summation order: dense-box order (dz, dy, dx ascending), from +0.0, one fused
// multiply-add per term, so results equal an unblocked sweep bit for bit.
#pragma once
#include "tb3d_impl.hpp"

namespace stencil_impl {
namespace tb3dd {

using tb3d::BX;
using tb3d::kThreads;
using tb3d::LX;
using tb3d::LY;
using tb3d::TX;

// Iterations between a level's output and its use by the next level: 3 for
// radius 1 and 4 for radius 2, so that the unrolled iteration period
// lcm(2R, LAG, Z0) stays short (6 and 4); the ring holds 2 LAG slots per tile.
constexpr int lag_of(int r) { return r == 1 ? 3 : 4; }
constexpr int ring_of(int r) { return 2 * lag_of(r); }
// Input planes in flight per lane. One workgroup per CU streams 64 x 16
// cells per plane, so by Little's law (bytes in flight = bandwidth x
// latency, paper Section 6.1) a deep prefetch is what keeps HBM busy: two
// planes (16 KB FP64 per CU) measured at about 1.4 TB/s. Deep FP64 variants
// keep fewer for their registers. A divisor-friendly count keeps the unrolled
// period lcm(2R, LAG, Z0) at 6 (radius 1) and 4 (radius 2).
constexpr int z0_of(bool f64, int r, int depth) {
  if (r == 1) return (f64 && depth > 4) ? 3 : 6;
  return 4;
}

// LDS of one level (the level's input plane), per iteration:
//   side faces [2][R][H]: left (x = X0 - R + c) then right (x = X0 + TX + c),
//     y = Y0 - R + j, H = TY + 2R rows (the corner rows included);
//   rows [BY][BX][NLS] (element-major over "lane slots"): the lanes' own
//     cells, plus VR virtual lane rows above and below the tile that hold the
//     top and bottom faces, so the rows above and below a lane always sit at
//     a fixed distance from its own slot.
template <int R, int BY>
struct Lvl {
  static constexpr int TY = LY * BY;
  static constexpr int H = TY + 2 * R;
  static constexpr int VR = (R + BY - 1) / BY;    // virtual lane rows above / below
  static constexpr int NLS = (LY + 2 * VR) * LX;  // lane slots
  static constexpr int kSide = 2 * R * H;
  static constexpr int kRows = BY * BX * NLS;
  static constexpr int kStride = kSide + kRows + 1;  // elements per level (+1: a slot no one reads)
  static constexpr int kPerPlane = 2 * R * H + 2 * R * TX;  // face entries per plane
  static constexpr int KF = (kPerPlane + kThreads - 1) / kThreads;
};

// One level's published edges of one plane, in the halo ring (cells):
//   top [R][TX] (tile rows 0..R-1), bottom [R][TX] (rows TY-R..TY-1),
//   left [R][TY] (columns 0..R-1), right [R][TY] (columns TX-R..TX-1).
// A cell takes one 64-bit ring word per 32 bits of value: (value word, tag).
template <int R, int BY>
struct Strips {
  static constexpr int TY = LY * BY;
  static constexpr int kTop = 0;
  static constexpr int kBottom = R * TX;
  static constexpr int kLeft = 2 * R * TX;
  static constexpr int kRight = 2 * R * TX + R * TY;
  static constexpr int kPerLevel = 2 * R * (TX + TY);
};

template <typename Real>
constexpr int words_of() { return sizeof(Real) / 4; }  // 64-bit ring words per cell

// Published levels per ring slot (the ring's level stride).
constexpr int ring_levels(int depth) { return depth > 1 ? depth - 1 : 1; }

// LDS: the levels' areas, then the staging area of the edges a tile
// publishes: [ring_levels(DEPTH)][Strips::kPerLevel] cells.
template <typename Real, int R, int BY, int DEPTH>
struct DevLds {
  static constexpr size_t kLevels = (size_t)DEPTH * Lvl<R, BY>::kStride;
  static constexpr size_t kStage = (size_t)(DEPTH > 1 ? DEPTH - 1 : 1) * (2 * R * (TX + LY * BY));
  static constexpr size_t kBytes = (kLevels + kStage) * sizeof(Real);
};

// Ring cells per tile (all slots and levels).
template <int R, int BY>
constexpr int64_t ring_per_tile(int depth) {
  return (int64_t)ring_of(R) * ring_levels(depth) * Strips<R, BY>::kPerLevel;
}

// Cache policy of the ring's loads and stores: device scope (SC1). A store
// is written through to the point of device coherence; a load reads there.
constexpr int kDeviceScope = 16;

// Byte offset beyond every buffer's range (buffers stay below 2 GiB): a load
// there returns zero and a store there is dropped. Inactive lanes and planes
// outside the grid use it instead of a branch, so every iteration issues the
// same memory instructions and the compiler's wait counts stay exact (a
// branch around a load or store makes them path-dependent, and it then
// waits for everything).
constexpr uint32_t kOff = 0x80000000u;

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// (value word, tag) pairs of one cell.
template <typename Real>
struct Tagged {
  u32x2 w[words_of<Real>()];
};

template <typename Real>
__device__ __forceinline__ void ring_put(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff, Real v,
                                         unsigned tag) {
  constexpr int W = words_of<Real>();
  unsigned bits[W];
  __builtin_memcpy(bits, &v, sizeof(Real));
#pragma unroll
  for (int k = 0; k < W; ++k)
    __builtin_amdgcn_raw_buffer_store_b64(u32x2{bits[k], tag}, rs, voff + 8 * k, soff, kDeviceScope);
}
template <typename Real>
__device__ __forceinline__ Tagged<Real> ring_get(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff) {
  Tagged<Real> t;
#pragma unroll
  for (int k = 0; k < words_of<Real>(); ++k)
    t.w[k] = __builtin_amdgcn_raw_buffer_load_b64(rs, voff + 8 * k, soff, kDeviceScope);
  return t;
}
template <typename Real>
__device__ __forceinline__ bool tag_ok(const Tagged<Real>& t, unsigned tag) {
  bool ok = true;
#pragma unroll
  for (int k = 0; k < words_of<Real>(); ++k) ok = ok && t.w[k].y == tag;
  return ok;
}
template <typename Real>
__device__ __forceinline__ Real tag_value(const Tagged<Real>& t) {
  unsigned bits[words_of<Real>()];
#pragma unroll
  for (int k = 0; k < words_of<Real>(); ++k) bits[k] = t.w[k].x;
  Real v;
  __builtin_memcpy(&v, bits, sizeof(Real));
  return v;
}
template <typename Real>
__device__ __forceinline__ Tagged<Real> tag_make(Real v, unsigned tag) {
  Tagged<Real> t;
  unsigned bits[words_of<Real>()];
  __builtin_memcpy(bits, &v, sizeof(Real));
#pragma unroll
  for (int k = 0; k < words_of<Real>(); ++k) t.w[k] = u32x2{bits[k], tag};
  return t;
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
  constexpr int CB = 8 * words_of<Real>();  // ring bytes per cell
  constexpr int NL = ring_levels(DEPTH);
  constexpr int kLag = lag_of(R);
  constexpr int kRing = ring_of(R);
  constexpr int Z0 = z0_of(S == 8, R, DEPTH);
  constexpr int UNROLL = tb3d::lcm_3d(tb3d::lcm_3d(2 * R, kLag), Z0);
  extern __shared__ char lds_raw[];
  Real* lds = (Real*)lds_raw;  // [DEPTH][kStride]
  __shared__ int s_fail;

  const int tid = threadIdx.x;
  const int lx = tid % LX;
  const int ly = tid / LX;
  const int tile = blockIdx.x;
  const int gx = a.gx;
  const int tx = tile % gx, ty = tile / gx;
  const int P = (int)a.P, Qy = (int)a.Qy, Qz = (int)a.Qz;
  const int X0 = R + tx * TX, Y0 = R + ty * TY;
  const Real* __restrict__ w = a.w;
  const uint32_t row_bytes = (uint32_t)(P * S);
  const uint32_t plane_bytes = (uint32_t)((int64_t)P * Qy * S);
  const uint32_t grid_bytes = (uint32_t)((int64_t)Qz * P * Qy * S);
  const __amdgpu_buffer_rsrc_t rs = stencil_dev::make_rsrc(a.src, grid_bytes);
  const __amdgpu_buffer_rsrc_t rd = stencil_dev::make_rsrc(a.dst, grid_bytes);
  const uint32_t ring_bytes = (uint32_t)((int64_t)gx * a.gy * ring_per_tile<R, BY>(DEPTH) * CB);
  const __amdgpu_buffer_rsrc_t rr = stencil_dev::make_rsrc(a.ring, ring_bytes);
  const uint32_t blk_off = (uint32_t)(((Y0 + ly * BY) * P + X0 + lx * BX) * S);
  const int own_slot = (ly + VR) * LX + lx;  // the lane's slot in the rows area
  const uint32_t tile_ring = (uint32_t)(tile * ring_per_tile<R, BY>(DEPTH) * CB);

  // face entries of this thread: entry e = tid + k * 256; f_lds is its place
  // in a level's LDS area
  int f_kind[KF];
  uint32_t f_src[KF], f_ring[KF];
  int f_lds[KF];
#pragma unroll
  for (int k = 0; k < KF; ++k) {
    const int e = tid + k * kThreads;
    f_kind[k] = kNone;
    f_src[k] = kOff;
    f_ring[k] = kOff;
    f_lds[k] = LV::kStride - 1;
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
      } else if (SHAPE == kStar && corner) {
        // never read
      } else {
        // owner tile and the strip entry holding this cell
        const int otx = (fx - R) / TX, oty = (fy - R) / TY;
        const int xl = fx - R - otx * TX, yl = fy - R - oty * TY;
        int off;
        if (otx != tx) off = otx < tx ? SL::kRight + (xl - (TX - R)) * TY + yl : SL::kLeft + xl * TY + yl;
        else off = oty < ty ? SL::kBottom + (yl - (TY - R)) * TX + xl : SL::kTop + yl * TX + xl;
        f_kind[k] = kRingFace;
        f_ring[k] = (uint32_t)(((int64_t)(oty * gx + otx) * ring_per_tile<R, BY>(DEPTH) + off) * CB);
      }
    }
  }
  // level 1 reads every face from the input plane (f_src); levels >= 2 read
  // only the Dirichlet faces from it (f_srcd), the others from the ring
  uint32_t f_srcd[KF];
#pragma unroll
  for (int k = 0; k < KF; ++k) f_srcd[k] = f_kind[k] == kSrc ? f_src[k] : kOff;
  // Publication: during an iteration the lanes holding edge cells write them
  // into the LDS staging area (strip layout); at the start of the next
  // iteration the whole workgroup stores the staged cells to the ring with
  // dense, fully used stores (about kPerLevel / 64 instructions per level
  // instead of a mostly idle store per edge cell in every wave).
  Real* stage = lds + DEPTH * LV::kStride;  // [NL][kPerLevel]
  const bool edge_lane = ly * BY < R || ly * BY + BY > TY - R || lx == 0 || lx == LX - 1;

  Real A[DEPTH][2 * R][BY][BX];
  Real lag[NL][kLag][BY][BX];
  Real L0[Z0][BY][BX];
  Real F0[Z0][KF];
  Tagged<Real> G[NL][KF];
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
    for (int k = 0; k < KF; ++k) G[s][k] = tag_make<Real>(Real(0), 0u);
  // planes 0 .. Z0-1 and their faces
#pragma unroll
  for (int p = 0; p < Z0; ++p) {
    const uint32_t pb = p < Qz ? (uint32_t)p * plane_bytes : kOff;
#pragma unroll
    for (int j = 0; j < BY; ++j) stencil_dev::load_vec<Real, BX>(rs, blk_off + (uint32_t)j * row_bytes, pb, L0[p][j]);
#pragma unroll
    for (int k = 0; k < KF; ++k) F0[p][k] = stencil_dev::load_one<Real>(rs, f_src[k], pb);
  }
  if (tid == 0) s_fail = 0;
  __syncthreads();

  const int n_iter = Qz + R + (DEPTH - 1) * (R + kLag);
  const unsigned tag0 = a.flag_base + 1u;  // tag of iteration 0 of this pass
  const int64_t t_limit = a.timeout_ticks;
  bool failed = false;

  // One iteration: i is the plane that enters level 1, ph = i mod UNROLL (a
  // constant once the calls below are unrolled, so that every register ring
  // is indexed at compile time).
  auto iteration = [&](const int i, const int ph) __attribute__((always_inline)) {
      // ---- 1. every wave is done with the LDS of the previous iteration
      __syncthreads();
      // publish the edges the previous iteration staged (levels 1..DEPTH-1)
      if (DEPTH > 1) {
        const int ip = i - 1;
        const unsigned tag_prev = tag0 + (unsigned)ip;
        const uint32_t slot_base = tile_ring + (uint32_t)(((ip >= 0 ? ip : 0) % kRing) * NL) * (uint32_t)(SL::kPerLevel * CB);
        constexpr int kCells = NL * SL::kPerLevel;
#pragma unroll
        for (int e0 = 0; e0 < kCells; e0 += kThreads) {
          const int e = e0 + tid;
          // iteration -1 does not exist; cells past the end are dropped
          const uint32_t voff = (ip >= 0 && e < kCells) ? (uint32_t)(e * CB) : kOff;
          ring_put<Real>(rr, voff, slot_base, stage[e < kCells ? e : 0], tag_prev);
        }
      }

      // ---- 2. this iteration's faces (the neighbours' words checked) and
      // own rows into LDS
      Real x1[BY][BX];
#pragma unroll
      for (int j = 0; j < BY; ++j)
#pragma unroll
        for (int q = 0; q < BX; ++q) x1[j][q] = L0[ph % Z0][j][q];
      {
        // the neighbours' words for the faces of levels >= 2 are of their
        // iteration i - LAG. Level 2's words are checked every iteration, even
        // when its plane is outside the grid: that keeps every tile within LAG
        // iterations of its neighbours, which the ring's reuse relies on.
        const int src_it = i - kLag;
        const unsigned want = tag0 + (unsigned)src_it;
        const int slot = src_it >= 0 ? src_it % kRing : 0;
#pragma unroll
        for (int k = 0; k < KF; ++k) {
          lds[f_lds[k]] = F0[ph % Z0][k];
#pragma unroll
          for (int s = 2; s <= DEPTH; ++s) {
            const int u = i - (s - 1) * (R + kLag);
            const bool needed = s == 2 ? src_it >= 0 : (u >= 0 && u < Qz);
            if (f_kind[k] == kRingFace && needed && !tag_ok<Real>(G[s - 2][k], want)) {
              // not yet published: re-load until the tag arrives
              const uint32_t soff = (uint32_t)((slot * NL + (s - 2)) * SL::kPerLevel * CB);
              const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
              while (true) {
                __builtin_amdgcn_s_sleep(1);
                G[s - 2][k] = ring_get<Real>(rr, f_ring[k], soff);
                if (tag_ok<Real>(G[s - 2][k], want)) break;
                if (__hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
                    (int64_t)(__builtin_amdgcn_s_memrealtime() - t0) > t_limit) {
                  __hip_atomic_store(a.err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                  s_fail = 1;
                  break;
                }
              }
            }
            lds[(s - 1) * LV::kStride + f_lds[k]] = tag_value<Real>(G[s - 2][k]);
          }
        }
      }
#pragma unroll
      for (int s = 1; s <= DEPTH; ++s) {
        Real* xs = lds + (s - 1) * LV::kStride + LV::kSide + own_slot;
#pragma unroll
        for (int j = 0; j < BY; ++j)
#pragma unroll
          for (int q = 0; q < BX; ++q) xs[(j * BX + q) * NLS] = s == 1 ? x1[j][q] : lag[s - 2][ph % kLag][j][q];
      }
      __syncthreads();
      // a failed wait ends the launch at the end of this block of iterations
      // (later waits see the error word and return at once)
      if (__builtin_amdgcn_readfirstlane(s_fail) != 0) failed = true;

      // ---- 3. loads ahead: input plane i + Z0 and its faces, and the
      // neighbours' words for the faces of levels 2..DEPTH of iteration i + 1
      {
        const int ip = i + Z0;
        const uint32_t pbi = ip < Qz ? (uint32_t)ip * plane_bytes : kOff;
#pragma unroll
        for (int j = 0; j < BY; ++j)
          stencil_dev::load_vec<Real, BX>(rs, blk_off + (uint32_t)j * row_bytes, pbi, L0[ph % Z0][j]);
#pragma unroll
        for (int k = 0; k < KF; ++k) F0[ph % Z0][k] = stencil_dev::load_one<Real>(rs, f_src[k], pbi);
        const int in1 = i + 1;
        const int src_it = in1 - kLag;
        const int slot = src_it >= 0 ? src_it % kRing : 0;
        const unsigned want = tag0 + (unsigned)src_it;
#pragma unroll
        for (int s = 2; s <= DEPTH; ++s) {
          const int u = in1 - (s - 1) * (R + kLag);
          const bool needed = s == 2 ? src_it >= 0 : (u >= 0 && u < Qz);
          const uint32_t soff = needed ? (uint32_t)((slot * NL + (s - 2)) * SL::kPerLevel * CB) : kOff;
          const uint32_t pb = (u >= 0 && u < Qz) ? (uint32_t)u * plane_bytes : kOff;
#pragma unroll
          for (int k = 0; k < KF; ++k) {
            // every thread issues both loads; the one that does not apply
            // reads out of range
            const Tagged<Real> rg = ring_get<Real>(rr, f_ring[k], soff);
            const Real sv = stencil_dev::load_one<Real>(rs, f_srcd[k], pb);
            G[s - 2][k] = f_kind[k] == kRingFace ? rg : tag_make<Real>(sv, want);
          }
        }
      }

      // ---- 4. every level, top down (a level reads the lag slot before the
      // level below overwrites it)
#pragma unroll
      for (int s = DEPTH; s >= 1; --s) {
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
        if (s < DEPTH) {
          // the next level takes it LAG iterations from now; its edges go to
          // the ring for the neighbours (every iteration, valid plane or not)
#pragma unroll
          for (int j = 0; j < BY; ++j)
#pragma unroll
            for (int q = 0; q < BX; ++q) lag[s - 1 < NL ? s - 1 : 0][ph % kLag][j][q] = out[j][q];
          if (edge_lane) {
            Real* sg = stage + (s - 1) * SL::kPerLevel;
#pragma unroll
            for (int j = 0; j < BY; ++j) {
              const int yl = ly * BY + j;
#pragma unroll
              for (int q = 0; q < BX; ++q) {
                const int xl = lx * BX + q;
                if (yl < R) sg[SL::kTop + yl * TX + xl] = out[j][q];
                if (yl >= TY - R) sg[SL::kBottom + (yl - (TY - R)) * TX + xl] = out[j][q];
                if (xl < R) sg[SL::kLeft + xl * TY + yl] = out[j][q];
                if (xl >= TX - R) sg[SL::kRight + (xl - (TX - R)) * TY + yl] = out[j][q];
              }
            }
          }
        } else {
          const uint32_t pb = (o >= 0 && o < Qz) ? (uint32_t)o * plane_bytes : kOff;
#pragma unroll
          for (int j = 0; j < BY; ++j)
            stencil_dev::store_vec<Real, BX>(rd, blk_off + (uint32_t)j * row_bytes, pb, out[j]);
        }
      }
  };

  // whole blocks of UNROLL iterations (no exit inside a block, so the wait
  // counts of one block carry over to the next), then the remainder
  const int nfull = n_iter / UNROLL;
  for (int b = 0; b < nfull; ++b) {
#pragma unroll
    for (int ph = 0; ph < UNROLL; ++ph) iteration(b * UNROLL + ph, ph);
    if (failed) return;
  }
#pragma unroll
  for (int ph = 0; ph < UNROLL; ++ph)
    if (nfull * UNROLL + ph < n_iter) iteration(nfull * UNROLL + ph, ph);
}

// Deepest compiled depth of a device-tiled variant (0: none).
constexpr int dev_max_depth_c(int dtype, int r, int shape) {
  if (r == 1 && shape == kStar) return dtype == kF64 ? 6 : 9;
  if (r == 2 && shape == kStar) return dtype == kF64 ? 2 : 6;
  if (r == 1 && shape == kBox) return dtype == kF64 ? 6 : 7;
  return 0;
}

template <typename Real, int R, int SHAPE, int D>
hipError_t dev_launch_depth(int cdepth, const Tb3dDevParams<Real>* p, hipStream_t s) {
  if constexpr (D == 0) {
    return hipErrorInvalidValue;
  } else {
    if (cdepth == D) {
      constexpr int BY = 1;  // every pass runs the kernel compiled for its own depth
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
