// tb3d_impl.hpp -- temporally blocked 3D stencil pass for gfx950 (kernel templates).
//
// One pass advances a padded 3D grid (z slowest, x fastest) by DEPTH Jacobi
// steps (paper Section 2.1) reading and writing every cell of HBM once.
//
// Decomposition: overlapped "SM tiling" with N.5-D streaming along z (paper
// Sections 2.1.2-2.1.3, 3.5-D blocking; Section 4.1 SM tiling):
//   * One workgroup of four waves owns an xy tile of 64 x (16 BY) cells and
//     streams a z segment of it. The 256 lanes form a 16 x 16 grid; lane
//     (lx, ly) holds a 4 x BY block of cells (x = 4 lx .. 4 lx + 3,
//     y = BY ly .. BY ly + BY - 1), BY = 4 or 2 (cells_y).
//     Wave w holds lane rows 4w .. 4w + 3, so one 16-lane DPP row is one lane
//     row of the tile.
//   * Time levels form a skewed wavefront along z: when input plane z arrives,
//     level s completes plane z - s*r. Each level keeps 2r partial-sum planes of
//     the lane's 16 cells in registers, and an arriving plane is pushed into the
//     partial sums of the 2r+1 output planes it touches (the paper's
//     multi-queue, Section 4.2, one queue per time level, rotated at compile
//     time).
//   * In-plane neighbours: x through DPP row shifts (row_shr:1 / row_shl:1
//     inside a lane row); y through an LDS exchange of each lane's top and
//     bottom r rows (extended by r cells on each side), one workgroup barrier
//     per level.
//   * Tile faces: the four faces of the tile (r cells thick, corners included)
//     are read from HBM for every input plane and kept in an LDS circular queue
//     indexed by plane modulo a power of two (the computed-address circular
//     multi-queue of Section 4.2.2). Lanes on the tile edge take their outside
//     neighbours from it, at every level. For a tile that touches the grid
//     boundary these are Dirichlet halo cells, which never change, so the
//     values are exact; inside the grid they are stale and their error moves
//     inward r cells per level, inside the redundant margin of the overlapped
//     tile (valid fraction of paper Section 5.2.1).
//   * Tiles start at the first interior cell of the grid, so no tile computes a
//     halo cell. Halo planes (z) are detected per workgroup (uniform branch).
//
// Summation order: dense-box order (dz, dy, dx ascending), from +0.0, one fused
// multiply-add per term; the push along z adds the dz groups in ascending
// order, so results equal an unblocked sweep bit for bit.
//
// Memory safety: every global access goes through a buffer descriptor bounded
// to the planes of the segment; LDS indices are bounded by construction.
#pragma once
#include "device_common.hpp"
#include "launch.hpp"

namespace stencil_impl {
using namespace stencil_dev;

namespace tb3d {

constexpr int BX = 4;      // cells per lane along x
constexpr int LX = 16;     // lanes along x (one DPP row)
constexpr int LY = 16;     // lanes along y (four waves)
constexpr int TX = LX * BX;  // tile extent in x (64)
constexpr int kThreads = LX * LY;

// Cells per lane along y (BY; the tile is LY * BY tall). FP64 tiles other
// than the radius-1 box hold 4 x 2 cells per lane: radius 2 does not fit the
// register file with 4 x 4 even at depth 1, and the 7-point star reaches
// depth 4 with four planes in flight (636 against 504 GCells/s for 4 x 4 at
// depth 2 on 512^3); the 27-point box is faster with 4 x 4 at depth 2.
constexpr int cells_y(bool f64, int r, int shape) { return (f64 && (r >= 2 || shape != kBox)) ? 2 : 4; }
constexpr int kRing = 16;  // planes in the face queue (power of two)

constexpr int pmod(int a, int m) { return ((a % m) + m) % m; }
constexpr int gcd_3d(int a, int b) { return b == 0 ? a : gcd_3d(b, a % b); }
constexpr int lcm_3d(int a, int b) { return a / gcd_3d(a, b) * b; }

// DPP row shifts by one lane inside each 16-lane row; lanes whose source is
// outside the row keep `old`.
constexpr int kDppRowShr1 = 0x111;
constexpr int kDppRowShl1 = 0x101;

template <int CTRL>
__device__ __forceinline__ double dpp_keep(double old, double v) {
  unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  unsigned long long o = __builtin_bit_cast(unsigned long long, old);
  int lo = __builtin_amdgcn_update_dpp((int)(unsigned)(o & 0xffffffffull),
                                       (int)(unsigned)(b & 0xffffffffull), CTRL, 0xf, 0xf, false);
  int hi = __builtin_amdgcn_update_dpp((int)(unsigned)(o >> 32), (int)(unsigned)(b >> 32), CTRL,
                                       0xf, 0xf, false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_keep(float old, float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old),
                                                               __builtin_bit_cast(int, v), CTRL,
                                                               0xf, 0xf, false));
}

// Face queue layout per plane slot (Real elements):
//   left  [R][TY]            x = X0 - R + c, y = Y0 + j
//   right [R][TY]            x = X0 + TX + c
//   top   [R][TX + 2R]       y = Y0 - R + c, x = X0 - R + i
//   bottom[R][TX + 2R]       y = Y0 + TY + c
template <int R, int BY>
struct FaceLayout {
  static constexpr int TY = LY * BY;
  static constexpr int kLeft = 0;
  static constexpr int kRight = R * TY;
  static constexpr int kTop = 2 * R * TY;
  static constexpr int kBottom = 2 * R * TY + R * (TX + 2 * R);
  static constexpr int kPerPlane = 2 * R * TY + 2 * R * (TX + 2 * R);
};

// Exchange buffer layout, element-major so that consecutive lanes touch
// consecutive words (no bank conflicts): element e of lane l at e * 256 + l,
// elements = top R rows then bottom R rows of the lane's block, each
// (BX + 2R) wide (x-extended).
template <int R>
struct XchgLayout {
  static constexpr int kRowW = BX + 2 * R;
  static constexpr int kPerLane = 2 * R * kRowW;
  static constexpr int kPerBuf = kThreads * kPerLane;
  static constexpr int kBufs = (R == 1) ? 2 : 1;
};

template <typename Real, int R, int BY>
struct Lds {
  static constexpr int kFaces = kRing * FaceLayout<R, BY>::kPerPlane;
  static constexpr int kXchg = XchgLayout<R>::kBufs * XchgLayout<R>::kPerBuf;
  static constexpr size_t kBytes = (size_t)(kFaces + kXchg) * sizeof(Real);
};

// Planes in flight per lane (loaded Z0 - 1 iterations before use). Deeper
// rings hide more HBM latency (one workgroup per CU has little else to hide
// it with); FP64 star and box variants at depth 2 keep 2, the most their
// registers allow without spilling.
//
// Ablation switch (paper Section 7, breakdown study; see
// paper_2305_07390_amd/ablation.py): STENCIL_ABL_PLANES caps the planes in
// flight (at least 2, one plane ahead: the ring also carries the face values
// of the next plane).
#ifndef STENCIL_ABL_PLANES
#define STENCIL_ABL_PLANES 4
#endif
static_assert(STENCIL_ABL_PLANES >= 2, "the plane ring holds at least the next plane");
constexpr int plane_ring_full(bool f64, int r, int shape, int depth) {
  if (!f64 || shape == kGeneral) return 4;
  if (shape == kStar) return (r == 1 || depth == 1) ? 4 : 2;
  return 2;
}
constexpr int plane_ring(bool f64, int r, int shape, int depth) {
  return plane_ring_full(f64, r, shape, depth) < STENCIL_ABL_PLANES ? plane_ring_full(f64, r, shape, depth)
                                                                     : STENCIL_ABL_PLANES;
}

template <typename Real, int R, int DEPTH, int Z0_, int BY>
struct State {
  static constexpr int Z0 = Z0_;  // plane prefetch ring
  Real L0[Z0][BY][BX];
  Real A[DEPTH][2 * R][BY][BX];
  Real F[Z0][3];  // face values this lane loads for planes in flight (<= 3 per lane)
};

struct Tile {
  __amdgpu_buffer_rsrc_t rs, rd;
  uint32_t blk_off;     // byte offset of the lane's block (row 0) inside a plane
  uint32_t st_off;      // same, or past the descriptor for lanes outside the valid range
  uint32_t plane_bytes, row_bytes;
  int zs, Z0, Z1, Qz, n_iter;
  int d;  // levels of this pass (<= the compiled depth)
  int lo[13];
  // face cells this lane loads (plane-relative byte offset, face queue index)
  uint32_t f_off[3];
  int f_idx[3];
  int n_f;
};

template <typename Real, int R, int SHAPE, int BY>
__device__ __forceinline__ void add_plane(Real (&acc)[BY][BX], const Real (&ext)[BY + 2 * R][BX + 2 * R],
                                          const Real* __restrict__ w, int dz) {
  constexpr int SIDE = 2 * R + 1;
#pragma unroll
  for (int dy = -R; dy <= R; ++dy) {
#pragma unroll
    for (int dx = -R; dx <= R; ++dx) {
      if (SHAPE == kStar && ((dz != 0) + (dy != 0) + (dx != 0)) > 1) continue;
      const Real c = w[((dz + R) * SIDE + (dy + R)) * SIDE + (dx + R)];
      if (SHAPE == kGeneral && c == Real(0)) continue;
#pragma unroll
      for (int j = 0; j < BY; ++j)
#pragma unroll
        for (int i = 0; i < BX; ++i) acc[j][i] = fma_t(c, ext[j + R + dy][i + R + dx], acc[j][i]);
    }
  }
}

// One input plane through all levels (iteration i, phase ph).
template <typename Real, int R, int SHAPE, int DEPTH, bool GENERAL, int Z0, int BY>
__device__ __forceinline__ void plane_step(State<Real, R, DEPTH, Z0, BY>& st, const Tile& t,
                                           const Real* __restrict__ w, Real* faces, Real* xchg,
                                           const int lx, const int ly, const int ph, const int i) {
  using FL = FaceLayout<R, BY>;
  constexpr int TY = FL::TY;
  using XL = XchgLayout<R>;
  constexpr int S = sizeof(Real);
  const int lane_id_t = ly * LX + lx;

  // Faces of plane i+1 (loaded one iteration ago) go into the queue now; they
  // are read no earlier than the next iteration, after at least one barrier.
  if (!GENERAL || i + 1 < t.n_iter) {
    const int zq = t.zs + i + 1;
    Real(&fv)[3] = st.F[(ph + 1) % Z0];
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (k < t.n_f) faces[(zq & (kRing - 1)) * FL::kPerPlane + t.f_idx[k]] = fv[k];
  }
  // This iteration's plane leaves its ring slot, which then receives plane
  // i + 2 (two planes in flight per workgroup).
  Real x[BY][BX];
#pragma unroll
  for (int j = 0; j < BY; ++j)
#pragma unroll
    for (int q = 0; q < BX; ++q) x[j][q] = st.L0[ph % Z0][j][q];
  {
    const int ip = i + Z0;
    if (!GENERAL || ip < t.n_iter) {
      const uint32_t pb = (uint32_t)ip * t.plane_bytes;
      Real(&dst)[BY][BX] = st.L0[ph % Z0];
#pragma unroll
      for (int j = 0; j < BY; ++j)
        load_vec<Real, BX>(t.rs, t.blk_off + pb + (uint32_t)j * t.row_bytes, 0, dst[j]);
      Real(&fv)[3] = st.F[ph % Z0];
#pragma unroll
      for (int k = 0; k < 3; ++k)
        if (k < t.n_f) fv[k] = load_one<Real>(t.rs, t.f_off[k] + pb, 0);
    }
  }
  const int z = t.zs + i;
  const int Qz = t.Qz;

#pragma unroll
  for (int s = 1; s <= DEPTH; ++s) {
    if (s > t.d) break;
    const int u = z - (s - 1) * R;  // plane of level s-1 arriving now
    const bool ok = !GENERAL || ((u >= t.lo[s - 1]) && (u < Qz));
    const Real* fp = faces + ((u < 0 ? 0 : u) & (kRing - 1)) * FL::kPerPlane;

    // x extension: DPP inside the lane row; edge lanes take the face values
    Real ext[BY + 2 * R][BX + 2 * R];
#pragma unroll
    for (int j = 0; j < BY; ++j) {
#pragma unroll
      for (int q = 0; q < BX; ++q) ext[j + R][q + R] = x[j][q];
      const int yrow = ly * BY + j;
#pragma unroll
      for (int c = 0; c < R; ++c) {
        const Real oldl = fp[FL::kLeft + c * TY + yrow];
        const Real oldr = fp[FL::kRight + c * TY + yrow];
        ext[j + R][c] = dpp_keep<kDppRowShr1>(oldl, x[j][BX - R + c]);
        ext[j + R][BX + R + c] = dpp_keep<kDppRowShl1>(oldr, x[j][c]);
      }
    }
    // y extension through LDS: publish own top/bottom r extended rows. With two
    // buffers they alternate with the running level count (even per unrolled
    // block), so one barrier per level separates every write from the last
    // read of the same buffer.
    // a star tap off the plane row has dx = 0, so only the lane's own columns
    // of the rows above and below are needed; other patterns also read the
    // corners (the x-extended columns)
    constexpr int kQa = SHAPE == kStar ? R : 0;
    constexpr int kQb = SHAPE == kStar ? R + BX : XL::kRowW;
    Real* xb = xchg + (XL::kBufs == 2 ? ((ph * t.d + s) & 1) * XL::kPerBuf : 0);
    {
#pragma unroll
      for (int c = 0; c < R; ++c)
#pragma unroll
        for (int q = kQa; q < kQb; ++q) {
          xb[(c * XL::kRowW + q) * kThreads + lane_id_t] = ext[R + c][q];            // top rows
          xb[((R + c) * XL::kRowW + q) * kThreads + lane_id_t] = ext[BY + c][q];     // bottom rows
        }
    }
    __syncthreads();
    {
      // rows above: bottom rows of the lane above, or the top face; rows below:
      // top rows of the lane below, or the bottom face
      const bool in_a = ly > 0, in_b = ly < LY - 1;
      const Real* above = in_a ? xb + R * XL::kRowW * kThreads + (lane_id_t - LX)
                               : fp + FL::kTop + lx * BX;
      const int a_c = in_a ? XL::kRowW * kThreads : TX + 2 * R;
      const int a_q = in_a ? kThreads : 1;
      const Real* below = in_b ? xb + (lane_id_t + LX) : fp + FL::kBottom + lx * BX;
      const int b_c = in_b ? XL::kRowW * kThreads : TX + 2 * R;
      const int b_q = in_b ? kThreads : 1;
#pragma unroll
      for (int c = 0; c < R; ++c)
#pragma unroll
        for (int q = kQa; q < kQb; ++q) {
          ext[c][q] = above[c * a_c + q * a_q];
          ext[R + BY + c][q] = below[c * b_c + q * b_q];
        }
    }
    if (XL::kBufs == 1) __syncthreads();

    // 1) output completed by this arrival (dz = +r)
    Real out[BY][BX];
    {
      const int o = u - R;
      const int sl = ph % (2 * R);
      const bool halo = GENERAL && ((o < R) || (o >= Qz - R));
      if (ok && !halo) add_plane<Real, R, SHAPE, BY>(st.A[s - 1][sl], ext, w, R);
#pragma unroll
      for (int j = 0; j < BY; ++j)
#pragma unroll
        for (int q = 0; q < BX; ++q) out[j][q] = st.A[s - 1][sl][j][q];
    }
    // 2) open outputs and the newly started one
    if (ok) {
#pragma unroll
      for (int dz = R - 1; dz >= -R; --dz) {
        const int o = u - dz;
        const int sl = pmod(ph - dz - R, 2 * R);
        const bool halo = GENERAL && ((o < R) || (o >= Qz - R));
        if (halo) {
          if (dz == 0) {
#pragma unroll
            for (int j = 0; j < BY; ++j)
#pragma unroll
              for (int q = 0; q < BX; ++q) st.A[s - 1][sl][j][q] = x[j][q];
          }
        } else {
          if (dz == -R) {
#pragma unroll
            for (int j = 0; j < BY; ++j)
#pragma unroll
              for (int q = 0; q < BX; ++q) st.A[s - 1][sl][j][q] = Real(0);
          }
          add_plane<Real, R, SHAPE, BY>(st.A[s - 1][sl], ext, w, dz);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < BY; ++j)
#pragma unroll
      for (int q = 0; q < BX; ++q) x[j][q] = out[j][q];
    if (s == t.d) {
      // the last level completed plane z - d*r
      const int o = z - s * R;
      if (!GENERAL || (o >= t.Z0 && o < t.Z1)) {
        const uint32_t pb = (uint32_t)(o - t.Z0) * t.plane_bytes;
#pragma unroll
        for (int j = 0; j < BY; ++j)
          store_vec<Real, BX>(t.rd, t.st_off + pb + (uint32_t)j * t.row_bytes, 0, x[j]);
      }
    }
  }
}

// Geometry of tile (tx, ty) of an sx x sy tiling with hx / hy redundant lanes.
struct Tb3dGeom {
  int X0, lxa, lxb, Y0, lya, lyb;
};
template <int R, int BY>
__device__ __forceinline__ Tb3dGeom tb3d_geom(int tx, int ty, int sx, int sy, int P, int Qy, int HX,
                                              int HY) {
  constexpr int TY = LY * BY;
  Tb3dGeom g;
  // a single tile exactly as wide (tall) as the interior has halo on both sides
  if (sx == 1) { g.X0 = R; g.lxa = 0; g.lxb = LX; }
  else if (tx == 0) { g.X0 = R; g.lxa = 0; g.lxb = LX - HX; }
  else if (tx == sx - 1) { g.X0 = P - R - TX; g.lxa = HX; g.lxb = LX; }
  else { g.X0 = R + (LX - HX) * BX + (tx - 1) * (LX - 2 * HX) * BX - HX * BX; g.lxa = HX; g.lxb = LX - HX; }
  if (sy == 1) { g.Y0 = R; g.lya = 0; g.lyb = LY; }
  else if (ty == 0) { g.Y0 = R; g.lya = 0; g.lyb = LY - HY; }
  else if (ty == sy - 1) { g.Y0 = Qy - R - TY; g.lya = HY; g.lyb = LY; }
  else { g.Y0 = R + (LY - HY) * BY + (ty - 1) * (LY - 2 * HY) * BY - HY * BY; g.lya = HY; g.lyb = LY - HY; }
  return g;
}

// One workgroup tile of one pass: d (<= DEPTH) levels from src to dst over the
// planes [Zs0, Zs1) of the xy tile g. Every thread of the workgroup calls it.
// Z0: planes in flight (plane_ring by default; the fused batch kernel, whose
// one register allocation serves every variant, passes 2).
template <typename Real, int R, int SHAPE, int DEPTH,
          int Z0 = plane_ring(sizeof(Real) == 8, R, SHAPE, DEPTH), int BY = cells_y(sizeof(Real) == 8, R, SHAPE)>
__device__ __forceinline__ void tb3d_tile(const Real* __restrict__ w, const void* src, void* dst,
                                          const int P, const int Qy, const int Qz,
                                          const Tb3dGeom g, const int Zs0, const int Zs1,
                                          const int d, Real* faces, Real* xchg) {
  using FL = FaceLayout<R, BY>;
  constexpr int TY = FL::TY;
  constexpr int UNROLL = lcm_3d(2 * R, Z0);
  constexpr int S = sizeof(Real);
  const int tid = threadIdx.x;
  const int lx = tid % LX;
  const int ly = tid / LX;
  const int X0 = g.X0, Y0 = g.Y0;

  Tile t;
  t.d = d;
  t.Qz = Qz;
  t.Z0 = Zs0;
  t.Z1 = Zs1;
  t.zs = Zs0 - d * R > 0 ? Zs0 - d * R : 0;
  const int ze = Zs1 - 1 + d * R;
  t.n_iter = ze - t.zs + 1;
  t.row_bytes = (uint32_t)(P * S);
  t.plane_bytes = (uint32_t)((int64_t)P * Qy * S);
  int64_t range = (int64_t)(Qz - t.zs) * P * Qy * S;
  if (range > 0xffffffffll) range = 0xffffffffll;
  t.rs = make_rsrc((const char*)src + (int64_t)t.zs * P * Qy * S, (uint32_t)range);
  t.rd = make_rsrc((char*)dst + (int64_t)Zs0 * P * Qy * S,
                   (uint32_t)((int64_t)(Zs1 - Zs0) * P * Qy * S));
  t.blk_off = (uint32_t)(((Y0 + ly * BY) * P + X0 + lx * BX) * S);
  const bool valid = lx >= g.lxa && lx < g.lxb && ly >= g.lya && ly < g.lyb;
  t.st_off = valid ? t.blk_off : 0x80000000u;
  t.lo[0] = t.zs;
#pragma unroll
  for (int s = 1; s <= DEPTH; ++s) {
    const int b = Zs0 - (d - s) * R;
    t.lo[s] = b > 0 ? b : 0;
  }
  // face cells handled by this thread: thread k takes face entries k, k+256, ...
  t.n_f = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int e = tid + k * kThreads;
    t.f_off[k] = 0;
    t.f_idx[k] = 0;
    if (e < FL::kPerPlane) {
      int fx, fy;
      if (e < FL::kRight) { const int c = e / TY, j = e % TY; fx = X0 - R + c; fy = Y0 + j; }
      else if (e < FL::kTop) { const int f = e - FL::kRight; const int c = f / TY, j = f % TY; fx = X0 + TX + c; fy = Y0 + j; }
      else if (e < FL::kBottom) { const int f = e - FL::kTop; const int c = f / (TX + 2 * R), q = f % (TX + 2 * R); fy = Y0 - R + c; fx = X0 - R + q; }
      else { const int f = e - FL::kBottom; const int c = f / (TX + 2 * R), q = f % (TX + 2 * R); fy = Y0 + TY + c; fx = X0 - R + q; }
      // cells outside the padded plane are never needed by a valid cell: clamp
      fx = fx < 0 ? 0 : (fx >= P ? P - 1 : fx);
      fy = fy < 0 ? 0 : (fy >= Qy ? Qy - 1 : fy);
      t.f_off[k] = (uint32_t)((fy * P + fx) * S);
      t.f_idx[k] = e;
      t.n_f = k + 1;
    }
  }

  State<Real, R, DEPTH, Z0, BY> st;
#pragma unroll
  for (int zz = 0; zz < Z0; ++zz) {
#pragma unroll
    for (int j = 0; j < BY; ++j)
#pragma unroll
      for (int q = 0; q < BX; ++q) st.L0[zz][j][q] = Real(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) st.F[zz][k] = Real(0);
  }
#pragma unroll
  for (int s = 0; s < DEPTH; ++s)
#pragma unroll
    for (int sl = 0; sl < 2 * R; ++sl)
#pragma unroll
      for (int j = 0; j < BY; ++j)
#pragma unroll
        for (int q = 0; q < BX; ++q) st.A[s][sl][j][q] = Real(0);

  // prologue: the first Z0 planes (blocks and faces), face queue slot of plane 0
  __syncthreads();  // the previous tile is done with the LDS queues
#pragma unroll
  for (int p = 0; p < Z0; ++p) {
    if (p < t.n_iter) {
      const uint32_t pb = (uint32_t)p * t.plane_bytes;
#pragma unroll
      for (int j = 0; j < BY; ++j)
        load_vec<Real, BX>(t.rs, t.blk_off + pb + (uint32_t)j * t.row_bytes, 0, st.L0[p][j]);
#pragma unroll
      for (int k = 0; k < 3; ++k)
        if (k < t.n_f) st.F[p][k] = load_one<Real>(t.rs, t.f_off[k] + pb, 0);
    }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k)
    if (k < t.n_f) faces[(t.zs & (kRing - 1)) * FL::kPerPlane + t.f_idx[k]] = st.F[0][k];
  __syncthreads();

  // steady planes: every level valid, no halo plane touched, output stored
  const int lo_dm1 = Zs0 - R > 0 ? Zs0 - R : 0;  // lowest valid plane of level d-1
  int z_a = lo_dm1 + (d - 1) * R;
  if (z_a < (d + 1) * R) z_a = (d + 1) * R;
  if (z_a < Zs0 + d * R) z_a = Zs0 + d * R;
  int z_b = Qz - 2 * R;
  if (z_b > ze + 1) z_b = ze + 1;
  int i_a = z_a - t.zs;
  i_a = (i_a + UNROLL - 1) / UNROLL * UNROLL;
  int i_b = (z_b - t.zs) / UNROLL * UNROLL;
  if (i_a > t.n_iter) i_a = (t.n_iter / UNROLL) * UNROLL;
  if (i_b < i_a) i_b = i_a;

  int base = 0;
  for (; base < i_a; base += UNROLL) {
#pragma unroll
    for (int ph = 0; ph < UNROLL; ++ph)
      if (base + ph < t.n_iter)
        plane_step<Real, R, SHAPE, DEPTH, true, Z0, BY>(st, t, w, faces, xchg, lx, ly, ph, base + ph);
  }
  for (; base < i_b; base += UNROLL) {
#pragma unroll
    for (int ph = 0; ph < UNROLL; ++ph)
      plane_step<Real, R, SHAPE, DEPTH, false, Z0, BY>(st, t, w, faces, xchg, lx, ly, ph, base + ph);
  }
  for (; base < t.n_iter; base += UNROLL) {
#pragma unroll
    for (int ph = 0; ph < UNROLL; ++ph)
      if (base + ph < t.n_iter)
        plane_step<Real, R, SHAPE, DEPTH, true, Z0, BY>(st, t, w, faces, xchg, lx, ly, ph, base + ph);
  }
}

template <typename Real, int R, int SHAPE, int DEPTH>
__global__ __launch_bounds__(kThreads) void tb3d_kernel(const Tb3dParams<Real> a) {
  constexpr int BY = cells_y(sizeof(Real) == 8, R, SHAPE);
  using FL = FaceLayout<R, BY>;
  extern __shared__ char lds_raw[];
  Real* faces = (Real*)lds_raw;
  Real* xchg = faces + kRing * FL::kPerPlane;
  const int P = (int)a.P, Qy = (int)a.Qy, Qz = (int)a.Qz;
  for (int tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
    const int seg = tile / (a.sx * a.sy);
    const int rem = tile - seg * a.sx * a.sy;
    const int ty = rem / a.sx;
    const int tx = rem - ty * a.sx;
    const Tb3dGeom g = tb3d_geom<R, BY>(tx, ty, a.sx, a.sy, P, Qy, a.hx, a.hy);
    const int Zs0 = seg * a.seg_len;
    const int Zs1 = (Zs0 + a.seg_len < Qz) ? Zs0 + a.seg_len : Qz;
    tb3d_tile<Real, R, SHAPE, DEPTH>(a.w, a.src, a.dst, P, Qy, Qz, g, Zs0, Zs1, DEPTH, faces, xchg);
  }
}

// Deepest compiled variant per (dtype, radius, shape) that compiles without
// scratch spills: the partial planes of every level live in registers
// (2r planes x BX x BY cells per lane per level).
constexpr int max_depth_c(int dtype, int r, int shape) {
  if (dtype == kF64) {
    if (shape == kStar) return r == 1 ? 4 : 2;
    if (shape == kBox) return r == 1 ? 2 : 1;
    return r == 1 ? 2 : 1;
  }
  if (shape == kStar) return r == 1 ? 4 : r == 2 ? 2 : 0;
  if (shape == kBox) return r == 1 ? 3 : 0;
  return r == 1 ? 2 : 0;
}
template <typename Real>
constexpr int dtype_code() { return sizeof(Real) == 8 ? kF64 : kF32; }

template <typename Real, int R, int SHAPE, int D>
hipError_t launch_depth(int depth, const Tb3dParams<Real>* p, int grid, hipStream_t s) {
  if constexpr (D == 0) {
    return hipErrorInvalidValue;
  } else {
    if (depth == D) {
      const void* fn = (const void*)&tb3d_kernel<Real, R, SHAPE, D>;
      constexpr size_t lds = Lds<Real, R, cells_y(sizeof(Real) == 8, R, SHAPE)>::kBytes;
      hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      void* args[] = {(void*)p};
      return hipLaunchKernel(fn, dim3(grid), dim3(kThreads), args, lds, s);
    }
    return launch_depth<Real, R, SHAPE, D - 1>(depth, p, grid, s);
  }
}

}  // namespace tb3d

template <typename Real, int R>
hipError_t tb3d_launch_r(int shape, int depth, const Tb3dParams<Real>* p, int grid, hipStream_t s) {
  using namespace tb3d;
  switch (shape) {
    case kStar:
      if constexpr (max_depth_c(dtype_code<Real>(), R, kStar) > 0)
        return launch_depth<Real, R, kStar, max_depth_c(dtype_code<Real>(), R, kStar)>(depth, p, grid, s);
      return hipErrorInvalidValue;
    case kBox:
      if constexpr (max_depth_c(dtype_code<Real>(), R, kBox) > 0)
        return launch_depth<Real, R, kBox, max_depth_c(dtype_code<Real>(), R, kBox)>(depth, p, grid, s);
      return hipErrorInvalidValue;
    case kGeneral:
      if constexpr (max_depth_c(dtype_code<Real>(), R, kGeneral) > 0)
        return launch_depth<Real, R, kGeneral, max_depth_c(dtype_code<Real>(), R, kGeneral)>(depth, p, grid, s);
      return hipErrorInvalidValue;
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace stencil_impl
