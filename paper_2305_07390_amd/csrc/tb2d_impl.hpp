// tb2d_impl.hpp -- temporally blocked 2D stencil pass for gfx950 (kernel templates).
// Each tb2d_<dtype>_r<r>.hip translation unit instantiates one (dtype, radius)
// so the variants compile in parallel.
//
// One pass advances a padded 2D grid by DEPTH Jacobi steps (paper Section 2.1)
// with a single read and a single write of every cell in HBM, which is the
// point of temporal blocking (paper Section 2.1.2 and Section 3).
//
// Decomposition (overlapped tiling, paper Sections 2.1.2-2.1.3 and 4.1 "SM
// tiling", taken here to the granularity of one wavefront):
//   * The grid is cut into vertical strips of W = 64*V columns; lane l of the
//     wave owns the V consecutive columns X0 + l*V .. X0 + l*V + V - 1.
//   * A strip is cut into row segments [Y0, Y1). The wave streams the segment
//     top to bottom (N.5-D streaming along y), reading rows
//     Y0 - DEPTH*r .. Y1 - 1 + DEPTH*r once from HBM.
//   * The DEPTH time levels form a skewed wavefront: when input row y arrives,
//     level s completes output row y - s*r. Each level keeps 2r partial-sum
//     rows in registers; a newly arrived row is pushed into the partial sums of
//     the 2r+1 output rows it touches (the paper's multi-queue, one queue per
//     time level, Section 4.2, held in VGPRs with a compile-time rotation in
//     place of the computed-address ring, since register arrays cannot be
//     indexed at run time).
//   * x-neighbours come from the adjacent lanes through DPP wave shifts; y
//     neighbours are implicit in the streaming order. No LDS and no barrier:
//     the waves of a workgroup are independent tiles.
//   * Errors from the missing neighbours at the strip edges move inward by r
//     columns per level, so an interior strip keeps HL >= ceil(DEPTH*r/V) lanes
//     of redundant work on each side (valid fraction of paper Section 5.2.1).
//     HL comes from the plan (the deepest pass), so that every pass of a plan
//     uses the same strip layout and no interior strip reaches the halo.
//     A strip that touches the left or right edge of the grid needs no
//     redundancy on that side: the Dirichlet halo never changes.
//
// Summation order: every output cell accumulates its terms in dense-box order
// (rows dy = -r..r, within a row dx = -r..r), from +0.0, one fused
// multiply-add per term. Rows of an output arrive in increasing dy, so the
// push order reproduces exactly that order and results are bit-identical to
// an unblocked sweep that uses the same order.
//
// Dirichlet halo (width r, held at its initial values): halo rows are detected
// per wave (uniform branch) and take the value of their own row at the
// previous level; halo columns exist only in the first and last strip, at
// fixed register positions, and are patched by a per-lane select.
//
// Memory safety: loads and stores go through buffer descriptors limited to the
// rows of the tile; out-of-range loads read zero and out-of-range stores are
// dropped by the hardware.
#pragma once
#include "device_common.hpp"
#include "launch.hpp"

// Ablation switches (paper Section 7, breakdown study): each names one
// optimisation of this kernel. The library is built with every one on (the
// defaults); paper_2305_07390_amd/ablation.py builds variants with some off to
// measure what each is worth.
//   STENCIL_ABL_PREFETCH       level-0 rows are loaded ahead of their use into
//                              a register ring (0: each row is loaded when used)
//   STENCIL_ABL_SCHED_BARRIER  each row's prefetch stays at the head of its row
//   STENCIL_ABL_SPLIT_BODY     interior strips run a tile body without halo reads
//   STENCIL_ABL_XCD_ORDER      each XCD runs a run of consecutive tile groups
#ifndef STENCIL_ABL_PREFETCH
#define STENCIL_ABL_PREFETCH 1
#endif
#ifndef STENCIL_ABL_SCHED_BARRIER
#define STENCIL_ABL_SCHED_BARRIER 1
#endif
#ifndef STENCIL_ABL_SPLIT_BODY
#define STENCIL_ABL_SPLIT_BODY 1
#endif
#ifndef STENCIL_ABL_XCD_ORDER
#define STENCIL_ABL_XCD_ORDER 1
#endif

namespace stencil_impl {
using namespace stencil_dev;

namespace {

constexpr int cdiv(int a, int b) { return (a + b - 1) / b; }
constexpr int gcd_c(int a, int b) { return b == 0 ? a : gcd_c(b, a % b); }
constexpr int lcm_c(int a, int b) { return a / gcd_c(a, b) * b; }
constexpr int pmod(int a, int m) { return ((a % m) + m) % m; }

enum Edge { kInterior = 0, kLeftEdge = 1, kRightEdge = 2, kBothEdges = 3 };

// Tile `tile` of a pass -> its strip's place in x and its rows [Y0, Y1).
// Without edge tiles, tile = seg * ns + strip. With edge_tiles > 0 the two
// edge strips come first, two tiles (left, right) per segment of seg_len_e
// rows, then the interior strips by segments of seg_len rows.
struct Tile2D {
  int edge, X0, la, lb, Y0, Y1;
};

__device__ __forceinline__ Tile2D locate_2d(int tile, int ns, int seg_len, int seg_len_e,
                                            int edge_tiles, int P, int Q, int R, int V, int HL) {
  int strip, Y0, len;
  if (tile < edge_tiles) {
    const int seg = tile >> 1;
    strip = (tile & 1) ? ns - 1 : 0;
    Y0 = seg * seg_len_e;
    len = seg_len_e;
  } else if (edge_tiles > 0) {
    const int t = tile - edge_tiles, ni = ns - 2;
    const int seg = t / ni;
    strip = 1 + (t - seg * ni);
    Y0 = seg * seg_len;
    len = seg_len;
  } else {
    const int seg = tile / ns;
    strip = tile - seg * ns;
    Y0 = seg * seg_len;
    len = seg_len;
  }
  Tile2D g;
  g.Y0 = Y0;
  g.Y1 = (Y0 + len < Q) ? Y0 + len : Q;
  if (ns == 1) {
    // one strip exactly as wide as the interior: both sides are halo
    g.edge = kBothEdges; g.X0 = R; g.la = 0; g.lb = kWave;
  } else if (strip == 0) {
    g.edge = kLeftEdge; g.X0 = R; g.la = 0; g.lb = kWave - HL;
  } else if (strip == ns - 1) {
    g.edge = kRightEdge; g.X0 = P - R - kWave * V; g.la = HL; g.lb = kWave;
  } else {
    g.edge = kInterior;
    g.X0 = R + (kWave - HL) * V + (strip - 1) * (kWave - 2 * HL) * V - HL * V;
    g.la = HL; g.lb = kWave - HL;
  }
  return g;
}

// Register rings of a tile: `slots` partial-sum rows per level and `z0`
// level-0 rows in flight (prefetch distance + 1), both rotated at compile time
// over an unroll of lcm(slots, z0) rows.
//
// With 2r slots the output a row completes and the output it opens share a
// slot: both are live at once, so unless the unroll lets the allocator rotate
// 2r + 1 registers, every level copies the completed row. Radius-2 boxes
// (the 25-point box: the most FMAs per row) take 2r + 1 slots and five rows
// in flight, an unroll of five that rotates both rings (measured on 8192^2
// FP64: +3 % at depths 5 and 6). WIDE = false keeps 2r slots (the fused batch
// kernels, whose one register allocation has no room for the extra row).
template <int R, int SHAPE, bool WIDE>
struct LevelRing {
  static constexpr bool wide = WIDE && R == 2 && SHAPE == kBox;
  static constexpr int slots = wide ? 2 * R + 1 : 2 * R;
  static constexpr int z0 = !STENCIL_ABL_PREFETCH ? 1 : wide ? 5 : (2 * R >= 4) ? 2 * R : 4;
};

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <typename Real, int R, int SHAPE, int V>
__device__ __forceinline__ void add_row(Real (&acc)[V], const Real (&x)[V],
                                        const Real (&xe)[V + 2 * R], const Real* __restrict__ w,
                                        int dy) {
  constexpr int SIDE = 2 * R + 1;
  if (SHAPE == kStar && dy != 0) {
    const Real c = w[(dy + R) * SIDE + R];
#pragma unroll
    for (int v = 0; v < V; ++v) acc[v] = fma_t(c, x[v], acc[v]);
  } else {
#pragma unroll
    for (int dx = -R; dx <= R; ++dx) {
      const Real c = w[(dy + R) * SIDE + dx + R];
      if (SHAPE == kGeneral && c == Real(0)) continue;
#pragma unroll
      for (int v = 0; v < V; ++v) acc[v] = fma_t(c, xe[v + R + dx], acc[v]);
    }
  }
}

template <int CTRL, typename Real>
__device__ __forceinline__ Real dpp_or(Real old, Real v);
template <int CTRL>
__device__ __forceinline__ double dpp_or(double old, double v) {
  // lanes whose source lane does not exist keep `old`
  unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  unsigned long long o = __builtin_bit_cast(unsigned long long, old);
  int lo = __builtin_amdgcn_update_dpp((int)(unsigned)(o & 0xffffffffull),
                                       (int)(unsigned)(b & 0xffffffffull), CTRL, 0xf, 0xf, false);
  int hi = __builtin_amdgcn_update_dpp((int)(unsigned)(o >> 32), (int)(unsigned)(b >> 32), CTRL,
                                       0xf, 0xf, false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_or(float old, float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old),
                                                               __builtin_bit_cast(int, v), CTRL,
                                                               0xf, 0xf, false));
}

// Row x of V values per lane -> extended row with r neighbours on each side.
// Lane 0 takes its left neighbours from `el` and lane 63 its right neighbours
// from `er` (the Dirichlet halo of the row when the strip touches the grid's
// edge; ignored otherwise); every other lane reads the adjacent lane.
template <typename Real, int R, int V>
__device__ __forceinline__ void extend_row(const Real (&x)[V], const Real (&el)[R],
                                           const Real (&er)[R], Real (&xe)[V + 2 * R]) {
#pragma unroll
  for (int v = 0; v < V; ++v) xe[R + v] = x[v];
#pragma unroll
  for (int j = 0; j < R; ++j) {
    xe[j] = dpp_or<kDppWaveShr1>(el[j], x[V - R + j]);
    xe[R + V + j] = dpp_or<kDppWaveShl1>(er[j], x[j]);
  }
}

// Interior strips: the first and last HL lanes are redundant, so the lanes
// without a source lane may take any value (bound_ctrl writes zero) and no
// halo values are read.
template <int CTRL>
__device__ __forceinline__ double dpp_open(double v) {
  unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)(b & 0xffffffffull), CTRL, 0xf, 0xf, true);
  int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, true);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_open(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xf,
                                                            0xf, true));
}

template <typename Real, int R, int V>
__device__ __forceinline__ void extend_row_open(const Real (&x)[V], Real (&xe)[V + 2 * R]) {
#pragma unroll
  for (int v = 0; v < V; ++v) xe[R + v] = x[v];
#pragma unroll
  for (int j = 0; j < R; ++j) {
    xe[j] = dpp_open<kDppWaveShr1>(x[V - R + j]);
    xe[R + V + j] = dpp_open<kDppWaveShl1>(x[j]);
  }
}

// Mutable per-tile streaming state (kept in registers after inlining).
template <typename Real, int DEPTH, int V, int NS, int Z0>
struct Tb2dState {
  Real L0[Z0][V];       // level-0 rows in flight (prefetch ring)
  Real A[DEPTH][NS][V]; // per level: partial sums of the open output rows
};

// Per-tile constants.
struct Tb2dTile {
  __amdgpu_buffer_rsrc_t rs, rd;
  uint32_t col_off, st_off, row_bytes;
  int ys, Y0, Y1, Q, n_iter;
  int d;  // levels of this pass (<= the compiled depth)
  int lo[17];
};

// One streamed row (iteration i, phase ph of the unrolled loop).
// GENERAL: warm-up/drain rows -- checks which levels hold valid rows and
// handles the Dirichlet halo rows. Steady rows skip every check.
template <typename Real, int R, int SHAPE, int DEPTH, int V, int NS, int Z0, bool EDGE, bool GENERAL>
__device__ __forceinline__ void tb2d_row(Tb2dState<Real, DEPTH, V, NS, Z0>& st, const Tb2dTile& t,
                                         const Real* __restrict__ w, const Real* hq, const int ph,
                                         const int i) {
  {
    const int ip = i + Z0 - 1;
    if (!GENERAL || ip < t.n_iter)
      load_vec<Real, V>(t.rs, t.col_off + (uint32_t)ip * t.row_bytes, 0, st.L0[(ph + Z0 - 1) % Z0]);
    // keep the prefetch at the head of its row: the scheduler otherwise sinks
    // the loads of an unrolled iteration towards its end, and the next
    // iteration then waits on all of them (vmcnt also counts the stores)
    if (!GENERAL && STENCIL_ABL_SCHED_BARRIER) __builtin_amdgcn_sched_barrier(0);
  }
  Real x[V];
#pragma unroll
  for (int v = 0; v < V; ++v) x[v] = st.L0[ph % Z0][v];
  const int y = t.ys + i;
  const int Q = t.Q;

#pragma unroll
  for (int s = 1; s <= DEPTH; ++s) {
    if (s > t.d) break;
    const int u = y - (s - 1) * R;  // row of level s-1 arriving now
    const bool ok = !GENERAL || ((u >= t.lo[s - 1]) && (u < Q));
    Real xe[V + 2 * R];
    if constexpr (EDGE) {
      // halo values of row u (two copies, so each DPP gets its own register)
      Real el[R], er[R];
      int hrow = u - t.ys;
      if (GENERAL) hrow = hrow < 0 ? 0 : hrow;
#pragma unroll
      for (int j = 0; j < R; ++j) {
        el[j] = hq[hrow * 2 * R + j];
        er[j] = hq[hrow * 2 * R + R + j];
      }
      extend_row<Real, R, V>(x, el, er, xe);
    } else {
      extend_row_open<Real, R, V>(x, xe);
    }

    // 1) the output completed by this arrival (dy = +r); it was started 2r
    //    arrivals ago in the same slot (an output keeps the slot it opened in:
    //    phase minus dy + r, modulo the slot count)
    Real out[V];
    {
      const int o = u - R;
      const int sl = pmod(ph - 2 * R, NS);
      const bool halo_row = GENERAL && ((o < R) || (o >= Q - R));
      if (ok && !halo_row) add_row<Real, R, SHAPE, V>(st.A[s - 1][sl], x, xe, w, R);
#pragma unroll
      for (int v = 0; v < V; ++v) out[v] = st.A[s - 1][sl][v];
    }
    // 2) open outputs (dy = r-1 .. -r+1) and the newly started one (dy = -r)
    if (ok) {
#pragma unroll
      for (int dy = R - 1; dy >= -R; --dy) {
        const int o = u - dy;
        const int sl = pmod(ph - dy - R, NS);
        const bool halo_row = GENERAL && ((o < R) || (o >= Q - R));
        if (halo_row) {
          if (dy == 0) {
#pragma unroll
            for (int v = 0; v < V; ++v) st.A[s - 1][sl][v] = x[v];
          }
        } else {
          if (dy == -R) {
#pragma unroll
            for (int v = 0; v < V; ++v) st.A[s - 1][sl][v] = Real(0);
          }
          add_row<Real, R, SHAPE, V>(st.A[s - 1][sl], x, xe, w, dy);
        }
      }
    }
#pragma unroll
    for (int v = 0; v < V; ++v) x[v] = out[v];
    if (s == t.d) {
      // the last level completed row y - d*r
      const int o = y - s * R;
      if (!GENERAL || (o >= t.Y0 && o < t.Y1))
        store_vec<Real, V>(t.rd, t.st_off + (uint32_t)(o - t.Y0) * t.row_bytes, 0, x);
    }
  }
}

// One wave tile of one pass: d (<= DEPTH) levels from src to dst. EDGE: the
// strip touches the left or right side of the grid (edge != kInterior).
template <typename Real, int R, int SHAPE, int DEPTH, int V, bool EDGE, bool WIDE = true>
__device__ __forceinline__ void tb2d_tile_impl(const Real* __restrict__ w, const void* src, void* dst,
                                          const void* orig, const int P, const int Q, Real* hq,
                                          const int lane, const int edge, const int X0,
                                          const int la, const int lb, const int Y0, const int Y1,
                                          const int d) {
  using Ring = LevelRing<R, SHAPE, WIDE>;
  constexpr int NS = Ring::slots;
  constexpr int Z0 = Ring::z0;
  constexpr int UNROLL = lcm_c(NS, Z0);
  constexpr int S = sizeof(Real);

  Tb2dTile t;
  t.d = d;
  t.Q = Q;
  t.Y0 = Y0;
  t.Y1 = Y1;
  t.ys = Y0 - d * R > 0 ? Y0 - d * R : 0;
  const int ye = Y1 - 1 + d * R;
  t.n_iter = ye - t.ys + 1;
  int64_t src_range = (int64_t)(Q - t.ys) * P * S;
  if (src_range > 0xffffffffll) src_range = 0xffffffffll;
  t.rs = make_rsrc((const char*)src + (int64_t)t.ys * P * S, (uint32_t)src_range);
  t.rd = make_rsrc((char*)dst + (int64_t)Y0 * P * S, (uint32_t)((int64_t)(Y1 - Y0) * P * S));
  t.row_bytes = (uint32_t)(P * S);
  t.col_off = (uint32_t)((X0 + lane * V) * S);
  // lanes outside the store range get an offset past the descriptor: the
  // hardware drops their stores
  t.st_off = (lane >= la && lane < lb) ? t.col_off : 0x80000000u;
  t.lo[0] = t.ys;
#pragma unroll
  for (int s = 1; s <= DEPTH; ++s) {
    const int b = Y0 - (d - s) * R;
    t.lo[s] = b > 0 ? b : 0;
  }

  // Edge strips: stage the Dirichlet halo columns of the tile's rows in LDS
  // (left strip: columns 0..r-1, right strip: columns P-r..P-1), two copies
  // per row.
  if (EDGE && edge != kInterior) {
    const int rows = (ye < Q - 1 ? ye : Q - 1) - t.ys + 1;
    const __amdgpu_buffer_rsrc_t rin =
        make_rsrc((const char*)orig + (int64_t)t.ys * P * S, (uint32_t)src_range);
    for (int k = lane; k < rows * R; k += kWave) {
      const int row = k / R, j = k - row * R;
      // left copy feeds lane 0, right copy feeds lane 63
      const Real hl = load_one<Real>(rin, (uint32_t)(row * P + j) * S, 0);
      const Real hr = load_one<Real>(rin, (uint32_t)(row * P + P - R + j) * S, 0);
      hq[row * 2 * R + j] = edge == kRightEdge ? hr : hl;
      hq[row * 2 * R + R + j] = edge == kLeftEdge ? hl : hr;
    }
  }

  Tb2dState<Real, DEPTH, V, NS, Z0> st;
#pragma unroll
  for (int z = 0; z < Z0; ++z)
#pragma unroll
    for (int v = 0; v < V; ++v) st.L0[z][v] = Real(0);
#pragma unroll
  for (int s = 0; s < DEPTH; ++s)
#pragma unroll
    for (int j = 0; j < NS; ++j)
#pragma unroll
      for (int v = 0; v < V; ++v) st.A[s][j][v] = Real(0);

#pragma unroll
  for (int p = 0; p < Z0 - 1; ++p)
    if (p < t.n_iter) load_vec<Real, V>(t.rs, t.col_off + (uint32_t)p * t.row_bytes, 0, st.L0[p]);

  // Steady rows: every level holds valid rows, no halo row is touched and the
  // completed row is stored.
  const int lo_dm1 = Y0 - R > 0 ? Y0 - R : 0;  // lowest valid row of level d-1
  int y_a = lo_dm1 + (d - 1) * R;
  if (y_a < (d + 1) * R) y_a = (d + 1) * R;
  if (y_a < Y0 + d * R) y_a = Y0 + d * R;
  int y_b = Q - 2 * R;
  if (y_b > ye + 1) y_b = ye + 1;
  int i_a = y_a - t.ys;
  i_a = (i_a + UNROLL - 1) / UNROLL * UNROLL;
  int i_b = (y_b - t.ys) / UNROLL * UNROLL;
  if (i_a > t.n_iter) i_a = (t.n_iter / UNROLL) * UNROLL;
  if (i_b < i_a) i_b = i_a;

  int base = 0;
  for (; base < i_a; base += UNROLL) {
#pragma unroll
    for (int ph = 0; ph < UNROLL; ++ph)
      if (base + ph < t.n_iter) tb2d_row<Real, R, SHAPE, DEPTH, V, NS, Z0, EDGE, true>(st, t, w, hq, ph, base + ph);
  }
  for (; base < i_b; base += UNROLL) {
#pragma unroll
    for (int ph = 0; ph < UNROLL; ++ph) tb2d_row<Real, R, SHAPE, DEPTH, V, NS, Z0, EDGE, false>(st, t, w, hq, ph, base + ph);
  }
  for (; base < t.n_iter; base += UNROLL) {
#pragma unroll
    for (int ph = 0; ph < UNROLL; ++ph)
      if (base + ph < t.n_iter) tb2d_row<Real, R, SHAPE, DEPTH, V, NS, Z0, EDGE, true>(st, t, w, hq, ph, base + ph);
  }
}

template <typename Real, int R, int SHAPE, int DEPTH, int V, bool WIDE = true>
__device__ __forceinline__ void tb2d_tile(const Real* __restrict__ w, const void* src, void* dst,
                                          const void* orig, const int P, const int Q, Real* hq,
                                          const int lane, const int edge, const int X0,
                                          const int la, const int lb, const int Y0, const int Y1,
                                          const int d) {
  if (edge == kInterior && STENCIL_ABL_SPLIT_BODY)
    tb2d_tile_impl<Real, R, SHAPE, DEPTH, V, false, WIDE>(w, src, dst, orig, P, Q, hq, lane, edge, X0,
                                                          la, lb, Y0, Y1, d);
  else
    tb2d_tile_impl<Real, R, SHAPE, DEPTH, V, true, WIDE>(w, src, dst, orig, P, Q, hq, lane, edge, X0,
                                                         la, lb, Y0, Y1, d);
}

template <typename Real, int R, int SHAPE, int DEPTH>
__global__ __launch_bounds__(256) void tb2d_kernel(const Tb2dParams<Real> a) {
  constexpr int V = tb2d_cols(sizeof(Real) == 8, R, SHAPE);
  extern __shared__ char lds_raw[];
  const int lane = lane_id();
  const int waves = blockDim.x / kWave;
  const int wid = uniform((int)(threadIdx.x / kWave));
  Real* hq = (Real*)lds_raw + (size_t)wid * a.hq_rows * 2 * R;
  const int stride = gridDim.x * waves;
  const int ns = a.n_strips;
  const int P = (int)a.P;
  const int Q = (int)a.Q;
  // strip layout shared by every pass of the plan: hl * V >= DEPTH * r
  const int HL = a.hl;
  // Workgroups are dispatched round-robin over the 8 XCDs. Give each XCD a
  // run of consecutive tile groups, so that adjacent strips, which re-read each
  // other's margin columns, share an L2 (a bijection for any grid size).
  const int g = (int)gridDim.x, xcd = (int)blockIdx.x % 8, slot = (int)blockIdx.x / 8;
  const int per = g / 8, extra = g % 8;
  const int swz = STENCIL_ABL_XCD_ORDER ? xcd * per + (xcd < extra ? xcd : extra) + slot : (int)blockIdx.x;
  for (int tile = swz * waves + wid; tile < a.ntiles; tile += stride) {
    const Tile2D g = locate_2d(tile, ns, a.seg_len, a.seg_len_e, a.edge_tiles, P, Q, R, V, HL);
    tb2d_tile<Real, R, SHAPE, DEPTH, V>(a.w, a.src, a.dst, a.orig, P, Q, hq, lane, g.edge, g.X0,
                                        g.la, g.lb, g.Y0, g.Y1, DEPTH);
  }
}

// Deepest compiled variant per (dtype, radius, shape): at most the deepest
// that compiles without scratch spills on gfx950 (each level holds 2r partial
// rows of V values per lane), and no deeper than the deepest that still runs
// faster where the levels past the VGPRs live in AGPRs (measured at 8192^2:
// the radius-1 star stops at 12, the radius-3 star at 5). The general pattern
// (runtime zero skipping) is a fallback; for r >= 3 it has no blocked variant.
constexpr int max_depth_c(bool f64, int r, int shape) {
  if (shape == kStar) return r == 1 ? 12 : r == 2 ? 8 : r == 3 ? 5 : 2;
  if (shape == kBox) return r == 1 ? 10 : r == 2 ? (f64 ? 6 : 5) : r == 3 ? 3 : 2;
  return r == 1 ? 3 : r == 2 ? 2 : 0;
}

template <typename Real, int R, int SHAPE, int D>
hipError_t launch_depth(int depth, const Tb2dParams<Real>* p, int grid, int block, size_t lds,
                        hipStream_t s) {
  if constexpr (D == 0) {
    return hipErrorInvalidValue;
  } else {
    if (depth == D) {
      const void* fn = (const void*)&tb2d_kernel<Real, R, SHAPE, D>;
      // the edge strips' halo queues may take more than the default 64 KB
      if (lds > (size_t)64 * 1024) {
        const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
      }
      void* args[] = {(void*)p};
      return hipLaunchKernel(fn, dim3(grid), dim3(block), args, lds, s);
    }
    return launch_depth<Real, R, SHAPE, D - 1>(depth, p, grid, block, lds, s);
  }
}

}  // namespace

template <typename Real, int R>
hipError_t tb2d_launch_r(int shape, int depth, const Tb2dParams<Real>* p, int grid, int block,
                         size_t lds, hipStream_t s) {
  switch (shape) {
    case kStar:
      return launch_depth<Real, R, kStar, max_depth_c(sizeof(Real) == 8, R, kStar)>(depth, p, grid, block, lds, s);
    case kBox:
      return launch_depth<Real, R, kBox, max_depth_c(sizeof(Real) == 8, R, kBox)>(depth, p, grid, block, lds, s);
    case kGeneral:
      return launch_depth<Real, R, kGeneral, max_depth_c(sizeof(Real) == 8, R, kGeneral)>(depth, p, grid, block,
                                                                                        lds, s);
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace stencil_impl
