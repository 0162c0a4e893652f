// Launch parameters shared by the host runtime (capi.cpp) and the HIP kernels.
// Internal to the library: not part of the public C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stencil_impl {

enum ShapeClass : int { kStar = 0, kBox = 1, kGeneral = 2 };
enum DType : int { kF32 = 0, kF64 = 1 };

constexpr int kMaxR = 4;
constexpr int kMaxBox2D = (2 * kMaxR + 1) * (2 * kMaxR + 1);
constexpr int kMaxBox3D = (2 * kMaxR + 1) * (2 * kMaxR + 1) * (2 * kMaxR + 1);
constexpr int kWave = 64;

// Columns per lane of the blocked 2D kernels: two 16-byte words per lane.
constexpr int tb2d_cols(bool f64, int r, int shape) {
  (void)r;
  (void)shape;
  return f64 ? 4 : 8;
}

// One pass of the temporally blocked 2D kernel: DEPTH steps from src to dst.
// Both arrays are padded (P columns x Q rows, x fastest). The grid is cut into
// n_strips x n_segs wave tiles (see tb2d.hip for the geometry).
// `orig` is the operation's original input (its halo is the Dirichlet data).
// The interior columns r .. P-r-1 are cut into n_strips strips (at least two)
// laid out with hl redundant lanes on each open side (hl * V >= depth * r for
// every pass of the plan); rows into n_segs segments of seg_len rows. With
// edge_tiles > 0 the two edge strips have their own segments of seg_len_e rows
// and their tiles come first. Each wave keeps hq_rows x 2r halo values in LDS.
template <typename Real>
struct Tb2dParams {
  const void* src;
  void* dst;
  const void* orig;
  int64_t P, Q;
  int32_t n_strips, n_segs, seg_len, ntiles, hq_rows, hl;
  int32_t seg_len_e, edge_tiles;  // edge-strip segments (edge_tiles = 0: none)
  Real w[kMaxBox2D];  // dense (2r+1)^2 coefficient box, dense-box order
};

// One pass of the temporally blocked 3D kernel (tb3d_impl.hpp): padded extents
// P (x), Qy, Qz; the interior xy plane is cut into sx x sy overlapped 64 x 64
// tiles with hx / hy redundant lanes (4 cells each) per open side, z into
// n_segs segments of seg_len planes; ntiles = sx * sy * n_segs workgroups.
template <typename Real>
struct Tb3dParams {
  const void* src;
  void* dst;
  int64_t P, Qy, Qz;
  int32_t sx, sy, n_segs, seg_len, ntiles, hx, hy;
  Real w[kMaxBox3D > 125 ? 125 : kMaxBox3D];  // dense (2r+1)^3 box, r <= 2
};

// One pass of the device-tiled 3D kernel (tb3d_dev_impl.hpp): the interior xy
// plane is cut into gx x gy non-overlapping 64 x 16 tiles, one workgroup each
// (all resident at once); every workgroup streams all Qz planes through
// `depth` levels and exchanges tile edges through `ring` (tb3d_dev_ring_elems
// cells per tile, each stored as (32-bit word, tag) pairs: 2 x sizeof(Real)
// bytes), zeroed before the first pass; iteration i of the pass tags its
// words flag_base + i + 1. A bounded wait that expires sets *err.
template <typename Real>
struct Tb3dDevParams {
  const void* src;
  void* dst;
  void* ring;
  unsigned int* err;
  int64_t P, Qy, Qz;
  int32_t gx, gy, depth;
  uint32_t flag_base;
  int64_t timeout_ticks;
  Real w[125];  // dense (2r+1)^3 box, r <= 2
};

// ---- batched persistent execution ----------------------------------------
// A batch runs many independent grids in one persistent launch per dtype.
// Work items are a workgroup's share of one (job, pass): a 3D tile, or up to
// four 2D wave tiles. Items are listed as chunks (job, pass) in an order where
// every pass of a job follows its previous pass, and the item counter walks
// them. Tiles of pass p of job j start once all tiles of pass p-1 of job j are
// done (done[j] >= p * tiles), which also covers the reuse of the ping-pong
// buffers.
struct BatchQueue {
  const int32_t* chunk_job;
  const int32_t* chunk_pass;
  const int64_t* chunk_first;  // nchunks + 1 prefix sums of item counts
  int32_t nchunks;
  int64_t nitems;
  unsigned long long* cursor;  // next item
  unsigned int* done;          // per job: tiles finished, all passes
  unsigned int* err;           // set when a bounded wait expires
  int64_t timeout_ticks;       // s_memrealtime ticks (100 MHz)
};

// Variant index of a batched job: 2D variants 0..11, 3D variants 12..23.
constexpr int kBatch3DBase = 12;
constexpr int batch_variant(int ndim, int r, int shape) {
  return (ndim - 2) * kBatch3DBase + (r - 1) * 3 + shape;
}

// One batched grid. 2D: P = padded x extent, Qy = padded y extent, strips x
// segments tiles of one wave. 3D: P, Qy, Qz padded extents, sx x sy x
// segments tiles of one workgroup.
template <typename Real>
struct BatchJob {
  const void* in;
  void* out;
  void* ws;
  int64_t P, Qy, Qz;
  int32_t variant, tiles, strips, seg_len, hl, sx, sy, hx, hy, npass, depth, depth_last;
  int32_t seg_len_e, edge_tiles;
  Real w[125];
};

template <typename Real>
struct BatchParams {
  const BatchJob<Real>* jobs;
  BatchQueue q;
  int32_t hq_stride;  // LDS halo-queue elements per wave (2D tiles)
};

// Halo-frame copies for many grids in one launch.
struct FrameCopyJob {
  const void* src;
  void* dst;
  int64_t ext[3];
  int32_t r[3];
};

// The fused persistent batch kernel of a dtype (grid workgroups of 256).
// aux: the auxiliary kernel (batch_aux_depth) instead of the fused one
hipError_t batch_launch(int dtype, const void* params, int grid, size_t lds_bytes, hipStream_t stream,
                        bool aux = false);
// Deepest compiled depth of a batched variant (0: none), and the LDS bytes a
// 3D variant needs.
int batch_max_depth(int dtype, int ndim, int r, int shape);
// Single-variant persistent kernel of `variant` (batch_variant id): one plan's
// passes in one launch at the variant's single-grid depth.
hipError_t batch_launch_single(int dtype, int variant, const void* params, int grid, size_t lds_bytes,
                               hipStream_t stream);
bool batch_single_supported(int dtype, int ndim, int r, int shape);
int batch_single_depth(int dtype, int ndim, int r, int shape);
// Deepest variant of the auxiliary batch kernel (0: none), for variants the
// fused kernel leaves out.
int batch_aux_depth(int dtype, int ndim, int r, int shape);
size_t batch_lds_3d(int dtype, int r, int shape);
// Device-wide barrier probe (one workgroup per CU), see stencil_probe_grid_sync.
hipError_t grid_sync_probe_launch(unsigned int* ctr, unsigned int* err, int rounds, int grid,
                                  long long timeout_ticks, hipStream_t stream);
hipError_t frame_copy_batch_launch(int dtype, const FrameCopyJob* jobs_dev, int njobs,
                                   hipStream_t stream);
// OR a launch's own error word into a report word (one small kernel on `stream`).
hipError_t error_fold_launch(const unsigned int* src, unsigned int* dst, hipStream_t stream);

// One step of the plain kernel, any ndim <= 3 (padded extents ext[0..2],
// slowest first; unused leading extents are 1 with zero halo). The non-zero
// taps (linear offset, weight) are passed by value in dense-box order.
constexpr int kMaxNaiveTaps = 128;
template <typename Real>
struct NaiveParams {
  const void* src;
  void* dst;
  int64_t ext[3];
  int32_t lo[3], hi[3];  // interior index range per axis
  int32_t ntaps;
  int64_t off[kMaxNaiveTaps];
  Real w[kMaxNaiveTaps];
};

// Host entry points implemented in the .hip files.
// Returns hipErrorInvalidValue when no kernel variant matches.
hipError_t tb2d_launch(int dtype, int r, int shape, int depth, const void* params, int grid,
                       int block, size_t lds_bytes, hipStream_t stream);
// Largest depth with a compiled variant (0 if none).
int tb2d_max_depth(int dtype, int r, int shape);
// Columns per lane for the given dtype.
int tb2d_cols_per_lane(int dtype, int r, int shape);

hipError_t naive_launch(int dtype, const void* params, int64_t cells, hipStream_t stream);

// Cells per lane along y of the 3D tiles for (dtype, radius, shape): the
// tile is 64 x 16 * that.
int tb3d_cells_y(int dtype, int r, int shape);
hipError_t tb3d_launch(int dtype, int r, int shape, int depth, const void* params, int grid,
                       hipStream_t stream);
int tb3d_max_depth(int dtype, int r, int shape);

// Device-tiled 3D passes: launch the kernel compiled for depth `cdepth` (each
// pass runs the variant of its own depth).
hipError_t tb3d_dev_launch(int dtype, int r, int shape, int cdepth, const void* params, hipStream_t stream);
int tb3d_dev_max_depth(int dtype, int r, int shape);
// Tile extent in y (x is 64), halo-ring elements per tile for a plan of
// depth `cdepth`, and iterations of one pass of depth d over Qz planes.
int tb3d_dev_tile_y();
int64_t tb3d_dev_ring_elems(int r, int cdepth);
int64_t tb3d_dev_iterations(int r, int d, int64_t Qz);
// Zero n 32-bit words (a small kernel, so that it may be captured in graphs).
hipError_t fill_zero_u32_launch(unsigned int* p, int64_t n, hipStream_t stream);

// Copy the halo frame (width r[j] on axis j; ext slowest first, unused leading
// axes have extent 1 and width 0) from src to dst.
hipError_t frame_copy_launch(int dtype, const void* src, void* dst, const int64_t ext[3],
                             const int r[3], hipStream_t stream);

}  // namespace stencil_impl
