// Host runtime behind include/stencil.h: argument validation, pattern
// classification, planning (scheme, temporal depth, tiles), the pass schedule
// and kernel launches. Compiled with hipcc for gfx950.
#include "../../include/stencil.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "launch.hpp"
#include "plan.hpp"

using namespace stencil_impl;

namespace stencil_impl {

thread_local std::string g_last_error;

stencil_status fail(stencil_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

stencil_status hip_fail(hipError_t e, const char* what) {
  return fail(STENCIL_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

DeviceInfo device_info() {
  static std::mutex mu;
  static std::vector<DeviceInfo> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return DeviceInfo{};
  std::lock_guard<std::mutex> lock(mu);
  if ((int)cache.size() <= dev) cache.resize(dev + 1);
  if (!cache[dev].ok) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return DeviceInfo{};
    cache[dev].cus = prop.multiProcessorCount;
    cache[dev].ok = true;
  }
  return cache[dev];
}

}  // namespace stencil_impl

namespace {

constexpr int64_t kLdsBudget = 128 * 1024;

bool classify(int ndim, int r, const double* c, int* pattern, int* points) {
  const int side = 2 * r + 1;
  const int count = ndim == 2 ? side * side : side * side * side;
  bool star_full = true, box_full = true, any = false;
  int k = 0;
  for (int idx = 0; idx < count; ++idx) {
    int rem = idx, nz_axes = 0;
    for (int d = 0; d < ndim; ++d) {
      if (rem % side != r) ++nz_axes;
      rem /= side;
    }
    const bool on_star = nz_axes <= 1;
    const bool nz = c[idx] != 0.0;
    if (!std::isfinite(c[idx])) return false;
    if (nz) { ++k; any = true; }
    if (on_star != nz) star_full = false;
    if (!nz) box_full = false;
  }
  *points = k;
  if (!any) *pattern = STENCIL_GENERAL;
  else if (star_full) *pattern = STENCIL_STAR;
  else if (box_full) *pattern = STENCIL_BOX;
  else *pattern = STENCIL_GENERAL;
  return true;
}

void plan_2d_tiles(stencil_plan_s* p, int depth, int seg_hint, int cus, bool edge_split) {
  const int V = tb2d_cols_per_lane(p->dtype, p->r, p->pattern);
  const int W = kWave * V;
  const int HL = (depth * p->r + V - 1) / V;
  const int64_t nx = p->n[2];
  const int64_t Q = p->ext[1];
  const int64_t side_valid = (int64_t)(kWave - HL) * V;
  const int64_t mid_valid = (int64_t)(kWave - 2 * HL) * V;
  int64_t n_int = 0;
  if (nx > 2 * side_valid) n_int = (nx - 2 * side_valid + mid_valid - 1) / mid_valid;
  // an interior exactly one wave tile wide is one strip with halo on both sides
  p->strips = nx == (int64_t)kWave * V ? 1 : (int)(2 + n_int);
  p->hl = HL;
  (void)W;
  int seg;
  if (seg_hint > 0) {
    seg = seg_hint;
  } else {
    // One tile per SIMD (four waves per CU, one workgroup per CU): the tile
    // count must not exceed the wave slots, or a second round of tiles
    // doubles the pass time.
    const int64_t slots = (int64_t)cus * 4;
    int64_t nseg = std::max<int64_t>(1, slots / p->strips);
    seg = (int)((Q + nseg - 1) / nseg);
    const int min_seg = std::max(16, 4 * depth * p->r);
    if (seg < min_seg) seg = min_seg;
  }
  // keep a tile's byte offsets within 31 bits
  const int64_t row_bytes = p->ext[2] * (int64_t)p->elem;
  const int64_t max_rows = ((int64_t)1 << 31) / row_bytes - 2 * depth * p->r - 16;
  if (seg > max_rows) seg = (int)std::max<int64_t>(1, max_rows);
  // the per-wave LDS halo queue (4 waves x rows x 2r values) stays within
  // 128 KB of the CU's 160 KB (the launch raises the kernel's LDS limit)
  const int64_t lds_rows = kLdsBudget / (4 * 2 * p->r * (int64_t)p->elem) - 2 * depth * p->r - 8;
  if (seg > lds_rows) seg = (int)std::max<int64_t>(1, lds_rows);
  if (seg > Q) seg = (int)Q;
  p->seg_len = seg;
  p->segs = (int)((Q + seg - 1) / seg);
  p->tiles = p->strips * p->segs;
  p->seg_len_e = seg;
  p->edge_tiles = 0;
  if (edge_split && p->strips > 2) {
    // Edge-strip tiles also apply the Dirichlet columns and cost more per
    // row; a pass whose tiles all run at once ends with its slowest tile.
    // Cut the two edge strips into shorter segments that take the wave slots
    // the interior tiles leave free (down to two thirds of the interior
    // length, which covers the measured extra cost).
    const int64_t slots = (int64_t)cus * 4;
    const int64_t spare = slots - (int64_t)(p->strips - 2) * p->segs;
    if (spare / 2 > p->segs) {
      int64_t se = (Q + spare / 2 - 1) / (spare / 2);
      se = std::max<int64_t>(se, (2 * (int64_t)seg + 2) / 3);
      se = std::max<int64_t>(se, std::min<int64_t>(seg, std::max(16, 4 * depth * p->r)));
      const int64_t segs_e = (Q + se - 1) / se;
      if (se < seg && segs_e > p->segs) {
        p->seg_len_e = (int)se;
        p->edge_tiles = (int)(2 * segs_e);
        p->tiles = p->edge_tiles + (p->strips - 2) * p->segs;
      }
    }
  }
  p->hq_rows = seg + 2 * depth * p->r + 8;
  p->block = 256;
  p->grid = (p->tiles + 3) / 4;
}

// Redundant lanes per side of a 3D tile along an axis with B cells per lane.
int halo_lanes_3d(int depth, int r, int B) { return (depth * r + B - 1) / B; }

void plan_3d_tiles(stencil_plan_s* p, int depth, int seg_hint, int cus) {
  constexpr int L = 16;  // lanes along x and along y
  const int BX = 4, BY = tb3d_cells_y(p->dtype == STENCIL_F64 ? kF64 : kF32, p->r, p->pattern);
  auto strips = [&](int64_t n, int B, int H) {
    const int64_t side = (int64_t)(L - H) * B, mid = (int64_t)(L - 2 * H) * B;
    int64_t k = 0;
    if (n == (int64_t)L * B) return 1;  // one tile exactly covers the interior
    if (n > 2 * side) k = (n - 2 * side + mid - 1) / mid;
    return (int)(2 + k);
  };
  p->hx = halo_lanes_3d(depth, p->r, BX);
  p->hy = halo_lanes_3d(depth, p->r, BY);
  p->sx = strips(p->n[2], BX, p->hx);
  p->sy = strips(p->n[1], BY, p->hy);
  const int64_t Qz = p->ext[0];
  const int64_t xy = (int64_t)p->sx * p->sy;
  int seg;
  if (seg_hint > 0) {
    seg = seg_hint;
  } else {
    // One workgroup per CU (the LDS queues take most of a CU's 160 KB), so
    // tiles run in rounds of `cus`. A pass costs about (rounds) x (planes a
    // tile streams: its segment plus the 2 d r warm-up planes); pick the
    // segment count that minimises it (more, shorter segments fill the last
    // round better but stream more warm-up planes).
    const int64_t halo = 2 * (int64_t)depth * p->r;
    const int min_seg = std::max(8, 4 * depth * p->r);
    int64_t best_cost = -1;
    seg = (int)Qz;
    for (int64_t nseg = 1; nseg <= 64; ++nseg) {
      const int64_t s_len = (Qz + nseg - 1) / nseg;
      if (s_len < min_seg && nseg > 1) break;
      const int64_t real_segs = (Qz + s_len - 1) / s_len;
      const int64_t rounds = (xy * real_segs + cus - 1) / cus;
      const int64_t cost = rounds * (s_len + halo);
      if (best_cost < 0 || cost < best_cost) {
        best_cost = cost;
        seg = (int)s_len;
      }
    }
  }
  const int64_t plane_bytes = p->ext[1] * p->ext[2] * (int64_t)p->elem;
  const int64_t max_planes = ((int64_t)1 << 31) / plane_bytes - 2 * depth * p->r - 4;
  if (seg > max_planes) seg = (int)std::max<int64_t>(1, max_planes);
  if (seg > Qz) seg = (int)Qz;
  p->seg_len = seg;
  p->segs = (int)((Qz + seg - 1) / seg);
  p->tiles = (int)(xy * p->segs);
  p->block = 256;
  p->grid = p->tiles;
}

// Device tiling (tb3d_dev) applies to this 3D plan at `depth`: tiles of
// 64 x 16 interior cells cover the plane exactly, one per CU at most, and the
// padded grid and the halo ring stay below 2 GiB (the kernel addresses them
// with 32-bit offsets and uses offsets from 2 GiB up for dropped accesses).
bool device_tiling_fits(const stencil_plan_s* p, int depth, int cus) {
  const int dt = p->dtype == STENCIL_F64 ? kF64 : kF32;
  if (p->ndim != 3 || depth < 1 || depth > tb3d_dev_max_depth(dt, p->r, p->pattern)) return false;
  const int ty = tb3d_dev_tile_y();
  if (p->n[2] % 64 != 0 || p->n[1] % ty != 0) return false;
  const int64_t tiles = (p->n[2] / 64) * (p->n[1] / ty);
  if (tiles < 1 || tiles > cus) return false;
  const int64_t grid_bytes = p->padded_elems * (int64_t)p->elem;
  const int64_t ring_bytes = tiles * tb3d_dev_ring_elems(p->r, depth) * 2 * (int64_t)p->elem;
  return grid_bytes < ((int64_t)1 << 31) && ring_bytes < ((int64_t)1 << 31);
}

// Device-tiled geometry and workspace layout: [ping-pong grid][halo ring]
// [error word].
void plan_device_3d(stencil_plan_s* p, int depth) {
  p->scheme = STENCIL_SCHEME_DEVICE_3D;
  p->depth = depth;
  p->sx = (int)(p->n[2] / 64);
  p->sy = (int)(p->n[1] / tb3d_dev_tile_y());
  p->hx = p->hy = 0;
  p->seg_len = (int)p->ext[0];
  p->segs = 1;
  p->tiles = p->sx * p->sy;
  p->grid = p->tiles;
  p->block = 256;
}

stencil_status validate(const double* coeffs, int32_t radius, const stencil_shape* shape,
                        stencil_dtype dtype, int64_t T) {
  if (!coeffs) return fail(STENCIL_ERR_INVALID, "coeffs is NULL");
  if (!shape) return fail(STENCIL_ERR_INVALID, "shape is NULL");
  if (shape->ndim != 2 && shape->ndim != 3)
    return fail(STENCIL_ERR_INVALID, "ndim must be 2 or 3 (got %d)", shape->ndim);
  if (radius < 0 || radius > kMaxR)
    return fail(STENCIL_ERR_INVALID, "radius must be in [0, %d] (got %d)", kMaxR, radius);
  if (T < 0) return fail(STENCIL_ERR_INVALID, "T must be >= 0 (got %lld)", (long long)T);
  if (dtype != STENCIL_F32 && dtype != STENCIL_F64)
    return fail(STENCIL_ERR_INVALID, "unknown dtype %d", (int)dtype);
  for (int d = 0; d < shape->ndim; ++d) {
    if (shape->n[d] < 1)
      return fail(STENCIL_ERR_INVALID, "extent n[%d] must be >= 1 (got %lld)", d,
                  (long long)shape->n[d]);
    if (shape->n[d] > ((int64_t)1 << 30))
      return fail(STENCIL_ERR_INVALID, "extent n[%d] too large", d);
  }
  return STENCIL_OK;
}

}  // namespace

namespace {

template <typename Real>
stencil_status run_blocked_2d(const stencil_plan_s* p, const void* in, void* out, void* ws,
                              hipStream_t stream) {
  const size_t npass = p->pass_depth.size();
  // the pass sequence alternates between two buffers and ends in `out`
  void* bufs[2];
  if (npass % 2 == 1) { bufs[0] = out; bufs[1] = ws; }
  else { bufs[0] = ws; bufs[1] = out; }
  // halo frame of every buffer a pass writes: copied once from `in`
  hipError_t e = frame_copy_launch(p->dtype == STENCIL_F64 ? kF64 : kF32, in, out, p->ext, p->rad, stream);
  if (e != hipSuccess) return hip_fail(e, "halo copy");
  if (npass >= 2) {
    e = frame_copy_launch(p->dtype == STENCIL_F64 ? kF64 : kF32, in, ws, p->ext, p->rad, stream);
    if (e != hipSuccess) return hip_fail(e, "halo copy");
  }
  Tb2dParams<Real> prm;
  std::memset(&prm, 0, sizeof(prm));
  prm.orig = in;
  prm.P = p->ext[2];
  prm.Q = p->ext[1];
  prm.n_strips = p->strips;
  prm.n_segs = p->segs;
  prm.seg_len = p->seg_len;
  prm.ntiles = p->tiles;
  prm.hq_rows = p->hq_rows;
  prm.hl = p->hl;
  prm.seg_len_e = p->seg_len_e;
  prm.edge_tiles = p->edge_tiles;
  for (size_t i = 0; i < p->coeffs.size(); ++i) prm.w[i] = (Real)p->coeffs[i];
  const size_t lds = (size_t)4 * p->hq_rows * 2 * p->r * sizeof(Real);
  const void* src = in;
  for (size_t k = 0; k < npass; ++k) {
    prm.src = src;
    prm.dst = bufs[k % 2];
    e = tb2d_launch(p->dtype == STENCIL_F64 ? kF64 : kF32, p->r, p->pattern, p->pass_depth[k], &prm,
                    p->grid, p->block, lds, stream);
    if (e != hipSuccess) return hip_fail(e, "blocked 2D pass launch");
    src = bufs[k % 2];
  }
  return STENCIL_OK;
}

template <typename Real>
stencil_status run_blocked_3d(const stencil_plan_s* p, const void* in, void* out, void* ws,
                              hipStream_t stream) {
  const size_t npass = p->pass_depth.size();
  void* bufs[2];
  if (npass % 2 == 1) { bufs[0] = out; bufs[1] = ws; }
  else { bufs[0] = ws; bufs[1] = out; }
  const int dt = p->dtype == STENCIL_F64 ? kF64 : kF32;
  hipError_t e = frame_copy_launch(dt, in, out, p->ext, p->rad, stream);
  if (e != hipSuccess) return hip_fail(e, "halo copy");
  if (npass >= 2) {
    e = frame_copy_launch(dt, in, ws, p->ext, p->rad, stream);
    if (e != hipSuccess) return hip_fail(e, "halo copy");
  }
  Tb3dParams<Real> prm;
  std::memset(&prm, 0, sizeof(prm));
  prm.P = p->ext[2];
  prm.Qy = p->ext[1];
  prm.Qz = p->ext[0];
  prm.sx = p->sx;
  prm.sy = p->sy;
  prm.n_segs = p->segs;
  prm.seg_len = p->seg_len;
  prm.ntiles = p->tiles;
  prm.hx = p->hx;
  prm.hy = p->hy;
  for (size_t i = 0; i < p->coeffs.size() && i < 125; ++i) prm.w[i] = (Real)p->coeffs[i];
  const void* src = in;
  for (size_t k = 0; k < npass; ++k) {
    prm.src = src;
    prm.dst = bufs[k % 2];
    e = tb3d_launch(dt, p->r, p->pattern, p->pass_depth[k], &prm, p->grid, stream);
    if (e != hipSuccess) return hip_fail(e, "blocked 3D pass launch");
    src = bufs[k % 2];
  }
  return STENCIL_OK;
}

// Device-tiled 3D passes: each pass is one launch of gx x gy workgroups (all
// resident). The halo ring is zeroed once per execution; the tags of its words
// grow monotonically over the passes (pass k starts from the sum of the
// earlier passes' iterations), so nothing is reset between passes.
template <typename Real>
stencil_status run_device_3d(const stencil_plan_s* p, const void* in, void* out, void* ws,
                             hipStream_t stream) {
  const size_t npass = p->pass_depth.size();
  char* wsb = (char*)ws;
  void* grid2 = npass >= 2 ? ws : nullptr;
  void* bufs[2];
  if (npass % 2 == 1) { bufs[0] = out; bufs[1] = grid2; }
  else { bufs[0] = grid2; bufs[1] = out; }
  const int dt = p->dtype == STENCIL_F64 ? kF64 : kF32;
  unsigned int* report = stream_report_word(stream);
  if (!report) return fail(STENCIL_ERR_NOMEM, "device error word allocation failed");
  hipError_t e = frame_copy_launch(dt, in, out, p->ext, p->rad, stream);
  if (e != hipSuccess) return hip_fail(e, "halo copy");
  if (grid2) {
    e = frame_copy_launch(dt, in, grid2, p->ext, p->rad, stream);
    if (e != hipSuccess) return hip_fail(e, "halo copy");
  }
  unsigned int* ctl = (unsigned int*)(wsb + p->dev_ctl_off);
  e = fill_zero_u32_launch((unsigned int*)(wsb + p->dev_ring_off), (int64_t)(p->dev_ring_bytes / 4), stream);
  if (e == hipSuccess) e = fill_zero_u32_launch(ctl, 1, stream);
  if (e != hipSuccess) return hip_fail(e, "halo ring reset");
  Tb3dDevParams<Real> prm;
  std::memset(&prm, 0, sizeof(prm));
  prm.ring = wsb + p->dev_ring_off;
  prm.err = ctl;
  prm.P = p->ext[2];
  prm.Qy = p->ext[1];
  prm.Qz = p->ext[0];
  prm.gx = p->sx;
  prm.gy = p->sy;
  prm.timeout_ticks = watchdog_ticks();
  for (size_t i = 0; i < p->coeffs.size() && i < 125; ++i) prm.w[i] = (Real)p->coeffs[i];
  const void* src = in;
  uint32_t base = 0;
  for (size_t k = 0; k < npass; ++k) {
    prm.src = src;
    prm.dst = bufs[k % 2];
    prm.depth = p->pass_depth[k];
    prm.flag_base = base;
    e = tb3d_dev_launch(dt, p->r, p->pattern, p->pass_depth[k], &prm, stream);
    if (e != hipSuccess) return hip_fail(e, "device-tiled 3D pass launch");
    base += (uint32_t)tb3d_dev_iterations(p->r, p->pass_depth[k], p->ext[0]);
    src = bufs[k % 2];
  }
  e = error_fold_launch(prm.err, report, stream);
  return e == hipSuccess ? STENCIL_OK : hip_fail(e, "device-tiled error report");
}

template <typename Real>
stencil_status run_naive(const stencil_plan_s* p, const void* in, void* out, void* ws,
                         hipStream_t stream) {
  const size_t bytes = (size_t)p->padded_elems * p->elem;
  const size_t npass = p->pass_depth.size();
  void* work = npass >= 2 ? ws : nullptr;
  hipError_t e = hipMemcpyAsync(out, in, bytes, hipMemcpyDeviceToDevice, stream);
  if (e != hipSuccess) return hip_fail(e, "copy in->out");
  if (work) {
    e = hipMemcpyAsync(work, in, bytes, hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) return hip_fail(e, "copy in->workspace");
  }
  void* bufs[2];
  if (npass % 2 == 1) { bufs[0] = out; bufs[1] = work; }
  else { bufs[0] = work; bufs[1] = out; }
  NaiveParams<Real> prm;
  std::memset(&prm, 0, sizeof(prm));
  for (int d = 0; d < 3; ++d) {
    prm.ext[d] = p->ext[d];
    prm.lo[d] = p->rad[d];
    prm.hi[d] = (int32_t)(p->ext[d] - p->rad[d]);
  }
  prm.ntaps = (int32_t)p->tap_off.size();
  for (size_t i = 0; i < p->tap_off.size(); ++i) {
    prm.off[i] = p->tap_off[i];
    prm.w[i] = (Real)p->tap_w[i];
  }
  const void* src = in;
  for (size_t k = 0; k < npass; ++k) {
    prm.src = src;
    prm.dst = bufs[k % 2];
    e = naive_launch(p->dtype == STENCIL_F64 ? kF64 : kF32, &prm, p->cells, stream);
    if (e != hipSuccess) return hip_fail(e, "plain step launch");
    src = bufs[k % 2];
  }
  return STENCIL_OK;
}

}  // namespace

namespace stencil_impl {

// Pass schedule of plan p for T steps (ceil(T / depth) passes, the last one
// taking the remainder; one step per pass for the plain kernel; none for a
// copy) and the workspace it needs: one padded grid for the ping-pong when
// there are two or more passes, plus the halo ring and control words of a
// device-tiled plan. The tile geometry is T's own business only through the
// depth, so a plan made for one T serves any other T with this.
void plan_schedule(stencil_plan_s* p, int64_t T) {
  p->T = T;
  if (T == 0) {
    p->scheme = STENCIL_SCHEME_COPY;
    p->pass_depth.clear();
  } else if (p->scheme == STENCIL_SCHEME_BLOCKED_2D || p->scheme == STENCIL_SCHEME_BLOCKED_3D ||
             p->scheme == STENCIL_SCHEME_DEVICE_3D) {
    const int64_t q = T / p->depth, rem = T % p->depth;
    p->pass_depth.assign((size_t)q, p->depth);
    if (rem) p->pass_depth.push_back((int)rem);
  } else if (p->scheme != STENCIL_SCHEME_COPY) {
    p->pass_depth.assign((size_t)T, 1);
  }
  const size_t bytes = (size_t)p->padded_elems * p->elem;
  p->workspace = p->pass_depth.size() >= 2 ? bytes : 0;
  if (p->scheme == STENCIL_SCHEME_DEVICE_3D) {
    auto align = [](size_t v) { return (v + 255) / 256 * 256; };
    p->dev_ring_off = align(p->workspace);
    // each ring cell is stored as (32-bit word, tag) pairs: twice its size
    p->dev_ring_bytes = (size_t)p->tiles * (size_t)tb3d_dev_ring_elems(p->r, p->depth) * 2 * p->elem;
    p->dev_ctl_off = align(p->dev_ring_off + p->dev_ring_bytes);
    p->workspace = p->dev_ctl_off + align(sizeof(unsigned int));
  }
}

}  // namespace stencil_impl

extern "C" {

const char* stencil_last_error(void) { return g_last_error.c_str(); }

stencil_status stencil_plan(stencil_plan_t* out_plan, const double* coeffs, int32_t radius,
                            const stencil_shape* shape, stencil_dtype dtype, int64_t T,
                            const stencil_tuning* hint) {
  if (!out_plan) return fail(STENCIL_ERR_INVALID, "plan is NULL");
  *out_plan = nullptr;
  stencil_status st = validate(coeffs, radius, shape, dtype, T);
  if (st != STENCIL_OK) return st;

  stencil_plan_s* p = new (std::nothrow) stencil_plan_s();
  if (!p) return fail(STENCIL_ERR_NOMEM, "host allocation failed");
  p->ndim = shape->ndim;
  p->r = radius;
  p->dtype = dtype;
  p->T = T;
  p->elem = dtype == STENCIL_F64 ? 8 : 4;
  const int side = 2 * radius + 1;
  const int count = p->ndim == 2 ? side * side : side * side * side;
  p->coeffs.assign(coeffs, coeffs + count);
  if (!classify(p->ndim, radius, coeffs, &p->pattern, &p->points)) {
    delete p;
    return fail(STENCIL_ERR_INVALID, "coefficients must be finite");
  }
  const int off = 3 - p->ndim;
  p->cells = 1;
  p->padded_elems = 1;
  for (int d = 0; d < p->ndim; ++d) {
    p->n[off + d] = shape->n[d];
    p->ext[off + d] = shape->n[d] + 2 * radius;
    p->rad[off + d] = radius;
    p->cells *= shape->n[d];
    p->padded_elems *= p->ext[off + d];
  }
  // taps for the plain kernel
  for (int idx = 0; idx < count; ++idx) {
    if (coeffs[idx] == 0.0) continue;
    int rem = idx;
    int64_t o = 0, stride = 1;
    for (int d = 2; d >= off; --d) {
      const int pd = rem % side - radius;
      rem /= side;
      o += (int64_t)pd * stride;
      stride *= p->ext[d];
    }
    p->tap_off.push_back(o);
    p->tap_w.push_back(coeffs[idx]);
  }

  const bool force_naive = hint && (hint->flags & STENCIL_FLAG_NAIVE);
  // without a depth or segment hint, take the autotuner's cached choice
  stencil_tuning tuned;
  std::memset(&tuned, 0, sizeof(tuned));
  const bool use_cache = !(hint && (hint->flags & STENCIL_FLAG_NO_CACHE)) &&
                         !(hint && (hint->depth > 0 || hint->tile[0] > 0));
  if (use_cache && T > 0) {
    int d = 0, seg = 0, sfl = 0;
    if (tune_lookup_plan(p, false, &d, &seg, &sfl)) {
      tuned.depth = d;
      tuned.tile[0] = seg;
      // the measured scheme, unless the caller forbade or required one
      const int caller = hint ? hint->flags : 0;
      const int scheme_bits = STENCIL_FLAG_DEVICE_TILING | STENCIL_FLAG_OVERLAPPED_TILING;
      tuned.flags = (caller & scheme_bits) ? caller : (caller | sfl);
      hint = &tuned;
    }
  }
  if (T == 0) {
    p->scheme = STENCIL_SCHEME_COPY;
    p->depth = 0;
  } else {
    p->scheme = STENCIL_SCHEME_NAIVE;
    p->depth = 1;
    DeviceInfo di = device_info();
    const int cus = di.ok ? di.cus : machine().cus;
    const int dt = dtype == STENCIL_F64 ? kF64 : kF32;
    const int hint_depth = hint ? hint->depth : 0;
    const int hint_seg = hint ? hint->tile[0] : 0;
    const int hflags = hint ? hint->flags : 0;
    // Candidates are the feasible (scheme, depth) pairs; a depth hint fixes the
    // depth, otherwise the model's predicted rate decides (paper Sections 5-6).
    // The model resolves rates to a few percent and leaves out per-pass costs
    // (launches, halo-frame copies, a serving round's quantum of passes), so
    // among the candidates within 3% of the best prediction the deepest (the
    // fewest passes) wins.
    std::vector<std::pair<double, stencil_plan_s>> cands;
    p->shared = (hflags & STENCIL_FLAG_UNIFORM_TILES) != 0;
    auto consider = [&](const stencil_plan_s& c) { cands.emplace_back(plan_model_rate(&c), c); };
    if (!force_naive && p->ndim == 2 && radius >= 1 && p->points > 0) {
      const int V = tb2d_cols_per_lane(dtype, radius, p->pattern);
      const int maxd = tb2d_max_depth(dtype, radius, p->pattern);
      int lo = 1, hi = maxd;
      // (a variant without a blocked kernel, maxd = 0, has no candidate)
      if (hint_depth > 0 && maxd >= 1) lo = hi = std::min(hint_depth, maxd);
      for (int depth = lo; depth <= hi && (int64_t)depth <= T; ++depth) {
        // every strip must lie inside the interior, and its edge redundancy fit in the wave
        const int HL = (depth * radius + V - 1) / V;
        if (p->n[2] < (int64_t)kWave * V || 2 * HL >= kWave) continue;
        stencil_plan_s c = *p;
        c.scheme = STENCIL_SCHEME_BLOCKED_2D;
        c.depth = depth;
        plan_2d_tiles(&c, depth, hint_seg, cus, !(hflags & STENCIL_FLAG_UNIFORM_TILES));
        consider(c);
      }
      if (hint_depth > 0 && cands.empty() && maxd >= 1 && T >= 1) {
        // a hint deeper than T: the deepest feasible depth not above T
        for (int depth = std::min<int64_t>(maxd, T); depth >= 1 && cands.empty(); --depth) {
          const int HL = (depth * radius + V - 1) / V;
          if (p->n[2] < (int64_t)kWave * V || 2 * HL >= kWave) continue;
          stencil_plan_s c = *p;
          c.scheme = STENCIL_SCHEME_BLOCKED_2D;
          c.depth = depth;
          plan_2d_tiles(&c, depth, hint_seg, cus, !(hflags & STENCIL_FLAG_UNIFORM_TILES));
          consider(c);
        }
      }
    }
    if (!force_naive && p->ndim == 3 && radius >= 1 && p->points > 0) {
      const bool no_dev = (hflags & STENCIL_FLAG_OVERLAPPED_TILING) != 0;
      const bool only_dev = (hflags & STENCIL_FLAG_DEVICE_TILING) != 0 && !no_dev;
      const int by = tb3d_cells_y(dt, radius, p->pattern);
      auto depths = [&](int maxd, int* lo, int* hi) {
        *lo = 1;
        *hi = (int)std::min<int64_t>(maxd, T);
        if (hint_depth > 0) *lo = *hi = (int)std::min<int64_t>(std::min(hint_depth, maxd), T);
        if (*lo < 1) {  // no blocked kernel for this variant: no candidate
          *lo = 1;
          *hi = 0;
        }
      };
      int lo, hi;
      // device tiling: non-overlapping tiles exchanging edges every z-step
      if (!no_dev) {
        depths(tb3d_dev_max_depth(dt, radius, p->pattern), &lo, &hi);
        for (int depth = lo; depth <= hi; ++depth) {
          if (!device_tiling_fits(p, depth, cus)) continue;
          stencil_plan_s c = *p;
          plan_device_3d(&c, depth);
          consider(c);
        }
      }
      // overlapped tiles (when device tiling was asked for, only if it does not apply)
      if (!(only_dev && !cands.empty())) {
        depths(tb3d_max_depth(dt, radius, p->pattern), &lo, &hi);
        for (int depth = lo; depth <= hi; ++depth) {
          // tiles of 64 x 16*by interior cells; each needs its redundant margins inside
          const int hx = halo_lanes_3d(depth, radius, 4), hy = halo_lanes_3d(depth, radius, by);
          if (!(p->n[2] >= 64 && p->n[1] >= 16 * by && 2 * hx < 16 && 2 * hy < 16 && p->plan_ok_3d(depth))) continue;
          stencil_plan_s c = *p;
          c.scheme = STENCIL_SCHEME_BLOCKED_3D;
          c.depth = depth;
          plan_3d_tiles(&c, depth, hint_seg, cus);
          consider(c);
        }
      }
    }
    if (!cands.empty()) {
      double top = 0.0;
      for (const auto& c : cands) top = std::max(top, c.first);
      const stencil_plan_s* pick = nullptr;
      for (const auto& c : cands)
        if (c.first >= 0.97 * top && (!pick || c.second.depth > pick->depth ||
                                      (c.second.depth == pick->depth && c.first > plan_model_rate(pick))))
          pick = &c.second;
      *p = *pick;
    }
    const bool want_persistent = hint && (hint->flags & STENCIL_FLAG_PERSISTENT);
    if (want_persistent &&
        (p->scheme == STENCIL_SCHEME_BLOCKED_2D || p->scheme == STENCIL_SCHEME_BLOCKED_3D)) {
      // one persistent kernel per variant, at the launches' depths where its
      // registers allow
      const int cap = batch_single_depth(dtype == STENCIL_F64 ? kF64 : kF32, p->ndim, radius, p->pattern);
      if (cap >= 1) {
        p->persistent = true;
        if (p->depth > cap) {
          DeviceInfo di = device_info();
          const int cus = di.ok ? di.cus : 256;
          p->depth = cap;
          if (p->scheme == STENCIL_SCHEME_BLOCKED_2D)
            plan_2d_tiles(p, cap, hint->tile[0], cus, !(hint->flags & STENCIL_FLAG_UNIFORM_TILES));
          else plan_3d_tiles(p, cap, hint->tile[0], cus);
        }
      }
    }
  }
  plan_schedule(p, T);
  if (p->scheme == STENCIL_SCHEME_NAIVE && p->tap_off.size() > (size_t)kMaxNaiveTaps) {
    delete p;
    return fail(STENCIL_ERR_UNSUPPORTED, "more than %d non-zero coefficients without a blocked kernel",
                kMaxNaiveTaps);
  }
  *out_plan = p;
  return STENCIL_OK;
}

stencil_status stencil_plan_workspace(stencil_plan_t plan, size_t* bytes) {
  if (!plan || !bytes) return fail(STENCIL_ERR_INVALID, "NULL argument");
  *bytes = plan->workspace;
  return STENCIL_OK;
}

stencil_status stencil_plan_describe(stencil_plan_t plan, stencil_plan_info* info) {
  if (!plan || !info) return fail(STENCIL_ERR_INVALID, "NULL argument");
  std::memset(info, 0, sizeof(*info));
  info->scheme = plan->scheme;
  info->pattern = plan->pattern;
  info->points = plan->points;
  info->depth = plan->depth;
  info->passes = (int64_t)plan->pass_depth.size();
  info->tiles = plan->tiles;
  info->strips = plan->strips;
  info->seg_len = plan->seg_len;
  info->edge_seg_len = plan->scheme == STENCIL_SCHEME_BLOCKED_2D ? plan->seg_len_e : 0;
  info->edge_tiles = plan->scheme == STENCIL_SCHEME_BLOCKED_2D ? plan->edge_tiles : 0;
  info->cols_per_lane = plan->scheme == STENCIL_SCHEME_BLOCKED_2D ? tb2d_cols_per_lane(plan->dtype, plan->r, plan->pattern)
                        : plan->scheme == STENCIL_SCHEME_BLOCKED_3D ? 4 : 1;
  info->redundant_lanes = plan->scheme == STENCIL_SCHEME_BLOCKED_3D ? plan->hx
                          : plan->scheme == STENCIL_SCHEME_DEVICE_3D ? 0
                                                                     : plan->hl;
  if (plan->scheme == STENCIL_SCHEME_BLOCKED_3D || plan->scheme == STENCIL_SCHEME_DEVICE_3D)
    info->strips = plan->sx * plan->sy;
  if (plan->scheme == STENCIL_SCHEME_DEVICE_3D) info->cols_per_lane = 4;
  info->grid = plan->grid;
  info->block = plan->block;
  info->cells = plan->cells;
  info->padded_bytes = plan->padded_elems * (int64_t)plan->elem;
  info->workspace_bytes = (int64_t)plan->workspace;
  info->model_cells_per_s = plan_model_rate(plan);
  return STENCIL_OK;
}

stencil_status stencil_plan_destroy(stencil_plan_t plan) {
  delete plan;
  return STENCIL_OK;
}

stencil_status stencil_execute(stencil_plan_t plan, const void* in, void* out, void* workspace,
                               void* stream) {
  if (!plan) return fail(STENCIL_ERR_INVALID, "plan is NULL");
  if (!in || !out) return fail(STENCIL_ERR_INVALID, "in/out is NULL");
  const size_t bytes = (size_t)plan->padded_elems * plan->elem;
  const char* a = (const char*)in;
  const char* b = (const char*)out;
  if (a < b + bytes && b < a + bytes) return fail(STENCIL_ERR_ALIAS, "in and out overlap");
  if (plan->workspace > 0) {
    if (!workspace) return fail(STENCIL_ERR_INVALID, "workspace of %zu bytes required", plan->workspace);
    const char* w = (const char*)workspace;
    const size_t wb = plan->workspace;
    if ((w < a + bytes && a < w + wb) || (w < b + bytes && b < w + wb))
      return fail(STENCIL_ERR_ALIAS, "workspace overlaps in or out");
  }
  hipStream_t s = (hipStream_t)stream;
  if (plan->scheme == STENCIL_SCHEME_COPY) {
    hipError_t e = hipMemcpyAsync(out, in, bytes, hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? STENCIL_OK : hip_fail(e, "copy");
  }
  if (plan->persistent) {
    // every pass in one persistent launch, passes separated by the grid-wide
    // count of finished tiles
    std::vector<stencil_plan_s*> plans{plan};
    std::vector<const void*> ins{in};
    std::vector<void*> outs{out}, wss{workspace};
    return batch_run(plans, ins, outs, wss, s);
  }
  if (plan->scheme == STENCIL_SCHEME_BLOCKED_2D) {
    return plan->dtype == STENCIL_F64 ? run_blocked_2d<double>(plan, in, out, workspace, s)
                                      : run_blocked_2d<float>(plan, in, out, workspace, s);
  }
  if (plan->scheme == STENCIL_SCHEME_BLOCKED_3D) {
    return plan->dtype == STENCIL_F64 ? run_blocked_3d<double>(plan, in, out, workspace, s)
                                      : run_blocked_3d<float>(plan, in, out, workspace, s);
  }
  if (plan->scheme == STENCIL_SCHEME_DEVICE_3D) {
    return plan->dtype == STENCIL_F64 ? run_device_3d<double>(plan, in, out, workspace, s)
                                      : run_device_3d<float>(plan, in, out, workspace, s);
  }
  return plan->dtype == STENCIL_F64 ? run_naive<double>(plan, in, out, workspace, s)
                                    : run_naive<float>(plan, in, out, workspace, s);
}

stencil_status stencil_run(const double* coeffs, int32_t radius, const stencil_shape* shape,
                           stencil_dtype dtype, int64_t T, const void* in, void* out,
                           void* stream) {
  stencil_status st = validate(coeffs, radius, shape, dtype, T);
  if (st != STENCIL_OK) return st;
  if (!in || !out) return fail(STENCIL_ERR_INVALID, "in/out is NULL");
  stencil_plan_t plan = nullptr;
  st = stencil_plan(&plan, coeffs, radius, shape, dtype, T, nullptr);
  if (st != STENCIL_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  void* ws = nullptr;
  if (plan->workspace) {
    const size_t wbytes = plan->workspace;
    hipError_t e = hipMallocAsync(&ws, wbytes, s);
    if (e != hipSuccess) {
      stencil_plan_destroy(plan);
      return fail(STENCIL_ERR_NOMEM, "workspace allocation of %zu bytes failed: %s", wbytes,
                  hipGetErrorString(e));
    }
  }
  st = stencil_execute(plan, in, out, ws, stream);
  if (ws) {
    hipError_t e = hipFreeAsync(ws, s);
    if (e != hipSuccess && st == STENCIL_OK) st = hip_fail(e, "workspace release");
  }
  stencil_plan_destroy(plan);
  return st;
}

}  // extern "C"
