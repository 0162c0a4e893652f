// Machine parameters of the attainable-performance model (paper Section 5.1:
// global and on-chip bandwidth, compute throughput; Section 5.2.2: the cost of
// a synchronisation) and the planner's use of the model: the predicted rate
// of a concrete plan, from its exact tile geometry.
//
// The defaults are MI355X values measured with this library's probes
// (stencil_probe_*): a streaming copy, LDS reads over all CUs, a device-wide
// barrier and a neighbour-counter round; the vector FP64 peak is the chip's
// 256 CUs x 4 SIMDs x 16 FMA lanes x 2 flops at the clock measured under the
// stencil kernels (about 2.15 GHz); FP32 runs at the same rate as built
// (packed FP32 off). stencil_machine_calibrate replaces the measured ones
// with fresh probe results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "launch.hpp"
#include "plan.hpp"

namespace stencil_impl {
namespace {

stencil_machine defaults() {
  stencil_machine m;
  std::memset(&m, 0, sizeof(m));
  m.hbm_bytes_per_s = 5.1e12;
  m.lds_bytes_per_s = 68.7e12;
  m.fp64_flops = 256.0 * 4 * 16 * 2 * 2.15e9;
  m.fp32_flops = m.fp64_flops;
  m.grid_sync_s = 9.5e-6;
  m.neighbor_sync_s = 3.3e-6;
  m.hbm_latency_s = 184e-9;
  m.lds_latency_s = 25e-9;
  m.fma_latency_s = 2.6e-9;
  m.cus = 256;
  return m;
}

std::mutex g_mu;
stencil_machine g_machine = defaults();

bool valid(const stencil_machine& m) {
  return m.hbm_bytes_per_s > 0 && m.lds_bytes_per_s > 0 && m.fp64_flops > 0 && m.fp32_flops > 0 &&
         m.grid_sync_s >= 0 && m.neighbor_sync_s >= 0 && m.cus > 0;
}

// T = max(T_gm, T_sm, T_cmp) of one pass through stencil_model_eval (Section
// 5.1), with the counts of the whole pass: D_gm cells moved through HBM (one
// access each), D_sm cells through LDS, D_cmp cell-steps computed.
double pass_time(const stencil_machine& m, bool f64, double hbm_cells, double lds_cells, double cmp_cells,
                 int points) {
  stencil_model_params q;
  std::memset(&q, 0, sizeof(q));
  q.B_gm = m.hbm_bytes_per_s;
  q.B_sm = lds_cells > 0 ? m.lds_bytes_per_s : 0.0;
  q.thr_cmp = f64 ? m.fp64_flops : m.fp32_flops;
  q.cell_bytes = f64 ? 8.0 : 4.0;
  q.a_gm = 1.0;
  q.a_sm = 1.0;
  q.a_cmp = 2.0 * points;
  q.D_gm = hbm_cells;
  q.D_sm = lds_cells;
  q.D_cmp = cmp_cells;
  q.D_all = 1.0;
  q.t = 1.0;
  q.tiling = STENCIL_MODEL_NO_TILING;
  stencil_model_result r;
  if (stencil_model_eval(&q, &r) != STENCIL_OK) return INFINITY;
  return r.T_stencil;
}

}  // namespace

stencil_machine machine() {
  std::lock_guard<std::mutex> lock(g_mu);
  return g_machine;
}

// Predicted cells/s of valid output of a full-depth pass of plan p (0 when
// the scheme is not blocked). Each scheme's counts follow its kernel:
//   blocked 2D: every tile computes and reads its 64V-column strip over its
//     segment plus 2 d r warm-up rows; writes are the valid cells; no LDS in
//     the level loop (registers and DPP); tiles run in rounds of one per
//     SIMD (a batched plan's rounds are filled by the other jobs);
//   blocked 3D: every tile computes and reads 64 x 16 BY cells over its
//     segment plus 2 d r warm-up planes; per level the lanes exchange their
//     top and bottom rows through LDS; tiles run in rounds of one per CU;
//   device 3D: no redundant cells; the halo ring adds (d - 1) levels of
//     edges per z-step, written and read (two 64-bit words per FP64 cell);
//     each z-step ends with one neighbour synchronisation, whose cost gives
//     the valid proportion T_step / (T_step + t_sync) of Section 5.2.2.
double plan_model_rate(const stencil_plan_s* p) {
  if (!p || p->depth < 1) return 0.0;
  const stencil_machine m = machine();
  const bool f64 = p->dtype == STENCIL_F64;
  const double d = p->depth, r = p->r;
  const double N = (double)p->cells;
  double t_pass = 0.0;
  if (p->scheme == STENCIL_SCHEME_BLOCKED_2D) {
    const double V = tb2d_cols_per_lane(p->dtype, p->r, p->pattern);
    const double cols = kWave * V;
    const double Q = (double)p->ext[1];
    auto rows = [&](double seg) { return std::min(seg + 2.0 * d * r, Q); };
    double computed;
    if (p->edge_tiles > 0)
      computed = cols * (p->edge_tiles * rows(p->seg_len_e) + (double)(p->strips - 2) * p->segs * rows(p->seg_len));
    else
      computed = cols * (double)p->strips * p->segs * rows(p->seg_len);
    t_pass = pass_time(m, f64, computed + N, 0.0, computed * d, p->points);
    // one tile per SIMD at a time: tiles run in rounds over the wave slots,
    // and a round with fewer tiles than slots leaves the rest idle (unless
    // other jobs' tiles fill it)
    const double slots = 4.0 * m.cus;
    if (!p->shared) t_pass *= std::ceil(p->tiles / slots) * slots / (double)p->tiles;
  } else if (p->scheme == STENCIL_SCHEME_BLOCKED_3D) {
    const double BY = tb3d_cells_y(f64 ? kF64 : kF32, p->r, p->pattern);
    const double tile_cells = 64.0 * 16.0 * BY;
    const double planes = std::min((double)p->seg_len + 2.0 * d * r, (double)p->ext[0]);
    const double computed = (double)p->sx * p->sy * p->segs * tile_cells * planes;
    // per level and cell: its rows shared with the lanes above and below
    const double lds_cells = computed * d * (1.0 + 2.0 * std::min(r, BY) / BY);
    t_pass = pass_time(m, f64, computed + N, lds_cells, computed * d, p->points);
    // one tile per CU at a time: the last round runs part-empty (unless
    // other jobs' tiles fill it)
    const double rounds = std::ceil((double)p->tiles / m.cus);
    if (!p->shared) t_pass *= rounds * m.cus / (double)p->tiles;
  } else if (p->scheme == STENCIL_SCHEME_DEVICE_3D) {
    const double zsteps = (double)tb3d_dev_iterations(p->r, p->depth, p->ext[0]);
    const double edge_cells = (double)p->tiles * 2.0 * r * (64.0 + tb3d_dev_tile_y());
    const double ring_cells = zsteps * (d - 1.0) * edge_cells * 2.0 /* write + read */ * 2.0 /* tags */;
    const double lds_cells = N * d * (1.0 + 2.0 * r);
    const double t_work = pass_time(m, f64, 2.0 * N + ring_cells, lds_cells, N * d, p->points);
    const double t_step = t_work / zsteps;
    t_pass = zsteps * (t_step + m.neighbor_sync_s);
  } else {
    return 0.0;
  }
  return t_pass > 0 ? N * d / t_pass : 0.0;
}

}  // namespace stencil_impl

using namespace stencil_impl;

extern "C" {

stencil_status stencil_machine_get(stencil_machine* out) {
  if (!out) return fail(STENCIL_ERR_INVALID, "NULL result");
  *out = machine();
  return STENCIL_OK;
}

stencil_status stencil_machine_set(const stencil_machine* m) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!m) {
    g_machine = defaults();
    return STENCIL_OK;
  }
  if (!valid(*m)) return fail(STENCIL_ERR_INVALID, "machine parameters must be positive (syncs >= 0)");
  g_machine = *m;
  return STENCIL_OK;
}

stencil_status stencil_machine_calibrate(void* stream, stencil_machine* out) {
  stencil_machine m = machine();
  double v = 0;
  stencil_status st = stencil_probe_copy((int64_t)1 << 30, stream, &v);
  if (st != STENCIL_OK) return st;
  m.hbm_bytes_per_s = v;
  if ((st = stencil_probe_lds_bandwidth(stream, &v)) != STENCIL_OK) return st;
  m.lds_bytes_per_s = v;
  if ((st = stencil_probe_grid_sync(2000, stream, &v)) != STENCIL_OK) return st;
  m.grid_sync_s = v;
  uint64_t bad = 0;
  if ((st = stencil_probe_neighbor_sync(1, 2000, 0, stream, &v, &bad)) != STENCIL_OK) return st;
  if (bad != 0) return fail(STENCIL_ERR_DEVICE, "neighbour probe read %llu stale words", (unsigned long long)bad);
  m.neighbor_sync_s = v;
  if ((st = stencil_probe_latency(STENCIL_PROBE_HBM_LATENCY, stream, &v)) != STENCIL_OK) return st;
  m.hbm_latency_s = v;
  if ((st = stencil_probe_latency(STENCIL_PROBE_LDS_LATENCY, stream, &v)) != STENCIL_OK) return st;
  m.lds_latency_s = v;
  if ((st = stencil_probe_latency(STENCIL_PROBE_FMA64_LATENCY, stream, &v)) != STENCIL_OK) return st;
  m.fma_latency_s = v;
  DeviceInfo di = device_info();
  if (di.ok) m.cus = di.cus;
  if ((st = stencil_machine_set(&m)) != STENCIL_OK) return st;
  if (out) *out = m;
  return STENCIL_OK;
}

}  // extern "C"
