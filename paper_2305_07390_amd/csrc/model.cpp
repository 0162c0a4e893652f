// Practical attainable performance model (paper Section 5) and the design
// rules derived from it (Section 6): desired depth, minimum 3D tile, valid
// proportions of SM and device tiling. Host code; its outputs are pinned
// against the numbers the paper prints for an A100. The planner and the
// autotuner evaluate it for each candidate plan with the MI355X machine
// parameters (machine.cpp).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "../../include/stencil.h"

namespace {

// Valid proportion of SM (overlapped) tiling, Section 5.2.1: each tiled
// dimension loses t*rad cells on both sides.
double v_smtile(const stencil_model_params& m) {
  double v = 1.0;
  const int nd = m.tiled_dims < 1 ? 1 : (m.tiled_dims > 2 ? 2 : m.tiled_dims);
  for (int d = 0; d < nd; ++d) {
    const double tile = m.tile[d];
    if (tile <= 0) return 0.0;
    v *= std::max(0.0, (tile - 2.0 * m.t * m.rad) / tile);
  }
  return v;
}

}  // namespace

extern "C" {

stencil_status stencil_model_eval(const stencil_model_params* m, stencil_model_result* out) {
  if (!m || !out) return STENCIL_ERR_INVALID;
  if (!(m->B_gm > 0) || !(m->thr_cmp > 0) || !(m->cell_bytes > 0) || !(m->t > 0))
    return STENCIL_ERR_INVALID;
  std::memset(out, 0, sizeof(*out));
  // Equations for T_gm, T_sm, T_com (Section 5.1)
  out->T_gm = m->a_gm * m->D_gm / m->B_gm * m->cell_bytes;
  out->T_sm = m->B_sm > 0 ? m->a_sm * m->D_sm * m->t / m->B_sm * m->cell_bytes : 0.0;
  out->T_cmp = m->a_cmp * m->D_cmp * m->t / m->thr_cmp;
  out->T_stencil = std::max(out->T_gm, std::max(out->T_sm, out->T_cmp));
  out->bottleneck = out->T_stencil == out->T_gm ? 0 : (out->T_stencil == out->T_sm ? 1 : 2);
  out->P = m->D_all * m->t / out->T_stencil;
  // Valid proportion (Section 5.2)
  if (m->tiling == STENCIL_MODEL_SM_TILING) {
    out->V = v_smtile(*m);
  } else if (m->tiling == STENCIL_MODEL_DEVICE_TILING) {
    out->V = out->T_stencil / (out->T_stencil + m->t_dsync * m->n_sync);
  } else {
    out->V = 1.0;
  }
  out->PP = out->P * out->V;

  // Desired depth (Section 6.2): the smallest t with
  //   a_sm * t * D_sm / B_sm >= a_gm * D_gm(t) / B_gm,
  // where device tiling adds the tile halo to the global traffic:
  //   D_gm(t) = tile_x * tile_y + (tile_x + tile_y) * 2 * t * rad.
  if (m->B_sm > 0 && m->a_sm > 0 && m->D_sm > 0) {
    const double lhs = m->a_sm * m->D_sm / m->B_sm;
    if (m->tiling == STENCIL_MODEL_DEVICE_TILING) {
      const double area = m->tile[0] * m->tile[1];
      const double perim = (m->tile[0] + m->tile[1]) * 2.0 * m->rad;
      const double denom = lhs - m->a_gm * perim / m->B_gm;
      out->t_desired = denom > 0 ? (m->a_gm * area / m->B_gm) / denom : INFINITY;
    } else {
      out->t_desired = (m->a_gm * m->D_gm / m->B_gm) / lhs;
    }
    // Minimum square tile for a 3D device tile (Section 6.4):
    //   tile_x * tile_y * a_sm / B_sm > (tile_x + tile_y) * 2 * a_gm * rad / B_gm
    out->min_tile = 4.0 * m->a_gm * m->B_sm / (m->a_sm * m->B_gm) * m->rad;
  }
  return STENCIL_OK;
}

}  // extern "C"
