// Internal to the library: the plan object and helpers shared by capi.cpp
// (single grids) and batch_host.cpp (batches).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/stencil.h"
#include "launch.hpp"

namespace stencil_impl {

stencil_status fail(stencil_status st, const char* fmt, ...);
stencil_status hip_fail(hipError_t e, const char* what);

struct DeviceInfo {
  int cus = 0;
  bool ok = false;
};
DeviceInfo device_info();

}  // namespace stencil_impl

struct stencil_plan_s;
namespace stencil_impl {
// Autotuner cache lookup for a plan's stencil class and size (tune.cpp).
// flags (may be NULL) receives the entry's scheme flags (3D: device or
// overlapped tiling).
bool tune_lookup_plan(const stencil_plan_s* pl, bool batched, int* depth, int* seg, int* flags = nullptr);
// Prepared plans through the persistent batch kernel (batch_host.cpp).
// stencil_batch_submit with explicit batch tile lengths (2D rows, 3D planes);
// the launch's device memory comes from `pool` (NULL: the device's default
// stream-ordered pool).
stencil_status batch_submit_tiles(const stencil_job* jobs, int32_t n, void* stream,
                                  stencil_status* per_job_status, int seg2d, int seg3d,
                                  hipMemPool_t pool = nullptr);
// One batch job's plan: its depth, else the autotuner's batched depth, else
// the model's, on uniform tiles of seg2d rows / seg3d planes, capped at the
// fused kernel's depth (a job with no batched variant: a single-grid plan).
stencil_status plan_batch_job(const stencil_job& j, int seg2d, int seg3d, stencil_plan_s** out);
// Prepared plans (not owned) run for steps[i] steps each in one batch (a
// copy of each plan rescheduled with plan_schedule), from ins[i] to outs[i].
// The plans' memory must not overlap (not checked).
stencil_status batch_submit_planned(const std::vector<const stencil_plan_s*>& plans,
                                    const std::vector<int64_t>& steps, const std::vector<const void*>& ins,
                                    const std::vector<void*>& outs, hipStream_t s, hipMemPool_t pool);
int serve_seg_2d();
int serve_seg_3d();
// The model's machine parameters and its predicted rate of a plan
// (machine.cpp).
stencil_machine machine();
// Pass schedule and workspace of plan p for T steps at its depth (capi.cpp).
void plan_schedule(stencil_plan_s* p, int64_t T);
double plan_model_rate(const stencil_plan_s* p);
// Watchdog limit of in-kernel bounded waits (s_memrealtime ticks), and the
// per-stream report word that stencil_sync reads (batch_host.cpp).
int64_t watchdog_ticks();
unsigned int* stream_report_word(hipStream_t s);
stencil_status batch_run(const std::vector<stencil_plan_s*>& plans, const std::vector<const void*>& ins,
                         const std::vector<void*>& outs, const std::vector<void*>& wsg, hipStream_t s,
                         hipMemPool_t pool = nullptr);
}  // namespace stencil_impl

struct stencil_plan_s {
  int ndim = 0;
  int r = 0;
  int64_t n[3] = {1, 1, 1};
  // ^ interior extents, slowest first (padded to three axes)
  int64_t ext[3] = {1, 1, 1};  // padded extents padded to 3 axes (leading 1s for 2D)
  int rad[3] = {0, 0, 0};      // halo width per padded axis
  stencil_dtype dtype = STENCIL_F64;
  int64_t T = 0;
  std::vector<double> coeffs;  // dense box
  int pattern = STENCIL_GENERAL;
  int points = 0;
  int scheme = STENCIL_SCHEME_NAIVE;
  int depth = 1;
  std::vector<int> pass_depth;  // depth of each pass
  // 2D blocked geometry
  int strips = 0, segs = 0, seg_len = 0, tiles = 0, hq_rows = 0, hl = 0;
  // edge strips with their own (shorter) segments: edge_tiles > 0 lists them
  // first, two per segment (left, right)
  int seg_len_e = 0, edge_tiles = 0;
  // 3D blocked geometry
  int sx = 0, sy = 0, hx = 0, hy = 0;
  int grid = 0, block = 0;
  int64_t cells = 0;
  int64_t padded_elems = 0;
  size_t elem = 8;
  size_t workspace = 0;
  // plain kernel taps (offset, weight), dense-box order
  std::vector<int64_t> tap_off;
  std::vector<double> tap_w;
  bool persistent = false;  // all passes in one persistent launch
  // planned for a batch: its tiles share the device with other jobs', so a
  // round of tiles left part-empty by this grid is filled by theirs
  bool shared = false;
  // device-tiled 3D plan: byte offsets of the halo ring and of the control
  // words (progress counters, then the error word) in the workspace
  size_t dev_ring_off = 0, dev_ring_bytes = 0, dev_ctl_off = 0;
  bool plan_ok_3d(int) const { return r <= 2; }
};

