// Host side of batched execution (stencil_batch_submit, stencil_sync).
//
// Every job is planned like a single grid, with longer tiles so that small
// grids are not cut into slivers. Jobs with a blocked variant are grouped by
// dtype; each group becomes one persistent launch of the fused batch kernel
// over a work list of (job, pass) chunks ordered by the fraction of the job
// completed after the chunk, so that long and short jobs progress together
// and finish together. Device memory for workspaces, job descriptors, the
// work list and counters is one stream-ordered allocation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "launch.hpp"
#include "plan.hpp"
#include "worklist.hpp"

using namespace stencil_impl;

namespace {

constexpr int64_t kTimeoutTicks = 500000000;  // 5 s of the 100 MHz realtime clock

// Watchdog limit of a launch's bounded waits: 5 s, or STENCIL_WATCHDOG_US
// microseconds when that variable is set (tests shorten it to force expiry).
int64_t timeout_ticks() {
  const char* v = std::getenv("STENCIL_WATCHDOG_US");
  if (v && *v) {
    char* end = nullptr;
    const long long us = std::strtoll(v, &end, 10);
    if (end != v && us >= 0) return (int64_t)us * 100;  // 100 ticks per microsecond
  }
  return kTimeoutTicks;
}
// Batch tiles are longer than single-grid ones (fewer warm-up rows per tile),
// but a job's passes run one after another, so a tile also bounds how fast
// a long job can finish: measured on the 128-grid batch, 512 rows and 128
// planes are the best of {128, 256, 512, 1024} x {32, 64, 128, 256} (FP64 3D
// tiles of 256 planes make the longest jobs' pass chain the critical path).
constexpr int kBatchSeg2D = 512;              // rows per 2D batch tile
constexpr int kBatchSeg3D = 128;              // planes per 3D batch tile
// Tiles of the serving loop's rounds: a round runs a few passes of every
// active request, so shorter tiles keep rounds, and latency, short.
constexpr int kServeSeg2D = 256;
constexpr int kServeSeg3D = 64;

// Report word of a (device, stream): every launch on the stream has its own
// error word, zeroed with its control block, which its kernels set when a
// bounded wait expires; a small kernel after the launch ORs it into the
// stream's report word, which only stencil_sync reads and clears. So an
// expiry never leaks into another launch's waits, and each stream reports
// its own.
unsigned int* report_word(hipStream_t s) {
  static std::mutex mu;
  static std::map<std::pair<int, hipStream_t>, unsigned int*> words;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  const auto key = std::make_pair(dev, s);
  auto it = words.find(key);
  if (it != words.end()) return it->second;
  unsigned int* w = nullptr;
  if (hipMalloc(&w, 256) != hipSuccess) return nullptr;
  if (hipMemset(w, 0, 256) != hipSuccess) return nullptr;
  words[key] = w;
  return w;
}

// Pinned host staging for the control block of a batch, per device. Copies
// from pinned memory go by DMA; pageable ones go through staging kernels.
// The buffer is reused: a new upload waits (on the host) until the previous
// one has left it.
struct ControlStaging {
  std::mutex mu;
  void* buf = nullptr;
  size_t cap = 0;
  hipEvent_t done = nullptr;
  bool pending = false;
};

ControlStaging* control_staging() {
  static std::mutex mu;
  static std::map<int, ControlStaging*> per_device;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  auto it = per_device.find(dev);
  if (it != per_device.end()) return it->second;
  ControlStaging* cs = new ControlStaging();
  if (hipEventCreateWithFlags(&cs->done, hipEventDisableTiming) != hipSuccess) {
    delete cs;
    return nullptr;
  }
  per_device[dev] = cs;
  return cs;
}

// Upload `bytes` from `src` to device `dst` on s through the staging buffer
// (pageable copy if pinned memory is not available).
hipError_t upload_control(void* dst, const void* src, size_t bytes, hipStream_t s) {
  ControlStaging* cs = control_staging();
  if (!cs) return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
  std::lock_guard<std::mutex> lock(cs->mu);
  if (cs->pending) {
    (void)hipEventSynchronize(cs->done);
    cs->pending = false;
  }
  if (cs->cap < bytes) {
    if (cs->buf) (void)hipHostFree(cs->buf);
    cs->buf = nullptr;
    cs->cap = 0;
    const size_t want = std::max(bytes * 2, (size_t)1 << 20);
    if (hipHostMalloc(&cs->buf, want, hipHostMallocDefault) == hipSuccess) cs->cap = want;
  }
  if (!cs->buf) return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
  std::memcpy(cs->buf, src, bytes);
  hipError_t e = hipMemcpyAsync(dst, cs->buf, bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && hipEventRecord(cs->done, s) == hipSuccess) cs->pending = true;
  return e;
}

// Pinned host word per device for reading the error word back by DMA.
struct PinnedWord {
  std::mutex mu;
  unsigned int* p = nullptr;
};

PinnedWord* pinned_word() {
  static std::mutex mu;
  static std::map<int, PinnedWord*> per_device;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  auto it = per_device.find(dev);
  if (it != per_device.end()) return it->second;
  PinnedWord* w = new PinnedWord();
  if (hipHostMalloc((void**)&w->p, 256, hipHostMallocDefault) != hipSuccess) {
    delete w;
    return nullptr;
  }
  per_device[dev] = w;
  return w;
}

struct Group {
  int dtype;
  bool aux = false;       // runs on the auxiliary batch kernel
  std::vector<int> jobs;  // indices into the batch
};
constexpr int kAuxGroup = 2;  // groups: kF32, kF64, then the FP64 auxiliary group

// Work-list items of one pass: a 3D tile, or up to four 2D wave tiles.
int64_t items_per_pass(const stencil_plan_s* p) { return worklist::items_per_pass(p->ndim, p->tiles); }

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Work list of a group (worklist::build): every pass of a job follows its
// previous pass.
void build_worklist(const std::vector<stencil_plan_s*>& plans, const std::vector<int>& members,
                    std::vector<int32_t>& cj, std::vector<int32_t>& cp, std::vector<int64_t>& cf) {
  std::vector<worklist::JobShape> shapes;
  for (int i : members) shapes.push_back({(int32_t)plans[i]->pass_depth.size(), items_per_pass(plans[i])});
  worklist::build(shapes, cj, cp, cf);
}

template <typename Real>
BatchJob<Real> make_job(const stencil_plan_s* p, const void* in, void* out, void* ws) {
  BatchJob<Real> J;
  std::memset(&J, 0, sizeof(J));
  J.in = in;
  J.out = out;
  J.ws = ws;
  J.variant = batch_variant(p->ndim, p->r, p->pattern);
  J.tiles = p->tiles;
  J.npass = (int32_t)p->pass_depth.size();
  J.depth = p->pass_depth.front();
  J.depth_last = p->pass_depth.back();
  J.P = p->ext[2];
  J.Qy = p->ext[1];
  J.Qz = p->ext[0];
  J.seg_len = p->seg_len;
  if (p->ndim == 2) {
    J.strips = p->strips;
    J.hl = p->hl;
    J.seg_len_e = p->seg_len_e;
    J.edge_tiles = p->edge_tiles;
  } else {
    J.sx = p->sx;
    J.sy = p->sy;
    J.hx = p->hx;
    J.hy = p->hy;
  }
  const size_t nw = std::min(p->coeffs.size(), sizeof(J.w) / sizeof(J.w[0]));
  for (size_t i = 0; i < nw; ++i) J.w[i] = (Real)p->coeffs[i];
  return J;
}

}  // namespace

namespace stencil_impl {

// Runs prepared plans (not owned; NULL entries are skipped) from ins[i] to
// outs[i] on stream s: blocked plans in one persistent launch per dtype, the
// others with their plain kernels. wsg[i], when not NULL, is the caller's
// workspace for plan i; the rest of the workspace and control memory is one
// stream-ordered allocation (from `pool`, else the device's default pool)
// released on s.
stencil_status batch_run(const std::vector<stencil_plan_s*>& plans, const std::vector<const void*>& ins,
                         const std::vector<void*>& outs, const std::vector<void*>& wsg, hipStream_t s,
                         hipMemPool_t pool) {
  const int n = (int)plans.size();
  // groups of blocked jobs by dtype (the fused kernel), FP64 jobs of the
  // auxiliary kernel's variants; everything else runs alone
  Group groups[3];
  groups[kF32].dtype = kF32;
  groups[kF64].dtype = kF64;
  groups[kAuxGroup].dtype = kF64;
  groups[kAuxGroup].aux = true;
  std::vector<int> alone;
  // a persistent single-grid plan runs on its variant's own persistent kernel
  int single_variant = -1;
  if (n == 1 && plans[0] && plans[0]->persistent) {
    stencil_plan_s* p = plans[0];
    const int dt = p->dtype == STENCIL_F64 ? kF64 : kF32;
    single_variant = batch_variant(p->ndim, p->r, p->pattern);
    groups[dt].jobs.push_back(0);
  }
  for (int i = 0; i < n && single_variant < 0; ++i) {
    stencil_plan_s* p = plans[i];
    if (!p) continue;
    const int dt = p->dtype == STENCIL_F64 ? kF64 : kF32;
    const bool blocked = p->scheme == STENCIL_SCHEME_BLOCKED_2D || p->scheme == STENCIL_SCHEME_BLOCKED_3D;
    if (blocked && p->depth <= batch_max_depth(dt, p->ndim, p->r, p->pattern))
      groups[dt].jobs.push_back(i);
    else if (blocked && dt == kF64 && p->depth <= batch_aux_depth(dt, p->ndim, p->r, p->pattern))
      groups[kAuxGroup].jobs.push_back(i);
    else
      alone.push_back(i);
  }

  // device memory: workspaces, then per-group control blocks, then frame-copy lists
  char* dev = nullptr;
  std::vector<size_t> ws_off(n, 0);
  size_t total = 0;
  for (int i = 0; i < n; ++i) {
    if (!plans[i] || plans[i]->workspace == 0 || wsg[i]) continue;
    ws_off[i] = total;
    total = align256(total + plans[i]->workspace);
  }
  auto ws_of = [&](int i) -> void* {
    if (!plans[i]->workspace) return nullptr;
    return wsg[i] ? wsg[i] : (void*)(dev + ws_off[i]);
  };
  struct GroupMem {
    size_t jobs_off = 0, cj_off = 0, cp_off = 0, cf_off = 0, cursor_off = 0, done_off = 0;
    std::vector<int32_t> cj, cp;
    std::vector<int64_t> cf;
    int64_t hq_stride = 0;  // LDS halo elements per wave (2D jobs)
    size_t lds = 0;
  };
  GroupMem gmem[3];
  for (int gi = 0; gi < 3; ++gi) {
    Group& g = groups[gi];
    if (g.jobs.empty()) continue;
    const int d = g.dtype;
    GroupMem& m = gmem[gi];
    build_worklist(plans, g.jobs, m.cj, m.cp, m.cf);
    const size_t job_sz = d == kF64 ? sizeof(BatchJob<double>) : sizeof(BatchJob<float>);
    const size_t elem = d == kF64 ? 8 : 4;
    m.jobs_off = total;
    total = align256(total + job_sz * g.jobs.size());
    m.cj_off = total;
    total = align256(total + 4 * m.cj.size());
    m.cp_off = total;
    total = align256(total + 4 * m.cp.size());
    m.cf_off = total;
    total = align256(total + 8 * m.cf.size());
    m.cursor_off = total;
    total = align256(total + 8);
    m.done_off = total;
    total = align256(total + 4 * g.jobs.size());
    for (int i : g.jobs) {
      const stencil_plan_s* p = plans[i];
      if (p->ndim == 2) m.hq_stride = std::max<int64_t>(m.hq_stride, (int64_t)p->hq_rows * 2 * p->r);
      else m.lds = std::max(m.lds, batch_lds_3d(d, p->r, p->pattern));
    }
    m.lds = std::max(m.lds, (size_t)(4 * m.hq_stride) * elem);
  }
  // this launch's own error word (zeroed with the control block)
  const size_t err_off = total;
  total = align256(total + sizeof(unsigned int));
  std::vector<FrameCopyJob> frames[2];  // per dtype
  for (int gi = 0; gi < 3; ++gi)
    for (int i : groups[gi].jobs) {
      const int d = groups[gi].dtype;
      const stencil_plan_s* p = plans[i];
      FrameCopyJob f;
      std::memset(&f, 0, sizeof(f));
      f.src = ins[i];
      for (int k = 0; k < 3; ++k) {
        f.ext[k] = p->ext[k];
        f.r[k] = p->rad[k];
      }
      f.dst = outs[i];
      frames[d].push_back(f);
      if (p->workspace) {
        f.dst = nullptr;  // filled once the block address is known
        frames[d].push_back(f);
      }
    }
  size_t frames_off[2];
  for (int d = 0; d < 2; ++d) {
    frames_off[d] = total;
    total = align256(total + sizeof(FrameCopyJob) * frames[d].size());
  }
  for (int gi = 0; gi < 3; ++gi)
    if (gmem[gi].lds > (size_t)160 * 1024) {
      return fail(STENCIL_ERR_UNSUPPORTED, "batch needs %zu bytes of LDS per workgroup", gmem[gi].lds);
    }

  if (total) {
    hipError_t e = pool ? hipMallocFromPoolAsync((void**)&dev, total, pool, s) : hipMallocAsync((void**)&dev, total, s);
    if (e != hipSuccess) {
      return fail(STENCIL_ERR_NOMEM, "batch allocation of %zu bytes failed: %s", total,
                  hipGetErrorString(e));
    }
  }
  unsigned int* report = report_word(s);
  if (!report) {
    if (dev) hipFreeAsync(dev, s);
    return fail(STENCIL_ERR_NOMEM, "device error word allocation failed");
  }
  unsigned int* err = (unsigned int*)(dev + err_off);

  // host image of the control region (everything after the workspaces is
  // small); counters start at zero
  size_t ctl_lo = std::min(total, err_off);
  for (int gi = 0; gi < 3; ++gi)
    if (!groups[gi].jobs.empty()) ctl_lo = std::min(ctl_lo, gmem[gi].jobs_off);
  for (int d = 0; d < 2; ++d) ctl_lo = std::min(ctl_lo, frames_off[d]);
  std::vector<char> img(total - ctl_lo, 0);
  auto put = [&](size_t off, const void* src, size_t bytes) {
    if (bytes) std::memcpy(img.data() + (off - ctl_lo), src, bytes);
  };
  for (int gi = 0; gi < 3; ++gi) {
    Group& g = groups[gi];
    GroupMem& m = gmem[gi];
    const int d = g.dtype;
    for (size_t local = 0; local < g.jobs.size(); ++local) {
      const int i = g.jobs[local];
      const stencil_plan_s* p = plans[i];
      void* ws = ws_of(i);
      if (d == kF64) {
        const BatchJob<double> J = make_job<double>(p, ins[i], outs[i], ws);
        put(m.jobs_off + local * sizeof(J), &J, sizeof(J));
      } else {
        const BatchJob<float> J = make_job<float>(p, ins[i], outs[i], ws);
        put(m.jobs_off + local * sizeof(J), &J, sizeof(J));
      }
    }
    if (g.jobs.empty()) continue;
    put(m.cj_off, m.cj.data(), 4 * m.cj.size());
    put(m.cp_off, m.cp.data(), 4 * m.cp.size());
    put(m.cf_off, m.cf.data(), 8 * m.cf.size());
  }
  {
    // second entry of a pair targets the job's workspace (same order as above)
    size_t k[2] = {0, 0};
    for (int gi = 0; gi < 3; ++gi) {
      const int d = groups[gi].dtype;
      for (int i : groups[gi].jobs) {
        ++k[d];  // the `out` entry
        if (plans[i]->workspace) frames[d][k[d]++].dst = ws_of(i);
      }
    }
    for (int d = 0; d < 2; ++d)
      put(frames_off[d], frames[d].data(), sizeof(FrameCopyJob) * frames[d].size());
  }
  hipError_t e = hipSuccess;
  if (!img.empty()) e = upload_control(dev + ctl_lo, img.data(), img.size(), s);
  stencil_status st = STENCIL_OK;
  if (e != hipSuccess) st = hip_fail(e, "batch control upload");

  DeviceInfo di = device_info();
  const int cus = di.ok ? di.cus : 256;
  for (int d = 0; d < 2 && st == STENCIL_OK; ++d) {
    e = frame_copy_batch_launch(d, (const FrameCopyJob*)(dev + frames_off[d]), (int)frames[d].size(), s);
    if (e != hipSuccess) st = hip_fail(e, "batch halo copy");
  }
  for (int gi = 0; gi < 3 && st == STENCIL_OK; ++gi) {
    Group& g = groups[gi];
    if (g.jobs.empty()) continue;
    GroupMem& m = gmem[gi];
    const int d = g.dtype;
    BatchQueue q;
    q.chunk_job = (const int32_t*)(dev + m.cj_off);
    q.chunk_pass = (const int32_t*)(dev + m.cp_off);
    q.chunk_first = (const int64_t*)(dev + m.cf_off);
    q.nchunks = (int32_t)m.cj.size();
    q.nitems = m.cf.back();
    q.cursor = (unsigned long long*)(dev + m.cursor_off);
    q.done = (unsigned int*)(dev + m.done_off);
    q.err = err;
    q.timeout_ticks = timeout_ticks();
    // one workgroup per CU, never more than there are items
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(cus, q.nitems));
    if (d == kF64) {
      BatchParams<double> prm{(const BatchJob<double>*)(dev + m.jobs_off), q, (int32_t)m.hq_stride};
      e = single_variant >= 0 ? batch_launch_single(d, single_variant, &prm, grid, m.lds, s)
                              : batch_launch(d, &prm, grid, m.lds, s, g.aux);
    } else {
      BatchParams<float> prm{(const BatchJob<float>*)(dev + m.jobs_off), q, (int32_t)m.hq_stride};
      e = single_variant >= 0 ? batch_launch_single(d, single_variant, &prm, grid, m.lds, s)
                              : batch_launch(d, &prm, grid, m.lds, s);
    }
    if (e != hipSuccess) st = hip_fail(e, "batch launch");
  }
  // the launches' expiries go to the stream's report word
  if (st == STENCIL_OK) {
    e = error_fold_launch(err, report, s);
    if (e != hipSuccess) st = hip_fail(e, "batch error report");
  }
  // jobs without a blocked variant: the plain path, workspace from the block
  for (int i : alone) {
    if (st != STENCIL_OK) break;
    st = stencil_execute(plans[i], ins[i], outs[i], ws_of(i), s);
  }
  if (dev) {
    e = hipFreeAsync(dev, s);
    if (e != hipSuccess && st == STENCIL_OK) st = hip_fail(e, "batch release");
  }
  return st;
}

// Plans one job of a batch (host only): the caller's depth, else the
// autotuner's batched depth for its stencil class and size, else the model's,
// on uniform tiles of segments seg2d / seg3d rows or planes; blocked plans are
// capped at the fused kernel's depth for their variant, and a job with no
// batched variant gets the single-grid planner's own plan (it runs alone).
stencil_status plan_batch_job(const stencil_job& j, int seg2d, int seg3d, stencil_plan_s** out) {
  *out = nullptr;
  stencil_tuning hint;
  std::memset(&hint, 0, sizeof(hint));
  hint.depth = j.depth;
  hint.tile[0] = j.shape.ndim == 2 ? seg2d : seg3d;
  // the jobs share the wave slots; the fused kernel runs overlapped tiles
  hint.flags = STENCIL_FLAG_UNIFORM_TILES | STENCIL_FLAG_OVERLAPPED_TILING;
  stencil_plan_t pl = nullptr;
  stencil_status st = stencil_plan(&pl, j.coeffs, j.radius, &j.shape, j.dtype, j.T, &hint);
  int tuned_depth = 0, tuned_seg = 0;
  if (st == STENCIL_OK && j.depth <= 0 && tune_lookup_plan(pl, true, &tuned_depth, &tuned_seg) &&
      tuned_depth != pl->depth) {
    // the autotuner's depth for batched tiles of this stencil class and size
    stencil_plan_destroy(pl);
    pl = nullptr;
    hint.depth = tuned_depth;
    st = stencil_plan(&pl, j.coeffs, j.radius, &j.shape, j.dtype, j.T, &hint);
  }
  if (st == STENCIL_OK && (pl->scheme == STENCIL_SCHEME_BLOCKED_2D || pl->scheme == STENCIL_SCHEME_BLOCKED_3D)) {
    // the fused batch kernel's own depth limit for this variant
    const int dt = pl->dtype == STENCIL_F64 ? kF64 : kF32;
    int cap = batch_max_depth(dt, pl->ndim, pl->r, pl->pattern);
    if (cap == 0) cap = batch_aux_depth(dt, pl->ndim, pl->r, pl->pattern);
    if (cap >= 1 && pl->depth > cap) {
      stencil_plan_destroy(pl);
      pl = nullptr;
      hint.depth = cap;
      st = stencil_plan(&pl, j.coeffs, j.radius, &j.shape, j.dtype, j.T, &hint);
    } else if (cap == 0) {
      // no batched variant: the job runs alone after the persistent launch,
      // with the single-grid planner's own segments (enough tiles to fill
      // the device on its own, unlike the batch's long segments)
      stencil_plan_destroy(pl);
      pl = nullptr;
      hint.tile[0] = 0;
      hint.flags = 0;
      st = stencil_plan(&pl, j.coeffs, j.radius, &j.shape, j.dtype, j.T, &hint);
    }
  }
  if (st == STENCIL_OK) *out = pl;
  return st;
}

stencil_status batch_submit_tiles(const stencil_job* jobs, int32_t n, void* stream,
                                  stencil_status* per_job_status, int seg2d, int seg3d, hipMemPool_t pool) {
  if (!jobs || n <= 0) return fail(STENCIL_ERR_INVALID, "no jobs");
  hipStream_t s = (hipStream_t)stream;
  std::vector<stencil_status> status(n, STENCIL_OK);
  std::vector<stencil_plan_s*> plans(n, nullptr);

  // plan every job (host only)
  for (int i = 0; i < n; ++i) {
    const stencil_job& j = jobs[i];
    if (!j.in || !j.out) {
      status[i] = fail(STENCIL_ERR_INVALID, "job %d: in/out is NULL", i);
      continue;
    }
    stencil_plan_t pl = nullptr;
    status[i] = plan_batch_job(j, seg2d, seg3d, &pl);
    if (status[i] == STENCIL_OK) {
      const size_t bytes = (size_t)pl->padded_elems * pl->elem;
      const char* a = (const char*)j.in;
      const char* b = (const char*)j.out;
      if (a < b + bytes && b < a + bytes) {
        status[i] = fail(STENCIL_ERR_ALIAS, "job %d: in and out overlap", i);
        stencil_plan_destroy(pl);
        pl = nullptr;
      }
    }
    plans[i] = pl;
  }
  // no two valid jobs may share memory
  for (int i = 0; i < n; ++i) {
    if (!plans[i]) continue;
    const size_t bi = (size_t)plans[i]->padded_elems * plans[i]->elem;
    for (int k = i + 1; k < n; ++k) {
      if (!plans[k]) continue;
      const size_t bk = (size_t)plans[k]->padded_elems * plans[k]->elem;
      const char* ri[2] = {(const char*)jobs[i].in, (const char*)jobs[i].out};
      const char* rk[2] = {(const char*)jobs[k].in, (const char*)jobs[k].out};
      for (int u = 0; u < 2; ++u)
        for (int v = 0; v < 2; ++v) {
          if (u == 0 && v == 0) continue;  // two jobs may read the same input
          if (ri[u] < rk[v] + bk && rk[v] < ri[u] + bi) {
            for (auto* p : plans) stencil_plan_destroy(p);
            return fail(STENCIL_ERR_ALIAS, "jobs %d and %d share memory", i, k);
          }
        }
    }
  }
  if (per_job_status)
    for (int i = 0; i < n; ++i) per_job_status[i] = status[i];
  int valid = 0;
  for (int i = 0; i < n; ++i) valid += plans[i] != nullptr;
  if (!valid) return fail(STENCIL_ERR_INVALID, "no valid job in the batch");

  std::vector<const void*> ins(n);
  std::vector<void*> outs(n), wsg(n, nullptr);
  for (int i = 0; i < n; ++i) {
    ins[i] = jobs[i].in;
    outs[i] = jobs[i].out;
  }
  stencil_status st = batch_run(plans, ins, outs, wsg, s, pool);
  for (auto* p : plans) stencil_plan_destroy(p);
  return st;
}

stencil_status batch_submit_planned(const std::vector<const stencil_plan_s*>& plans,
                                    const std::vector<int64_t>& steps, const std::vector<const void*>& ins,
                                    const std::vector<void*>& outs, hipStream_t s, hipMemPool_t pool) {
  const size_t n = plans.size();
  std::vector<stencil_plan_s> copies(n);
  std::vector<stencil_plan_s*> run(n, nullptr);
  for (size_t i = 0; i < n; ++i) {
    if (!plans[i]) continue;
    copies[i] = *plans[i];
    plan_schedule(&copies[i], steps[i]);
    run[i] = &copies[i];
  }
  std::vector<void*> wsg(n, nullptr);
  return batch_run(run, ins, outs, wsg, s, pool);
}

int serve_seg_2d() { return kServeSeg2D; }
int serve_seg_3d() { return kServeSeg3D; }

}  // namespace stencil_impl

namespace stencil_impl {
int64_t watchdog_ticks() { return timeout_ticks(); }
unsigned int* stream_report_word(hipStream_t s) { return report_word(s); }
}  // namespace stencil_impl

extern "C" {

stencil_status stencil_batch_submit(const stencil_job* jobs, int32_t n, void* stream,
                                    stencil_status* per_job_status) {
  return batch_submit_tiles(jobs, n, stream, per_job_status, kBatchSeg2D, kBatchSeg3D);
}

stencil_status stencil_batch_describe(const stencil_job* job, stencil_plan_info* info) {
  if (!job || !info) return fail(STENCIL_ERR_INVALID, "NULL argument");
  stencil_plan_s* pl = nullptr;
  stencil_status st = plan_batch_job(*job, kBatchSeg2D, kBatchSeg3D, &pl);
  if (st != STENCIL_OK) return st;
  st = stencil_plan_describe(pl, info);
  stencil_plan_destroy(pl);
  return st;
}

stencil_status stencil_probe_grid_sync(int32_t rounds, void* stream, double* seconds_per_sync) {
  if (!seconds_per_sync || rounds < 1 || rounds > 1000000)
    return fail(STENCIL_ERR_INVALID, "rounds in [1, 1e6] and a result pointer");
  *seconds_per_sync = 0;
  hipStream_t s = (hipStream_t)stream;
  unsigned int* report = report_word(s);
  if (!report) return fail(STENCIL_ERR_NOMEM, "device error word allocation failed");
  DeviceInfo di = device_info();
  if (!di.ok) return fail(STENCIL_ERR_DEVICE, "no device");
  unsigned int* ctr = nullptr;
  hipError_t e = hipMallocAsync((void**)&ctr, 512, s);
  if (e != hipSuccess) return hip_fail(e, "probe counter");
  unsigned int* err = ctr + 64;  // the probe's own error word
  hipEvent_t e0 = nullptr, e1 = nullptr;
  stencil_status st = STENCIL_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = fail(STENCIL_ERR_DEVICE, "events");
  // one launch to warm up, then the timed one
  for (int rep = 0; rep < 2 && st == STENCIL_OK; ++rep) {
    e = hipMemsetAsync(ctr, 0, 512, s);
    if (e == hipSuccess && rep == 1) e = hipEventRecord(e0, s);
    if (e == hipSuccess) e = grid_sync_probe_launch(ctr, err, rounds, di.cus, timeout_ticks(), s);
    if (e == hipSuccess && rep == 1) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = error_fold_launch(err, report, s);
    if (e != hipSuccess) st = hip_fail(e, "grid sync probe");
  }
  if (st == STENCIL_OK) st = stencil_sync(stream);
  if (st == STENCIL_OK) {
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    *seconds_per_sync = ms * 1e-3 / rounds;
  }
  (void)hipFreeAsync(ctr, s);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return st;
}

stencil_status stencil_sync(void* stream) {
  hipStream_t s = (hipStream_t)stream;
  unsigned int* err = report_word(s);
  PinnedWord* pw = err ? pinned_word() : nullptr;
  unsigned int h = 0;
  hipError_t e;
  if (pw) {
    // the read rides on the stream: one synchronisation covers both
    std::lock_guard<std::mutex> lock(pw->mu);
    e = hipMemcpyAsync(pw->p, err, sizeof(unsigned int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "stream synchronize");
    h = *pw->p;
  } else {
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "stream synchronize");
    if (err) {
      e = hipMemcpy(&h, err, sizeof(h), hipMemcpyDeviceToHost);
      if (e != hipSuccess) return hip_fail(e, "error word read");
    }
  }
  if (worklist::status_of_report(h) != STENCIL_OK) {
    e = hipMemsetAsync(err, 0, sizeof(unsigned int), s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "error word reset");
    return fail(worklist::status_of_report(h), "a bounded device wait expired; affected results are undefined");
  }
  return STENCIL_OK;
}

}  // extern "C"
