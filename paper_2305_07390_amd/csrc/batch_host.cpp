// Host side of batched execution (stencil_batch_submit, stencil_sync).
//
// Every job is planned like a single grid, with longer tiles so that small
// grids are not cut into slivers. Jobs with a blocked variant are grouped by
// kernel variant (dimension, dtype, radius, pattern); each group becomes one
// persistent launch over a work list of (job, pass) chunks ordered by the
// fraction of the job completed after the chunk, so that long and short jobs
// progress together and finish together. Device memory for workspaces, job
// descriptors, the work list and counters is one stream-ordered allocation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "launch.hpp"
#include "plan.hpp"

using namespace stencil_impl;

namespace {

constexpr int64_t kTimeoutTicks = 500000000;  // 5 s of the 100 MHz realtime clock
constexpr int kBatchSeg2D = 256;              // rows per 2D batch tile
constexpr int kBatchSeg3D = 64;               // planes per 3D batch tile

// Per-device error word shared by all batch launches on that device.
unsigned int* device_error_word() {
  static std::mutex mu;
  static std::map<int, unsigned int*> words;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  auto it = words.find(dev);
  if (it != words.end()) return it->second;
  unsigned int* w = nullptr;
  if (hipMalloc(&w, 256) != hipSuccess) return nullptr;
  if (hipMemset(w, 0, 256) != hipSuccess) return nullptr;
  words[dev] = w;
  return w;
}

struct Group {
  int ndim, dtype, r, pattern;
  std::vector<int> jobs;  // indices into the batch
};

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Work list of a group: chunks (job, pass) in order of progress after the
// chunk; ties by job index. Every pass of a job follows its previous pass.
void build_worklist(const std::vector<stencil_plan_s*>& plans, const std::vector<int>& members,
                    std::vector<int32_t>& cj, std::vector<int32_t>& cp, std::vector<int64_t>& cf) {
  struct C { double key; int job, pass; };
  std::vector<C> chunks;
  for (int local = 0; local < (int)members.size(); ++local) {
    const stencil_plan_s* p = plans[members[local]];
    const int np = (int)p->pass_depth.size();
    for (int k = 0; k < np; ++k) chunks.push_back({(double)(k + 1) / np, local, k});
  }
  std::stable_sort(chunks.begin(), chunks.end(), [](const C& a, const C& b) {
    if (a.key != b.key) return a.key < b.key;
    if (a.job != b.job) return a.job < b.job;
    return a.pass < b.pass;
  });
  cj.clear();
  cp.clear();
  cf.assign(1, 0);
  for (const C& c : chunks) {
    cj.push_back(c.job);
    cp.push_back(c.pass);
    cf.push_back(cf.back() + plans[members[c.job]]->tiles);
  }
}

template <typename Job, typename Real>
void fill_common(Job& J, const stencil_plan_s* p, const void* in, void* out, void* ws) {
  J.in = in;
  J.out = out;
  J.ws = ws;
  J.npass = (int32_t)p->pass_depth.size();
  J.depth = p->pass_depth.front();
  J.depth_last = p->pass_depth.back();
  const size_t nw = std::min(p->coeffs.size(), sizeof(J.w) / sizeof(J.w[0]));
  for (size_t i = 0; i < nw; ++i) J.w[i] = (Real)p->coeffs[i];
}

}  // namespace

extern "C" {

stencil_status stencil_batch_submit(const stencil_job* jobs, int32_t n, void* stream,
                                    stencil_status* per_job_status) {
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
    stencil_tuning hint;
    std::memset(&hint, 0, sizeof(hint));
    hint.depth = j.depth;
    hint.tile[0] = j.shape.ndim == 2 ? kBatchSeg2D : kBatchSeg3D;
    stencil_plan_t pl = nullptr;
    status[i] = stencil_plan(&pl, j.coeffs, j.radius, &j.shape, j.dtype, j.T, &hint);
    int tuned_depth = 0, tuned_seg = 0;
    if (status[i] == STENCIL_OK && j.depth <= 0 &&
        tune_lookup_plan(pl, true, &tuned_depth, &tuned_seg) && tuned_depth != pl->depth) {
      // the autotuner's depth for batched tiles of this stencil class and size
      stencil_plan_destroy(pl);
      pl = nullptr;
      hint.depth = tuned_depth;
      status[i] = stencil_plan(&pl, j.coeffs, j.radius, &j.shape, j.dtype, j.T, &hint);
    }
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

  // groups of blocked jobs by kernel variant; everything else runs alone
  std::map<std::tuple<int, int, int, int>, Group> groups;
  std::vector<int> alone;
  for (int i = 0; i < n; ++i) {
    stencil_plan_s* p = plans[i];
    if (!p) continue;
    if (p->scheme == STENCIL_SCHEME_BLOCKED_2D || p->scheme == STENCIL_SCHEME_BLOCKED_3D) {
      const int dt = p->dtype == STENCIL_F64 ? kF64 : kF32;
      auto key = std::make_tuple(p->ndim, dt, p->r, p->pattern);
      Group& g = groups[key];
      g.ndim = p->ndim;
      g.dtype = dt;
      g.r = p->r;
      g.pattern = p->pattern;
      g.jobs.push_back(i);
    } else {
      alone.push_back(i);
    }
  }

  // device memory: workspaces, then per-group control blocks, then frame-copy lists
  std::vector<size_t> ws_off(n, 0);
  size_t total = 0;
  for (int i = 0; i < n; ++i) {
    if (!plans[i] || plans[i]->workspace == 0) continue;
    ws_off[i] = total;
    total = align256(total + plans[i]->workspace);
  }
  struct GroupMem {
    size_t jobs_off, cj_off, cp_off, cf_off, cursor_off, done_off;
    std::vector<int32_t> cj, cp;
    std::vector<int64_t> cf;
    int hq_rows = 0;
  };
  std::vector<GroupMem> gmem;
  std::vector<Group*> glist;
  for (auto& kv : groups) {
    Group& g = kv.second;
    GroupMem m;
    build_worklist(plans, g.jobs, m.cj, m.cp, m.cf);
    const size_t job_sz = g.ndim == 2 ? (g.dtype == kF64 ? sizeof(BatchJob2D<double>) : sizeof(BatchJob2D<float>))
                                      : (g.dtype == kF64 ? sizeof(BatchJob3D<double>) : sizeof(BatchJob3D<float>));
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
    for (int i : g.jobs) m.hq_rows = std::max(m.hq_rows, plans[i]->hq_rows);
    gmem.push_back(std::move(m));
    glist.push_back(&g);
  }
  std::vector<FrameCopyJob> frames[2];  // per dtype
  for (auto* g : glist)
    for (int i : g->jobs) {
      const stencil_plan_s* p = plans[i];
      FrameCopyJob f;
      std::memset(&f, 0, sizeof(f));
      f.src = jobs[i].in;
      for (int d = 0; d < 3; ++d) {
        f.ext[d] = p->ext[d];
        f.r[d] = p->rad[d];
      }
      f.dst = jobs[i].out;
      frames[g->dtype].push_back(f);
      if (p->workspace) {
        f.dst = nullptr;  // filled once the block address is known
        frames[g->dtype].push_back(f);
      }
    }
  size_t frames_off[2];
  for (int d = 0; d < 2; ++d) {
    frames_off[d] = total;
    total = align256(total + sizeof(FrameCopyJob) * frames[d].size());
  }
  const size_t ctl_begin = 0;
  (void)ctl_begin;

  char* dev = nullptr;
  if (total) {
    hipError_t e = hipMallocAsync((void**)&dev, total, s);
    if (e != hipSuccess) {
      for (auto* p : plans) stencil_plan_destroy(p);
      return fail(STENCIL_ERR_NOMEM, "batch allocation of %zu bytes failed: %s", total,
                  hipGetErrorString(e));
    }
  }
  unsigned int* err = device_error_word();
  if (!err) {
    if (dev) hipFreeAsync(dev, s);
    for (auto* p : plans) stencil_plan_destroy(p);
    return fail(STENCIL_ERR_NOMEM, "device error word allocation failed");
  }

  // host image of the control region (everything after the first workspace
  // bytes is small); counters start at zero
  size_t ctl_lo = total;
  for (auto& m : gmem) ctl_lo = std::min(ctl_lo, m.jobs_off);
  for (int d = 0; d < 2; ++d) ctl_lo = std::min(ctl_lo, frames_off[d]);
  std::vector<char> img(total - ctl_lo, 0);
  auto put = [&](size_t off, const void* src, size_t bytes) {
    if (bytes) std::memcpy(img.data() + (off - ctl_lo), src, bytes);
  };
  for (size_t gi = 0; gi < glist.size(); ++gi) {
    Group& g = *glist[gi];
    GroupMem& m = gmem[gi];
    for (size_t local = 0; local < g.jobs.size(); ++local) {
      const int i = g.jobs[local];
      const stencil_plan_s* p = plans[i];
      void* ws = p->workspace ? (void*)(dev + ws_off[i]) : nullptr;
      if (g.ndim == 2) {
        auto fill2 = [&](auto* proto) {
          using J = std::remove_pointer_t<decltype(proto)>;
          J jd;
          std::memset(&jd, 0, sizeof(jd));
          using Real = std::remove_reference_t<decltype(jd.w[0])>;
          fill_common<J, Real>(jd, p, jobs[i].in, jobs[i].out, ws);
          jd.P = p->ext[2];
          jd.Q = p->ext[1];
          jd.strips = p->strips;
          jd.segs = p->segs;
          jd.seg_len = p->seg_len;
          jd.tiles = p->tiles;
          jd.hl = p->hl;
          put(m.jobs_off + local * sizeof(J), &jd, sizeof(J));
        };
        if (g.dtype == kF64) fill2((BatchJob2D<double>*)nullptr);
        else fill2((BatchJob2D<float>*)nullptr);
      } else {
        auto fill3 = [&](auto* proto) {
          using J = std::remove_pointer_t<decltype(proto)>;
          J jd;
          std::memset(&jd, 0, sizeof(jd));
          using Real = std::remove_reference_t<decltype(jd.w[0])>;
          fill_common<J, Real>(jd, p, jobs[i].in, jobs[i].out, ws);
          jd.P = p->ext[2];
          jd.Qy = p->ext[1];
          jd.Qz = p->ext[0];
          jd.sx = p->sx;
          jd.sy = p->sy;
          jd.segs = p->segs;
          jd.seg_len = p->seg_len;
          jd.tiles = p->tiles;
          jd.hx = p->hx;
          jd.hy = p->hy;
          put(m.jobs_off + local * sizeof(J), &jd, sizeof(J));
        };
        if (g.dtype == kF64) fill3((BatchJob3D<double>*)nullptr);
        else fill3((BatchJob3D<float>*)nullptr);
      }
    }
    put(m.cj_off, m.cj.data(), 4 * m.cj.size());
    put(m.cp_off, m.cp.data(), 4 * m.cp.size());
    put(m.cf_off, m.cf.data(), 8 * m.cf.size());
  }
  for (int d = 0; d < 2; ++d) {
    // second entry of a pair targets the job's workspace
    size_t k = 0;
    for (auto* g : glist) {
      if (g->dtype != d) continue;
      for (int i : g->jobs) {
        ++k;  // the `out` entry
        if (plans[i]->workspace) frames[d][k++].dst = dev + ws_off[i];
      }
    }
    put(frames_off[d], frames[d].data(), sizeof(FrameCopyJob) * frames[d].size());
  }
  hipError_t e = hipSuccess;
  if (!img.empty()) e = hipMemcpyAsync(dev + ctl_lo, img.data(), img.size(), hipMemcpyHostToDevice, s);
  stencil_status st = STENCIL_OK;
  if (e != hipSuccess) st = hip_fail(e, "batch control upload");

  DeviceInfo di = device_info();
  const int cus = di.ok ? di.cus : 256;
  for (int d = 0; d < 2 && st == STENCIL_OK; ++d) {
    e = frame_copy_batch_launch(d, (const FrameCopyJob*)(dev + frames_off[d]), (int)frames[d].size(), s);
    if (e != hipSuccess) st = hip_fail(e, "batch halo copy");
  }
  for (size_t gi = 0; gi < glist.size() && st == STENCIL_OK; ++gi) {
    Group& g = *glist[gi];
    GroupMem& m = gmem[gi];
    BatchQueue q;
    q.chunk_job = (const int32_t*)(dev + m.cj_off);
    q.chunk_pass = (const int32_t*)(dev + m.cp_off);
    q.chunk_first = (const int64_t*)(dev + m.cf_off);
    q.nchunks = (int32_t)m.cj.size();
    q.nitems = m.cf.back();
    q.cursor = (unsigned long long*)(dev + m.cursor_off);
    q.done = (unsigned int*)(dev + m.done_off);
    q.err = err;
    q.timeout_ticks = kTimeoutTicks;
    if (g.ndim == 2) {
      const size_t elem = g.dtype == kF64 ? 8 : 4;
      const size_t lds = (size_t)4 * m.hq_rows * 2 * g.r * elem;
      if (g.dtype == kF64) {
        Batch2DParams<double> prm{(const BatchJob2D<double>*)(dev + m.jobs_off), q, m.hq_rows};
        e = tb2d_batch_launch(g.dtype, g.r, g.pattern, 0, &prm, cus, lds, s);
      } else {
        Batch2DParams<float> prm{(const BatchJob2D<float>*)(dev + m.jobs_off), q, m.hq_rows};
        e = tb2d_batch_launch(g.dtype, g.r, g.pattern, 0, &prm, cus, lds, s);
      }
    } else {
      if (g.dtype == kF64) {
        Batch3DParams<double> prm{(const BatchJob3D<double>*)(dev + m.jobs_off), q};
        e = tb3d_batch_launch(g.dtype, g.r, g.pattern, 0, &prm, cus, s);
      } else {
        Batch3DParams<float> prm{(const BatchJob3D<float>*)(dev + m.jobs_off), q};
        e = tb3d_batch_launch(g.dtype, g.r, g.pattern, 0, &prm, cus, s);
      }
    }
    if (e != hipSuccess) st = hip_fail(e, "batch launch");
  }
  // jobs without a blocked variant: the plain path, workspace from the block
  for (int i : alone) {
    if (st != STENCIL_OK) break;
    void* ws = plans[i]->workspace ? (void*)(dev + ws_off[i]) : nullptr;
    st = stencil_execute(plans[i], jobs[i].in, jobs[i].out, ws, stream);
  }
  if (dev) {
    e = hipFreeAsync(dev, s);
    if (e != hipSuccess && st == STENCIL_OK) st = hip_fail(e, "batch release");
  }
  for (auto* p : plans) stencil_plan_destroy(p);
  return st;
}

stencil_status stencil_sync(void* stream) {
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "stream synchronize");
  unsigned int* err = device_error_word();
  if (!err) return STENCIL_OK;
  unsigned int h = 0;
  e = hipMemcpy(&h, err, sizeof(h), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "error word read");
  if (h) {
    hipMemset(err, 0, sizeof(unsigned int));
    return fail(STENCIL_ERR_TIMEOUT, "a bounded device wait expired; affected results are undefined");
  }
  return STENCIL_OK;
}

}  // extern "C"
