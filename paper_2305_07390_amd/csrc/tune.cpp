// Autotuner: choose the temporal depth and the streamed segment length of a
// blocked plan by measurement, with the attainable-performance model of paper
// Section 5 pruning the candidates (Section 6.2: a depth below the one that
// moves the bound off global memory is not worth timing; Section 3.4: the
// final depth comes from an empirical search around the model's value).
//
// Results live in a process-wide cache keyed by (gfx arch, CU count, ndim,
// pattern class, radius, points, dtype, size bucket, single/batched), which can
// be saved to and merged from a small JSON file. Plans made without a hint and
// batch jobs without a depth consult the cache.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "plan.hpp"

using namespace stencil_impl;

namespace {

struct Entry {
  int depth = 0;
  int seg = 0;
  int flags = 0;  // STENCIL_FLAG_DEVICE_TILING or _OVERLAPPED_TILING for 3D plans
  double sec_per_step = 0;
  int candidates = 0;
};

std::mutex g_mu;
std::map<std::string, Entry> g_cache;

std::string arch_name(int dev) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

// Half-octave size bucket of one extent, powers of two at bucket centres;
// grids whose extents share buckets share a tuning entry.
int bucket(int64_t n) { return (int)std::lround(2.0 * std::log2((double)std::max<int64_t>(n, 1))); }

const char* pattern_name(int p) {
  return p == STENCIL_STAR ? "star" : p == STENCIL_BOX ? "box" : "general";
}

// Cache key; `pl` supplies the classification of the coefficients.
std::string make_key(const stencil_plan_s* pl, bool batched) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  const DeviceInfo di = device_info();
  char buf[256];
  const int off = 3 - pl->ndim;
  std::string b;
  for (int d = off; d < 3; ++d) {
    b += std::to_string(bucket(pl->n[d]));
    if (d < 2) b += ".";
  }
  std::snprintf(buf, sizeof(buf), "%s/%d/%dd/%s/r%d/k%d/%s/b%s/%s", arch_name(dev).c_str(),
                di.ok ? di.cus : 0, pl->ndim, pattern_name(pl->pattern), pl->r, pl->points,
                pl->dtype == STENCIL_F64 ? "f64" : "f32", b.c_str(), batched ? "batch" : "single");
  return buf;
}

// Plan for classification only (T = 1, no hint and no cache).
stencil_status probe_plan(const double* coeffs, int32_t radius, const stencil_shape* shape,
                          stencil_dtype dtype, stencil_plan_t* out) {
  stencil_tuning h;
  std::memset(&h, 0, sizeof(h));
  h.flags = STENCIL_FLAG_NO_CACHE;
  return stencil_plan(out, coeffs, radius, shape, dtype, 1, &h);
}

struct Candidate {
  int depth, seg, flags;
  double model;  // plan_model_rate of the candidate plan (cells/s of valid output)
  size_t workspace;
};

// Device buffers for timing runs.
struct Buffers {
  std::vector<void*> ptrs;
  ~Buffers() {
    for (void* p : ptrs)
      if (p) (void)hipFree(p);
  }
  void* alloc(size_t bytes) {
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    ptrs.push_back(p);
    return p;
  }
};

// Timed runs per candidate (after one untimed run); the best one counts.
constexpr int kTuneReps = 3;

// Time `fn` (enqueues on s) once untimed, then `reps` times; best seconds.
template <typename F>
stencil_status time_best(hipStream_t s, int reps, F&& fn, double* best) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return hip_fail(hipErrorUnknown, "hipEventCreate");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(hipErrorUnknown, "hipEventCreate");
  }
  stencil_status st = fn();
  *best = INFINITY;
  for (int i = 0; i < reps && st == STENCIL_OK; ++i) {
    (void)hipEventRecord(e0, s);
    st = fn();
    (void)hipEventRecord(e1, s);
    if (st != STENCIL_OK) break;
    if (hipEventSynchronize(e1) != hipSuccess) {
      st = hip_fail(hipErrorUnknown, "hipEventSynchronize");
      break;
    }
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    *best = std::min(*best, ms * 1e-3);
  }
  if (st == STENCIL_OK) st = stencil_sync(s);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

}  // namespace

namespace stencil_impl {

// Cached choice for a plan about to be made, if any (used by stencil_plan and
// stencil_batch_submit).
bool tune_lookup_plan(const stencil_plan_s* pl, bool batched, int* depth, int* seg, int* flags) {
  const std::string key = make_key(pl, batched);
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_cache.find(key);
  if (it == g_cache.end()) return false;
  *depth = it->second.depth;
  *seg = it->second.seg;
  if (flags) *flags = it->second.flags;
  return true;
}

}  // namespace stencil_impl

extern "C" {

stencil_status stencil_tune(const double* coeffs, int32_t radius, const stencil_shape* shape,
                            stencil_dtype dtype, int32_t flags, void* stream,
                            stencil_tune_result* result) {
  if (!result) return fail(STENCIL_ERR_INVALID, "result is NULL");
  std::memset(result, 0, sizeof(*result));
  stencil_plan_t base = nullptr;
  stencil_status st = probe_plan(coeffs, radius, shape, dtype, &base);
  if (st != STENCIL_OK) return st;
  const bool batched = (flags & STENCIL_TUNE_BATCH) != 0;
  const std::string key = make_key(base, batched);
  if (!(flags & STENCIL_TUNE_FORCE)) {
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
      result->depth = it->second.depth;
      result->seg_len = it->second.seg;
      result->seconds_per_step = it->second.sec_per_step;
      result->candidates = it->second.candidates;
      result->flags = it->second.flags;
      result->from_cache = 1;
      stencil_plan_destroy(base);
      return STENCIL_OK;
    }
  }
  const int scheme = base->scheme;
  const int ndim = base->ndim;
  if (scheme != STENCIL_SCHEME_BLOCKED_2D && scheme != STENCIL_SCHEME_BLOCKED_3D &&
      scheme != STENCIL_SCHEME_DEVICE_3D) {
    stencil_plan_destroy(base);
    return fail(STENCIL_ERR_UNSUPPORTED, "no blocked kernel for this stencil and shape: nothing to tune");
  }
  const int dt = dtype == STENCIL_F64 ? kF64 : kF32;

  // Candidates: every compiled depth of every applicable scheme (3D: the
  // overlapped tiles and, single grids only, device tiling), each with the
  // planner's segment for it and (single grids, overlapped tiles) half and
  // double that segment; batched tiles keep the batch segment. The model
  // (plan_model_rate with the machine parameters) prunes candidates predicted
  // below 60% of its best; measurement decides among the rest.
  std::vector<Candidate> cand;
  double best_model = 0;
  auto add = [&](int d, int seg, int fl) {
    stencil_tuning h;
    std::memset(&h, 0, sizeof(h));
    h.depth = d;
    h.tile[0] = seg;
    h.flags = STENCIL_FLAG_NO_CACHE | fl;
    stencil_plan_t p = nullptr;
    if (stencil_plan(&p, coeffs, radius, shape, dtype, 4 * (int64_t)d, &h) != STENCIL_OK) return -1;
    int got = -1;
    const bool want_dev = (fl & STENCIL_FLAG_DEVICE_TILING) != 0;
    const bool is_dev = p->scheme == STENCIL_SCHEME_DEVICE_3D;
    if (p->depth == d && p->scheme != STENCIL_SCHEME_NAIVE && want_dev == is_dev) {
      const double m = plan_model_rate(p);
      best_model = std::max(best_model, m);
      cand.push_back({d, batched ? 0 : p->seg_len, fl, m, p->workspace});
      got = p->seg_len;
    }
    stencil_plan_destroy(p);
    return got;
  };
  const int fl_ov = ndim == 3 ? STENCIL_FLAG_OVERLAPPED_TILING : 0;
  const int maxd = ndim == 2 ? tb2d_max_depth(dt, radius, base->pattern) : tb3d_max_depth(dt, radius, base->pattern);
  for (int d = 1; d <= maxd; ++d) {
    const int seg0 = add(d, 0, fl_ov);
    if (seg0 > 0 && !batched) {
      const int lo = seg0 / 2, hi = seg0 * 2;
      if (lo >= 8) add(d, lo, fl_ov);
      if (hi <= (ndim == 2 ? base->n[1] : base->n[0])) add(d, hi, fl_ov);
    }
  }
  if (ndim == 3 && !batched)
    for (int d = 1; d <= tb3d_dev_max_depth(dt, radius, base->pattern); ++d) add(d, 0, STENCIL_FLAG_DEVICE_TILING);
  stencil_plan_destroy(base);
  std::vector<Candidate> keep;
  for (const Candidate& c : cand)
    if (c.model >= 0.6 * best_model) keep.push_back(c);
  if (keep.empty()) return fail(STENCIL_ERR_UNSUPPORTED, "no candidate plan");

  hipStream_t s = (hipStream_t)stream;
  Buffers buf;
  const int64_t padded = [&] {
    int64_t e = 1;
    for (int d = 0; d < shape->ndim; ++d) e *= shape->n[d] + 2 * radius;
    return e;
  }();
  const size_t bytes = (size_t)padded * (dtype == STENCIL_F64 ? 8 : 4);
  const int64_t cells = [&] {
    int64_t c = 1;
    for (int d = 0; d < shape->ndim; ++d) c *= shape->n[d];
    return c;
  }();
  // Batched tuning fills the machine with replicas of the grid (sharing one
  // input), as a batch of many grids would.
  int replicas = 1;
  if (batched) {
    const int64_t target_cells = (int64_t)64 << 20;
    replicas = (int)std::max<int64_t>(1, std::min<int64_t>(64, target_cells / std::max<int64_t>(cells, 1)));
    while (replicas > 1 && (size_t)replicas * bytes > ((size_t)2 << 30)) --replicas;
  }
  void* in = buf.alloc(bytes);
  if (!in) return fail(STENCIL_ERR_NOMEM, "tuning buffers (%zu bytes)", bytes);
  if (hipMemsetAsync(in, 0, bytes, s) != hipSuccess) return hip_fail(hipErrorUnknown, "hipMemsetAsync");
  std::vector<void*> outs;
  for (int i = 0; i < replicas; ++i) {
    void* o = buf.alloc(bytes);
    if (!o) return fail(STENCIL_ERR_NOMEM, "tuning buffers (%zu bytes)", bytes);
    outs.push_back(o);
  }
  void* ws = nullptr;
  if (!batched) {
    size_t wbytes = bytes;
    for (const Candidate& c : keep) wbytes = std::max(wbytes, c.workspace);
    ws = buf.alloc(wbytes);
    if (!ws) return fail(STENCIL_ERR_NOMEM, "tuning workspace (%zu bytes)", wbytes);
  }

  double best_t = INFINITY;
  Candidate best = keep.front();
  int measured = 0;
  for (const Candidate& c : keep) {
    // enough passes to time about ten milliseconds of work, at least four:
    // neighbouring depths of one stencil can differ by 1-2 %, so a timing
    // needs less noise than that
    const int64_t per_pass = cells * c.depth * replicas;
    int64_t passes = std::max<int64_t>(4, (int64_t)(8.0e9 / (double)std::max<int64_t>(per_pass, 1)));
    passes = std::min<int64_t>(passes, 64);
    const int64_t Tp = passes * c.depth;
    double t = INFINITY;
    if (!batched) {
      stencil_tuning h;
      std::memset(&h, 0, sizeof(h));
      h.depth = c.depth;
      h.tile[0] = c.seg;
      h.flags = STENCIL_FLAG_NO_CACHE | c.flags;
      stencil_plan_t p = nullptr;
      st = stencil_plan(&p, coeffs, radius, shape, dtype, Tp, &h);
      if (st != STENCIL_OK) return st;
      st = time_best(s, kTuneReps, [&] { return stencil_execute(p, in, outs[0], ws, s); }, &t);
      stencil_plan_destroy(p);
    } else {
      std::vector<stencil_job> jobs(replicas);
      for (int i = 0; i < replicas; ++i) {
        stencil_job& j = jobs[i];
        std::memset(&j, 0, sizeof(j));
        j.coeffs = coeffs;
        j.radius = radius;
        j.shape = *shape;
        j.dtype = dtype;
        j.T = Tp;
        j.in = in;
        j.out = outs[i];
        j.tag = (uint64_t)i;
        j.depth = c.depth;
      }
      st = time_best(s, kTuneReps, [&] { return stencil_batch_submit(jobs.data(), replicas, s, nullptr); }, &t);
    }
    if (st != STENCIL_OK) return st;
    ++measured;
    const double sps = t / ((double)Tp * replicas);
    if (sps < best_t) {
      best_t = sps;
      best = c;
    }
  }
  Entry e;
  e.depth = best.depth;
  e.seg = best.seg;
  e.flags = best.flags;
  e.sec_per_step = best_t;
  e.candidates = measured;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    g_cache[key] = e;
  }
  result->depth = e.depth;
  result->seg_len = e.seg;
  result->seconds_per_step = e.sec_per_step;
  result->candidates = e.candidates;
  result->model_cells_per_s = best.model;
  result->flags = e.flags;
  result->from_cache = 0;
  return STENCIL_OK;
}

stencil_status stencil_tune_lookup(const double* coeffs, int32_t radius, const stencil_shape* shape,
                                   stencil_dtype dtype, int32_t flags, stencil_tuning* out,
                                   int32_t* found) {
  if (!out || !found) return fail(STENCIL_ERR_INVALID, "NULL argument");
  std::memset(out, 0, sizeof(*out));
  *found = 0;
  stencil_plan_t p = nullptr;
  stencil_status st = probe_plan(coeffs, radius, shape, dtype, &p);
  if (st != STENCIL_OK) return st;
  int depth = 0, seg = 0;
  int sflags = 0;
  if (tune_lookup_plan(p, (flags & STENCIL_TUNE_BATCH) != 0, &depth, &seg, &sflags)) {
    out->depth = depth;
    out->tile[0] = seg;
    out->flags = sflags;
    *found = 1;
  }
  stencil_plan_destroy(p);
  return STENCIL_OK;
}

stencil_status stencil_tune_cache_clear(void) {
  std::lock_guard<std::mutex> lock(g_mu);
  g_cache.clear();
  return STENCIL_OK;
}

stencil_status stencil_tune_cache_save(const char* path) {
  if (!path) return fail(STENCIL_ERR_INVALID, "path is NULL");
  std::lock_guard<std::mutex> lock(g_mu);
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(STENCIL_ERR_INVALID, "cannot write %s", path);
  std::fprintf(f, "{\n  \"version\": 1,\n  \"entries\": [");
  bool first = true;
  for (const auto& kv : g_cache) {
    std::fprintf(f, "%s\n    {\"key\": \"%s\", \"depth\": %d, \"seg\": %d, \"flags\": %d, "
                    "\"sec_per_step\": %.6e, \"candidates\": %d}",
                 first ? "" : ",", kv.first.c_str(), kv.second.depth, kv.second.seg, kv.second.flags,
                 kv.second.sec_per_step, kv.second.candidates);
    first = false;
  }
  std::fprintf(f, "\n  ]\n}\n");
  const bool ok = std::fclose(f) == 0;
  return ok ? STENCIL_OK : fail(STENCIL_ERR_INVALID, "cannot write %s", path);
}

// Reads the format written above: one object per entry with a string "key"
// and integer "depth" and "seg" (other fields optional). Merges into the cache.
stencil_status stencil_tune_cache_load(const char* path, int32_t* loaded) {
  if (!path) return fail(STENCIL_ERR_INVALID, "path is NULL");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(STENCIL_ERR_INVALID, "cannot read %s", path);
  std::string text;
  char chunk[4096];
  size_t got;
  while ((got = std::fread(chunk, 1, sizeof(chunk), f)) > 0) text.append(chunk, got);
  std::fclose(f);
  auto field_num = [](const std::string& obj, const char* name, double* v) {
    const std::string pat = std::string("\"") + name + "\"";
    size_t p = obj.find(pat);
    if (p == std::string::npos) return false;
    p = obj.find(':', p + pat.size());
    if (p == std::string::npos) return false;
    char* end = nullptr;
    *v = std::strtod(obj.c_str() + p + 1, &end);
    return end != obj.c_str() + p + 1;
  };
  int n = 0;
  std::map<std::string, Entry> parsed;
  size_t pos = text.find("\"entries\"");
  if (pos == std::string::npos) return fail(STENCIL_ERR_INVALID, "%s: no \"entries\"", path);
  while (true) {
    const size_t a = text.find('{', pos);
    if (a == std::string::npos) break;
    const size_t b = text.find('}', a);
    if (b == std::string::npos) return fail(STENCIL_ERR_INVALID, "%s: unterminated entry", path);
    const std::string obj = text.substr(a, b - a + 1);
    pos = b + 1;
    size_t k = obj.find("\"key\"");
    if (k == std::string::npos) return fail(STENCIL_ERR_INVALID, "%s: entry without key", path);
    k = obj.find('"', obj.find(':', k) + 1);
    const size_t k2 = obj.find('"', k + 1);
    if (k == std::string::npos || k2 == std::string::npos)
      return fail(STENCIL_ERR_INVALID, "%s: malformed key", path);
    Entry e;
    double d = 0, s = 0, t = 0, c = 0, fl = 0;
    if (!field_num(obj, "depth", &d) || !field_num(obj, "seg", &s) || d < 1 || d > 64 || s < 0)
      return fail(STENCIL_ERR_INVALID, "%s: entry needs depth >= 1 and seg >= 0", path);
    field_num(obj, "sec_per_step", &t);
    field_num(obj, "candidates", &c);
    field_num(obj, "flags", &fl);
    e.depth = (int)d;
    e.seg = (int)s;
    e.flags = (int)fl & (STENCIL_FLAG_DEVICE_TILING | STENCIL_FLAG_OVERLAPPED_TILING);
    e.sec_per_step = t;
    e.candidates = (int)c;
    parsed[obj.substr(k + 1, k2 - k - 1)] = e;
    ++n;
  }
  {
    std::lock_guard<std::mutex> lock(g_mu);
    for (auto& kv : parsed) g_cache[kv.first] = kv.second;
  }
  if (loaded) *loaded = n;
  return STENCIL_OK;
}

stencil_status stencil_tune_cache_key(const double* coeffs, int32_t radius, const stencil_shape* shape,
                                      stencil_dtype dtype, int32_t flags, char* buf, size_t len) {
  if (!buf || len == 0) return fail(STENCIL_ERR_INVALID, "buffer is NULL");
  stencil_plan_t p = nullptr;
  stencil_status st = probe_plan(coeffs, radius, shape, dtype, &p);
  if (st != STENCIL_OK) return st;
  const std::string key = make_key(p, (flags & STENCIL_TUNE_BATCH) != 0);
  stencil_plan_destroy(p);
  if (key.size() + 1 > len) return fail(STENCIL_ERR_INVALID, "buffer too small for key");
  std::memcpy(buf, key.c_str(), key.size() + 1);
  return STENCIL_OK;
}

}  // extern "C"
