// worklist.hpp -- the work-list protocol of the persistent kernels (the
// batch kernels and single-grid persistent launches), shared by the device
// code and host code.
//
// A launch's work is a list of items, each a group of tiles of one pass of
// one job; consecutive items of one (job, pass) form a chunk. Workgroups
// claim items in list order from one counter. An item of pass k > 0 first
// waits until its job's count of finished tiles reaches k x tiles (every
// tile of pass k - 1), then runs, then adds its tiles to the count with
// release semantics (paper Section 4.1, tile-by-tile execution, extended
// across grids). Every pass of a job comes after its previous pass in the
// list and items are claimed in order by running workgroups, so each wait
// depends only on items already held by running workgroups and ends. Waits
// are bounded by a watchdog: an expired wait sets the launch's error word,
// every later wait of the launch then returns at once, and the launch
// drains with its results undefined.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "../../include/stencil.h"

namespace stencil_impl {
namespace worklist {

// Tiles per item: 2D items are four tiles (one per wave of the workgroup),
// 3D items one tile (all four waves).
__host__ __device__ constexpr int tiles_per_item(int ndim) { return ndim == 2 ? 4 : 1; }

__host__ __device__ constexpr int64_t items_per_pass(int ndim, int64_t tiles) {
  return (tiles + tiles_per_item(ndim) - 1) / tiles_per_item(ndim);
}

// Tiles of item `sub` of a pass (the last item of a 2D pass may hold fewer).
__host__ __device__ constexpr unsigned item_tiles(int ndim, int tiles, int sub) {
  const int first = tiles_per_item(ndim) * sub;
  return (unsigned)(tiles - first < tiles_per_item(ndim) ? tiles - first : tiles_per_item(ndim));
}

// Finished tiles a job must count before pass `pass` may run.
__host__ __device__ constexpr unsigned need_before(int pass, int tiles) { return (unsigned)pass * (unsigned)tiles; }

struct JobShape {
  int32_t npass;
  int64_t items_per_pass;
};

// The list of a launch: chunks (job, pass) ordered by the job's progress
// after the chunk, (pass + 1) / npass, so that short and long jobs advance
// together; ties by job, then pass. cf receives the nchunks + 1 prefix sums
// of the chunks' item counts.
inline void build(const std::vector<JobShape>& jobs, std::vector<int32_t>& cj, std::vector<int32_t>& cp,
                  std::vector<int64_t>& cf) {
  struct C {
    double key;
    int job, pass;
  };
  std::vector<C> chunks;
  for (int j = 0; j < (int)jobs.size(); ++j)
    for (int k = 0; k < jobs[j].npass; ++k) chunks.push_back({(double)(k + 1) / jobs[j].npass, j, k});
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
    cf.push_back(cf.back() + jobs[c.job].items_per_pass);
  }
}

// Chunk holding item `it`: the largest c with first[c] <= it (first holds
// nchunks + 1 prefix sums).
__host__ __device__ inline int find_chunk(const int64_t* first, int nchunks, int64_t it) {
  int lo = 0, hi = nchunks;  // first[lo] <= it < first[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (first[mid] <= it) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Waits until *ctr >= need. Returns false if the watchdog expired here (then
// sets *err) or an earlier wait of the launch already failed. The counter is
// polled with relaxed loads and one acquire fence follows the load that sees
// it reach `need` (on the device an acquire load at agent scope invalidates
// cache lines at every poll, under the workgroups still streaming). P
// supplies the memory operations and the clock:
//   unsigned load_relaxed(const unsigned*), void acquire_fence(),
//   void raise(unsigned*) (store 1, relaxed), uint64_t now(), void pause().
template <class P>
__host__ __device__ inline bool wait_count(const unsigned* ctr, unsigned need, unsigned* err,
                                           int64_t timeout_ticks) {
  const uint64_t t0 = P::now();
  while (true) {
    if (P::load_relaxed(ctr) >= need) {
      P::acquire_fence();
      return true;
    }
    if (P::load_relaxed(err) != 0u) return false;
    if ((int64_t)(P::now() - t0) > timeout_ticks) {
      P::raise(err);
      return false;
    }
    P::pause();
  }
}

// Status that a stream's report word (the OR of its launches' error words)
// stands for.
constexpr stencil_status status_of_report(unsigned word) { return word ? STENCIL_ERR_TIMEOUT : STENCIL_OK; }

}  // namespace worklist
}  // namespace stencil_impl
