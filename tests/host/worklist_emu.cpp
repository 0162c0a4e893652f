// Host emulation of the persistent kernels' work-list protocol: one thread
// per workgroup runs the item loop of the batch kernel over the library's own
// list builder, chunk lookup, item tile counts, bounded wait and report
// mapping (worklist.hpp), with std atomics in place of the device's.
//
//   worklist_emu ok   SEED   every item runs, each after all tiles of its
//                            job's previous pass; no wait expires
//   worklist_emu held SEED   the workgroup that claims one early item holds
//                            it without publishing: the waits behind it
//                            expire, the error word is set, every other
//                            workgroup drains, and the report maps to
//                            STENCIL_ERR_TIMEOUT
//
// Prints one line "result ..." and exits 0 when the expected behaviour holds.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <random>
#include <thread>
#include <vector>

#include "worklist.hpp"

using namespace stencil_impl;

namespace {

struct HostWait {
  static unsigned load_relaxed(const unsigned* p) { return __atomic_load_n(p, __ATOMIC_RELAXED); }
  static void acquire_fence() { __atomic_thread_fence(__ATOMIC_ACQUIRE); }
  static void raise(unsigned* p) { __atomic_store_n(p, 1u, __ATOMIC_RELAXED); }
  static uint64_t now() {  // 100 MHz ticks, as the device's realtime clock
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch()).count() / 10;
  }
  static void pause() { std::this_thread::yield(); }
};

struct Job {
  int ndim, tiles, npass;
};

}  // namespace

// One launch over `jobs` by `workers` threads; returns the exit status.
int launch(const std::vector<Job>& jobs, bool held, const char* name) {
  const int njobs = (int)jobs.size(), workers = 8;
  std::vector<worklist::JobShape> shapes;
  for (const Job& b : jobs) shapes.push_back({b.npass, worklist::items_per_pass(b.ndim, b.tiles)});
  std::vector<int32_t> cj, cp;
  std::vector<int64_t> cf;
  worklist::build(shapes, cj, cp, cf);
  const int nchunks = (int)cj.size();
  const int64_t nitems = cf.back();
  // the list puts every pass of a job after its previous pass
  for (int c = 0; c < nchunks; ++c)
    for (int d = c + 1; d < nchunks; ++d)
      if (cj[d] == cj[c] && cp[d] < cp[c]) {
        std::printf("result list-order chunk %d\n", c);
        return 1;
      }
  // the held item: job 0's first item of pass 0
  int64_t held_item = -1;
  for (int c = 0; c < nchunks && held_item < 0; ++c)
    if (cj[c] == 0 && cp[c] == 0) held_item = cf[c];

  std::atomic<unsigned long long> cursor{0};
  std::vector<unsigned> done(njobs, 0u);
  unsigned err = 0;
  std::vector<std::vector<std::atomic<int>>> prog(njobs);  // passes finished per tile
  for (int j = 0; j < njobs; ++j) prog[j] = std::vector<std::atomic<int>>(jobs[j].tiles);
  std::atomic<int> violations{0}, executed{0}, exited{0};
  std::atomic<bool> let_go{false};
  const int64_t timeout = held ? 2000000 : 500000000;  // 20 ms / 5 s of 100 MHz ticks

  auto workgroup = [&](int w) {
    std::mt19937 r2(1000u + (unsigned)w);
    while (true) {
      const int64_t it = (int64_t)cursor.fetch_add(1);
      if (it >= nitems) break;
      const int c = worklist::find_chunk(cf.data(), nchunks, it);
      const int job = cj[c], pass = cp[c], sub = (int)(it - cf[c]);
      const Job& J = jobs[job];
      const bool ok = pass == 0 ||
                      worklist::wait_count<HostWait>(&done[job], worklist::need_before(pass, J.tiles), &err, timeout);
      if (held && it == held_item) {
        // a workgroup that never gets to run its item
        while (!let_go.load()) std::this_thread::sleep_for(std::chrono::milliseconds(1));
        break;
      }
      const unsigned nt = worklist::item_tiles(J.ndim, J.tiles, sub);
      const int first = worklist::tiles_per_item(J.ndim) * sub;
      if (ok) {
        // the pass reads its neighbours' results: every tile of the job must
        // have finished the previous pass. (Once a wait has expired, skipped
        // items still publish their counts so that the launch drains, and the
        // launch's results are undefined: only items that saw the error word
        // clear after their wait are held to this.)
        const bool clean = __atomic_load_n(&err, __ATOMIC_ACQUIRE) == 0u;
        for (int u = 0; u < J.tiles && clean; ++u)
          if (prog[job][u].load(std::memory_order_relaxed) < pass) violations++;
        std::this_thread::sleep_for(std::chrono::microseconds(r2() % 200));
        for (unsigned t = 0; t < nt; ++t) prog[job][first + t].store(pass + 1, std::memory_order_relaxed);
        executed++;
      }
      __atomic_fetch_add(&done[job], nt, __ATOMIC_RELEASE);  // published, run or skipped
    }
    exited++;
  };
  std::vector<std::thread> pool;
  for (int w = 0; w < workers; ++w) pool.emplace_back(workgroup, w);
  // every workgroup but a held one must drain
  const auto t0 = std::chrono::steady_clock::now();
  while (exited.load() < workers - (held ? 1 : 0)) {
    if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(20)) {
      std::printf("result %s no-drain exited=%d\n", name, exited.load());
      std::fflush(stdout);
      std::_Exit(2);
    }
    std::this_thread::sleep_for(std::chrono::milliseconds(1));
  }
  let_go = true;
  for (auto& t : pool) t.join();
  unsigned report = 0;
  report |= __atomic_load_n(&err, __ATOMIC_RELAXED);  // the launch's error word folded into the stream's
  const stencil_status st = worklist::status_of_report(report);
  int complete = 1;
  for (int j = 0; j < njobs; ++j)
    for (int u = 0; u < jobs[j].tiles; ++u) complete &= prog[j][u].load() == jobs[j].npass;
  std::printf("result %s items=%lld executed=%d violations=%d err=%u status=%d complete=%d\n", name,
              (long long)nitems, executed.load(), violations.load(), report, (int)st, complete);
  if (violations.load() != 0) return 1;
  if (!held) return (st == STENCIL_OK && complete && executed.load() == nitems) ? 0 : 1;
  return (st == STENCIL_ERR_TIMEOUT && !complete && executed.load() < nitems) ? 0 : 1;
}

int main(int argc, char** argv) {
  if (argc < 3) return 64;
  const bool held = std::strcmp(argv[1], "held") == 0;
  std::mt19937 rng((unsigned)std::atoi(argv[2]));
  // a mix of 24 jobs, 2D and 3D, as a batch
  std::vector<Job> mix;
  for (int j = 0; j < 24; ++j) {
    Job b{2 + (int)(rng() % 2), 1 + (int)(rng() % 13), 1 + (int)(rng() % 7)};
    if (j == 0) b.npass = 5;  // the held item's job has later passes
    mix.push_back(b);
  }
  if (held) return launch(mix, true, "mix");
  // one long 3D job, as a persistent single-grid launch: the items of pass
  // k + 1 are claimed while those of pass k still run
  const std::vector<Job> single = {{3, 13, 12}};
  const int a = launch(mix, false, "mix");
  const int b = launch(single, false, "single");
  return a != 0 ? a : b;
}
