// Host emulation of the serving loop's admission wait (server_admission.hpp)
// with a fake executor: a submitter thread, a scheduler thread that admits
// requests and runs rounds (a sleep stands in for the batched launch), and a
// collector thread that takes results in submission order and releases their
// memory. The budget is small, so the head of the queue often does not fit
// until a collection frees memory.
//
//   admission_emu fixed  the scheduler sleeps until the head fits (the
//                        library's Admission::wait_admissible): every
//                        request completes and the scheduler wakes a bounded
//                        number of times
//   admission_emu queue  the scheduler waits on "queue not empty" instead:
//                        with a head that does not fit it spins holding the
//                        mutex, the collector never releases memory, and a
//                        watchdog finds no progress (expected to fail)
//
// Prints one line "result ..."; exits 0 when every request completed.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "server_admission.hpp"

using namespace stencil_impl;
using Clock = std::chrono::steady_clock;

namespace {

struct Req {
  size_t need = 0;
  bool done = false;
};

}  // namespace

int main(int argc, char** argv) {
  if (argc < 2) return 64;
  const bool fixed = std::strcmp(argv[1], "fixed") == 0;
  const int n = 300;
  std::mt19937 rng(7);
  std::vector<Req> reqs(n);
  for (auto& r : reqs) r.need = 10 + rng() % 91;  // 10 .. 100 of a budget of 120
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  Admission<Req> adm;
  adm.budget = 120;
  adm.slots = 4;
  std::atomic<bool> stop{false};
  std::atomic<int> collected{0};
  long wakeups = 0, rounds = 0;

  std::thread scheduler([&] {
    std::unique_lock<std::mutex> lock(mu);
    while (!stop.load()) {
      adm.admit([](Req*) { return true; });
      std::vector<Req*> round;
      for (Req* r : adm.resident)
        if (!r->done) round.push_back(r);
      if (round.empty()) {
        ++wakeups;
        if (fixed) adm.wait_admissible(cv_work, lock, [&] { return stop.load(); });
        else cv_work.wait(lock, [&] { return stop.load() || !adm.queue.empty(); });
        continue;
      }
      lock.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(300));  // the round's launch
      lock.lock();
      ++rounds;
      for (Req* r : round) r->done = true;
      cv_done.notify_all();
    }
  });
  std::thread collector([&] {
    for (int k = 0; k < n; ++k) {
      std::unique_lock<std::mutex> lock(mu);
      cv_done.wait(lock, [&] { return reqs[k].done || stop.load(); });
      if (stop.load()) return;
      adm.release(&reqs[k]);
      collected++;
      cv_work.notify_all();  // a slot and memory are free again
    }
  });
  std::thread submitter([&] {
    std::mt19937 r2(11);
    for (int k = 0; k < n && !stop.load(); ++k) {
      std::this_thread::sleep_for(std::chrono::microseconds(r2() % 400));
      std::lock_guard<std::mutex> lock(mu);
      adm.queue.push_back(&reqs[k]);
      cv_work.notify_all();
    }
  });
  // watchdog: no collection for 2 s is a live-lock
  int last = -1;
  auto t_last = Clock::now();
  while (collected.load() < n) {
    std::this_thread::sleep_for(std::chrono::milliseconds(10));
    const int c = collected.load();
    if (c != last) {
      last = c;
      t_last = Clock::now();
    } else if (Clock::now() - t_last > std::chrono::seconds(2)) {
      break;
    }
  }
  const int got = collected.load();
  stop = true;
  {
    std::lock_guard<std::mutex> lock(mu);
    cv_work.notify_all();
    cv_done.notify_all();
  }
  submitter.join();
  collector.join();
  scheduler.join();
  std::printf("result collected=%d of %d rounds=%ld wakeups=%ld peak=%zu budget=%zu\n", got, n, rounds, wakeups,
              adm.peak, adm.budget);
  if (got != n) return 2;
  // the scheduler sleeps until the head fits: at most one wake per
  // submission and per collection, plus spurious ones
  if (wakeups > 4L * n) return 3;
  if (adm.peak > adm.budget) return 4;
  return 0;
}
