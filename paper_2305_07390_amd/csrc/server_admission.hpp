// server_admission.hpp -- the serving loop's admission state: a FIFO of
// submitted requests, the set of resident ones, and the rule that admits the
// head of the queue when a slot is free and its device memory fits in the
// budget. Host-only and free of device calls, so the server (server.cpp) and
// host tests of its waiting discipline share it.
//
// Req needs a `size_t need` member: the device bytes the request holds while
// resident. Every member function is called with the owner's mutex held.
#pragma once
#include <algorithm>
#include <condition_variable>
#include <cstddef>
#include <deque>
#include <mutex>
#include <vector>

namespace stencil_impl {

template <class Req>
struct Admission {
  size_t budget = 0;  // device bytes that resident requests may hold
  int slots = 1;      // resident requests at most
  std::deque<Req*> queue;     // submitted, not yet admitted (arrival order)
  std::vector<Req*> resident; // admitted, not yet released
  size_t in_use = 0, peak = 0;

  // Whether the head of the queue can be admitted now.
  bool head_fits() const {
    return !queue.empty() && (int)resident.size() < slots && in_use + queue.front()->need <= budget;
  }

  // Admits queued requests in arrival order while the head fits (a request
  // that does not fit blocks the ones behind it: no overtaking). start(r)
  // begins the request's upload and returns false if it could not; such a
  // request leaves the queue without becoming resident. Returns the number
  // admitted.
  template <class Start>
  int admit(Start&& start) {
    int n = 0;
    while (head_fits()) {
      Req* r = queue.front();
      queue.pop_front();
      if (!start(r)) continue;
      in_use += r->need;
      peak = std::max(peak, in_use);
      resident.push_back(r);
      ++n;
    }
    return n;
  }

  // Gives back a resident request's slot and memory (no-op otherwise).
  // Returns whether it was resident.
  bool release(Req* r) {
    auto it = std::find(resident.begin(), resident.end(), r);
    if (it == resident.end()) return false;
    resident.erase(it);
    in_use -= r->need;
    return true;
  }

  // Blocks until a queued request fits or stop() holds. The predicate is
  // "the head fits", not "the queue is not empty": with a head that does not
  // fit the latter returns at once, and the caller's loop would spin holding
  // the mutex that submissions and collections (the only events that can
  // make the head fit) need.
  template <class Stop>
  void wait_admissible(std::condition_variable& cv, std::unique_lock<std::mutex>& lock, Stop&& stop) {
    cv.wait(lock, [&] { return stop() || head_fits(); });
  }
};

}  // namespace stencil_impl
